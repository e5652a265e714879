"""Writes droplet_2d_convergence.json: the oracle's relative L2 error of phi
(Sec. 3.1, the norm of the convergence study) for the 2D static droplet
(Cn = 0.06, La = 1, tau_rho = 0.02) after two viscous times t0 = eta D/(2 sigma)
at L0 = 50, 100 and 200. Calls only the oracle and the input generator
(the 200 case runs about 7 minutes on one core)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2407_12263_amd import inputs  # noqa: E402


def main():
    out = {"description": "oracle ||phi - phi0||_2 / ||phi0||_2 after T = round(2 t0) steps",
           "Cn": 0.06, "La": 1.0, "tau_rho": 0.02, "M": 0.02, "runs": {}}
    for L0 in [int(a) for a in sys.argv[1:]] or (50, 100, 200):
        w = inputs.droplet_2d(L0)
        T = int(round(2 * w.meta["t0"]))
        o = oracle.Oracle(oracle.OracleParams(**w.params()), w.phi0, w.u0, w.p0)
        o.step(T)
        phi, u, _ = o.fields()
        err = float(np.sqrt(((phi - w.phi0) ** 2).sum() / (w.phi0 ** 2).sum()))
        umax = float(np.sqrt((u ** 2).sum(0)).max())
        out["runs"][str(L0)] = {"steps": T, "phi_l2_error": err, "umax": umax}
        print(L0, T, err, umax, flush=True)
    with open(os.path.join(HERE, "droplet_2d_convergence.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
