"""Shared helpers of the GPU tests: run the HIP library and the oracle on the
same seeded workload, and map PDFs between the two lattice orders."""
import sys

import numpy as np

import oracle
from paper_2407_12263_amd import lbm


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def order_maps(q=19):
    """perm such that gpu[i] = oracle[perm[i]] (lattice q = 19 or 27)."""
    eg, _ = lbm.lbm_lattice_q(q)
    eo, _ = oracle.lattice(q)
    perm = [next(k for k in range(q) if tuple(eo[k]) == tuple(eg[i])) for i in range(q)]
    inv = [perm.index(k) for k in range(q)]
    return np.array(perm), np.array(inv)


# parameters of the GPU solver only (the oracle has no phase-mass bookkeeping
# and no storage modes)
SOLVER_ONLY = ("mass_fix_every", "check_every", "store_log2", "p_ref")


def oracle_run(w, steps, **over):
    prm = w.params()
    prm.update({k: v for k, v in over.items() if k not in SOLVER_ONLY})
    o = oracle.Oracle(oracle.OracleParams(**prm), w.phi0, w.u0, w.p0)
    o.step(steps)
    return o


def gpu_solver(w, precision, **over):
    prm = w.params()
    prm.update(over)
    prm["precision"] = precision
    return lbm.Solver(prm, w.phi0, w.u0, w.p0)


def gpu_fields(sol):
    phi, u, p = sol.fields()
    return phi.cpu().numpy(), u.cpu().numpy(), p.cpu().numpy()
