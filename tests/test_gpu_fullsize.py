"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (default tile order and plane pitch; interior and
wall-slab launches): the GPU evolves each lattice for 40 steps. Its state is
then read back (the decoded FP64 values of what it stores) and loaded into
the oracle, and both take one step from that identical state; every node's
phi, u, p and PDFs are compared. A trajectory comparison at these sizes
would instead measure the scheme's amplification of rounding differences,
not the kernels.

Tolerances: the stated ones per storage mode (phi: FP64 1e-12, FP32 1e-5,
16-bit 2e-3), and for one step the tighter bounds of its arithmetic, on
phi and every PDF:
  FP64  1e-13  (a few roundings of O(1) sums; measured <= 9e-16)
  FP32  2e-6   (about ten FP32 roundings through propagation and collision
               of PDFs up to 1/3: ~3e-8 each; measured <= 5e-7)
  FP16  1e-4   (each stored deviation rounds to 2^-11 relative, deviations
               up to ~0.05, 19 taps per moment; measured <= 1.5e-5)
  BF16  5e-4   (2^-8 relative, 8x FP16; measured <= 8e-5)
"""
import numpy as np
import pytest

import oracle
from paper_2407_12263_amd import inputs

from gpu_common import gpu_solver, order_maps, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


FULL = {
    "rt": inputs.rayleigh_taylor,            # 128 x 512 x 128, walls in y (the benchmark)
    "bubble": inputs.rising_bubble,          # 128 x 128 x 256, walls on all faces
    "tg": lambda: inputs.taylor_green_breakup(n=256),   # 256^3 periodic
    "emulsion": lambda: inputs.emulsion(n=256),          # 256^3 periodic, 200 droplets
}
TOL = {"fp64": (1e-12, 1e-12, 1e-12), "fp32": (1e-5, 1e-5, 1e-5), "fp16": (2e-3, 2e-3, 2e-3),
       "bf16": (2e-3, 2e-3, 2e-3)}
ONE_STEP = {"fp64": 1e-13, "fp32": 2e-6, "fp16": 1e-4, "bf16": 5e-4}


@pytest.mark.parametrize("name,prec", [("rt", "fp16"), ("rt", "bf16"), ("rt", "fp32"),
                                       ("rt", "fp64"), ("bubble", "fp16"), ("bubble", "fp64"),
                                       ("tg", "fp16"), ("tg", "fp32"), ("emulsion", "fp16")])
def test_full_size_one_step_parity(name, prec):
    w = FULL[name]()
    say(f"[full] {w.name} {w.nx}x{w.ny}x{w.nz} {prec}: 40 GPU steps, then one step on both")
    _, inv = order_maps()
    sol = gpu_solver(w, prec)
    sol.step(40)
    f, g = sol.get_pdfs()
    f, g = f.cpu().numpy(), g.cpu().numpy()
    o = oracle.Oracle(oracle.OracleParams(**w.params()), w.phi0, w.u0, w.p0)
    o.set_pdfs(f[inv], g[inv])
    del f, g
    o.step(1)
    sol.step(1)
    phi, u, p = (a.cpu().numpy() for a in sol.fields())
    po, uo, qo = o.fields()
    e = (np.abs(phi - po).max(), np.abs(u - uo).max(), np.abs(p - qo).max())
    fo, go = o.pdfs()
    del o
    fg, gg = sol.get_pdfs()
    perm, _ = order_maps()
    ef = np.abs(fg.cpu().numpy() - fo[perm]).max()
    del fo
    eg = np.abs(gg.cpu().numpy() - go[perm]).max()
    say(f"   max|dphi| {e[0]:.2e}  max|du| {e[1]:.2e}  max|dp| {e[2]:.2e}  "
        f"max|df| {ef:.2e}  max|dg| {eg:.2e}")
    tp, tu, tq = TOL[prec]
    assert np.isfinite(phi).all()
    assert e[0] <= tp and e[1] <= tu and e[2] <= tq
    assert max(ef, eg) <= tp
    assert max(e[0], ef, eg) <= ONE_STEP[prec]


def test_largest_lattice_fp16():
    """The largest lattice whose 19 population planes of 16-bit storage fit
    one 32-bit buffer range: 512 x 512 x 215 (56.4 M nodes; the last plane
    starts 3.99 GB into the range). 216 planes are rejected. The initial
    moments return phi0 at every node, and 20 steps keep the phase mass to
    1e-6 and every value finite."""
    import torch
    from paper_2407_12263_amd import lbm
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes(lbm.make_params(512, 512, 216, precision="fp16"))
    w = inputs.static_droplet(n=512, R=40.0, nz=215, sigma=1e-3)
    say(f"[full] largest lattice {w.nx}x{w.ny}x{w.nz} fp16: init, 20 steps")
    sol = gpu_solver(w, "fp16")
    phi0 = torch.as_tensor(w.phi0, device="cuda")
    e0 = float((sol.fields()[0] - phi0).abs().max())
    m0 = float(phi0.sum())
    del phi0
    sol.step(20)
    d = sol.diagnostics()
    drift = abs(d["sum_phi"] - m0) / m0
    say(f"   init max|dphi| {e0:.2e}, mass drift after 20 steps {drift:.2e}, umax {d['umax']:.2e}")
    assert e0 < 2e-3
    assert np.isfinite(d["sum_phi"]) and np.isfinite(d["umax"]) and d["umax"] < 1e-2
    assert drift < 1e-6
