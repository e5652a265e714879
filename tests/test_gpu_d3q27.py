"""The method on D3Q27 (all 27 vectors of {-1,0,1}^3, weights 8/27, 2/27,
1/54, 1/216): the HIP library with lattice = 27 against the D3Q27 build of
the oracle, at the tolerances of the D3Q19 path.

* trajectories: the static droplet (32^3, 100 steps) in every storage mode
  (FP64 1e-12, FP32 1e-5, FP16/BF16 storage 2e-3); FP64 runs with walls on
  all faces (corner vectors bounce back along both wall axes), with walls in
  y, on a ragged lattice, on a periodic Taylor-Green field and with exact
  streaming (c = 1);
* the step map from identical states (the oracle's state at t = 30 loaded
  into the GPU), with and without walls, c = 0.997 and 1: every PDF to 1e-14;
* at full size (Rayleigh-Taylor 128 x 512 x 128, walls in y, the launch
  configuration of the D3Q19 benchmark): one step from the GPU's own state
  at t = 40, every node's phi and PDFs, FP16 storage 1e-4, FP32 2e-6;
* phase mass over 10^4 FP16 steps (relative drift <= 1e-6) and bitwise
  checkpoint / restart.
"""
import numpy as np
import pytest

import oracle
from paper_2407_12263_amd import inputs

from gpu_common import gpu_fields, gpu_solver, oracle_run, order_maps, say

pytestmark = pytest.mark.gpu

Q27 = dict(lattice=27)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_12263_amd import lbm
    lbm.load_library()


def _cmp(w, precision, steps, tol_phi, tol_u=None, **over):
    over = dict(Q27, **over)
    say(f"[d3q27] {w.name} {w.nx}x{w.ny}x{w.nz} {precision} steps={steps} over={over}")
    o = oracle_run(w, steps, **over)
    sol = gpu_solver(w, precision, **over)
    sol.step(steps)
    phi, u, p = gpu_fields(sol)
    po, uo, qo = o.fields()
    e_phi, e_u, e_p = np.abs(phi - po).max(), np.abs(u - uo).max(), np.abs(p - qo).max()
    say(f"   max|dphi|={e_phi:.3e} max|du|={e_u:.3e} max|dp|={e_p:.3e}")
    assert np.isfinite(phi).all()
    assert e_phi <= tol_phi
    if tol_u is not None:
        assert e_u <= tol_u and e_p <= tol_u


SMALL = {
    "rt": lambda: inputs.rayleigh_taylor(nx=32, ny=128, nz=16),
    "bubble": lambda: inputs.rising_bubble(nx=32, ny=32, nz=64, R=8, zc=20, g=2e-5),
    "box": lambda: inputs.rising_bubble(nx=6, ny=5, nz=12, R=2.0, zc=6.0, g=1e-4),
    "tg": lambda: inputs.taylor_green_breakup(n=32),
    "ragged": lambda: inputs.static_droplet(n=13, R=3.5, ny=7, nz=9, sigma=2e-3),
}


@pytest.mark.parametrize("prec,tol,tol_u", [("fp64", 1e-12, 1e-13), ("fp32", 1e-5, 1e-6),
                                            ("fp16", 2e-3, None), ("bf16", 2e-3, None)])
def test_static_droplet_100_steps(prec, tol, tol_u):
    _cmp(inputs.static_droplet(), prec, 100, tol, tol_u)


@pytest.mark.parametrize("name,steps", [("bubble", 100), ("box", 50), ("rt", 10), ("tg", 100),
                                        ("ragged", 50)])
def test_fp64_trajectory(name, steps):
    _cmp(SMALL[name](), "fp64", steps, 1e-12, 1e-13)


def test_fp64_exact_streaming_c1():
    _cmp(inputs.static_droplet(courant=1.0), "fp64", 20, 1e-12, 1e-13)


@pytest.mark.parametrize("name", ["rt", "box", "ragged"])
@pytest.mark.parametrize("courant", [0.997, 1.0])
def test_one_step_parity_from_oracle_state(name, courant):
    w = SMALL[name]().with_(courant=courant)
    say(f"[d3q27 one-step] {w.name} c={courant}")
    perm, _ = order_maps(27)
    o = oracle_run(w, 30, **Q27)
    f, g = o.pdfs()
    sol = gpu_solver(w, "fp64", **Q27)
    sol.set_pdfs(f[perm], g[perm])
    assert np.abs(gpu_fields(sol)[0] - o.fields()[0]).max() < 1e-14
    o.step(1)
    sol.step(1)
    phi, u, p = gpu_fields(sol)
    po, uo, qo = o.fields()
    fg, gg = sol.get_pdfs()
    fo, go = o.pdfs()
    e = [np.abs(phi - po).max(), np.abs(u - uo).max(), np.abs(p - qo).max(),
         np.abs(fg.cpu().numpy() - fo[perm]).max(), np.abs(gg.cpu().numpy() - go[perm]).max()]
    say("   " + " ".join(f"{x:.2e}" for x in e))
    assert max(e) < 1e-14


@pytest.mark.parametrize("prec,tol", [("fp16", 1e-4), ("fp32", 2e-6)])
def test_full_size_one_step(prec, tol):
    w = inputs.rayleigh_taylor()
    say(f"[d3q27 full] {w.name} {w.nx}x{w.ny}x{w.nz} {prec}: 40 GPU steps, then one on both")
    perm, inv = order_maps(27)
    sol = gpu_solver(w, prec, **Q27)
    sol.step(40)
    f, g = sol.get_pdfs()
    f, g = f.cpu().numpy(), g.cpu().numpy()
    o = oracle.Oracle(oracle.OracleParams(**w.params(), **Q27), w.phi0, w.u0, w.p0)
    o.set_pdfs(f[inv], g[inv])
    del f, g
    o.step(1)
    sol.step(1)
    phi = sol.fields()[0].cpu().numpy()
    po = o.fields()[0]
    fo, go = o.pdfs()
    del o
    fg, gg = sol.get_pdfs()
    ef = np.abs(fg.cpu().numpy() - fo[perm]).max()
    del fo
    eg = np.abs(gg.cpu().numpy() - go[perm]).max()
    e = np.abs(phi - po).max()
    say(f"   max|dphi| {e:.2e}  max|df| {ef:.2e}  max|dg| {eg:.2e}")
    assert max(e, ef, eg) <= tol


def test_phase_mass_drift_fp16_10k_steps():
    w = inputs.static_droplet()
    say("[d3q27 mass] static droplet fp16, 10000 steps")
    sol = gpu_solver(w, "fp16", mass_fix_every=10, **Q27)
    m0 = float(w.phi0.sum())
    worst = 0.0
    for t in (2500, 5000, 10000):
        sol.step(t - sol.t)
        worst = max(worst, abs(sol.diagnostics()["sum_phi"] - m0) / m0)
    say(f"   max relative drift {worst:.2e}")
    assert worst <= 1e-6


def test_checkpoint_restart_bitwise():
    w = SMALL["tg"]()
    say("[d3q27 restart] tg fp32")
    a = gpu_solver(w, "fp32", mass_fix_every=0, **Q27)
    a.step(100)
    b = gpu_solver(w, "fp32", mass_fix_every=0, **Q27)
    b.step(50)
    f, g = b.get_pdfs()
    assert f.shape[0] == 27
    c = gpu_solver(w, "fp32", mass_fix_every=0, **Q27)
    c.set_pdfs(f, g)
    c.step(50)
    assert np.array_equal(a.fields()[0].cpu().numpy(), c.fields()[0].cpu().numpy())


def test_lattices_give_different_runs():
    """D3Q19 and D3Q27 are two discretisations of the same equations: their
    runs differ (the corner vectors enter), by far less than the interface."""
    w = inputs.static_droplet()
    a = gpu_solver(w, "fp64")
    b = gpu_solver(w, "fp64", **Q27)
    a.step(100)
    b.step(100)
    d = np.abs(gpu_fields(a)[0] - gpu_fields(b)[0]).max()
    say(f"[d3q27] D3Q19 vs D3Q27 after 100 steps: max|dphi| = {d:.2e}")
    assert 1e-8 < d < 0.05
