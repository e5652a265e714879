"""The plain solver as the surrogate's fallback: every way a window can fail
is driven through the real schedule (``accel.accelerated_run``) with a
predictor that returns a bad change, on a 64^3 emulsion (32^3 coarse).
A window that fails its checks is discarded and the solver runs the cycle,
so the run must end in exactly the plain solver's state; a window whose
prolonged fields the solver rejects takes the reset path. Also the reset
contract of the C ABI: a rejected reset leaves no usable state, and
lbm_step refuses to run on it until a reset succeeds."""
import math

import numpy as np
import pytest

from paper_2407_12263_amd import inputs

from gpu_common import say

pytestmark = pytest.mark.gpu

WINDOWS, CYCLE, NSUR = 8, 4, 3


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_12263_amd import accel, lbm, surrogate as sur
    w = inputs.emulsion(n=64, n_drops=6, rmin=6.0, rmax=10.0, seed=3)
    return dict(torch=torch, accel=accel, lbm=lbm, sur=sur, w=w)


def _fresh(env):
    accel, lbm = env["accel"], env["lbm"]
    w = env["w"]
    sol = lbm.Solver(dict(w.params(), precision="fp16"), w.phi0, w.u0, w.p0)
    cp = accel.Coupler(sol, accel.state_scale(0.02))
    return sol, cp


def _plain_phi(env):
    sol, _ = _fresh(env)
    sol.step(WINDOWS * env["accel"].K_STEPS)
    return sol.fields()[0].cpu().numpy()


def _bad_change(env, cp, kind):
    """A predicted change (units of rscale = 1, FP32 [Pc][16]) that fails the
    check named by kind and no earlier one."""
    torch = env["torch"]
    nx, ny, nz = cp.coarse
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.zeros((cp.P, 16), dtype=np.float32)
    if kind == "nonfinite":
        d[7, 0] = np.nan
    elif kind == "range":
        # a mass-neutral checkerboard of +-0.3 in phi: max phi about 1.3
        d[:, 0] = (0.3 * (1 - 2 * ((x + y + z) % 2))).ravel()
    elif kind == "mass":
        # 1% of the phase mass, spread evenly (phi stays inside its range)
        d[:, 0] = 0.01 * env["w"].phi0.mean()
    elif kind == "divergence":
        # u_x += U sin(2 pi x / nx): RMS divergence 2 pi / nx / sqrt(2) = 0.14
        d[:, 1] = np.sin(2 * np.pi * x / nx).ravel()
    return torch.as_tensor(d).to(cp.solver.device)


@pytest.mark.parametrize("kind", ["nonfinite", "range", "mass", "divergence"])
def test_failed_window_falls_back_to_the_plain_solver(env, kind):
    accel = env["accel"]
    say(f"[fallback] 64^3 emulsion FP16, predictor failing '{kind}'")
    ref = _plain_phi(env)
    sol, cp = _fresh(env)
    bad = _bad_change(env, cp, kind)
    limits = accel.CheckLimits(div_rms=0.05)
    st = accel.accelerated_run(cp, None, np.ones(16, np.float32), WINDOWS, nsur=NSUR,
                               cycle=CYCLE, limits=limits, predictor=lambda s: bad,
                               warmup_windows=0)
    cycles = WINDOWS // CYCLE
    say(f"   fallbacks {st.fallbacks} {st.fail_reasons}, surrogate windows {st.sur_windows}")
    assert st.fallbacks == cycles
    assert st.fail_reasons == {kind: cycles}
    assert st.sur_windows == 0 and st.lbm_windows == WINDOWS
    assert sol.t == WINDOWS * accel.K_STEPS
    # nothing of the discarded windows reached the solver
    phi = sol.fields()[0].cpu().numpy()
    assert np.array_equal(phi, ref), np.abs(phi - ref).max()


def test_rejected_fields_take_the_reset_path(env):
    """Checks loose enough to pass a +-2 checkerboard in phi; its plain
    trilinear prolongation puts fine phi far outside what lbm_reset
    accepts, so the solver is rebuilt from the cycle-start fields and runs
    the cycle itself."""
    accel, torch = env["accel"], env["torch"]
    say("[fallback] 64^3 emulsion FP16, prolonged fields rejected by lbm_reset")
    sol, cp = _fresh(env)
    nx, ny, nz = cp.coarse
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.zeros((cp.P, 16), dtype=np.float32)
    d[:, 0] = (2.0 * (1 - 2 * ((x // 2 + y // 2 + z // 2) % 2))).ravel()
    bad = torch.as_tensor(d).to(sol.device)
    limits = accel.CheckLimits(mass_tol=1e9, phi_lo=-1e9, phi_hi=1e9, div_rms=1e9)
    m0 = float(env["w"].phi0.sum())
    st = accel.accelerated_run(cp, None, np.ones(16, np.float32), WINDOWS, nsur=NSUR,
                               cycle=CYCLE, limits=limits, predictor=lambda s: bad,
                               linear=True, warmup_windows=0, judge_tol=None)
    say(f"   fallbacks {st.fallbacks} {st.fail_reasons}")
    assert st.fail_reasons == {"reset": WINDOWS // CYCLE}
    assert st.sur_windows == 0 and st.lbm_windows == WINDOWS
    assert sol.t == WINDOWS * accel.K_STEPS
    d1 = sol.diagnostics()
    assert math.isfinite(d1["sum_phi"]) and 0.0 <= d1["phi_max"] < 1.1
    assert abs(d1["sum_phi"] - m0) / m0 < 1e-6


def test_rejected_reset_leaves_the_context_refusing_steps(env):
    lbm, torch = env["lbm"], env["torch"]
    say("[fallback] lbm_reset with phi = 2, then lbm_step")
    sol, _ = _fresh(env)
    sol.step(3)
    phi, u, p = sol.fields()
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_reset(sol.ctx, torch.full_like(phi, 2.0), u, p, sol.t)
    assert e.value.status == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        sol.step(1)
    assert e.value.status == lbm.LBM_ESTATE
    lbm.lbm_reset(sol.ctx, phi, u, p, 3)
    sol.step(2)
    assert sol.t == 5
    assert math.isfinite(sol.diagnostics()["sum_phi"])
