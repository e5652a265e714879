"""The coupling kernels of the surrogate (coarsen, prolong, level-set update
with mass restoration, features, window checks, residual updates) through the
sur_* C ABI against the coupling oracle, on a ragged coarse grid (point
counts that are not multiples of the 256-thread blocks) and at the full size
(128^3 coarse, 256^3 fine)."""
import numpy as np
import pytest

from oracle import coupling_oracle as co

from gpu_common import say

pytestmark = pytest.mark.gpu

SCALE = np.array([1.0, 0.02, 0.02, 0.02, 4e-4] + [1.0] * 11, dtype=np.float32)

# coarse nx, ny, nz: ragged (480 points) and the emulsion's full coarse grid
@pytest.fixture(params=[(10, 6, 8), (128, 128, 128)], ids=["ragged", "full"])
def cg(request):
    return request.param


@pytest.fixture(scope="module")
def sur():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_12263_amd import surrogate
    surrogate.load_library()
    return surrogate


def _dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def _fine_fields(rng, cg):
    nx, ny, nz = (2 * n for n in cg)
    shp = (nz, ny, nx)
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[:, None, None]
    # two droplets with tanh profiles plus noise; velocity and pressure at
    # their physical magnitudes
    r1 = np.sqrt((x - 0.365 * nx) ** 2 + (y - 0.425 * ny) ** 2 + (z - 0.4125 * nz) ** 2)
    r2 = np.sqrt((x - 0.71 * nx) ** 2 + (y - 0.533 * ny) ** 2 + (z - 0.6125 * nz) ** 2)
    phi = np.maximum(co.profile(4.5 - r1, 4.0), co.profile(3.5 - r2, 4.0))
    phi = phi + 1e-3 * rng.standard_normal(shp)
    u = 0.02 * rng.standard_normal((3,) + shp)
    p = 4e-4 * rng.standard_normal(shp)
    return phi, u, p


def _coarse(s, cg):
    nx, ny, nz = cg
    return s.reshape(nz, ny, nx, 16)


def test_coarsen_and_prolong_add(sur, cg):
    import torch
    say("[coupling] coarsen / prolong_add")
    rng = np.random.default_rng(1)
    phi, u, p = _fine_fields(rng, cg)
    phi32, u32, p32 = (a.astype(np.float32) for a in (phi, u, p))
    out = torch.full((np.prod(cg), 16), 7.0, dtype=torch.float32, device="cuda")
    outb = torch.empty((np.prod(cg), 16), dtype=torch.int16, device="cuda")
    sur.sur_coarsen(_dev(phi32, torch.float32), _dev(u32, torch.float32), _dev(p32, torch.float32),
                    tuple(2 * n for n in cg), _dev(SCALE, torch.float32), out, outb)
    ref = co.coarsen(phi32.astype(np.float64), u32.astype(np.float64), p32.astype(np.float64),
                     SCALE.astype(np.float64))
    got = _coarse(out.cpu().numpy(), cg)
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()
    bits = outb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    assert np.abs(_coarse(bits.view(np.float32), cg) - got).max() <= 2 ** -8 * np.abs(got).max()
    delta = (0.1 * rng.standard_normal(got.shape)).astype(np.float32)
    dphi, du, dp = _dev(phi, torch.float64), _dev(u, torch.float64), _dev(p, torch.float64)
    sur.sur_prolong_add(_dev(delta.reshape(-1, 16), torch.float32), cg, _dev(SCALE, torch.float32),
                        dphi, du, dp)
    rphi, ru, rp = co.prolong_add(delta.astype(np.float64), SCALE.astype(np.float64), phi, u, p)
    for g, r, sc in ((dphi, rphi, 1.0), (du, ru, 0.02), (dp, rp, 4e-4)):
        assert np.abs(g.cpu().numpy() - r).max() <= 1e-6 * sc


def test_level_set_update_with_mass_restoration(sur, cg):
    import torch
    say("[coupling] prolong_update (level set) + mass fix")
    rng = np.random.default_rng(2)
    phi, u, p = _fine_fields(rng, cg)
    s0 = co.coarsen(phi, u, p, SCALE.astype(np.float64)).astype(np.float32)
    s1 = s0.copy()
    s1[..., :5] += (np.array([0.05, 0.3, 0.3, 0.3, 0.5]) * rng.standard_normal(s0[..., :5].shape)).astype(np.float32)
    dphi, du, dp = _dev(phi, torch.float64), _dev(u, torch.float64), _dev(p, torch.float64)
    scr = torch.empty(sur.sur_prolong_update_scratch_doubles(cg), dtype=torch.float64, device="cuda")
    sums = torch.empty(4, dtype=torch.float64, device="cuda")
    sur.sur_prolong_update(_dev(s0.reshape(-1, 16), torch.float32), _dev(s1.reshape(-1, 16), torch.float32),
                           cg, _dev(SCALE, torch.float32), 4.0, dphi, du, dp, scr, sums)
    rphi, ru, rp, rsums = co.prolong_update(s0.astype(np.float64), s1.astype(np.float64),
                                            SCALE.astype(np.float64), 4.0, phi, u, p)
    gphi = dphi.cpu().numpy()
    # coarse psi is taken in FP32 on the GPU: phi agrees to ~1e-6 of its range
    e = np.abs(gphi - rphi).max()
    say(f"   max|dphi| {e:.2e}")
    assert e < 2e-5
    assert np.abs(du.cpu().numpy() - ru).max() <= 1e-6 * 0.02
    assert np.abs(dp.cpu().numpy() - rp).max() <= 1e-6 * 4e-4
    g = sums.cpu().numpy()
    assert abs(g[0] - rsums[0]) <= 1e-12 * abs(rsums[0])
    assert abs(g[2] - rsums[2]) <= 1e-6 * abs(rsums[2])
    # the phase mass of the input is restored to FP64 rounding
    assert abs(gphi.sum() - phi.sum()) <= 1e-11 * phi.sum()


def test_features_and_checks(sur, cg):
    import torch
    say("[coupling] features / checks")
    rng = np.random.default_rng(3)
    s = np.zeros(cg[::-1] + (16,), dtype=np.float32)
    s[..., :5] = rng.standard_normal(s[..., :5].shape)
    s[..., 0] = rng.random(s[..., 0].shape)
    s[..., 12:] = 5.0
    ds = _dev(s.reshape(-1, 16), torch.float32)
    sur.sur_features(ds, cg)
    ref = co.features(s.astype(np.float64))
    got = _coarse(ds.cpu().numpy(), cg)
    assert np.abs(got - ref).max() <= 1e-5
    assert np.all(got[..., 12:] == 5.0)
    scr = torch.empty(7 * (np.prod(cg) // 256 + 1), dtype=torch.float64, device="cuda")
    out = torch.empty(7, dtype=torch.float64, device="cuda")
    sur.sur_checks(ds, cg, scr, out)
    c = out.cpu().numpy()
    rc = co.checks(got.astype(np.float64))
    assert c[1] == rc[1] and c[2] == rc[2] and c[5] == rc[5]
    for k in (0, 3, 4, 6):
        assert abs(c[k] - rc[k]) <= 1e-12 * abs(rc[k]), k


def test_residual_updates_and_coarse_mass_fix(sur, cg):
    import torch
    say("[coupling] apply_residual / residual_target / fix_mass")
    rng = np.random.default_rng(4)
    P = int(np.prod(cg))
    s0 = np.zeros((P, 16), dtype=np.float32)
    s0[:, :5] = rng.random((P, 5))
    out = rng.standard_normal((P, 16)).astype(np.float32)
    r = np.array([0.01, 0.2, 0.2, 0.2, 0.5] + [1.0] * 11, dtype=np.float32)
    ds = _dev(s0, torch.float32)
    sur.sur_apply_residual(ds, _dev(out, torch.float32), _dev(r, torch.float32), 5, P)
    s1 = co.apply_residual(s0.astype(np.float64), out.astype(np.float64), r.astype(np.float64))
    assert np.abs(ds.cpu().numpy() - s1).max() <= 1e-6
    t = torch.empty((P, 16), dtype=torch.float32, device="cuda")
    sur.sur_residual_target(_dev(s0, torch.float32), ds, _dev(r, torch.float32), 5, P, t)
    rt = co.residual_target(s0.astype(np.float64), ds.cpu().numpy().astype(np.float64), r.astype(np.float64))
    assert np.abs(t.cpu().numpy() - rt).max() <= 1e-4
    scr = torch.empty(7 * (P // 256 + 1), dtype=torch.float64, device="cuda")
    chk = torch.empty(7, dtype=torch.float64, device="cuda")
    sur.sur_checks(ds, cg, scr, chk)
    pre = ds.cpu().numpy().astype(np.float64).reshape(cg[::-1] + (16,))
    target = torch.tensor([float(s0[:, 0].astype(np.float64).sum())], dtype=torch.float64, device="cuda")
    sur.sur_fix_mass(ds, P, chk, target)
    got = ds.cpu().numpy()
    ref = co.fix_mass(pre, co.checks(pre), float(target.item())).reshape(P, 16)
    assert np.abs(got - ref).max() <= 1e-6
    # FP32 storage of the fixed phi: the mass is back to FP32 rounding
    assert abs(got[:, 0].astype(np.float64).sum() - target.item()) <= 1e-6 * target.item()


def test_level_set_residual_kernels(sur, cg):
    import torch
    say("[coupling] apply_residual / residual_target in level-set mode")
    rng = np.random.default_rng(5)
    P = int(np.prod(cg))
    W = 4.0
    s0 = np.zeros((P, 16), dtype=np.float32)
    s0[:, :5] = rng.random((P, 5)).astype(np.float32)
    s0[:7, 0] = [0.0, 1.0, 1e-6, 1 - 1e-6, 0.5, -0.01, 1.02]   # clamp edges
    out = (0.5 * rng.standard_normal((P, 16))).astype(np.float32)
    r = np.array([0.2, 0.2, 0.2, 0.2, 0.5] + [1.0] * 11, dtype=np.float32)
    ds = _dev(s0, torch.float32)
    sur.sur_apply_residual(ds, _dev(out, torch.float32), _dev(r, torch.float32), 5, P, W)
    ref = co.apply_residual(s0.astype(np.float64), out.astype(np.float64), r.astype(np.float64),
                            width=W)
    got = ds.cpu().numpy()
    say(f"   max|d| {np.abs(got - ref).max():.2e}")
    assert np.abs(got - ref).max() <= 2e-6
    t = torch.empty((P, 16), dtype=torch.float32, device="cuda")
    sur.sur_residual_target(_dev(s0, torch.float32), ds, _dev(r, torch.float32), 5, P, t, W)
    rt = co.residual_target(s0.astype(np.float64), got.astype(np.float64), r.astype(np.float64),
                            width=W)
    # Psi is steep near the clamp: compare where phi is away from it
    mid = (s0[:, 0] > 1e-3) & (s0[:, 0] < 1 - 1e-3) & (got[:, 0] > 1e-3) & (got[:, 0] < 1 - 1e-3)
    assert np.abs(t.cpu().numpy()[mid] - rt[mid]).max() <= 2e-4
    assert np.abs(t.cpu().numpy()[:, 1:5] - rt[:, 1:5]).max() <= 1e-4
