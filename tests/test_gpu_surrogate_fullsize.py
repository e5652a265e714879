"""The surrogate's convolution kernels at the network's full sizes (the
128^3 and 64^3 levels of the coarse grid, LDS-tiled persistent kernels in
the launch configuration the network uses): the forward and the flipped,
masked data gradient on 4096 sampled output points, each computed by the
definition Y[p][o] = sum_t sum_i X[p + d_t][i] W[t][o][i] (+ b) in FP64
from the same BF16 inputs; the weight gradient in full against the oracle.
"""
import numpy as np
import pytest

from oracle import surrogate_oracle as so

from gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sur():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_12263_amd import surrogate
    surrogate.load_library()
    return surrogate


def _bits(a):
    import torch
    r = so.bf16_round(np.asarray(a, dtype=np.float32))
    return torch.as_tensor(r.view(np.uint32).__rshift__(16).astype(np.uint16).view(np.int16)).cuda()


def _f32(a):
    import torch
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).cuda()


def _sampled_conv(x, w, b, pts, flip):
    """Y at sampled points (z, y, x) by the definition (periodic), FP64."""
    nz, ny, nx, _ = x.shape
    s = -1 if flip else 1
    out = np.zeros((len(pts), w.shape[1]))
    for t, (dx, dy, dz) in enumerate(so.TAPS):
        zz = (pts[:, 0] + s * dz) % nz
        yy = (pts[:, 1] + s * dy) % ny
        xx = (pts[:, 2] + s * dx) % nx
        out += x[zz, yy, xx].astype(np.float64) @ w[t].T
    if b is not None:
        out += b
    return out


@pytest.mark.parametrize("n,cin,cout,flip", [(128, 16, 16, 0), (128, 48, 16, 0), (128, 16, 48, 1),
                                             (128, 48, 16, 1), (64, 80, 32, 0), (64, 32, 32, 1)])
def test_conv_full_size_sampled(sur, n, cin, cout, flip):
    import torch
    say(f"[sur-full] conv {n}^3 {cin}->{cout} flip={flip}: 4096 sampled points")
    rng = np.random.default_rng(n + cin + cout + flip)
    x = so.bf16_round(rng.standard_normal((n, n, n, cin)).astype(np.float32))
    w = so.bf16_round((rng.standard_normal((27, cout, cin)) * 0.1).astype(np.float32))
    b = rng.standard_normal(cout).astype(np.float32)
    wf = torch.empty((27, cout, cin), dtype=torch.int16, device="cuda")
    wd = torch.empty((27, cin, cout), dtype=torch.int16, device="cuda")
    P = n ** 3
    y = torch.empty((P, cout), dtype=torch.float32, device="cuda")
    if not flip:
        sur.sur_pack_weights(_f32(w), cin, cout, wf, None)
        sur.sur_conv3d(_bits(x.reshape(-1, cin)), cin, wf, _f32(b), cout, (n, n, n), relu=1,
                       y_f32=y)
    else:
        # the data gradient of a layer with cout -> cin: weights packed
        # transposed per tap, mask = the layer input's ReLU pattern
        wl = so.bf16_round((rng.standard_normal((27, cin, cout)) * 0.1).astype(np.float32))
        sur.sur_pack_weights(_f32(wl), cout, cin, None, wd)
        mask = so.bf16_round(np.maximum(rng.standard_normal((n, n, n, cout)), 0).astype(np.float32))
        sur.sur_conv3d(_bits(x.reshape(-1, cin)), cin, wd, None, cout, (n, n, n), flip=1,
                       mask=_bits(mask.reshape(-1, cout)), y_f32=y)
        w = np.transpose(wl, (0, 2, 1))  # Wd[t][o][i] = Wl[t][i][o]
        b = None
    pts = rng.integers(0, n, size=(4096, 3))
    ref = _sampled_conv(x, w.astype(np.float64), None if b is None else b.astype(np.float64),
                        pts, flip)
    if flip:
        ref = ref * (mask[pts[:, 0], pts[:, 1], pts[:, 2]] > 0)
    else:
        ref = np.maximum(ref, 0.0)
    got = y.cpu().numpy().reshape(n, n, n, cout)[pts[:, 0], pts[:, 1], pts[:, 2]]
    e = np.abs(got - ref).max()
    say(f"   max|dy| {e:.2e} (scale {np.abs(ref).max():.2f})")
    assert e <= 1e-5 * (1 + np.abs(ref).max())


@pytest.mark.parametrize("n,cin,cout", [(128, 16, 16), (128, 48, 16), (64, 80, 32)])
def test_conv_weight_gradient_full_size(sur, n, cin, cout):
    import torch
    say(f"[sur-full] weight gradient {n}^3 {cin}->{cout}")
    rng = np.random.default_rng(3 * n + cin + cout)
    x = so.bf16_round(rng.standard_normal((n, n, n, cin)).astype(np.float32))
    dy = so.bf16_round(rng.standard_normal((n, n, n, cout)).astype(np.float32))
    grid = (n, n, n)
    scratch = torch.empty(sur.sur_wgrad_scratch_floats(cin, cout, grid), dtype=torch.float32,
                          device="cuda")
    dw = torch.empty((27, cout, cin), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    sur.sur_conv3d_wgrad(_bits(x.reshape(-1, cin)), cin, _bits(dy.reshape(-1, cout)), cout, grid,
                         scratch, dw, db)
    rdw, rdb = so.conv3d_wgrad(x.astype(np.float64), dy.astype(np.float64))
    e = np.abs(dw.cpu().numpy() - rdw).max()
    eb = np.abs(db.cpu().numpy() - rdb).max()
    say(f"   max|ddw| {e:.2e} (scale {np.abs(rdw).max():.1f}), max|ddb| {eb:.2e}")
    # FP32 sums of n^3 BF16 products: rounding grows like sqrt(n^3)
    P = n ** 3
    assert e <= 1e-5 * (1 + np.abs(rdw).max()) * np.sqrt(P) / 64
    assert eb <= 1e-5 * (1 + np.abs(rdb).max()) * np.sqrt(P) / 64


@pytest.mark.parametrize("n,cc,fc,cout", [(128, 32, 16, 16), (64, 32, 32, 32), (64, 48, 32, 32)])
def test_conv_reading_the_concat_in_place_full_size_sampled(sur, n, cc, fc, cout, monkeypatch):
    """The decoder's first 128^3 convolution (32 upsampled channels of the
    64^3 level + 16 skip channels -> 16) reading its concat in place, and
    64^3 ones with two output tiles (weights resident, or five chunks staged
    per chunk; all on eight-wavefront blocks), on 4096
    sampled points against the definition over the concatenated input; the
    output bits equal those of the four-wavefront form (SUR_CONV_WV=4)."""
    import torch
    say(f"[sur-full] conv of the concat in place {n}^3 ({cc} up + {fc} skip) -> {cout}: 4096 points")
    rng = np.random.default_rng(77 + n + cout)
    xc = so.bf16_round(rng.standard_normal((n // 2, n // 2, n // 2, cc)).astype(np.float32))
    xf = so.bf16_round(rng.standard_normal((n, n, n, fc)).astype(np.float32))
    w = so.bf16_round((rng.standard_normal((27, cout, cc + fc)) * 0.1).astype(np.float32))
    b = rng.standard_normal(cout).astype(np.float32)
    wf = torch.empty((27, cout, cc + fc), dtype=torch.int16, device="cuda")
    sur.sur_pack_weights(_f32(w), cc + fc, cout, wf, None)
    y = torch.empty((n ** 3, cout), dtype=torch.float32, device="cuda")
    sur.sur_conv3d_cat(_bits(xc.reshape(-1, cc)), cc, _bits(xf.reshape(-1, fc)), fc, wf, _f32(b),
                       cout, (n, n, n), relu=1, y_f32=y)
    pts = rng.integers(0, n, size=(4096, 3))
    ref = np.zeros((len(pts), cout))
    for t, (dx, dy, dz) in enumerate(so.TAPS):
        zz, yy, xx = (pts[:, 0] + dz) % n, (pts[:, 1] + dy) % n, (pts[:, 2] + dx) % n
        xin = np.concatenate([xc[zz // 2, yy // 2, xx // 2], xf[zz, yy, xx]], axis=1).astype(np.float64)
        ref += xin @ w[t].astype(np.float64).T
    ref = np.maximum(ref + b, 0.0)
    got = y.cpu().numpy().reshape(n, n, n, cout)[pts[:, 0], pts[:, 1], pts[:, 2]]
    e = np.abs(got - ref).max()
    say(f"   max|dy| {e:.2e} (scale {np.abs(ref).max():.2f})")
    assert e <= 1e-5 * (1 + np.abs(ref).max())
    monkeypatch.setenv("SUR_CONV_WV", "4")
    y4 = torch.empty_like(y)
    sur.sur_conv3d_cat(_bits(xc.reshape(-1, cc)), cc, _bits(xf.reshape(-1, fc)), fc, wf, _f32(b),
                       cout, (n, n, n), relu=1, y_f32=y4)
    assert torch.equal(y, y4)


@pytest.mark.parametrize("n,cin,cout", [(128, 16, 16), (64, 32, 32), (32, 48, 48)])
def test_conv_with_pooling_full_size_sampled(sur, n, cin, cout, monkeypatch):
    """The encoders' second convolutions with their pooling in one pass (the
    128^3 and 64^3 levels on eight-wavefront blocks, the 32^3 level on the
    small grids' one-tile blocks, all pooled through LDS; the bits equal
    those of the four-wavefront two-tile form, or of the two passes for 16
    outputs): the BF16 output on 4096 sampled points against
    the definition, and the pooled output on 4096 sampled cells equal to the
    mean of the cell's eight stored BF16 values (summed x, y, z in FP32)."""
    import torch
    say(f"[sur-full] conv + pooling {n}^3 {cin}->{cout}: 4096 points and cells")
    rng = np.random.default_rng(5 * n + cin)
    x = so.bf16_round(rng.standard_normal((n, n, n, cin)).astype(np.float32))
    w = so.bf16_round((rng.standard_normal((27, cout, cin)) * 0.1).astype(np.float32))
    b = rng.standard_normal(cout).astype(np.float32)
    wf = torch.empty((27, cout, cin), dtype=torch.int16, device="cuda")
    sur.sur_pack_weights(_f32(w), cin, cout, wf, None)
    yb = torch.empty((n ** 3, cout), dtype=torch.int16, device="cuda")
    yp = torch.empty((n ** 3 // 8, cout), dtype=torch.int16, device="cuda")
    sur.sur_conv3d_pool(_bits(x.reshape(-1, cin)), cin, wf, _f32(b), cout, (n, n, n), relu=1,
                        y_bf16=yb, y_pool=yp)
    ybits = yb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    yv = ybits.view(np.float32).reshape(n, n, n, cout)
    pts = rng.integers(0, n, size=(4096, 3))
    ref = np.maximum(_sampled_conv(x, w.astype(np.float64), b.astype(np.float64), pts, False), 0.0)
    got = yv[pts[:, 0], pts[:, 1], pts[:, 2]]
    e = np.abs(got - ref).max()
    say(f"   max|dy| {e:.2e} (scale {np.abs(ref).max():.2f})")
    assert e <= 2 ** -8 * np.abs(ref).max() + 1e-5 * (1 + np.abs(ref).max())
    cells = rng.integers(0, n // 2, size=(4096, 3))
    s = np.zeros((len(cells), cout), dtype=np.float32)
    for k in range(8):
        dx, dy, dz = k & 1, (k >> 1) & 1, k >> 2
        s = s + yv[2 * cells[:, 0] + dz, 2 * cells[:, 1] + dy, 2 * cells[:, 2] + dx]
    want = so.bf16_round(np.float32(0.125) * s)
    pbits = yp.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    pv = pbits.view(np.float32).reshape(n // 2, n // 2, n // 2, cout)
    assert np.array_equal(pv[cells[:, 0], cells[:, 1], cells[:, 2]], want)
    monkeypatch.setenv("SUR_CONV_WV", "4")
    monkeypatch.setenv("SUR_CONV_SPLITN", "0")
    yb4, yp4 = torch.empty_like(yb), torch.empty_like(yp)
    sur.sur_conv3d_pool(_bits(x.reshape(-1, cin)), cin, wf, _f32(b), cout, (n, n, n), relu=1,
                        y_bf16=yb4, y_pool=yp4)
    assert torch.equal(yb, yb4) and torch.equal(yp, yp4)


@pytest.mark.parametrize("grid,cin,cout,flip", [((128, 128, 128), 16, 16, 0), ((64, 64, 64), 32, 32, 1),
                                                ((128, 64, 32), 48, 16, 0), ((64, 32, 64), 16, 48, 0)])
def test_conv_xcd_slab_order_same_bits(sur, grid, cin, cout, flip, monkeypatch):
    """On power-of-two grids with at least 8 tile rows the convolution deals
    its tiles to the XCDs in slabs of tile rows; every output bit equals
    that of the x-fastest order (SUR_CONV_XCD=0): both orders visit each
    tile once."""
    import torch
    nx, ny, nz = grid
    P = nx * ny * nz
    say(f"[sur-full] conv tile order {grid} {cin}->{cout} flip={flip}")
    rng = np.random.default_rng(nx + ny + nz + cin + cout + flip)
    x = so.bf16_round(rng.standard_normal((P, cin)).astype(np.float32))
    w = so.bf16_round((rng.standard_normal((27, cout, cin)) * 0.1).astype(np.float32))
    b = rng.standard_normal(cout).astype(np.float32)
    mask = so.bf16_round(np.maximum(rng.standard_normal((P, cout)), 0).astype(np.float32))
    wf = torch.empty((27, cout, cin), dtype=torch.int16, device="cuda")
    sur.sur_pack_weights(_f32(w), cin, cout, wf, None)
    xb, mb = _bits(x), _bits(mask)
    outs = []
    for order in (None, "0"):
        if order is not None:
            monkeypatch.setenv("SUR_CONV_XCD", order)
        y = torch.empty((P, cout), dtype=torch.float32, device="cuda")
        yb = torch.empty((P, cout), dtype=torch.int16, device="cuda")
        sur.sur_conv3d(xb, cin, wf, None if flip else _f32(b), cout, grid, flip=flip,
                       relu=0 if flip else 1, mask=mb if flip else None, y_bf16=yb, y_f32=y)
        torch.cuda.synchronize()
        outs.append((y, yb))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("grid,cin,cout,flip", [((96, 96, 64), 32, 16, 0), ((80, 96, 128), 16, 16, 1),
                                                ((128, 64, 128), 48, 16, 0), ((64, 64, 64), 32, 32, 0),
                                                ((64, 64, 64), 64, 48, 1), ((128, 64, 64), 16, 32, 0)])
def test_conv_eight_wavefront_tiles_sampled(sur, grid, cin, cout, flip):
    """Layers on large grids run eight wavefronts per block on 16 x 4 x 8
    point tiles (one output tile with at least four tiles per CU, powers of
    two or not; two output tiles where the tiles make whole rounds of the
    CUs, with up to four input chunks' weights resident): 4096 sampled
    points against the definition, and every output bit equal to the same
    layer on four-wavefront 16 x 4 x 4 tiles (SUR_CONV_WV=4)."""
    import os
    import torch
    nx, ny, nz = grid
    P = nx * ny * nz
    say(f"[sur-full] conv on 16x4x8 tiles {grid} {cin}->{cout} flip={flip}: 4096 points")
    rng = np.random.default_rng(nx + 3 * ny + 5 * nz + cin + flip)
    x = so.bf16_round(rng.standard_normal((nz, ny, nx, cin)).astype(np.float32))
    w = so.bf16_round((rng.standard_normal((27, cout, cin)) * 0.1).astype(np.float32))
    b = rng.standard_normal(cout).astype(np.float32)
    mask = so.bf16_round(np.maximum(rng.standard_normal((nz, ny, nx, cout)), 0).astype(np.float32))
    wf = torch.empty((27, cout, cin), dtype=torch.int16, device="cuda")
    sur.sur_pack_weights(_f32(w), cin, cout, wf, None)
    xb, mb = _bits(x.reshape(-1, cin)), _bits(mask.reshape(-1, cout))
    outs = []
    old = os.environ.get("SUR_CONV_WV")
    try:
        for wv in (None, "4"):
            if wv is None:
                os.environ.pop("SUR_CONV_WV", None)
            else:
                os.environ["SUR_CONV_WV"] = wv
            y = torch.empty((P, cout), dtype=torch.float32, device="cuda")
            yb = torch.empty((P, cout), dtype=torch.int16, device="cuda")
            sur.sur_conv3d(xb, cin, wf, None if flip else _f32(b), cout, grid, flip=flip,
                           relu=0 if flip else 1, mask=mb if flip else None, y_bf16=yb, y_f32=y)
            outs.append((y.cpu().numpy(), yb.cpu().numpy()))
    finally:
        if old is None:
            os.environ.pop("SUR_CONV_WV", None)
        else:
            os.environ["SUR_CONV_WV"] = old
    pts = np.stack([rng.integers(0, nz, 4096), rng.integers(0, ny, 4096), rng.integers(0, nx, 4096)], 1)
    ref = _sampled_conv(x, w.astype(np.float64), None if flip else b.astype(np.float64), pts, flip)
    ref = ref * (mask[pts[:, 0], pts[:, 1], pts[:, 2]] > 0) if flip else np.maximum(ref, 0.0)
    got = outs[0][0].reshape(nz, ny, nx, cout)[pts[:, 0], pts[:, 1], pts[:, 2]]
    e = np.abs(got - ref).max()
    say(f"   max|dy| {e:.2e} (scale {np.abs(ref).max():.2f})")
    assert e <= 1e-5 * (1 + np.abs(ref).max())
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
