"""The surrogate's HIP kernels (through the sur_* C ABI) against the NumPy
oracle on identical BF16-rounded inputs: convolution forward, data and weight
gradients, pooling/upsampling/concat, loss, Adam, and the whole U-Net
forward and backward."""
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
    """float array -> BF16 bit pattern (int16 torch tensor on the GPU)."""
    import torch
    r = so.bf16_round(np.asarray(a, dtype=np.float32))
    return torch.as_tensor(r.view(np.uint32).__rshift__(16).astype(np.uint16).view(np.int16)).cuda()


def _from_bits(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32)


def _f32(a):
    import torch
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(1e-30, np.linalg.norm(np.ravel(b))))


GRID = (10, 6, 8)  # nx, ny, nz -> P = 480 (not a multiple of 256)
# grids of the convolution's two kernels: sizes not multiples of its 16 x 4 x 4
# tile (the general kernel), 2 x 2 x 2 tiles, and one tile whose halo wraps
# onto itself (the LDS-tiled kernel)
CONV_GRIDS = [GRID, (32, 8, 8), (16, 4, 4)]


@pytest.mark.parametrize("grid", CONV_GRIDS)
@pytest.mark.parametrize("cin,cout,relu", [(16, 16, 1), (32, 48, 0), (112, 48, 1), (80, 32, 1),
                                           (48, 64, 0), (48, 112, 1)])
def test_conv_forward(sur, cin, cout, relu, grid):
    import torch
    say(f"[sur] conv fwd cin={cin} cout={cout} relu={relu} grid={grid}")
    rng = np.random.default_rng(cin + cout)
    nx, ny, nz = grid
    x = so.bf16_round(rng.standard_normal((nz, ny, nx, cin)).astype(np.float32))
    w = rng.standard_normal((27, cout, cin)).astype(np.float32) * 0.1
    b = rng.standard_normal(cout).astype(np.float32)
    wf = torch.empty((27, cout, cin), dtype=torch.int16, device="cuda")
    sur.sur_pack_weights(_f32(w), cin, cout, wf, None)
    yf = torch.empty((nx * ny * nz, cout), dtype=torch.float32, device="cuda")
    yb = torch.empty((nx * ny * nz, cout), dtype=torch.int16, device="cuda")
    sur.sur_conv3d(_bits(x.reshape(-1, cin)), cin, wf, _f32(b), cout, grid, relu=relu,
                   y_bf16=yb, y_f32=yf)
    ref = so.conv3d(x.astype(np.float64), so.bf16_round(w).astype(np.float64), b.astype(np.float64))
    if relu:
        ref = so.relu(ref)
    got = yf.cpu().numpy().reshape(ref.shape)
    assert np.abs(got - ref).max() <= 1e-5 * (1 + np.abs(ref).max())
    gb = _from_bits(yb).reshape(ref.shape)
    assert np.array_equal(gb, so.bf16_round(got.astype(np.float32)))


@pytest.mark.parametrize("grid", CONV_GRIDS)
@pytest.mark.parametrize("cin,cout", [(16, 32), (112, 48), (48, 16)])
def test_conv_data_gradient_with_mask(sur, cin, cout, grid):
    import torch
    say(f"[sur] conv dgrad cin={cin} cout={cout} grid={grid}")
    rng = np.random.default_rng(7 + cin)
    nx, ny, nz = grid
    dy = so.bf16_round(rng.standard_normal((nz, ny, nx, cout)).astype(np.float32))
    w = rng.standard_normal((27, cout, cin)).astype(np.float32) * 0.1
    act = so.bf16_round(np.maximum(rng.standard_normal((nz, ny, nx, cin)), 0).astype(np.float32))
    wd = torch.empty((27, cin, cout), dtype=torch.int16, device="cuda")
    sur.sur_pack_weights(_f32(w), cin, cout, None, wd)
    dx = torch.empty((nx * ny * nz, cin), dtype=torch.float32, device="cuda")
    sur.sur_conv3d(_bits(dy.reshape(-1, cout)), cout, wd, None, cin, grid, flip=1,
                   mask=_bits(act.reshape(-1, cin)), y_f32=dx)
    ref = so.conv3d_dgrad(dy.astype(np.float64), so.bf16_round(w).astype(np.float64)) * (act > 0)
    got = dx.cpu().numpy().reshape(ref.shape)
    assert np.abs(got - ref).max() <= 1e-5 * (1 + np.abs(ref).max())


# fine grids of the in-place concat: power-of-two sizes, others (the general
# index path), one tile whose halo wraps onto itself
CAT_GRIDS = [(32, 8, 8), (48, 12, 8), (16, 4, 4)]


@pytest.mark.parametrize("grid", CAT_GRIDS)
@pytest.mark.parametrize("cc,fc,cout,relu", [(32, 16, 16, 1), (64, 48, 48, 1), (48, 32, 32, 0),
                                             (16, 16, 64, 1)])
def test_conv_reading_the_concat_in_place(sur, cc, fc, cout, relu, grid):
    """sur_conv3d_cat = the convolution of [up2(xc), xf]: within 1e-5 of the
    oracle's, and bitwise the concat pass followed by sur_conv3d."""
    import torch
    say(f"[sur] conv of the concat in place cc={cc} fc={fc} cout={cout} grid={grid}")
    rng = np.random.default_rng(cc + 3 * fc + cout)
    nx, ny, nz = grid
    P = nx * ny * nz
    cin = cc + fc
    xc = so.bf16_round(rng.standard_normal((nz // 2, ny // 2, nx // 2, cc)).astype(np.float32))
    xf = so.bf16_round(rng.standard_normal((nz, ny, nx, fc)).astype(np.float32))
    w = rng.standard_normal((27, cout, cin)).astype(np.float32) * 0.1
    b = rng.standard_normal(cout).astype(np.float32)
    wf = torch.empty((27, cout, cin), dtype=torch.int16, device="cuda")
    sur.sur_pack_weights(_f32(w), cin, cout, wf, None)
    xcb, xfb, bb = _bits(xc.reshape(-1, cc)), _bits(xf.reshape(-1, fc)), _f32(b)
    yf = torch.empty((P, cout), dtype=torch.float32, device="cuda")
    yb = torch.empty((P, cout), dtype=torch.int16, device="cuda")
    sur.sur_conv3d_cat(xcb, cc, xfb, fc, wf, bb, cout, grid, relu=relu, y_bf16=yb, y_f32=yf)
    cat = np.concatenate([so.up2(xc.astype(np.float64)), xf.astype(np.float64)], axis=-1)
    ref = so.conv3d(cat, so.bf16_round(w).astype(np.float64), b.astype(np.float64))
    if relu:
        ref = so.relu(ref)
    got = yf.cpu().numpy().reshape(ref.shape)
    assert np.abs(got - ref).max() <= 1e-5 * (1 + np.abs(ref).max())
    # the two-pass form on the GPU gives the same bits
    catb = torch.empty((P, cin), dtype=torch.int16, device="cuda")
    sur.sur_concat_up2(xcb, cc, xfb, fc, grid, catb)
    yf2 = torch.empty_like(yf)
    yb2 = torch.empty_like(yb)
    sur.sur_conv3d(catb, cin, wf, bb, cout, grid, relu=relu, y_bf16=yb2, y_f32=yf2)
    assert torch.equal(yf, yf2) and torch.equal(yb, yb2)


# forms of the small grids' layers: one-tile blocks with the weights
# prefetched (the default), two-tile blocks with and without the prefetch
SMALL_FORMS = {"one-tile": {}, "two-tile": {"SUR_CONV_SPLITN": "0"},
               "two-tile-staged": {"SUR_CONV_SPLITN": "0", "SUR_CONV_WPF": "0"}}


@pytest.mark.parametrize("form", list(SMALL_FORMS))
@pytest.mark.parametrize("grid", CAT_GRIDS + [(64, 16, 12)])
@pytest.mark.parametrize("cin,cout", [(16, 16), (32, 32), (48, 48), (16, 64), (64, 16)])
def test_conv_with_pooling_in_the_same_pass(sur, cin, cout, grid, form, monkeypatch):
    """sur_conv3d_pool = sur_conv3d then sur_pool2, bitwise, and the pooled
    output within BF16 rounding of the oracle's pool2 of the BF16 output;
    in every form of the small grids' layers."""
    import torch
    for k, v in SMALL_FORMS[form].items():
        monkeypatch.setenv(k, v)
    say(f"[sur] conv + pooling in one pass cin={cin} cout={cout} grid={grid} form={form}")
    rng = np.random.default_rng(cin * 7 + cout)
    nx, ny, nz = grid
    P = nx * ny * nz
    x = so.bf16_round(rng.standard_normal((nz, ny, nx, cin)).astype(np.float32))
    w = rng.standard_normal((27, cout, cin)).astype(np.float32) * 0.1
    b = rng.standard_normal(cout).astype(np.float32)
    wf = torch.empty((27, cout, cin), dtype=torch.int16, device="cuda")
    sur.sur_pack_weights(_f32(w), cin, cout, wf, None)
    xb, bb = _bits(x.reshape(-1, cin)), _f32(b)
    yb = torch.empty((P, cout), dtype=torch.int16, device="cuda")
    yp = torch.empty((P // 8, cout), dtype=torch.int16, device="cuda")
    sur.sur_conv3d_pool(xb, cin, wf, bb, cout, grid, relu=1, y_bf16=yb, y_pool=yp)
    yb2 = torch.empty_like(yb)
    yp2 = torch.empty_like(yp)
    sur.sur_conv3d(xb, cin, wf, bb, cout, grid, relu=1, y_bf16=yb2)
    sur.sur_pool2(yb2, cout, grid, yp2)
    assert torch.equal(yb, yb2) and torch.equal(yp, yp2)
    ref = so.pool2(_from_bits(yb).reshape(nz, ny, nx, cout).astype(np.float64))
    got = _from_bits(yp).reshape(ref.shape)
    assert np.abs(got - ref).max() <= 2 ** -8 * (np.abs(ref).max() + 1e-30)


@pytest.mark.parametrize("cin,cout,grid,flip", [(32, 48, (32, 32, 32), 0), (112, 48, (32, 32, 32), 0),
                                                (48, 48, (32, 32, 32), 1), (64, 64, (16, 16, 16), 0),
                                                (64, 48, (16, 16, 16), 1), (48, 32, (48, 16, 12), 1)])
def test_conv_small_grid_forms_agree(sur, cin, cout, grid, flip, monkeypatch):
    """The small grids' one-tile form gives the bits of the two-tile forms
    (with and without the weight prefetch), forward and flipped with mask;
    all within 1e-5 of the oracle's convolution."""
    import torch
    say(f"[sur] small-grid forms cin={cin} cout={cout} grid={grid} flip={flip}")
    rng = np.random.default_rng(cin + 5 * cout + flip)
    nx, ny, nz = grid
    P = nx * ny * nz
    x = so.bf16_round(rng.standard_normal((nz, ny, nx, cin)).astype(np.float32))
    w = so.bf16_round((rng.standard_normal((27, cout, cin)) * 0.1).astype(np.float32))
    b = rng.standard_normal(cout).astype(np.float32)
    mask = so.bf16_round(np.maximum(rng.standard_normal((nz, ny, nx, cout)), 0).astype(np.float32))
    wf = torch.empty((27, cout, cin), dtype=torch.int16, device="cuda")
    sur.sur_pack_weights(_f32(w), cin, cout, wf, None)
    xb, mb = _bits(x.reshape(-1, cin)), _bits(mask.reshape(-1, cout))
    outs = {}
    for form, env in SMALL_FORMS.items():
        for k in ("SUR_CONV_SPLITN", "SUR_CONV_WPF"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        y = torch.empty((P, cout), dtype=torch.float32, device="cuda")
        yb = torch.empty((P, cout), dtype=torch.int16, device="cuda")
        sur.sur_conv3d(xb, cin, wf, None if flip else _f32(b), cout, grid, flip=flip,
                       relu=0 if flip else 1, mask=mb if flip else None, y_bf16=yb, y_f32=y)
        outs[form] = (y.cpu().numpy(), yb.cpu().numpy())
    for form in SMALL_FORMS:
        assert np.array_equal(outs[form][0], outs["one-tile"][0]), form
        assert np.array_equal(outs[form][1], outs["one-tile"][1]), form
    wt = w.astype(np.float64)
    if flip:
        ref = so.conv3d(x.astype(np.float64), wt, None, flip=True) * (mask > 0)
    else:
        ref = so.relu(so.conv3d(x.astype(np.float64), wt, b.astype(np.float64)))
    got = outs["one-tile"][0].reshape(ref.shape)
    assert np.abs(got - ref).max() <= 1e-5 * (1 + np.abs(ref).max())


def test_conv_cat_rejects_grids_off_its_tile(sur):
    """Sizes that are not multiples of the 16 x 4 x 4 tile are refused on the
    host by the concat and pooling forms (the caller takes two passes)."""
    import torch
    grid = (8, 8, 8)
    xc = torch.zeros((64, 32), dtype=torch.int16, device="cuda")
    xf = torch.zeros((512, 16), dtype=torch.int16, device="cuda")
    wf = torch.zeros((27, 16, 48), dtype=torch.int16, device="cuda")
    yb = torch.empty((512, 16), dtype=torch.int16, device="cuda")
    assert not sur.conv_cat_fits(grid)
    with pytest.raises(RuntimeError):
        sur.sur_conv3d_cat(xc, 32, xf, 16, wf, None, 16, grid, y_bf16=yb)
    yp = torch.empty((64, 16), dtype=torch.int16, device="cuda")
    w16 = torch.zeros((27, 16, 16), dtype=torch.int16, device="cuda")
    with pytest.raises(RuntimeError):
        sur.sur_conv3d_pool(xf, 16, w16, None, 16, grid, y_bf16=yb, y_pool=yp)


def test_unet_inference_forward_equals_training_forward(sur):
    """The forward that reads the decoder concats in place gives the bits of
    the one that writes them (the training step's); a backward after the
    former is refused."""
    import torch
    say("[sur] unet 32^3 forward, concat in place vs written")
    net = sur.UNet((32, 32, 32), channels=(16, 32, 48, 64), seed=9)
    g = torch.Generator(device="cuda").manual_seed(1)
    x = torch.randint(0, 1 << 14, (32 ** 3, 16), dtype=torch.int16, device="cuda", generator=g)
    a = net.forward(x).clone()
    with pytest.raises(RuntimeError):
        net.backward(net.dout)
    b = net.forward(x, keep_cat=True).clone()
    assert torch.equal(a, b)


# the first seven grids are multiples of the 16 x 4 x 4 tile (the LDS-tiled
# kernel, one to 48 tiles, every output-channel count; the two with 8 tile
# rows and a multiple of 8 blocks deal the tiles to the XCDs in slabs of
# rows, one of them with 3 tiles in x), the rest are not
@pytest.mark.parametrize("cin,cout,grid", [(16, 16, (16, 8, 12)), (112, 48, (32, 8, 8)),
                                           (48, 64, (16, 4, 4)), (80, 32, (16, 8, 4)),
                                           (32, 16, (48, 4, 8)), (16, 16, (48, 32, 8)),
                                           (48, 16, (16, 64, 8)),
                                           (112, 48, (8, 8, 8)), (48, 64, (10, 6, 8)),
                                           (80, 32, (4, 4, 4))])
def test_conv_weight_gradient(sur, cin, cout, grid):
    import torch
    say(f"[sur] conv wgrad cin={cin} cout={cout} grid={grid}")
    rng = np.random.default_rng(11 + cout)
    nx, ny, nz = grid
    P = nx * ny * nz
    x = so.bf16_round(rng.standard_normal((nz, ny, nx, cin)).astype(np.float32))
    dy = so.bf16_round(rng.standard_normal((nz, ny, nx, cout)).astype(np.float32))
    scratch = torch.empty(sur.sur_wgrad_scratch_floats(cin, cout, grid), dtype=torch.float32,
                          device="cuda")
    dw = torch.empty((27, cout, cin), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    sur.sur_conv3d_wgrad(_bits(x.reshape(-1, cin)), cin, _bits(dy.reshape(-1, cout)), cout, grid,
                         scratch, dw, db)
    rdw, rdb = so.conv3d_wgrad(x.astype(np.float64), dy.astype(np.float64))
    assert np.abs(dw.cpu().numpy() - rdw).max() <= 1e-5 * (1 + np.abs(rdw).max()) * np.sqrt(P)
    assert np.abs(db.cpu().numpy() - rdb).max() <= 1e-5 * (1 + np.abs(rdb).max()) * np.sqrt(P)


@pytest.mark.parametrize("c", [16, 12, 6])  # 16-byte (c % 8 == 0), 4-channel (c % 4 == 0), per element
def test_grid_layers(sur, c):
    import torch
    say(f"[sur] pool / upsample / concat / masks, {c} channels")
    rng = np.random.default_rng(3)
    nx, ny, nz = 8, 4, 6
    P = nx * ny * nz
    cs = 3 * c  # concat stride; pieces at offsets 0 and c
    x = so.bf16_round(rng.standard_normal((nz, ny, nx, c)).astype(np.float32))
    y = torch.empty((P // 8, c), dtype=torch.int16, device="cuda")
    sur.sur_pool2(_bits(x.reshape(-1, c)), c, (nx, ny, nz), y)
    assert np.abs(_from_bits(y).reshape(nz // 2, ny // 2, nx // 2, c)
                  - so.bf16_round(so.pool2(x).astype(np.float32))).max() == 0.0
    xc = so.bf16_round(rng.standard_normal((nz // 2, ny // 2, nx // 2, c)).astype(np.float32))
    cat = torch.zeros((P, cs), dtype=torch.int16, device="cuda")
    sur.sur_upsample2(_bits(xc.reshape(-1, c)), c, (nx // 2, ny // 2, nz // 2), cat, cs, 0)
    sur.sur_copy_channels(_bits(x.reshape(-1, c)), c, P, cat, cs, c)
    got = _from_bits(cat).reshape(nz, ny, nx, cs)
    assert np.array_equal(got[..., :c], so.up2(xc))
    assert np.array_equal(got[..., c:2 * c], x)
    assert not got[..., 2 * c:].any()
    # the decoder's concat in one pass equals the two passes
    cat2 = torch.empty((P, 2 * c), dtype=torch.int16, device="cuda")
    sur.sur_concat_up2(_bits(xc.reshape(-1, c)), c, _bits(x.reshape(-1, c)), c, (nx, ny, nz), cat2)
    got2 = _from_bits(cat2).reshape(nz, ny, nx, 2 * c)
    assert np.array_equal(got2[..., :c], so.up2(xc))
    assert np.array_equal(got2[..., c:], x)
    dy = rng.standard_normal((P, cs)).astype(np.float32)
    du = torch.empty((P // 8, c), dtype=torch.float32, device="cuda")
    sur.sur_upsample2_bwd(_f32(dy), cs, c, c, (nx // 2, ny // 2, nz // 2), du)
    ref = so.up2_bwd(dy.reshape(nz, ny, nx, cs)[..., c:2 * c].astype(np.float64))
    assert np.abs(du.cpu().numpy().reshape(ref.shape) - ref).max() < 1e-5
    dx = torch.zeros((P, c), dtype=torch.float32, device="cuda")
    sur.sur_pool2_bwd(_f32(dy[:P // 8, :c]), c, (nx, ny, nz), dx)
    ref = so.pool2_bwd(dy[:P // 8, :c].reshape(nz // 2, ny // 2, nx // 2, c).astype(np.float64))
    assert np.abs(dx.cpu().numpy().reshape(ref.shape) - ref).max() < 1e-6
    g = _f32(dy[:, :c])
    sur.sur_relu_mask(g, _bits(x.reshape(-1, c)))
    assert np.array_equal(g.cpu().numpy(), dy[:, :c] * (x.reshape(-1, c) > 0))
    # the fused encoder gradient: pooled path + skip columns c .. 2c of dy,
    # through the ReLU of x; bitwise the same as the four separate passes
    fused = torch.empty((P, c), dtype=torch.float32, device="cuda")
    fused_b = torch.empty((P, c), dtype=torch.int16, device="cuda")
    sur.sur_pool2_bwd_skip(_f32(dy[:P // 8, :c]), c, (nx, ny, nz), _f32(dy), cs, c,
                           _bits(x.reshape(-1, c)), dx=fused, dx_bf16=fused_b)
    sep = torch.zeros((P, c), dtype=torch.float32, device="cuda")
    sur.sur_pool2_bwd(_f32(dy[:P // 8, :c]), c, (nx, ny, nz), sep)
    sur.sur_add_channels(_f32(dy), cs, c, c, P, sep)
    sur.sur_relu_mask(sep, _bits(x.reshape(-1, c)))
    assert np.array_equal(fused.cpu().numpy(), sep.cpu().numpy())
    ref = (so.pool2_bwd(dy[:P // 8, :c].reshape(nz // 2, ny // 2, nx // 2, c).astype(np.float64))
           .reshape(P, c) + dy[:, c:2 * c]) * (x.reshape(-1, c) > 0)
    assert np.abs(fused.cpu().numpy() - ref).max() < 1e-6
    sb = torch.empty((P, c), dtype=torch.int16, device="cuda")
    sur.sur_to_bf16(sep, sb)
    assert torch.equal(fused_b, sb)
    # upsampling backward through the coarse ReLU, into BF16: the same as
    # upsample2_bwd, relu_mask and to_bf16 in turn
    actc = xc.reshape(-1, c)
    um = torch.empty((P // 8, c), dtype=torch.int16, device="cuda")
    sur.sur_upsample2_bwd_mask(_f32(dy), cs, c, c, (nx // 2, ny // 2, nz // 2), _bits(actc), um)
    us = torch.empty((P // 8, c), dtype=torch.float32, device="cuda")
    sur.sur_upsample2_bwd(_f32(dy), cs, c, c, (nx // 2, ny // 2, nz // 2), us)
    sur.sur_relu_mask(us, _bits(actc))
    ub = torch.empty((P // 8, c), dtype=torch.int16, device="cuda")
    sur.sur_to_bf16(us, ub)
    assert torch.equal(um, ub)


def test_loss_and_adam(sur):
    import torch
    say("[sur] mse and adam")
    rng = np.random.default_rng(9)
    P = 700
    pred = rng.standard_normal((P, 16)).astype(np.float32)
    tgt = rng.standard_normal((P, 16)).astype(np.float32)
    wch = np.array([4.0, 1.0, 1.0, 1.0, 0.5], dtype=np.float32)
    grad = torch.empty((P, 16), dtype=torch.float32, device="cuda")
    scratch = torch.empty(P // 256 + 2, dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    sur.sur_mse(_f32(pred), _f32(tgt), 5, 16, P, _f32(wch), grad, scratch, loss)
    rl, rg = so.mse(pred.reshape(P, 1, 1, 16).astype(np.float64),
                    tgt.reshape(P, 1, 1, 16).astype(np.float64), wch.astype(np.float64))
    assert abs(float(loss.item()) - rl) < 1e-6 * rl
    assert np.abs(grad.cpu().numpy() - rg.reshape(P, 16)).max() < 1e-7
    # the BF16 gradient is the rounding of the FP32 one (both outputs at once)
    gb = torch.empty((P, 16), dtype=torch.int16, device="cuda")
    sur.sur_mse(_f32(pred), _f32(tgt), 5, 16, P, _f32(wch), grad, scratch, loss, grad_bf16=gb)
    gr = torch.empty((P, 16), dtype=torch.int16, device="cuda")
    sur.sur_to_bf16(grad, gr)
    assert torch.equal(gb, gr)
    w0 = rng.standard_normal(1000).astype(np.float32)
    g = rng.standard_normal(1000).astype(np.float32)
    w, m, v = _f32(w0), torch.zeros(1000, device="cuda"), torch.zeros(1000, device="cuda")
    ref = (w0.astype(np.float64), np.zeros(1000), np.zeros(1000))
    for t in range(1, 4):
        sur.sur_adam(w, m, v, _f32(g * t), 1e-2, 0.9, 0.999, 1e-8, t)
        ref = so.adam(ref[0], ref[1], ref[2], (g * t).astype(np.float64), t, lr=1e-2)
    assert np.abs(w.cpu().numpy() - ref[0]).max() < 1e-6


def test_unet_forward_backward_matches_oracle(sur):
    """4-level U-Net (16-32-48-64) on a 16^3 coarse grid: output and every
    layer's weight gradient agree with the oracle run on the same BF16
    rounding of inputs, weights and stored activations."""
    import torch
    say("[sur] unet 16^3 forward/backward")
    rng = np.random.default_rng(21)
    grid = (16, 16, 16)
    net = sur.UNet(grid, channels=(16, 32, 48, 64), seed=3)
    params = net.get_params()
    qparams = [(so.bf16_round(w.astype(np.float32)).astype(np.float64), b) for w, b in params]
    x = np.zeros((16, 16, 16, 16), dtype=np.float32)
    x[..., :5] = rng.standard_normal((16, 16, 16, 5))
    x = so.bf16_round(x)
    tgt = np.zeros_like(x)
    tgt[..., :5] = 0.1 * rng.standard_normal((16, 16, 16, 5))
    wch = np.array([1.0, 1.0, 1.0, 1.0, 1.0], dtype=np.float32)
    out = net.forward(_bits(x.reshape(-1, 16)), keep_cat=True)
    loss = net.loss_and_grad(_f32(tgt.reshape(-1, 16)), _f32(wch))
    net.backward(net.dout)
    torch.cuda.synchronize()
    q = lambda a: so.bf16_round(a.astype(np.float32)).astype(np.float64)
    rout, cache = so.unet_forward(x.astype(np.float64), qparams, (16, 32, 48, 64), quant=q)
    rl, rdout = so.mse(rout, tgt.astype(np.float64), wch.astype(np.float64))
    rgrads = so.unet_backward(rdout, qparams, (16, 32, 48, 64), cache)
    e_out = _rel(out.cpu().numpy(), rout.reshape(-1, 16))
    say(f"   output rel err {e_out:.2e}, loss {float(loss.item()):.6e} vs {rl:.6e}")
    assert e_out < 1e-2
    assert abs(float(loss.item()) - rl) < 2e-2 * rl
    worst = 0.0
    for k, (gw, gb) in enumerate(rgrads):
        ew = _rel(net.gw[k].cpu().numpy(), gw)
        worst = max(worst, ew)
    say(f"   worst layer weight-gradient rel err {worst:.2e}")
    assert worst < 2e-2


def test_training_trajectory_matches_oracle(sur):
    """60 Adam steps of the 4-level U-Net on an 8^3 grid (smooth input, target
    half the one-cell shift of the input): the GPU loss curve follows the
    oracle's (same initial weights, BF16 rounding of weights and activations
    emulated in the oracle's forward pass) and falls by more than 20x."""
    from scipy.ndimage import gaussian_filter
    say("[sur] training trajectory 8^3 vs oracle")
    ch = (16, 32, 48, 64)
    n = 8
    rng = np.random.default_rng(5)
    x = np.zeros((n, n, n, 16))
    for c in range(5):
        x[..., c] = 3.0 * gaussian_filter(rng.standard_normal((n, n, n)), 1.0, mode="wrap")
    x = so.bf16_round(x.astype(np.float32)).astype(np.float64)
    tgt = np.zeros_like(x)
    tgt[..., :5] = 0.5 * (np.roll(x[..., :5], 1, axis=2) - x[..., :5])
    net = sur.UNet((n, n, n), channels=ch, seed=4)
    params = net.get_params()
    xb, tg, wch = _bits(x.reshape(-1, 16)), _f32(tgt.reshape(-1, 16)), _f32(np.ones(5))
    lr, steps = 1e-3, 60
    q = lambda a: so.bf16_round(a.astype(np.float32)).astype(np.float64)
    st = [(np.zeros_like(w), np.zeros_like(w), np.zeros_like(b), np.zeros_like(b)) for w, b in params]
    gpu, ref = [], []
    for t in range(1, steps + 1):
        gpu.append(float(net.train_step(xb, tg, wch, lr=lr).item()))
        qp = [(q(w), b) for w, b in params]
        out, cache = so.unet_forward(x, qp, ch, quant=q)
        loss, dout = so.mse(out, tgt, np.ones(5))
        grads = so.unet_backward(dout, qp, ch, cache)
        ref.append(loss)
        new_p, new_s = [], []
        for (w, b), (gw, gb), (mw, vw, mb, vb) in zip(params, grads, st):
            w, mw, vw = so.adam(w, mw, vw, gw, t, lr=lr)
            b, mb, vb = so.adam(b, mb, vb, gb, t, lr=lr)
            new_p.append((w, b))
            new_s.append((mw, vw, mb, vb))
        params, st = new_p, new_s
    gpu, ref = np.array(gpu), np.array(ref)
    say("   step   gpu loss    oracle loss")
    for t in (0, 9, 19, 39, 59):
        say(f"   {t + 1:4d}  {gpu[t]:.5e}  {ref[t]:.5e}")
    # same weights at step 1: the losses agree to BF16 forward rounding
    assert abs(gpu[0] - ref[0]) < 1e-4 * ref[0]
    # later steps: the GPU's BF16 gradients (not emulated in the oracle)
    # slow the descent a little; the curves stay within a factor 1.6
    assert np.all(np.abs(np.log(gpu / ref)) < np.log(1.6))
    assert ref[-1] < 0.05 * ref[0] and gpu[-1] < 0.05 * gpu[0]


def test_pack_weights_all_equals_per_layer(sur):
    """One packing launch over several layers (weights at offsets of a flat
    buffer) writes the same BF16 packings as one launch per layer."""
    import torch
    say("[sur] packing of three layers in one launch")
    rng = np.random.default_rng(5)
    shapes = [(16, 16), (48, 16), (32, 64)]  # (cin, cout)
    w_off, off = [], 0
    for ci, co in shapes:
        w_off.append(off)
        off += 27 * ci * co + co  # a bias after each layer's weights
    flat = _f32(rng.standard_normal(off).astype(np.float32))
    n = sum(27 * ci * co for ci, co in shapes)
    wf = torch.empty(n, dtype=torch.int16, device="cuda")
    wd = torch.empty(n, dtype=torch.int16, device="cuda")
    sur.sur_pack_weights_all(flat, w_off, [ci for ci, _ in shapes], [co for _, co in shapes], wf, wd)
    p = 0
    for (ci, co), o in zip(shapes, w_off):
        m = 27 * ci * co
        f1 = torch.empty((27, co, ci), dtype=torch.int16, device="cuda")
        d1 = torch.empty((27, ci, co), dtype=torch.int16, device="cuda")
        sur.sur_pack_weights(flat[o:o + m].view(27, co, ci), ci, co, f1, d1)
        assert torch.equal(wf[p:p + m], f1.view(-1))
        assert torch.equal(wd[p:p + m], d1.view(-1))
        p += m
