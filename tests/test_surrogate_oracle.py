"""Pins of the NumPy surrogate oracle: definitions checked against brute-force
loops, adjoint identities, central finite differences of the whole U-Net in
FP64, and the closed-form first Adam step."""
import numpy as np
import pytest

from oracle import surrogate_oracle as so


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_conv_matches_brute_force_loops():
    rng = _rng(1)
    nz, ny, nx, I, O = 3, 4, 5, 2, 3
    x = rng.standard_normal((nz, ny, nx, I))
    w = rng.standard_normal((27, O, I))
    b = rng.standard_normal(O)
    y = so.conv3d(x, w, b)
    ref = np.zeros((nz, ny, nx, O))
    for z in range(nz):
        for yy in range(ny):
            for xx in range(nx):
                acc = b.copy()
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            t = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)
                            v = x[(z + dz) % nz, (yy + dy) % ny, (xx + dx) % nx]
                            acc += w[t] @ v
                ref[z, yy, xx] = acc
    assert np.abs(y - ref).max() < 1e-12


def test_conv_delta_kernel_is_identity_and_linear():
    rng = _rng(2)
    x = rng.standard_normal((4, 4, 4, 3))
    w = np.zeros((27, 3, 3))
    w[13] = np.eye(3)
    assert np.abs(so.conv3d(x, w) - x).max() == 0.0
    w = rng.standard_normal((27, 2, 3))
    x2 = rng.standard_normal(x.shape)
    lhs = so.conv3d(2.0 * x - 3.0 * x2, w)
    rhs = 2.0 * so.conv3d(x, w) - 3.0 * so.conv3d(x2, w)
    assert np.abs(lhs - rhs).max() < 1e-12


def test_conv_gradients_are_adjoints():
    rng = _rng(3)
    x = rng.standard_normal((4, 6, 4, 3))
    w = rng.standard_normal((27, 5, 3))
    dy = rng.standard_normal((4, 6, 4, 5))
    y = so.conv3d(x, w)
    dx = so.conv3d_dgrad(dy, w)
    dw, db = so.conv3d_wgrad(x, dy)
    ip = float((y * dy).sum())
    assert abs(ip - float((x * dx).sum())) < 1e-10 * abs(ip)
    assert abs(ip - float((w * dw).sum())) < 1e-10 * abs(ip)
    assert np.abs(db - dy.reshape(-1, 5).sum(0)).max() < 1e-12
    # data gradient = flipped conv with the per-tap transposed weights
    wd = np.transpose(w, (0, 2, 1))
    assert np.abs(so.conv3d(dy, wd, flip=True) - dx).max() < 1e-12


def test_pool_and_upsample_adjoints():
    rng = _rng(4)
    x = rng.standard_normal((4, 6, 8, 2))
    yc = rng.standard_normal((2, 3, 4, 2))
    assert abs(float((so.pool2(x) * yc).sum()) - float((x * so.pool2_bwd(yc)).sum())) < 1e-12
    yf = rng.standard_normal(x.shape)
    assert abs(float((so.up2(yc) * yf).sum()) - float((yc * so.up2_bwd(yf)).sum())) < 1e-12
    assert np.abs(so.pool2(so.up2(yc)) - yc).max() < 1e-15


@pytest.mark.parametrize("ch,n", [((4, 6), 4), ((2, 3, 4, 5), 8)])
def test_unet_gradient_by_finite_differences(ch, n):
    """U-Net in FP64, two levels (channels 4, 6) on 4^3 and four levels (the
    product's depth; channels 2, 3, 4, 5) on 8^3, whose coarsest level is a
    single point: every sampled weight and bias gradient of every layer
    agrees with a central finite difference of the loss."""
    rng = _rng(5)
    layers = so.unet_layers(ch, cin=3, cout=3)
    assert len(layers) == 4 * len(ch) - 1
    params = [(0.3 * rng.standard_normal((27, o, i)), 0.1 * rng.standard_normal(o))
              for _, i, o, _ in layers]
    x = rng.standard_normal((n, n, n, 3))
    tgt = rng.standard_normal((n, n, n, 3))
    wch = [1.0, 0.5, 2.0]

    def loss_of(params):
        out, _ = so.unet_forward(x, params, ch)
        return so.mse(out, tgt, wch)[0]

    out, cache = so.unet_forward(x, params, ch)
    _, dout = so.mse(out, tgt, wch)
    grads = so.unet_backward(dout, params, ch, cache)
    h = 1e-6
    worst = 0.0
    for k, (w, b) in enumerate(params):
        for idx in [(0, 0, 0), (13, w.shape[1] - 1, w.shape[2] - 1), (26, 0, w.shape[2] // 2)]:
            wp = [(ww.copy(), bb.copy()) for ww, bb in params]
            wm = [(ww.copy(), bb.copy()) for ww, bb in params]
            wp[k][0][idx] += h
            wm[k][0][idx] -= h
            fd = (loss_of(wp) - loss_of(wm)) / (2 * h)
            an = grads[k][0][idx]
            worst = max(worst, abs(fd - an) / max(1e-8, abs(fd) + abs(an)))
        bp = [(ww.copy(), bb.copy()) for ww, bb in params]
        bm = [(ww.copy(), bb.copy()) for ww, bb in params]
        bp[k][1][0] += h
        bm[k][1][0] -= h
        fd = (loss_of(bp) - loss_of(bm)) / (2 * h)
        worst = max(worst, abs(fd - grads[k][1][0]) / max(1e-8, abs(fd) + abs(grads[k][1][0])))
    assert worst < 1e-6, worst


def test_adam_first_step_is_signed_learning_rate():
    rng = _rng(6)
    g = rng.standard_normal(100)
    w0 = rng.standard_normal(100)
    w1, m, v = so.adam(w0, np.zeros(100), np.zeros(100), g, t=1, lr=1e-2, eps=1e-12)
    assert np.abs((w1 - w0) + 1e-2 * np.sign(g)).max() < 1e-10


def test_adam_bias_correction_over_three_steps():
    """Kingma & Ba's bias correction in closed form: with a constant gradient
    g the corrected moments are g and g^2 at every t, so each of the first
    three steps moves w by -lr sign(g) (without the correction, or with it
    at a fixed t, steps 2 and 3 differ); with g then -g the second step is
    +lr (1 - b1)/(1 + b1) sign(g), since m_2/(1 - b1^2) = -(1 - b1)/(1 + b1) g
    and v_2/(1 - b2^2) = g^2."""
    rng = _rng(7)
    g = rng.standard_normal(50)
    w0 = rng.standard_normal(50)
    lr, b1, b2 = 1e-2, 0.9, 0.999
    w, m, v = w0, np.zeros(50), np.zeros(50)
    for t in (1, 2, 3):
        w1, m, v = so.adam(w, m, v, g, t=t, lr=lr, b1=b1, b2=b2, eps=1e-14)
        assert np.abs((w1 - w) + lr * np.sign(g)).max() < 1e-11, t
        w = w1
    assert np.abs(w - (w0 - 3 * lr * np.sign(g))).max() < 1e-11
    w1, m, v = so.adam(w0, np.zeros(50), np.zeros(50), g, t=1, lr=lr, b1=b1, b2=b2, eps=1e-14)
    w2, m, v = so.adam(w1, m, v, -g, t=2, lr=lr, b1=b1, b2=b2, eps=1e-14)
    assert np.abs((w2 - w1) - lr * (1 - b1) / (1 + b1) * np.sign(g)).max() < 1e-11


def test_bf16_rounding_ties_to_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5, 0.0],
                    dtype=np.float32)
    r = so.bf16_round(vals)
    assert r.tolist() == [1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.5, 0.0]
