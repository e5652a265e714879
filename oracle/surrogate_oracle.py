"""NumPy reference of the coarse-grid U-Net surrogate (test infrastructure).

Plain definitions, channels-last arrays of shape (nz, ny, nx, C):

* conv3d: y[p, o] = b[o] + sum_t sum_i x[p + s d_t, i] w[t, o, i], 27 taps
  t = (dx+1) + 3 (dy+1) + 9 (dz+1), periodic wrap, s = +1 (s = -1 with the
  [27][cin][cout] weights gives the data gradient);
* its gradients: dw[t, o, i] = sum_p dy[p, o] x[p + d_t, i], db = sum_p dy,
  dx[q, i] = sum_t sum_o dy[q - d_t, o] w[t, o, i];
* 2x2x2 average pooling, nearest 2x upsampling, ReLU, channel concat;
* residual MSE  L = sum_p sum_c w_c (pred - target)^2 / (P n_c);
* Adam (Kingma & Ba 2015) with bias correction;
* the U-Net: per level two 3x3x3 conv + ReLU on the way down, 2x pooling,
  a bottom level, nearest upsampling, concat with the skip, two conv + ReLU,
  and a final linear 3x3x3 conv; the prediction is the residual.

Only the test-suite uses this module; it imports nothing from the GPU path.
"""
from __future__ import annotations

import numpy as np

TAPS = [((t % 3) - 1, ((t // 3) % 3) - 1, (t // 9) - 1) for t in range(27)]  # (dx, dy, dz)


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(a32.shape)


def shift(x, d, s=1):
    """x[p + s*d] for every p (periodic)."""
    dx, dy, dz = d
    return np.roll(x, shift=(-s * dz, -s * dy, -s * dx), axis=(0, 1, 2))


def conv3d(x, w, b=None, flip=False):
    """x (nz,ny,nx,I), w (27,O,I) -> (nz,ny,nx,O)."""
    s = -1 if flip else 1
    y = np.zeros(x.shape[:3] + (w.shape[1],), dtype=np.float64)
    for t, d in enumerate(TAPS):
        y += shift(x, d, s) @ w[t].T
    if b is not None:
        y += b
    return y


def conv3d_wgrad(x, dy):
    """dw (27,O,I), db (O,) of y = conv3d(x, w, b)."""
    O, I = dy.shape[-1], x.shape[-1]
    dyf = dy.reshape(-1, O)
    dw = np.zeros((27, O, I))
    for t, d in enumerate(TAPS):
        dw[t] = dyf.T @ shift(x, d).reshape(-1, I)
    return dw, dyf.sum(axis=0)


def conv3d_dgrad(dy, w):
    """dx of y = conv3d(x, w): sum_t dy[q - d_t] @ w[t]."""
    dx = np.zeros(dy.shape[:3] + (w.shape[2],))
    for t, d in enumerate(TAPS):
        dx += shift(dy, d, -1) @ w[t]
    return dx


def pool2(x):
    nz, ny, nx, c = x.shape
    return x.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).mean(axis=(1, 3, 5))


def pool2_bwd(dy):
    return up2(dy) / 8.0


def up2(x):
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def up2_bwd(dy):
    nz, ny, nx, c = dy.shape
    return dy.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2, c).sum(axis=(1, 3, 5))


def relu(x):
    return np.maximum(x, 0.0)


def mse(pred, target, wch):
    cu = len(wch)
    P = int(np.prod(pred.shape[:3]))
    d = pred[..., :cu] - target[..., :cu]
    loss = float((d * d * np.asarray(wch)).sum() / (P * cu))
    g = np.zeros_like(pred)
    g[..., :cu] = 2.0 * d * np.asarray(wch) / (P * cu)
    return loss, g


def adam(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- the U-Net

def unet_layers(channels, cin=16, cout=16):
    """(name, cin, cout, relu) of every conv, in parameter order."""
    L = []
    prev = cin
    for lv, c in enumerate(channels):
        L.append((f"enc{lv}a", prev, c, True))
        L.append((f"enc{lv}b", c, c, True))
        prev = c
    for lv in range(len(channels) - 2, -1, -1):
        c = channels[lv]
        L.append((f"dec{lv}a", prev + c, c, True))
        L.append((f"dec{lv}b", c, c, True))
        prev = c
    L.append(("out", prev, cout, False))
    return L


def unet_forward(x, params, channels, quant=None):
    """params: list of (w, b) in unet_layers order. quant: optional rounding
    applied to every stored activation (e.g. bf16_round) to mirror BF16
    storage. Returns (output, cache)."""
    q = quant or (lambda a: a)
    layers = unet_layers(channels, x.shape[-1])
    cache = {"in": x}
    k = 0
    h = x
    skips = []
    for lv in range(len(channels)):
        for part in "ab":
            w, b = params[k]
            pre = conv3d(h, w, b)
            h = q(relu(pre))
            cache[layers[k][0]] = h
            k += 1
        if lv < len(channels) - 1:
            skips.append(h)
            h = q(pool2(h))
            cache[f"pool{lv}"] = h
    for lv in range(len(channels) - 2, -1, -1):
        u = up2(h)
        h = np.concatenate([u, skips[lv]], axis=-1)
        cache[f"cat{lv}"] = h
        for part in "ab":
            w, b = params[k]
            h = q(relu(conv3d(h, w, b)))
            cache[layers[k][0]] = h
            k += 1
    w, b = params[k]
    out = conv3d(h, w, b)
    return out, cache


def unet_backward(dout, params, channels, cache):
    """Gradients (dw, db) per layer of the loss whose gradient at the output
    is dout (backprop through the graph of unet_forward)."""
    layers = unet_layers(channels, cache["in"].shape[-1])
    grads = [None] * len(layers)
    k = len(layers) - 1
    # final conv: input = last decoder activation (or bottom if one level)
    inp_name = layers[k - 1][0]
    x_in = cache[inp_name]
    w, b = params[k]
    grads[k] = conv3d_wgrad(x_in, dout)
    dh = conv3d_dgrad(dout, w)
    nlev = len(channels)
    # walk the decoder backwards
    dskip = [None] * (nlev - 1)
    for lv in range(0, nlev - 1):
        for part in "ba":
            k -= 1
            act = cache[layers[k][0]]
            dpre = dh * (act > 0)
            x_in = cache[f"cat{lv}"] if part == "a" else cache[layers[k - 1][0]]
            w, b = params[k]
            grads[k] = conv3d_wgrad(x_in, dpre)
            dh = conv3d_dgrad(dpre, w)
        cup = dh.shape[-1] - channels[lv]
        dskip[lv] = dh[..., cup:]
        dh = up2_bwd(dh[..., :cup])
    # encoder, bottom first
    for lv in range(nlev - 1, -1, -1):
        if lv < nlev - 1:
            dh = pool2_bwd(dh) + dskip[lv]
        for part in "ba":
            k -= 1
            act = cache[layers[k][0]]
            dpre = dh * (act > 0)
            if part == "b":
                x_in = cache[layers[k - 1][0]]
            else:
                x_in = cache["in"] if lv == 0 else cache[f"pool{lv - 1}"]
            w, b = params[k]
            grads[k] = conv3d_wgrad(x_in, dpre)
            dh = conv3d_dgrad(dpre, w)
    return grads
