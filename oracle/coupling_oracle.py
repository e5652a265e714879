"""Oracle of the coupling between the LBM solver and the coarse-grid surrogate
(test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use it).

Plain NumPy in FP64 of what the transfer and check kernels compute; arrays
are (z, y, x) for fine fields and (z, y, x, 16) for coarse states:

  coarsen        2x2x2 mean of (phi, ux, uy, uz, p), divided by scale.
  prolong        cell-centred trilinear interpolation, periodic: fine node i
                 sits at coarse coordinate (i + 1/2)/2 - 1/2.
  prolong_add    fine += scale * prolong(delta).
  psi / profile  the signed distance of the equilibrium tanh profile of the
                 phase field (width W) and its inverse.
  prolong_update u, p get the prolonged change; phi moves its level set by
                 the prolonged change of psi; then the phase mass is restored.
  features       periodic central differences and products used as network
                 inputs.
  checks         the per-window check sums.
  apply_residual / residual_target / fix_mass  the state updates of a window
                 (phi's change optionally in level-set coordinates).

The paper has no learned component, so nothing here follows a passage of it
except the equilibrium profile (the tanh interface of width delta used for the
droplet tests, Sec. 3.1) that the level-set transform inverts.
"""
from __future__ import annotations

import numpy as np

NCH = 16
NUSE = 5
LS_EPS = 1e-4


def coarsen(phi, u, p, scale):
    nz, ny, nx = phi.shape
    out = np.zeros((nz // 2, ny // 2, nx // 2, NCH))
    fields = [phi, u[0], u[1], u[2], p]
    for c, f in enumerate(fields):
        m = f.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5))
        out[..., c] = m / scale[c]
    return out


def _interp_axis(c, axis):
    """Doubles one axis: fine 2I takes 3/4 of I and 1/4 of I - 1, fine 2I + 1
    takes 3/4 of I and 1/4 of I + 1 (periodic)."""
    lo = np.roll(c, 1, axis=axis)
    hi = np.roll(c, -1, axis=axis)
    even = 0.75 * c + 0.25 * lo
    odd = 0.75 * c + 0.25 * hi
    shp = list(c.shape)
    shp[axis] *= 2
    out = np.empty(shp)
    sl = [slice(None)] * c.ndim
    sl[axis] = slice(0, None, 2)
    out[tuple(sl)] = even
    sl[axis] = slice(1, None, 2)
    out[tuple(sl)] = odd
    return out


def prolong(c):
    """c: (cz, cy, cx) -> (2cz, 2cy, 2cx)."""
    out = c
    for axis in range(3):
        out = _interp_axis(out, axis)
    return out


def prolong_add(delta, scale, phi, u, p):
    phi = phi + scale[0] * prolong(delta[..., 0])
    u = np.stack([u[a] + scale[1 + a] * prolong(delta[..., 1 + a]) for a in range(3)])
    p = p + scale[4] * prolong(delta[..., 4])
    return phi, u, p


def psi(f, W):
    f = np.clip(f, LS_EPS, 1.0 - LS_EPS)
    return 0.25 * W * np.log(f / (1.0 - f))


def profile(s, W):
    return 0.5 * (1.0 + np.tanh(2.0 * s / W))


def field_sums(phi):
    return float(phi.sum()), float(np.maximum(phi * (1.0 - phi), 0.0).sum())


def prolong_update(s0, s1, scale, W, phi, u, p):
    """Returns the updated (phi, u, p) and the sums {sum phi, sum w} before
    and after the level-set move (before the mass fix)."""
    before = field_sums(phi)
    dpsi = prolong(psi(scale[0] * s1[..., 0], W) - psi(scale[0] * s0[..., 0], W))
    so = psi(phi, W)
    phi1 = phi + (profile(so + dpsi, W) - profile(so, W))
    u1 = np.stack([u[a] + scale[1 + a] * prolong(s1[..., 1 + a] - s0[..., 1 + a]) for a in range(3)])
    p1 = p + scale[4] * prolong(s1[..., 4] - s0[..., 4])
    after = field_sums(phi1)
    c = (before[0] - after[0]) / after[1] if after[1] > 0 else 0.0
    phi1 = phi1 + c * np.maximum(phi1 * (1.0 - phi1), 0.0)
    return phi1, u1, p1, before + after


def _cd(f, axis):
    """Periodic central difference along a (z, y, x) axis."""
    return 0.5 * (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis))


def features(s):
    out = s.copy()
    phi = s[..., 0]
    gx, gy, gz = _cd(phi, 2), _cd(phi, 1), _cd(phi, 0)
    out[..., 5], out[..., 6], out[..., 7] = gx, gy, gz
    out[..., 8] = s[..., 1] * gx + s[..., 2] * gy + s[..., 3] * gz
    out[..., 9] = _cd(s[..., 1], 2) + _cd(s[..., 2], 1) + _cd(s[..., 3], 0)
    out[..., 10] = phi * (1.0 - phi)
    out[..., 11] = np.sqrt(gx * gx + gy * gy + gz * gz)
    return out


def checks(s):
    phi = s[..., 0]
    div = _cd(s[..., 1], 2) + _cd(s[..., 2], 1) + _cd(s[..., 3], 0)
    return np.array([phi.sum(), phi.min(), phi.max(), (div * div).sum(),
                     (s[..., 1:4] ** 2).sum(), phi.size,
                     np.maximum(phi * (1.0 - phi), 0.0).sum()])


def apply_residual(s, out, rscale, cu=NUSE, width=0.0):
    """s + rscale * out on the first cu channels; with width > 0 channel 0
    (phi) moves in level-set coordinates: phi + Phi(Psi(phi) + d) - Phi(Psi(phi))."""
    s = s.copy()
    d = rscale[:cu] * out[..., :cu]
    if width > 0:
        phi = s[..., 0]
        so = psi(phi, width)
        s[..., 0] = phi + (profile(so + d[..., 0], width) - profile(so, width))
        s[..., 1:cu] += d[..., 1:cu]
    else:
        s[..., :cu] += d
    return s


def residual_target(s0, s1, rscale, cu=NUSE, width=0.0):
    """(s1 - s0)/rscale on the first cu channels (channel 0 as the change of
    Psi(phi) when width > 0), 0 beyond."""
    t = np.zeros_like(s0)
    t[..., :cu] = (s1[..., :cu] - s0[..., :cu]) / rscale[:cu]
    if width > 0:
        t[..., 0] = (psi(s1[..., 0], width) - psi(s0[..., 0], width)) / rscale[0]
    return t


def fix_mass(s, chk, target):
    s = s.copy()
    c = (target - chk[0]) / chk[6] if chk[6] > 0 else 0.0
    phi = s[..., 0]
    s[..., 0] = phi + c * np.maximum(phi * (1.0 - phi), 0.0)
    return s
