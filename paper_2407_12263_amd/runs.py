"""The paper's three-dimensional test problems run over their configured
horizons on one GPU, with the observables each is judged by (Sec. 3):

* Rayleigh-Taylor (Sec. 3.2): the fronts of the phi = 1/2 contour where the
  heavy phase falls (spike, x = Lx/2) and the light phase rises (bubble,
  x = 0), the phase mass, and how far FP16 storage departs from FP32;
* the rising bubble (Sec. 3.3): the centroid C_m = sum phi z / sum phi and
  the rise velocity V_d = sum phi u_z / sum phi of the bubble phase, the
  mass sum rho phi (not an invariant: with the bubble's rho1 = 0.1 it is
  0.1 sum phi + 0.9 sum phi (1 - phi), and the interface term changes as
  the bubble deforms) and the drift of sum phi, which is conserved;
* bubble breakup in a Taylor-Green vortex (Sec. 3.4): the number of
  fragments (6-connected regions of phi > 1/2, the box periodic), the
  kinetic energy sum rho |u|^2 / 2 and sum phi.

Every step is the library's (lbm_step); this module sequences the runs and
reads diagnostics and fields back at the reporting times. The fragment
count labels the phase field on the host.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs, lbm


def fragments(phi: np.ndarray, periodic=(True, True, True), level: float = 0.5) -> int:
    """Number of 6-connected regions of phi > level in a (nz, ny, nx) field;
    along a periodic axis the first and last layers are neighbours.
    periodic is given as (x, y, z)."""
    return len(fragment_sizes(phi, periodic, level))


def fragment_sizes(phi: np.ndarray, periodic=(True, True, True), level: float = 0.5) -> np.ndarray:
    """Node counts of the fragments of fragments(), largest first."""
    from scipy import ndimage
    lab, n = ndimage.label(phi > level)
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    parent = np.arange(n + 1)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for flag, axis in zip(periodic, (2, 1, 0)):
        if not flag:
            continue
        a = np.take(lab, 0, axis=axis).ravel()
        b = np.take(lab, -1, axis=axis).ravel()
        both = (a > 0) & (b > 0)
        for u, v in set(zip(a[both].tolist(), b[both].tolist())):
            ru, rv = find(u), find(v)
            if ru != rv:
                parent[max(ru, rv)] = min(ru, rv)
    counts = np.bincount(lab.ravel(), minlength=n + 1)
    size = {}
    for k in range(1, n + 1):
        rk = find(k)
        size[rk] = size.get(rk, 0) + int(counts[k])
    return np.array(sorted(size.values(), reverse=True), dtype=np.int64)


def _crossing(col: np.ndarray, from_top: bool, level: float = 0.5) -> float:
    """Position (in node units, linear interpolation) where a column leaves
    the phase it starts in: from the top down to the first node below level
    (the spike front), or from the bottom up to the first node above it (the
    bubble front); nan if the column never crosses."""
    n = len(col)
    col = np.asarray(col, dtype=np.float64)
    if from_top:
        for y in range(n - 1, 0, -1):
            if col[y] >= level > col[y - 1]:
                return float(y - (col[y] - level) / (col[y] - col[y - 1]))
    else:
        for y in range(n - 1):
            if col[y] < level <= col[y + 1]:
                return float(y + (level - col[y]) / (col[y + 1] - col[y]))
    return float("nan")


def rayleigh_taylor(steps: int = 20000, every: int = 1000, precisions=("fp16", "fp32"),
                    log=print, **kw) -> dict:
    w = inputs.rayleigh_taylor(**kw)
    t0 = w.meta["t0"]
    out = dict(workload=w.name, grid=[w.nx, w.ny, w.nz], steps=steps, t0_steps=t0, runs={})
    final = {}
    for prec in precisions:
        sol = lbm.Solver(dict(w.params(), precision=prec), w.phi0, w.u0, w.p0)
        m0 = float(w.phi0.sum())
        rec = []
        tw = time.perf_counter()
        while sol.t < steps:
            sol.step(min(every, steps - sol.t))
            phi = sol.fields(dtype=sol.torch.float32)[0][0].cpu().numpy()   # plane z = 0
            d = sol.diagnostics()
            rec.append(dict(t=sol.t, t_over_t0=sol.t / t0,
                            spike_y=_crossing(phi[:, w.nx // 2], True),
                            bubble_y=_crossing(phi[:, 0], False),
                            sum_phi_drift=(d["sum_phi"] - m0) / m0, umax=float(d["umax"])))
        final[prec] = sol.fields()[0].cpu().numpy()
        out["runs"][prec] = dict(seconds=time.perf_counter() - tw, series=rec)
        log(f"[runs] {w.name} {prec}: spike y {rec[-1]['spike_y']:.2f}, bubble y "
            f"{rec[-1]['bubble_y']:.2f} at t/t0 = {rec[-1]['t_over_t0']:.2f}, drift "
            f"{rec[-1]['sum_phi_drift']:.2e}")
        del sol
    if "fp16" in final and "fp32" in final:
        out["fp16_vs_fp32_max_dphi"] = float(np.abs(final["fp16"] - final["fp32"]).max())
        out["fp16_vs_fp32_l2"] = float(np.sqrt(((final["fp16"] - final["fp32"]) ** 2).sum()
                                               / (final["fp32"] ** 2).sum()))
    return out


def rising_bubble(steps: int = 30000, every: int = 1000, precisions=("fp16", "fp32"),
                  log=print, **kw) -> dict:
    w = inputs.rising_bubble(**kw)
    out = dict(workload=w.name, grid=[w.nx, w.ny, w.nz], steps=steps, runs={})
    for prec in precisions:
        sol = lbm.Solver(dict(w.params(), precision=prec), w.phi0, w.u0, w.p0)
        d0 = sol.diagnostics()
        rec = []
        tw = time.perf_counter()
        while sol.t < steps:
            sol.step(min(every, steps - sol.t))
            d = sol.diagnostics()
            rec.append(dict(t=sol.t, centroid_z=d["com"][2] / d["sum_phi"],
                            rise_velocity=d["phiu"][2] / d["sum_phi"],
                            mass=d["mass"], mass_drift=(d["mass"] - d0["mass"]) / d0["mass"],
                            sum_phi_drift=(d["sum_phi"] - d0["sum_phi"]) / d0["sum_phi"]))
        out["runs"][prec] = dict(seconds=time.perf_counter() - tw, series=rec)
        log(f"[runs] {w.name} {prec}: C_m {rec[-1]['centroid_z']:.2f}, V_d "
            f"{rec[-1]['rise_velocity']:.3e}, mass drift {rec[-1]['mass_drift']:.2e}")
        del sol
    return out


def taylor_green(steps: int = 40000, every: int = 4000, precisions=("fp16", "fp32"),
                 log=print, **kw) -> dict:
    w = inputs.taylor_green_breakup(**kw)
    out = dict(workload=w.name, grid=[w.nx, w.ny, w.nz], steps=steps, runs={})
    for prec in precisions:
        sol = lbm.Solver(dict(w.params(), precision=prec), w.phi0, w.u0, w.p0)
        d0 = sol.diagnostics()
        # a fragment counts as resolved from the volume of a droplet one
        # interface width across
        vmin = math.pi / 6.0 * w.delta ** 3

        def frag(phi):
            sz = fragment_sizes(phi)
            return dict(fragments=len(sz), fragments_resolved=int((sz >= vmin).sum()),
                        largest_fraction=float(sz[0] / sz.sum()) if len(sz) else 0.0)

        rec = [dict(t=0, ekin=d0["ekin"], sum_phi_drift=0.0, **frag(w.phi0))]
        tw = time.perf_counter()
        while sol.t < steps:
            sol.step(min(every, steps - sol.t))
            d = sol.diagnostics()
            phi = sol.fields(dtype=sol.torch.float32)[0].cpu().numpy()
            rec.append(dict(t=sol.t, ekin=d["ekin"],
                            sum_phi_drift=(d["sum_phi"] - d0["sum_phi"]) / d0["sum_phi"],
                            **frag(phi)))
        out["runs"][prec] = dict(seconds=time.perf_counter() - tw, series=rec)
        log(f"[runs] {w.name} {prec}: fragments {[r['fragments'] for r in rec]}, resolved "
            f"{[r['fragments_resolved'] for r in rec]}, E_k "
            f"{rec[0]['ekin']:.3e} -> {rec[-1]['ekin']:.3e}, drift {rec[-1]['sum_phi_drift']:.2e}")
        del sol
    return out


def horizons(log=print) -> dict:
    """All three problems at their configured sizes and horizons."""
    return dict(rayleigh_taylor=rayleigh_taylor(log=log), rising_bubble=rising_bubble(log=log),
                taylor_green=taylor_green(log=log))


if __name__ == "__main__":
    import json
    import sys
    print(json.dumps(horizons(log=lambda *a: print(*a, file=sys.stderr, flush=True))), flush=True)
