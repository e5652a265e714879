"""Seeded synthetic workloads: initial fields and parameter sets.

This module holds no arithmetic of the method itself. It builds the initial
order parameter, velocity and pressure of the paper's test problems
(Sec. 3) at the sizes the benchmarks and tests use, and states each
workload's parameters as plain numbers in the solver's convention:
grid units (dx = dt = 1), discrete velocities c*e^_i with the Courant
number c, relaxation times tau as in the paper (relaxation rate
1/(tau + 1/2), nu = tau*c^2/3, M = tau_phi*c^2/3).

Both the GPU library's tests and the oracle's tests take their inputs from
here, so both sides see bit-identical inputs.

Arrays: numpy float64 with shape (nz, ny, nx) for scalars and
(3, nz, ny, nx) for vectors (x fastest in memory).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

COURANT = 0.997  # the paper's fixed Courant number (Sec. 2.2)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    wall: tuple = (0, 0, 0)      # per axis: 1 = no-slip walls on both faces
    courant: float = COURANT
    rho1: float = 1.0            # density of the phi = 1 phase
    rho2: float = 1.0            # density of the phi = 0 phase
    tau_rho1: float = 0.3
    tau_rho2: float = 0.3
    tau_phi: float = 0.3
    sigma: float = 0.0
    delta: float = 4.0
    G: tuple = (0.0, 0.0, 0.0)
    k1_eps: float = 1e-4         # normal set to 0 where |K1| <= k1_eps
    steps: int = 100
    phi0: np.ndarray = field(default=None, repr=False)
    u0: np.ndarray = field(default=None, repr=False)
    p0: np.ndarray = field(default=None, repr=False)
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    def params(self) -> dict:
        """Solver parameters as a plain dict (no fields)."""
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, wall=tuple(self.wall),
                    courant=self.courant, rho1=self.rho1, rho2=self.rho2,
                    tau_rho1=self.tau_rho1, tau_rho2=self.tau_rho2, tau_phi=self.tau_phi,
                    sigma=self.sigma, delta=self.delta, G=tuple(self.G), k1_eps=self.k1_eps)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def cs2_of(courant: float) -> float:
    """Squared lattice sound speed for velocities c*e^_i (unit conversion only)."""
    return courant * courant / 3.0


def tau_from_mobility(M: float, courant: float = COURANT) -> float:
    return M / cs2_of(courant)


def tau_from_kinematic(nu: float, courant: float = COURANT) -> float:
    return nu / cs2_of(courant)


# ---------------------------------------------------------------- geometry

def _grid(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def _min_image(d, n, periodic):
    if periodic:
        return d - n * np.round(d / n)
    return d


def sphere_distance(shape, center, wall=(0, 0, 0)):
    """Distance to ``center`` (x, y, z), minimum image along periodic axes."""
    nz, ny, nx = shape
    x, y, z = _grid(shape)
    dx = _min_image(x - center[0], nx, not wall[0])
    dy = _min_image(y - center[1], ny, not wall[1])
    dz = _min_image(z - center[2], nz, not wall[2])
    return np.sqrt(dx * dx + dy * dy + dz * dz)


def tanh_drop(r, R, W):
    """Equilibrium profile of a dispersed phase (phi = 1 inside), Sec. 3.1."""
    return 0.5 * (1.0 - np.tanh(2.0 * (r - R) / W))


# -------------------------------------------------------------- workloads

def static_droplet(n: int = 32, R: float = 8.0, W: float = 4.0, sigma: float = 1e-3,
                   tau_bgk: float = 0.8, M: float = 0.02, courant: float = COURANT,
                   steps: int = 500, ny: int | None = None, nz: int | None = None,
                   center=None) -> Workload:
    """Static droplet in a periodic box (Sec. 3.1; 3D form).

    tau_bgk is a BGK relaxation time (relaxation rate 1/tau_bgk), so the
    paper's tau_rho = tau_bgk - 1/2; the mobility M fixes tau_phi.
    """
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    shape = (nz, ny, n)
    if center is None:
        center = (n / 2, ny / 2, nz / 2)
    r = sphere_distance(shape, center)
    phi0 = tanh_drop(r, R, W)
    tau = tau_bgk - 0.5
    return Workload(name=f"static_droplet_{n}x{ny}x{nz}", nx=n, ny=ny, nz=nz, courant=courant,
                    rho1=1.0, rho2=1.0, tau_rho1=tau, tau_rho2=tau,
                    tau_phi=tau_from_mobility(M, courant), sigma=sigma, delta=W, steps=steps,
                    phi0=phi0, u0=np.zeros((3,) + shape), p0=np.zeros(shape),
                    meta=dict(R=R, W=W, center=center))


def droplet_2d(L0: int = 100, Cn: float = 0.06, La: float = 1.0, tau_rho: float = 0.02,
               M: float = 0.02, courant: float = COURANT) -> Workload:
    """Static droplet in 2D (Sec. 3.1: the convergence study): diameter
    D = L0/2 in a periodic L0 x L0 box, interface width delta = Cn D,
    rho1 = rho2 = 1, equal viscosities from tau_rho, sigma from
    La = sigma rho D / eta, t0 = eta D / (2 sigma). The lattice is D3Q19 on a
    single z-plane (nz = 1, periodic): the z-moving populations stay in the
    plane and the projected weights are those of D2Q9 (4/9, 1/9, 1/36).
    The floor on the normal is 1e-5 (3/W)^2: the droplet has no walls or
    body force, so K1 carries no non-gradient part for the floor to remove
    beyond rounding noise, and below the floor the profile's tail diffuses
    without sharpening. |K1| of a profile falls as 1/W, so a fixed floor
    would cut a band of the profile that widens with the resolution, an
    error that does not shrink and puts a floor under a convergence study;
    falling as W^-2, the band narrows faster than the O(W^2) error does."""
    cs2 = cs2_of(courant)
    D = L0 / 2.0
    W = Cn * D
    eta = tau_rho * cs2
    sigma = La * eta / D
    shape = (1, L0, L0)
    r = sphere_distance(shape, (L0 / 2.0, L0 / 2.0, 0.0))
    phi0 = tanh_drop(r, D / 2.0, W)
    return Workload(name=f"droplet_2d_{L0}", nx=L0, ny=L0, nz=1, courant=courant,
                    rho1=1.0, rho2=1.0, tau_rho1=tau_rho, tau_rho2=tau_rho,
                    tau_phi=tau_from_mobility(M, courant), sigma=sigma, delta=W,
                    k1_eps=1e-5 * (3.0 / W) ** 2, steps=0, phi0=phi0, u0=np.zeros((3,) + shape), p0=np.zeros(shape),
                    meta=dict(D=D, W=W, t0=eta * D / (2.0 * sigma), sigma=sigma, eta=eta))


def rayleigh_taylor(nx: int = 128, ny: int = 512, nz: int = 128, W: float = 4.0,
                    Re: float = 256.0, U: float = 0.04, sigma: float = 5e-5,
                    M: float = 0.02, amp_frac: float = 0.05, courant: float = COURANT,
                    steps: int = 20000, mode3d: bool = False) -> Workload:
    """Rayleigh-Taylor instability (Sec. 3.2 in 3D): heavy phase (phi = 1,
    rho1 = 1) on top of a light one (rho2 = 1/3, At = 0.5), equal dynamic
    viscosities, no-slip walls at the bottom and top (y), periodic in x, z.
    Velocity scale U = sqrt(g Lx) sets g; Re = rho1 U Lx / eta sets eta.
    """
    shape = (nz, ny, nx)
    x, y, z = _grid(shape)
    amp = amp_frac * nx
    yi = ny / 2.0 + amp * np.cos(2.0 * math.pi * x / nx)
    if mode3d:
        yi = ny / 2.0 + amp * np.cos(2.0 * math.pi * x / nx) * np.cos(2.0 * math.pi * z / nz)
    phi0 = 0.5 * (1.0 + np.tanh(2.0 * (y - yi) / W))
    rho1, rho2 = 1.0, 1.0 / 3.0
    g = U * U / nx
    eta = rho1 * U * nx / Re
    cs2 = cs2_of(courant)
    return Workload(name=f"rayleigh_taylor_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, wall=(0, 1, 0),
                    courant=courant, rho1=rho1, rho2=rho2,
                    tau_rho1=eta / (rho1 * cs2), tau_rho2=eta / (rho2 * cs2),
                    tau_phi=tau_from_mobility(M, courant), sigma=sigma, delta=W,
                    G=(0.0, -g, 0.0), steps=steps, phi0=phi0,
                    u0=np.zeros((3,) + shape), p0=np.zeros(shape),
                    meta=dict(g=g, eta=eta, t0=math.sqrt(2.0 * nx / g), At=0.5, Re=Re))


def rising_bubble(nx: int = 128, ny: int = 128, nz: int = 256, R: float = 16.0,
                  zc: float = 48.0, W: float = 4.0, g: float = 2e-6, Eo: float = 10.0,
                  Mo: float = 1e-3, M: float = 0.02, courant: float = COURANT,
                  steps: int = 30000) -> Workload:
    """Single rising bubble (Sec. 3.3 in 3D): bubble phase phi = 1 with
    rho1 = 0.1 in a liquid rho2 = 1, equal kinematic viscosities (viscosity
    ratio 10), walls on all faces, gravity along -z. Eo = drho g D^2/sigma
    fixes sigma; Mo = g eta_l^4 drho/(rho_l^2 sigma^3) fixes eta_l."""
    shape = (nz, ny, nx)
    rho_l, rho_g = 1.0, 0.1
    drho = rho_l - rho_g
    D = 2.0 * R
    sigma = drho * g * D * D / Eo
    eta_l = (Mo * rho_l ** 2 * sigma ** 3 / (g * drho)) ** 0.25
    nu = eta_l / rho_l
    tau = tau_from_kinematic(nu, courant)
    r = sphere_distance(shape, (nx / 2.0, ny / 2.0, zc), wall=(1, 1, 1))
    phi0 = tanh_drop(r, R, W)
    return Workload(name=f"rising_bubble_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, wall=(1, 1, 1),
                    courant=courant, rho1=rho_g, rho2=rho_l, tau_rho1=tau, tau_rho2=tau,
                    tau_phi=tau_from_mobility(M, courant), sigma=sigma, delta=W,
                    G=(0.0, 0.0, -g), steps=steps, phi0=phi0,
                    u0=np.zeros((3,) + shape), p0=np.zeros(shape),
                    meta=dict(R=R, zc=zc, eta_l=eta_l, Eo=Eo, Mo=Mo))


def taylor_green_fields(shape, u0: float, rho0: float = 1.0, p_ref: float = 0.0):
    """3D Taylor-Green cell with period = box (Sec. 3.4): u, v, w, p."""
    nz, ny, nx = shape
    x, y, z = _grid(shape)
    kx, ky, kz = 2 * math.pi / nx, 2 * math.pi / ny, 2 * math.pi / nz
    u = u0 * np.sin(kx * x) * np.cos(ky * y) * np.cos(kz * z)
    v = -u0 * np.cos(kx * x) * np.sin(ky * y) * np.cos(kz * z)
    w = np.zeros(shape)
    p = p_ref + rho0 * u0 * u0 / 16.0 * (np.cos(2 * kx * x) + np.cos(2 * ky * y)) * \
        (np.cos(2 * kz * z) + 2.0)
    return np.stack([u, v, w]), p


def taylor_green_breakup(n: int = 256, R: float | None = None, u0: float = 0.04,
                         sigma: float = 2e-4, W: float = 4.0, tau_bgk: float = 0.55,
                         M: float = 0.02, courant: float = COURANT,
                         steps: int = 40000) -> Workload:
    """Bubble breakup in a decaying Taylor-Green vortex (Sec. 3.4): periodic
    cube, density ratio 1, bubble of radius R (n/8 by default) at the centre."""
    shape = (n, n, n)
    R = n / 8.0 if R is None else R
    r = sphere_distance(shape, (n / 2.0, n / 2.0, n / 2.0))
    phi0 = tanh_drop(r, R, W)
    u, p = taylor_green_fields(shape, u0)
    tau = tau_bgk - 0.5
    return Workload(name=f"taylor_green_{n}", nx=n, ny=n, nz=n, courant=courant,
                    rho1=1.0, rho2=1.0, tau_rho1=tau, tau_rho2=tau,
                    tau_phi=tau_from_mobility(M, courant), sigma=sigma, delta=W, steps=steps,
                    phi0=phi0, u0=u, p0=p, meta=dict(R=R, u0=u0))


def random_solenoidal(shape, kmax: float = 4.0, rms: float = 0.02, seed: int = 0):
    """Random divergence-free velocity from integer wavevectors 1 <= |k| <= kmax:
    complex Gaussian amplitudes (drawn for those modes only) projected
    perpendicular to k; the field is the real part of the inverse FFT (the
    Hermitian part of the spectrum), rescaled to the given rms."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    K = int(math.floor(kmax))
    ks = np.arange(-K, K + 1)
    kz, ky, kx = [a.ravel() for a in np.meshgrid(ks, ks, ks, indexing="ij")]
    k2 = kx * kx + ky * ky + kz * kz
    keep = (k2 >= 1) & (k2 <= kmax * kmax)
    kv = np.stack([kx[keep], ky[keep], kz[keep]]).astype(float)
    m = kv.shape[1]
    amp = rng.standard_normal((3, m)) + 1j * rng.standard_normal((3, m))
    amp -= kv * (kv * amp).sum(0) / (kv * kv).sum(0)
    # inverse DFT restricted to the few nonzero wavenumbers per axis, one axis
    # at a time: u(x) = (1/N) sum_k amp(k) exp(2 pi i k.x / n)
    E = [np.exp(2j * np.pi * np.outer(ks, np.arange(L)) / L) for L in (nx, ny, nz)]
    u = np.empty((3,) + shape)
    for a in range(3):
        B = np.zeros((2 * K + 1,) * 3, dtype=complex)
        np.add.at(B, (kv[2].astype(int) + K, kv[1].astype(int) + K, kv[0].astype(int) + K), amp[a])
        T = np.einsum("abk,kx->abx", B, E[0])                 # (kz, ky, x)
        T = np.einsum("ky,akx->ayx", E[1], T)                 # (kz, y, x)
        T = T.reshape(2 * K + 1, ny * nx)
        u[a] = ((E[2].real.T @ T.real) - (E[2].imag.T @ T.imag)).reshape(shape) / (nx * ny * nz)
    cur = math.sqrt(float(np.mean(np.sum(u * u, axis=0))))
    if cur > 0:
        u *= rms / cur
    return u


def emulsion(n: int = 256, n_drops: int = 200, rmin: float = 6.0, rmax: float = 16.0,
             W: float = 4.0, seed: int = 1, rms: float = 0.02, sigma: float = 2e-4,
             tau_rho: float = 0.05, M: float = 0.02, courant: float = COURANT,
             max_tries: int = 200000) -> Workload:
    """Emulsion: n_drops non-overlapping droplets (radii uniform in
    [rmin, rmax], minimum-image gap >= r_a + r_b + 2W, rejection sampling)
    in a periodic cube plus a random solenoidal velocity (rms ``rms``).
    phi is the maximum of the droplets' tanh profiles; each profile is
    evaluated in a periodic box reaching 7W beyond its radius, where it has
    fallen below 1e-12."""
    shape = (n, n, n)
    rng = np.random.default_rng(seed)
    centres, radii = [], []
    tries = 0
    while len(centres) < n_drops and tries < max_tries:
        tries += 1
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0.0, n, size=3)
        if centres:
            d = np.asarray(centres) - c
            d -= n * np.round(d / n)
            if (np.sqrt((d * d).sum(1)) < r + np.asarray(radii) + 2.0 * W).any():
                continue
        centres.append(c)
        radii.append(r)
    # profiles are written into a padded copy with plain slices, then the
    # padding is folded back periodically (max over the periodic images)
    H = int(math.ceil(rmax + 7.0 * W)) + 1
    if 2 * H >= n:
        phi0 = np.zeros(shape)
        for c, r in zip(centres, radii):
            np.maximum(phi0, tanh_drop(sphere_distance(shape, tuple(c)), r, W), out=phi0)
    else:
        P = np.zeros((n + 2 * H,) * 3)
        for c, r in zip(centres, radii):
            h = int(math.ceil(r + 7.0 * W))
            lo = [int(math.floor(c[a])) - h for a in range(3)]
            ax = [np.arange(lo[a], lo[a] + 2 * h + 2) - c[a] for a in range(3)]
            d = np.sqrt(ax[0][None, None, :] ** 2 + ax[1][None, :, None] ** 2
                        + ax[2][:, None, None] ** 2)
            sl = tuple(slice(lo[a] + H, lo[a] + H + 2 * h + 2) for a in (2, 1, 0))
            np.maximum(P[sl], tanh_drop(d, r, W), out=P[sl])
        for axis in range(3):
            core = [slice(None)] * 3
            left = [slice(None)] * 3
            right = [slice(None)] * 3
            core[axis] = slice(H, H + n)
            left[axis] = slice(0, H)
            right[axis] = slice(H + n, n + 2 * H)
            c_lo = list(core)
            c_lo[axis] = slice(H + n - H, H + n)
            c_hi = list(core)
            c_hi[axis] = slice(H, 2 * H)
            np.maximum(P[tuple(c_lo)], P[tuple(left)], out=P[tuple(c_lo)])
            np.maximum(P[tuple(c_hi)], P[tuple(right)], out=P[tuple(c_hi)])
            P = P[tuple(core)]
        phi0 = np.ascontiguousarray(P)
    u0 = random_solenoidal(shape, rms=rms, seed=seed + 7919)
    return Workload(name=f"emulsion_{n}_seed{seed}", nx=n, ny=n, nz=n, courant=courant,
                    rho1=1.0, rho2=1.0, tau_rho1=tau_rho, tau_rho2=tau_rho,
                    tau_phi=tau_from_mobility(M, courant), sigma=sigma, delta=W,
                    steps=16, phi0=phi0, u0=u0, p0=np.zeros(shape),
                    meta=dict(centres=np.array(centres), radii=np.array(radii), seed=seed))
