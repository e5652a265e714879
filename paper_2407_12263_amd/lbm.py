"""Thin Python binding of the C ABI in ``include/lbm.h`` (``liblbm.so``).

The functions here carry the C names and only marshal arguments: device
pointers and the stream come from PyTorch tensors and
``torch.cuda.current_stream()``; every step of the solver runs in the HIP
library. There is no fallback: if ``liblbm.so`` is missing or no GPU is
present, the calls raise.

:class:`Solver` is a convenience wrapper that owns the workspace tensor and
the context.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
# algorithmic HBM bytes per lattice update of the fused step (2 x 19 values
# read once and written once, plus phi_s for 16-bit storage)
BYTES_PER_LU = {"fp64": 608, "fp32": 304, "fp16": 160, "bf16": 160}
# the same on D3Q27 (2 x 27 values)
BYTES_PER_LU_Q27 = {"fp64": 864, "fp32": 432, "fp16": 224, "bf16": 224}


class LbmParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("precision", C.c_int32),
                ("wall", C.c_int32 * 3),
                ("store_log2", C.c_int32 * 2),
                ("check_every", C.c_int32),
                ("mass_fix_every", C.c_int32),
                ("normal_fd", C.c_int32),
                ("courant", C.c_double),
                ("rho1", C.c_double), ("rho2", C.c_double),
                ("tau_rho1", C.c_double), ("tau_rho2", C.c_double),
                ("tau_phi", C.c_double), ("sigma", C.c_double), ("delta", C.c_double),
                ("G", C.c_double * 3),
                ("k1_eps", C.c_double),
                ("p_ref", C.c_double),
                ("lattice", C.c_int32),
                ("wetting", C.c_int32),
                ("cos_theta", C.c_double)]


class LbmDiag(C.Structure):
    _fields_ = [("step", C.c_int64), ("sum_phi", C.c_double), ("mass", C.c_double),
                ("mom", C.c_double * 3), ("ekin", C.c_double), ("umax", C.c_double),
                ("phi_min", C.c_double), ("phi_max", C.c_double),
                ("com", C.c_double * 3), ("phiu", C.c_double * 3),
                ("l2_num", C.c_double), ("l2_den", C.c_double)]


class LbmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} (status {status})")


_lib = None


def hip_runtime_first():
    """Loads PyTorch's HIP runtime before any of this package's libraries.
    PyTorch ships its own libamdhip64 with the same soname as the system's;
    a library of ours opened first would bring in the system copy and
    PyTorch then a second one, and streams and device memory of one runtime
    are invalid in the other (lbm_init then fails with LBM_EDEVICE). Opened
    after PyTorch, our libraries bind to the runtime it already holds."""
    import torch  # noqa: F401


def load_library(path: str | None = None):
    """Loads liblbm.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FileNotFoundError(f"HIP library {p} is not built; run __graft_entry__.build()")
    hip_runtime_first()
    lib = C.CDLL(p)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    lib.lbm_lattice.argtypes = [C.POINTER(C.c_int32), dp]
    lib.lbm_lattice.restype = None
    lib.lbm_lattice_q.argtypes = [C.c_int32, C.POINTER(C.c_int32), dp]
    lib.lbm_lattice_q.restype = C.c_int
    lib.lbm_workspace_bytes.argtypes = [C.POINTER(LbmParams), C.POINTER(C.c_size_t)]
    lib.lbm_init.argtypes = [C.POINTER(LbmParams), vp, C.c_size_t, vp, vp, vp, vp,
                             C.POINTER(vp)]
    lib.lbm_step.argtypes = [vp, C.c_int64]
    lib.lbm_fields.argtypes = [vp, vp, vp, vp, C.c_int32]
    lib.lbm_diagnostics.argtypes = [vp, vp, C.POINTER(LbmDiag)]
    lib.lbm_get_pdfs.argtypes = [vp, vp, vp]
    lib.lbm_set_pdfs.argtypes = [vp, vp, vp]
    lib.lbm_reset.argtypes = [vp, vp, vp, vp, C.c_int64]
    lib.lbm_time.argtypes = [vp]
    lib.lbm_time.restype = C.c_int64
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_destroy.restype = None
    lib.lbm_strerror.argtypes = [C.c_int]
    lib.lbm_strerror.restype = C.c_char_p
    if path is None:
        _lib = lib
    return lib


def strerror(status: int) -> str:
    try:
        return load_library().lbm_strerror(int(status)).decode()
    except FileNotFoundError:
        return "unknown"


def _check(rc: int, where: str):
    if rc != LBM_OK:
        raise LbmError(rc, where)


def make_params(nx, ny, nz, precision="fp32", wall=(0, 0, 0), courant=0.997, rho1=1.0,
                rho2=1.0, tau_rho1=0.3, tau_rho2=0.3, tau_phi=0.3, sigma=0.0, delta=4.0,
                G=(0.0, 0.0, 0.0), k1_eps=1e-4, p_ref=0.0, store_log2=(10, 10),
                check_every=0, mass_fix_every=None, normal_fd=0, lattice=19, wetting=0,
                cos_theta=0.0) -> LbmParams:
    """mass_fix_every: None picks 10 for FP32 and 16-bit storage (FP32 rounding
    alone drifts the phase mass by ~1e-8 of it per step on a quasi-steady
    interface), 0 for FP64. lattice: 19 (D3Q19) or 27 (D3Q27). wetting = 1 with
    cos_theta: contact angle theta at the walls."""
    p = LbmParams()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for a in range(3):
        p.wall[a] = int(wall[a])
        p.G[a] = float(G[a])
    p.store_log2[0], p.store_log2[1] = int(store_log2[0]), int(store_log2[1])
    p.check_every = int(check_every)
    if mass_fix_every is None:
        mass_fix_every = 0 if p.precision == PRECISIONS["fp64"] else 10
    p.mass_fix_every = int(mass_fix_every)
    p.normal_fd = int(normal_fd)
    p.courant = float(courant)
    p.rho1, p.rho2 = float(rho1), float(rho2)
    p.tau_rho1, p.tau_rho2 = float(tau_rho1), float(tau_rho2)
    p.tau_phi, p.sigma, p.delta = float(tau_phi), float(sigma), float(delta)
    p.k1_eps, p.p_ref = float(k1_eps), float(p_ref)
    p.lattice = int(lattice)
    p.wetting = int(wetting)
    p.cos_theta = float(cos_theta)
    return p


# ------------------------------------------------------- C names, marshalled

def lbm_lattice():
    lib = load_library()
    e = (C.c_int32 * 57)()
    t = (C.c_double * 19)()
    lib.lbm_lattice(e, t)
    return np.array(list(e), dtype=np.int64).reshape(19, 3), np.array(list(t))


def lbm_lattice_q(q: int = 19):
    lib = load_library()
    e = (C.c_int32 * (3 * max(int(q), 1)))()
    t = (C.c_double * max(int(q), 1))()
    _check(lib.lbm_lattice_q(int(q), e, t), "lbm_lattice_q")
    return np.array(list(e), dtype=np.int64).reshape(q, 3), np.array(list(t))


def lbm_workspace_bytes(params: LbmParams) -> int:
    n = C.c_size_t()
    _check(load_library().lbm_workspace_bytes(C.byref(params), C.byref(n)), "lbm_workspace_bytes")
    return int(n.value)


def lbm_init(params: LbmParams, workspace, stream, phi0, u0=None, p0=None):
    """workspace, phi0, u0, p0: CUDA tensors (float64 fields). Returns the
    context handle (c_void_p)."""
    h = C.c_void_p()
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    rc = load_library().lbm_init(C.byref(params), ptr(workspace), workspace.numel() * workspace.element_size(),
                                 C.c_void_p(stream), ptr(phi0), ptr(u0), ptr(p0), C.byref(h))
    _check(rc, "lbm_init")
    return h


def lbm_step(ctx, n: int):
    _check(load_library().lbm_step(ctx, C.c_int64(int(n))), "lbm_step")


def lbm_fields(ctx, phi=None, u=None, p=None, dtype: int = 0):
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    _check(load_library().lbm_fields(ctx, ptr(phi), ptr(u), ptr(p), int(dtype)), "lbm_fields")


def lbm_diagnostics(ctx, phi_ref=None) -> dict:
    d = LbmDiag()
    ref = None if phi_ref is None else C.c_void_p(phi_ref.data_ptr())
    _check(load_library().lbm_diagnostics(ctx, ref, C.byref(d)), "lbm_diagnostics")
    return dict(step=int(d.step), sum_phi=d.sum_phi, mass=d.mass, mom=list(d.mom),
                ekin=d.ekin, umax=d.umax, phi_min=d.phi_min, phi_max=d.phi_max,
                com=list(d.com), phiu=list(d.phiu), l2_num=d.l2_num, l2_den=d.l2_den)


def lbm_get_pdfs(ctx, f, g):
    _check(load_library().lbm_get_pdfs(ctx, C.c_void_p(f.data_ptr()), C.c_void_p(g.data_ptr())),
           "lbm_get_pdfs")


def lbm_set_pdfs(ctx, f, g):
    _check(load_library().lbm_set_pdfs(ctx, C.c_void_p(f.data_ptr()), C.c_void_p(g.data_ptr())),
           "lbm_set_pdfs")


def lbm_reset(ctx, phi, u=None, p=None, t: int = 0):
    ptr = lambda x: None if x is None else C.c_void_p(x.data_ptr())
    _check(load_library().lbm_reset(ctx, ptr(phi), ptr(u), ptr(p), C.c_int64(int(t))), "lbm_reset")


def lbm_time(ctx) -> int:
    return int(load_library().lbm_time(ctx))


def lbm_destroy(ctx):
    load_library().lbm_destroy(ctx)


# ------------------------------------------------------------ convenience

class Solver:
    """One simulation on one GPU. ``params`` is a dict of lbm_params fields
    (see :func:`make_params`); fields are numpy or torch arrays shaped
    (nz, ny, nx) / (3, nz, ny, nx)."""

    def __init__(self, params: dict, phi0, u0=None, p0=None, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP solver needs a GPU; none is visible")
        self.torch = torch
        self.device = torch.device(device)
        self.params = make_params(**params)
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.Q = 27 if self.params.lattice == 27 else 19
        self.N = self.params.nx * self.params.ny * self.params.nz
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            nbytes = lbm_workspace_bytes(self.params)
            # 256-byte aligned: the caching allocator returns 512-byte aligned blocks
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            dev = lambda a, shp: None if a is None else torch.as_tensor(
                np.asarray(a) if not isinstance(a, torch.Tensor) else a,
                dtype=torch.float64).to(self.device).reshape(shp).contiguous()
            phi0_d = dev(phi0, self.shape)
            u0_d = dev(u0, (3,) + self.shape)
            p0_d = dev(p0, self.shape)
            self.ctx = lbm_init(self.params, self.workspace, self.stream.cuda_stream, phi0_d,
                                u0_d, p0_d)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                self.stream.synchronize()
            finally:
                lbm_destroy(ctx)
            self.ctx = None

    @property
    def t(self) -> int:
        return lbm_time(self.ctx)

    def step(self, n: int = 1):
        lbm_step(self.ctx, n)

    def fields(self, dtype=None):
        torch = self.torch
        dt = torch.float64 if dtype in (None, torch.float64) else torch.float32
        phi = torch.empty(self.shape, dtype=dt, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=dt, device=self.device)
        p = torch.empty(self.shape, dtype=dt, device=self.device)
        lbm_fields(self.ctx, phi, u, p, 0 if dt == torch.float64 else 1)
        return phi, u, p

    def diagnostics(self, phi_ref=None) -> dict:
        ref = None
        if phi_ref is not None:
            ref = self.torch.as_tensor(np.asarray(phi_ref) if not isinstance(phi_ref, self.torch.Tensor)
                                       else phi_ref, dtype=self.torch.float64).to(self.device).contiguous()
        return lbm_diagnostics(self.ctx, ref)

    def get_pdfs(self):
        torch = self.torch
        f = torch.empty((self.Q,) + self.shape, dtype=torch.float64, device=self.device)
        g = torch.empty((self.Q,) + self.shape, dtype=torch.float64, device=self.device)
        lbm_get_pdfs(self.ctx, f, g)
        return f, g

    def set_pdfs(self, f, g):
        torch = self.torch
        cv = lambda a: torch.as_tensor(np.asarray(a) if not isinstance(a, torch.Tensor) else a,
                                       dtype=torch.float64).to(self.device).reshape((self.Q,) + self.shape).contiguous()
        fd, gd = cv(f), cv(g)
        lbm_set_pdfs(self.ctx, fd, gd)
        self.stream.synchronize()

    def reset(self, phi, u=None, p=None, t=None):
        """Rebuild the state from device FP64 fields (torch tensors)."""
        torch = self.torch
        cv = lambda a, shp: None if a is None else torch.as_tensor(a, dtype=torch.float64).to(
            self.device).reshape(shp).contiguous()
        lbm_reset(self.ctx, cv(phi, self.shape), cv(u, (3,) + self.shape), cv(p, self.shape),
                  self.t if t is None else t)

    def synchronize(self):
        self.stream.synchronize()
