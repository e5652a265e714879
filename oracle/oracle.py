"""ctypes binding of the C oracle (test infrastructure, see package docstring).

Arrays are numpy float64, structure-of-arrays with x fastest:
scalar fields have shape (nz, ny, nx), vector fields (3, nz, ny, nx) and
PDF fields (Q, nz, ny, nx) with Q = 19 (D3Q19) or 27 (D3Q27), chosen by
``OracleParams.lattice``; the two lattices are two builds of the same C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpf_oracle.c")
LATTICES = (19, 27)
Q = 19   # the default lattice


def _lib_path(q: int) -> str:
    return os.path.join(_HERE, "libcpf_oracle.so" if q == 19 else f"libcpf_oracle_q{q}.so")


_LIB_PATH = _lib_path(19)

DIAG_NAMES = ("sum_phi", "mass", "momx", "momy", "momz", "ekin", "umax", "phi_min",
              "phi_max", "comx", "comy", "comz", "phiux", "phiuy", "phiuz", "l2_num",
              "l2_den")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math),
    once per lattice; returns the D3Q19 library's path."""
    for q in LATTICES:
        path = _lib_path(q)
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                   "-Wall", f"-DORC_Q={q}", "-o", tmp, _SRC, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(tmp, path)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("wall", C.c_int * 3),
                ("courant", C.c_double),
                ("rho1", C.c_double), ("rho2", C.c_double),
                ("tau_rho1", C.c_double), ("tau_rho2", C.c_double),
                ("tau_phi", C.c_double), ("sigma", C.c_double), ("delta", C.c_double),
                ("G", C.c_double * 3),
                ("normal_fd", C.c_int),
                ("k1_eps", C.c_double),
                ("wetting", C.c_int),
                ("cos_theta", C.c_double)]


@dataclass
class OracleParams:
    nx: int
    ny: int
    nz: int
    wall: tuple = (0, 0, 0)
    courant: float = 0.997
    rho1: float = 1.0
    rho2: float = 1.0
    tau_rho1: float = 0.3
    tau_rho2: float = 0.3
    tau_phi: float = 0.3
    sigma: float = 0.0
    delta: float = 4.0
    G: tuple = (0.0, 0.0, 0.0)
    normal_fd: int = 0
    k1_eps: float = 1e-4
    lattice: int = 19        # 19 (D3Q19) or 27 (D3Q27): which build runs
    wetting: int = 0         # 1: contact angle at the walls (see cpf_oracle.c)
    cos_theta: float = 0.0

    def to_c(self) -> _Params:
        p = _Params()
        p.nx, p.ny, p.nz = int(self.nx), int(self.ny), int(self.nz)
        for a in range(3):
            p.wall[a] = int(self.wall[a])
            p.G[a] = float(self.G[a])
        p.courant = float(self.courant)
        p.rho1, p.rho2 = float(self.rho1), float(self.rho2)
        p.tau_rho1, p.tau_rho2 = float(self.tau_rho1), float(self.tau_rho2)
        p.tau_phi, p.sigma, p.delta = float(self.tau_phi), float(self.sigma), float(self.delta)
        p.normal_fd = int(self.normal_fd)
        p.k1_eps = float(self.k1_eps)
        p.wetting = int(self.wetting)
        p.cos_theta = float(self.cos_theta)
        return p

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    @property
    def Q(self):
        return _check_q(self.lattice)


_libs = {}
_dp = C.POINTER(C.c_double)


def _check_q(q) -> int:
    q = int(q)
    if q not in LATTICES:
        raise ValueError(f"lattice must be one of {LATTICES}, got {q}")
    return q


def _load(q: int = 19):
    q = _check_q(q)
    if q not in _libs:
        if not os.path.exists(_lib_path(q)):
            build(force=False)
        lib = C.CDLL(_lib_path(q))
        lib.orc_create.argtypes = [C.POINTER(_Params), _dp, _dp, _dp, C.POINTER(C.c_void_p)]
        lib.orc_create.restype = C.c_int
        lib.orc_destroy.argtypes = [C.c_void_p]
        lib.orc_step.argtypes = [C.c_void_p, C.c_long]
        lib.orc_time.argtypes = [C.c_void_p]
        lib.orc_time.restype = C.c_long
        lib.orc_fields.argtypes = [C.c_void_p, _dp, _dp, _dp]
        lib.orc_diag.argtypes = [C.c_void_p, _dp, _dp]
        lib.orc_get_pdfs.argtypes = [C.c_void_p, _dp, _dp]
        lib.orc_set_pdfs.argtypes = [C.c_void_p, _dp, _dp]
        lib.orc_lattice.argtypes = [C.POINTER(C.c_int), _dp]
        lib.orc_node_equilibria.argtypes = [C.POINTER(_Params), C.c_double, _dp, C.c_double,
                                            _dp, _dp, _dp, _dp, _dp]
        lib.orc_node_macro.argtypes = [C.POINTER(_Params), _dp, _dp, _dp]
        lib.orc_propagate.argtypes = [C.POINTER(_Params), _dp, _dp]
        lib.orc_fd_gradient.argtypes = [C.POINTER(_Params), _dp, _dp]
        lib.orc_num_threads.restype = C.c_int
        lib.orc_set_num_threads.argtypes = [C.c_int]
        _libs[q] = lib
    return _libs[q]


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def num_threads(q: int = 19) -> int:
    return int(_load(q).orc_num_threads())


def set_num_threads(n: int, q: int = 19):
    _load(q).orc_set_num_threads(int(n))


def lattice(q: int = 19):
    """(e^ (q,3) int, t (q,)) of the oracle's own D3Q19 or D3Q27 table."""
    lib = _load(q)
    e = (C.c_int * (q * 3))()
    t = np.zeros(q)
    lib.orc_lattice(e, _ptr(t))
    return np.array(list(e), dtype=np.int64).reshape(q, 3), t


def node_equilibria(P: OracleParams, phi, u, p, gradphi):
    lib = _load(P.Q)
    cp = P.to_c()
    u = _f64(u, (3,))
    gp = _f64(gradphi, (3,))
    out = [np.zeros(P.Q) for _ in range(4)]
    lib.orc_node_equilibria(C.byref(cp), float(phi), _ptr(u), float(p), _ptr(gp),
                            *[_ptr(o) for o in out])
    return tuple(out)  # feq, geq, S_i, R_i


def node_macro(P: OracleParams, fb, g):
    lib = _load(P.Q)
    cp = P.to_c()
    out = np.zeros(10)
    lib.orc_node_macro(C.byref(cp), _ptr(_f64(fb, (P.Q,))), _ptr(_f64(g, (P.Q,))), _ptr(out))
    return dict(phi=out[0], rho=out[1], tau_rho=out[2], u=out[3:6].copy(), p=out[6],
                gradphi=out[7:10].copy())


def propagate(P: OracleParams, fin):
    lib = _load(P.Q)
    cp = P.to_c()
    fin = _f64(fin, (P.Q,) + P.shape)
    out = np.empty_like(fin)
    lib.orc_propagate(C.byref(cp), _ptr(fin), _ptr(out))
    return out


def fd_gradient(P: OracleParams, phi):
    lib = _load(P.Q)
    cp = P.to_c()
    phi = _f64(phi, P.shape)
    out = np.empty((3,) + P.shape)
    lib.orc_fd_gradient(C.byref(cp), _ptr(phi), _ptr(out))
    return out


class Oracle:
    """A running FP64 CPU simulation (the oracle's own state at time t)."""

    def __init__(self, P: OracleParams, phi0, u0=None, p0=None):
        self.P = P
        self._lib = _load(P.Q)
        self._cp = P.to_c()
        phi0 = _f64(phi0, P.shape)
        u0 = _f64(u0, (3,) + P.shape) if u0 is not None else None
        p0 = _f64(p0, P.shape) if p0 is not None else None
        h = C.c_void_p()
        rc = self._lib.orc_create(C.byref(self._cp), _ptr(phi0), _ptr(u0), _ptr(p0), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle rejected the input (status {rc})")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    @property
    def t(self) -> int:
        return int(self._lib.orc_time(self._h))

    def step(self, n: int = 1):
        self._lib.orc_step(self._h, int(n))

    def fields(self):
        P = self.P
        phi = np.empty(P.shape)
        u = np.empty((3,) + P.shape)
        p = np.empty(P.shape)
        self._lib.orc_fields(self._h, _ptr(phi), _ptr(u), _ptr(p))
        return phi, u, p

    def diag(self, phi_ref=None) -> dict:
        out = np.zeros(len(DIAG_NAMES))
        ref = _f64(phi_ref, self.P.shape) if phi_ref is not None else None
        self._lib.orc_diag(self._h, _ptr(ref), _ptr(out))
        return dict(zip(DIAG_NAMES, out.tolist()))

    def pdfs(self):
        P = self.P
        f = np.empty((P.Q,) + P.shape)
        g = np.empty((P.Q,) + P.shape)
        self._lib.orc_get_pdfs(self._h, _ptr(f), _ptr(g))
        return f, g

    def set_pdfs(self, f, g):
        P = self.P
        self._lib.orc_set_pdfs(self._h, _ptr(_f64(f, (P.Q,) + P.shape)),
                               _ptr(_f64(g, (P.Q,) + P.shape)))
