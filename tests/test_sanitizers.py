"""The oracle and the host side of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU. Each is built with the sanitizers
into a temporary directory and exercised in a child process that preloads
the matching runtime; any report aborts the child.

* The oracle (gcc, ASan + UBSan) runs ragged, walled, finite-difference,
  wetting and D3Q27 cases through every exported call.
* liblbm.so's host code (hipcc, the sanitizers given to the host pass only with
  -Xarch_host) runs parameter validation, the workspace layout, the lattice
  tables and the error strings over valid and invalid parameter sets (the
  kernels are built too, and never launched)."""
import os
import shutil
import subprocess
import sys

import pytest

pytestmark = pytest.mark.slow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:detect_odr_violation=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "OMP_NUM_THREADS": "2"}

ORACLE_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
from oracle import oracle as om
libs = {19: sys.argv[2], 27: sys.argv[3]}
om._lib_path = lambda q: libs[q]
from paper_2407_12263_amd import inputs
cases = [inputs.static_droplet(n=13, R=3.5, ny=7, nz=9, sigma=2e-3),
         inputs.rising_bubble(nx=6, ny=5, nz=12, R=2.0, zc=6.0, g=1e-4),
         inputs.rayleigh_taylor(nx=8, ny=16, nz=4)]
n = 0
for q in (19, 27):
    om.lattice(q)
    for w in cases:
        variants = [{}]
        if q == 19:
            variants.append({"normal_fd": 1})
        if any(w.wall):
            variants.append({"wetting": 1, "cos_theta": 0.5})
        for over in variants:
            P = om.OracleParams(**dict(w.params(), lattice=q, **over))
            o = om.Oracle(P, w.phi0, w.u0, w.p0)
            o.step(5)
            o.fields()
            o.diag(w.phi0)
            f, g = o.pdfs()
            o.set_pdfs(f, g)
            om.propagate(P, f)
            om.fd_gradient(P, w.phi0)
            om.node_macro(P, f[:, 0, 0, 0], g[:, 0, 0, 0])
            om.node_equilibria(P, 0.3, [1e-3, 0, 0], 0.0, [0.1, 0.0, 0.0])
            n += 1
try:
    om.Oracle(om.OracleParams(nx=4, ny=4, nz=4, courant=2.0), np.zeros((4, 4, 4)))
except ValueError:
    pass
print("CHILD_OK", n, flush=True)
"""

LBM_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import ctypes as C
from paper_2407_12263_amd import lbm
lib = C.CDLL(sys.argv[2])
lib.lbm_workspace_bytes.argtypes = [C.POINTER(lbm.LbmParams), C.POINTER(C.c_size_t)]
lib.lbm_lattice_q.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
lib.lbm_strerror.restype = C.c_char_p
good = dict(nx=13, ny=7, nz=9, precision="fp16", wall=(0, 1, 0))
cases = [good, dict(good, precision="fp32"), dict(good, precision="fp64", lattice=27),
         dict(good, normal_fd=1), dict(good, wetting=1, cos_theta=0.3),
         dict(good, nx=512, ny=512, nz=215), dict(good, nx=512, ny=512, nz=216),
         dict(good, nx=0), dict(good, courant=1.5), dict(good, k1_eps=-1.0),
         dict(good, store_log2=(30, 0)), dict(good, G=(float("nan"), 0, 0)),
         dict(good, wall=(1, 0, 0), nx=1), dict(good, lattice=27, normal_fd=1),
         dict(good, tau_phi=-0.6), dict(good, rho1=0.0)]
ok = 0
for c in cases:
    p = lbm.make_params(**c)
    n = C.c_size_t()
    rc = lib.lbm_workspace_bytes(C.byref(p), C.byref(n))
    ok += rc == 0
    lib.lbm_strerror(rc)
for q in (19, 27, 5):
    e = (C.c_int32 * 81)()
    t = (C.c_double * 27)()
    lib.lbm_lattice_q(q, e, t)
lib.lbm_workspace_bytes(None, None)
print("CHILD_OK", ok, len(cases), flush=True)
"""


def _run(code, args, preload):
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=preload)
    r = subprocess.run([sys.executable, "-c", code, ROOT, *args], capture_output=True, text=True,
                       timeout=600, env=env)
    assert r.returncode == 0 and "CHILD_OK" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
    return r.stdout


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc has no AddressSanitizer runtime")
    out = {}
    for q in (19, 27):
        out[q] = str(tmp_path / f"liborc{q}.so")
        subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                        "-ffp-contract=off", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", f"-DORC_Q={q}",
                        "-o", out[q], os.path.join(ROOT, "oracle", "cpf_oracle.c"), "-lm"],
                       check=True)
    stdout = _run(ORACLE_CHILD, [out[19], out[27]], asan)
    assert int(stdout.split()[-1]) >= 10


def test_lbm_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc")
    rt = [p for p in __import__("glob").glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")]
    if not hipcc or not rt:
        pytest.skip("no hipcc or no clang AddressSanitizer runtime")
    so = str(tmp_path / "liblbm_host_san.so")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
                    "-fPIC", "-shared", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                    "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
                    "-Xarch_host", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2407_12263_amd", "csrc"), "-o", so,
                    os.path.join(ROOT, "paper_2407_12263_amd", "csrc", "lbm.hip")], check=True,
                   capture_output=True)
    stdout = _run(LBM_CHILD, [so], rt[0])
    ok, n = map(int, stdout.split()[-2:])
    assert 0 < ok < n      # valid sets accepted, invalid ones rejected, no report either way
