"""The C-ABI library loads and exports every symbol include/lbm.h declares;
host-only entry points behave (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2407_12263_amd import lbm
    return lbm


def test_surrogate_library_exports_every_declared_symbol():
    """libsur.so exports every function include/sur.h declares."""
    from paper_2407_12263_amd import surrogate
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "sur.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(sur_[a-z0-9_]+)\s*\(", src)))
    assert "sur_conv3d" in names and "sur_pool2_bwd_skip" in names
    so = surrogate.load_library()
    for n in names:
        assert hasattr(so, n), n


def test_probe_library_exports_every_declared_symbol():
    from paper_2407_12263_amd import probe
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "probe.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(probe_[a-z0-9_]+)\s*\(", src)))
    assert names == ["probe_copy"]
    so = probe.load_library()
    for n in names:
        assert hasattr(so, n), n


def test_library_exports_every_declared_symbol(lib):
    names = _declared()
    assert "lbm_init" in names and "lbm_step" in names and "lbm_diagnostics" in names
    so = lib.load_library()
    for n in names:
        assert hasattr(so, n), n


def test_lattice_is_d3q19(lib, orc):
    e, t = lib.lbm_lattice()
    eo, to = orc.lattice()
    assert sorted(map(tuple, e)) == sorted(map(tuple, eo))
    # weights by speed class, same as the oracle's
    for i in range(19):
        j = [k for k in range(19) if tuple(eo[k]) == tuple(e[i])][0]
        assert t[i] == to[j]
    assert e[0].tolist() == [0, 0, 0]


def test_lattice_q27_matches_oracle(lib, orc):
    """lbm_lattice_q(27): the oracle's D3Q27 vectors and weights, the D3Q19
    order as its first 19 entries, opposite directions adjacent (i, i + 1
    for odd i, which the collision's pair evaluation relies on)."""
    e, t = lib.lbm_lattice_q(27)
    eo, to = orc.lattice(27)
    assert sorted(map(tuple, e)) == sorted(map(tuple, eo))
    for i in range(27):
        j = [k for k in range(27) if tuple(eo[k]) == tuple(e[i])][0]
        assert t[i] == to[j]
    e19, _ = lib.lbm_lattice()
    assert np.array_equal(e[:19], e19)
    for i in range(1, 27, 2):
        assert np.array_equal(e[i], -e[i + 1])
    assert np.array_equal(lib.lbm_lattice_q(19)[0], e19)
    with pytest.raises(lib.LbmError):
        lib.lbm_lattice_q(15)


def test_workspace_bytes_and_validation(lib):
    p = lib.make_params(32, 32, 32, precision="fp32")
    n32 = lib.lbm_workspace_bytes(p)
    N = 32 ** 3
    assert n32 >= 2 * 2 * 19 * N * 4
    p16 = lib.make_params(32, 32, 32, precision="fp16")
    n16 = lib.lbm_workspace_bytes(p16)
    assert 2 * (2 * 19 * N * 2 + 4 * N) <= n16 < n32
    bad = [dict(courant=1.5), dict(courant=0.0), dict(tau_phi=0.0), dict(rho1=-1.0),
           dict(delta=0.0), dict(wall=(0, 0, 2)), dict(precision=7), dict(sigma=-1.0),
           dict(k1_eps=-1.0), dict(store_log2=(30, 0)), dict(G=(float("nan"), 0, 0)),
           dict(normal_fd=2), dict(nx=0), dict(ny=0), dict(nz=-1)]
    for kw in bad:
        kw = dict(dict(nx=8, ny=8, nz=8), **kw)
        with pytest.raises(lib.LbmError) as ei:
            lib.lbm_workspace_bytes(lib.make_params(**kw))
        assert ei.value.status == lib.LBM_EINVAL
    with pytest.raises(lib.LbmError):
        lib.lbm_workspace_bytes(lib.make_params(8, 1, 8, wall=(0, 1, 0)))
    with pytest.raises(lib.LbmError):
        lib.lbm_workspace_bytes(lib.make_params(1024, 1024, 128))  # 19 N >= 2^31
    # D3Q27: 27 planes per field; the comparison FD scheme is D3Q19 only
    n27 = lib.lbm_workspace_bytes(lib.make_params(32, 32, 32, precision="fp32", lattice=27))
    assert n27 >= 2 * 2 * 27 * N * 4 and n27 > n32
    for kw in (dict(lattice=23), dict(lattice=27, normal_fd=1), dict(wetting=2),
               dict(wetting=1, cos_theta=1.5), dict(wetting=1, cos_theta=float("nan")),
               dict(wetting=1, normal_fd=1)):
        with pytest.raises(lib.LbmError) as ei:
            lib.lbm_workspace_bytes(lib.make_params(8, 8, 8, **kw))
        assert ei.value.status == lib.LBM_EINVAL
    # 19 planes of 512 x 512 x 160 FP32 fit one 32-bit buffer range, 27 do not
    lib.lbm_workspace_bytes(lib.make_params(512, 512, 160))
    with pytest.raises(lib.LbmError):
        lib.lbm_workspace_bytes(lib.make_params(512, 512, 160, lattice=27))


def test_strerror(lib):
    assert lib.strerror(0) == "ok"
    assert "invalid" in lib.strerror(-1)


def test_init_rejects_null_workspace(lib):
    so = lib.load_library()
    p = lib.make_params(8, 8, 8)
    h = C.c_void_p()
    assert so.lbm_init(C.byref(p), None, 0, None, None, None, None, C.byref(h)) == lib.LBM_EINVAL
    assert not h.value
    assert so.lbm_step(None, 1) == lib.LBM_EINVAL
