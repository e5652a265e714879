"""Binding of libprobe.so (include/probe.h): the achievable HBM bandwidth of a
plain streaming copy on the current GPU, the yardstick beside the nominal
peak for the HBM-bound solver step. Argument marshalling and HIP-event
timing only; the copy is the library's kernel."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprobe.so")
_lib = None


def load_library():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        from .lbm import hip_runtime_first
        hip_runtime_first()  # one HIP runtime per process (see there)
        lib = C.CDLL(LIB_PATH)
        lib.probe_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_int32,
                                   C.c_void_p]
        lib.probe_copy.restype = C.c_int
        _lib = lib
    return _lib


def probe_copy(src, dst, nbytes: int, nontemporal: bool, blocks: int, stream):
    rc = load_library().probe_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                   C.c_size_t(nbytes), int(bool(nontemporal)), int(blocks),
                                   C.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"probe_copy failed with status {rc}")


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 10, blocks=(0, 2048, 8192, 32768),
                   device="cuda:0") -> dict:
    """GB/s of a copy of nbytes (bytes read + bytes written per second), for
    each variant (nontemporal or not, block count) the median of `reps`
    launches timed with HIP events on the current stream, and the best."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream(device)
    out = {}
    for nt in (True, False):
        for b in blocks:
            probe_copy(src, dst, nbytes, nt, b, st.cuda_stream)
            ts = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(st)
                probe_copy(src, dst, nbytes, nt, b, st.cuda_stream)
                e1.record(st)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            ts.sort()
            out[f"{'nt' if nt else 'plain'}_{b or 'per_thread'}"] = 2 * nbytes / ts[len(ts) // 2] / 1e9
    if not torch.equal(src[:: 1 << 16], dst[:: 1 << 16]):
        raise RuntimeError("probe_copy: the copy is wrong")
    best = max(out, key=out.get)
    return dict(copy_gbs=round(out[best], 1), best=best, bytes=nbytes,
                variants={k: round(v, 1) for k, v in out.items()})
