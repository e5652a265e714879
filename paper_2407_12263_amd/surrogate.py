"""Coarse-grid 3D U-Net surrogate: Python orchestration of the HIP kernels in
``libsur.so`` (C ABI ``include/sur.h``).

The network advances the coarsened state (phi, u, p) of the LBM solver by a
window of K steps: state(t + K) = state(t) + UNet(state(t)). Every layer is a
``sur_*`` kernel launch on the current stream (3x3x3 convolutions on BF16
matrix cores with FP32 accumulation, pooling, upsampling, concat, residual
MSE, Adam); this module only allocates the tensors (PyTorch) and sequences
the calls. There is no fallback: without the library or a GPU it raises.

Architecture (channels per level, e.g. 16-32-48-64): per level two
conv + ReLU, 2x average pooling between levels, nearest 2x upsampling and
concat with the skip on the way up, two conv + ReLU, a final linear conv.
Input and output have 16 channels of which the first 5 are used.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsur.so")
NCH = 16          # stored channels of the state
NUSE = 5          # phi, ux, uy, uz, p

_lib = None


def load_library(path: str | None = None):
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FileNotFoundError(f"HIP library {p} is not built; run __graft_entry__.build()")
    from .lbm import hip_runtime_first
    hip_runtime_first()  # one HIP runtime per process (see there)
    lib = C.CDLL(p)
    vp, i32, i64, fl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
    lib.sur_conv3d.argtypes = [vp, i32, vp, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp]
    lib.sur_conv3d_cat.argtypes = [vp, i32, vp, i32, vp, vp, i32, i32, i32, i32, i32, vp, vp, vp]
    lib.sur_conv3d_pool.argtypes = [vp, i32, vp, vp, i32, i32, i32, i32, i32, vp, vp, vp]
    lib.sur_wgrad_scratch_floats.argtypes = [i32, i32, i32, i32, i32]
    lib.sur_wgrad_scratch_floats.restype = sz
    lib.sur_conv3d_wgrad.argtypes = [vp, i32, vp, i32, i32, i32, i32, vp, sz, vp, vp, vp]
    lib.sur_pack_weights.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.sur_pool2.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    lib.sur_pool2_bwd.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    lib.sur_pool2_bwd_skip.argtypes = [vp, i32, i32, i32, i32, vp, i32, i32, vp, vp, vp, vp]
    lib.sur_upsample2_bwd_mask.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp, vp]
    lib.sur_concat_up2.argtypes = [vp, i32, vp, i32, i32, i32, i32, vp, vp]
    lib.sur_pack_weights_all.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.sur_upsample2.argtypes = [vp, i32, i32, i32, i32, vp, i32, i32, vp]
    lib.sur_upsample2_bwd.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp]
    lib.sur_copy_channels.argtypes = [vp, i32, i64, vp, i32, i32, vp]
    lib.sur_add_channels.argtypes = [vp, i32, i32, i32, i64, vp, vp]
    lib.sur_to_bf16.argtypes = [vp, i64, vp, vp]
    lib.sur_relu_mask.argtypes = [vp, vp, i64, vp]
    lib.sur_mse.argtypes = [vp, vp, i32, i32, i64, vp, vp, vp, vp, vp, vp]
    lib.sur_adam.argtypes = [vp, vp, vp, vp, i64, fl, fl, fl, fl, i32, vp]
    lib.sur_coarsen.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp, vp]
    lib.sur_prolong_add.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.sur_checks.argtypes = [vp, i32, i32, i32, vp, vp, vp]
    lib.sur_checks_noalloc.argtypes = [vp, i32, i32, i32, vp, vp]
    lib.sur_apply_residual.argtypes = [vp, vp, vp, i32, i64, C.c_double, vp]
    lib.sur_residual_target.argtypes = [vp, vp, vp, i32, i64, C.c_double, vp, vp]
    lib.sur_fix_mass.argtypes = [vp, i64, vp, vp, vp]
    lib.sur_features.argtypes = [vp, i32, i32, i32, vp]
    lib.sur_prolong_update_scratch_doubles.argtypes = [i32, i32, i32]
    lib.sur_prolong_update_scratch_doubles.restype = sz
    lib.sur_prolong_update.argtypes = [vp, vp, i32, i32, i32, vp, C.c_double, vp, vp, vp, vp, vp, vp]
    for n in ["sur_features", "sur_prolong_update", "sur_apply_residual", "sur_residual_target", "sur_fix_mass", "sur_conv3d", "sur_conv3d_cat", "sur_conv3d_pool", "sur_conv3d_wgrad", "sur_pack_weights", "sur_pool2", "sur_pool2_bwd",
              "sur_upsample2", "sur_upsample2_bwd", "sur_copy_channels", "sur_add_channels",
              "sur_to_bf16", "sur_relu_mask", "sur_mse", "sur_adam", "sur_coarsen",
              "sur_prolong_add", "sur_checks", "sur_checks_noalloc", "sur_pool2_bwd_skip", "sur_upsample2_bwd_mask",
              "sur_concat_up2", "sur_pack_weights_all"]:
        getattr(lib, n).restype = C.c_int
    if path is None:
        _lib = lib
    return lib


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ok(rc, where):
    if rc != 0:
        raise RuntimeError(f"{where} failed with status {rc}")


# ------------------------------------------------------------ C names

def sur_conv3d(x, cin, w, bias, cout, grid, flip=0, relu=0, mask=None, y_bf16=None, y_f32=None):
    nx, ny, nz = grid
    _ok(load_library().sur_conv3d(_p(x), cin, _p(w), _p(bias), cout, nx, ny, nz, flip, relu,
                                  _p(mask), _p(y_bf16), _p(y_f32), _stream()), "sur_conv3d")


def sur_conv3d_cat(xc, cc, xf, fc, w, bias, cout, grid, relu=0, y_bf16=None, y_f32=None):
    nx, ny, nz = grid
    _ok(load_library().sur_conv3d_cat(_p(xc), cc, _p(xf), fc, _p(w), _p(bias), cout, nx, ny, nz,
                                      relu, _p(y_bf16), _p(y_f32), _stream()), "sur_conv3d_cat")


def sur_conv3d_pool(x, cin, w, bias, cout, grid, relu=0, y_bf16=None, y_pool=None):
    nx, ny, nz = grid
    _ok(load_library().sur_conv3d_pool(_p(x), cin, _p(w), _p(bias), cout, nx, ny, nz, relu,
                                       _p(y_bf16), _p(y_pool), _stream()), "sur_conv3d_pool")


def conv_cat_fits(grid):
    """Whether sur_conv3d_cat and sur_conv3d_pool take these (fine-grid)
    sizes: their tiled kernel's 16 x 4 x 4 point tile."""
    nx, ny, nz = grid
    return nx % 16 == 0 and ny % 4 == 0 and nz % 4 == 0


def sur_wgrad_scratch_floats(cin, cout, grid):
    return int(load_library().sur_wgrad_scratch_floats(cin, cout, *grid))


def sur_conv3d_wgrad(x, cin, dy, cout, grid, scratch, dw, dbias):
    nx, ny, nz = grid
    _ok(load_library().sur_conv3d_wgrad(_p(x), cin, _p(dy), cout, nx, ny, nz, _p(scratch),
                                        scratch.numel(), _p(dw), _p(dbias), _stream()),
        "sur_conv3d_wgrad")


def sur_pack_weights(w, cin, cout, wf, wd):
    _ok(load_library().sur_pack_weights(_p(w), cin, cout, _p(wf), _p(wd), _stream()),
        "sur_pack_weights")


def sur_pool2(x, c, grid, y):
    _ok(load_library().sur_pool2(_p(x), c, *grid, _p(y), _stream()), "sur_pool2")


def sur_pool2_bwd(dy, c, grid, dx):
    _ok(load_library().sur_pool2_bwd(_p(dy), c, *grid, _p(dx), _stream()), "sur_pool2_bwd")


def sur_pool2_bwd_skip(dy, c, grid, skip, skip_stride, skip_off, act, dx=None, dx_bf16=None):
    _ok(load_library().sur_pool2_bwd_skip(_p(dy), c, *grid, _p(skip), skip_stride, skip_off,
                                          _p(act), _p(dx), _p(dx_bf16), _stream()),
        "sur_pool2_bwd_skip")


def sur_upsample2_bwd_mask(dy, dystride, dyoff, c, grid, act, dx_bf16):
    _ok(load_library().sur_upsample2_bwd_mask(_p(dy), dystride, dyoff, c, *grid, _p(act),
                                              _p(dx_bf16), _stream()), "sur_upsample2_bwd_mask")


def sur_pack_weights_all(w_flat, w_off, cin, cout, wf_flat, wd_flat):
    n = len(w_off)
    offs = (C.c_int64 * n)(*[int(o) for o in w_off])
    ci = (C.c_int32 * n)(*[int(c) for c in cin])
    co = (C.c_int32 * n)(*[int(c) for c in cout])
    _ok(load_library().sur_pack_weights_all(_p(w_flat), n, offs, ci, co, _p(wf_flat), _p(wd_flat),
                                            _stream()), "sur_pack_weights_all")


def sur_concat_up2(xc, hc, xf, fc, grid, y):
    _ok(load_library().sur_concat_up2(_p(xc), hc, _p(xf), fc, *grid, _p(y), _stream()),
        "sur_concat_up2")


def sur_upsample2(x, c, grid, y, ystride, yoff):
    _ok(load_library().sur_upsample2(_p(x), c, *grid, _p(y), ystride, yoff, _stream()),
        "sur_upsample2")


def sur_upsample2_bwd(dy, dystride, dyoff, c, grid, dx):
    _ok(load_library().sur_upsample2_bwd(_p(dy), dystride, dyoff, c, *grid, _p(dx), _stream()),
        "sur_upsample2_bwd")


def sur_copy_channels(x, c, P, y, ystride, yoff):
    _ok(load_library().sur_copy_channels(_p(x), c, P, _p(y), ystride, yoff, _stream()),
        "sur_copy_channels")


def sur_add_channels(dy, dystride, dyoff, c, P, dx):
    _ok(load_library().sur_add_channels(_p(dy), dystride, dyoff, c, P, _p(dx), _stream()),
        "sur_add_channels")


def sur_to_bf16(x, y):
    _ok(load_library().sur_to_bf16(_p(x), x.numel(), _p(y), _stream()), "sur_to_bf16")


def sur_relu_mask(dx, act):
    _ok(load_library().sur_relu_mask(_p(dx), _p(act), dx.numel(), _stream()), "sur_relu_mask")


def sur_mse(pred, target, cu, cs, P, wch, grad, scratch, loss_out, grad_bf16=None):
    _ok(load_library().sur_mse(_p(pred), _p(target), cu, cs, P, _p(wch), _p(grad), _p(grad_bf16),
                               _p(scratch), _p(loss_out), _stream()), "sur_mse")


def sur_adam(w, m, v, g, lr, b1, b2, eps, t):
    _ok(load_library().sur_adam(_p(w), _p(m), _p(v), _p(g), w.numel(), lr, b1, b2, eps, t,
                                _stream()), "sur_adam")


def sur_coarsen(phi, u, p, grid, scale, coarse_f32, coarse_bf16=None):
    _ok(load_library().sur_coarsen(_p(phi), _p(u), _p(p), *grid, _p(scale), _p(coarse_f32),
                                   _p(coarse_bf16), _stream()), "sur_coarsen")


def sur_prolong_add(delta, cgrid, scale, phi, u, p):
    _ok(load_library().sur_prolong_add(_p(delta), *cgrid, _p(scale), _p(phi), _p(u), _p(p),
                                       _stream()), "sur_prolong_add")


def sur_checks(state, grid, scratch, out):
    _ok(load_library().sur_checks(_p(state), *grid, _p(scratch), _p(out), _stream()), "sur_checks")


def sur_checks_noalloc(state, grid, out):
    """sur_checks with the library's own partials buffer (no scratch)."""
    _ok(load_library().sur_checks_noalloc(_p(state), *grid, _p(out), _stream()),
        "sur_checks_noalloc")


CHECKS_NOALLOC_MAX_POINTS = 1 << 22


def sur_apply_residual(state, out, rscale, cu, P, width=0.0):
    _ok(load_library().sur_apply_residual(_p(state), _p(out), _p(rscale), cu, P, float(width),
                                          _stream()), "sur_apply_residual")


def sur_residual_target(s0, s1, rscale, cu, P, target, width=0.0):
    _ok(load_library().sur_residual_target(_p(s0), _p(s1), _p(rscale), cu, P, float(width),
                                           _p(target), _stream()), "sur_residual_target")


def sur_fix_mass(state, P, checks_out, target_mass):
    _ok(load_library().sur_fix_mass(_p(state), P, _p(checks_out), _p(target_mass), _stream()),
        "sur_fix_mass")


def sur_features(state, grid):
    _ok(load_library().sur_features(_p(state), *grid, _stream()), "sur_features")


def sur_prolong_update_scratch_doubles(cgrid):
    return int(load_library().sur_prolong_update_scratch_doubles(*cgrid))


def sur_prolong_update(s0, s1, cgrid, scale, width, phi, u, p, scratch, sums):
    _ok(load_library().sur_prolong_update(_p(s0), _p(s1), *cgrid, _p(scale), float(width), _p(phi),
                                          _p(u), _p(p), _p(scratch), _p(sums), _stream()),
        "sur_prolong_update")


# ---------------------------------------------------------------- the U-Net

def unet_layers(channels, cin=NCH, cout=NCH):
    """(name, cin, cout, relu) of every conv in parameter order (encoder
    levels a/b, decoder levels from the bottom up, final conv)."""
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


class UNet:
    """Parameters, Adam state and activation buffers of one U-Net on a fixed
    coarse grid (nx, ny, nz), each divisible by 2^(levels-1)."""

    def __init__(self, grid, channels=(16, 32, 48, 64), seed=0, device="cuda:0", out_scale=0.1):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate runs on the GPU; none is visible")
        load_library()
        self.torch = torch
        self.dev = torch.device(device)
        self.channels = tuple(channels)
        self.layers = unet_layers(self.channels)
        self.nlev = len(self.channels)
        nx, ny, nz = grid
        for n in grid:
            if n % (2 ** (self.nlev - 1)):
                raise ValueError("grid sizes must be divisible by 2^(levels-1)")
        self.grids = [(nx >> l, ny >> l, nz >> l) for l in range(self.nlev)]
        self.P = [a * b * c for (a, b, c) in self.grids]
        g = torch.Generator().manual_seed(seed)
        # every layer's weights and bias are views of one flat FP32 buffer (and
        # so are their Adam moments and gradients), so that one Adam launch
        # updates all parameters
        sizes = []
        for name, ci, co, relu in self.layers:
            sizes += [27 * co * ci, co]
        ntot = sum(sizes)
        self.flat = {k: torch.zeros(ntot, dtype=torch.float32, device=self.dev)
                     for k in ("w", "m", "v", "g")}

        def views(buf):
            out, off = [], 0
            for k, (name, ci, co, relu) in enumerate(self.layers):
                out.append(buf[off:off + 27 * co * ci].view(27, co, ci))
                off += 27 * co * ci
                out.append(buf[off:off + co])
                off += co
            return out[0::2], out[1::2]

        self.w, self.b = views(self.flat["w"])
        self.mw, self.mb = views(self.flat["m"])
        self.vw, self.vb = views(self.flat["v"])
        self.gw, self.gb = views(self.flat["g"])
        for k, (name, ci, co, relu) in enumerate(self.layers):
            std = math.sqrt(2.0 / (27 * ci)) * (1.0 if relu else out_scale)
            self.w[k].copy_((torch.randn((27, co, ci), generator=g) * std).to(self.dev))
        # BF16 packings, back to back in two flat buffers (one packing launch)
        npk = [27 * co * ci for name, ci, co, relu in self.layers]
        self.pk_flat = {k: torch.empty(sum(npk), dtype=torch.int16, device=self.dev)
                        for k in ("f", "d")}
        self.wf, self.wd, off = [], [], 0
        for (name, ci, co, relu), n in zip(self.layers, npk):
            self.wf.append(self.pk_flat["f"][off:off + n].view(27, co, ci))
            self.wd.append(self.pk_flat["d"][off:off + n].view(27, ci, co))
            off += n
        self._w_off = [w.storage_offset() - self.flat["w"].storage_offset() for w in self.w]
        self.adam_t = 0
        self._alloc()
        self.pack()

    # -------------------------------------------------------------- buffers
    def _alloc(self):
        torch = self.torch
        bf = lambda P, c: torch.empty((P, c), dtype=torch.int16, device=self.dev)
        f32 = lambda P, c: torch.zeros((P, c), dtype=torch.float32, device=self.dev)
        self.act = {}
        for k, (name, ci, co, relu) in enumerate(self.layers):
            lv = self._level(name)
            if relu:
                self.act[name] = bf(self.P[lv], co)
        for lv in range(self.nlev - 1):
            self.act[f"pool{lv}"] = bf(self.P[lv + 1], self.channels[lv])
        for lv in range(self.nlev - 1):
            # [upsampled output of level lv + 1, skip of level lv]
            self.act[f"cat{lv}"] = bf(self.P[lv], self.channels[lv + 1] + self.channels[lv])
        self.out = f32(self.P[0], NCH)
        sc = 0
        for k, (name, ci, co, relu) in enumerate(self.layers):
            sc = max(sc, sur_wgrad_scratch_floats(ci, co, self.grids[self._level(name)]))
        self.scratch = torch.empty(sc, dtype=torch.float32, device=self.dev)
        self.loss_scratch = torch.empty(self.P[0] // 256 + 2, dtype=torch.float64, device=self.dev)
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=self.dev)
        # the loss gradient only feeds the output layer's backward: BF16
        self.dout = torch.empty((self.P[0], NCH), dtype=torch.int16, device=self.dev)

    @staticmethod
    def _level(name):
        return 0 if name == "out" else int(name[3:-1])

    def pack(self):
        sur_pack_weights_all(self.flat["w"], self._w_off, [ci for _, ci, _, _ in self.layers],
                             [co for _, _, co, _ in self.layers], self.pk_flat["f"],
                             self.pk_flat["d"])

    def n_params(self):
        return sum(w.numel() + b.numel() for w, b in zip(self.w, self.b))

    # -------------------------------------------------------------- forward
    def forward(self, x_bf16, keep_cat=False):
        """x_bf16: int16 tensor [P0, 16] (BF16 bits). Returns the FP32 output
        [P0, 16] (the residual in scaled units). The decoder convolutions read
        their concat in place (sur_conv3d_cat) unless keep_cat is set (the
        training step: the weight gradient reads the concat) or the grid does
        not fit that kernel; both ways give the same bits."""
        k = 0
        h = x_bf16
        hc = NCH
        for lv in range(self.nlev):
            g = self.grids[lv]
            for part in "ab":
                name, ci, co, relu = self.layers[k]
                if part == "b" and lv < self.nlev - 1 and conv_cat_fits(g):
                    # the pooled output in the same pass
                    sur_conv3d_pool(h, ci, self.wf[k], self.b[k], co, g, relu=1,
                                    y_bf16=self.act[name], y_pool=self.act[f"pool{lv}"])
                    pooled = True
                else:
                    sur_conv3d(h, ci, self.wf[k], self.b[k], co, g, relu=1, y_bf16=self.act[name])
                    pooled = False
                h, hc = self.act[name], co
                k += 1
            if lv < self.nlev - 1:
                if not pooled:
                    sur_pool2(h, hc, g, self.act[f"pool{lv}"])
                h = self.act[f"pool{lv}"]
        self._cat_kept = True
        for lv in range(self.nlev - 2, -1, -1):
            skip = self.act[f"enc{lv}b"]
            if not keep_cat and conv_cat_fits(self.grids[lv]):
                self._cat_kept = False
                name, ci, co, relu = self.layers[k]
                sur_conv3d_cat(h, hc, skip, self.channels[lv], self.wf[k], self.b[k], co,
                               self.grids[lv], relu=1, y_bf16=self.act[name])
                h, hc = self.act[name], co
                k += 1
                parts = "b"
            else:
                cat = self.act[f"cat{lv}"]
                sur_concat_up2(h, hc, skip, self.channels[lv], self.grids[lv], cat)
                h, hc = cat, cat.shape[1]
                parts = "ab"
            for part in parts:
                name, ci, co, relu = self.layers[k]
                sur_conv3d(h, ci, self.wf[k], self.b[k], co, self.grids[lv], relu=1,
                           y_bf16=self.act[name])
                h, hc = self.act[name], co
                k += 1
        name, ci, co, relu = self.layers[k]
        sur_conv3d(h, ci, self.wf[k], self.b[k], co, self.grids[0], relu=0, y_f32=self.out)
        self._last_input = x_bf16
        return self.out

    # ------------------------------------------------------------- backward
    def _conv_back(self, k, x_in, dy, grid, mask, out_bf16=False):
        """Weight/bias gradients of layer k and the input gradient (masked by
        mask > 0 if given): FP32, or BF16 bits (int16) with ``out_bf16`` when
        it only feeds the next layer's backward. dy is FP32 or BF16 bits."""
        torch = self.torch
        name, ci, co, relu = self.layers[k]
        lv = self._level(name)
        P = self.P[lv]
        if dy.dtype == torch.int16:
            dyb = dy
        else:
            dyb = torch.empty((P, co), dtype=torch.int16, device=self.dev)
            sur_to_bf16(dy, dyb)
        sur_conv3d_wgrad(x_in, ci, dyb, co, grid, self.scratch, self.gw[k], self.gb[k])
        if out_bf16:
            dx = torch.empty((P, ci), dtype=torch.int16, device=self.dev)
            sur_conv3d(dyb, co, self.wd[k], None, ci, grid, flip=1, relu=0, mask=mask, y_bf16=dx)
        else:
            dx = torch.empty((P, ci), dtype=torch.float32, device=self.dev)
            sur_conv3d(dyb, co, self.wd[k], None, ci, grid, flip=1, relu=0, mask=mask, y_f32=dx)
        return dx

    def backward(self, dout):
        """dout: FP32 [P0, 16] gradient at the output. Fills gw, gb. Needs the
        concat buffers of the last forward (forward with keep_cat=True)."""
        if not getattr(self, "_cat_kept", False):
            raise RuntimeError("UNet.backward needs the forward pass run with keep_cat=True")
        torch = self.torch
        k = len(self.layers) - 1
        nlev = self.nlev
        last = self.layers[k - 1][0]
        # gradients that only feed the next layer's backward stay BF16 (the
        # rounding it would apply anyway); those that are split, upsampled
        # or pooled first are FP32
        dh = self._conv_back(k, self.act[last], dout, self.grids[0], mask=self.act[last],
                             out_bf16=True)
        dskip = [None] * (nlev - 1)
        for lv in range(0, nlev - 1):
            for part in "ba":
                k -= 1
                name, ci, co, relu = self.layers[k]
                x_in = self.act[f"cat{lv}"] if part == "a" else self.act[self.layers[k - 1][0]]
                if part == "b":
                    mask = self.act[self.layers[k - 1][0]]
                else:
                    mask = None  # input is the concat: split below, masks come from its parts
                dh = self._conv_back(k, x_in, dh, self.grids[lv], mask, out_bf16=part == "b")
            cup = dh.shape[1] - self.channels[lv]
            # skip part: gradient w.r.t. enc{lv}b output, channels cup .. of dh
            # (added and masked later with the encoder's pooled path)
            dskip[lv] = (dh, dh.shape[1], cup)
            # upsampled part: gradient w.r.t. the lower level's output, a ReLU
            # activation (bottom or decoder b of lv + 1); BF16, it only feeds
            # that layer's backward
            below = f"enc{lv + 1}b" if lv + 1 == nlev - 1 else f"dec{lv + 1}b"
            du = torch.empty((self.P[lv + 1], cup), dtype=torch.int16, device=self.dev)
            sur_upsample2_bwd_mask(dh, dh.shape[1], 0, cup, self.grids[lv + 1], self.act[below], du)
            dh = du
        for lv in range(nlev - 1, -1, -1):
            if lv < nlev - 1:
                # gradient w.r.t. enc{lv}b output = pooled path + skip path,
                # through its ReLU (one pass)
                dfull = torch.empty((self.P[lv], self.channels[lv]), dtype=torch.int16,
                                    device=self.dev)
                skip, sstride, soff = dskip[lv]
                sur_pool2_bwd_skip(dh, self.channels[lv], self.grids[lv], skip, sstride, soff,
                                   self.act[f"enc{lv}b"], dx_bf16=dfull)
                dh = dfull
            for part in "ba":
                k -= 1
                name, ci, co, relu = self.layers[k]
                if part == "b":
                    x_in = self.act[self.layers[k - 1][0]]
                    mask = x_in
                else:
                    x_in = self._last_input if lv == 0 else self.act[f"pool{lv - 1}"]
                    mask = None
                dh = self._conv_back(k, x_in, dh, self.grids[lv], mask, out_bf16=part == "b")
        return dh

    def loss_and_grad(self, target_f32, wch):
        """Residual MSE on the used channels; gradient into self.dout."""
        sur_mse(self.out, target_f32, NUSE, NCH, self.P[0], wch, None, self.loss_scratch,
                self.loss_dev, grad_bf16=self.dout)
        return self.loss_dev

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.adam_t += 1
        f = self.flat
        sur_adam(f["w"], f["m"], f["v"], f["g"], lr, b1, b2, eps, self.adam_t)
        self.pack()

    def train_step(self, x_bf16, target_f32, wch, lr=1e-3):
        self.forward(x_bf16, keep_cat=True)
        loss = self.loss_and_grad(target_f32, wch)
        self.backward(self.dout)
        self.adam_step(lr)
        return loss

    # ------------------------------------------------------------ host I/O
    def get_params(self):
        return [(w.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64))
                for w, b in zip(self.w, self.b)]

    def set_params(self, params):
        torch = self.torch
        for k, (w, b) in enumerate(params):
            self.w[k].copy_(torch.as_tensor(np.asarray(w, dtype=np.float32)))
            self.b[k].copy_(torch.as_tensor(np.asarray(b, dtype=np.float32)))
        self.pack()

    def state_dict(self):
        return {"channels": list(self.channels),
                "w": [w.cpu() for w in self.w], "b": [b.cpu() for b in self.b]}


def bf16_bits_from_f32(t):
    """Round an FP32 torch tensor to BF16 (ties to even) on the GPU and return
    the bit pattern as int16 (the format the kernels read)."""
    import torch
    out = torch.empty(t.shape, dtype=torch.int16, device=t.device)
    sur_to_bf16(t.contiguous(), out)
    return out


def _main(argv=None):
    """Times the U-Net on an n^3 coarse grid: `reps` forward passes, then
    `reps` training steps (forward, both gradients, Adam with lr 0), with
    HIP events on the stream the kernels run on."""
    import argparse
    import torch
    ap = argparse.ArgumentParser(description=_main.__doc__)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args(argv)
    g = (a.grid,) * 3
    net = UNet(g, channels=(16, 32, 48, 64), seed=0)
    P = a.grid ** 3
    x = torch.zeros((P, NCH), dtype=torch.int16, device=net.dev)
    x.random_(0, 1 << 14)  # BF16 bit patterns of values in [0, 2)
    tgt = torch.zeros((P, NCH), dtype=torch.float32, device=net.dev)
    wch = torch.ones(NUSE, dtype=torch.float32, device=net.dev)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    flop = sum(2 * 27 * ci * co * net.P[net._level(n)] for n, ci, co, _ in net.layers)
    for what, fn in (("forward", lambda: net.forward(x)),
                     ("train step", lambda: net.train_step(x, tgt, wch, lr=0.0))):
        for _ in range(3):
            fn()
        e0.record(st)
        for _ in range(a.reps):
            fn()
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / a.reps
        extra = f", {flop / (ms * 1e-3) / 1e12:.1f} TFLOP/s" if what == "forward" else ""
        print(f"unet {a.grid}^3 {what}: {ms:.3f} ms{extra}", flush=True)


if __name__ == "__main__":
    _main()
