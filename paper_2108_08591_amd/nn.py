"""Learned warm start for steady MDF-LBM cavity solves.

A U-Net-style convolutional encoder-decoder (4 levels, 32/64/128/256
channels, ~1.9 M parameters, BF16 matrix-core products with FP32
accumulation) maps a cavity description -- solid mask, Reynolds number, lid
speed and the node coordinates -- to the steady fields (P, u, v, du/dx,
du/dy, dv/dx, dv/dy).  Its prediction initialises the solver with f^eq + f^ne
(the inverse of eq. 3-16, MDF_INIT_FIELDS_GRAD); the solver then runs to its
own residual, and a cold start from rest stays the fallback.

Every layer runs in the kernels of include/mdfnn.h (libmdf.so); this module
marshals arguments and orders the calls.  torch provides device memory.
"""
from __future__ import annotations

import ctypes
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

from . import mdf

FEATURES = 6          # solid mask, Re feature, lid-speed feature, x, y, wall distance
COARSE_FEATURES = 8   # optional, once or twice: a coarse-grid solution in target scales (7) and its flag
IN_CH = 32            # features padded to the 32-channel granularity of the kernels
OUT_CH = 7            # P, u, v, du/dx, du/dy, dv/dx, dv/dy
LEVELS = (32, 64, 128, 256)

_DECLARED = False


def _lib():
    global _DECLARED
    L = mdf.lib()
    if not _DECLARED:
        vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_float
        sz = ctypes.c_size_t
        L.mdfnn_conv3x3_fwd.argtypes = [vp, i32, vp, i32, vp, vp, i32, i32, i32, i32, i32, vp, vp, vp, vp]
        L.mdfnn_conv3x3_flip.argtypes = [vp, i32, i32, vp, vp]
        L.mdfnn_wgrad_scratch_bytes.argtypes = [i32, i32, i32, i32, i32]
        L.mdfnn_wgrad_scratch_bytes.restype = sz
        L.mdfnn_conv3x3_wgrad.argtypes = [vp, i32, vp, i32, vp, i32, i32, i32, i32, vp, vp, vp, vp]
        L.mdfnn_avgpool2_fwd.argtypes = [vp, i32, i32, i32, i32, vp, vp]
        L.mdfnn_avgpool2_bwd.argtypes = [vp, i32, i32, i32, i32, vp, vp]
        L.mdfnn_upsample2_fwd.argtypes = [vp, i32, i32, i32, i32, vp, vp]
        L.mdfnn_upsample2_bwd.argtypes = [vp, i32, i32, i32, i32, vp, vp]
        L.mdfnn_add.argtypes = [vp, vp, vp, i64, vp, vp]
        L.mdfnn_head_fwd.argtypes = [vp, i32, i32, vp, vp, i32, vp, vp]
        L.mdfnn_head_scratch_bytes.argtypes = [i32, i32, i32]
        L.mdfnn_head_scratch_bytes.restype = sz
        L.mdfnn_head_bwd.argtypes = [vp, vp, i32, i32, vp, i32, vp, vp, vp, vp, vp, vp]
        L.mdfnn_loss_scratch_bytes.argtypes = [i32]
        L.mdfnn_loss_scratch_bytes.restype = sz
        L.mdfnn_mse.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp]
        L.mdfnn_mse_noalloc.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
        L.mdfnn_adam.argtypes = [vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp, vp]
        L.mdfnn_to_bf16.argtypes = [vp, i64, vp, vp]
        L.mdfnn_to_f32.argtypes = [vp, i64, vp, vp]
        for n in ("mdfnn_conv3x3_fwd", "mdfnn_conv3x3_flip", "mdfnn_conv3x3_wgrad", "mdfnn_avgpool2_fwd",
                  "mdfnn_avgpool2_bwd", "mdfnn_upsample2_fwd", "mdfnn_upsample2_bwd", "mdfnn_add",
                  "mdfnn_head_fwd", "mdfnn_head_bwd", "mdfnn_mse", "mdfnn_mse_noalloc", "mdfnn_adam",
                  "mdfnn_to_bf16", "mdfnn_to_f32"):
            getattr(L, n).restype = ctypes.c_int
        _DECLARED = True
    return L


NN_EXPORTED = ["mdfnn_conv3x3_fwd", "mdfnn_conv3x3_flip", "mdfnn_wgrad_scratch_bytes", "mdfnn_conv3x3_wgrad",
               "mdfnn_avgpool2_fwd", "mdfnn_avgpool2_bwd", "mdfnn_upsample2_fwd", "mdfnn_upsample2_bwd",
               "mdfnn_add", "mdfnn_head_fwd", "mdfnn_head_scratch_bytes", "mdfnn_head_bwd",
               "mdfnn_loss_scratch_bytes", "mdfnn_mse", "mdfnn_mse_noalloc", "mdfnn_adam", "mdfnn_to_bf16",
               "mdfnn_to_f32"]


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _st(stream):
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def _ok(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with status {rc}")


# ---------------------------------------------------------------- thin op wrappers
# bf16 tensors are torch.int16 views of the bit patterns.

def bf16_empty(shape, device):
    return torch.empty(shape, dtype=torch.int16, device=device)


def to_bf16(x: torch.Tensor, stream=None) -> torch.Tensor:
    x = x.contiguous().float()
    y = bf16_empty(x.shape, x.device)
    _ok(_lib().mdfnn_to_bf16(_p(x), x.numel(), _p(y), _st(stream)), "to_bf16")
    return y


def to_f32(x: torch.Tensor, stream=None) -> torch.Tensor:
    y = torch.empty(x.shape, dtype=torch.float32, device=x.device)
    _ok(_lib().mdfnn_to_f32(_p(x), x.numel(), _p(y), _st(stream)), "to_f32")
    return y


def conv_fwd(x1, x2, w, bias, relu, mask=None, out_bf16=None, out_f32=None, stream=None):
    B, H, W, c1 = x1.shape
    c2 = 0 if x2 is None else x2.shape[3]
    cout = w.shape[0]
    _ok(_lib().mdfnn_conv3x3_fwd(_p(x1), c1, _p(x2), c2, _p(w), _p(bias), B, H, W, cout, int(relu), _p(mask),
                                 _p(out_bf16), _p(out_f32), _st(stream)), "conv3x3_fwd")


def conv_flip(w, wt, stream=None):
    cout, _, cin = w.shape
    _ok(_lib().mdfnn_conv3x3_flip(_p(w), cout, cin, _p(wt), _st(stream)), "conv3x3_flip")


def conv_wgrad(x1, x2, dy, dw, db, scratch, stream=None):
    B, H, W, c1 = x1.shape
    c2 = 0 if x2 is None else x2.shape[3]
    _ok(_lib().mdfnn_conv3x3_wgrad(_p(x1), c1, _p(x2), c2, _p(dy), B, H, W, dy.shape[3], _p(dw), _p(db),
                                   _p(scratch), _st(stream)), "conv3x3_wgrad")


def wgrad_scratch_bytes(B, H, W, cin, cout):
    return int(_lib().mdfnn_wgrad_scratch_bytes(B, H, W, cin, cout))


def avgpool2(x, y, stream=None):
    B, H, W, C = x.shape
    _ok(_lib().mdfnn_avgpool2_fwd(_p(x), B, H, W, C, _p(y), _st(stream)), "avgpool2_fwd")


def avgpool2_bwd(dy, dx, stream=None):
    B, H, W, C = dx.shape
    _ok(_lib().mdfnn_avgpool2_bwd(_p(dy), B, H, W, C, _p(dx), _st(stream)), "avgpool2_bwd")


def upsample2(x, y, stream=None):
    B, H, W, C = x.shape
    _ok(_lib().mdfnn_upsample2_fwd(_p(x), B, H, W, C, _p(y), _st(stream)), "upsample2_fwd")


def upsample2_bwd(dy, dx, stream=None):
    B, H, W, C = dx.shape
    _ok(_lib().mdfnn_upsample2_bwd(_p(dy), B, H, W, C, _p(dx), _st(stream)), "upsample2_bwd")


def add(a, b, mask, out, stream=None):
    _ok(_lib().mdfnn_add(_p(a), _p(b), _p(mask), a.numel(), _p(out), _st(stream)), "add")


def head_fwd(x, w, b, y, stream=None):
    P = x.numel() // x.shape[-1]
    _ok(_lib().mdfnn_head_fwd(_p(x), P, x.shape[-1], _p(w), _p(b), w.shape[0], _p(y), _st(stream)), "head_fwd")


def head_bwd(x, dy, w, mask, dx, dw, db, scratch, stream=None):
    P = x.numel() // x.shape[-1]
    _ok(_lib().mdfnn_head_bwd(_p(x), _p(dy), P, x.shape[-1], _p(w), w.shape[0], _p(mask), _p(dx), _p(dw), _p(db),
                              _p(scratch), _st(stream)), "head_bwd")


def head_scratch_bytes(P, cin, cout):
    return int(_lib().mdfnn_head_scratch_bytes(P, cin, cout))


def mse(y, t, wt, dy, loss, scratch, stream=None):
    P, C = y.shape[0], y.shape[1]
    _ok(_lib().mdfnn_mse(_p(y), _p(t), _p(wt), P, C, _p(dy), _p(loss), _p(scratch), _st(stream)), "mse")


def mse_noalloc(y, t, wt, dy, loss, stream=None):
    """mse() without a scratch buffer (mdfnn_mse_noalloc): the partial sums
    live in the library's static device array; at most MSE_NOALLOC_MAX_P
    pixels."""
    P, C = y.shape[0], y.shape[1]
    _ok(_lib().mdfnn_mse_noalloc(_p(y), _p(t), _p(wt), P, C, _p(dy), _p(loss), _st(stream)), "mse_noalloc")


MSE_NOALLOC_MAX_P = 1 << 23


def loss_scratch_bytes(P):
    return int(_lib().mdfnn_loss_scratch_bytes(P))


def adam(p, g, m, v, lr, t, p_bf16=None, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    _ok(_lib().mdfnn_adam(_p(p), _p(g), _p(m), _p(v), p.numel(), lr, b1, b2, eps, int(t), _p(p_bf16),
                          _st(stream)), "adam")


# ---------------------------------------------------------------- the network

class UNet:
    """Encoder: at level l two 3x3 convs (ReLU) then 2x2 average pooling
    (not after the last level).  Decoder: nearest 2x up-sampling, channel
    concatenation with the encoder output of the same level, two 3x3 convs
    (ReLU).  Head: 1x1 conv to OUT_CH channels (FP32).  Parameters live in
    one flat FP32 buffer (master weights) with a BF16 mirror for the
    matrix-core products."""

    def __init__(self, device="cuda:0", seed=0, levels=LEVELS):
        self.device = torch.device(device)
        self.levels = levels
        specs = []        # (name, cin1, cin2, cout)
        cin = IN_CH
        for l, c in enumerate(levels):
            specs.append((f"enc{l}a", cin, 0, c))
            specs.append((f"enc{l}b", c, 0, c))
            cin = c
        for l in range(len(levels) - 2, -1, -1):
            c = levels[l]
            specs.append((f"dec{l}a", levels[l + 1], c, c))
            specs.append((f"dec{l}b", c, 0, c))
        self.convs = specs
        self.layout: Dict[str, Tuple[int, Tuple[int, ...]]] = {}
        off = 0
        for name, c1, c2, co in specs:
            self.layout[name + ".w"] = (off, (co, 9, c1 + c2))
            off += co * 9 * (c1 + c2)
            self.layout[name + ".b"] = (off, (co,))
            off += co
        self.layout["head.w"] = (off, (OUT_CH, levels[0]))
        off += OUT_CH * levels[0]
        self.layout["head.b"] = (off, (OUT_CH,))
        off += OUT_CH
        self.nparams = off
        rng = np.random.default_rng(seed)
        flat = np.zeros(off, np.float32)
        for name, c1, c2, co in specs:
            o, shp = self.layout[name + ".w"]
            fan_in = 9 * (c1 + c2)
            flat[o:o + np.prod(shp)] = rng.normal(0, math.sqrt(2.0 / fan_in), size=np.prod(shp))
        o, shp = self.layout["head.w"]
        flat[o:o + np.prod(shp)] = rng.normal(0, math.sqrt(1.0 / levels[0]), size=np.prod(shp))
        self.params = torch.tensor(flat, device=self.device)
        self.params_bf16 = to_bf16(self.params)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_count = 0
        self.norm = {"mean": np.zeros(OUT_CH, np.float32), "std": np.ones(OUT_CH, np.float32)}
        self._bufs = {}

    # views into the flat buffers
    def view(self, name, which="f32"):
        o, shp = self.layout[name]
        n = int(np.prod(shp))
        src = {"f32": self.params, "bf16": self.params_bf16, "grad": self.grads}[which]
        return src[o:o + n].view(shp)

    def state_dict(self):
        return {"params": self.params.cpu().numpy(), "mean": self.norm["mean"], "std": self.norm["std"],
                "levels": np.array(self.levels)}

    def load_state_dict(self, d):
        self.params.copy_(torch.tensor(d["params"], device=self.device))
        self.params_bf16 = to_bf16(self.params)
        self.norm = {"mean": np.asarray(d["mean"], np.float32), "std": np.asarray(d["std"], np.float32)}

    # -------------------------------------------------------------- buffers
    def _buffers(self, B, H, W):
        key = (B, H, W)
        if key in self._bufs:
            return self._bufs[key]
        dev = self.device
        bf = {}
        h, w = H, W
        for l, c in enumerate(self.levels):
            bf[f"enc{l}a"] = bf16_empty((B, h, w, c), dev)
            bf[f"enc{l}b"] = bf16_empty((B, h, w, c), dev)
            bf[f"g_enc{l}a"] = bf16_empty((B, h, w, c), dev)
            bf[f"g_enc{l}b"] = bf16_empty((B, h, w, c), dev)
            if l + 1 < len(self.levels):
                bf[f"pool{l}"] = bf16_empty((B, h // 2, w // 2, c), dev)
                bf[f"g_pool{l}"] = bf16_empty((B, h // 2, w // 2, c), dev)
                bf[f"g_skip{l}"] = bf16_empty((B, h, w, c), dev)
                bf[f"g_tmp{l}"] = bf16_empty((B, h, w, c), dev)
                h, w = h // 2, w // 2
        h, w = H, W
        for l in range(len(self.levels) - 1):
            c_up = self.levels[l + 1]
            c = self.levels[l]
            hh, ww = H >> l, W >> l
            bf[f"up{l}"] = bf16_empty((B, hh, ww, c_up), dev)
            bf[f"g_up{l}"] = bf16_empty((B, hh, ww, c_up), dev)
            bf[f"dec{l}a"] = bf16_empty((B, hh, ww, c), dev)
            bf[f"dec{l}b"] = bf16_empty((B, hh, ww, c), dev)
            bf[f"g_dec{l}a"] = bf16_empty((B, hh, ww, c), dev)
            bf[f"g_dec{l}b"] = bf16_empty((B, hh, ww, c), dev)
        P = B * H * W
        bf["out"] = torch.empty((P, OUT_CH), dtype=torch.float32, device=dev)
        bf["g_out"] = torch.empty((P, OUT_CH), dtype=torch.float32, device=dev)
        bf["loss"] = torch.zeros(1, dtype=torch.float32, device=dev)
        maxw = max(wgrad_scratch_bytes(B, H >> l, W >> l, c1 + c2, co)
                   for l_name, c1, c2, co in self.convs
                   for l in [int(l_name[3])])
        bf["scratch"] = torch.empty(max(maxw, head_scratch_bytes(P, self.levels[0], OUT_CH),
                                        loss_scratch_bytes(P)), dtype=torch.uint8, device=dev)
        cmax = max((c1 + c2) * co * 9 for _, c1, c2, co in self.convs)
        bf["wt"] = bf16_empty((cmax,), dev)
        self._bufs[key] = bf
        return bf

    # -------------------------------------------------------------- forward
    def forward(self, x, stream=None):
        """x: bf16 [B, H, W, IN_CH] (H, W divisible by 2^(levels-1)).
        Returns the FP32 output [B*H*W, OUT_CH] (normalised targets)."""
        B, H, W, _ = x.shape
        bf = self._buffers(B, H, W)
        inp = x
        nl = len(self.levels)
        for l in range(nl):
            conv_fwd(inp, None, self.view(f"enc{l}a.w", "bf16"), self.view(f"enc{l}a.b"), True,
                     out_bf16=bf[f"enc{l}a"], stream=stream)
            conv_fwd(bf[f"enc{l}a"], None, self.view(f"enc{l}b.w", "bf16"), self.view(f"enc{l}b.b"), True,
                     out_bf16=bf[f"enc{l}b"], stream=stream)
            if l + 1 < nl:
                avgpool2(bf[f"enc{l}b"], bf[f"pool{l}"], stream)
                inp = bf[f"pool{l}"]
        low = bf[f"enc{nl - 1}b"]
        for l in range(nl - 2, -1, -1):
            upsample2(low, bf[f"up{l}"], stream)
            conv_fwd(bf[f"up{l}"], bf[f"enc{l}b"], self.view(f"dec{l}a.w", "bf16"), self.view(f"dec{l}a.b"), True,
                     out_bf16=bf[f"dec{l}a"], stream=stream)
            conv_fwd(bf[f"dec{l}a"], None, self.view(f"dec{l}b.w", "bf16"), self.view(f"dec{l}b.b"), True,
                     out_bf16=bf[f"dec{l}b"], stream=stream)
            low = bf[f"dec{l}b"]
        head_fwd(low, self.view("head.w"), self.view("head.b"), bf["out"], stream)
        self._last_input = x
        return bf["out"]

    # -------------------------------------------------------------- backward
    def _conv_back(self, name, x1, x2, gy, gx1, gx1_mask, gx2, stream):
        """gy: gradient at this conv's output already multiplied by the ReLU
        derivative; accumulates the weight/bias gradients; writes the input
        gradients (masked by gx1_mask if given) unless gx1 is None."""
        B, H, W, _ = x1.shape
        bf = self._buffers(*self._last_input.shape[:3])
        conv_wgrad(x1, x2, gy, self.view(name + ".w", "grad"), self.view(name + ".b", "grad"), bf["scratch"],
                   stream)
        if gx1 is None:
            return
        w = self.view(name + ".w", "bf16")
        cout, _, cin = w.shape
        wt = bf["wt"][: cout * 9 * cin].view(cin, 9, cout)
        conv_flip(w, wt, stream)
        c1 = x1.shape[3]
        conv_fwd(gy, None, wt[:c1], None, False, mask=gx1_mask, out_bf16=gx1, stream=stream)
        if x2 is not None:
            conv_fwd(gy, None, wt[c1:], None, False, mask=None, out_bf16=gx2, stream=stream)

    def backward(self, g_out, stream=None):
        """g_out: FP32 [P, OUT_CH] gradient of the loss at the output.  Fills
        self.grads."""
        x = self._last_input
        B, H, W, _ = x.shape
        bf = self._buffers(B, H, W)
        nl = len(self.levels)
        top = bf["dec0b"] if nl > 1 else bf["enc0b"]
        g_top = bf["g_dec0b"] if nl > 1 else bf["g_enc0b"]
        head_bwd(top, g_out, self.view("head.w"), top, g_top, self.view("head.w", "grad"),
                 self.view("head.b", "grad"), bf["scratch"], stream)
        # decoder, top to bottom
        for l in range(0, nl - 1):
            self._conv_back(f"dec{l}b", bf[f"dec{l}a"], None, bf[f"g_dec{l}b"], bf[f"g_dec{l}a"], bf[f"dec{l}a"],
                            None, stream)
            self._conv_back(f"dec{l}a", bf[f"up{l}"], bf[f"enc{l}b"], bf[f"g_dec{l}a"], bf[f"g_up{l}"], None,
                            bf[f"g_skip{l}"], stream)
            if l + 1 < nl - 1:
                upsample2_bwd(bf[f"g_up{l}"], bf[f"g_dec{l + 1}b"], stream)
                add(bf[f"g_dec{l + 1}b"], None, bf[f"dec{l + 1}b"], bf[f"g_dec{l + 1}b"], stream)
            else:
                upsample2_bwd(bf[f"g_up{l}"], bf[f"g_enc{nl - 1}b"], stream)
                add(bf[f"g_enc{nl - 1}b"], None, bf[f"enc{nl - 1}b"], bf[f"g_enc{nl - 1}b"], stream)
        # encoder, bottom to top
        for l in range(nl - 1, -1, -1):
            if l < nl - 1:
                # output of enc{l}b feeds the pool (gradient from level l+1) and the skip
                avgpool2_bwd(bf[f"g_pool{l}"], bf[f"g_tmp{l}"], stream)
                add(bf[f"g_tmp{l}"], bf[f"g_skip{l}"], bf[f"enc{l}b"], bf[f"g_enc{l}b"], stream)
            self._conv_back(f"enc{l}b", bf[f"enc{l}a"], None, bf[f"g_enc{l}b"], bf[f"g_enc{l}a"], bf[f"enc{l}a"],
                            None, stream)
            if l > 0:
                self._conv_back(f"enc{l}a", bf[f"pool{l - 1}"], None, bf[f"g_enc{l}a"], bf[f"g_pool{l - 1}"], None,
                                None, stream)
            else:
                self._conv_back("enc0a", x, None, bf["g_enc0a"], None, None, None, stream)

    def adam_step(self, lr, stream=None):
        self.step_count += 1
        adam(self.params, self.grads, self.m, self.v, lr, self.step_count, self.params_bf16, stream=stream)

    def loss_and_grad(self, target, weight, stream=None):
        bf = self._buffers(*self._last_input.shape[:3])
        mse(bf["out"], target, weight, bf["g_out"], bf["loss"], bf["scratch"], stream)
        return bf["loss"], bf["g_out"]


# ---------------------------------------------------------------- data

def input_features(N, mask, Re, U, coarse=None, coarse2=None):
    """Per-node features: solid flag, (log10 Re - 2), U / 0.1 - 0.75, the
    node coordinates in [-1, 1] and the distance to the nearest solid node or
    cavity wall (in units of N; 0 inside solids); optionally one or two
    interpolated coarse-grid solutions with their flags; zero-padded to IN_CH
    channels.  Returns float32 [N, N, IN_CH] ([y, x, c])."""
    from scipy.ndimage import distance_transform_edt
    f = np.zeros((N, N, IN_CH), np.float32)
    f[..., 0] = mask.astype(np.float32)
    f[..., 1] = math.log10(Re) - 2.0
    f[..., 2] = U / 0.1 - 0.75
    c = (np.arange(N) + 0.5) / N * 2 - 1
    f[..., 3] = c[None, :]
    f[..., 4] = c[:, None]
    # walls sit halfway outside the first and last nodes: a solid ring one
    # node wide around the grid, distances shifted by the half node
    fluid = np.zeros((N + 2, N + 2), bool)
    fluid[1:-1, 1:-1] = mask == 0
    d = distance_transform_edt(fluid)[1:-1, 1:-1]
    f[..., 5] = np.where(mask == 0, (d - 0.5) / N, 0.0)
    if coarse is not None:
        # an interpolated coarse-grid steady solution in the scales of
        # raw_targets ([N, N, OUT_CH]) and a flag saying it exists
        f[..., FEATURES:FEATURES + OUT_CH] = coarse
        f[..., FEATURES + OUT_CH] = 1.0
    if coarse2 is not None:
        # a second, coarser solution in the same scales: with the first it
        # tells the network how the solution moves with the grid spacing
        k = FEATURES + COARSE_FEATURES
        f[..., k:k + OUT_CH] = coarse2
        f[..., k + OUT_CH] = 1.0
    return f


def raw_targets(fields: Dict[str, torch.Tensor], N, U, Re):
    """Steady fields of one case in scales that keep every case O(1):
    P Re / U^2 (the cavity pressure of this scheme follows the viscous
    scaling P ~ U^2 / Re over the whole Re range), u / U, v / U and
    grad u * N / U, as float32 [N, N, OUT_CH]."""
    P = fields["P"] - fields["P"].mean()
    g = fields["grad"]
    out = torch.stack([P * (Re / (U * U)), fields["u"][0] / U, fields["u"][1] / U,
                       g[0, 0] * N / U, g[0, 1] * N / U, g[1, 0] * N / U, g[1, 1] * N / U], dim=-1)
    return out.float()


def scaled_fields(fl: np.ndarray, N, U, Re, mask) -> np.ndarray:
    """Channel-major [P, u, v, grad(4)] fields in lattice units -> the scales
    of raw_targets, [N, N, OUT_CH] float32 (P with its fluid mean removed)."""
    fluid = mask == 0
    out = np.zeros((N, N, OUT_CH), np.float32)
    P = fl[0] - (fl[0][fluid].mean() if fluid.any() else 0.0)
    out[..., 0] = P * (Re / (U * U))
    out[..., 1] = fl[1] / U
    out[..., 2] = fl[2] / U
    for k in range(4):
        out[..., 3 + k] = fl[3 + k] * N / U
    return out


def fields_from_prediction(pred: np.ndarray, N, U, Re, mask, norm, base=None):
    """Inverse of raw_targets for one case: [N, N, OUT_CH] normalised
    network output (plus `base`, a field in target scales, when the network
    predicts a correction to it) -> channel-major [P, u, v, grad(4)] init
    data (float64) with solid nodes zeroed."""
    y = pred * norm["std"] + norm["mean"]
    if base is not None:
        y = y + base
    fl = np.zeros((7, N, N))
    fl[0] = y[..., 0] * (U * U / Re)
    fl[1] = y[..., 1] * U
    fl[2] = y[..., 2] * U
    for k in range(4):
        fl[3 + k] = y[..., 3 + k] * U / N
    # the gradient from the network need not be trace-free; remove the
    # divergence so that the initial pressure is not shifted (eq. 3-15)
    div = fl[3] + fl[6]
    fl[3] -= 0.5 * div
    fl[6] -= 0.5 * div
    fl[:, mask.astype(bool)] = 0.0
    return fl
