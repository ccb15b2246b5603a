"""ctypes binding of the learned-initialiser kernels (C ABI in include/msl_nn.h).

Argument marshalling only: every operation runs in libmsl.  Tensors are
device tensors; bfloat16 arrays are torch.int16 / torch.uint16-compatible
16-bit tensors holding the bfloat16 bit patterns (torch.int16 is used).
"""
from __future__ import annotations

import ctypes
from ctypes import c_double, c_float, c_int32, c_int64, c_void_p

import torch

from . import msl

EXPORTS = ("msl_nn_gemm_bf16", "msl_nn_gemm_bf16_splitk", "msl_nn_im2col3x3", "msl_nn_col2im3x3", "msl_nn_upsample2",
           "msl_nn_upsample2_adjoint", "msl_nn_rowpool", "msl_nn_rowpool_adjoint", "msl_nn_relu_adjoint",
           "msl_nn_add", "msl_nn_to_bf16", "msl_nn_rowsum", "msl_nn_mse", "msl_nn_adam", "msl_nn_logmap",
           "msl_nn_render_pools", "msl_nn_pool_average", "msl_nn_row_features", "msl_nn_add_row_bias",
           "msl_nn_row_bias_adjoint", "msl_nn_conv3x3", "msl_nn_conv3x3_adjoint", "msl_nn_conv3x3_weight_grad",
           "msl_nn_conv3x3_scratch_elems", "msl_nn_grad_prep")

MAX_BOXES = 64   # MSL_NN_MAX_BOXES
MAX_CUTS = 132   # MSL_NN_MAX_CUTS

_ready = False


def lib():
    global _ready
    L = msl.lib()
    if not _ready:
        P = c_void_p
        I = c_int32
        sig = {
            "msl_nn_gemm_bf16": [I, I, I, P, I, I, P, I, I, P, I, c_float, P, I, P, P],
            "msl_nn_gemm_bf16_splitk": [I, I, I, P, I, I, P, I, I, P, I, I, P, P],
            "msl_nn_im2col3x3": [I, I, I, I, I, P, P, P],
            "msl_nn_col2im3x3": [I, I, I, I, I, P, P, P],
            "msl_nn_upsample2": [I, I, I, I, P, P, I, P],
            "msl_nn_upsample2_adjoint": [I, I, I, I, P, P, P],
            "msl_nn_rowpool": [I, I, I, I, P, P, P],
            "msl_nn_rowpool_adjoint": [I, I, I, I, P, P, P],
            "msl_nn_relu_adjoint": [c_int64, P, P, P],
            "msl_nn_add": [c_int64, P, P, P],
            "msl_nn_to_bf16": [c_int64, P, P, P],
            "msl_nn_rowsum": [I, I, P, P, P, P],
            "msl_nn_mse": [c_int64, P, P, P, P, P, P],
            "msl_nn_adam": [c_int64, P, P, P, P, P, c_float, c_float, c_float, c_float, I, P],
            "msl_nn_logmap": [c_int64, P, c_float, c_float, c_float, P, P],
            "msl_nn_render_pools": [I, I, I, I, c_float, c_float, P, P, P, P, P, I, P, P, P],
            "msl_nn_pool_average": [I, I, I, I, I, P, P, P, I, P, c_float, P, P],
            "msl_nn_row_features": [I, I, I, P, P, P, P, P],
            "msl_nn_add_row_bias": [I, I, I, P, P, P],
            "msl_nn_row_bias_adjoint": [I, I, I, P, P, P],
            "msl_nn_conv3x3": [I, I, I, I, I, I, P, P, I, P, I, P, I, P, P],
            "msl_nn_conv3x3_adjoint": [I, I, I, I, I, I, P, P, P, I, P, P],
            "msl_nn_conv3x3_weight_grad": [I, I, I, I, I, I, P, P, I, P, I, P, P],
            "msl_nn_grad_prep": [I, I, P, I, P, P, P, P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.restype = c_int32
            f.argtypes = args
        L.msl_nn_conv3x3_scratch_elems.restype = c_int64
        L.msl_nn_conv3x3_scratch_elems.argtypes = [I, I]
        _ready = True
    return L


def _p(t, dtype=None):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


def _ck(st):
    msl._check(st)


def _s():
    return msl._stream()


BF16 = torch.int16   # storage dtype of bfloat16 bit patterns


def _act(t):
    """(pointer, 1 if bfloat16 bits) of an activation held as float32 or as bfloat16 bits."""
    if t is None:
        return None, 0
    if t.dtype == BF16:
        return _p(t, BF16), 1
    return _p(t, torch.float32), 0


def gemm(M, N, K, A, lda, transA, B, ldb, transB, C, ldc, beta=0.0, bias=None, relu=False, C16=None):
    _ck(lib().msl_nn_gemm_bf16(M, N, K, _p(A, BF16), lda, int(transA), _p(B, BF16), ldb, int(transB),
                               _p(C, torch.float32), ldc, float(beta), _p(bias, torch.float32), int(relu),
                               _p(C16, BF16), _s()))


def gemm_splitk(M, N, K, A, lda, transA, B, ldb, transB, C, ldc, splits, partials):
    _ck(lib().msl_nn_gemm_bf16_splitk(M, N, K, _p(A, BF16), lda, int(transA), _p(B, BF16), ldb, int(transB),
                                      _p(C, torch.float32), ldc, int(splits), _p(partials, torch.float32), _s()))


_scratch = {}


def conv_scratch(Co, C, device):
    """Packed-weight scratch of msl_nn_conv3x3 / _adjoint (msl_nn_conv3x3_scratch_elems), one growing
    buffer per device, reused by every call on it (the calls of one stream run in order)."""
    n = int(lib().msl_nn_conv3x3_scratch_elems(Co, C))
    buf = _scratch.get(device)
    if buf is None or buf.numel() < n:
        buf = torch.empty(max(n, 1 << 16), dtype=BF16, device=device)
        _scratch[device] = buf
    return buf


def conv3x3(Co, C, B, H, W, stride, w16, x, y, bias=None, relu=False, scratch=None):
    """msl_nn_conv3x3; x and y each float32 or bfloat16 bits (BF16 storage)."""
    ws = scratch if scratch is not None else conv_scratch(Co, C, x.device)
    xp, xb = _act(x)
    yp, yb = _act(y)
    _ck(lib().msl_nn_conv3x3(Co, C, B, H, W, stride, _p(w16, BF16), xp, xb, _p(bias, torch.float32),
                             int(relu), yp, yb, _p(ws, BF16), _s()))


def conv3x3_adjoint(Co, C, B, H, W, stride, w16, dy16, dx, scratch=None, accumulate=False):
    ws = scratch if scratch is not None else conv_scratch(Co, C, dx.device)
    _ck(lib().msl_nn_conv3x3_adjoint(Co, C, B, H, W, stride, _p(w16, BF16), _p(dy16, BF16), _p(dx, torch.float32),
                                     int(accumulate), _p(ws, BF16), _s()))


def grad_prep(M, N, y, dy, dy16, bias_grad, parts):
    """msl_nn_grad_prep: dy16 = bf16(dy masked by y > 0, or unmasked when y is None), bias_grad = row sums;
    y float32 or bfloat16 bits."""
    yp, yb = _act(y)
    _ck(lib().msl_nn_grad_prep(M, N, yp, yb, _p(dy, torch.float32), _p(dy16, BF16),
                               _p(bias_grad, torch.float32), _p(parts, torch.float32), _s()))


def conv3x3_weight_grad(Co, C, B, H, W, stride, dy16, x, dw, splits, partials):
    """msl_nn_conv3x3_weight_grad; x float32 or bfloat16 bits."""
    xp, xb = _act(x)
    _ck(lib().msl_nn_conv3x3_weight_grad(Co, C, B, H, W, stride, _p(dy16, BF16), xp, xb,
                                         _p(dw, torch.float32), int(splits), _p(partials, torch.float32), _s()))


def im2col(C, B, H, W, stride, x, col):
    _ck(lib().msl_nn_im2col3x3(C, B, H, W, stride, _p(x, torch.float32), _p(col, BF16), _s()))


def col2im(C, B, H, W, stride, col, dx):
    _ck(lib().msl_nn_col2im3x3(C, B, H, W, stride, _p(col, torch.float32), _p(dx, torch.float32), _s()))


def upsample2(C, B, H, W, x, y):
    """msl_nn_upsample2; x and y both float32 or both bfloat16 bits."""
    xp, xb = _act(x)
    yp, yb = _act(y)
    if xb != yb:
        raise ValueError("upsample2: x and y must have the same dtype")
    _ck(lib().msl_nn_upsample2(C, B, H, W, xp, yp, xb, _s()))


def upsample2_adjoint(C, B, H, W, dy, dx):
    _ck(lib().msl_nn_upsample2_adjoint(C, B, H, W, _p(dy, torch.float32), _p(dx, torch.float32), _s()))


def rowpool(B, H, W, f, x, y):
    _ck(lib().msl_nn_rowpool(B, H, W, f, _p(x, torch.float32), _p(y, torch.float32), _s()))


def rowpool_adjoint(B, H, W, f, dy, dx):
    _ck(lib().msl_nn_rowpool_adjoint(B, H, W, f, _p(dy, torch.float32), _p(dx, torch.float32), _s()))


def row_features(B, H, W, x, f16, shift=None, scale=None):
    _ck(lib().msl_nn_row_features(B, H, W, _p(x, torch.float32), _p(shift, torch.float32),
                                  _p(scale, torch.float32), _p(f16, BF16), _s()))


def add_row_bias(B, R, W, p, y):
    _ck(lib().msl_nn_add_row_bias(B, R, W, _p(p, torch.float32), _p(y, torch.float32), _s()))


def row_bias_adjoint(B, R, W, dy, dp):
    _ck(lib().msl_nn_row_bias_adjoint(B, R, W, _p(dy, torch.float32), _p(dp, torch.float32), _s()))


def relu_adjoint(y, dy):
    _ck(lib().msl_nn_relu_adjoint(y.numel(), _p(y, torch.float32), _p(dy, torch.float32), _s()))


def add_(x, y):
    _ck(lib().msl_nn_add(x.numel(), _p(x, torch.float32), _p(y, torch.float32), _s()))


def to_bf16(x, y16):
    _ck(lib().msl_nn_to_bf16(x.numel(), _p(x, torch.float32), _p(y16, BF16), _s()))


def rowsum(M, N, X, out, parts):
    """parts: float32 scratch of at least M * 64 values."""
    _ck(lib().msl_nn_rowsum(M, N, _p(X, torch.float32), _p(out, torch.float32), _p(parts, torch.float32), _s()))


_mse_parts = {}


def mse(pred, target, grad, loss):
    parts = _mse_parts.get(pred.device)
    if parts is None:
        parts = torch.empty(256, dtype=torch.float64, device=pred.device)
        _mse_parts[pred.device] = parts
    _ck(lib().msl_nn_mse(pred.numel(), _p(pred, torch.float32), _p(target, torch.float32),
                         _p(grad, torch.float32), _p(loss, torch.float64), _p(parts, torch.float64), _s()))


def adam(w, g, m, v, w16, lr, beta1, beta2, eps, t):
    _ck(lib().msl_nn_adam(w.numel(), _p(w, torch.float32), _p(g, torch.float32), _p(m, torch.float32),
                          _p(v, torch.float32), _p(w16, BF16), float(lr), float(beta1), float(beta2), float(eps),
                          int(t), _s()))


def logmap(x, eps, a, b, out):
    _ck(lib().msl_nn_logmap(x.numel(), _p(x, torch.float32), float(eps), float(a), float(b),
                            _p(out, torch.float32), _s()))


def render_pools(n_samples, ny, nz, substrate_rows, sub_delta, sub_beta, boxes, nf, cuts, npool, pool_off,
                 max_pool, pool_delta, pool_beta):
    _ck(lib().msl_nn_render_pools(n_samples, ny, nz, substrate_rows, float(sub_delta), float(sub_beta),
                                  _p(boxes, torch.float32), _p(nf, torch.int32), _p(cuts, torch.int32),
                                  _p(npool, torch.int32), _p(pool_off, torch.int64), max_pool,
                                  _p(pool_delta, torch.float32), _p(pool_beta, torch.float32), _s()))


def pool_average(n_samples, ny, nz, y0, rows, w, npool, pool_off, max_pool, pool, scale, out):
    _ck(lib().msl_nn_pool_average(n_samples, ny, nz, y0, rows, _p(w, torch.float32), _p(npool, torch.int32),
                                  _p(pool_off, torch.int64), max_pool, _p(pool, torch.float32), float(scale),
                                  _p(out, torch.float32), _s()))
