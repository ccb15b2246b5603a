"""FP64 CPU oracle for the learned initialiser's network.

TEST INFRASTRUCTURE ONLY, like ``msl_oracle``: only the test-suite, the
package smoke check and the benchmark's ``cpu_baseline`` leg may import it.
It shares no code with the HIP path.

The network is not part of the paper: it supplies the initial guess that the
paper's gradient reconstruction (Sec. 4.1) refines.  This module defines it
plainly: 3x3 convolutions with zero padding (stride 1 or 2) by their
definition (a sum over the nine taps of shifted inputs), ReLU, nearest 2x
upsampling, channel concatenation, a row mean, the mean squared error, and
their adjoints, all in float64; and the global head: per-row summaries of the
input image (means and the centre column), two dense layers, and the
broadcast of its output along the columns.

Where the library rounds to bfloat16 (the matrix-core inputs: activations and
weights entering a convolution, and the output gradient entering the
backward products) this oracle rounds the same values the same way (round to
nearest even, from float32), so both sides take that quantisation decision in
the same precision; everything else is float64 here and float32 there.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to bfloat16 (nearest even) from float32, returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    special = (u & 0x7F800000) == 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(special, u & 0xFFFF0000, r).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def conv3x3(x, w, bias=None, stride=1):
    """y[o, b, i, j] = sum_c sum_{dy, dx in -1..1} w[o, c, dy+1, dx+1] x[c, b, s i + dy, s j + dx] (+ bias[o]),
    x [C][B][H][W] zero outside, w [O][C][3][3]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    C, B, H, W = x.shape
    Ho, Wo = H // stride, W // stride
    xp = np.zeros((C, B, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    y = np.zeros((w.shape[0], B, Ho, Wo))
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + stride * Ho:stride, dx:dx + stride * Wo:stride]
            y += np.einsum("oc,cbij->obij", w[:, :, dy, dx], patch)
    if bias is not None:
        y += np.asarray(bias, np.float64)[:, None, None, None]
    return y


def conv3x3_adjoint(x, w, dy, stride=1):
    """(dL/dx, dL/dw, dL/dbias) of ``conv3x3`` given dL/dy."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    dy = np.asarray(dy, np.float64)
    C, B, H, W = x.shape
    Ho, Wo = H // stride, W // stride
    xp = np.zeros((C, B, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ty in range(3):
        for tx in range(3):
            sl = (slice(None), slice(None), slice(ty, ty + stride * Ho, stride), slice(tx, tx + stride * Wo, stride))
            dw[:, :, ty, tx] = np.einsum("obij,cbij->oc", dy, xp[sl])
            dxp[sl] += np.einsum("oc,obij->cbij", w[:, :, ty, tx], dy)
    return dxp[:, :, 1:H + 1, 1:W + 1], dw, dy.sum(axis=(1, 2, 3))


def relu(x):
    return np.maximum(x, 0.0)


def upsample2(x):
    return np.repeat(np.repeat(np.asarray(x, np.float64), 2, axis=2), 2, axis=3)


def upsample2_adjoint(dy):
    d = np.asarray(dy, np.float64)
    return d[:, :, 0::2, 0::2] + d[:, :, 0::2, 1::2] + d[:, :, 1::2, 0::2] + d[:, :, 1::2, 1::2]


def rowpool(x, f):
    """[B][H][W] -> [B][H/f][W], mean of f consecutive rows."""
    x = np.asarray(x, np.float64)
    B, H, W = x.shape
    return x.reshape(B, H // f, f, W).mean(axis=2)


def rowpool_adjoint(dy, f):
    return np.repeat(np.asarray(dy, np.float64), f, axis=1) / f


def row_features(x0):
    """x0 [B][H][W] -> [B][3H]: per row the mean over all columns, the centre column W/2, and the
    mean over the seven columns W/2-3 .. W/2+3."""
    x0 = np.asarray(x0, np.float64)
    B, H, W = x0.shape
    c = W // 2
    return np.concatenate([x0.mean(axis=2), x0[:, :, c], x0[:, :, c - 3:c + 4].mean(axis=2)], axis=1)


def add_row_bias(y, p):
    """y [B][R][W] + p[r][b] at every column."""
    return np.asarray(y, np.float64) + np.asarray(p, np.float64).T[:, :, None]


def add_row_bias_adjoint(dy):
    """dL/dp [R][B] from dL/dy [B][R][W]."""
    return np.asarray(dy, np.float64).sum(axis=2).T


def mse(p, t):
    d = np.asarray(p, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


# ---------------------------------------------------------------------------
# the network: a four-level U-Net, channels c, 2c, 4c, 8c

def layer_specs(c=32, in_ch=2):
    """(name, in channels, out channels, stride, relu) of every convolution, in order."""
    c1, c2, c3, c4 = c, 2 * c, 4 * c, 8 * c
    return [("e1a", in_ch, c1, 1, True), ("e1b", c1, c1, 1, True),
            ("e2a", c1, c2, 2, True), ("e2b", c2, c2, 1, True),
            ("e3a", c2, c3, 2, True), ("e3b", c3, c3, 1, True),
            ("e4a", c3, c4, 2, True), ("e4b", c4, c4, 1, True),
            ("d3", c4 + c3, c3, 1, True), ("d2", c3 + c2, c2, 1, True), ("d1", c2 + c1, c1, 1, True),
            ("out", c1, 1, 1, False)]


def unet_forward(params, x, rows_per_output=4, quantize=True, offset=None, feat_norm=None):
    """x [C][B][H][W] -> pred [B][H/rows_per_output][W] (+ offset [H/rows_per_output][W]);
    params[name] = (w [O][C][3][3], bias [O]) for the convolutions, and optionally the global
    head "g1" (w [hidden][3H], bias [hidden]; ReLU) and "g2" (w [H/rows_per_output][hidden],
    bias [H/rows_per_output]); feat_norm = (shift [3H], scale [3H]) normalises the head's inputs.
    Returns (pred, cache) for ``unet_adjoint``.  quantize=False skips the bfloat16 rounding
    (the exact function, for finite-difference checks)."""
    q = bf16 if quantize else (lambda a: np.asarray(a, np.float64))
    cache = {"q": q}

    def conv(name, inp, stride, act):
        w, b = params[name]
        xin = q(inp)
        y = conv3x3(xin, q(w), b, stride)
        y = relu(y) if act else y
        cache[name] = (xin, y, stride, act)
        return y

    e1 = conv("e1b", conv("e1a", x, 1, True), 1, True)
    e2 = conv("e2b", conv("e2a", e1, 2, True), 1, True)
    e3 = conv("e3b", conv("e3a", e2, 2, True), 1, True)
    e4 = conv("e4b", conv("e4a", e3, 2, True), 1, True)
    d3 = conv("d3", np.concatenate([upsample2(e4), e3]), 1, True)
    d2 = conv("d2", np.concatenate([upsample2(d3), e2]), 1, True)
    d1 = conv("d1", np.concatenate([upsample2(d2), e1]), 1, True)
    out = conv("out", d1, 1, False)
    pred = rowpool(out[0], rows_per_output)
    if "g1" in params:
        # global head: dense layers on shift-invariant row summaries of the first input channel,
        # its output added to every column of the corresponding output row
        (w1, b1), (w2, b2) = params["g1"], params["g2"]
        feat = row_features(x[0])                        # [B][3H]
        if feat_norm is not None:
            feat = (feat - np.asarray(feat_norm[0], np.float64)) * np.asarray(feat_norm[1], np.float64)
        feat = q(feat)
        h1 = relu(q(w1) @ feat.T + np.asarray(b1, np.float64)[:, None])   # [hidden][B]
        h1q = q(h1)
        p = q(w2) @ h1q + np.asarray(b2, np.float64)[:, None]              # [R][B]
        pred = add_row_bias(pred, p)
        cache["head"] = (feat, h1, h1q)
    if offset is not None:
        pred = pred + np.asarray(offset, np.float64)[None]
    cache["shapes"] = {"e4": e4.shape[0], "d3": d3.shape[0], "d2": d2.shape[0]}
    return pred, cache


def unet_adjoint(params, cache, dpred, rows_per_output=4):
    """Gradients {name: (dw, dbias)} of a loss with dL/dpred through ``unet_forward``."""
    grads = {}
    q = cache["q"]

    def back(name, dy):
        xin, y, stride, act = cache[name]
        if act:
            dy = dy * (y > 0)
        w, _ = params[name]
        dx, dw, _ = conv3x3_adjoint(xin, q(w), q(dy), stride)
        grads[name] = (dw, dy.sum(axis=(1, 2, 3)))
        return dx

    ch = cache["shapes"]
    if "head" in cache:
        feat, h1, h1q = cache["head"]
        w2, _ = params["g2"]
        dp = add_row_bias_adjoint(dpred)                 # [R][B]
        grads["g2"] = (q(dp) @ h1q.T, dp.sum(axis=1))
        dh1 = (q(w2).T @ q(dp)) * (h1 > 0)
        grads["g1"] = (q(dh1) @ feat, dh1.sum(axis=1))
    dout = rowpool_adjoint(dpred, rows_per_output)[None]
    dd1 = back("out", dout)
    dcat = back("d1", dd1)
    dd2, de1 = upsample2_adjoint(dcat[:ch["d2"]]), dcat[ch["d2"]:]
    dcat = back("d2", dd2)
    dd3, de2 = upsample2_adjoint(dcat[:ch["d3"]]), dcat[ch["d3"]:]
    dcat = back("d3", dd3)
    de4, de3 = upsample2_adjoint(dcat[:ch["e4"]]), dcat[ch["e4"]:]
    de3 = de3 + back("e4a", back("e4b", de4))
    de2 = de2 + back("e3a", back("e3b", de3))
    de1 = de1 + back("e2a", back("e2b", de2))
    back("e1a", back("e1b", de1))
    return grads
