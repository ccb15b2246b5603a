"""Learned initialiser for the gradient reconstruction (NEXT to the paper's Sec. 4.1).

A four-level U-Net (channels c, 2c, 4c, 8c; 3x3 convolutions, stride-2
convolutions down, nearest 2x upsampling and skip concatenation up) maps the
far-field log-intensity image of a sample (Ny x Nz) to the delta cross-section
of the unknown rows (mean over the beam direction, rows pooled 4:1), which is
extruded along the beam as the ADAM starting point.  Every layer runs in
libmsl's kernels (``nn.py``): convolutions are bfloat16 matrix-core products
(weights x 3x3 patches) with float32 accumulation; master weights, activations
and gradients are float32.  This module only sequences the calls and owns the
buffers.

Training data come from the model itself: samples of the bars-on-substrate
generator (feature boxes drawn on the host, slice pools rendered on the
device), their far fields from the batched forward, and as targets the
slice-length-weighted mean of the pools over the unknown rows.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import msl, nn, synth

BF16 = nn.BF16


def layer_specs(c=32):
    """(name, in channels, out channels, stride, relu) of every convolution, in order."""
    c1, c2, c3, c4 = c, 2 * c, 4 * c, 8 * c
    return [("e1a", 1, c1, 1, True), ("e1b", c1, c1, 1, True),
            ("e2a", c1, c2, 2, True), ("e2b", c2, c2, 1, True),
            ("e3a", c2, c3, 2, True), ("e3b", c3, c3, 1, True),
            ("e4a", c3, c4, 2, True), ("e4b", c4, c4, 1, True),
            ("d3", c4 + c3, c3, 1, True), ("d2", c3 + c2, c2, 1, True), ("d1", c2 + c1, c1, 1, True),
            ("out", c1, 1, 1, False)]


class UNet:
    """Parameters (flat float32 master copy, bfloat16 copy, ADAM moments) and the pass buffers."""

    def __init__(self, c=32, rows_per_output=4, device="cuda:0", seed=0):
        self.c, self.f, self.dev = c, rows_per_output, torch.device(device)
        self.specs = layer_specs(c)
        self.off = {}
        o = 0
        for name, ci, co, s, act in self.specs:
            self.off[name] = (o, o + co * ci * 9, co, ci, s, act)   # weights, then biases
            o += co * ci * 9 + co
        self.n_params = o
        self.w = torch.zeros(o, dtype=torch.float32, device=self.dev)
        self.g = torch.zeros_like(self.w)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.w16 = torch.zeros(o, dtype=BF16, device=self.dev)
        self.t = 0
        self.init(seed)
        self._bufs = None

    # -- parameters ---------------------------------------------------------
    def init(self, seed):
        """He-normal weights (seeded host draws), zero biases."""
        rng = np.random.Generator(np.random.PCG64(seed))
        host = np.zeros(self.n_params, np.float32)
        for name, ci, co, s, act in self.specs:
            wo, bo, *_ = self.off[name]
            host[wo:bo] = rng.standard_normal(co * ci * 9) * math.sqrt(2.0 / (9 * ci))
        self.set_flat(host)

    def set_flat(self, host):
        self.w.copy_(torch.from_numpy(np.ascontiguousarray(host, np.float32)))
        nn.to_bf16(self.w, self.w16)
        self.m.zero_()
        self.v.zero_()
        self.t = 0

    def params_numpy(self):
        """{name: (w [co][ci][3][3], bias [co])} float64 copies (for checks)."""
        host = self.w.cpu().numpy().astype(np.float64)
        out = {}
        for name, ci, co, s, act in self.specs:
            wo, bo, *_ = self.off[name]
            out[name] = (host[wo:bo].reshape(co, ci, 3, 3), host[bo:bo + co])
        return out

    def grads_numpy(self):
        host = self.g.cpu().numpy().astype(np.float64)
        out = {}
        for name, ci, co, s, act in self.specs:
            wo, bo, *_ = self.off[name]
            out[name] = (host[wo:bo].reshape(co, ci, 3, 3), host[bo:bo + co])
        return out

    def _wb(self, name):
        wo, bo, co, ci, s, act = self.off[name]
        return self.w16[wo:bo], self.w[bo:bo + co], self.g[wo:bo], self.g[bo:bo + co]

    # -- buffers ------------------------------------------------------------
    def _buffers(self, B, H, W):
        key = (B, H, W)
        if self._bufs is not None and self._bufs["key"] == key:
            return self._bufs
        c1, c2, c3, c4 = self.c, 2 * self.c, 4 * self.c, 8 * self.c
        d = self.dev
        z = lambda *shape: torch.zeros(shape, dtype=torch.float32, device=d)
        hw = [(H, W), (H // 2, W // 2), (H // 4, W // 4), (H // 8, W // 8)]
        b = {"key": key}
        b["x"] = z(1, B, H, W)
        b["e1a"] = z(c1, B, *hw[0])
        b["cat1"] = z(c2 + c1, B, *hw[0])          # [up(d2); e1]
        b["e2a"] = z(c2, B, *hw[1])
        b["cat2"] = z(c3 + c2, B, *hw[1])          # [up(d3); e2]
        b["e3a"] = z(c3, B, *hw[2])
        b["cat3"] = z(c4 + c3, B, *hw[2])          # [up(e4); e3]
        b["e4a"] = z(c4, B, *hw[3])
        b["e4"] = z(c4, B, *hw[3])
        b["d3"] = z(c3, B, *hw[2])
        b["d2"] = z(c2, B, *hw[1])
        b["d1"] = z(c1, B, *hw[0])
        b["out"] = z(1, B, H, W)
        b["pred"] = z(B, H // self.f, W)
        kmax = max(ci * 9 for _, ci, _, _, _ in self.specs)
        nmax = B * H * W
        b["col"] = torch.zeros(kmax * nmax, dtype=BF16, device=d)
        b["dcol"] = torch.zeros(kmax * nmax, dtype=torch.float32, device=d)
        comax = max(co for _, _, co, _, _ in self.specs)
        b["dy16"] = torch.zeros(comax * nmax, dtype=BF16, device=d)
        # gradient buffers with the activations' shapes
        for k in ("e1a", "cat1", "e2a", "cat2", "e3a", "cat3", "e4a", "e4", "d3", "d2", "d1", "out"):
            b["d_" + k] = torch.zeros_like(b[k])
        b["t1"] = z(c1, B, *hw[0])   # encoder gradient parts before the skip sum
        b["t2"] = z(c2, B, *hw[1])
        b["t3"] = z(c3, B, *hw[2])
        b["d_pred"] = torch.zeros_like(b["pred"])
        b["loss"] = torch.zeros((), dtype=torch.float64, device=d)
        self._bufs = b
        return b

    # -- layers -------------------------------------------------------------
    def _conv(self, name, x, y, B, H, W):
        """y = act(W * patches(x) + b); x [ci][B][H][W] -> y [co][B][H/s][W/s]."""
        wo, bo, co, ci, s, act = self.off[name]
        bf = self._bufs
        Ho, Wo = H // s, W // s
        N = B * Ho * Wo
        col = bf["col"][:ci * 9 * N]
        nn.im2col(ci, B, H, W, s, x, col)
        w16, bias, _, _ = self._wb(name)
        nn.gemm(co, N, ci * 9, w16, ci * 9, 0, col, N, 0, y, N, bias=bias, relu=act)

    def _conv_back(self, name, x, y, dy, dx, B, H, W):
        """Weight and bias gradients of layer `name` into self.g; dx (may be None) = dL/dx."""
        wo, bo, co, ci, s, act = self.off[name]
        bf = self._bufs
        Ho, Wo = H // s, W // s
        N = B * Ho * Wo
        if act:
            nn.relu_adjoint(y, dy)
        dy16 = bf["dy16"][:co * N]
        nn.to_bf16(dy, dy16)
        w16, _, gw, gb = self._wb(name)
        nn.rowsum(co, N, dy, gb)
        col = bf["col"][:ci * 9 * N]
        nn.im2col(ci, B, H, W, s, x, col)
        nn.gemm(co, ci * 9, N, dy16, N, 0, col, N, 1, gw, ci * 9)
        if dx is not None:
            dcol = bf["dcol"][:ci * 9 * N]
            nn.gemm(ci * 9, N, co, w16, ci * 9, 1, dy16, N, 0, dcol, N)
            nn.col2im(ci, B, H, W, s, dcol, dx)

    def forward(self, x=None, B=None, H=256, W=256):
        """Network output for the input already in the buffer x (or copied from `x`)."""
        if x is not None:
            B, H, W = x.shape[1], x.shape[2], x.shape[3]
        bf = self._buffers(B, H, W)
        if x is not None:
            bf["x"].copy_(x)
        c1, c2, c3, c4 = self.c, 2 * self.c, 4 * self.c, 8 * self.c
        e1 = bf["cat1"][c2:]
        e2 = bf["cat2"][c3:]
        e3 = bf["cat3"][c4:]
        self._conv("e1a", bf["x"], bf["e1a"], B, H, W)
        self._conv("e1b", bf["e1a"], e1, B, H, W)
        self._conv("e2a", e1, bf["e2a"], B, H, W)
        self._conv("e2b", bf["e2a"], e2, B, H // 2, W // 2)
        self._conv("e3a", e2, bf["e3a"], B, H // 2, W // 2)
        self._conv("e3b", bf["e3a"], e3, B, H // 4, W // 4)
        self._conv("e4a", e3, bf["e4a"], B, H // 4, W // 4)
        self._conv("e4b", bf["e4a"], bf["e4"], B, H // 8, W // 8)
        nn.upsample2(c4, B, H // 8, W // 8, bf["e4"], bf["cat3"][:c4])
        self._conv("d3", bf["cat3"], bf["d3"], B, H // 4, W // 4)
        nn.upsample2(c3, B, H // 4, W // 4, bf["d3"], bf["cat2"][:c3])
        self._conv("d2", bf["cat2"], bf["d2"], B, H // 2, W // 2)
        nn.upsample2(c2, B, H // 2, W // 2, bf["d2"], bf["cat1"][:c2])
        self._conv("d1", bf["cat1"], bf["d1"], B, H, W)
        self._conv("out", bf["d1"], bf["out"], B, H, W)
        nn.rowpool(B, H, W, self.f, bf["out"], bf["pred"])
        return bf["pred"]

    def backward(self, dpred):
        """Parameter gradients (into self.g) of a loss with dL/dpred, after ``forward``."""
        bf = self._bufs
        B, H, W = bf["key"]
        c1, c2, c3, c4 = self.c, 2 * self.c, 4 * self.c, 8 * self.c
        e1, e2, e3 = bf["cat1"][c2:], bf["cat2"][c3:], bf["cat3"][c4:]
        nn.rowpool_adjoint(B, H, W, self.f, dpred, bf["d_out"])
        self._conv_back("out", bf["d1"], bf["out"], bf["d_out"], bf["d_d1"], B, H, W)
        self._conv_back("d1", bf["cat1"], bf["d1"], bf["d_d1"], bf["d_cat1"], B, H, W)
        nn.upsample2_adjoint(c2, B, H // 2, W // 2, bf["d_cat1"][:c2], bf["d_d2"])
        self._conv_back("d2", bf["cat2"], bf["d2"], bf["d_d2"], bf["d_cat2"], B, H // 2, W // 2)
        nn.upsample2_adjoint(c3, B, H // 4, W // 4, bf["d_cat2"][:c3], bf["d_d3"])
        self._conv_back("d3", bf["cat3"], bf["d3"], bf["d_d3"], bf["d_cat3"], B, H // 4, W // 4)
        nn.upsample2_adjoint(c4, B, H // 8, W // 8, bf["d_cat3"][:c4], bf["d_e4"])
        # encoder: skip gradients are the second parts of the concatenations
        de3, de2, de1 = bf["d_cat3"][c4:], bf["d_cat2"][c3:], bf["d_cat1"][c2:]
        self._conv_back("e4b", bf["e4a"], bf["e4"], bf["d_e4"], bf["d_e4a"], B, H // 8, W // 8)
        self._conv_back("e4a", e3, bf["e4a"], bf["d_e4a"], bf["t3"], B, H // 4, W // 4)
        nn.add_(bf["t3"], de3)
        self._conv_back("e3b", bf["e3a"], e3, de3, bf["d_e3a"], B, H // 4, W // 4)
        self._conv_back("e3a", e2, bf["e3a"], bf["d_e3a"], bf["t2"], B, H // 2, W // 2)
        nn.add_(bf["t2"], de2)
        self._conv_back("e2b", bf["e2a"], e2, de2, bf["d_e2a"], B, H // 2, W // 2)
        self._conv_back("e2a", e1, bf["e2a"], bf["d_e2a"], bf["t1"], B, H, W)
        nn.add_(bf["t1"], de1)
        self._conv_back("e1b", bf["e1a"], e1, de1, bf["d_e1a"], B, H, W)
        self._conv_back("e1a", bf["x"], bf["e1a"], bf["d_e1a"], None, B, H, W)

    def loss_and_grad(self, target):
        """MSE against target [B][H/f][W]; fills the gradients; returns the loss (device float64)."""
        bf = self._bufs
        nn.mse(bf["pred"], target, bf["d_pred"], bf["loss"])
        self.backward(bf["d_pred"])
        return bf["loss"]

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        nn.adam(self.w, self.g, self.m, self.v, self.w16, lr, beta1, beta2, eps, self.t)
