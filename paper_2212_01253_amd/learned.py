"""Learned initialiser for the gradient reconstruction (NEXT to the paper's Sec. 4.1).

A four-level U-Net (channels c, 2c, 4c, 8c; 3x3 convolutions, stride-2
convolutions down, nearest 2x upsampling and skip concatenation up) maps the
far-field log-intensity image of a sample (Ny x Nz) to the delta cross-section
of the unknown rows (mean over the beam direction, rows pooled 4:1), which is
extruded along the beam as the ADAM starting point.  A second input channel
holds the row coordinate (a convolutional network is otherwise blind to
absolute position, and the cross-section's rows are heights), and the output
is a correction to a fixed offset map (the training targets' mean).  A global
head adds a per-row term: two dense layers on shift-invariant summaries of
each image row (its mean, the centre column and the mean of the seven central
columns), broadcast along the row.  Shifting a structure cyclically across
the beam leaves the far-field intensity unchanged, so what an image
determines is shift-invariant (heights, densities), and the row summaries
carry it to every output column, which 3x3 convolutions cannot.  Every layer
runs in libmsl's kernels (``nn.py``): convolutions are bfloat16 matrix-core
products (weights x 3x3 patches, formed while loading) with float32
accumulation; master weights, activations and gradients are float32.  This module only sequences the calls and owns the
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
SPLIT_PARTS = 2048  # most parts of a split weight-gradient product


def layer_specs(c=32, in_ch=2):
    """(name, in channels, out channels, stride, relu) of every convolution, in order."""
    c1, c2, c3, c4 = c, 2 * c, 4 * c, 8 * c
    return [("e1a", in_ch, c1, 1, True), ("e1b", c1, c1, 1, True),
            ("e2a", c1, c2, 2, True), ("e2b", c2, c2, 1, True),
            ("e3a", c2, c3, 2, True), ("e3b", c3, c3, 1, True),
            ("e4a", c3, c4, 2, True), ("e4b", c4, c4, 1, True),
            ("d3", c4 + c3, c3, 1, True), ("d2", c3 + c2, c2, 1, True), ("d1", c2 + c1, c1, 1, True),
            ("out", c1, 1, 1, False)]


class UNet:
    """Parameters (flat float32 master copy, bfloat16 copy, ADAM moments) and the pass buffers."""

    def __init__(self, c=32, rows_per_output=4, device="cuda:0", seed=0, n=256, hidden=None):
        self.c, self.f, self.dev = c, rows_per_output, torch.device(device)
        self.n = n                      # image rows (the global head's input and output sizes)
        self.hidden = hidden or 8 * c   # global head's hidden width
        self.specs = layer_specs(c)
        self.offset = None   # [rows][W] added to every output (set_offset)
        self.off = {}
        o = 0
        n_real = 0
        for name, ci, co, s, act in self.specs:
            o = (o + 7) // 8 * 8   # weight rows start 16-byte aligned (vector loads in the products)
            self.off[name] = (o, o + co * ci * 9, co, ci, s, act)   # weights, then biases
            o += co * ci * 9 + co
            n_real += co * ci * 9 + co
        # global head: dense layers on shift-invariant row summaries (msl_nn_row_features),
        # its output added along every output row
        self.head_off = {}
        for name, ni, no in (("g1", 3 * n, self.hidden), ("g2", self.hidden, n // rows_per_output)):
            o = (o + 7) // 8 * 8
            self.head_off[name] = (o, o + no * ni, no, ni)
            o += no * ni + no
            n_real += no * ni + no
        self.n_params = n_real   # parameters (the flat arrays also hold alignment gaps, always zero)
        self.n_flat = o
        self.w = torch.zeros(o, dtype=torch.float32, device=self.dev)
        self.g = torch.zeros_like(self.w)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.w16 = torch.zeros(o, dtype=BF16, device=self.dev)
        # normalisation of the head's inputs (fixed, from the training set: set_feature_norm)
        self.feat_shift = torch.zeros(3 * n, dtype=torch.float32, device=self.dev)
        self.feat_scale = torch.ones(3 * n, dtype=torch.float32, device=self.dev)
        self.t = 0
        self.init(seed)
        self._bufs = None

    # -- parameters ---------------------------------------------------------
    def init(self, seed):
        """He-normal weights (seeded host draws), zero biases."""
        rng = np.random.Generator(np.random.PCG64(seed))
        host = np.zeros(self.n_flat, np.float32)
        for name, ci, co, s, act in self.specs:
            wo, bo, *_ = self.off[name]
            host[wo:bo] = rng.standard_normal(co * ci * 9) * math.sqrt(2.0 / (9 * ci))
        for name, gain in (("g1", 2.0), ("g2", 0.01)):
            wo, bo, no, ni = self.head_off[name]
            host[wo:bo] = rng.standard_normal(no * ni) * math.sqrt(gain / ni)
        self.set_flat(host)

    def set_flat(self, host):
        self.w.copy_(torch.from_numpy(np.ascontiguousarray(host, np.float32)))
        nn.to_bf16(self.w, self.w16)
        self.m.zero_()
        self.v.zero_()
        self.t = 0

    def _unflatten(self, host):
        out = {}
        for name, ci, co, s, act in self.specs:
            wo, bo, *_ = self.off[name]
            out[name] = (host[wo:bo].reshape(co, ci, 3, 3), host[bo:bo + co])
        for name, (wo, bo, no, ni) in self.head_off.items():
            out[name] = (host[wo:bo].reshape(no, ni), host[bo:bo + no])
        return out

    def params_numpy(self):
        """{name: (w, bias)} float64 copies (for checks): convolutions w [co][ci][3][3],
        head layers w [out][in]."""
        return self._unflatten(self.w.cpu().numpy().astype(np.float64))

    def grads_numpy(self):
        return self._unflatten(self.g.cpu().numpy().astype(np.float64))

    def _wb(self, name):
        if name in self.head_off:
            wo, bo, co, _ = self.head_off[name]
        else:
            wo, bo, co, ci, s, act = self.off[name]
        return self.w16[wo:bo], self.w[bo:bo + co], self.g[wo:bo], self.g[bo:bo + co]

    # -- buffers ------------------------------------------------------------
    def _buffers(self, B, H, W):
        key = (B, H, W)
        if self._bufs is not None and self._bufs["key"] == key:
            return self._bufs
        if H != self.n:
            raise ValueError(f"the network was built for {self.n}-row images, got {H}")
        c1, c2, c3, c4 = self.c, 2 * self.c, 4 * self.c, 8 * self.c
        d = self.dev
        z = lambda *shape: torch.zeros(shape, dtype=torch.float32, device=d)
        # ReLU activations are stored as bfloat16 bits: every layer that reads them (convolutions,
        # their weight gradients) rounds its input to bfloat16 anyway, the ReLU adjoint only needs
        # their sign, and upsampling and concatenation copy them, so the network computes the same
        # values with half the activation traffic.  The input, the output layer and all gradients
        # stay float32.
        z16 = lambda *shape: torch.zeros(shape, dtype=BF16, device=d)
        hw = [(H, W), (H // 2, W // 2), (H // 4, W // 4), (H // 8, W // 8)]
        b = {"key": key}
        b["x"] = z(2, B, H, W)
        ramp = torch.linspace(-1.0, 1.0, H, device=d)   # channel 1: the row coordinate
        b["x"][1].copy_(ramp.view(1, H, 1).expand(B, H, W))
        b["e1a"] = z16(c1, B, *hw[0])
        b["cat1"] = z16(c2 + c1, B, *hw[0])          # [up(d2); e1]
        b["e2a"] = z16(c2, B, *hw[1])
        b["cat2"] = z16(c3 + c2, B, *hw[1])          # [up(d3); e2]
        b["e3a"] = z16(c3, B, *hw[2])
        b["cat3"] = z16(c4 + c3, B, *hw[2])          # [up(e4); e3]
        b["e4a"] = z16(c4, B, *hw[3])
        b["e4"] = z16(c4, B, *hw[3])
        b["d3"] = z16(c3, B, *hw[2])
        b["d2"] = z16(c2, B, *hw[1])
        b["d1"] = z16(c1, B, *hw[0])
        b["out"] = z(1, B, H, W)
        b["pred"] = z(B, H // self.f, W)
        nmax = B * H * W
        comax = max(co for _, _, co, _, _ in self.specs)
        b["dy16"] = torch.zeros(comax * nmax, dtype=BF16, device=d)
        need = 0
        for name, ci, co, s, act in self.specs:
            # pixel level of the layer's output (its gradient's columns)
            lvl = {"e1a": 0, "e1b": 0, "e2a": 1, "e2b": 1, "e3a": 2, "e3b": 2, "e4a": 3, "e4b": 3,
                   "d3": 2, "d2": 1, "d1": 0, "out": 0}[name]
            npix = B * hw[lvl][0] * hw[lvl][1]
            need = max(need, max(1, min(SPLIT_PARTS, npix // 1024)) * co * ci * 9)
        b["parts"] = torch.zeros(need, dtype=torch.float32, device=d)
        # gradient buffers with the activations' shapes
        for k in ("e1a", "cat1", "e2a", "cat2", "e3a", "cat3", "e4a", "e4", "d3", "d2", "d1", "out"):
            b["d_" + k] = torch.zeros(b[k].shape, dtype=torch.float32, device=d)
        b["d_pred"] = torch.zeros_like(b["pred"])
        b["loss"] = torch.zeros((), dtype=torch.float64, device=d)
        # global head
        hid, R = self.hidden, H // self.f
        b["feat16"] = torch.zeros(B * 3 * H, dtype=BF16, device=d)
        b["h1"] = z(hid, B)
        b["h1_16"] = torch.zeros(hid * B, dtype=BF16, device=d)
        b["hp"] = z(R, B)
        b["dp"] = z(R, B)
        b["dp16"] = torch.zeros(R * B, dtype=BF16, device=d)
        b["dh1"] = z(hid, B)
        b["dh1_16"] = torch.zeros(hid * B, dtype=BF16, device=d)
        self._bufs = b
        return b

    # -- layers -------------------------------------------------------------
    def _conv(self, name, x, y, B, H, W):
        """y = act(W * patches(x) + b); x [ci][B][H][W] -> y [co][B][H/s][W/s] (implicit product)."""
        wo, bo, co, ci, s, act = self.off[name]
        w16, bias, _, _ = self._wb(name)
        nn.conv3x3(co, ci, B, H, W, s, w16, x, y, bias=bias, relu=act)

    def _conv_back(self, name, x, y, dy, dx, B, H, W, accumulate=False):
        """Weight and bias gradients of layer `name` into self.g; dx (may be None) = dL/dx, or
        dx += dL/dx with accumulate (an input that also feeds a skip connection)."""
        wo, bo, co, ci, s, act = self.off[name]
        bf = self._bufs
        Ho, Wo = H // s, W // s
        N = B * Ho * Wo
        dy16 = bf["dy16"][:co * N]
        w16, _, gw, gb = self._wb(name)
        # ReLU adjoint, bfloat16 copy and bias gradient in one pass (dy itself is not rewritten)
        nn.grad_prep(co, N, y if act else None, dy, dy16, gb, bf["parts"])
        # weight gradient: a short, wide product over the long pixel axis, split along it
        splits = max(1, min(SPLIT_PARTS, N // 1024))
        nn.conv3x3_weight_grad(co, ci, B, H, W, s, dy16, x, gw, splits, bf["parts"])
        if dx is not None:
            nn.conv3x3_adjoint(co, ci, B, H, W, s, w16, dy16, dx, accumulate=accumulate)

    def forward(self, x=None, B=None, H=256, W=256):
        """Network output for the input already in the buffer x (or copied from `x`)."""
        if x is not None:
            B, H, W = x.shape[1], x.shape[2], x.shape[3]
        bf = self._buffers(B, H, W)
        if x is not None:
            bf["x"][0].copy_(x[0])
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
        self._head(B, H, W)
        if self.offset is not None:
            if "offset" not in bf:
                bf["offset"] = self.offset.unsqueeze(0).expand(B, -1, -1).contiguous()
            nn.add_(bf["offset"], bf["pred"])
        return bf["pred"]

    def _head(self, B, H, W):
        """pred[b][r][:] += g2(relu(g1(row summaries of input channel 0)))[r][b]."""
        bf = self._bufs
        hid, R, F = self.hidden, H // self.f, 3 * H
        nn.row_features(B, H, W, bf["x"][0], bf["feat16"], self.feat_shift, self.feat_scale)
        w1, b1, _, _ = self._wb("g1")
        nn.gemm(hid, B, F, w1, F, 0, bf["feat16"], F, 1, bf["h1"], B, bias=b1, relu=True, C16=bf["h1_16"])
        w2, b2, _, _ = self._wb("g2")
        nn.gemm(R, B, hid, w2, hid, 0, bf["h1_16"], B, 0, bf["hp"], B, bias=b2)
        nn.add_row_bias(B, R, W, bf["hp"], bf["pred"])

    def _head_back(self, dpred, B, H, W):
        bf = self._bufs
        hid, R, F = self.hidden, H // self.f, 3 * H
        _, _, gw1, gb1 = self._wb("g1")
        w2, _, gw2, gb2 = self._wb("g2")
        nn.row_bias_adjoint(B, R, W, dpred, bf["dp"])
        nn.rowsum(R, B, bf["dp"], gb2, bf["parts"])
        nn.to_bf16(bf["dp"], bf["dp16"])
        nn.gemm(R, hid, B, bf["dp16"], B, 0, bf["h1_16"], B, 1, gw2, hid)
        nn.gemm(hid, B, R, w2, hid, 1, bf["dp16"], B, 0, bf["dh1"], B)
        nn.relu_adjoint(bf["h1"], bf["dh1"])
        nn.rowsum(hid, B, bf["dh1"], gb1, bf["parts"])
        nn.to_bf16(bf["dh1"], bf["dh1_16"])
        nn.gemm(hid, F, B, bf["dh1_16"], B, 0, bf["feat16"], F, 0, gw1, F)

    def set_feature_norm(self, shift, scale):
        """The head's inputs become (summary - shift) * scale (float32 [3n] each)."""
        self.feat_shift.copy_(shift.to(self.dev).float())
        self.feat_scale.copy_(scale.to(self.dev).float())

    def set_offset(self, offset):
        """Fixed map [rows][W] added to the output (None: no offset)."""
        self.offset = None if offset is None else offset.to(self.dev).float().contiguous()
        if self._bufs is not None:
            self._bufs.pop("offset", None)

    def backward(self, dpred):
        """Parameter gradients (into self.g) of a loss with dL/dpred, after ``forward``."""
        bf = self._bufs
        B, H, W = bf["key"]
        c1, c2, c3, c4 = self.c, 2 * self.c, 4 * self.c, 8 * self.c
        e1, e2, e3 = bf["cat1"][c2:], bf["cat2"][c3:], bf["cat3"][c4:]
        self._head_back(dpred, B, H, W)
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
        # each stride-2 layer's input gradient is added onto the skip gradient of the same tensor
        self._conv_back("e4a", e3, bf["e4a"], bf["d_e4a"], de3, B, H // 4, W // 4, accumulate=True)
        self._conv_back("e3b", bf["e3a"], e3, de3, bf["d_e3a"], B, H // 4, W // 4)
        self._conv_back("e3a", e2, bf["e3a"], bf["d_e3a"], de2, B, H // 2, W // 2, accumulate=True)
        self._conv_back("e2b", bf["e2a"], e2, de2, bf["d_e2a"], B, H // 2, W // 2)
        self._conv_back("e2a", e1, bf["e2a"], bf["d_e2a"], de1, B, H, W, accumulate=True)
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


# ---------------------------------------------------------------------------
# training data from the forward model

INPUT_A = 0.25   # network input: INPUT_A * log(I + eps_of(n))


def eps_of(n):
    """Intensity floor of the input map: one photon of a 1e6-photon image of an n x n unit field."""
    return n * n / 1e6


def slice_index_of(cuts):
    """Pool index of every slice from the pool boundaries."""
    return np.repeat(np.arange(len(cuts) - 1, dtype=np.int32), np.diff(cuts))


class TrainingSet:
    """Network inputs [S][n][n] and targets [S][rows/f... rows][n] on the device, from the model."""

    def __init__(self, n_samples, seed0=20000, n=256, n_slices=1024, rows=None, f=4, chunk=128, log=False):
        self.n, self.f = n, f
        self.rows = rows or n // 4            # unknown rows: the n/4 rows above the n/4-row substrate
        dev = torch.device("cuda")
        self.x = torch.zeros((n_samples, n, n), dtype=torch.float32, device=dev)
        self.y = torch.zeros((n_samples, self.rows, n), dtype=torch.float32, device=dev)
        t0 = time.perf_counter()
        for c0 in range(0, n_samples, chunk):
            ids = list(range(c0, min(n_samples, c0 + chunk)))
            smp = [synth.training_sample(seed0 + i, n=n, n_slices=n_slices) for i in ids]
            k = len(smp)
            nps = np.array([len(c) - 1 for _, _, c in smp], np.int32)
            offs = np.concatenate([[0], np.cumsum(nps)[:-1]]).astype(np.int64)
            boxes = np.zeros((k, nn.MAX_BOXES, 8), np.float32)
            cuts = np.zeros((k, nn.MAX_CUTS), np.int32)
            wts = np.zeros((k, nn.MAX_CUTS), np.float32)
            nfs = np.zeros(k, np.int32)
            for q, (g, b, c) in enumerate(smp):
                boxes[q, :len(b)] = b
                nfs[q] = len(b)
                cuts[q, :len(c)] = c
                wts[q, :len(c) - 1] = np.diff(c) / g.n_slices
            pd = torch.empty((int(nps.sum()), n, n), dtype=torch.float32, device=dev)
            pb = torch.empty_like(pd)
            T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
            Tn, Toff = T(nps), T(offs)
            nn.render_pools(k, n, n, n // 4, synth.SUBSTRATE_DELTA, synth.SUBSTRATE_BETA, T(boxes), T(nfs), T(cuts),
                            Tn, Toff, int(nps.max()), pd, pb)
            nn.pool_average(k, n, n, n // 4, self.rows, T(wts), Tn, Toff, int(nps.max()), pd, 1e5,
                            self.y[ids[0]:ids[-1] + 1])
            I = torch.empty((k, n, n), dtype=torch.float32, device=dev)
            items = []
            for q, (g, b, c) in enumerate(smp):
                items.append({"geom": g, "pool_delta": pd[offs[q]:offs[q] + nps[q]],
                              "pool_beta": pb[offs[q]:offs[q] + nps[q]], "slice_index": T(slice_index_of(c)),
                              "field": torch.empty((n, n), dtype=torch.complex64, device=dev), "intensity": I[q]})
            msl.forward_batch(items)
            nn.logmap(I, eps_of(n), INPUT_A, 0.0, self.x[ids[0]:ids[-1] + 1])
            if log and (c0 // chunk) % 20 == 0:
                torch.cuda.synchronize()
                print(f"# training set: {c0 + k}/{n_samples} samples ({time.perf_counter() - t0:.1f} s)", flush=True)
        torch.cuda.synchronize()
        self.seconds = time.perf_counter() - t0

    def __len__(self):
        return self.x.shape[0]


def feature_norm(data, chunk=256):
    """Shift (mean) and scale (1 / standard deviation) of the head's row summaries over a
    training set, float32 [3n] each (the same summaries msl_nn_row_features forms)."""
    n = data.n
    c = n // 2
    s1 = torch.zeros(3 * n, dtype=torch.float64, device=data.x.device)
    s2 = torch.zeros_like(s1)
    for s0 in range(0, len(data), chunk):
        x = data.x[s0:s0 + chunk].double()
        f = torch.cat([x.mean(dim=2), x[:, :, c], x[:, :, c - 3:c + 4].mean(dim=2)], dim=1)
        s1 += f.sum(dim=0)
        s2 += (f * f).sum(dim=0)
    m = s1 / len(data)
    sd = torch.sqrt(torch.clamp(s2 / len(data) - m * m, min=0.0)) + 1e-6
    return m.float(), (1.0 / sd).float()


def mean_target(data, chunk=256):
    """Mean of the training targets, [rows][n] (the network's output offset)."""
    acc = torch.zeros(data.y.shape[1:], dtype=torch.float64, device=data.y.device)
    for s0 in range(0, len(data), chunk):
        acc += data.y[s0:s0 + chunk].double().sum(0)
    return (acc / len(data)).float()


def steps_per_epoch(n_samples, batch):
    """Minibatches per epoch: every sample at least once (the last batch may wrap around)."""
    return max(1, -(-n_samples // batch))


def train(net, data, steps, batch=32, lr=1e-3, seed=1, log_every=0, val=None):
    """ADAM on the mean squared error over minibatches that walk the training set in a fresh
    seeded permutation each epoch (every sample at least once per epoch: the last batch of an
    epoch is filled up from the start of that epoch's permutation); returns the loss history
    and the seconds taken."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = data.n
    xb = torch.empty((1, batch, n, n), dtype=torch.float32, device="cuda")
    yb = torch.empty((batch, data.rows, n), dtype=torch.float32, device="cuda")
    hist = []
    per_epoch = steps_per_epoch(len(data), batch)
    order = None
    t0 = time.perf_counter()
    for it in range(steps):
        if it % per_epoch == 0:
            order = rng.permutation(len(data))
        k = it % per_epoch
        sel = order[k * batch:(k + 1) * batch]
        if len(sel) < batch:
            sel = np.concatenate([sel, np.resize(order, batch - len(sel))])
        idx = torch.from_numpy(sel).cuda()
        torch.index_select(data.x, 0, idx, out=xb[0])
        torch.index_select(data.y, 0, idx, out=yb)
        net.forward(xb)
        L = net.loss_and_grad(yb)
        net.adam_step(lr)
        if log_every and (it % log_every == 0 or it == steps - 1):
            Lh = float(L.item())
            hist.append((it, Lh))
            msg = f"# step {it}: loss {Lh:.5f} ({time.perf_counter() - t0:.1f} s)"
            if val is not None:
                msg += f", validation {evaluate(net, val, batch):.5f}"
            print(msg, flush=True)
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def predict(net, x, batch=64):
    """Network output for inputs x [S][n][n] in batches; returns [S][rows][n] (device)."""
    S, n = x.shape[0], x.shape[1]
    out = []
    for s0 in range(0, S, batch):
        xb = x[s0:s0 + batch].unsqueeze(0).contiguous()
        out.append(net.forward(xb).clone())
    return torch.cat(out)


def evaluate(net, data, batch=64):
    """Mean squared error of the network on a data set (library loss kernel per batch)."""
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    total, count = 0.0, 0
    for s0 in range(0, len(data), batch):
        xb = data.x[s0:s0 + batch].unsqueeze(0).contiguous()
        pred = net.forward(xb)
        nn.mse(pred, data.y[s0:s0 + batch].contiguous(), None, loss)
        k = xb.shape[1]
        total += float(loss.item()) * k
        count += k
    return total / count


def train_initialiser(n_samples=50000, steps=None, batch=32, lr=1e-3, n=256, n_slices=1024, seed=0, log_every=0,
                      n_val=256, epochs=1):
    """Training set from the model, the network with the targets' mean as output offset, ADAM
    over `epochs` passes through the training set (or `steps` minibatches when given).
    Returns (net, info) with the data and training times and the validation error of the network
    next to that of the offset alone (the population-mean cross-section); info["companions"]
    keeps the validation inputs (images the network never trained on) for batched inference."""
    if steps is None:
        steps = epochs * steps_per_epoch(n_samples, batch)
    data = TrainingSet(n_samples, n=n, n_slices=n_slices)
    val = TrainingSet(n_val, seed0=900000, n=n, n_slices=n_slices)
    net = UNet(c=32, seed=seed, n=n)
    mt = mean_target(data)
    net.set_offset(mt)
    net.set_feature_norm(*feature_norm(data))
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    nn.mse(mt.unsqueeze(0).expand(len(val), -1, -1).contiguous(), val.y, None, loss)
    base = float(loss.item())
    hist, secs = train(net, data, steps, batch=batch, lr=lr, log_every=log_every)
    # A cyclic shift of the structure across the beam (along z) leaves the far-field intensity
    # unchanged, so where a feature sits in z cannot be read from the image; what an image
    # determines is shift-invariant, such as the row profile (the mean over z of each row).
    # Its error is reported beside the per-pixel one, for the network and for the mean map.
    pred = predict(net, val.x)
    rt = val.y.mean(dim=2)
    row_net = float(((pred.mean(dim=2) - rt) ** 2).mean())
    row_mean = float(((mt.mean(dim=1).unsqueeze(0) - rt) ** 2).mean())
    info = {"samples": n_samples, "steps": steps, "batch": batch, "lr": lr, "data_seconds": data.seconds,
            "train_seconds": secs, "ms_per_step": 1e3 * secs / max(1, steps), "params": net.n_params,
            "val_mse": evaluate(net, val), "val_mse_mean_map": base,
            "val_row_profile_mse": row_net, "val_row_profile_mse_mean_map": row_mean,
            "epochs": steps / steps_per_epoch(n_samples, batch)}
    info["companions"] = val.x[:63].clone()
    del data, val
    return net, info


def step_flops(net, batch, H=256, W=256):
    """Multiply-add flops (2 per product) of one forward pass and of one training step: every
    convolution's product in the forward; in the backward, its weight gradient and (all layers but
    the first, whose input needs none) its input gradient; the global head's two dense layers the
    same way.  Elementwise work is not counted."""
    fwd = bwd = 0.0
    h, w = H, W
    for name, ci, co, s, _ in net.specs:
        if name == "d3":
            h, w = H // 4, W // 4   # decoder levels follow the upsampling
        elif name == "d2":
            h, w = H // 2, W // 2
        elif name == "d1":
            h, w = H, W
        h, w = h // s, w // s
        f = 2.0 * co * ci * 9 * batch * h * w
        fwd += f
        bwd += f if name == "e1a" else 2 * f
    for name, (o0, o1, no, ni) in net.head_off.items():
        f = 2.0 * no * ni * batch
        fwd += f
        bwd += 2 * f
    return fwd, fwd + bwd


def _speed(batch, steps=5):
    """Times training steps and forward passes of the 256 x 256 network at a batch size."""
    net = UNet(c=32, seed=0)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(1, batch, 256, 256, device="cuda", generator=g) * 0.1
    y = torch.randn(batch, 64, 256, device="cuda", generator=g) * 0.1
    for _ in range(2):
        net.forward(x)
        net.loss_and_grad(y)
        net.adam_step(1e-3)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        net.forward(x)
        net.loss_and_grad(y)
        net.adam_step(1e-3)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    t = time.perf_counter()
    for _ in range(steps):
        net.forward(x)
    torch.cuda.synchronize()
    df = (time.perf_counter() - t) / steps
    ff, ft = step_flops(net, batch)
    print(f"batch {batch}: training step {dt * 1e3:.1f} ms ({ft / dt / 1e12:.0f} TFLOP/s of {ft / 1e12:.2f} TFLOP), "
          f"forward {df * 1e3:.1f} ms ({ff / df / 1e12:.0f} TFLOP/s)", flush=True)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="learned initialiser: timing of the network's passes")
    ap.add_argument("--speed", type=int, default=32, metavar="BATCH")
    _speed(ap.parse_args().speed)
