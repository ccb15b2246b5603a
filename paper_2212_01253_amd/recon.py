"""Gradient reconstruction driver (arXiv 2212.01253, Sec. 4.1).

The paper refines a 3-D object by minimising the amplitude loss of Eq. (4)
between a measured (Poisson-noised) detector image and the multislice model,
with gradients of that loss and the ADAM optimiser.  Here the unknowns are the
delta values of a box of voxels (beta tied to delta by a fixed ratio) over a
known stack (the substrate), and one iteration is:

    pack slices -> forward sweep (checkpoints) -> far field -> amplitude loss
    -> [stop if the loss is at or below the threshold]
    -> far-field adjoint -> adjoint sweep -> ADAM step on the box (+ scatter)

Every step runs in libmsl's kernels through the C ABI (``msl.py``); this
module only sequences the calls and reads the loss back once per iteration.

Detector model: counts C ~ Poisson(s I_true) with the photon scale s fixed;
the loss compares sqrt(s I) with sqrt(C), which is s times the amplitude loss
of I against sqrt(C / s), so the library's loss is evaluated with the
measured amplitudes sqrt(C / s) and multiplied by s (and so is its gradient).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field, replace

import numpy as np
import torch

from . import msl, synth


@dataclass
class Adam:
    lr: float = 1.25e-5   # from a sweep on the 256x256x1024 workload (7e-6 ... 3e-5), plain start
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-12
    lo: float = 0.0
    hi: float = 1e-3

    def c(self):
        return msl.CAdam(self.lr, self.beta1, self.beta2, self.eps, self.lo, self.hi)


@dataclass
class ReconResult:
    losses: list = field(default_factory=list)   # detector loss after each evaluation
    times: list = field(default_factory=list)    # seconds from start when each loss was known
    iters_to_threshold: int | None = None        # ADAM steps taken before the first iterate at or below it
    secs_to_threshold: float | None = None
    threshold: float | None = None
    stalled: bool = False                        # stopped by the stall detector (see Reconstructor.run)


class StallWatch:
    """Progress test of a descent: the loss must fall by a fraction `gain` below its last marked
    value within every `window` iterations (window 0: never stalls).  A loss that is not a number
    never counts as progress."""

    def __init__(self, window, gain):
        self.window, self.gain = int(window), float(gain)
        self.mark, self.mark_it = math.inf, 0

    def stalled(self, it, loss):
        if loss <= self.mark * (1.0 - self.gain):
            self.mark, self.mark_it = loss, it
            return False
        return self.window > 0 and it - self.mark_it >= self.window


class Reconstructor:
    """Holds the device state of one reconstruction (stacks, workspace, ADAM moments)."""

    def __init__(self, geom, known_delta, known_beta, region, counts, scale, probe=None, ckpt_every=32,
                 adam: Adam | None = None, device="cuda:0", graphs=False):
        self.g = msl.geometry(geom)
        self.r = msl.region(region)
        self.adam = adam or Adam()
        self.k = max(1, min(int(ckpt_every), self.g.n_slices))
        self.scale = float(scale)
        dev = torch.device(device)
        ny, nz, ns = self.g.ny, self.g.nz, self.g.n_slices
        box = (self.r.ns, self.r.ny, self.r.nz)
        self.D = torch.as_tensor(np.ascontiguousarray(known_delta, np.float32)).to(dev)
        self.B = torch.as_tensor(np.ascontiguousarray(known_beta, np.float32)).to(dev)
        assert tuple(self.D.shape) == (ns, ny, nz) and tuple(self.B.shape) == (ns, ny, nz)
        amp = np.sqrt(np.asarray(counts, np.float64) / self.scale).astype(np.float32)
        self.meas = torch.as_tensor(amp).to(dev)
        self.probe = None if probe is None else torch.as_tensor(np.asarray(probe, np.complex64)).to(dev)
        self.ws = msl.workspace(self.g, self.k, dev)
        self.field = torch.empty((ny, nz), dtype=torch.complex64, device=dev)
        self.ck = torch.empty((msl.checkpoint_count(self.g, self.k), ny, nz), dtype=torch.complex64, device=dev)
        self.I = torch.empty((ny, nz), dtype=torch.float32, device=dev)
        self.gpsi = torch.empty((ny, nz), dtype=torch.complex64, device=dev)
        self.gd = torch.empty((ns, ny, nz), dtype=torch.float32, device=dev)
        self.gb = torch.empty((ns, ny, nz), dtype=torch.float32, device=dev)
        self.theta = torch.zeros(box, dtype=torch.float32, device=dev)
        self.m = torch.zeros(box, dtype=torch.float32, device=dev)
        self.v = torch.zeros(box, dtype=torch.float32, device=dev)
        self.t = 0
        self._loss = torch.zeros((), dtype=torch.float64, device=dev)
        self._gI = torch.zeros((ny, nz), dtype=torch.float32, device=dev)
        # with graphs, the loss evaluation and the adjoint are each captured once in a HIP graph
        # (thousands of kernel launches per iteration become one launch each)
        self.graphs = graphs
        self._g_loss = self._g_adj = None

    def set_theta(self, theta):
        """Start from theta (box values); resets the ADAM moments."""
        self.theta.copy_(torch.as_tensor(np.ascontiguousarray(theta, np.float32)))
        self.m.zero_()
        self.v.zero_()
        self.t = 0
        msl.region_scatter(self.g, self.r, self.theta, self.D, self.B)

    def _loss_calls(self):
        msl.pack_slices(self.g, self.D, self.B, self.ws)
        msl.forward(self.g, self.D, self.B, self.probe, self.k, ws=self.ws, out=self.field, ckpt=self.ck,
                    reuse_pack=True)
        msl.far_field(self.g, self.field, ws=self.ws, out=self.I)
        msl.amp_loss(self.g, self.I, self.meas, ws=self.ws, loss=self._loss, gI=self._gI)

    def _adjoint_calls(self):
        msl.far_field_adjoint(self.g, self.field, self._gI, ws=self.ws, out=self.gpsi)
        msl.adjoint(self.g, self.D, self.B, self.ck, self.k, self.gpsi, probe=self.probe, ws=self.ws,
                    gd=self.gd, gb=self.gb, want_probe=False, reuse_pack=True)

    def _capture(self, calls):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(graph, stream=s):
                calls()
        torch.cuda.current_stream().wait_stream(s)
        return graph

    def _run(self, which):
        calls = self._loss_calls if which == "loss" else self._adjoint_calls
        if not self.graphs:
            calls()
            return
        attr = "_g_loss" if which == "loss" else "_g_adj"
        if getattr(self, attr) is None:
            calls()            # eager once (warms every table and stream), then capture
            torch.cuda.synchronize()
            setattr(self, attr, self._capture(calls))
            torch.cuda.synchronize()
        getattr(self, attr).replay()

    def loss(self):
        """Forward model and amplitude loss of the current theta against sqrt(C / s): a device
        float64 scalar, s times smaller than the detector loss."""
        self._run("loss")
        return self._loss

    def gradient_step(self):
        """Adjoint of the last ``loss()`` and one ADAM step on theta."""
        self._run("adjoint")
        self.t += 1
        msl.region_adam_step(self.g, self.r, self.adam.c(), self.t, self.gd, self.gb, self.theta, self.m,
                             self.v, self.D, self.B, grad_scale=self.scale)

    def stack_gradients(self):
        """(dL/d delta, dL/d beta) of the last ``loss()``, for the detector loss (scaled by s
        inside the ADAM step, not here); runs the adjoint without updating theta."""
        self._run("adjoint")
        return self.gd, self.gb

    def snap(self, levels):
        """The paper's nearest-index filter: theta <- nearest of `levels` (resets nothing else)."""
        msl.region_snap(self.g, self.r, levels, self.theta, self.D, self.B)

    def shrinkwrap(self, sigmas, threshold):
        """Shrink-wrap support on theta: zero where the blurred |theta| is not above threshold x max."""
        if getattr(self, "_sw_scratch", None) is None:
            self._sw_scratch = torch.empty(2 * self.theta.numel() + 1024, dtype=torch.float32, device=self.theta.device)
        msl.region_shrinkwrap(self.g, self.r, sigmas, threshold, self.theta, self.D, self.B, self._sw_scratch)

    def run(self, theta0, max_iters, threshold=None, log_every=0, snap_levels=None, snap_every=0,
            wrap_every=0, wrap_sigmas=(0.0, 1.5, 1.5), wrap_threshold=0.1, stall_window=0, stall_gain=0.01):
        """ADAM from theta0 until the loss is <= threshold or max_iters steps; wall-clock timed.
        With snap_levels and snap_every, every snap_every-th step is followed by the
        nearest-index filter (the paper applies it after 20 epochs); with wrap_every, every
        wrap_every-th step by the shrink-wrap support (the paper: every 20 epochs).  With
        stall_window, the run also stops (result.stalled) once stall_window iterations pass
        without the loss falling by a fraction stall_gain below its last such improvement."""
        res = ReconResult(threshold=threshold)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.set_theta(theta0)
        watch = StallWatch(stall_window, stall_gain)
        for it in range(max_iters + 1):
            L = float(self.loss().item()) * self.scale
            now = time.perf_counter() - t0
            res.losses.append(L)
            res.times.append(now)
            if log_every and it % log_every == 0:
                print(f"# iter {it}: loss {L:.6g} ({now:.2f} s)", flush=True)
            if threshold is not None and L <= threshold:
                res.iters_to_threshold = it
                res.secs_to_threshold = now
                break
            if it == max_iters:
                break
            if watch.stalled(it, L):
                res.stalled = True
                break
            self.gradient_step()
            if snap_levels is not None and snap_every and self.t % snap_every == 0:
                self.snap(snap_levels)
            if wrap_every and self.t % wrap_every == 0:
                self.shrinkwrap(wrap_sigmas, wrap_threshold)
        return res


@dataclass
class Problem:
    """A reconstruction workload: what is known, the data, and the ground truth for the threshold."""
    geom: synth.Geometry
    region: dict
    known_delta: np.ndarray
    known_beta: np.ndarray
    counts: np.ndarray
    scale: float
    truth: np.ndarray        # ground-truth box values (only used for the loss threshold)


def make_problem(seed_gt=4242, seed_noise=4243, n=256, n_slices=1024, photons=1e6) -> Problem:
    """The gradient workload: bars-on-substrate truth, unknown box = all slices and columns of the
    n/4 rows above the substrate (beta = delta/20), Poisson data at `photons` total from the
    model's own intensity (computed here by libmsl)."""
    w = synth.recon_256(seed_gt, n_slices=n_slices, n=n)
    g = w.geom
    region = synth.pattern_region(g, n // 4, n // 4)
    kd, kb = synth.known_stack(w, region)
    D = torch.from_numpy(w.delta).cuda()
    B = torch.from_numpy(w.beta).cuda()
    f, _ = msl.forward(g, D, B)
    I = msl.far_field(g, f).cpu().numpy()
    del D, B
    counts, s = synth.poisson_counts(I, photons, seed_noise)
    return Problem(g, region, kd, kb, counts, s, synth.box_values(w, region))


def seconds_to_threshold(p: Problem, init, factor=1.10, max_iters=5000, adam: Adam | None = None, ckpt_every=32,
                         log_every=0, graphs=True):
    """Plain reconstruction from `init`: time to the first iterate whose loss is <= factor * L(truth)."""
    R = Reconstructor(p.geom, p.known_delta, p.known_beta, p.region, p.counts, p.scale, ckpt_every=ckpt_every,
                      adam=adam, graphs=graphs)
    R.set_theta(p.truth)
    L_truth = float(R.loss().item()) * p.scale
    R.stack_gradients()   # the adjoint graph is captured here, before the clock starts
    res = R.run(init, max_iters, factor * L_truth, log_every=log_every)
    return L_truth, res


def learned_initial_guesses(net, problems, companions=None, batch=64):
    """Box values from the network for several problems in one inference batch: each problem's
    measured counts as an intensity estimate (counts / s) through the network's input map, the
    predicted cross-section (rows x columns, in units of 1e-5) clamped at 0 and repeated along
    the beam over the box's slices.  `companions` ([S][n][n] device tensor of inputs already
    through the input map, e.g. other measured images) fill the batch up to `batch` images, as in
    a run that infers many samples at once; only the problems' guesses are returned."""
    from . import learned, nn
    n = problems[0].geom.ny
    k = len(problems)
    B = max(batch, k)
    x = torch.zeros((1, B, n, n), dtype=torch.float32, device="cuda")
    for i, p in enumerate(problems):
        I = torch.from_numpy(np.ascontiguousarray(p.counts / p.scale, np.float32)).cuda()
        nn.logmap(I, learned.eps_of(n), learned.INPUT_A, 0.0, x[0, i])
    if companions is not None and B > k:
        m = min(B - k, companions.shape[0])
        x[0, k:k + m] = companions[:m]
    pred = net.forward(x)[:k].cpu().numpy().astype(np.float64) * 1e-5
    out = []
    for p, q in zip(problems, pred):
        cs = np.clip(q, 0.0, None).astype(np.float32)
        out.append(np.ascontiguousarray(np.broadcast_to(cs, (p.region["ns"],) + cs.shape)))
    return out


def learned_initial_guess(net, p: Problem, companions=None, batch=64):
    """``learned_initial_guesses`` for one problem (in a batch of `batch` images)."""
    return learned_initial_guesses(net, [p], companions, batch)[0]


REFINE_LR = 5e-6        # ADAM step from a learned start (sweep 4e-6 ... 8.5e-6 on the same workload)
REFINE_BUDGET = 400     # most ADAM steps from a learned start before the plain start takes over
STALL_WINDOW = 50       # ... or this many steps without the loss falling by STALL_GAIN
STALL_GAIN = 0.01


@dataclass
class LearnedRun:
    """Outcome of a reconstruction from a learned start with its error judge and fallback."""
    L_truth: float
    result: ReconResult          # the whole run (judging, learned attempt, plain fallback), one clock
    start: str                   # "learned", "plain" (judge) or "learned, then plain" (fallback)
    loss_learned_start: float
    loss_plain_start: float
    learned_iters: int | None    # ADAM steps of the learned attempt (None: not tried)
    stalled: bool = False


def seconds_to_threshold_learned(p: Problem, net, plain_init, factor=1.10, max_iters=5000, adam: Adam | None = None,
                                 ckpt_every=32, log_every=0, graphs=True, refine_lr=REFINE_LR, companions=None,
                                 batch=64, budget=REFINE_BUDGET, stall_window=STALL_WINDOW, stall_gain=STALL_GAIN):
    """Learned start with an error judge and a fallback.  Network inference (in a batch of
    `batch` images with `companions`), then the losses of the learned and the plain start are
    compared and ADAM starts from the lower one (the plain start when the learned guess is worse
    or not finite).  From the learned start ADAM takes the refinement step refine_lr (None: keep
    adam's) and is watched: if it has not reached the threshold within `budget` steps, or stalls
    (stall_window steps without a stall_gain fall of the loss), the plain start takes over with
    adam's own step.  One clock covers inference, judging, a failed attempt and the fallback."""
    R = Reconstructor(p.geom, p.known_delta, p.known_beta, p.region, p.counts, p.scale, ckpt_every=ckpt_every,
                      adam=adam, graphs=graphs)
    R.set_theta(p.truth)
    L_truth = float(R.loss().item()) * p.scale
    R.stack_gradients()   # the adjoint graph is captured here, before the clock starts
    threshold = factor * L_truth
    base_adam = R.adam
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    guess = learned_initial_guess(net, p, companions, batch)
    R.set_theta(guess)
    L_learned = float(R.loss().item()) * p.scale
    R.set_theta(plain_init)
    L_plain = float(R.loss().item()) * p.scale
    chose = bool(np.isfinite(L_learned) and L_learned < L_plain)
    t_judge = time.perf_counter() - t0
    out = ReconResult(threshold=threshold)

    def append(res, offset):
        out.losses += res.losses
        out.times += [t + offset for t in res.times]

    learned_iters, stalled, start = None, False, "plain"
    offset = t_judge
    if chose:
        R.adam = replace(base_adam, lr=float(refine_lr)) if refine_lr is not None else base_adam
        res = R.run(guess, min(budget, max_iters), threshold, log_every=log_every, stall_window=stall_window,
                    stall_gain=stall_gain)
        append(res, offset)
        learned_iters = len(res.losses) - 1
        stalled = res.stalled
        if res.secs_to_threshold is not None:
            out.iters_to_threshold = res.iters_to_threshold
            out.secs_to_threshold = res.secs_to_threshold + offset
            return LearnedRun(L_truth, out, "learned", L_learned, L_plain, learned_iters, stalled)
        offset += res.times[-1]
        start = "learned, then plain"
        R.adam = base_adam
    res = R.run(plain_init, max_iters, threshold, log_every=log_every)
    append(res, offset)
    if res.secs_to_threshold is not None:
        out.iters_to_threshold = res.iters_to_threshold + (learned_iters or 0)
        out.secs_to_threshold = res.secs_to_threshold + offset
    return LearnedRun(L_truth, out, start, L_learned, L_plain, learned_iters, stalled)
