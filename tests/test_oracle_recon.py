"""Pins of the reconstruction oracle (ADAM step, box parameterisation) on the CPU.

ADAM (Kingma and Ba 2014, the optimiser of Sec. 4.1) has closed forms that
do not need the oracle's own formula: after the first step, and after any
number of steps under a constant gradient, the bias-corrected moments equal
g and g^2 exactly, so each step moves every parameter by lr g / (|g| + eps).
The box gradient (beta tied to delta) is pinned by central finite
differences of the FP64 forward model.
"""
import numpy as np
import pytest

from oracle import msl_oracle as O
from oracle import recon_oracle as R
from paper_2212_01253_amd import synth


def test_adam_first_step_is_a_signed_lr_step():
    rng = np.random.default_rng(1)
    th = rng.standard_normal(1000)
    g = rng.standard_normal(1000) * 10.0 ** rng.uniform(-3, 3, 1000)
    lr, eps = 1e-3, 1e-20   # eps / |g| <= 1e-14 here
    t1, m, v = R.adam_step(th, g, np.zeros(1000), np.zeros(1000), 1, lr, 0.9, 0.999, eps)
    assert np.allclose(t1, th - lr * np.sign(g), rtol=0, atol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


@pytest.mark.parametrize("b1,b2", [(0.9, 0.999), (0.5, 0.9), (0.0, 0.0)])
def test_adam_constant_gradient_moves_linearly(b1, b2):
    rng = np.random.default_rng(2)
    th0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-2, 1e-3
    th, m, v = th0, np.zeros(50), np.zeros(50)
    for t in range(1, 31):
        th, m, v = R.adam_step(th, g, m, v, t, lr, b1, b2, eps)
        assert np.allclose(th, th0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)


def test_adam_clamps_to_the_box():
    th, _, _ = R.adam_step(np.array([0.0, 1.0, 0.5]), np.array([1.0, -1.0, 0.0]), np.zeros(3), np.zeros(3), 1,
                           0.3, lo=0.0, hi=1.1)
    assert th.tolist() == [0.0, 1.1, 0.5]


def test_adam_minimises_a_quadratic():
    rng = np.random.default_rng(3)
    a = rng.uniform(0.1, 10, 20)
    c = rng.standard_normal(20)
    th, m, v = np.zeros(20), np.zeros(20), np.zeros(20)
    for t in range(1, 3001):
        lr = 0.05 if t < 2000 else 0.005
        th, m, v = R.adam_step(th, a * (th - c), m, v, t, lr)
    assert np.max(np.abs(th - c)) < 1e-2


def test_box_gradient_matches_finite_differences():
    # tiny geometry; the box covers rows 2..4, columns 1..5, slices 1..3
    g = synth.Geometry(8, 8, 4, 1.0, 1.0, 10.0, 0.1, 0.004, 0)
    rng = np.random.default_rng(4)
    kd = np.zeros((4, 8, 8))
    kb = np.zeros((4, 8, 8))
    kd[:, :2] = 7.6e-6
    kb[:, :2] = 1.7e-7
    region = {"s0": 1, "ns": 2, "y0": 2, "ny": 3, "z0": 1, "nz": 5, "beta_over_delta": 0.05}
    theta = rng.uniform(0, 3e-5, (2, 3, 5))
    meas = np.abs(rng.standard_normal((8, 8)))
    L, gth = R.region_loss_and_gradient(g, kd, kb, region, theta, meas)
    h = 1e-9
    for idx in [(0, 0, 0), (1, 2, 4), (0, 1, 3), (1, 0, 2)]:
        tp, tm = theta.copy(), theta.copy()
        tp[idx] += h
        tm[idx] -= h
        fd = (R.region_loss_and_gradient(g, kd, kb, region, tp, meas)[0]
              - R.region_loss_and_gradient(g, kd, kb, region, tm, meas)[0]) / (2 * h)
        assert fd == pytest.approx(gth[idx], rel=1e-5, abs=1e-9 * abs(gth).max())
    # the tie to beta matters: dropping it changes the gradient
    _, gd, gb, _, _, _ = O.loss_and_gradient(g, *R.scatter(kd, kb, region, theta), meas)
    ix = R.box_slices(region)
    assert np.max(np.abs(gd[ix] - gth)) > 1e-3 * np.max(np.abs(gth))


def test_scatter_sets_only_the_box():
    kd = np.full((3, 4, 4), 2.0)
    kb = np.full((3, 4, 4), 3.0)
    region = {"s0": 1, "ns": 1, "y0": 1, "ny": 2, "z0": 0, "nz": 3, "beta_over_delta": 0.5}
    d, b = R.scatter(kd, kb, region, np.full((1, 2, 3), 8.0))
    assert d.sum() == 2.0 * 48 + 6 * 6.0 and b.sum() == 3.0 * 48 + 6 * 1.0
    assert d[1, 1, 0] == 8.0 and b[1, 2, 2] == 4.0 and d[1, 1, 3] == 2.0 and d[0, 1, 0] == 2.0


def test_poisson_scale_identity():
    # the detector loss sum (sqrt(s I) - sqrt(C))^2 equals s times the amplitude loss against sqrt(C/s)
    rng = np.random.default_rng(5)
    I = rng.uniform(0, 2, (16, 16))
    C, s = synth.poisson_counts(I, 1e6, 7)
    assert C.sum() == pytest.approx(1e6, rel=0.01)
    Ldet = np.sum((np.sqrt(s * I) - np.sqrt(C.astype(np.float64))) ** 2)
    L, _, _ = O.amp_loss(I, R.poisson_loss_scale(C, s))
    assert s * L == pytest.approx(Ldet, rel=1e-12)


def test_snap_picks_the_nearest_level_by_brute_force():
    rng = np.random.default_rng(8)
    levels = [0.0, 7.6e-6, 1.5e-5, 3e-5]
    th = rng.uniform(-1e-5, 4e-5, 500).astype(np.float32)
    th[:4] = [3.8e-6, 1.13e-5, 2.25e-5, -0.0]   # near midpoints and zero
    got = R.snap(th, levels)
    for t, s in zip(th, got):
        dists = [abs(float(np.float32(t) - np.float32(l))) for l in levels]
        best = min(range(len(levels)), key=lambda i: (dists[i], i))
        assert s == np.float32(levels[best])


def test_shrinkwrap_properties():
    rng = np.random.default_rng(10)
    th = rng.standard_normal((6, 10, 12))
    # no blur: the support is |theta| above the fraction of its maximum
    out, b = R.shrinkwrap(th, (0, 0, 0), 0.4)
    assert np.array_equal(out, np.where(np.abs(th) > 0.4 * np.abs(th).max(), th, 0.0))
    # the blur of an interior impulse keeps its sum and is symmetric
    imp = np.zeros((21, 21, 21))
    imp[10, 10, 10] = 1.0
    _, b = R.shrinkwrap(imp, (1.5, 2.0, 1.0), 0.0)
    assert b.sum() == pytest.approx(1.0, rel=1e-12)
    assert np.allclose(b, b[::-1, ::-1, ::-1]) and b[10, 10, 10] == b.max()
    # a higher threshold keeps a subset
    lo, _ = R.shrinkwrap(th, (1.0, 1.0, 1.0), 0.2)
    hi, _ = R.shrinkwrap(th, (1.0, 1.0, 1.0), 0.5)
    assert np.all((hi != 0) <= (lo != 0)) and np.count_nonzero(hi) < np.count_nonzero(lo)
