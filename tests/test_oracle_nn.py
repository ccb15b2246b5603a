"""Pins of the network oracle (CPU): convolution against a library correlation, adjoints by
dot-product identities and finite differences, bfloat16 rounding against its definition."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import nn_oracle as N


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 2, 12, 10))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    for s in (1, 2):
        y = N.conv3x3(x, w, b, s)
        for o in range(4):
            for bb in range(2):
                ref = sum(correlate2d(x[c, bb], w[o, c], mode="same") for c in range(3)) + b[o]
                assert np.allclose(y[o, bb], ref[::s, ::s], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("s", [1, 2])
def test_conv_adjoint_identities(s):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 2, 8, 8))
    w = rng.standard_normal((5, 3, 3, 3))
    dy = rng.standard_normal((5, 2, 8 // s, 8 // s))
    dx, dw, db = N.conv3x3_adjoint(x, w, dy, s)
    y = N.conv3x3(x, w, None, s)
    assert np.sum(y * dy) == pytest.approx(np.sum(x * dx), rel=1e-12)   # linear in x
    assert np.sum(y * dy) == pytest.approx(np.sum(w * dw), rel=1e-12)   # linear in w
    assert np.allclose(db, dy.sum(axis=(1, 2, 3)))


def test_resampling_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 4, 5))
    y = rng.standard_normal((2, 3, 8, 10))
    assert np.sum(N.upsample2(x) * y) == pytest.approx(np.sum(x * N.upsample2_adjoint(y)), rel=1e-12)
    p = rng.standard_normal((3, 16, 5))
    q = rng.standard_normal((3, 4, 5))
    assert np.sum(N.rowpool(p, 4) * q) == pytest.approx(np.sum(p * N.rowpool_adjoint(q, 4)), rel=1e-12)
    assert np.allclose(N.rowpool(np.arange(8.0).reshape(1, 8, 1), 4)[0, :, 0], [1.5, 5.5])


def test_bf16_rounding_by_definition():
    rng = np.random.default_rng(4)
    vals = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.uniform(-30, 30, 2000),
                           [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 0.0, -0.0, 3.0e38]]).astype(np.float32)
    got = N.bf16(vals)
    for v, r in zip(vals.astype(np.float64), got):
        # the two bfloat16 neighbours of v (truncation and next up in magnitude)
        u = np.array([v], np.float32).view(np.uint32)[0]
        lo = np.array([u & 0xFFFF0000], np.uint32).view(np.float32)[0].astype(np.float64)
        hi = np.array([(u & 0xFFFF0000) + 0x10000], np.uint32).view(np.float32)[0].astype(np.float64)
        dlo, dhi = abs(v - lo), abs(v - hi)
        if dlo < dhi:
            assert r == lo
        elif dhi < dlo:
            assert r == hi
        else:   # tie: the even one (last kept bit 0)
            assert r == (lo if ((u >> 16) & 1) == 0 else hi)
    assert np.isnan(N.bf16(np.float32(np.nan))) and N.bf16(np.float32(np.inf)) == np.inf


def small_params(rng, c):
    return {name: (rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (9 * ci)), rng.standard_normal(co) * 0.1)
            for name, ci, co, s, act in N.layer_specs(c)}


def test_unet_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    c = 2
    params = small_params(rng, c)
    x = rng.standard_normal((2, 2, 16, 16))
    t = rng.standard_normal((2, 4, 16))

    def loss(p):
        pred, _ = N.unet_forward(p, x, quantize=False)
        return N.mse(pred, t)[0]

    pred, cache = N.unet_forward(params, x, quantize=False)
    L, dpred = N.mse(pred, t)
    grads = N.unet_adjoint(params, cache, dpred)
    h = 1e-6
    for name in ("e1a", "e3b", "e4b", "d3", "d1", "out"):
        w, b = params[name]
        for idx in [(0, 0, 1, 1), (w.shape[0] - 1, w.shape[1] - 1, 2, 0)]:
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            fd = (loss({**params, name: (wp, b)}) - loss({**params, name: (wm, b)})) / (2 * h)
            assert fd == pytest.approx(grads[name][0][idx], rel=1e-5, abs=1e-9)
        bp, bm = b.copy(), b.copy()
        bp[0] += h
        bm[0] -= h
        fd = (loss({**params, name: (w, bp)}) - loss({**params, name: (w, bm)})) / (2 * h)
        assert fd == pytest.approx(grads[name][1][0], rel=1e-5, abs=1e-9)


def test_row_features_closed_forms():
    # rows that are affine in the column index: mean over all columns = value at (W-1)/2, centre
    # column = value at W/2, seven-column mean = value at W/2
    B, H, W = 2, 3, 16
    a = np.arange(B * H, dtype=np.float64).reshape(B, H, 1)
    x = a + 0.5 * np.arange(W)[None, None, :]
    f = N.row_features(x)
    assert np.allclose(f[:, :H], a[:, :, 0] + 0.5 * (W - 1) / 2)
    assert np.allclose(f[:, H:2 * H], a[:, :, 0] + 0.5 * (W // 2))
    assert np.allclose(f[:, 2 * H:], a[:, :, 0] + 0.5 * (W // 2))
    # the summaries are invariant under a cyclic shift of the columns only for the full mean;
    # the centre terms pick up the shifted columns
    xs = np.roll(x, 3, axis=2)
    assert np.allclose(N.row_features(xs)[:, :H], f[:, :H])


def test_row_bias_adjoint_identity():
    rng = np.random.default_rng(9)
    p = rng.standard_normal((5, 3))
    dy = rng.standard_normal((3, 5, 7))
    y0 = np.zeros((3, 5, 7))
    lhs = np.sum(N.add_row_bias(y0, p) * dy)
    rhs = np.sum(p * N.add_row_bias_adjoint(dy))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_global_head_gradient_matches_finite_differences():
    rng = np.random.default_rng(6)
    c, H, hid = 2, 16, 8
    params = small_params(rng, c)
    params["g1"] = (rng.standard_normal((hid, 3 * H)) * 0.3, rng.standard_normal(hid) * 0.1)
    params["g2"] = (rng.standard_normal((H // 4, hid)) * 0.3, rng.standard_normal(H // 4) * 0.1)
    x = rng.standard_normal((2, 2, H, H))
    t = rng.standard_normal((2, H // 4, H))

    def loss(p):
        pred, _ = N.unet_forward(p, x, quantize=False)
        return N.mse(pred, t)[0]

    pred, cache = N.unet_forward(params, x, quantize=False)
    L, dpred = N.mse(pred, t)
    grads = N.unet_adjoint(params, cache, dpred)
    h = 1e-6
    for name in ("g1", "g2", "e2b"):
        w, b = params[name]
        for idx in [tuple(0 for _ in w.shape), tuple(n - 1 for n in w.shape)]:
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            fd = (loss({**params, name: (wp, b)}) - loss({**params, name: (wm, b)})) / (2 * h)
            assert fd == pytest.approx(grads[name][0][idx], rel=1e-5, abs=1e-9)
        bp, bm = b.copy(), b.copy()
        bp[-1] += h
        bm[-1] -= h
        fd = (loss({**params, name: (w, bp)}) - loss({**params, name: (w, bm)})) / (2 * h)
        assert fd == pytest.approx(grads[name][1][-1], rel=1e-5, abs=1e-9)
