"""GPU parity of the learned-initialiser kernels and network against the FP64 oracle."""
import numpy as np
import pytest

from oracle import nn_oracle as N
from oracle import recon_oracle as RO
from paper_2212_01253_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import nn
    nn.lib()
    return nn


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def bf16_bits(x):
    """bfloat16 bit patterns (int16) of values that are already bfloat16-representable."""
    f = np.ascontiguousarray(np.asarray(x, np.float32))
    return (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_matches_float64_products(T, ta, tb):
    import torch
    rng = np.random.default_rng(1)
    M, Nn, K = 70, 130, 45
    a = N.bf16(rng.standard_normal((M, K)))
    b = N.bf16(rng.standard_normal((K, Nn)))
    A = a.T.copy() if ta else a
    Bm = b.T.copy() if tb else b
    bias = rng.standard_normal(M).astype(np.float32)
    C0 = rng.standard_normal((M, Nn)).astype(np.float32)
    C = dev(C0)
    C16 = torch.zeros((M, Nn), dtype=torch.int16, device="cuda")
    T.gemm(M, Nn, K, dev(bf16_bits(A)), A.shape[1], ta, dev(bf16_bits(Bm)), Bm.shape[1], tb, C, Nn,
           beta=0.5, bias=dev(bias), relu=True, C16=C16)
    torch.cuda.synchronize()
    ref = np.maximum(a @ b + 0.5 * C0 + bias[:, None], 0)
    scale = np.abs(a) @ np.abs(b) + 1.0
    got = C.cpu().numpy()
    assert np.all(np.abs(got - ref) <= 4e-6 * scale)
    g16 = C16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    assert np.array_equal(g16.view(np.float32), N.bf16(got).astype(np.float32))


@pytest.mark.parametrize("s", [1, 2])
def test_convolution_through_patches_matches_the_oracle(T, s):
    import torch
    rng = np.random.default_rng(2)
    C, B, H, W, O = 5, 2, 12, 8, 7
    x = rng.standard_normal((C, B, H, W)).astype(np.float32)
    w = rng.standard_normal((O, C, 3, 3))
    wb = N.bf16(w)
    bias = rng.standard_normal(O).astype(np.float32)
    Ho, Wo = H // s, W // s
    col = torch.zeros(C * 9 * B * Ho * Wo, dtype=torch.int16, device="cuda")
    T.im2col(C, B, H, W, s, dev(x), col)
    y = torch.zeros((O, B, Ho, Wo), dtype=torch.float32, device="cuda")
    T.gemm(O, B * Ho * Wo, C * 9, dev(bf16_bits(wb.reshape(O, -1))), C * 9, 0, col, B * Ho * Wo, 0, y, B * Ho * Wo,
           bias=dev(bias))
    # backward data: dcol = W^T dy, dx = col2im(dcol)
    dy = N.bf16(rng.standard_normal((O, B, Ho, Wo)))
    dcol = torch.zeros(C * 9 * B * Ho * Wo, dtype=torch.float32, device="cuda")
    T.gemm(C * 9, B * Ho * Wo, O, dev(bf16_bits(wb.reshape(O, -1))), C * 9, 1, dev(bf16_bits(dy.reshape(O, -1))),
           B * Ho * Wo, 0, dcol, B * Ho * Wo)
    dx = torch.zeros((C, B, H, W), dtype=torch.float32, device="cuda")
    T.col2im(C, B, H, W, s, dcol, dx)
    torch.cuda.synchronize()
    ref = N.conv3x3(N.bf16(x), wb, bias, s)
    rdx, rdw, _ = N.conv3x3_adjoint(N.bf16(x), wb, dy, s)
    assert rel(y.cpu().numpy(), ref) <= 1e-6
    assert rel(dx.cpu().numpy(), rdx) <= 1e-6


@pytest.mark.parametrize("C,B,H,W,O,s", [(5, 2, 12, 8, 7, 1), (5, 2, 12, 8, 7, 2), (2, 3, 16, 16, 70, 1),
                                         (16, 2, 8, 24, 9, 2), (8, 1, 32, 32, 4, 1), (20, 2, 6, 72, 130, 1),
                                         (33, 1, 10, 40, 40, 2), (130, 1, 9, 70, 17, 1), (3, 2, 64, 64, 1, 1),
                                         (24, 2, 20, 48, 40, 2)])
def test_implicit_convolution(T, C, B, H, W, O, s):
    # the products on halo tiles sum in another order than the explicit ones (patch matrix, then
    # product; split product for the weight gradient), so the two agree to float32 rounding, and all
    # match the oracle; so does the input gradient.  Shapes cover ragged tiles (output widths 24, 40,
    # 70, 72; heights not multiples of the tile), channel counts that are not multiples of the 16- or
    # 32-channel chunks, row counts over one 128-row block, and both weight-gradient paths (halo
    # tiles when the output width is a multiple of 8, the patch-column product otherwise).
    import torch
    rng = np.random.default_rng(C * 100 + O)
    x = rng.standard_normal((C, B, H, W)).astype(np.float32)
    w = rng.standard_normal((O, C, 3, 3))
    wb = N.bf16(w)
    w16 = dev(bf16_bits(wb.reshape(O, -1)))
    bias = rng.standard_normal(O).astype(np.float32)
    Ho, Wo = H // s, W // s
    n = B * Ho * Wo
    col = torch.zeros(C * 9 * n, dtype=torch.int16, device="cuda")
    T.im2col(C, B, H, W, s, dev(x), col)
    y_exp = torch.zeros((O, B, Ho, Wo), dtype=torch.float32, device="cuda")
    T.gemm(O, n, C * 9, w16, C * 9, 0, col, n, 0, y_exp, n, bias=dev(bias), relu=True)
    y = torch.zeros((O, B, Ho, Wo), dtype=torch.float32, device="cuda")
    T.conv3x3(O, C, B, H, W, s, w16, dev(x), y, bias=dev(bias), relu=True)
    dy = N.bf16(rng.standard_normal((O, B, Ho, Wo)))
    dy16 = dev(bf16_bits(dy))
    dx = torch.full((C, B, H, W), float("nan"), dtype=torch.float32, device="cuda")
    T.conv3x3_adjoint(O, C, B, H, W, s, w16, dy16, dx)
    dx2 = dx.clone()
    T.conv3x3_adjoint(O, C, B, H, W, s, w16, dy16, dx2, accumulate=True)   # dx2 = dx + dx, exactly
    splits = 3
    parts = torch.zeros(splits * O * C * 9, dtype=torch.float32, device="cuda")
    dw_exp = torch.zeros((O, C * 9), dtype=torch.float32, device="cuda")
    T.gemm_splitk(O, C * 9, n, dy16, n, 0, col, n, 1, dw_exp, C * 9, splits, parts)
    dw = torch.full((O, C * 9), float("nan"), dtype=torch.float32, device="cuda")
    T.conv3x3_weight_grad(O, C, B, H, W, s, dy16, dev(x), dw, splits, parts)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), y_exp.cpu().numpy()) <= 1e-6
    assert rel(dw.cpu().numpy(), dw_exp.cpu().numpy()) <= 1e-6
    ref = np.maximum(N.conv3x3(N.bf16(x), wb, bias, s), 0.0)
    rdx, rdw, _ = N.conv3x3_adjoint(N.bf16(x), wb, dy, s)
    assert rel(y.cpu().numpy(), ref) <= 1e-6
    assert rel(dx.cpu().numpy(), rdx) <= 1e-6
    assert np.array_equal(dx2.cpu().numpy(), 2 * dx.cpu().numpy())
    assert rel(dw.cpu().numpy(), rdw.reshape(O, C * 9)) <= 1e-6
    # bfloat16 activations: the same values as bfloat16 bits stage the same operands, so the
    # convolution and its weight gradient equal the float32-input results bit for bit, and a
    # bfloat16 output is the float32 output rounded to nearest even
    x16 = dev(bf16_bits(N.bf16(x)))
    yb = torch.zeros((O, B, Ho, Wo), dtype=torch.float32, device="cuda")
    T.conv3x3(O, C, B, H, W, s, w16, x16, yb, bias=dev(bias), relu=True)
    y16 = torch.zeros((O, B, Ho, Wo), dtype=torch.int16, device="cuda")
    T.conv3x3(O, C, B, H, W, s, w16, x16, y16, bias=dev(bias), relu=True)
    ry16 = torch.zeros(O * n, dtype=torch.int16, device="cuda")
    T.to_bf16(y, ry16)
    torch.cuda.synchronize()
    assert np.array_equal(yb.cpu().numpy(), y.cpu().numpy())
    assert np.array_equal(y16.cpu().numpy().ravel(), ry16.cpu().numpy())
    dwb = torch.full((O, C * 9), float("nan"), dtype=torch.float32, device="cuda")
    T.conv3x3_weight_grad(O, C, B, H, W, s, dy16, x16, dwb, splits, parts)   # both paths (Wo % 8)
    torch.cuda.synchronize()
    assert np.array_equal(dwb.cpu().numpy(), dw.cpu().numpy())


def test_resampling_and_elementwise_kernels(T):
    import torch
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 2, 4, 6)).astype(np.float32)
    y = torch.zeros((3, 2, 8, 12), dtype=torch.float32, device="cuda")
    T.upsample2(3, 2, 4, 6, dev(x), y)
    dy = rng.standard_normal((3, 2, 8, 12)).astype(np.float32)
    dx = torch.zeros((3, 2, 4, 6), dtype=torch.float32, device="cuda")
    T.upsample2_adjoint(3, 2, 4, 6, dev(dy), dx)
    p = rng.standard_normal((2, 16, 5)).astype(np.float32)
    q = torch.zeros((2, 4, 5), dtype=torch.float32, device="cuda")
    T.rowpool(2, 16, 5, 4, dev(p), q)
    dq = rng.standard_normal((2, 4, 5)).astype(np.float32)
    dp = torch.zeros((2, 16, 5), dtype=torch.float32, device="cuda")
    T.rowpool_adjoint(2, 16, 5, 4, dev(dq), dp)
    r = dev(rng.standard_normal(1000).astype(np.float32))
    dr = rng.standard_normal(1000).astype(np.float32)
    drd = dev(dr)
    T.relu_adjoint(r, drd)
    s = torch.zeros(7, dtype=torch.float32, device="cuda")
    X = rng.standard_normal((7, 333)).astype(np.float32)
    T.rowsum(7, 333, dev(X), s, torch.zeros(7 * 64, dtype=torch.float32, device="cuda"))
    pr, tg = rng.standard_normal(5000).astype(np.float32), rng.standard_normal(5000).astype(np.float32)
    gr = torch.zeros(5000, dtype=torch.float32, device="cuda")
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    T.mse(dev(pr), dev(tg), gr, loss)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), N.upsample2(x).astype(np.float32))
    # bfloat16 bits are copied unchanged (aligned pair stores, and the scalar path for an odd offset)
    xb = N.bf16(x).astype(np.float32)
    for off in (0, 1):
        y16 = torch.zeros(3 * 2 * 8 * 12 + off, dtype=torch.int16, device="cuda")
        T.upsample2(3, 2, 4, 6, dev(bf16_bits(xb)), y16[off:])
        torch.cuda.synchronize()
        assert np.array_equal(y16[off:].cpu().numpy(), bf16_bits(N.upsample2(xb)).ravel())
    assert np.allclose(dx.cpu().numpy(), N.upsample2_adjoint(dy), rtol=1e-6, atol=1e-6)
    assert np.allclose(q.cpu().numpy(), N.rowpool(p, 4), rtol=1e-6, atol=1e-6)
    assert np.allclose(dp.cpu().numpy(), N.rowpool_adjoint(dq, 4), rtol=1e-6, atol=0)
    rr = r.cpu().numpy()
    assert np.array_equal(drd.cpu().numpy(), np.where(rr > 0, dr, 0).astype(np.float32))
    assert np.allclose(s.cpu().numpy(), X.astype(np.float64).sum(axis=1), rtol=1e-5, atol=1e-4)
    L, g = N.mse(pr, tg)
    assert float(loss.cpu()) == pytest.approx(L, rel=1e-12)
    assert np.allclose(gr.cpu().numpy(), g, rtol=1e-6, atol=0)


@pytest.mark.parametrize("M,N", [(7, 333), (5, 4096), (3, 1030)])
def test_gradient_preparation_in_one_pass(T, M, N):
    # msl_nn_grad_prep: the same bfloat16 copy as the ReLU adjoint followed by the conversion, bit
    # for bit, and the row sums of the masked gradient (other summation order: float32 rounding);
    # with y None no mask.  dy is left as it was.  N = 4096 takes the four-column path, 333 and 1030
    # the single-column one (1030 is not a multiple of 4).
    import torch
    rng = np.random.default_rng(M * 1000 + N)
    y = rng.standard_normal((M, N)).astype(np.float32)
    dy = rng.standard_normal((M, N)).astype(np.float32)
    parts = torch.zeros(M * 64, dtype=torch.float32, device="cuda")
    for relu in (True, False):
        dyd = dev(dy)
        d16 = torch.zeros(M * N, dtype=torch.int16, device="cuda")
        gb = torch.zeros(M, dtype=torch.float32, device="cuda")
        T.grad_prep(M, N, dev(y) if relu else None, dyd, d16, gb, parts)
        g = np.where(y > 0, dy, 0).astype(np.float32) if relu else dy
        ref16 = torch.zeros(M * N, dtype=torch.int16, device="cuda")
        T.to_bf16(dev(g), ref16)
        torch.cuda.synchronize()
        assert np.array_equal(dyd.cpu().numpy(), dy)
        assert np.array_equal(d16.cpu().numpy(), ref16.cpu().numpy())
        assert np.allclose(gb.cpu().numpy(), g.astype(np.float64).sum(axis=1), rtol=1e-5, atol=1e-4)
    # y as bfloat16 bits masks like the float32 values they hold: bit for bit the same outputs
    from oracle import nn_oracle as nno          # (N is the column count here)
    yb = nno.bf16(y).astype(np.float32)
    yb[0, :5] = 0.0                               # exact zeros and a negative zero mask too
    yb[0, 5] = -0.0
    outs = []
    for yt in (dev(yb), dev(bf16_bits(yb))):
        d16 = torch.zeros(M * N, dtype=torch.int16, device="cuda")
        gb = torch.zeros(M, dtype=torch.float32, device="cuda")
        T.grad_prep(M, N, yt, dev(dy), d16, gb, parts)
        torch.cuda.synchronize()
        outs.append((d16.cpu().numpy(), gb.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_global_head_kernels(T):
    import torch
    rng = np.random.default_rng(8)
    B, H, W, R = 3, 12, 20, 6
    x = rng.standard_normal((B, H, W)).astype(np.float32)
    f16 = torch.zeros(B * 3 * H, dtype=torch.int16, device="cuda")
    T.row_features(B, H, W, dev(x), f16)
    shift = rng.standard_normal(3 * H).astype(np.float32)
    scale = rng.uniform(0.5, 4.0, 3 * H).astype(np.float32)
    n16 = torch.zeros(B * 3 * H, dtype=torch.int16, device="cuda")
    T.row_features(B, H, W, dev(x), n16, dev(shift), dev(scale))
    p = rng.standard_normal((R, B)).astype(np.float32)
    y0 = rng.standard_normal((B, R, W)).astype(np.float32)
    y = dev(y0)
    T.add_row_bias(B, R, W, dev(p), y)
    dy = rng.standard_normal((B, R, W)).astype(np.float32)
    dp = torch.zeros((R, B), dtype=torch.float32, device="cuda")
    T.row_bias_adjoint(B, R, W, dev(dy), dp)
    torch.cuda.synchronize()
    # bfloat16 features: within half an ulp of the float64 values rounded the same way, after the
    # float32 sums (one ulp apart at most where the sum order decides a tie)
    got = f16.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    got = got.view(np.float32).astype(np.float64).reshape(B, 3 * H)
    ref = N.row_features(x)
    assert np.allclose(got, N.bf16(ref), rtol=2 ** -7, atol=0)
    assert np.array_equal(got[:, H:2 * H], N.bf16(x[:, :, W // 2]))   # the centre column: a pure copy
    gotn = (n16.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert np.allclose(gotn.reshape(B, 3 * H), N.bf16((ref - shift) * scale), rtol=2 ** -7, atol=1e-6)
    assert np.allclose(y.cpu().numpy(), N.add_row_bias(y0, p), rtol=1e-6, atol=1e-6)
    assert np.allclose(dp.cpu().numpy(), N.add_row_bias_adjoint(dy), rtol=1e-5, atol=1e-5)


def test_weight_adam_matches_the_oracle(T):
    import torch
    rng = np.random.default_rng(4)
    w0 = rng.standard_normal(3000).astype(np.float32)
    w, m, v = dev(w0), dev(np.zeros(3000, np.float32)), dev(np.zeros(3000, np.float32))
    w16 = torch.zeros(3000, dtype=torch.int16, device="cuda")
    rw, rm, rv = w0.astype(np.float64), np.zeros(3000), np.zeros(3000)
    for t in range(1, 4):
        g = rng.standard_normal(3000).astype(np.float32)
        T.adam(w, dev(g), m, v, w16, 1e-3, 0.9, 0.999, 1e-8, t)
        rw, rm, rv = RO.adam_step(rw, g, rm, rv, t, 1e-3, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    got = w.cpu().numpy()
    assert np.max(np.abs(got - rw)) <= 1e-4 * 1e-3 + 1e-6 * np.abs(rw).max()
    g16 = w16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    assert np.array_equal(g16.view(np.float32), N.bf16(got).astype(np.float32))


def test_rendered_pools_equal_the_host_generator(T):
    import torch
    samples = [synth.training_sample(7000 + i, n=64, n_slices=96) for i in range(5)]
    nfs = [len(b) for _, b, _ in samples]
    nps = [len(c) - 1 for _, _, c in samples]
    offs = np.cumsum([0] + nps[:-1]).astype(np.int64)
    boxes = np.zeros((5, T.MAX_BOXES, 8), np.float32)
    cuts = np.zeros((5, T.MAX_CUTS), np.int32)
    wts = np.zeros((5, T.MAX_CUTS), np.float32)
    for i, (g, b, c) in enumerate(samples):
        boxes[i, :len(b)] = b
        cuts[i, :len(c)] = c
        wts[i, :len(c) - 1] = np.diff(c) / g.n_slices
    pd = torch.zeros((sum(nps), 64, 64), dtype=torch.float32, device="cuda")
    pb = torch.zeros_like(pd)
    T.render_pools(5, 64, 64, 16, synth.SUBSTRATE_DELTA, synth.SUBSTRATE_BETA, dev(boxes), dev(np.array(nfs, np.int32)),
                   dev(cuts), dev(np.array(nps, np.int32)), dev(offs), max(nps), pd, pb)
    tgt = torch.zeros((5, 16, 64), dtype=torch.float32, device="cuda")
    T.pool_average(5, 64, 64, 16, 16, dev(wts), dev(np.array(nps, np.int32)), dev(offs), max(nps), pd, 1e5, tgt)
    torch.cuda.synchronize()
    for i, (g, b, c) in enumerate(samples):
        cs = synth.compact_bars_on_substrate(g, 7000 + i + 1, substrate_rows=16, n_bars=(8, 32), bar_height=(2, 40),
                                             bar_width=(4, 64), bar_len_frac=(1 / 8, 1.0), n_lines=(2, 8),
                                             line_height=(2, 40), line_width=(1, 4), delta_range=(5e-6, 3e-5),
                                             beta_over_delta=1 / 20)
        assert np.array_equal(pd[offs[i]:offs[i] + nps[i]].cpu().numpy(), cs.pool_delta)
        assert np.array_equal(pb[offs[i]:offs[i] + nps[i]].cpu().numpy(), cs.pool_beta)
        d, _ = cs.dense()
        ref = d[:, 16:32, :].astype(np.float64).mean(axis=0) * 1e5
        assert np.allclose(tgt[i].cpu().numpy(), ref, rtol=1e-5, atol=1e-6)


def test_unet_forward_and_gradients_match_the_oracle(T):
    import torch
    from paper_2212_01253_amd import learned
    net = learned.UNet(c=4, seed=3, n=32)
    rng = np.random.default_rng(5)
    B, H, W = 2, 32, 32
    x = rng.standard_normal((1, B, H, W)).astype(np.float32)
    tgt = rng.standard_normal((B, H // 4, W)).astype(np.float32)
    off = rng.standard_normal((H // 4, W)).astype(np.float32)
    net.set_offset(dev(off))
    # non-zero biases to exercise them
    host = net.w.cpu().numpy()
    for name, ci, co, s, act in learned.layer_specs(4):   # two input channels
        wo, bo, *_ = net.off[name]
        host[bo:bo + co] = rng.standard_normal(co) * 0.1
    for name, (wo, bo, no, ni) in net.head_off.items():   # the global head too
        host[bo:bo + no] = rng.standard_normal(no) * 0.1
        host[wo:bo] = rng.standard_normal(no * ni) * np.sqrt(1.0 / ni)
    net.set_flat(host)
    fshift = rng.standard_normal(3 * H).astype(np.float32) * 0.1
    fscale = rng.uniform(0.5, 2.0, 3 * H).astype(np.float32)
    net.set_feature_norm(dev(fshift), dev(fscale))
    pred = net.forward(dev(x))
    loss = net.loss_and_grad(dev(tgt))
    torch.cuda.synchronize()
    params = net.params_numpy()
    # the network's second input channel is the row coordinate, -1 .. 1 (as the buffer holds it)
    ramp = net._bufs["x"][1:].cpu().numpy()
    assert np.allclose(ramp[0, 0, :, 0], np.linspace(-1.0, 1.0, H), atol=1e-6) and np.all(ramp == ramp[:, :, :, :1])
    xin = np.concatenate([x, ramp]).astype(np.float64)
    rpred, cache = N.unet_forward(params, xin, offset=off, feat_norm=(fshift, fscale))
    rL, dpred = N.mse(rpred, tgt)
    rg = N.unet_adjoint(params, cache, dpred)
    print("pred", rel(pred.cpu().numpy(), rpred), "loss", abs(float(loss.cpu()) - rL) / rL)
    assert rel(pred.cpu().numpy(), rpred) <= 1e-5
    assert abs(float(loss.cpu()) - rL) <= 1e-4 * rL
    g = net.grads_numpy()
    errs = {}
    for name in params:
        errs[name] = (rel(g[name][0], rg[name][0]), rel(g[name][1], rg[name][1]))
        print(name, errs[name], np.linalg.norm(rg[name][0]), np.linalg.norm(rg[name][1]))
    # Both sides round the backward products' inputs to bfloat16 from float32 values that differ in
    # the last bits (float32 against float64 arithmetic), so now and then one element sits on a
    # rounding boundary and the two round it apart: one such element moves the gradients below it
    # by about 2^-8 of its share (~1e-4 relative here).  Every layer must stay within that, and
    # most layers, which no such element reaches, within float32 accuracy.
    for name, (e_w, e_b) in errs.items():
        assert e_w <= 1e-3 and e_b <= 1e-3, name
    tight = sum(1 for e_w, e_b in errs.values() if e_w <= 1e-6 and e_b <= 1e-6)
    assert tight >= 0.6 * len(errs), errs
    # Against the unquantised FP64 network (no bfloat16 rounding anywhere): the bfloat16 network
    # differs by first-order product rounding only.  Every quantised product rounds both of its
    # operands to bfloat16 (unit roundoff u = 2^-9), a relative error of at most 2u per product;
    # along the longest path, 12 convolutions and the head's 2 dense layers forward, then as many
    # products backward, so with unit amplification per layer the output is within 2 * 14 u and
    # the gradients within 2 * 28 u of the exact network's.
    u = 2.0 ** -9
    xpred, xcache = N.unet_forward(params, xin, offset=off, feat_norm=(fshift, fscale), quantize=False)
    _, xdpred = N.mse(xpred, tgt)
    xg = N.unet_adjoint(params, xcache, xdpred)
    e_pred = rel(pred.cpu().numpy(), xpred)
    gv = np.concatenate([np.concatenate([g[n][0].ravel(), g[n][1].ravel()]) for n in params])
    xv = np.concatenate([np.concatenate([xg[n][0].ravel(), xg[n][1].ravel()]) for n in params])
    e_grad = rel(gv, xv)
    print(f"against the unquantised network: prediction {e_pred:.2e} (bound {28 * u:.2e}), "
          f"gradients {e_grad:.2e} (bound {56 * u:.2e})")
    assert e_pred <= 2 * 14 * u
    assert e_grad <= 2 * 28 * u


@pytest.mark.parametrize("ta,tb,splits", [(0, 1, 7), (0, 0, 1), (1, 1, 33)])
def test_split_gemm_matches_float64_products(T, ta, tb, splits):
    import torch
    rng = np.random.default_rng(6)
    M, Nn, K = 40, 70, 5000
    a = N.bf16(rng.standard_normal((M, K)))
    b = N.bf16(rng.standard_normal((K, Nn)))
    A = a.T.copy() if ta else a
    Bm = b.T.copy() if tb else b
    C = torch.zeros((M, Nn), dtype=torch.float32, device="cuda")
    parts = torch.zeros(splits * M * Nn, dtype=torch.float32, device="cuda")
    T.gemm_splitk(M, Nn, K, dev(bf16_bits(A)), A.shape[1], ta, dev(bf16_bits(Bm)), Bm.shape[1], tb, C, Nn, splits,
                  parts)
    torch.cuda.synchronize()
    scale = np.abs(a) @ np.abs(b)
    assert np.all(np.abs(C.cpu().numpy() - a @ b) <= 4e-6 * scale)


def test_learned_start_and_its_judge(M=None):
    """The error judge on a held-out reconstruction (small grid, short training): the learned
    start has a much lower loss and is chosen; the judge falls back to the plain start when the
    learned guess is not usable (here: NaN offset)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import learned, recon
    net, info = learned.train_initialiser(n_samples=512, steps=60, batch=16, n=128, n_slices=128, n_val=64)
    info.pop("companions")
    print(info)
    assert np.isfinite(info["val_mse"]) and info["val_mse"] <= 1.5 * info["val_mse_mean_map"]
    p = recon.make_problem(seed_gt=4300, seed_noise=4301, n=128, n_slices=128, photons=1e7)
    init = synth.random_init(p.region, 4302)
    adam = recon.Adam()
    run = recon.seconds_to_threshold_learned(p, net, init, max_iters=0, adam=adam, ckpt_every=8)
    print("start losses: learned", run.loss_learned_start, "plain", run.loss_plain_start)
    # the judge picks the learned start (no steps here: max_iters=0, so the run ends right after)
    assert run.start.startswith("learned") and run.loss_learned_start < 0.7 * run.loss_plain_start   # 112784 / 232480
    net.set_offset(torch.full_like(net.offset, float("nan")))
    run2 = recon.seconds_to_threshold_learned(p, net, init, max_iters=800, adam=adam, ckpt_every=8)
    assert run2.start == "plain" and not np.isfinite(run2.loss_learned_start)
    assert run2.loss_plain_start == run.loss_plain_start
    assert run2.result.iters_to_threshold is not None   # the plain start reaches 1.1 x L(truth) (485 steps)


def test_refinement_that_misses_the_threshold_falls_back_to_the_plain_start():
    """A learned start whose refinement does not reach the threshold within its step budget hands
    over to the plain start; the failed attempt's time counts, and the run still reaches the
    threshold (the small network here: its start is chosen, but 12 steps do not suffice)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import learned, recon
    net, info = learned.train_initialiser(n_samples=512, steps=60, batch=16, n=128, n_slices=128, n_val=64)
    p = recon.make_problem(seed_gt=4300, seed_noise=4301, n=128, n_slices=128, photons=1e7)
    init = synth.random_init(p.region, 4302)
    run = recon.seconds_to_threshold_learned(p, net, init, max_iters=800, ckpt_every=8, budget=12,
                                             companions=info["companions"], batch=64)
    res = run.result
    print(run.start, run.learned_iters, res.iters_to_threshold, res.secs_to_threshold)
    assert run.start == "learned, then plain" and run.learned_iters == 12
    assert res.iters_to_threshold is not None and res.iters_to_threshold > 12
    assert res.secs_to_threshold > res.times[12]     # the learned attempt's 12 steps are on the clock
    assert res.losses[-1] <= res.threshold


def test_learned_start_reaches_the_threshold_sooner():
    """What the trained initialiser gains, in seconds to the loss threshold, on a held-out truth
    of the gradient workload (256 x 256 grid, 1024 slices; truth, noise and plain start seeds
    the training set does not use): the learned start, with inference in a batch of 64 and the
    error judge on the clock, reaches 1.1 x L(truth) in fewer seconds than the plain start."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import learned, recon
    net, info = learned.train_initialiser(n_samples=4096, steps=300)
    p = recon.make_problem(seed_gt=4270, seed_noise=4271)
    init = synth.random_init(p.region, 4272)
    L_truth, plain = recon.seconds_to_threshold(p, init)
    run = recon.seconds_to_threshold_learned(p, net, init, companions=info["companions"], batch=64)
    print(f"plain {plain.secs_to_threshold:.2f} s ({plain.iters_to_threshold} steps); learned "
          f"{run.result.secs_to_threshold:.2f} s ({run.result.iters_to_threshold} steps, start {run.start})")
    assert plain.secs_to_threshold is not None and run.result.secs_to_threshold is not None
    assert run.start == "learned"
    assert run.result.secs_to_threshold < plain.secs_to_threshold
