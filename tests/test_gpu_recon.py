"""GPU parity of the reconstruction support (box scatter, ADAM step, driver) against the oracle."""
import numpy as np
import pytest

from oracle import msl_oracle as O
from oracle import recon_oracle as RO
from paper_2212_01253_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import msl
    msl.lib()
    return msl


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


REGION = {"s0": 2, "ns": 5, "y0": 16, "ny": 24, "z0": 3, "nz": 50, "beta_over_delta": 0.05}
GEOM = synth.Geometry(64, 64, 9, 1.0, 1.0, 5.0, 0.1, 0.0035, 0)


def test_region_scatter(M):
    import torch
    rng = np.random.default_rng(1)
    d = rng.random((9, 64, 64)).astype(np.float32)
    b = rng.random((9, 64, 64)).astype(np.float32)
    th = rng.random((5, 24, 50)).astype(np.float32)
    D, B = dev(d), dev(b)
    M.region_scatter(GEOM, REGION, dev(th), D, B)
    torch.cuda.synchronize()
    rd, _ = RO.scatter(d, b, REGION, th)
    assert np.array_equal(D.cpu().numpy(), rd.astype(np.float32))
    eb = b.copy()
    eb[RO.box_slices(REGION)] = np.float32(0.05) * th   # one float32 product, as on the device
    assert np.array_equal(B.cpu().numpy(), eb)


def test_region_adam_matches_oracle(M):
    import torch
    rng = np.random.default_rng(2)
    box = (5, 24, 50)
    th = (rng.random(box) * 3e-5).astype(np.float32)
    D = dev(rng.random((9, 64, 64)).astype(np.float32))
    B = dev(rng.random((9, 64, 64)).astype(np.float32))
    outside = D.cpu().numpy().copy()
    T, Mm, V = dev(th), dev(np.zeros(box, np.float32)), dev(np.zeros(box, np.float32))
    rth, rm, rv = th.astype(np.float64), np.zeros(box), np.zeros(box)
    lr, scale = 2e-6, 37.5
    gmax = np.zeros(box)
    adam = M.CAdam(lr, 0.9, 0.999, 1e-12, 0.0, 2.5e-5)
    for t in range(1, 6):
        gd = (rng.standard_normal((9, 64, 64)) * 10.0 ** rng.uniform(-4, 2, (9, 64, 64))).astype(np.float32)
        gb = (rng.standard_normal((9, 64, 64)) * 10.0 ** rng.uniform(-4, 2, (9, 64, 64))).astype(np.float32)
        M.region_adam_step(GEOM, REGION, adam, t, dev(gd), dev(gb), T, Mm, V, D, B, grad_scale=scale)
        ix = RO.box_slices(REGION)
        g = scale * (gd[ix].astype(np.float64) + 0.05 * gb[ix].astype(np.float64))
        # float32 forms g from two terms that may cancel: its error is relative to their size
        gmax = np.maximum(gmax, scale * (np.abs(gd[ix]) + 0.05 * np.abs(gb[ix])))
        rth, rm, rv = RO.adam_step(rth, g, rm, rv, t, lr, 0.9, 0.999, 1e-12, 0.0, 2.5e-5)
    torch.cuda.synchronize()
    gth = T.cpu().numpy()
    # each step is lr * (a ratio computed in float32): the parameters agree to a small
    # fraction of one step; the moments to float32 rounding of the gradients they sum
    assert np.max(np.abs(gth - rth)) <= 1e-4 * lr + 4e-12
    assert np.all(np.abs(Mm.cpu().numpy() - rm) <= 1e-6 * gmax)
    assert np.all(np.abs(V.cpu().numpy() - rv) <= 2e-6 * gmax * gmax)
    assert np.all((gth >= 0) & (gth <= np.float32(2.5e-5)))
    d = D.cpu().numpy()
    assert np.array_equal(d[ix], gth)
    mask = np.ones(d.shape, bool)
    mask[ix] = False
    assert np.array_equal(d[mask], outside[mask])
    assert np.allclose(B.cpu().numpy()[ix], 0.05 * gth, rtol=1e-7, atol=0)


def _small_problem():
    w = synth.parity_small(3)
    ns = 32
    g = synth.Geometry(**{**w.geom.as_dict(), "n_slices": ns})
    d, b = w.delta[:ns].copy(), w.beta[:ns].copy()
    region = {"s0": 0, "ns": ns, "y0": 24, "ny": 24, "z0": 0, "nz": 64, "beta_over_delta": 0.05}
    ix = RO.box_slices(region)
    b[ix] = np.float32(0.05) * d[ix]          # tie beta to delta in the truth as well
    kd, kb = d.copy(), b.copy()
    kd[ix] = 0
    kb[ix] = 0
    I = O.far_field(g, O.forward(g, d, b))
    counts, s = synth.poisson_counts(I, 1e5, 11)
    init = synth.random_init(region, 12)
    return g, region, kd, kb, counts, s, d[ix].copy(), init


def test_reconstruction_iterations_match_the_oracle(M):
    from paper_2212_01253_amd import recon
    g, region, kd, kb, counts, s, truth, init = _small_problem()
    lr = 1e-5
    amp = RO.poisson_loss_scale(counts, s)
    # ADAM steps by about lr * g / (|g| + eps): with a negligible eps every voxel moves a full lr
    # in the direction of its gradient's sign, and for the few voxels whose gradient is near zero
    # (below 1e-5 of the largest) float32 rounding decides that sign (one such flip moves a voxel
    # by 2 lr, as large as its delta, and the loss by ~1e-4).  An eps of 1e-2 of the largest
    # first gradient lets those voxels take near-zero steps, so the comparison measures the
    # gradient and the update, not rounding-decided signs; the descent is as fast (the loss falls
    # 832 -> 71 in four steps).
    _, g1 = RO.region_loss_and_gradient(g, kd, kb, region, init.astype(np.float64), amp)
    eps = 1e-2 * float(np.abs(s * g1).max())
    R = recon.Reconstructor(g, kd, kb, region, counts, s, ckpt_every=8, adam=recon.Adam(lr=lr, eps=eps))
    res = R.run(init, 4)
    th_gpu = R.theta.cpu().numpy()
    th, m, v = init.astype(np.float64), np.zeros(init.shape), np.zeros(init.shape)
    ref = []
    for t in range(1, 6):
        L, gth = RO.region_loss_and_gradient(g, kd, kb, region, th, amp)
        ref.append(s * L)
        if t == 5:
            break
        th, m, v = RO.adam_step(th, s * gth, m, v, t, lr, 0.9, 0.999, eps, 0.0, 1e-3)
    rl = np.abs(np.array(res.losses) - np.array(ref)) / np.array(ref)
    dth = np.abs(th_gpu - th)
    print("loss rel", rl, "theta |diff| / lr: max", dth.max() / lr, "mean", dth.mean() / lr)
    assert ref[-1] < 0.2 * ref[0]
    assert np.all(rl <= 1e-4)
    assert dth.max() <= 0.05 * lr
    assert dth.mean() <= 1e-3 * lr


def test_reconstruction_reduces_the_loss(M):
    from paper_2212_01253_amd import recon
    g, region, kd, kb, counts, s, truth, init = _small_problem()
    R = recon.Reconstructor(g, kd, kb, region, counts, s, ckpt_every=8, adam=recon.Adam())
    R.set_theta(truth)
    L_truth = float(R.loss().item()) * s
    L_ref = s * O.amp_loss(O.far_field(g, O.forward(g, *RO.scatter(kd, kb, region, truth))),
                           RO.poisson_loss_scale(counts, s))[0]
    assert L_truth == pytest.approx(L_ref, rel=1e-4)
    res = R.run(init, 300, threshold=1.1 * L_ref)
    print("L0", res.losses[0], "L_truth", L_ref, "iterations", res.iters_to_threshold, "final", res.losses[-1])
    assert res.iters_to_threshold is not None and res.losses[-1] <= 1.1 * L_ref


def test_region_snap_matches_the_oracle_bitwise(M):
    import torch
    rng = np.random.default_rng(9)
    levels = [0.0, 7.6e-6, 1.5e-5, 3e-5]
    th = rng.uniform(-1e-5, 4e-5, (5, 24, 50)).astype(np.float32)
    D = dev(rng.random((9, 64, 64)).astype(np.float32))
    B = dev(rng.random((9, 64, 64)).astype(np.float32))
    T = dev(th)
    M.region_snap(GEOM, REGION, levels, T, D, B)
    torch.cuda.synchronize()
    ref = RO.snap(th, levels)
    assert np.array_equal(T.cpu().numpy(), ref)
    assert np.array_equal(D.cpu().numpy()[RO.box_slices(REGION)], ref)


@pytest.mark.parametrize("k", [8, 1])
def test_reconstruction_from_captured_graphs_equals_eager(M, k):
    # the loss evaluation and the adjoint captured once as HIP graphs and replayed every iteration
    # (with the eager ADAM step, loss read-backs and synchronisations between replays) give
    # bit-identical losses and parameters; k = 1 runs the adjoint without recompute
    from paper_2212_01253_amd import recon
    g, region, kd, kb, counts, s, truth, init = _small_problem()
    out = []
    for graphs in (False, True):
        R = recon.Reconstructor(g, kd, kb, region, counts, s, ckpt_every=k, adam=recon.Adam(), graphs=graphs)
        res = R.run(init, 6)
        out.append((res.losses, R.theta.cpu().numpy()))
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])


def test_region_shrinkwrap_matches_the_oracle(M):
    import torch
    rng = np.random.default_rng(11)
    th = (rng.random((5, 24, 50)) * 3e-5).astype(np.float32)
    th[:, :, 20:30] *= 8.0                       # a bright band: the support forms around it
    D = dev(rng.random((9, 64, 64)).astype(np.float32))
    B = dev(rng.random((9, 64, 64)).astype(np.float32))
    T = dev(th)
    M.region_shrinkwrap(GEOM, REGION, (1.0, 1.5, 2.0), 0.3, T, D, B)
    torch.cuda.synchronize()
    ref, blur = RO.shrinkwrap(th.astype(np.float64), (1.0, 1.5, 2.0), 0.3)
    got = T.cpu().numpy()
    band = np.abs(blur - 0.3 * blur.max()) <= 1e-5 * blur.max()   # float32 blur may decide either way
    assert np.array_equal(got[~band], ref[~band].astype(np.float32))
    assert 0 < np.count_nonzero(got) < got.size
    assert np.array_equal(D.cpu().numpy()[RO.box_slices(REGION)], got)
