"""GPU parity: the HIP library through its C ABI against the FP64 oracle.

Tolerances: exit field relative L2 <= 2e-5 and far-field intensity relative
L2 <= 1e-4 (complex64 on the GPU against complex128 on the CPU from the same
float32 inputs), and element by element: every field element and every
far-field amplitude sqrt(I) within the bounds that follow from the float32
error model (parity_gates.py).  Gradients: relative L2 <= 1e-3.
"""
import math

import numpy as np
import pytest

from oracle import msl_oracle as O
from paper_2212_01253_amd import synth
from parity_gates import check_field, check_forward, check_intensity, fmt

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

FIELD_TOL = 2e-5
INT_TOL = 1e-4
GRAD_TOL = 1e-3
SCHEDULES = [1, 2]  # per-pass launches, persistent cooperative kernel


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import msl
    msl.lib()
    yield msl
    msl.set_schedule(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_forward(M, g, d, b, probe=None, k=0, sched=1):
    M.set_schedule(sched)
    ws = M.workspace(g, k)
    f, ck = M.forward(g, dev(d), dev(b), None if probe is None else dev(probe.astype(np.complex64)),
                      ckpt_every=k, ws=ws)
    M.workspace_status(ws)   # raises if a persistent barrier gave up
    I = M.far_field(g, f, ws=ws)
    M.workspace_status(ws)
    torch.cuda.synchronize()
    return f.cpu().numpy(), I.cpu().numpy(), (None if ck is None else ck.cpu().numpy())


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_parity_64x64x128(M, sched, seed):
    w = synth.parity_small(seed)
    f, I, _ = run_forward(M, w.geom, w.delta, w.beta, sched=sched)
    rf = O.forward(w.geom, w.delta, w.beta)
    rI = O.far_field(w.geom, rf)
    print(f"seed {seed} sched {sched}: {fmt(check_forward(f, rf, I, rI))}")


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("ny,nz,ns", [(16, 16, 5), (32, 64, 9), (128, 32, 7), (16, 1024, 4), (1024, 16, 4),
                                      (256, 256, 12), (512, 128, 6), (1024, 1024, 3)])
def test_size_sweep(M, sched, ny, nz, ns):
    g = synth.Geometry(ny, nz, ns, 0.9, 1.2, 8.0, 0.12, math.radians(0.15), 0)
    d, b = synth.random_stack(ny, nz, ns, ny * 7 + nz + ns, 3e-5, 2e-6)
    p = synth.random_field(ny, nz, ny + nz)
    f, I, _ = run_forward(M, g, d, b, probe=p, sched=sched)
    rf = O.forward(g, d, b, p.astype(np.complex128))
    rI = O.far_field(g, rf)
    print(f"{ny}x{nz}x{ns}: {fmt(check_forward(f, rf, I, rI))}")


@pytest.mark.parametrize("sched", SCHEDULES)
def test_exact_propagator(M, sched):
    w = synth.parity_small(3)
    g = synth.Geometry(**{**w.geom.as_dict(), "propagator": 1})
    f, I, _ = run_forward(M, g, w.delta, w.beta, sched=sched)
    rf = O.forward(g, w.delta, w.beta)
    print(fmt(check_forward(f, rf, I, O.far_field(g, rf))))
    # and it is a different model from the paraxial one
    assert rel(rf, O.forward(w.geom, w.delta, w.beta)) > 1e-3


def test_checkpoints_hold_entrance_fields(M):
    w = synth.parity_small(4)
    g = synth.Geometry(**{**w.geom.as_dict(), "n_slices": 40})
    d, b = w.delta[:40], w.beta[:40]
    f, _, ck = run_forward(M, g, d, b, k=7)
    rf, kept = O.forward(g, d, b, keep=True)
    assert ck.shape == (6, 64, 64)
    for c in range(6):
        check_field(ck[c], kept[7 * c], what=f"checkpoint {c}")
    check_field(f, rf)


def test_vacuum_composition_on_gpu(M):
    ny, nz = 64, 32
    p = synth.random_field(ny, nz, 5)
    g = synth.Geometry(ny, nz, 16, 1.0, 1.0, 6.0, 0.1, 0.0, 0)
    g1 = synth.Geometry(ny, nz, 1, 1.0, 1.0, 96.0, 0.1, 0.0, 0)
    z = np.zeros((16, ny, nz), np.float32)
    f16, _, _ = run_forward(M, g, z, z, probe=p)
    f1, _, _ = run_forward(M, g1, z[:1], z[:1], probe=p)
    check_field(f16, f1)


def test_parseval_on_gpu(M):
    w = synth.parity_small(2)
    f, I, _ = run_forward(M, w.geom, w.delta, np.zeros_like(w.beta))
    n0 = w.geom.ny * w.geom.nz  # |probe|^2 = 1 per pixel
    assert abs(np.sum(np.abs(f.astype(np.complex128)) ** 2) / n0 - 1) <= 1e-5
    assert abs(I.astype(np.float64).sum() / np.sum(np.abs(f.astype(np.complex128)) ** 2) - 1) <= 1e-5


def test_deterministic_repeat(M):
    w = synth.parity_small(1)
    f1, I1, _ = run_forward(M, w.geom, w.delta, w.beta)
    f2, I2, _ = run_forward(M, w.geom, w.delta, w.beta)
    assert np.array_equal(f1, f2) and np.array_equal(I1, I2)


def test_far_field_and_loss(M):
    ny, nz = 64, 128
    g = synth.Geometry(ny, nz, 1, 1.0, 1.0, 10.0, 0.1, 0.0, 0)
    psi = synth.random_field(ny, nz, 11)
    meas = synth.random_measured_amplitude(ny, nz, 12, 3.0)
    fpsi = dev(psi)
    I = M.far_field(g, fpsi)
    loss, gI = M.amp_loss(g, I, dev(meas))
    gpsi = M.far_field_adjoint(g, fpsi, gI)
    torch.cuda.synchronize()
    rI = O.far_field(g, psi.astype(np.complex128))
    L, _, rgI = O.amp_loss(I.cpu().numpy().astype(np.float64), meas)
    check_intensity(I.cpu().numpy(), rI)
    assert abs(float(loss.cpu()) - L) <= 1e-9 * abs(L)
    assert rel(gI.cpu().numpy(), rgI) <= 1e-6
    rg = O.far_field_adjoint(g, psi.astype(np.complex128), gI.cpu().numpy().astype(np.float64))
    assert rel(gpsi.cpu().numpy(), rg) <= 1e-5


def test_loss_zero_intensity_pixels(M):
    ny, nz = 16, 16
    g = synth.Geometry(ny, nz, 1, 1.0, 1.0, 10.0, 0.1, 0.0, 0)
    I = np.zeros((ny, nz), np.float32)
    I[3, 4] = 4.0
    m = np.full((ny, nz), 0.5, np.float32)
    loss, gI = M.amp_loss(g, dev(I), dev(m))
    torch.cuda.synchronize()
    L, _, rgI = O.amp_loss(I, m)
    assert float(loss.cpu()) == pytest.approx(L, rel=1e-12)
    assert np.allclose(gI.cpu().numpy(), rgI, atol=1e-7)


def _grad_case(M, g, d, b, meas, k, sched=1, reuse_pack=False):
    M.set_schedule(sched)
    D, B = dev(d), dev(b)
    ws = M.workspace(g, k)
    f, ck = M.forward(g, D, B, ckpt_every=k, ws=ws)
    M.workspace_status(ws)
    I = M.far_field(g, f, ws=ws)
    loss, gI = M.amp_loss(g, I, dev(meas), ws=ws)
    gpsi = M.far_field_adjoint(g, f, gI, ws=ws)
    gd, gb, gp = M.adjoint(g, D, B, ck, k, gpsi, ws=ws, reuse_pack=reuse_pack)
    M.workspace_status(ws)
    torch.cuda.synchronize()
    return float(loss.cpu()), gd.cpu().numpy(), gb.cpu().numpy(), gp.cpu().numpy()


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("k", [1, 3, 32, 40])
def test_gradient_parity(M, sched, k):
    w = synth.parity_small(5)
    g = synth.Geometry(**{**w.geom.as_dict(), "n_slices": 40})
    d, b = w.delta[:40], w.beta[:40]
    meas = (np.sqrt(O.far_field(g, O.forward(g, d * 1.1, b * 1.1)))
            * (1 + 0.05 * np.random.default_rng(6).random((64, 64)))).astype(np.float32)
    L, gd, gb, gp = _grad_case(M, g, d, b, meas, k, sched)
    rL, rd, rb, rp, _, _ = O.loss_and_gradient(g, d, b, meas)
    print(f"k={k}: loss {abs(L - rL) / rL:.2e} gd {rel(gd, rd):.2e} gb {rel(gb, rb):.2e} gp {rel(gp, rp):.2e}")
    assert abs(L - rL) <= 1e-4 * abs(rL)
    assert rel(gd, rd) <= GRAD_TOL
    assert rel(gb, rb) <= GRAD_TOL
    assert rel(gp, rp) <= GRAD_TOL


def test_gradient_reusing_the_forward_slice_pack(M):
    w = synth.parity_small(8)
    g = synth.Geometry(**{**w.geom.as_dict(), "n_slices": 33})
    d, b = w.delta[:33], w.beta[:33]
    meas = (np.sqrt(O.far_field(g, O.forward(g, d * 1.1, b * 1.1)))).astype(np.float32)
    a = _grad_case(M, g, d, b, meas, 4)
    r = _grad_case(M, g, d, b, meas, 4, reuse_pack=True)
    for x, y in zip(a[1:], r[1:]):
        assert np.array_equal(x, y)


def test_forward_from_a_separate_slice_pack(M):
    # msl_pack_slices then msl_forward(MSL_REUSE_SLICE_PACK) equals msl_forward
    # packing by itself, bit for bit; the pack survives a forward with another
    # probe (it depends on delta, beta, wavelength and dx only)
    w = synth.parity_small(9)
    g = synth.Geometry(**{**w.geom.as_dict(), "n_slices": 37})
    D, B = dev(w.delta[:37]), dev(w.beta[:37])
    ws = M.workspace(g, 0)
    ref, _ = M.forward(g, D, B, ws=ws)
    ref = ref.cpu().numpy()
    ws2 = M.workspace(g, 0)
    M.pack_slices(g, D, B, ws2)
    p = dev(synth.random_field(64, 64, 3).astype(np.complex64))
    M.forward(g, D, B, p, ws=ws2, reuse_pack=True)
    f, _ = M.forward(g, D, B, ws=ws2, reuse_pack=True)
    torch.cuda.synchronize()
    assert np.array_equal(f.cpu().numpy(), ref)


def test_gradient_exact_propagator(M):
    w = synth.parity_small(6)
    g = synth.Geometry(**{**w.geom.as_dict(), "n_slices": 24, "propagator": 1})
    d, b = w.delta[:24], w.beta[:24]
    # measured amplitudes near the model's (the reconstruction regime); the
    # loss derivative 1 - m / sqrt(I) is singular at dark pixels otherwise
    meas = (np.sqrt(O.far_field(g, O.forward(g, d * 1.1, b * 1.1)))
            * (1 + 0.05 * np.random.default_rng(9).random((64, 64)))).astype(np.float32)
    L, gd, gb, gp = _grad_case(M, g, d, b, meas, 5)
    rL, rd, rb, rp, _, _ = O.loss_and_gradient(g, d, b, meas)
    assert rel(gd, rd) <= GRAD_TOL and rel(gb, rb) <= GRAD_TOL and rel(gp, rp) <= GRAD_TOL


def test_autograd_wrappers(M):
    w = synth.parity_small(7)
    g = synth.Geometry(**{**w.geom.as_dict(), "n_slices": 16})
    d = dev(w.delta[:16]).requires_grad_(True)
    b = dev(w.beta[:16]).requires_grad_(True)
    meas = (np.sqrt(O.far_field(g, O.forward(g, w.delta[:16] * 0.9, w.beta[:16] * 0.9)))
            * (1 + 0.05 * np.random.default_rng(10).random((64, 64)))).astype(np.float32)
    f = M.Multislice.apply(d, b, g, None, 4)
    I = M.FarField.apply(f, g)
    L = M.AmpLoss.apply(I, dev(meas), g)
    L.backward()
    rL, rd, rb, _, _, _ = O.loss_and_gradient(g, w.delta[:16], w.beta[:16], meas)
    assert abs(float(L.detach().cpu()) - rL) <= 1e-4 * rL
    assert rel(d.grad.cpu().numpy(), rd) <= GRAD_TOL
    assert rel(b.grad.cpu().numpy(), rb) <= GRAD_TOL


def _random_case(seed):
    """A seeded geometry: independent row and column counts, pitches, slice count, checkpoint
    interval, propagator and probe (None or a random field)."""
    rng = np.random.default_rng(seed)
    ny, nz = (int(v) for v in rng.choice([16, 32, 64, 128, 256], 2))
    ns = int(rng.integers(2, 49))
    k = int(rng.choice([1, 2, 5, 16, ns]))
    prop = int(rng.integers(0, 2))
    g = synth.Geometry(ny, nz, ns, float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.5, 2.0)),
                       float(rng.uniform(2.0, 20.0)), float(rng.uniform(0.08, 0.15)),
                       math.radians(float(rng.uniform(0.05, 0.5))), prop)
    d, b = synth.random_stack(ny, nz, ns, seed + 1, 3e-5, 2e-6)
    probe = None if rng.random() < 0.5 else synth.random_field(ny, nz, seed + 2)
    return g, d, b, probe, k


@pytest.mark.parametrize("seed", range(7000, 7012))
def test_random_geometries_forward_and_gradient(M, seed):
    g, d, b, probe, k = _random_case(seed)
    M.set_schedule(1)
    D, B = dev(d), dev(b)
    P = None if probe is None else dev(probe.astype(np.complex64))
    ws = M.workspace(g, k)
    f, ck = M.forward(g, D, B, P, k, ws=ws)
    I = M.far_field(g, f, ws=ws)
    rf = O.forward(g, d, b, None if probe is None else probe.astype(np.complex128))
    rI = O.far_field(g, rf)
    meas = (np.sqrt(O.far_field(g, O.forward(g, d * 1.1, b * 1.1,
                                             None if probe is None else probe.astype(np.complex128))))
            * (1 + 0.05 * np.random.default_rng(seed).random((g.ny, g.nz)))).astype(np.float32)
    loss, gI = M.amp_loss(g, I, dev(meas), ws=ws)
    gpsi = M.far_field_adjoint(g, f, gI, ws=ws)
    gd, gb, gp = M.adjoint(g, D, B, ck, k, gpsi, probe=P, ws=ws)
    torch.cuda.synchronize()
    rL, rd, rb, rp, _, _ = O.loss_and_gradient(g, d, b, meas, None if probe is None else probe.astype(np.complex128))
    errs = (rel(f.cpu().numpy(), rf), rel(I.cpu().numpy(), rI), abs(float(loss.cpu()) - rL) / rL,
            rel(gd.cpu().numpy(), rd), rel(gb.cpu().numpy(), rb), rel(gp.cpu().numpy(), rp))
    print(seed, g.ny, g.nz, g.n_slices, k, g.propagator, probe is not None, ["%.1e" % e for e in errs])
    print(seed, fmt(check_forward(f.cpu().numpy(), rf, I.cpu().numpy(), rI)))
    assert errs[0] <= FIELD_TOL and errs[1] <= INT_TOL and errs[2] <= 1e-4
    assert errs[3] <= GRAD_TOL and errs[4] <= GRAD_TOL and errs[5] <= GRAD_TOL


def test_persistent_barrier_that_gives_up_is_reported(M):
    # the host forces the bounded barrier wait to give up (spin limit 0: a block that finds
    # the others not yet arrived raises the error word at once); every kernel still exits
    # normally, the status query reports the failure and the working field holds NaN; with
    # the limit restored the same call is valid again and equals the per-pass schedule
    w = synth.parity_small(2)
    g = synth.Geometry(**{**w.geom.as_dict(), "n_slices": 24})
    D, B = dev(w.delta[:24]), dev(w.beta[:24])
    ws = M.workspace(g, 0)
    prev = M.set_barrier_spin_limit(0)
    try:
        M.set_schedule(2)
        f, _ = M.forward(g, D, B, ws=ws)
        with pytest.raises(M.MslError) as e:
            M.workspace_status(ws)
        assert e.value.status == M.ERR_HIP and "barrier" in str(e.value)
        assert torch.isnan(f).all()
    finally:
        M.set_barrier_spin_limit(prev)
    f, _ = M.forward(g, D, B, ws=ws)
    M.workspace_status(ws)
    M.set_schedule(1)
    ref, _ = M.forward(g, D, B, ws=ws)
    M.workspace_status(ws)
    torch.cuda.synchronize()
    check_field(f.cpu().numpy(), ref.cpu().numpy().astype(np.complex128))
