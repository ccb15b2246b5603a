"""Full-size parity on the throughput workload (512 x 512 grid, 2048 slices).

The benchmark's forward sweep, in the launch configuration the benchmark
uses, against the FP64 oracle on the same float32 inputs: exit field relative
L2 <= 2e-5 and far-field intensity relative L2 <= 1e-4, and element by
element (every field element, every far-field amplitude; parity_gates.py).  The oracle needs
about a minute of host CPU here.  A gradient check at the gradient workload's
full size (256 x 256 x 1024, checkpoints every 32 slices) compares the GPU
gradient with the oracle's on 16 sampled voxels and on its relative L2 norm;
the benchmark's own gradient step (512 x 512 x 2048, slice pack reused,
checkpoints every 32 slices, and again with one at every slice) gets the same
comparison.  The batched workload (96 instances in one call, as benchmarked)
is compared with the oracle on the instance with the fewest slices of every
grid size.
"""
import math
import time

import numpy as np
import pytest

from oracle import msl_oracle as O
from paper_2212_01253_amd import synth
from parity_gates import check_forward, fmt

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import msl
    msl.lib()
    msl.set_schedule(0)
    yield msl
    msl.set_schedule(0)


@pytest.mark.timeout(900)
def test_forward_512x512x2048(M):
    w = synth.throughput_512()
    g = w.geom
    print(f"workload {w.name} alpha {math.degrees(g.alpha_i_rad):.4f} deg", flush=True)
    D = torch.from_numpy(w.delta).cuda()
    B = torch.from_numpy(w.beta).cuda()
    f, _ = M.forward(g, D, B, ckpt_every=32)
    I = M.far_field(g, f)
    torch.cuda.synchronize()
    f = f.cpu().numpy()
    I = I.cpu().numpy()
    del D, B
    t0 = time.time()
    rf = O.forward(g, w.delta, w.beta)
    rI = O.far_field(g, rf)
    print(f"oracle {time.time() - t0:.1f} s", flush=True)
    print(fmt(check_forward(f, rf, I, rI)), flush=True)


@pytest.mark.timeout(900)
def test_gradient_256x256x1024(M):
    w = synth.recon_256()
    g = w.geom
    rng = np.random.default_rng(4243)
    # measured amplitudes from a perturbed structure with 5 % multiplicative noise
    t0 = time.time()
    meas = (np.sqrt(O.far_field(g, O.forward(g, w.delta * 1.05, w.beta * 1.05)))
            * (1 + 0.05 * rng.random((g.ny, g.nz)))).astype(np.float32)
    D = torch.from_numpy(w.delta).cuda()
    B = torch.from_numpy(w.beta).cuda()
    f, ck = M.forward(g, D, B, ckpt_every=32)
    I = M.far_field(g, f)
    loss, gI = M.amp_loss(g, I, torch.from_numpy(meas).cuda())
    gpsi = M.far_field_adjoint(g, f, gI)
    gd, gb, gp = M.adjoint(g, D, B, ck, 32, gpsi)
    torch.cuda.synchronize()
    gd, gb, gp = gd.cpu().numpy(), gb.cpu().numpy(), gp.cpu().numpy()
    L = float(loss.cpu())
    del D, B
    rL, rd, rb, rp, _, _ = O.loss_and_gradient(g, w.delta, w.beta, meas)
    pick = np.random.default_rng(4245)
    idx = [tuple(int(pick.integers(0, n)) for n in w.delta.shape) for _ in range(16)]
    scale = np.sqrt(np.mean(rd ** 2))
    worst = max(abs(gd[i] - rd[i]) / scale for i in idx)
    print(f"oracle {time.time() - t0:.1f} s; loss {abs(L - rL) / rL:.2e}; grad delta {rel(gd, rd):.2e} "
          f"beta {rel(gb, rb):.2e} probe {rel(gp, rp):.2e}; sampled voxels {worst:.2e}", flush=True)
    assert abs(L - rL) <= 1e-4 * rL
    assert rel(gd, rd) <= 1e-3 and rel(gb, rb) <= 1e-3 and rel(gp, rp) <= 1e-3
    assert worst <= 1e-3


@pytest.mark.timeout(900)
def test_gradient_512x512x2048_as_benchmarked(M):
    # the benchmark's gradient step (slice pack, forward with checkpoints every 32 slices reusing
    # the pack, far field, loss, far-field adjoint, adjoint reusing the pack) at its full size,
    # against the oracle's gradient; the same step with a checkpoint at every slice (no recompute)
    w = synth.throughput_512()
    g = w.geom
    rng = np.random.default_rng(2214)
    t0 = time.time()
    meas = (np.sqrt(O.far_field(g, O.forward(g, w.delta * 1.05, w.beta * 1.05)))
            * (1 + 0.05 * rng.random((g.ny, g.nz)))).astype(np.float32)
    print(f"measured amplitudes {time.time() - t0:.1f} s", flush=True)
    D = torch.from_numpy(w.delta).cuda()
    B = torch.from_numpy(w.beta).cuda()
    Mm = torch.from_numpy(meas).cuda()
    out = {}
    for k in (32, 1):
        ws = M.workspace(g, k, "cuda")
        M.pack_slices(g, D, B, ws)
        f, ck = M.forward(g, D, B, None, k, ws=ws, reuse_pack=True)
        I = M.far_field(g, f, ws=ws)
        loss, gI = M.amp_loss(g, I, Mm, ws=ws)
        gpsi = M.far_field_adjoint(g, f, gI, ws=ws)
        gd, gb, gp = M.adjoint(g, D, B, ck, k, gpsi, ws=ws, want_probe=True, reuse_pack=True)
        torch.cuda.synchronize()
        out[k] = (float(loss.cpu()), gd.cpu().numpy(), gb.cpu().numpy(), gp.cpu().numpy())
        del ws, ck, f, I, gI, gpsi, gd, gb, gp
        torch.cuda.empty_cache()
    del D, B, Mm
    L, gd, gb, gp = out[32]
    t0 = time.time()
    rL, rd, rb, rp, _, _ = O.loss_and_gradient(g, w.delta, w.beta, meas)
    pick = np.random.default_rng(2215)
    idx = [tuple(int(pick.integers(0, n)) for n in w.delta.shape) for _ in range(16)]
    scale = np.sqrt(np.mean(rd ** 2))
    worst = max(abs(gd[i] - rd[i]) / scale for i in idx)
    print(f"oracle {time.time() - t0:.1f} s; loss {abs(L - rL) / rL:.2e}; grad delta {rel(gd, rd):.2e} "
          f"beta {rel(gb, rb):.2e} probe {rel(gp, rp):.2e}; sampled voxels {worst:.2e}", flush=True)
    assert abs(L - rL) <= 1e-4 * rL
    assert rel(gd, rd) <= 1e-3 and rel(gb, rb) <= 1e-3 and rel(gp, rp) <= 1e-3
    assert worst <= 1e-3
    L1, gd1, gb1, gp1 = out[1]
    print(f"every-slice checkpoints: bitwise equal {np.array_equal(gd1, gd) and np.array_equal(gb1, gb)}", flush=True)
    assert L1 == L
    assert rel(gd1, gd) <= 1e-6 and rel(gb1, gb) <= 1e-6 and rel(gp1, gp) <= 1e-6


class _Slices:
    """Slice s of a compact stack as the oracle reads it (no dense copy)."""

    def __init__(self, pool, index):
        self.pool, self.index = pool, index

    def __getitem__(self, s):
        return self.pool[self.index[s]]


@pytest.mark.timeout(900)
def test_batched_workload_as_benchmarked_sampled_instances(M):
    # the benchmark's batched forward (all 96 instances in one call), then the oracle on the
    # instance with the fewest slices of every grid size and on the longest 512-point one
    stacks = synth.batch_workload(96)
    items = []
    for cs in stacks:
        g = cs.geom
        items.append({"geom": g, "pool_delta": torch.from_numpy(cs.pool_delta).cuda(),
                      "pool_beta": torch.from_numpy(cs.pool_beta).cuda(),
                      "slice_index": torch.from_numpy(cs.index.astype(np.int32)).cuda(),
                      "field": torch.empty((g.ny, g.nz), dtype=torch.complex64, device="cuda"),
                      "intensity": torch.empty((g.ny, g.nz), dtype=torch.float32, device="cuda")})
    ws = M.batch_workspace(items)
    M.forward_batch(items, ws)
    torch.cuda.synchronize()
    pick = {}
    for i, cs in enumerate(stacks):
        n = cs.geom.ny
        if n not in pick or cs.geom.n_slices < stacks[pick[n]].geom.n_slices:
            pick[n] = i
    assert sorted(pick) == [128, 256, 512, 1024]
    longest = max((i for i, cs in enumerate(stacks) if cs.geom.ny == 512), key=lambda i: stacks[i].geom.n_slices)
    for n, i in sorted(pick.items()) + [(512, longest)]:
        cs, it = stacks[i], items[i]
        t0 = time.time()
        rf = O.forward(cs.geom, _Slices(cs.pool_delta, cs.index), _Slices(cs.pool_beta, cs.index))
        rI = O.far_field(cs.geom, rf)
        print(f"instance {i} ({cs.name}): oracle {time.time() - t0:.1f} s", flush=True)
        errs = check_forward(it["field"].cpu().numpy(), rf, it["intensity"].cpu().numpy(), rI, what=f"instance {i}")
        print(f"instance {i}: {fmt(errs)}", flush=True)
