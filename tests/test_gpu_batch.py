"""GPU checks of the batched forward (compact slice stacks, many instances per call)."""
import numpy as np
import pytest

from oracle import msl_oracle as O
from paper_2212_01253_amd import synth
from parity_gates import check_forward, fmt

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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def small_batch():
    """Mixed grids (square and not), slice counts from 1 up, wavelengths and angles."""
    specs = [(64, 64, 40), (32, 32, 1), (32, 64, 17), (64, 64, 33), (16, 16, 9), (32, 32, 24), (64, 64, 2),
             (16, 32, 12)]
    out = []
    for i, (ny, nz, ns) in enumerate(specs):
        rng = np.random.default_rng(100 + i)
        g = synth.Geometry(ny, nz, ns, 1.0, 1.0, 5.0, float(rng.uniform(0.08, 0.15)),
                           np.radians(float(rng.uniform(0.05, 0.5))), 0)
        cs = synth.compact_bars_on_substrate(g, 200 + i, substrate_rows=ny // 4, n_bars=(2, 6),
                                             bar_height=(1, max(2, ny // 8)), bar_width=(1, nz // 4),
                                             bar_len_frac=(0.125, 1.0), n_lines=(1, 3),
                                             delta_range=(5e-6, 3e-5), beta_over_delta=0.05)
        out.append(cs)
    return out


def run_batch(M, stacks, probes=None, index_override=None):
    import torch
    items = []
    for i, cs in enumerate(stacks):
        g = cs.geom
        idx = cs.index if index_override is None or index_override[i] is None else index_override[i]
        items.append({"geom": g, "pool_delta": dev(cs.pool_delta), "pool_beta": dev(cs.pool_beta),
                      "slice_index": dev(idx.astype(np.int32)),
                      "probe": None if probes is None or probes[i] is None else dev(probes[i]),
                      "field": torch.empty((g.ny, g.nz), dtype=torch.complex64, device="cuda"),
                      "intensity": torch.empty((g.ny, g.nz), dtype=torch.float32, device="cuda")})
    M.forward_batch(items)
    torch.cuda.synchronize()
    return [(it["field"].cpu().numpy(), it["intensity"].cpu().numpy()) for it in items], items


def test_batch_equals_single_instance_calls_bitwise(M):
    import torch
    stacks = small_batch()
    probes = [None] * len(stacks)
    probes[3] = synth.random_field(64, 64, 7, 0.5)
    got, _ = run_batch(M, stacks, probes)
    for cs, p, (f, I) in zip(stacks, probes, got):
        d, b = cs.dense()
        ref, _ = M.forward(cs.geom, dev(d), dev(b), None if p is None else dev(p))
        rI = M.far_field(cs.geom, ref)
        torch.cuda.synchronize()
        assert np.array_equal(f, ref.cpu().numpy()), cs.geom
        assert np.array_equal(I, rI.cpu().numpy()), cs.geom


def test_batch_matches_the_oracle(M):
    stacks = small_batch()
    got, _ = run_batch(M, stacks)
    for cs, (f, I) in zip(stacks, got):
        d, b = cs.dense()
        rf = O.forward(cs.geom, d, b)
        rI = O.far_field(cs.geom, rf)
        print(cs.geom.ny, cs.geom.nz, cs.geom.n_slices, fmt(check_forward(f, rf, I, rI, what=str(cs.geom))))


def test_slice_index_is_clamped_to_the_pool(M):
    stacks = small_batch()[:3]
    bad = [cs.index.copy() for cs in stacks]
    bad[0][3] = -7
    bad[0][5] = stacks[0].pool_delta.shape[0] + 11
    clamped = [np.clip(x, 0, cs.pool_delta.shape[0] - 1) for x, cs in zip(bad, stacks)]
    a, _ = run_batch(M, stacks, index_override=bad)
    b, _ = run_batch(M, stacks, index_override=clamped)
    for (fa, Ia), (fb, Ib) in zip(a, b):
        assert np.array_equal(fa, fb) and np.array_equal(Ia, Ib)


def test_batch_replays_from_a_captured_graph(M):
    # the whole batched forward captured once and replayed; every replay equals the eager result
    import torch
    stacks = small_batch()
    eager, items = run_batch(M, stacks)
    ws = M.batch_workspace(items)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        M.forward_batch(items, ws)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            M.forward_batch(items, ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for it in items:
            it["field"].fill_(float("nan"))
            it["intensity"].fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        x = torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")  # eager work between replays
        torch.cuda.synchronize()
        for (f, I), it in zip(eager, items):
            assert np.array_equal(it["field"].cpu().numpy(), f)
            assert np.array_equal(it["intensity"].cpu().numpy(), I)
