"""GPU checks of the launch-shape settings and their autotuner.

The number of lines a workgroup handles changes only how lines are dealt to
the hardware, never the arithmetic of a line, so every allowed shape must give
bit-identical fields; the same holds for how many grid-size groups of a batch
run side by side.
"""
import numpy as np
import pytest

from paper_2212_01253_amd import synth

pytestmark = pytest.mark.gpu

LIMIT = {16: 64, 32: 32, 64: 16, 128: 8, 256: 4, 512: 2, 1024: 1}


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import msl
    msl.lib()
    before = msl.get_tuning()
    yield msl
    msl.set_tuning(before["lines_per_group"], before["batch_streams"])


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def stack(ny, nz, ns, seed):
    g = synth.Geometry(ny, nz, ns, 1.0, 1.0, 5.0, 0.1, np.radians(0.3), 0)
    d, b = synth.random_stack(ny, nz, ns, seed)
    return g, dev(d), dev(b)


def fwd(M, g, d, b):
    import torch
    f, _ = M.forward(g, d, b)
    torch.cuda.synchronize()
    return f.cpu().numpy()


@pytest.mark.parametrize("ny,nz,ns", [(512, 512, 9), (256, 256, 12), (128, 128, 20), (64, 128, 15), (32, 16, 7)])
def test_every_shape_gives_identical_fields(M, ny, nz, ns):
    g, d, b = stack(ny, nz, ns, 11)
    M.set_tuning({})
    ref = fwd(M, g, d, b)
    for n in sorted({ny, nz}):
        v = 1
        while v <= LIMIT[n]:
            M.set_tuning({n: v})
            got = fwd(M, g, d, b)
            print(ny, nz, n, v)
            assert np.array_equal(got, ref), (ny, nz, n, v)
            v *= 2
    M.set_tuning({})


def test_batch_streams_and_shapes_give_identical_fields(M):
    import torch
    specs = [(64, 64, 30), (128, 128, 17), (32, 32, 9), (128, 128, 5), (256, 256, 8)]
    items = []
    for i, (ny, nz, ns) in enumerate(specs):
        g = synth.Geometry(ny, nz, ns, 1.0, 1.0, 5.0, 0.1, np.radians(0.2), 0)
        cs = synth.compact_bars_on_substrate(g, 300 + i, substrate_rows=ny // 4, n_bars=(2, 5),
                                             bar_height=(1, ny // 8), bar_width=(1, nz // 4),
                                             bar_len_frac=(0.125, 1.0), n_lines=(1, 2),
                                             delta_range=(5e-6, 3e-5), beta_over_delta=0.05)
        items.append({"geom": g, "pool_delta": dev(cs.pool_delta), "pool_beta": dev(cs.pool_beta),
                      "slice_index": dev(cs.index.astype(np.int32)), "probe": None,
                      "field": torch.empty((ny, nz), dtype=torch.complex64, device="cuda"),
                      "intensity": torch.empty((ny, nz), dtype=torch.float32, device="cuda")})

    def run():
        M.forward_batch(items)
        torch.cuda.synchronize()
        return [(it["field"].cpu().numpy(), it["intensity"].cpu().numpy()) for it in items]

    M.set_tuning({})
    ref = run()
    for lpg, bs in [({}, 1), ({}, 2), ({128: 8, 256: 1}, 4), ({64: 2, 32: 32, 256: 4}, 3)]:
        M.set_tuning(lpg, bs)
        got = run()
        for (f, I), (rf, rI) in zip(got, ref):
            assert np.array_equal(f, rf) and np.array_equal(I, rI), (lpg, bs)
    M.set_tuning({})


def test_batch_autotune_picks_allowed_settings_and_keeps_results(M):
    import torch
    specs = [(64, 64, 30), (128, 128, 17), (32, 32, 9), (256, 256, 8)]
    items = []
    for i, (ny, nz, ns) in enumerate(specs):
        g = synth.Geometry(ny, nz, ns, 1.0, 1.0, 5.0, 0.1, np.radians(0.2), 0)
        cs = synth.compact_bars_on_substrate(g, 400 + i, substrate_rows=ny // 4, n_bars=(2, 5),
                                             bar_height=(1, ny // 8), bar_width=(1, nz // 4),
                                             bar_len_frac=(0.125, 1.0), n_lines=(1, 2),
                                             delta_range=(5e-6, 3e-5), beta_over_delta=0.05)
        items.append({"geom": g, "pool_delta": dev(cs.pool_delta), "pool_beta": dev(cs.pool_beta),
                      "slice_index": dev(cs.index.astype(np.int32)), "probe": None,
                      "field": torch.empty((ny, nz), dtype=torch.complex64, device="cuda"),
                      "intensity": torch.empty((ny, nz), dtype=torch.float32, device="cuda")})
    M.set_tuning({})
    M.forward_batch(items)
    torch.cuda.synchronize()
    ref = [(it["field"].cpu().numpy(), it["intensity"].cpu().numpy()) for it in items]
    t, ms = M.autotune_batch(items, reps=1)
    print(t, ms)
    assert ms > 0 and 0 <= t["batch_streams"] <= 4
    for n in (32, 64, 128, 256):
        v = t["lines_per_group"][n]
        assert v == 0 or (v & (v - 1) == 0 and 1 <= v <= LIMIT[n])
    assert M.get_tuning() == t
    M.forward_batch(items)
    torch.cuda.synchronize()
    for it, (rf, rI) in zip(items, ref):
        assert np.array_equal(it["field"].cpu().numpy(), rf) and np.array_equal(it["intensity"].cpu().numpy(), rI)
    M.set_tuning({})


def test_autotune_picks_an_allowed_shape_and_keeps_results(M):
    g, d, b = stack(256, 256, 64, 5)
    M.set_tuning({})
    ref = fwd(M, g, d, b)
    t, ms = M.autotune_forward(g, d, b, reps=2)
    print(t, ms)
    assert ms > 0
    v = t["lines_per_group"][256]
    assert v == 0 or (v & (v - 1) == 0 and 1 <= v <= LIMIT[256])
    assert M.get_tuning() == t
    assert np.array_equal(fwd(M, g, d, b), ref)
    M.set_tuning({})
