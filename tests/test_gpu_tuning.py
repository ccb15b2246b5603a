"""GPU checks of the launch-shape settings and their autotuner.

The number of lines a workgroup handles changes only how lines are dealt to
the hardware, never the arithmetic of a line, so at one points-per-lane
setting every allowed number of lines per workgroup must give bit-identical
fields; the same holds for how many grid-size groups of a batch run side by
side.  The points per lane (radix-4 or radix-8 FFT stages) change the order
of the float32 operations: each setting is held to the FP64 oracle by the
parity gates.
"""
import numpy as np
import pytest

from oracle import msl_oracle as O
from paper_2212_01253_amd import synth
from parity_gates import check_field, check_forward

pytestmark = pytest.mark.gpu


def limit(n, p):
    """Largest lines per workgroup: 256 threads of n / p lanes per line."""
    return 256 // (n // p)


def radices(n):
    return (4, 8) if n >= 64 else (4,)


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_01253_amd import msl
    msl.lib()
    before = msl.get_tuning()
    yield msl
    msl.restore_tuning(before)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def stack(ny, nz, ns, seed):
    g = synth.Geometry(ny, nz, ns, 1.0, 1.0, 5.0, 0.1, np.radians(0.3), 0)
    d, b = synth.random_stack(ny, nz, ns, seed, 3e-5, 2e-6)
    return g, d, b


def fwd(M, g, d, b):
    import torch
    f, _ = M.forward(g, d, b)
    torch.cuda.synchronize()
    return f.cpu().numpy()


@pytest.mark.parametrize("ny,nz,ns", [(512, 512, 9), (256, 256, 12), (128, 128, 20), (64, 128, 15), (32, 16, 7),
                                      (1024, 64, 5)])
def test_every_shape_gives_identical_fields(M, ny, nz, ns):
    g, dn, bn = stack(ny, nz, ns, 11)
    d, b = dev(dn), dev(bn)
    rf = O.forward(g, dn, bn)
    lens = sorted({ny, nz})
    for p in (4, 8):
        ppl = {n: p for n in lens if p in radices(n)}
        M.set_tuning({}, points_per_lane=ppl)
        ref = fwd(M, g, d, b)
        e, r = check_field(ref, rf, what=f"points per lane {ppl}")
        print(ny, nz, ppl, f"field {e:.2e} gates {r:.2f}")
        for n in lens:
            pn = ppl.get(n, 4 if n < 512 else 8)
            v = 1
            while v <= limit(n, pn):
                M.set_tuning({n: v}, points_per_lane=ppl)
                got = fwd(M, g, d, b)
                assert np.array_equal(got, ref), (ny, nz, n, v, ppl)
                v *= 2
    M.set_tuning({})


@pytest.mark.parametrize("ny,nz,ns", [(512, 512, 10), (1024, 512, 7)])
def test_forward_sweep_mapping_equals_the_checkpointing_one(M, ny, nz, ns):
    # forward row passes over 512-point lines that store no field take one line per wavefront,
    # those that store one (a checkpoint at every slice here) two lines interleaved over a
    # workgroup: same arithmetic per line, so the exit fields are bit-identical, and within the
    # parity gates
    g, dn, bn = stack(ny, nz, ns, 31)
    d, b = dev(dn), dev(bn)
    M.set_tuning({})
    f0, _ = M.forward(g, d, b, ckpt_every=0)
    f1, ck = M.forward(g, d, b, ckpt_every=1)
    import torch
    torch.cuda.synchronize()
    assert np.array_equal(f0.cpu().numpy(), f1.cpu().numpy())
    check_field(f0.cpu().numpy(), O.forward(g, dn, bn), what=f"{ny}x{nz}")


def batch_items(M, specs, seed0):
    import torch
    items = []
    for i, (ny, nz, ns) in enumerate(specs):
        g = synth.Geometry(ny, nz, ns, 1.0, 1.0, 5.0, 0.1, np.radians(0.2), 0)
        cs = synth.compact_bars_on_substrate(g, seed0 + i, substrate_rows=ny // 4, n_bars=(2, 5),
                                             bar_height=(1, ny // 8), bar_width=(1, nz // 4),
                                             bar_len_frac=(0.125, 1.0), n_lines=(1, 2),
                                             delta_range=(5e-6, 3e-5), beta_over_delta=0.05)
        items.append({"geom": g, "cs": cs, "pool_delta": dev(cs.pool_delta), "pool_beta": dev(cs.pool_beta),
                      "slice_index": dev(cs.index.astype(np.int32)), "probe": None,
                      "field": torch.empty((ny, nz), dtype=torch.complex64, device="cuda"),
                      "intensity": torch.empty((ny, nz), dtype=torch.float32, device="cuda")})
    return items


def run_batch(M, items):
    import torch
    M.forward_batch(items)
    torch.cuda.synchronize()
    return [(it["field"].cpu().numpy(), it["intensity"].cpu().numpy()) for it in items]


def oracle_batch(items):
    out = []
    for it in items:
        d, b = it["cs"].dense()
        g = it["geom"]
        rf = O.forward(g, d, b)
        out.append((rf, O.far_field(g, rf)))
    return out


def test_batch_streams_and_shapes_give_identical_fields(M):
    items = batch_items(M, [(64, 64, 30), (128, 128, 17), (32, 32, 9), (128, 128, 5), (256, 256, 8)], 300)
    M.set_tuning({})
    ref = run_batch(M, items)
    for lpg, bs in [({}, 1), ({}, 2), ({128: 8, 256: 1}, 4), ({64: 2, 32: 32, 256: 4}, 3)]:
        M.set_tuning(lpg, bs)
        got = run_batch(M, items)
        for (f, I), (rf, rI) in zip(got, ref):
            assert np.array_equal(f, rf) and np.array_equal(I, rI), (lpg, bs)
    # the other radix on every length that has one: within the parity gates, and again
    # bit-identical over the group shapes
    ppl = {64: 8, 128: 8, 256: 8}
    M.set_tuning({}, 0, ppl)
    ref8 = run_batch(M, items)
    for (f, I), (rf, rI) in zip(ref8, oracle_batch(items)):
        check_forward(f, rf, I, rI, what="points per lane 8")
    M.set_tuning({64: 16, 128: 2, 256: 4}, 2, ppl)
    for (f, I), (rf, rI) in zip(run_batch(M, items), ref8):
        assert np.array_equal(f, rf) and np.array_equal(I, rI)
    M.set_tuning({})


def test_batch_autotune_picks_allowed_settings_and_keeps_results(M):
    items = batch_items(M, [(64, 64, 30), (128, 128, 17), (32, 32, 9), (256, 256, 8)], 400)
    M.set_tuning({})
    t, ms = M.autotune_batch(items, reps=1)
    print(t, ms)
    assert ms > 0 and 0 <= t["batch_streams"] <= 4
    for n in (32, 64, 128, 256):
        p = t["points_per_lane"][n]
        assert p == 0 or p in radices(n)
        v = t["lines_per_group"][n]
        assert v == 0 or (v & (v - 1) == 0 and 1 <= v <= limit(n, p or 4))
    assert M.get_tuning() == t
    for (f, I), (rf, rI) in zip(run_batch(M, items), oracle_batch(items)):
        check_forward(f, rf, I, rI, what=f"autotuned {t}")
    M.set_tuning({})


def test_autotune_picks_an_allowed_shape_and_keeps_results(M):
    g, dn, bn = stack(256, 256, 64, 5)
    d, b = dev(dn), dev(bn)
    M.set_tuning({})
    ref = fwd(M, g, d, b)
    t, ms = M.autotune_forward(g, d, b, reps=2)
    print(t, ms)
    assert ms > 0
    p = t["points_per_lane"][256]
    assert p in (0, 4, 8)
    v = t["lines_per_group"][256]
    assert v == 0 or (v & (v - 1) == 0 and 1 <= v <= limit(256, p or 4))
    assert M.get_tuning() == t
    got = fwd(M, g, d, b)
    if p in (0, 4):
        assert np.array_equal(got, ref)
    check_field(got, O.forward(g, dn, bn), what=f"autotuned {t}")
    M.set_tuning({})
