"""Host checks of the seeded input generators (no method arithmetic here)."""
import numpy as np

from paper_2212_01253_amd import synth


def test_compact_stack_expands_to_the_dense_generator():
    g = synth.Geometry(64, 64, 300, 1.0, 1.0, 5.0, 0.1, 0.005, 0)
    kw = dict(substrate_rows=16, n_bars=(8, 32), bar_height=(2, 10), bar_width=(2, 16), bar_len_frac=(1 / 8, 1.0),
              n_lines=(2, 8), line_height=(2, 10), line_width=(1, 4), delta_range=(5e-6, 3e-5),
              beta_over_delta=0.05)
    for seed in (1, 5, 9):
        w = synth.bars_on_substrate(g, seed, **kw)
        c = synth.compact_bars_on_substrate(g, seed, **kw)
        d, b = c.dense()
        assert np.array_equal(d, w.delta) and np.array_equal(b, w.beta)
        assert c.pool_delta.shape[0] <= 2 * 32 + 1 + 8
        assert c.index.dtype == np.int32 and c.index.min() == 0 and c.index.max() == c.pool_delta.shape[0] - 1


def test_batch_instances_follow_the_recipe():
    insts = synth.batch_workload(12, grids=(16, 32), ns_range=(5, 40))
    for cs in insts:
        g = cs.geom
        assert g.ny == g.nz and g.ny in (16, 32) and 5 <= g.n_slices <= 40
        assert 0.08 <= g.wavelength_nm <= 0.15 and np.radians(0.05) <= g.alpha_i_rad <= np.radians(0.5)
        assert cs.index.shape == (g.n_slices,)
        d, b = cs.dense()
        assert np.all(d[:, : g.ny // 4] > 0) and np.allclose(b[d > 1e-5], d[d > 1e-5] / 20, rtol=1e-6)
    again = synth.batch_workload(12, grids=(16, 32), ns_range=(5, 40))
    assert all(np.array_equal(a.pool_delta, b.pool_delta) for a, b in zip(insts, again))
