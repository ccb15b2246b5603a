"""Host-side logic of the reconstruction driver (no GPU): the stall rule that decides when a
refinement from the learned start hands over to the plain start."""
import math

from paper_2212_01253_amd.recon import StallWatch


def test_steady_descent_never_stalls():
    w = StallWatch(10, 0.01)
    assert not any(w.stalled(it, 1000.0 * 0.98 ** it) for it in range(500))


def test_a_plateau_stalls_after_the_window():
    w = StallWatch(10, 0.01)
    losses = [100.0, 90.0, 80.0] + [79.5] * 20
    hits = [it for it, L in enumerate(losses) if w.stalled(it, L)]
    assert hits[0] == 12          # last 1 % fall at step 2, ten steps without one after it


def test_small_falls_below_the_gain_do_not_count():
    w = StallWatch(6, 0.05)
    losses = [100.0 * 0.99 ** it for it in range(40)]   # 1 % per step: a 5 % fall every 6 steps
    assert not any(w.stalled(it, L) for it, L in enumerate(losses))
    w = StallWatch(3, 0.05)
    assert any(w.stalled(it, L) for it, L in enumerate(losses))


def test_nan_is_never_progress_and_window_zero_never_stalls():
    w = StallWatch(3, 0.01)
    assert [w.stalled(it, L) for it, L in enumerate([5.0, math.nan, math.nan, math.nan])] == [False, False, False, True]
    w = StallWatch(0, 0.01)
    assert not any(w.stalled(it, 1.0) for it in range(100))
