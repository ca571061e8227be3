"""Host-side logic of the trainer (no GPU): the time-to-accuracy criteria
over a logged Y0 history."""
import numpy as np

from paper_1910_11623_amd.train import History, first_accurate_iteration, first_accurate_mean_iteration


def _hist(y, N):
    y = np.asarray(y, dtype=np.float64)
    return History(N=np.asarray(N), y0=y, loss=np.zeros_like(y), t=np.arange(1, y.size + 1) * 0.5,
                   level_seconds=[], params=None, y0_final=float(y[-1]))


def test_first_accurate_iteration_needs_the_finest_level_and_the_hold():
    # coarse level already accurate, then the finest level enters the band at index 30
    y = [100.0] * 20 + [90.0] * 10 + [100.4] * 150
    N = [4] * 20 + [8] * 160
    h = _hist(y, N)
    assert first_accurate_iteration(h, 100.0, rel=0.01, hold=100) == 30
    assert first_accurate_iteration(h, 100.0, rel=0.001, hold=100) is None
    # a single excursion inside the hold window restarts the count
    y2 = list(y)
    y2[60] = 95.0
    assert first_accurate_iteration(_hist(y2, N), 100.0, rel=0.01, hold=50) == 61
    assert first_accurate_iteration(_hist(y2, N), 100.0, rel=0.01, hold=120) is None  # 119 left after it


def test_first_accurate_mean_iteration_smooths_noise():
    rng = np.random.default_rng(0)
    n = 3000
    y = 100.0 + 1.5 * rng.standard_normal(n)      # noise above the 1% band, mean on target
    h = _hist(y, [32] * n)
    assert first_accurate_iteration(h, 100.0) is None
    k = first_accurate_mean_iteration(h, 100.0, window=100, hold=500)
    assert k is not None and 99 <= k < 400
    # a biased mean never qualifies
    assert first_accurate_mean_iteration(_hist(y + 2.0, [32] * n), 100.0) is None
    # coarse-level iterations are skipped: the window starts on the finest level
    h2 = _hist(np.concatenate([np.full(500, 100.0), y]), [16] * 500 + [32] * n)
    k2 = first_accurate_mean_iteration(h2, 100.0, window=100, hold=500)
    assert k2 is not None and k2 >= 500 + 99
