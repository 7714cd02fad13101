"""Pins of the oracle's peak finder (Sec. 4.2) on hand-made light curves."""
import math

import numpy as np

from oracle.peaks import CANDIDATE, TRUE_PEAK, find_peaks, is_candidate


def _h_over_sigma(a, n, b):
    mean = (a + n + b) / 3.0
    return (n - mean) / math.sqrt(mean)


def test_candidate_threshold_matches_definition():
    """h > 5 sigma with h = N - <N>, sigma = sqrt(<N>), checked in floating point
    on values away from the threshold, and the exact integer form at it."""
    rows = [(100, 200, 100), (100, 190, 100), (100, 185, 100), (100, 184, 100),
            (0, 30, 0), (0, 26, 0), (0, 25, 0), (1000, 1200, 1100), (1000, 1000, 900)]
    for a, n, b in rows:
        r = _h_over_sigma(a, n, b) if a + n + b else 0.0
        got = is_candidate([[a, n, b]], 0, 1)
        if abs(r - 5.0) > 1e-9:
            assert got == ((n > max(a, b)) and r > 5.0), (a, n, b, r)
    # 185: h = 56.667, 5 sigma = 56.642 -> candidate; 184: h = 56.0, 5 sigma = 56.569 -> not
    assert is_candidate([[100, 185, 100]], 0, 1)
    assert not is_candidate([[100, 184, 100]], 0, 1)
    # a local maximum is required even when h is large
    assert not is_candidate([[500, 500, 0]], 0, 1)


def test_ends_are_never_candidates():
    assert not is_candidate([[1000, 0, 0]], 0, 0)
    assert not is_candidate([[0, 0, 1000]], 0, 2)


def test_cross_validation_needs_both_sides():
    base = np.full((5, 9), 100, dtype=np.int64)
    spike = 400
    base[2, 4] = spike  # candidate in the middle curve
    base[1, 5] = spike  # left neighbour at j+1
    flags = find_peaks(base.tolist(), [2])
    assert flags[0][4] == CANDIDATE  # no candidate on the right yet
    base[3, 3] = spike  # right neighbour at j-1
    flags = find_peaks(base.tolist(), [1, 2, 3])
    assert flags[1][4] == CANDIDATE | TRUE_PEAK
    # the neighbours themselves lack a candidate on their far side
    assert flags[0][5] == CANDIDATE and flags[2][3] == CANDIDATE
    base[3, 3] = 100
    base[3, 1] = spike  # two columns away: not within the three neighbours
    assert find_peaks(base.tolist(), [2])[0][4] == CANDIDATE


def test_edge_curves_keep_no_true_peaks():
    base = np.full((3, 5), 10, dtype=np.int64)
    base[:, 2] = 200
    flags = find_peaks(base.tolist(), [0, 1, 2])
    assert flags[0][2] == CANDIDATE and flags[2][2] == CANDIDATE
    assert flags[1][2] == CANDIDATE | TRUE_PEAK


def test_poisson_noise_rarely_passes():
    """On a flat map with Poisson noise of mean 400, a 5 sigma three-point peak
    is rare (the paper's motivation for the threshold)."""
    rng = np.random.default_rng(1)
    m = rng.poisson(400, size=(40, 2000))
    flags = find_peaks(m.tolist(), list(range(1, 39)))
    cand = sum(f & CANDIDATE != 0 for row in flags for f in row)
    true = sum(f & TRUE_PEAK != 0 for row in flags for f in row)
    assert cand < 20
    assert true == 0


# ------------------------------------------------ statistics by distance (Sec. 4.2)

from oracle.peak_stats import bin_of_column, peak_stats  # noqa: E402


def test_peak_stats_on_placed_peaks():
    """Spikes placed by hand in three neighbouring rows (so the middle one is a
    true peak) at known columns: the histogram holds exactly those peaks, their
    counts, and the light-curve length per bin."""
    n_cols = 40
    base = np.full((7, n_cols), 100, dtype=np.int64)
    # columns 5 and 23: true peaks on row 3; column 31: a candidate only
    for col, h in ((5, 400), (23, 900)):
        base[2, col + 1] = base[3, col] = base[4, col - 1] = h
    base[3, 31] = 500
    src_x0, src_dx = -1.0, 0.25  # column p centred at -1 + (p + 1/2) / 4
    edges = [-1.0, 0.5, 4.0, 9.0]  # columns 0-5, 6-19, 20-39
    peaks, heights, pixels = peak_stats(base.tolist(), [3], edges, src_x0, src_dx)
    assert peaks == [1, 0, 1]
    assert heights == [400, 0, 900]
    assert pixels == [6, 14, 20]
    # two light curves: the outer rows hold candidates but no true peaks
    peaks2, _, pixels2 = peak_stats(base.tolist(), [2, 3], edges, src_x0, src_dx)
    assert peaks2 == [1, 0, 1] and pixels2 == [12, 28, 40]


def test_bin_of_column_edges_are_half_open():
    edges = [0.0, 1.0, 2.0]
    # centres 0.5, 1.5, 2.5 with dx = 1 from x0 = 0
    assert [bin_of_column(p, 0.0, 1.0, edges) for p in range(3)] == [0, 1, -1]
    # a centre exactly on an edge belongs to the bin it opens
    assert bin_of_column(0, 0.5, 1.0, edges) == 1
    assert bin_of_column(0, -0.5, 1.0, edges) == 0
    assert bin_of_column(0, -0.6, 1.0, edges) == -1
