"""Peak identification on light curves (Sec. 4.2), written out plainly.

TEST INFRASTRUCTURE (part of the oracle): independent of the library's kernel.

A light curve is column i of the source map: the counts N[i][j] of the pixels
with source-plane index i along the caustic and j across it (in the library's
row-major map, counts[q][p], the paper's column i is row q and j is p).

Candidate peak at (i, j) (the first step of Sec. 4.2):
    N_ij > max(N_i(j-1), N_i(j+1))  and  h_ij > k sigma_ij,
    h_ij = N_ij - <N>,  <N> = (N_i(j-1) + N_ij + N_i(j+1)) / 3,  sigma_ij = sqrt(<N>),
with k = 5.  Written with S = N_i(j-1) + N_ij + N_i(j+1), the second condition
is 3 N_ij - S > k sqrt(3 S), i.e. (3 N_ij - S)^2 > 3 k^2 S with 3 N_ij - S > 0, which
is decided exactly in integers here.  Pixels at the ends of a light curve
(j = 0 or the last j) have no two neighbours and are not candidates.

True peak at (i, j) (the cross-validation step): (i, j) is a candidate, one of
(i-1, j-1), (i-1, j), (i-1, j+1) is a candidate and one of (i+1, j-1),
(i+1, j), (i+1, j+1) is a candidate.  Light curves at the first or last i have
no neighbour on one side and keep no true peaks.
"""
from __future__ import annotations

CANDIDATE = 1
TRUE_PEAK = 2


def is_candidate(counts, i, j, k=5):
    """counts: 2-D indexable [i][j] of non-negative integers."""
    n_j = len(counts[i])
    if j <= 0 or j >= n_j - 1:
        return False
    a, n, b = int(counts[i][j - 1]), int(counts[i][j]), int(counts[i][j + 1])
    if not (n > a and n > b):
        return False
    s = a + n + b
    t = 3 * n - s
    return t > 0 and t * t > 3 * k * k * s


def find_peaks(counts, tracks, k=5):
    """Flags per listed light curve: list of lists of (CANDIDATE | TRUE_PEAK) bits."""
    n_i = len(counts)
    out = []
    for i in tracks:
        row = []
        n_j = len(counts[i])
        for j in range(n_j):
            f = 0
            if is_candidate(counts, i, j, k):
                f |= CANDIDATE
                if 0 < i < n_i - 1:
                    left = any(is_candidate(counts, i - 1, j + d, k) for d in (-1, 0, 1))
                    right = any(is_candidate(counts, i + 1, j + d, k) for d in (-1, 0, 1))
                    if left and right:
                        f |= TRUE_PEAK
            row.append(f)
        out.append(row)
    return out
