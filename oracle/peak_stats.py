"""Statistics of true peaks by distance to the caustic (Sec. 4.2, Figs. 4 and 5),
written out plainly.

TEST INFRASTRUCTURE (part of the oracle): independent of the library's kernel.

The paper counts the true peaks of its light curves and their heights as a
function of the source's distance to the caustic.  Here a light curve is a row
of the count map (see peaks.py), its pixels run across the caustic along
beta_x, and a pixel column p lies at the distance of its centre,
beta_x(p) = src_x0 + (p + 1/2) src_dx.  For distance bins [e_b, e_b+1):

  peaks[b]   number of true peaks on the listed rows whose centre lies in bin b
  heights[b] sum of the counts N_ij of those peaks
  pixels[b]  number of light-curve pixels whose centre lies in bin b

All three are integers; the paper's two statistics follow from them (the
number density per unit length of light curve, scaled by Eq. 14's N_cf and
s_f, and the mean peak magnification scaled by Eq. 15's prefactor).
"""
from __future__ import annotations

from .peaks import TRUE_PEAK, find_peaks


def bin_of_column(p, src_x0, src_dx, edges):
    """Distance bin of pixel column p (-1 outside every bin), by a plain scan."""
    centre = src_x0 + (float(p) + 0.5) * src_dx
    for b in range(len(edges) - 1):
        if edges[b] <= centre < edges[b + 1]:
            return b
    return -1


def peak_stats(counts, tracks, edges, src_x0, src_dx, k=5):
    """(peaks, heights, pixels) lists of len(edges) - 1 integers.

    counts: 2-D indexable [row][column] of non-negative integers (rows are the
    light curves); tracks: the rows to use."""
    nb = len(edges) - 1
    peaks, heights, pixels = [0] * nb, [0] * nb, [0] * nb
    n_cols = len(counts[0])
    bins = [bin_of_column(p, src_x0, src_dx, edges) for p in range(n_cols)]
    flags = find_peaks(counts, tracks, k)
    for t, i in enumerate(tracks):
        for p in range(n_cols):
            b = bins[p]
            if b < 0:
                continue
            pixels[b] += 1
            if flags[t][p] & TRUE_PEAK:
                peaks[b] += 1
                heights[b] += int(counts[i][p])
    return peaks, heights, pixels
