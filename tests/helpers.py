"""Shared helpers of the test suite (comparison metrics and geometry transfer)."""
import numpy as np

from oracle.geometry import OracleGeometry

_FIELDS = ("src_x0", "src_y0", "src_dx", "src_dy", "src_nx", "src_ny", "ray_x0", "ray_y0",
           "ray_dx", "ray_dy", "ray_nx", "ray_ny", "scheme", "coarse", "l1_kx", "l1_ky")


def oracle_geom(g):
    """OracleGeometry with the same numbers as a library lm_geometry."""
    return OracleGeometry(**{k: getattr(g, k) for k in _FIELDS}, halo=g.near_halo,
                          terms=g.taylor_terms, far_order=g.far_order)


def mismatch_fraction(a, b, rays):
    """Bin-mismatch fraction: half the L1 distance of two count maps over the rays shot."""
    return 0.5 * np.abs(a.astype(np.int64) - b.astype(np.int64)).sum() / float(rays)


def max_pixel_rel(a, b, min_count=10000):
    """Largest |a-b|/b over pixels with b >= min_count (0 if there are none)."""
    b64 = b.astype(np.float64)
    sel = b64 >= min_count
    if not sel.any():
        return 0.0
    return float((np.abs(a.astype(np.float64) - b64)[sel] / b64[sel]).max())
