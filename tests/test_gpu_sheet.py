"""GPU parity with the compensating sheet on the lenses' rectangle (Sec. 2,
Eq. 6): the rectangle's holomorphic part in every level-2 cell's
coefficients against the oracle's (whose series comes from its closed form
by contour sampling), maps against the oracle at the 1e-5 bar, partial cells
and a rectangle that is the lattice itself, the probes rebuilding a shot map,
and the entry point's error paths."""
import math
import os

import numpy as np
import pytest

import oracle
import paper_2308_14278_amd.lensmap as lm
from helpers import max_pixel_rel, mismatch_fraction, oracle_geom
from paper_2308_14278_amd import inputs

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    lm.load()
    oracle.build()


def _geom(w, **over):
    g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                              w.gamma, w.kappa_star, protect=w.protect, n_rays=w.n_rays or 0.0,
                              ray_nx=w.ray_nx or 0, ray_ny=w.ray_ny or 0, scheme=w.scheme,
                              coarse=w.coarse, mean_mass=w.mean_mass)
    for k, v in over.items():
        setattr(g, k, v)
    return g


def _pair(w, sheet=True, **over):
    g = _geom(w, **over)
    x, y, m = w.lenses()
    rect = w.sheet() if sheet else None
    mp = lm.Map(g, w.kappa, w.gamma, w.kappa_star, (x, y, m), sheet=rect)
    orc = oracle.Oracle(oracle_geom(g), w.kappa, w.gamma, w.kappa_star, x, y, m, sheet=rect)
    return g, mp, orc


def _small_fold(precision=lm.LM_PREC_AUTO, n_rays=4e7, hierarchical=False):
    """A fold map whose lenses fill the shooting region exactly, so the sheet's
    rectangle is the ray lattice itself; 22951 x 1743 rays in cells of 64
    leave a partial last column and row of level-2 cells.  hierarchical: the
    far field from the series of the near-square boxes of its 36 x 3 level-1
    cells."""
    k0, dx, dy, ks = 0.83, 2.0e-3, -1.5e-3, 0.01
    g = lm.lm_geometry_derive_fold(4.0, 4.0, 400, 400, k0, dx, ks, n_rays=n_rays, coarse=64)
    g.precision = precision
    if hierarchical:
        assert lm.lm_geometry_far_order(g) > 0
    hx, hy = g.ray_nx * g.ray_dx / 2, g.ray_ny * g.ray_dy / 2
    n = int(round(4 * hx * hy * ks / math.pi))
    rng = np.random.default_rng(31)
    x, y = rng.uniform(-hx, hx, n), rng.uniform(-hy, hy, n)
    m = np.ones(n)
    rect = (-hx, hx, -hy, hy)
    mp = lm.Map(g, kappa_star=ks, lenses=(x, y, m), fold=(k0, dx, dy), sheet=rect)
    orc = oracle.Oracle(oracle_geom(g), 0, 0, ks, x, y, m, fold=(k0, dx, dy), sheet=rect)
    return g, mp, orc


def _check_map(g, counts, n_out, ref, ref_out, rays, what):
    mis = mismatch_fraction(counts, ref, rays)
    pix = max_pixel_rel(counts, ref)
    print("%s: rays %d, mismatch %.2e, worst pixel %.2e, n_out %d / %d" %
          (what, rays, mis, pix, n_out, ref_out), flush=True)
    assert int(counts.sum()) + n_out == rays
    assert mis <= 1e-5
    assert pix <= 1e-3


@pytest.mark.parametrize("kind", ["near-fold", "fold-lattice"])
def test_sheet_coefficients_vs_oracle(kind):
    """Coefficients with the sheet against the oracle's, at cells spread over
    the lattice, its edges, corners and (fold-lattice) partial last cells,
    weighed as they move a ray of the cell: with h the cell's half-diagonal,
    |da_0| within 1e-11 and sum_n |da_n| h^n (n >= 1, FP32 storage) within
    3e-7 of the larger of the far and sheet parts' sum_n |a_n| h^n."""
    if kind == "near-fold":
        w = inputs.near_fold()
        g, mp, orc = _pair(w)
        orc0 = oracle.Oracle(oracle_geom(g), w.kappa, w.gamma, w.kappa_star, *w.lenses())
    else:
        g, mp, orc = _small_fold()
        orc0 = oracle.Oracle(oracle_geom(g), 0, 0, orc.kappa_star, orc.lx, orc.ly, orc.lm,
                             fold=(0.83, 2.0e-3, -1.5e-3))
    ncx, ncy = -(-g.ray_nx // g.coarse), -(-g.ray_ny // g.coarse)
    rng = np.random.default_rng(5)
    cells = [(0, 0), (ncx - 1, ncy - 1), (ncx - 1, 0), (0, ncy - 1), (ncx // 2, ncy // 2),
             (ncx - 1, ncy // 2), (ncx // 3, ncy - 1)]
    cells += [(int(rng.integers(ncx)), int(rng.integers(ncy))) for _ in range(12)]
    h = 0.5 * math.hypot(g.coarse * g.ray_dx, g.coarse * g.ray_dy)
    hn = h ** np.arange(g.taylor_terms)
    worst0 = worst = 0.0
    for ci, cj in cells:
        got = lm.lm_read_coeffs(mp.h, ci, cj, g.taylor_terms)
        ref = orc.coeffs(ci, cj)
        far = orc0.coeffs(ci, cj)
        scale = np.maximum(np.abs(far), np.abs(ref - far))
        worst0 = max(worst0, float(abs(got[0] - ref[0]) / scale[0]))
        worst = max(worst, float((np.abs(got[1:] - ref[1:]) * hn[1:]).sum() /
                                 (scale[1:] * hn[1:]).sum()))
    print("%s: a_0 rel err %.2e, a_1.. rel err %.2e" % (kind, worst0, worst))
    assert worst0 <= 1e-11
    assert worst <= 3e-7
    mp.close()


def test_sheet_near_fold_subrect_vs_oracle():
    """Near-fold workload (2000 lenses, R = 64) with the sheet on the lenses'
    rectangle: a 2.6e8-ray sub-rectangle against the oracle; the sheet moves
    rays (the map differs from the infinite sheet's)."""
    w = inputs.near_fold()
    g, mp, orc = _pair(w)
    ni, nj = 131072, 2048
    i0, j0 = (g.ray_nx - ni) // 2 + 999, (g.ray_ny - nj) // 2 - 77
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, _ = mp.counts()
    ref, ref_out = orc.shoot(i0, j0, ni, nj, nthreads=NTHREADS)
    _check_map(g, counts, n_out, ref, ref_out, ni * nj, "near-fold with sheet")
    g2, mp2, _ = _pair(w, sheet=False)
    mp2.shoot(i0, j0, ni, nj)
    c2, _, _ = mp2.counts()
    assert mismatch_fraction(counts, c2, ni * nj) > 1e-3
    mp.close()
    mp2.close()


@pytest.mark.parametrize("precision,hierarchical", [(lm.LM_PREC_AUTO, False),
                                                    (lm.LM_PREC_MIXED_FP64, False),
                                                    (lm.LM_PREC_MIXED_CENTRED, True)])
def test_sheet_fold_lattice_map_vs_oracle(precision, hierarchical):
    """Small fold map whose sheet rectangle is the lattice (partial last cells,
    corner cells included) against the oracle's map of the same scheme; the
    last case adds the hierarchical far field and the centred near sums, as
    the fold study of the bench combines them."""
    g, mp, orc = _small_fold(precision, hierarchical=hierarchical)
    mp.shoot()
    counts, n_out, n_shot = mp.counts()
    ref, ref_out = orc.shoot(nthreads=NTHREADS)
    _check_map(g, counts, n_out, ref, ref_out, g.n_rays, "fold lattice-rect sheet %d" %
               mp.precision()[0])
    mp.close()


def test_sheet_trace_rebuilds_shot_map():
    """The probes read the same coefficients: traced pixels of a shot
    sub-rectangle rebuild its counts bit for bit."""
    g, mp, _ = _small_fold()
    i0, j0, ni, nj = g.ray_nx - 700, g.ray_ny - 200, 700, 200  # the partial corner
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, _ = mp.counts()
    ii, jj = np.meshgrid(np.arange(i0, i0 + ni), np.arange(j0, j0 + nj))
    p, q = mp.trace(ii.ravel(), jj.ravel())
    inside = p >= 0
    rebuilt = np.zeros(g.src_nx * g.src_ny, dtype=np.int64)
    np.add.at(rebuilt, q[inside].astype(np.int64) * g.src_nx + p[inside], 1)
    np.testing.assert_array_equal(rebuilt.reshape(counts.shape), counts.astype(np.int64))
    assert int((~inside).sum()) == n_out
    mp.close()


def test_sheet_paper_scale_subrect_vs_oracle():
    """Paper-scale workload with the sheet on the lenses' rectangle (1.35x the
    shooting region per side): a 1.7e9-ray band through the middle of the
    lattice against the oracle, in the library's default precision."""
    w = inputs.paper_scale()
    g, mp, orc = _pair(w)
    nj = 4 * g.coarse
    ni = 230_000
    i0, j0 = g.ray_nx // 2 - ni // 2 + 13, g.ray_ny // 2 - nj // 2
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, _ = mp.counts()
    ref, ref_out = orc.shoot(i0, j0, ni, nj, nthreads=NTHREADS)
    _check_map(g, counts, n_out, ref, ref_out, ni * nj,
               "paper-scale with sheet (precision %d)" % mp.precision()[0])
    mp.close()


def test_sheet_error_paths():
    w = inputs.near_fold()
    g = _geom(w)
    mp = lm.Map(g, w.kappa, w.gamma, w.kappa_star, w.lenses())
    x0, x1 = g.ray_x0, g.ray_x0 + g.ray_nx * g.ray_dx
    y0, y1 = g.ray_y0, g.ray_y0 + g.ray_ny * g.ray_dy
    with pytest.raises(lm.LensmapError):  # does not hold the lattice
        lm.lm_set_sheet(mp.h, x0 + 1.0, x1, y0, y1)
    with pytest.raises(lm.LensmapError):  # empty
        lm.lm_set_sheet(mp.h, x1, x0, y0, y1)
    with pytest.raises(lm.LensmapError):
        lm.lm_set_sheet(mp.h, float("nan"), x1, y0, y1)
    lm.lm_set_sheet(mp.h, x0, x1, y0, y1)  # the lattice itself
    lm.lm_set_sheet(mp.h, 0.0, 0.0, 0.0, 0.0)  # back to the infinite sheet
    mp.shoot(0, 0, 64, 64)
    with pytest.raises(lm.LensmapError):  # counts present
        lm.lm_set_sheet(mp.h, x0, x1, y0, y1)
    mp.close()
    wd = inputs.plain_small()
    gd = _geom(wd)
    md = lm.Map(gd, wd.kappa, wd.gamma, wd.kappa_star, wd.lenses())
    with pytest.raises(lm.LensmapError):  # direct scheme
        lm.lm_set_sheet(md.h, -100.0, 100.0, -100.0, 100.0)
    md.close()


def test_sheet_batch_equals_per_map_and_follows_the_sheet():
    """The batch's coefficient graph carries the sheet: a batch of a map with
    the sheet on its lens rectangle and the same map with the infinite sheet
    reproduces each one's per-map counts bit for bit; moving a map's sheet
    after the graphs are built makes the batch rebuild them and follow."""
    w = inputs.near_fold()
    g = _geom(w)
    lenses = w.lenses()
    ni, nj = 65536, 1024
    i0, j0 = (g.ray_nx - ni) // 2, (g.ray_ny - nj) // 2
    maps = [lm.Map(g, w.kappa, w.gamma, w.kappa_star, lenses, sheet=w.sheet()),
            lm.Map(g, w.kappa, w.gamma, w.kappa_star, lenses)]
    ref = []
    for mp in maps:
        mp.shoot(i0, j0, ni, nj)
        ref.append(mp.counts())
        mp.reset()
    assert mismatch_fraction(ref[0][0], ref[1][0], ni * nj) > 1e-3
    b = lm.lm_batch_create([mp.h for mp in maps])
    for k in range(2):
        lm.lm_batch_set_rect(b, k, i0, j0, ni, nj)
    lm.lm_batch_shoot(b)
    for mp, (c, o, s) in zip(maps, ref):
        c2, o2, s2 = mp.counts()
        np.testing.assert_array_equal(c, c2)
        assert (o, s) == (o2, s2)
        mp.reset()
    # swap the sheets: the rebuilt graphs give each map the other's counts
    lm.lm_set_sheet(maps[0].h, 0.0, 0.0, 0.0, 0.0)
    lm.lm_set_sheet(maps[1].h, *w.sheet())
    lm.lm_batch_shoot(b)
    np.testing.assert_array_equal(maps[0].counts()[0], ref[1][0])
    np.testing.assert_array_equal(maps[1].counts()[0], ref[0][0])
    lm.lm_batch_destroy(b)
    for mp in maps:
        mp.close()
