"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (from the stated tolerances): bin-mismatch fraction <= 1e-5 of the rays
shot, per-pixel |dN|/N <= 1e-3 where the oracle count is >= 1e4, every ray
counted exactly, interpolated deflection within 1e-4 theta_E of the direct
sum.  Several maps are correct where a ray's exact image lies within rounding
of a pixel edge, so map parity is statistical (mismatch fraction), while
integer properties (ray conservation, additivity, batch == per-map, tuned ==
default, probe == kernel) are compared bit for bit.
"""
import os

import numpy as np
import pytest

import oracle
import paper_2308_14278_amd.lensmap as lm
from paper_2308_14278_amd import inputs
from helpers import max_pixel_rel, mismatch_fraction, oracle_geom

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


def _say(msg):
    print(msg, flush=True)


def _geom(w, **over):
    g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                              w.gamma, w.kappa_star, protect=w.protect, n_rays=w.n_rays or 0.0,
                              ray_nx=w.ray_nx or 0, ray_ny=w.ray_ny or 0, scheme=w.scheme,
                              coarse=w.coarse, mean_mass=w.mean_mass)
    for k, v in over.items():
        setattr(g, k, v)
    return g


def _pair(w, **over):
    """Library map and oracle on the same workload and lenses."""
    g = _geom(w, **over)
    x, y, m = w.lenses()
    mp = lm.Map(g, w.kappa, w.gamma, w.kappa_star, (x, y, m))
    orc = oracle.Oracle(oracle_geom(g), w.kappa, w.gamma, w.kappa_star, x, y, m)
    return g, mp, orc


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    lm.load()
    oracle.build()


def _compare(g, counts, n_out, ref, ref_out, rays, what):
    mis = mismatch_fraction(counts, ref, rays)
    pix = max_pixel_rel(counts, ref)
    _say("%s: rays=%d mismatch=%.3e max_pixel_rel=%.2e n_out gpu/oracle=%d/%d" %
         (what, rays, mis, pix, n_out, ref_out))
    assert int(counts.sum()) + n_out == rays
    assert int(ref.sum()) + ref_out == rays
    assert mis <= 1e-5
    assert pix <= 1e-3
    return mis


# ------------------------------------------------------------- direct sum


def test_plain_small_full_map():
    """Plain method, small: 100 unit lenses, 4096^2 rays, 256^2 map, direct sum."""
    w = inputs.plain_small()
    g, mp, orc = _pair(w)
    mp.shoot()
    counts, n_out, n_shot = mp.counts()
    assert n_shot == g.n_rays
    ref, ref_out = orc.shoot(nthreads=NTHREADS)
    _compare(g, counts, n_out, ref, ref_out, g.n_rays, "plain-small direct")
    mp.close()


def test_zero_lenses_exact_macro():
    """No lenses, no sheet, pixels of exactly 16 x 16 ray images: 256 per pixel."""
    g = lm.lm_geometry_derive(10.0, 10.0, 64, 64, 0.45, 0.5, 0.0, protect=0.0, ray_nx=1024,
                              ray_ny=1024, scheme=lm.LM_SCHEME_DIRECT, coarse=64)
    mp = lm.Map(g, 0.45, 0.5, 0.0, ([], [], []))
    mp.shoot()
    counts, n_out, _ = mp.counts()
    assert np.all(counts == 256) and n_out == 0
    mu = counts * mp.mu_factor()
    np.testing.assert_allclose(mu, 1.0 / abs(0.55 ** 2 - 0.25), rtol=1e-12)
    mp.close()


def test_single_lens_vs_oracle():
    """One unit lens at the origin (kappa = gamma = kappa_star = 0)."""
    g = lm.lm_geometry_derive(4.0, 4.0, 32, 32, 0.0, 0.0, 0.0, protect=2.0, ray_nx=2048,
                              ray_ny=2048, scheme=lm.LM_SCHEME_DIRECT, coarse=64)
    mp = lm.Map(g, 0.0, 0.0, 0.0, ([0.0], [0.0], [1.0]))
    mp.shoot()
    counts, n_out, _ = mp.counts()
    ref, ref_out = oracle.Oracle(oracle_geom(g), 0, 0, 0, [0.0], [0.0], [1.0]).shoot(
        nthreads=NTHREADS)
    _compare(g, counts, n_out, ref, ref_out, g.n_rays, "single lens")
    mp.close()


# ------------------------------------------------------ interpolated scheme


def test_near_fold_subrect_vs_oracle():
    """Near-fold map (2000 lenses, 64x64-ray cells): a ragged sub-rectangle of
    ~1.7e7 rays spanning many workgroup tiles, against the oracle."""
    w = inputs.near_fold()
    g, mp, orc = _pair(w)
    i0, j0, ni, nj = 900_037, 20_011, 5_777, 3_001
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, n_shot = mp.counts()
    ref, ref_out = orc.shoot(i0, j0, ni, nj, nthreads=NTHREADS)
    _compare(g, counts, n_out, ref, ref_out, ni * nj, "near-fold sub-rect")
    mp.close()


@pytest.mark.parametrize("precision", [lm.LM_PREC_MIXED, lm.LM_PREC_MIXED_FP64,
                                       lm.LM_PREC_MIXED_CENTRED])
def test_trace_probe_rebuilds_shot_map(precision):
    """lm_trace (one ray per thread) reproduces the shooting kernel bit for bit."""
    w = inputs.near_fold()
    g = _geom(w, precision=precision)
    x, y, m = w.lenses()
    mp = lm.Map(g, w.kappa, w.gamma, w.kappa_star, (x, y, m))
    i0, j0, ni, nj = 1_000_003, 30_000, 700, 333
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, _ = mp.counts()
    ii, jj = np.meshgrid(np.arange(i0, i0 + ni), np.arange(j0, j0 + nj))
    p, q = mp.trace(ii.ravel(), jj.ravel())
    inside = p >= 0
    rebuilt = np.zeros(g.src_nx * g.src_ny, dtype=np.int64)
    np.add.at(rebuilt, q[inside].astype(np.int64) * g.src_nx + p[inside], 1)
    np.testing.assert_array_equal(rebuilt.reshape(counts.shape), counts.astype(np.int64))
    assert (~inside).sum() == n_out
    mp.close()


@pytest.mark.parametrize("precision", [lm.LM_PREC_MIXED, lm.LM_PREC_MIXED_CENTRED])
def test_non_square_pixels(precision):
    """Pixels of different width and height (the near-fold source square in
    2000 x 1300 pixels): the FP32 sums in pixel units of each axis, and for the
    centred sums the y change carried from x pixels to y pixels.  The trace
    probe rebuilds the shot map bit for bit, and the map meets the bar against
    the oracle."""
    w = inputs.near_fold()
    g = lm.lm_geometry_derive(w.src_side, w.src_side, 2000, 1300, w.kappa, w.gamma,
                              w.kappa_star, protect=w.protect, n_rays=w.n_rays or 0.0,
                              ray_nx=w.ray_nx or 0, ray_ny=w.ray_ny or 0, scheme=w.scheme,
                              coarse=w.coarse, mean_mass=w.mean_mass)
    g.precision = precision
    assert abs(g.src_dx / g.src_dy - 1.3 / 2.0) < 1e-12
    x, y, m = w.lenses()
    mp = lm.Map(g, w.kappa, w.gamma, w.kappa_star, (x, y, m))
    orc = oracle.Oracle(oracle_geom(g), w.kappa, w.gamma, w.kappa_star, x, y, m)
    i0, j0, ni, nj = 1_000_000, 30_000, 20_000, 1_500
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, _ = mp.counts()
    ref, ref_out = orc.shoot(i0, j0, ni, nj, nthreads=NTHREADS)
    _compare(g, counts, n_out, ref, ref_out, ni * nj, "non-square pixels, precision %d" % precision)
    mp.reset()
    bi, bj = 900, 256
    mp.shoot(i0, j0, bi, bj)
    c2, o2, _ = mp.counts()
    ii, jj = np.meshgrid(np.arange(i0, i0 + bi), np.arange(j0, j0 + bj))
    p, q = mp.trace(ii.ravel(), jj.ravel())
    inside = p >= 0
    rebuilt = np.zeros(g.src_nx * g.src_ny, dtype=np.int64)
    np.add.at(rebuilt, q[inside].astype(np.int64) * g.src_nx + p[inside], 1)
    np.testing.assert_array_equal(rebuilt.reshape(c2.shape), c2.astype(np.int64))
    assert (~inside).sum() == o2
    mp.close()


def test_centred_sums_with_lenses_at_cell_centres():
    """Centred near sums where near lenses sit at (and next to) level-2 cell
    centres: those cells sum plainly (their centre's near deflection is not
    small), every other cell centred; the shot map against the oracle, and the
    trace probe rebuilds it bit for bit."""
    w = inputs.near_fold()
    g = _geom(w, precision=lm.LM_PREC_MIXED_CENTRED)
    x, y, m = w.lenses()
    i0, j0, ni, nj = 1_000_000, 30_000, 1_920, 640
    # move the first lenses onto cell centres (and within a tenth of a cell)
    # of the shot rectangle
    R = g.coarse
    x, y = x.copy(), y.copy()
    for t, (ci, cj, f) in enumerate(((i0 // R + 3, j0 // R + 2, 0.0), (i0 // R + 10, j0 // R + 5, 0.1),
                                     (i0 // R + 20, j0 // R + 1, 0.6))):
        x[t] = g.ray_x0 + (ci + 0.5 + f) * R * g.ray_dx
        y[t] = g.ray_y0 + (cj + 0.5) * R * g.ray_dy
    mp = lm.Map(g, w.kappa, w.gamma, w.kappa_star, (x, y, m))
    orc = oracle.Oracle(oracle_geom(g), w.kappa, w.gamma, w.kappa_star, x, y, m)
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, _ = mp.counts()
    ref, ref_out = orc.shoot(i0, j0, ni, nj, nthreads=NTHREADS)
    _compare(g, counts, n_out, ref, ref_out, ni * nj, "centred sums, lenses at cell centres")
    ii, jj = np.meshgrid(np.arange(i0, i0 + ni), np.arange(j0, j0 + nj))
    p, q = mp.trace(ii.ravel(), jj.ravel())
    inside = p >= 0
    rebuilt = np.zeros(g.src_nx * g.src_ny, dtype=np.int64)
    np.add.at(rebuilt, q[inside].astype(np.int64) * g.src_nx + p[inside], 1)
    np.testing.assert_array_equal(rebuilt.reshape(counts.shape), counts.astype(np.int64))
    mp.close()


@pytest.mark.parametrize("precision", [lm.LM_PREC_MIXED, lm.LM_PREC_MIXED_CENTRED])
def test_lenses_on_lattice_rays(precision):
    """Near lenses placed on lattice rays (two of the three FP32 offsets from
    the cell centre equal the rays' exactly): the floor on r^2 keeps every
    sum finite (a ray exactly on a lens gets no pull from it, where the
    oracle's FP64 offset is tiny but not zero: at most one ray per such lens
    differs).  A 2e7-ray region around them against the oracle (the strong
    fields next to the three lenses raise the flip rate of the FP32 sums over
    a few hundred rays around each), conservation, and the bitwise trace
    rebuild of the block that holds them."""
    w = inputs.near_fold()
    g = _geom(w, precision=precision)
    x, y, m = w.lenses()
    i0, j0, ni, nj = 1_000_000, 30_000, 1_920, 640
    x, y = x.copy(), y.copy()
    for t, (i, j) in enumerate(((i0 + 77, j0 + 13), (i0 + 1000, j0 + 300), (i0 + 1601, j0 + 600))):
        x[t] = g.ray_x0 + (i + 0.5) * g.ray_dx
        y[t] = g.ray_y0 + (j + 0.5) * g.ray_dy
    mp = lm.Map(g, w.kappa, w.gamma, w.kappa_star, (x, y, m))
    orc = oracle.Oracle(oracle_geom(g), w.kappa, w.gamma, w.kappa_star, x, y, m)
    bi, bj, bni, bnj = i0 - 2 * ni, j0 - 2 * nj, 5 * ni, 5 * nj
    mp.shoot(bi, bj, bni, bnj)
    counts, n_out, n_shot = mp.counts()
    assert int(counts.sum()) + n_out == n_shot == bni * bnj
    ref, ref_out = orc.shoot(bi, bj, bni, bnj, nthreads=NTHREADS)
    _compare(g, counts, n_out, ref, ref_out, bni * bnj,
             "lenses on lattice rays, precision %d" % precision)
    mp.reset()
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, _ = mp.counts()
    ii, jj = np.meshgrid(np.arange(i0, i0 + ni), np.arange(j0, j0 + nj))
    p, q = mp.trace(ii.ravel(), jj.ravel())
    inside = p >= 0
    rebuilt = np.zeros(g.src_nx * g.src_ny, dtype=np.int64)
    np.add.at(rebuilt, q[inside].astype(np.int64) * g.src_nx + p[inside], 1)
    np.testing.assert_array_equal(rebuilt.reshape(counts.shape), counts.astype(np.int64))
    assert (~inside).sum() == n_out
    mp.close()


def test_additivity_and_empty_shots():
    w = inputs.near_fold()
    g, mp, _ = _pair(w)
    i0, j0 = 500_000, 10_000
    mp.shoot(i0, j0, 1000, 0)  # empty
    mp.shoot(i0, j0, 0, 1000)  # empty
    mp.shoot(i0, j0, 2000, 700)
    a, na, _ = mp.counts()
    mp.reset()
    mp.shoot(i0, j0, 2000, 300)
    mp.shoot(i0, j0 + 300, 1, 400)
    mp.shoot(i0 + 1, j0 + 300, 1999, 400)
    b, nb, nshot = mp.counts()
    np.testing.assert_array_equal(a, b)
    assert na == nb and nshot == 2000 * 700
    mp.close()


@pytest.mark.parametrize("kind", ["paper-scale", "precision-stress"])
def test_full_size_sampled_rays_vs_oracle(kind):
    """Full-size lattices (1e13 and 4e12 rays): pixels of 3000 sampled rays from
    the probe that shares the kernel's arithmetic, against the oracle, one by one."""
    w = inputs.WORKLOADS[kind]()
    g, mp, orc = _pair(w)
    rng = np.random.default_rng(17)
    n = 3000
    ii = rng.integers(0, g.ray_nx, n)
    jj = rng.integers(0, g.ray_ny, n)
    p, q = mp.trace(ii, jj)
    _, pix = orc.trace(ii, jj)
    gpu_pix = np.where(p >= 0, q.astype(np.int64) * g.src_nx + p, -1)
    flips = int((gpu_pix != pix).sum())
    _say("%s: %d sampled rays, %d in map, %d flips" % (kind, n, int((pix >= 0).sum()), flips))
    assert flips <= 1
    mp.close()


def test_paper_scale_band_conservation_and_probe():
    """A 1e10-ray band of the paper-scale map through the timed launch path:
    every ray counted, and the counts of a small sub-block equal the traced
    pixels of its rays."""
    w = inputs.paper_scale()
    g, mp, _ = _pair(w)
    ni, nj = 2_000_000, 5_000
    i0, j0 = g.ray_nx // 2 - ni // 2, g.ray_ny // 2
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, n_shot = mp.counts()
    assert n_shot == ni * nj and int(counts.sum()) + n_out == ni * nj
    mp.reset()
    bi, bj = 3000, 200
    mp.shoot(i0, j0, bi, bj)
    c2, o2, _ = mp.counts()
    ii, jj = np.meshgrid(np.arange(i0, i0 + bi), np.arange(j0, j0 + bj))
    p, q = mp.trace(ii.ravel(), jj.ravel())
    rebuilt = np.zeros(g.src_nx * g.src_ny, dtype=np.int64)
    inside = p >= 0
    np.add.at(rebuilt, q[inside].astype(np.int64) * g.src_nx + p[inside], 1)
    np.testing.assert_array_equal(rebuilt.reshape(c2.shape), c2.astype(np.int64))
    mp.close()


@pytest.mark.parametrize("precision", [lm.LM_PREC_MIXED, lm.LM_PREC_MIXED_FP64,
                                       lm.LM_PREC_MIXED_CENTRED])
def test_paper_scale_subrect_map_vs_oracle(precision):
    """Paper-scale geometry (13000 lenses, ~1856-ray cells): a 2.2e7-ray map
    region against the oracle."""
    w = inputs.paper_scale()
    g, mp, orc = _pair(w, precision=precision)
    ni, nj = 40_000, 550
    i0, j0 = int(0.4 * g.ray_nx) + 17, g.ray_ny // 2 - 300
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, _ = mp.counts()
    ref, ref_out = orc.shoot(i0, j0, ni, nj, nthreads=NTHREADS)
    _compare(g, counts, n_out, ref, ref_out, ni * nj, "paper-scale sub-rect")
    assert ref_out < ni * nj // 10  # the block lands inside the map
    mp.close()


def test_deflection_interp_error_vs_direct():
    """Interpolated deflection from the GPU within 1e-4 theta_E of the direct
    sum (and within FP32 rounding of the oracle's interpolated value)."""
    w = inputs.paper_scale()
    g, mp, orc = _pair(w)
    rng = np.random.default_rng(5)
    n = 4000
    cx = g.ray_x0 + rng.uniform(0.3, 0.7, n) * g.ray_nx * g.ray_dx
    cy = g.ray_y0 + rng.uniform(0.05, 0.95, n) * g.ray_ny * g.ray_dy
    th = np.stack([cx, cy], axis=1)
    a_gpu = mp.deflect(th)
    a_dir = orc.deflect_direct(th)
    a_int = orc.deflect(th)
    err_dir = np.hypot(*(a_gpu - a_dir).T)
    err_int = np.hypot(*(a_gpu - a_int).T)
    scale = np.hypot(*a_int.T)
    _say("deflection: max |gpu-direct|=%.2e, max |gpu-oracle interp|=%.2e (|alpha| up to %.1f)" %
         (err_dir.max(), err_int.max(), scale.max()))
    assert err_dir.max() <= 1e-4
    assert np.all(err_int <= 1e-6 * np.maximum(1.0, scale))
    mp.close()


def test_precision_stress_region_vs_oracle():
    """Precision stress (lambda_t = 0.001, macro mu ~ 3300, 20000 lenses, 4e12-ray
    lattice, 4000^2 map): the 1e9-ray region at the centre of the lattice, whole
    map against the oracle, through the library's default precision choice."""
    w = inputs.precision_stress()
    g, mp, orc = _pair(w)
    nj = 8 * g.coarse
    ni = int(1e9 // nj)
    i0, j0 = g.ray_nx // 2 - ni // 2, g.ray_ny // 2 - nj // 2
    used, est, est_c = mp.precision()
    _say("precision stress: runs in precision %d (mismatch estimates %.2e plain, %.2e centred)" %
         (used, est, est_c))
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, _ = mp.counts()
    ref, ref_out = orc.shoot(i0, j0, ni, nj, nthreads=NTHREADS)
    _compare(g, counts, n_out, ref, ref_out, ni * nj, "precision-stress 1e9-ray region")
    mp.close()


def test_default_precision_choice_on_the_workloads():
    """The default (LM_PREC_AUTO) keeps FP32 near sums on the paper-scale and
    near-fold workloads (the estimated FP32 mismatch is well below the bar
    there), so the headline path is the FP32 one."""
    for kind in ("paper-scale", "near-fold"):
        w = inputs.WORKLOADS[kind]()
        g, mp, _ = _pair(w)
        assert g.precision == lm.LM_PREC_AUTO
        used, est, est_c = mp.precision()
        _say("%s: precision %d, mismatch estimates %.2e plain, %.2e centred" %
             (kind, used, est, est_c))
        assert used == lm.LM_PREC_MIXED and 0.0 <= est <= 5e-6
        mp.close()


def test_interp_error_of_kernel_arithmetic_1e6_rays():
    """Sec. 3.2 (the interpolation error of the near/far split, quoted as
    ~1e-7 theta_E): source positions of 1e6 sampled lattice rays of the
    paper-scale map as the shooting kernel computes them (lm_trace_beta: shared
    reciprocals, per-row Taylor re-expansion, FP32 near sums on rebased
    offsets) against the oracle's direct sum over all 13000 lenses: within
    1e-4 theta_E everywhere; and against the oracle's interpolated scheme:
    within FP32 rounding."""
    w = inputs.paper_scale()
    g, mp, orc = _pair(w)
    rng = np.random.default_rng(29)
    n = 1_000_000
    ii = rng.integers(0, g.ray_nx, n)
    jj = rng.integers(0, g.ray_ny, n)
    b_gpu = mp.trace_beta(ii, jj)
    x, y, m = w.lenses()
    gd = oracle_geom(g)
    gd.scheme = oracle.SCHEME_DIRECT
    b_dir, _ = oracle.Oracle(gd, w.kappa, w.gamma, w.kappa_star, x, y, m).trace(ii, jj)
    b_int, _ = orc.trace(ii, jj)
    th = np.stack([g.ray_x0 + (ii + 0.5) * g.ray_dx, g.ray_y0 + (jj + 0.5) * g.ray_dy], axis=1)
    a_mag = np.hypot(*orc.deflect(th).T)
    e_dir = np.hypot(*(b_gpu - b_dir).T)
    e_int = np.hypot(*(b_gpu - b_int).T)
    e_scheme = np.hypot(*(b_int - b_dir).T)
    _say("1e6 rays: max |beta_gpu - beta_direct| = %.2e (rms %.2e), max |beta_gpu - beta_interp| "
         "= %.2e (rms %.2e), oracle interp vs direct max %.2e theta_E" %
         (e_dir.max(), np.sqrt((e_dir ** 2).mean()), e_int.max(), np.sqrt((e_int ** 2).mean()),
          e_scheme.max()))
    assert e_dir.max() <= 1e-4
    # FP32 rounding is relative to the deflection, which grows as 1/r next to a lens
    assert np.all(e_int <= 1e-6 * np.maximum(1.0, a_mag))
    mp.close()


# ------------------------------------------------------------ batch path


def _small_batch(nmaps=6, rays_scale=1e-3):
    ws = inputs.batched_study(nmaps, rays_scale)
    maps = []
    for w in ws:
        g = _geom(w)
        maps.append((w, g, lm.Map(g, w.kappa, w.gamma, w.kappa_star, w.lenses())))
    return maps


def test_batch_equals_per_map_and_tuned_equals_default(tmp_path):
    maps = _small_batch()
    ref = []
    for w, g, mp in maps:
        mp.shoot()
        ref.append(mp.counts())
        mp.reset()
    b = lm.lm_batch_create([mp.h for _, _, mp in maps])
    lm.lm_batch_shoot(b)
    for (w, g, mp), (c, o, s) in zip(maps, ref):
        c2, o2, s2 = mp.counts()
        np.testing.assert_array_equal(c, c2)
        assert (o, s) == (o2, s2)
        mp.reset()
    cache = str(tmp_path / "tune.txt")
    lm.lm_batch_tune(b, cache)
    params = lm.lm_batch_params(b)
    _say("tuned params %s" % (params,))
    lm.lm_batch_shoot(b)
    lm.lm_batch_shoot(b)  # graph replay: counts double
    for (w, g, mp), (c, o, s) in zip(maps, ref):
        c2, o2, s2 = mp.counts()
        np.testing.assert_array_equal(2 * c.astype(np.int64), c2.astype(np.int64))
        assert 2 * o == o2 and 2 * s == s2
    # the cache is reused
    lm.lm_batch_tune(b, cache)
    assert lm.lm_batch_params(b) == params
    # every hand-set execution shape gives the same counts, every LDS layout included
    for nr, gs, wg, lay in ((4, 2, 0, 0), (16, 1, 2, 0), (8, 3, 1, 0), (16, 1, 0, 1),
                            (8, 2, 0, 2), (16, 1, 0, 3), (8, 1, 2, 3)):
        for _, _, mp in maps:
            mp.reset()
        lm.lm_batch_set_params(b, nr, gs, wg, lay)
        assert lm.lm_batch_params(b) == (nr, gs, wg, lay)
        lm.lm_batch_shoot(b)
        for (w, g, mp), (c, o, s) in zip(maps, ref):
            c2, o2, s2 = mp.counts()
            np.testing.assert_array_equal(c, c2)
            assert (o, s) == (o2, s2)
    lm.lm_batch_destroy(b)
    for _, _, mp in maps:
        mp.close()


def test_batch_map_vs_oracle():
    """One map of the batched study, shot by the batch kernel, against the oracle."""
    maps = _small_batch(nmaps=3, rays_scale=1e-4)
    b = lm.lm_batch_create([mp.h for _, _, mp in maps])
    w, g, mp = maps[1]
    rect = (g.ray_nx // 4, 0, min(6000, g.ray_nx // 2), g.ray_ny)
    for k, (_, gk, _) in enumerate(maps):
        if k != 1:
            lm.lm_batch_set_rect(b, k, 0, 0, min(1000, gk.ray_nx), min(1000, gk.ray_ny))
    lm.lm_batch_set_rect(b, 1, *rect)
    lm.lm_batch_shoot(b)
    counts, n_out, _ = mp.counts()
    x, y, m = w.lenses()
    ref, ref_out = oracle.Oracle(oracle_geom(g), w.kappa, w.gamma, w.kappa_star, x, y, m).shoot(
        *rect, nthreads=NTHREADS)
    _compare(g, counts, n_out, ref, ref_out, rect[2] * rect[3], "batched map 1")
    lm.lm_batch_destroy(b)
    for _, _, mp2 in maps:
        mp2.close()


def test_batch_follows_changes_to_its_maps():
    """A member map changed after the batch was built (lenses fewer and then
    more than before, so the lens buffers are reallocated; macro model; a
    caller-owned counts buffer) is shot by the next lm_batch_shoot with its
    new state, bit for bit as the per-map path shoots it."""
    import torch
    maps = _small_batch(nmaps=3, rays_scale=1e-4)
    b = lm.lm_batch_create([mp.h for _, _, mp in maps])
    lm.lm_batch_shoot(b)
    torch.cuda.synchronize()

    def per_map_reference():
        out = []
        for _, _, mp in maps:
            mp.reset()
            mp.shoot()
            out.append(mp.counts())
            mp.reset()
        return out

    w1, g1, mp1 = maps[1]
    x, y, m = w1.lenses()
    w0, g0, mp0 = maps[0]
    for step, n_keep in enumerate((len(x) // 3, len(x))):
        for _, _, mp in maps:
            mp.reset()
        lm.lm_set_lenses(mp1.h, x[:n_keep], y[:n_keep], m[:n_keep])
        if step == 0:
            lm.lm_set_macro(mp0.h, w0.kappa + 0.001, w0.gamma, w0.kappa_star)
        ref = per_map_reference()
        lm.lm_batch_shoot(b)
        for (_, _, mp), (c, o, s) in zip(maps, ref):
            c2, o2, s2 = mp.counts()
            np.testing.assert_array_equal(c, c2)
            assert (o, s) == (o2, s2)
    # counts bound to a caller-owned buffer after the batch was built
    for _, _, mp in maps:
        mp.reset()
    ref = per_map_reference()
    buf = torch.zeros(g1.src_ny * g1.src_nx, dtype=torch.int64, device="cuda")
    lm.lm_bind_counts(mp1.h, buf.data_ptr())
    lm.lm_batch_shoot(b)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(buf.cpu().numpy().reshape(ref[1][0].shape),
                                  ref[1][0].astype(np.int64))
    own = lm.lm_read_counts_region(mp1.h, 0, 0, g1.src_nx, g1.src_ny)
    np.testing.assert_array_equal(own, ref[1][0])
    lm.lm_bind_counts(mp1.h, None)
    lm.lm_batch_destroy(b)
    for _, _, mp in maps:
        mp.close()


def test_batched_study_map_at_full_geometry_vs_oracle():
    """A map of the 80-map study at its full geometry (the map with the fewest
    rays, ~1e11), shot by the persistent batch kernel on a centred rectangle of
    1e-2 of its rays, against the oracle; the other two maps of the batch shoot
    8e6-ray rectangles at the centres of their lattices in the same launch,
    each against the oracle too."""
    ws = inputs.batched_study(80, 1.0)
    k = int(np.argmin([w.n_rays for w in ws]))
    picks = [k, (k + 1) % 80, (k + 2) % 80]
    maps = []
    for idx in picks:
        g = _geom(ws[idx])
        maps.append((ws[idx], g, lm.Map(g, ws[idx].kappa, ws[idx].gamma, ws[idx].kappa_star,
                                        ws[idx].lenses())))
    b = lm.lm_batch_create([mp.h for _, _, mp in maps])
    w, g, mp = maps[0]
    nj = min(g.ray_ny, 4 * g.coarse)
    ni = min(g.ray_nx, int(1e-2 * g.n_rays / nj) + 1)
    rect = ((g.ray_nx - ni) // 2, (g.ray_ny - nj) // 2, ni, nj)
    assert ni * nj >= 1e-2 * g.n_rays
    lm.lm_batch_set_rect(b, 0, *rect)
    rects = {}
    for t in (1, 2):
        gt = maps[t][1]
        rni, rnj = min(8192, gt.ray_nx), min(1024, gt.ray_ny)
        rects[t] = ((gt.ray_nx - rni) // 2, (gt.ray_ny - rnj) // 2, rni, rnj)
        lm.lm_batch_set_rect(b, t, *rects[t])
    lm.lm_batch_shoot(b)
    counts, n_out, _ = mp.counts()
    x, y, m = w.lenses()
    ref, ref_out = oracle.Oracle(oracle_geom(g), w.kappa, w.gamma, w.kappa_star, x, y, m).shoot(
        *rect, nthreads=NTHREADS)
    _compare(g, counts, n_out, ref, ref_out, ni * nj,
             "study map %d (%.3g rays) through the batch kernel" % (k, g.n_rays))
    for t in (1, 2):
        wt, gt, mpt = maps[t]
        rt = rects[t]
        ct, ot, _ = mpt.counts()
        xt, yt, mt = wt.lenses()
        rf, ro = oracle.Oracle(oracle_geom(gt), wt.kappa, wt.gamma, wt.kappa_star, xt, yt,
                               mt).shoot(*rt, nthreads=NTHREADS)
        _compare(gt, ct, ot, rf, ro, rt[2] * rt[3],
                 "study map %d centre through the same launch" % picks[t])
    lm.lm_batch_destroy(b)
    for _, _, mp2 in maps:
        mp2.close()


# ---------------------------------------------------------- plain FP32 path


def test_plain_fp32_path_runs_and_is_worse():
    """The global-FP32 comparison path conserves rays; its error against the
    oracle is reported next to the mixed path's."""
    w = inputs.precision_stress()
    rng = np.random.default_rng(23)
    res = {}
    for prec in (lm.LM_PREC_MIXED, lm.LM_PREC_FP32):
        g, mp, orc = _pair(w, precision=prec)
        ii = rng.integers(0, g.ray_nx, 2000)
        jj = rng.integers(0, g.ray_ny, 2000)
        p, q = mp.trace(ii, jj)
        _, pix = orc.trace(ii, jj)
        gpu_pix = np.where(p >= 0, q.astype(np.int64) * g.src_nx + p, -1)
        res[prec] = float((gpu_pix != pix).mean())
        i0, j0 = g.ray_nx // 2, g.ray_ny // 2
        mp.shoot(i0, j0, 4096, 512)
        c, o, s = mp.counts()
        assert int(c.sum()) + o == s == 4096 * 512
        mp.close()
    _say("sampled flip rate: mixed %.2e, plain fp32 %.2e" % (res[0], res[1]))
    assert res[0] <= 1e-3
    assert res[1] > res[0]


# ------------------------------------------------------------ error paths


def test_error_paths():
    w = inputs.near_fold()
    g, mp, _ = _pair(w)
    with pytest.raises(lm.LensmapError) as e:
        mp.shoot(g.ray_nx - 10, 0, 11, 1)
    assert e.value.status == lm.LM_ERANGE
    mp.shoot(0, 0, 64, 64)
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_set_lenses(mp.h, [0.0], [0.0], [1.0])
    assert e.value.status == lm.LM_ESTATE
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_set_macro(mp.h, 0.1, 0.1, 0.1)
    assert e.value.status == lm.LM_ESTATE
    mp.reset()
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_set_lenses(mp.h, [0.0], [float("nan")], [1.0])
    assert e.value.status == lm.LM_EINVAL
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_set_lenses(mp.h, [0.0], [0.0], [-1.0])
    assert e.value.status == lm.LM_EINVAL
    with pytest.raises(lm.LensmapError) as e:
        mp.trace([g.ray_nx], [0])
    assert e.value.status == lm.LM_ERANGE
    b = lm.lm_batch_create([mp.h])
    for bad in ((5, 1, 0, 0), (8, 0, 0, 0), (8, 9, 0, 0), (8, 1, -1, 0), (8, 1, 9, 0),
                (8, 1, 0, 4)):
        with pytest.raises(lm.LensmapError) as e:
            lm.lm_batch_set_params(b, *bad)
        assert e.value.status == lm.LM_EINVAL
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_batch_set_params(b, 4, 1, 0, 2)  # layouts 1-3 need 8 or 16 rays per lane
    assert e.value.status == lm.LM_EUNSUPPORTED
    lm.lm_batch_destroy(b)
    mp.close()
