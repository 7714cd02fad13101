"""GPU parity at the edges of the scheme's parameters, against the FP64 oracle:
Taylor orders P = 1, 2 and 7 (the largest supported) and near halos H = 0 and
2; near lists longer than one LDS block (more than 64 near lenses, several
staging blocks per unit); the direct scheme over several 256-lens compensated
blocks; the FP64 near-sum mode with the largest P."""
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


def _near_fold(**over):
    w = inputs.near_fold()
    g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                              w.gamma, w.kappa_star, n_rays=w.n_rays, scheme=w.scheme,
                              coarse=w.coarse, mean_mass=w.mean_mass)
    for k, v in over.items():
        setattr(g, k, v)
    return w, g


def _run(w, g, rect, what, lenses=None, bar=1e-5):
    x, y, m = lenses if lenses is not None else w.lenses()
    mp = lm.Map(g, w.kappa, w.gamma, w.kappa_star, (x, y, m))
    orc = oracle.Oracle(oracle_geom(g), w.kappa, w.gamma, w.kappa_star, x, y, m)
    i0, j0, ni, nj = rect
    mp.shoot(i0, j0, ni, nj)
    counts, n_out, n_shot = mp.counts()
    ref, ref_out = orc.shoot(i0, j0, ni, nj, nthreads=NTHREADS)
    mis = mismatch_fraction(counts, ref, ni * nj)
    print("%s: rays %d, mismatch %.2e, worst pixel %.2e" % (what, ni * nj, mis,
                                                            max_pixel_rel(counts, ref)))
    assert int(counts.sum()) + n_out == n_shot == ni * nj
    assert int(ref.sum()) + ref_out == ni * nj
    assert mis <= bar
    assert max_pixel_rel(counts, ref) <= 1e-3
    mp.close()


@pytest.mark.parametrize("terms,halo,precision", [(1, 1, 0), (2, 1, 0), (7, 1, 0), (4, 0, 0),
                                                  (4, 2, 0), (7, 1, 2)])
def test_terms_and_halo(terms, halo, precision):
    w, g = _near_fold(taylor_terms=terms, near_halo=halo, precision=precision)
    _run(w, g, (700_011, 20_033, 3_001, 1_500),
         "near-fold P=%d H=%d prec=%d" % (terms, halo, precision))


@pytest.mark.parametrize("precision", [lm.LM_PREC_AUTO, lm.LM_PREC_MIXED_FP64])
def test_near_lists_longer_than_one_block(precision):
    """Level-1 cells 5x larger per side: ~100 near lenses per ray, so a unit
    stages its near list in several 64-lens blocks.  FP32 near sums round
    more with ~100 terms than with the method's ~9 (1.8e-5 of the rays move
    pixel), so the library's default precision choice must pick FP64 near
    sums here; both paths meet the 1e-5 bar."""
    w, g = _near_fold(precision=precision)
    g.l1_kx *= 5
    g.l1_ky *= 5
    lm_map = lm.Map(g, w.kappa, w.gamma, w.kappa_star, w.lenses())
    st = lm.lm_shot_stats(lm_map.h, 700_000, 20_000, 3_000, 1_500)
    used, est, _ = lm_map.precision()
    lm_map.close()
    pairs = st.near_pairs / st.rays
    print("near lenses per ray: %.1f; precision %d (FP32 mismatch estimate %.2e)" %
          (pairs, used, est))
    assert pairs > 80
    if precision == lm.LM_PREC_AUTO:
        # the lattice-mean estimate alone (~3e-6) would keep FP32: the near-list
        # length decides
        assert used == lm.LM_PREC_MIXED_FP64
    _run(w, g, (700_011, 20_033, 2_001, 1_100), "near-fold, long near lists, prec=%d" % precision)


def test_direct_scheme_several_blocks():
    """Direct sum over 700 lenses: three 256-lens compensated blocks."""
    w = inputs.plain_small()
    rng = np.random.default_rng(12)
    n = 700
    r, phi = 30.0 * np.sqrt(rng.random(n)), 2 * np.pi * rng.random(n)
    lenses = (r * np.cos(phi), r * np.sin(phi), np.ones(n))
    g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                              w.gamma, w.kappa_star, protect=w.protect, ray_nx=1536,
                              ray_ny=1536, scheme=lm.LM_SCHEME_DIRECT, coarse=64)
    _run(w, g, (0, 0, 1536, 1536), "direct, 700 lenses", lenses)
