"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the header declares, derives geometry by the paper's rules in
agreement with the oracle's independent derivation, and rejects bad input
before touching a device."""
import ctypes
import math

import numpy as np
import pytest

import paper_2308_14278_amd.lensmap as lm
from paper_2308_14278_amd import inputs
from oracle.geometry import derive_geometry


@pytest.fixture(scope="module")
def lib():
    return lm.load()


def test_exports_every_declared_symbol(lib):
    names = lm.header_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_struct_layout_matches_header(lib):
    # int32 fields are packed in pairs; the struct must be 8-byte aligned
    assert ctypes.sizeof(lm.lm_geometry) == 8 * 4 + 4 * 2 + 8 * 4 + 8 * 2 + 4 * 8


def test_version(lib):
    assert "gfx950" in lm.lm_version()


@pytest.mark.parametrize("kind", ["plain-small", "near-fold", "paper-scale", "precision-stress"])
def test_geometry_matches_oracle(kind):
    from paper_2308_14278_amd import inputs
    w = inputs.WORKLOADS[kind]()
    kw = dict(n_rays=w.n_rays, ray_nx=w.ray_nx, ray_ny=w.ray_ny, protect=w.protect,
              scheme=w.scheme, coarse=w.coarse)
    go = derive_geometry(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa, w.gamma,
                         w.kappa_star, mean_mass=w.mean_mass, **kw)
    gl = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                               w.gamma, w.kappa_star, mean_mass=w.mean_mass, **kw)
    for f in ("src_nx", "src_ny", "ray_nx", "ray_ny", "coarse"):
        assert getattr(gl, f) == getattr(go, f), f
    if w.scheme == 1:
        assert (gl.l1_kx, gl.l1_ky) == (go.l1_kx, go.l1_ky)
    for f in ("src_x0", "src_y0", "src_dx", "src_dy", "ray_x0", "ray_y0", "ray_dx", "ray_dy"):
        assert math.isclose(getattr(gl, f), getattr(go, f), rel_tol=1e-14), f
    assert gl.near_halo == 1 and gl.taylor_terms == 4


def test_paper_scale_geometry_numbers():
    """Paper-scale workload: 1e13 rays, level-2 cells of ~L1/20, level-1 ~ L0."""
    from paper_2308_14278_amd import inputs
    w = inputs.paper_scale()
    g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                              w.gamma, w.kappa_star, n_rays=w.n_rays, mean_mass=w.mean_mass)
    assert abs(g.n_rays / 1e13 - 1) < 1e-5
    l0 = math.sqrt(math.pi * w.mean_mass / w.kappa_star)
    assert abs(g.coarse * g.ray_dx * 20 / l0 - 1) < 0.05
    assert g.l1_kx == 20


def test_derive_rejects_bad_input():
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_geometry_derive(10, 10, 64, 64, 0.5, 0.5, 0.01, n_rays=1e6)  # lt = 0: singular
    assert e.value.status == lm.LM_EINVAL
    with pytest.raises(lm.LensmapError):
        lm.lm_geometry_derive(float("nan"), 10, 64, 64, 0.4, 0.5, 0.01, n_rays=1e6)
    with pytest.raises(lm.LensmapError):
        lm.lm_geometry_derive(10, 10, 0, 64, 0.4, 0.5, 0.01, n_rays=1e6)


def _good():
    return lm.lm_geometry_derive(10, 10, 64, 64, 0.45, 0.5, 0.01, n_rays=1e6, scheme=1, coarse=64)


@pytest.mark.parametrize("field,value", [("coarse", 100), ("coarse", 0), ("src_nx", 0),
                                         ("ray_dx", -1.0), ("taylor_terms", 9),
                                         ("scheme", 5), ("precision", 5), ("l1_kx", 0),
                                         ("ray_x0", float("inf"))])
def test_create_rejects_invalid_geometry(field, value):
    g = _good()
    setattr(g, field, value)
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_create(g)
    assert e.value.status == lm.LM_EINVAL
    assert lm.lm_last_error() != ""


def test_fp64_near_mode_needs_the_interpolated_scheme():
    g = lm.lm_geometry_derive(10, 10, 64, 64, 0.45, 0.5, 0.01, n_rays=1e6, scheme=0, coarse=64)
    g.precision = lm.LM_PREC_MIXED_FP64
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_create(g)
    assert e.value.status == lm.LM_EUNSUPPORTED


def test_far_order_validation():
    g = lm.lm_geometry_derive(20, 20, 200, 200, 0.45, 0.5, 0.01, n_rays=1e9, scheme=1)
    assert g.far_order == 0
    for q, status in ((3, lm.LM_EINVAL), (65, lm.LM_EINVAL), (8, lm.LM_EINVAL)):
        g.far_order = q  # below P, above 64, and elongated level-1 cells (no convergence)
        with pytest.raises(lm.LensmapError) as e:
            lm.lm_create(g)
        assert e.value.status == status
    g.far_order = 48
    g.precision = lm.LM_PREC_FP32
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_create(g)
    assert e.value.status == lm.LM_EUNSUPPORTED
    g2 = lm.lm_geometry_derive(10, 10, 64, 64, 0.45, 0.5, 0.01, n_rays=1e6, scheme=0, coarse=64)
    g2.far_order = 32
    with pytest.raises(lm.LensmapError) as e:
        lm.lm_create(g2)
    assert e.value.status == lm.LM_EINVAL


def test_far_order_choice():
    """The chosen order is the smallest meeting rho^Q / (1 - rho) <= 1e-9, with
    rho recomputed here from the geometry."""
    import math
    w = inputs.paper_scale()
    g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                              w.gamma, w.kappa_star, n_rays=w.n_rays, scheme=1,
                              mean_mass=w.mean_mass)
    q = lm.lm_geometry_far_order(g)
    l2x, l2y = g.coarse * g.ray_dx, g.coarse * g.ray_dy
    rho = math.hypot(0.5 * (g.l1_kx - 1) * l2x, 0.5 * (g.l1_ky - 1) * l2y) / (
        (g.near_halo + 0.5) * min(g.l1_kx * l2x, g.l1_ky * l2y))
    assert 0.4 < rho < 0.5 and q == g.far_order
    assert rho ** q / (1 - rho) <= 1e-9 < rho ** (q - 1) / (1 - rho)
    # elongated level-1 cells: about the cell centre no order converges; cut
    # into round(long / short) boxes of ceil(K / boxes) level-2 cells (the last
    # narrower), the ratio is that of the worst box
    g2 = lm.lm_geometry_derive(20, 20, 200, 200, 0.45, 0.5, 0.01, n_rays=1e9, scheme=1)
    l2x, l2y = g2.coarse * g2.ray_dx, g2.coarse * g2.ray_dy
    l1x, l1y = g2.l1_kx * l2x, g2.l1_ky * l2y
    H = g2.near_halo
    assert math.hypot(0.5 * (g2.l1_kx - 1) * l2x, 0.5 * (g2.l1_ky - 1) * l2y) / (
        (H + 0.5) * min(l1x, l1y)) > 1.0
    assert l1x > 1.5 * l1y
    nb = min(g2.l1_kx, max(1, math.floor(l1x / l1y + 0.5)))
    b = -(-g2.l1_kx // nb)
    widths = {b, g2.l1_kx - (nb - 1) * b}
    rho2 = max(math.hypot(0.5 * (wx - 1) * l2x, 0.5 * (g2.l1_ky - 1) * l2y) /
               min(H * l1x + 0.5 * wx * l2x, H * l1y + 0.5 * g2.l1_ky * l2y) for wx in widths)
    q2 = lm.lm_geometry_far_order(g2)
    assert rho2 < 0.5 and q2 == g2.far_order > 0
    assert rho2 ** q2 / (1 - rho2) <= 1e-9 < rho2 ** (q2 - 1) / (1 - rho2)


def test_null_handles_are_rejected(lib):
    assert lib.lm_shoot(None, 0, 0, 1, 1, None) == lm.LM_EINVAL
    assert lib.lm_set_macro(None, 0.0, 0.0, 0.0) == lm.LM_EINVAL
    assert lib.lm_read_counts(None, None, None, None) == lm.LM_EINVAL
    assert lib.lm_batch_shoot(None, None) == lm.LM_EINVAL
    assert lib.lm_batch_set_params(None, 8, 1, 0, 0) == lm.LM_EINVAL
    assert lib.lm_read_coeffs(None, 0, 0, None) == lm.LM_EINVAL
    lib.lm_destroy(None)
    lib.lm_batch_destroy(None)


@pytest.mark.parametrize("scale", [1.0, 1e-4])
def test_fold_geometry_matches_oracle(scale):
    from oracle.geometry import derive_fold_geometry
    from paper_2308_14278_amd import inputs
    w = inputs.paper_table1()
    k0, dx, dy = w.fold
    ny = int(w.extra["src_ny"] * scale) or 1
    nx = int(w.src_pixels * scale) or 1
    go = derive_fold_geometry(w.src_side, w.extra["src_ly"], nx, ny, k0, dx, w.kappa_star,
                              n_rays=w.n_rays * scale)
    gl = lm.lm_geometry_derive_fold(w.src_side, w.extra["src_ly"], nx, ny, k0, dx, w.kappa_star,
                                    n_rays=w.n_rays * scale)
    for f in ("src_nx", "src_ny", "ray_nx", "ray_ny", "coarse", "l1_kx", "l1_ky"):
        assert getattr(gl, f) == getattr(go, f), f
    for f in ("src_x0", "src_y0", "src_dx", "src_dy", "ray_x0", "ray_y0", "ray_dx", "ray_dy"):
        assert math.isclose(getattr(gl, f), getattr(go, f), rel_tol=1e-14), f


@pytest.mark.parametrize("kind", ["paper-scale", "near-fold", "precision-stress"])
def test_tuning_sample_is_the_same_rays_for_every_candidate(kind):
    """lm_batch_tune times every candidate on the same rays: the sample of a map
    is a function of its geometry, shot rectangle and the fraction only, so
    asking for it with each tile scale gives the same rectangle (whole level-2
    cells, inside the shot rectangle, about the requested fraction of its rays)
    while the number of workgroup tiles it spans changes with the tile scale."""
    w = inputs.WORKLOADS[kind]()
    g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                              w.gamma, w.kappa_star, protect=w.protect, n_rays=w.n_rays,
                              scheme=w.scheme, coarse=w.coarse, mean_mass=w.mean_mass)
    frac = min(1.0, 2e10 / g.n_rays)
    rects, tiles = set(), []
    for ts in range(1, 9):
        rect, nt = lm.lm_tune_sample(g, 0, 0, g.ray_nx, g.ray_ny, frac, ts)
        rects.add(rect)
        tiles.append(nt)
    assert len(rects) == 1
    i0, j0, ni, nj = rects.pop()
    R = g.coarse
    assert i0 % R == 0 and j0 % R == 0
    assert 0 <= i0 and i0 + ni <= g.ray_nx and 0 <= j0 and j0 + nj <= g.ray_ny
    assert ni % R == 0 or i0 + ni == g.ray_nx
    assert nj % R == 0 or j0 + nj == g.ray_ny
    assert 0.5 * frac * g.n_rays <= ni * nj <= 2.0 * frac * g.n_rays + 4 * R * R
    assert len(set(tiles)) > 1, tiles
    # a sub-rectangle: the sample stays inside it
    rect, _ = lm.lm_tune_sample(g, 1000, 7, g.ray_nx // 3, g.ray_ny // 2, 0.01, 1)
    assert rect[0] >= 1000 and rect[0] + rect[2] <= 1000 + g.ray_nx // 3
    assert rect[1] >= 7 and rect[1] + rect[3] <= 7 + g.ray_ny // 2
    with pytest.raises(lm.LensmapError):
        lm.lm_tune_sample(g, 0, 0, g.ray_nx, g.ray_ny, 0.0, 1)
    with pytest.raises(lm.LensmapError):
        lm.lm_tune_sample(g, 0, 0, g.ray_nx, g.ray_ny, 0.5, 9)


def test_default_precision_is_the_librarys_choice():
    """Derived geometries leave the near-sum precision to the library for the
    interpolated scheme (LM_PREC_AUTO) and use the compensated FP32 sums of
    the direct scheme (LM_PREC_MIXED)."""
    for kind in ("plain-small", "near-fold", "paper-scale"):
        w = inputs.WORKLOADS[kind]()
        g = lm.lm_geometry_derive(w.src_side, w.src_side, w.src_pixels, w.src_pixels, w.kappa,
                                  w.gamma, w.kappa_star, protect=w.protect, n_rays=w.n_rays or 0,
                                  ray_nx=w.ray_nx or 0, ray_ny=w.ray_ny or 0, scheme=w.scheme,
                                  coarse=w.coarse, mean_mass=w.mean_mass)
        want = lm.LM_PREC_AUTO if w.scheme == lm.LM_SCHEME_INTERP else lm.LM_PREC_MIXED
        assert g.precision == want, kind
    w = inputs.paper_table1()
    g = lm.lm_geometry_derive_fold(w.src_side, w.extra["src_ly"], w.src_pixels,
                                   w.extra["src_ny"], *w.fold[:2], w.kappa_star, n_rays=w.n_rays)
    assert g.precision == lm.LM_PREC_AUTO
