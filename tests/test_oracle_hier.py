"""Pins of the oracle's hierarchical far field (level-1 series re-expanded about
each level-2 centre) against closed forms and against the direct level-2
coefficients of Sec. 3.2.2.

For one far lens at z_k, with Z the level-1 centre, u = z_k - Z, w = z_c - Z
and rho = w/u, the Q-term series gives exactly
    a_0^(Q) = -(m/u) (1 - rho^Q) / (1 - rho),
    a_1^(Q) = -(m/u^2) (1 - Q rho^(Q-1) + (Q-1) rho^Q) / (1 - rho)^2,
the finite geometric sums (and their derivative) of the re-expansion; as Q
grows they tend to the direct coefficients -m/(z_k - z_c)^(n+1).
"""
import math

import numpy as np
import pytest

from oracle.geometry import OracleGeometry


def _geom(far_order, terms=4):
    # 512 x 512 rays of spacing 0.02 in 64-ray level-2 cells, 2 x 2 level-2
    # cells per level-1 cell: level-1 cells of 2.56 x 2.56 theta_E
    return OracleGeometry(src_x0=-4.0, src_y0=-4.0, src_dx=8 / 128, src_dy=8 / 128, src_nx=128,
                          src_ny=128, ray_x0=-5.12, ray_y0=-5.12, ray_dx=0.02, ray_dy=0.02,
                          ray_nx=512, ray_ny=512, scheme=1, coarse=64, l1_kx=2, l1_ky=2, halo=1,
                          terms=terms, far_order=far_order)


def _centres(g, ci, cj):
    L1x = g.l1_kx * g.coarse * g.ray_dx
    L1y = g.l1_ky * g.coarse * g.ray_dy
    I, J = ci // g.l1_kx, cj // g.l1_ky
    Z = complex(g.ray_x0 + (I + 0.5) * L1x, g.ray_y0 + (J + 0.5) * L1y)
    zc = complex(g.ray_x0 + (ci + 0.5) * g.coarse * g.ray_dx,
                 g.ray_y0 + (cj + 0.5) * g.coarse * g.ray_dy)
    return Z, zc


@pytest.mark.parametrize("Q", [6, 12, 24])
def test_single_far_lens_closed_forms(oracle_lib, Q):
    """a_0 and a_1 of one far lens equal the truncated geometric sums."""
    ci, cj = 3, 2
    g = _geom(Q)
    Z, zc = _centres(g, ci, cj)
    zk = complex(-0.9, 4.3)  # three level-1 cells above: far
    m = 0.7
    o = oracle_lib.Oracle(g, 0.0, 0.0, 0.0, [zk.real], [zk.imag], [m])
    assert not o.near_mask(ci, cj)[0]
    a = o.coeffs(ci, cj)
    u, w = zk - Z, zc - Z
    rho = w / u
    a0 = -(m / u) * (1 - rho ** Q) / (1 - rho)
    a1 = -(m / u ** 2) * (1 - Q * rho ** (Q - 1) + (Q - 1) * rho ** Q) / (1 - rho) ** 2
    assert abs(a[0] - a0) <= 1e-13 * abs(a0)
    assert abs(a[1] - a1) <= 1e-12 * abs(a1)


def test_single_far_lens_converges_to_direct(oracle_lib):
    """Every a_p tends to -m/(z_k - z_c)^(p+1) (Sec. 3.2.2) geometrically in Q."""
    ci, cj = 4, 5
    zk, m = complex(2.9, -3.7), 1.3
    Z, zc = _centres(_geom(8), ci, cj)
    rho = abs((zc - Z) / (zk - Z))
    exact = np.array([-m / (zk - zc) ** (p + 1) for p in range(4)])
    errs = []
    for Q in (8, 16, 24):
        o = oracle_lib.Oracle(_geom(Q), 0.0, 0.0, 0.0, [zk.real], [zk.imag], [m])
        errs.append(np.abs(o.coeffs(ci, cj) - exact) / np.abs(exact))
    for p in range(4):
        assert errs[1][p] < errs[0][p] * rho ** 8 * 50
        assert errs[2][p] < 1e-5
    assert errs[2][0] < 1e-9


def test_lens_field_matches_direct_coefficients(oracle_lib):
    """With many lenses, hierarchical and direct coefficients differ by no
    more than the summed single-lens truncation bounds; a wrong far set would
    differ by whole lens terms."""
    rng = np.random.default_rng(5)
    n = 300
    x, y = rng.uniform(-7, 7, n), rng.uniform(-7, 7, n)
    m = rng.uniform(0.1, 1.5, n)
    Q = 20
    gd, gh = _geom(0), _geom(Q)
    od = oracle_lib.Oracle(gd, 0.0, 0.0, 0.0, x, y, m)
    oh = oracle_lib.Oracle(gh, 0.0, 0.0, 0.0, x, y, m)
    for ci, cj in [(0, 0), (3, 4), (7, 7), (5, 1)]:
        Z, zc = _centres(gh, ci, cj)
        far = ~od.near_mask(ci, cj)
        u = (x + 1j * y)[far] - Z
        r = abs(zc - Z) / np.abs(u)
        assert r.max() < 0.5
        ad, ah = od.coeffs(ci, cj), oh.coeffs(ci, cj)
        for p in range(4):
            # |remainder| <= sum_k m_k/|u_k|^(p+1) sum_{n>=Q} C(n,p) r_k^(n-p)
            tail = sum(math.comb(k, p) * r ** (k - p) for k in range(Q, Q + 200))
            bound = float(np.sum(m[far] / np.abs(u) ** (p + 1) * tail)) + 1e-14
            assert abs(ah[p] - ad[p]) <= bound
            assert abs(ah[p] - ad[p]) <= 1e-4 * abs(ad[p]) + 1e-12


def test_hierarchical_map_matches_direct_map(oracle_lib):
    """Shooting with the hierarchical far field reproduces the direct-coefficient
    map except for rays within the truncation error of a pixel edge."""
    rng = np.random.default_rng(6)
    n = 400
    x, y = rng.uniform(-6, 6, n), rng.uniform(-6, 6, n)
    m = np.ones(n)
    od = oracle_lib.Oracle(_geom(0), 0.3, 0.1, 0.02, x, y, m)
    oh = oracle_lib.Oracle(_geom(24), 0.3, 0.1, 0.02, x, y, m)
    cd, od_out = od.shoot()
    ch, oh_out = oh.shoot()
    assert int(cd.sum()) + od_out == int(ch.sum()) + oh_out == 512 * 512
    mis = 0.5 * np.abs(cd.astype(np.int64) - ch.astype(np.int64)).sum() / (512 * 512)
    assert mis < 1e-5


# ------------------------------------------------- elongated level-1 cells


def _geom_long(far_order, kx, ky=2, terms=4, n=1024):
    # level-2 cells of 64 x 64 rays of spacing 0.02 (1.28 theta_E), kx x ky per
    # level-1 cell: level-1 cells of (1.28 kx) x (1.28 ky) theta_E
    return OracleGeometry(src_x0=-4.0, src_y0=-4.0, src_dx=8 / 128, src_dy=8 / 128, src_nx=128,
                          src_ny=128, ray_x0=-10.24, ray_y0=-5.12, ray_dx=0.02, ray_dy=0.02,
                          ray_nx=n, ray_ny=512, scheme=1, coarse=64, l1_kx=kx, l1_ky=ky, halo=1,
                          terms=terms, far_order=far_order)


def _box_centre_by_hand(g, ci, cj, b):
    """Centre of the box of b level-2 columns (counted from the level-1 cell's
    left edge) that holds level-2 cell (ci, cj); the box does not reach past
    the level-1 cell."""
    L2 = g.coarse * g.ray_dx
    I, J = ci // g.l1_kx, cj // g.l1_ky
    c0 = I * g.l1_kx + ((ci - I * g.l1_kx) // b) * b
    c1 = min(c0 + b, (I + 1) * g.l1_kx)
    return complex(g.ray_x0 + 0.5 * (c0 + c1) * L2,
                   g.ray_y0 + (J + 0.5) * g.l1_ky * g.coarse * g.ray_dy)


@pytest.mark.parametrize("kx,ci,b", [(8, 13, 2), (8, 8, 2), (7, 9, 2), (7, 13, 2), (7, 20, 2),
                                     (12, 17, 2)])
def test_elongated_cell_box_centre_closed_forms(oracle_lib, kx, ci, b):
    """A level-1 cell kx times longer than wide (in level-2 cells: kx x 2) is
    cut into round(kx / 2) boxes of ceil(kx / round(kx / 2)) level-2 cells,
    the last one narrower when they do not divide evenly (kx = 7: 2, 2, 2, 1);
    the series is taken about the centre of the box that holds the cell.  One
    far lens: a_0 and a_1 equal the truncated geometric sums about that
    centre."""
    Q, cj = 16, 3
    g = _geom_long(Q, kx)
    Z = _box_centre_by_hand(g, ci, cj, b)
    zc = complex(g.ray_x0 + (ci + 0.5) * g.coarse * g.ray_dx,
                 g.ray_y0 + (cj + 0.5) * g.coarse * g.ray_dy)
    zk, m = complex(2.3, 4.1), 0.8  # at least two level-1 rows above: far
    o = oracle_lib.Oracle(g, 0.0, 0.0, 0.0, [zk.real], [zk.imag], [m])
    assert not o.near_mask(ci, cj)[0]
    a = o.coeffs(ci, cj)
    u, w = zk - Z, zc - Z
    rho = w / u
    a0 = -(m / u) * (1 - rho ** Q) / (1 - rho)
    a1 = -(m / u ** 2) * (1 - Q * rho ** (Q - 1) + (Q - 1) * rho ** Q) / (1 - rho) ** 2
    assert abs(a[0] - a0) <= 1e-13 * abs(a0)
    assert abs(a[1] - a1) <= 1e-12 * abs(a1)


def test_elongated_cells_converge_where_the_cell_centre_would_not(oracle_lib):
    """Level-1 cells of 12 x 2 level-2 cells (15.4 x 2.6 theta_E): from the
    cell centre, far lenses beside the block lie closer than the cell's end
    cells (ratio above 1: that series diverges); from the boxes' centres every
    ratio stays below 0.5, and the hierarchical coefficients agree with the
    direct ones within the summed truncation bounds."""
    rng = np.random.default_rng(9)
    n = 400
    x, y = rng.uniform(-10, 10, n), rng.uniform(-5, 5, n)
    m = rng.uniform(0.1, 1.5, n)
    Q = 24
    gd, gh = _geom_long(0, 12), _geom_long(Q, 12)
    od = oracle_lib.Oracle(gd, 0.0, 0.0, 0.0, x, y, m)
    oh = oracle_lib.Oracle(gh, 0.0, 0.0, 0.0, x, y, m)
    worst_cell_centre = 0.0
    for ci, cj in [(12, 2), (17, 3), (23, 4), (0, 0), (6, 5)]:
        zc = complex(gh.ray_x0 + (ci + 0.5) * gh.coarse * gh.ray_dx,
                     gh.ray_y0 + (cj + 0.5) * gh.coarse * gh.ray_dy)
        Z = _box_centre_by_hand(gh, ci, cj, 2)
        I, J = ci // 12, cj // 2
        Zcell = complex(gh.ray_x0 + (I + 0.5) * 12 * 1.28, gh.ray_y0 + (J + 0.5) * 2 * 1.28)
        far = ~od.near_mask(ci, cj)
        zk = (x + 1j * y)[far]
        r = abs(zc - Z) / np.abs(zk - Z)
        assert r.max() < 0.5
        worst_cell_centre = max(worst_cell_centre, float((abs(zc - Zcell) / np.abs(zk - Zcell)).max()))
        ad, ah = od.coeffs(ci, cj), oh.coeffs(ci, cj)
        u = zk - Z
        for p in range(4):
            tail = sum(math.comb(k, p) * r ** (k - p) for k in range(Q, Q + 200))
            bound = float(np.sum(m[far] / np.abs(u) ** (p + 1) * tail)) + 1e-14
            assert abs(ah[p] - ad[p]) <= bound
    assert worst_cell_centre > 1.0
