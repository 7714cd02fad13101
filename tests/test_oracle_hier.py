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
