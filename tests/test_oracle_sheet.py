"""Pins of the oracle's compensating sheet (Sec. 2, Eq. 6) on the rectangle of
the lenses: its closed form against one-dimensional numerical integration of
the defining double integral, the infinite-sheet limit, the far-field
monopole, the divergence and curl that a uniform density fixes, and, through
the lens equation, that a dense lattice of point lenses filling the rectangle
is cancelled by it (the total density stays that of the macro model)."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle.geometry import OracleGeometry

RECT = (-5.0, 7.0, -2.0, 1.5)  # x0, x1, y0, y1
KS = 0.01


@pytest.fixture(scope="module")
def oracle_lib():
    oracle.build()
    return oracle


def _geom(scheme=0):
    # rays at multiples of 0.05, half a spacing from the lens lattice below
    return OracleGeometry(-10.0, -10.0, 0.05, 0.05, 400, 400, -10.025, -10.025, 0.05, 0.05,
                          400, 400, scheme=scheme)


def _sheet(oracle_lib, rect=RECT, ks=KS):
    return oracle_lib.Oracle(_geom(), 0.4, 0.1, ks, [], [], [], sheet=rect)


def _by_quadrature(ks, rect, tx, ty):
    """(ks / pi) int int (theta - t) / |theta - t|^2 d^2 t, the inner integral
    done by hand (an arctangent), the outer by adaptive quadrature."""
    x0, x1, y0, y1 = rect

    def fx(x):
        u = tx - x
        if u == 0.0:
            return 0.0
        return math.atan((ty - y0) / u) - math.atan((ty - y1) / u)

    def fy(y):
        v = ty - y
        if v == 0.0:
            return 0.0
        return math.atan((tx - x0) / v) - math.atan((tx - x1) / v)

    px = [tx] if x0 < tx < x1 else None
    py = [ty] if y0 < ty < y1 else None
    ax = integrate.quad(fx, x0, x1, points=px, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    ay = integrate.quad(fy, y0, y1, points=py, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    return ks / math.pi * ax, ks / math.pi * ay


@pytest.mark.parametrize("pt", [(0.3, -0.4), (6.9, 1.4), (-4.99, -1.99), (7.0, 0.0),
                                (12.0, 5.0), (-20.0, -1.0), (1.0, 1.5), (0.0, 30.0)])
def test_closed_form_matches_quadrature(oracle_lib, pt):
    got = _sheet(oracle_lib).sheet(np.array([pt]))[0]
    want = _by_quadrature(KS, RECT, *pt)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-13), (got, want)


def test_infinite_sheet_limit(oracle_lib):
    """Deep inside a huge square about the origin the term is kappa_star theta,
    the infinite sheet's (the remainder falls as |theta|^3 / L^2)."""
    big = 1e4
    o = _sheet(oracle_lib, rect=(-big, big, -big, big))
    th = np.array([[1.0, 0.5], [-30.0, 12.0], [250.0, -400.0], [40.0, 10.0]])
    rel = np.abs(o.sheet(th) / (KS * th) - 1.0)
    bound = 4.0 * (np.hypot(th[:, 0], th[:, 1]) / big) ** 2 + 1e-9
    assert (rel <= bound[:, None]).all(), (rel, bound)
    inf = oracle_lib.Oracle(_geom(), 0.4, 0.1, KS, [], [], [])
    assert np.array_equal(inf.sheet(th), KS * th)


def test_far_field_is_a_point_mass(oracle_lib):
    """Far away the rectangle deflects like its mass, kappa_star A / pi, at its
    centre; the next term falls as 1/d^3."""
    x0, x1, y0, y1 = RECT
    mass = KS * (x1 - x0) * (y1 - y0) / math.pi
    c = np.array([0.5 * (x0 + x1), 0.5 * (y0 + y1)])
    o = _sheet(oracle_lib)
    for d in (1e3, 1e4):
        for ang in (0.3, 2.0, 4.0):
            th = c + d * np.array([math.cos(ang), math.sin(ang)])
            r = th - c
            want = mass * r / (r @ r)
            got = o.sheet(th[None])[0]
            assert np.linalg.norm(got - want) <= 50.0 * mass / d ** 3


def test_divergence_and_curl(oracle_lib):
    """A uniform density: div s = 2 kappa_star inside the rectangle and 0
    outside, curl s = 0 everywhere (central differences)."""
    o = _sheet(oracle_lib)
    h = 1e-4
    for (tx, ty), inside in (((0.3, -0.4), True), ((5.5, 1.0), True), ((9.0, 0.0), False),
                             ((0.0, -3.0), False), ((-8.0, 4.0), False)):
        pts = np.array([[tx + h, ty], [tx - h, ty], [tx, ty + h], [tx, ty - h]])
        s = o.sheet(pts)
        dxx = (s[0, 0] - s[1, 0]) / (2 * h)
        dyy = (s[2, 1] - s[3, 1]) / (2 * h)
        dxy = (s[0, 1] - s[1, 1]) / (2 * h)
        dyx = (s[2, 0] - s[3, 0]) / (2 * h)
        assert abs(dxx + dyy - (2 * KS if inside else 0.0)) < 1e-7
        assert abs(dxy - dyx) < 1e-7


def test_mirror_symmetry(oracle_lib):
    """About its centre the rectangle's term is odd in each coordinate."""
    rect = (-3.0, 3.0, -1.0, 1.0)
    o = _sheet(oracle_lib, rect=rect)
    th = np.array([[0.7, 0.2], [-0.7, 0.2], [0.7, -0.2], [-0.7, -0.2]])
    s = o.sheet(th)
    assert np.allclose(s[1], [-s[0, 0], s[0, 1]], rtol=1e-13, atol=1e-16)
    assert np.allclose(s[2], [s[0, 0], -s[0, 1]], rtol=1e-13, atol=1e-16)
    assert np.allclose(s[3], -s[0], rtol=1e-13, atol=1e-16)


def test_lens_lattice_is_cancelled(oracle_lib):
    """Point lenses on a fine lattice filling the rectangle, each carrying the
    density of its lattice cell (m = kappa_star h^2 / pi), deflect like the
    sheet away from the lattice points, so with the sheet term the lens
    equation gives back the macro map (Sec. 2: the total density is that of
    the smooth model).  With an infinite sheet instead, the elongated
    rectangle leaves kappa_star (theta - s(theta)) uncancelled."""
    x0, x1, y0, y1 = RECT
    h = 0.05
    xs = np.arange(x0 + 0.5 * h, x1, h)
    ys = np.arange(y0 + 0.5 * h, y1, h)
    lx, ly = [a.ravel() for a in np.meshgrid(xs, ys)]
    lm = np.full(lx.size, KS * h * h / math.pi)
    g = _geom()
    kappa, gamma = 0.4, 0.1
    o = oracle_lib.Oracle(g, kappa, gamma, KS, lx, ly, lm, sheet=RECT)
    oinf = oracle_lib.Oracle(g, kappa, gamma, KS, lx, ly, lm)
    # rays at lattice-cell corners, away from every lens, inside and outside
    ii = np.array([[int(round((x - g.ray_x0) / g.ray_dx - 0.5)),
                    int(round((y - g.ray_y0) / g.ray_dy - 0.5))]
                   for x, y in ((0.0, 0.0), (3.0, -1.0), (6.5, 1.0), (-8.0, 3.0), (9.0, -6.0))])
    beta, _ = o.trace(ii[:, 0], ii[:, 1])
    beta_inf, _ = oinf.trace(ii[:, 0], ii[:, 1])
    th = np.stack([g.ray_x0 + (ii[:, 0] + 0.5) * g.ray_dx,
                   g.ray_y0 + (ii[:, 1] + 0.5) * g.ray_dy], axis=1)
    macro = th * np.array([1 - kappa - gamma, 1 - kappa + gamma])
    assert np.abs(beta - macro).max() < 1e-9
    left = KS * th - o.sheet(th)
    assert np.allclose(beta_inf - macro, left, atol=1e-9)
    assert np.abs(left).max() > 1e-3


# ------------------------------------------- interpolated scheme: series


def _lattice(scheme, nx, ny, terms=4):
    """Rays over [-8, 8] x [-4, 4] (16/nx and 8/ny apart), level-2 cells of 64
    rays; nx, ny need not be multiples of 64."""
    return OracleGeometry(-10.0, -6.0, 0.05, 0.05, 400, 240, -8.0, -4.0, 16.0 / nx, 8.0 / ny,
                          nx, ny, scheme=scheme, coarse=64, l1_kx=2, l1_ky=2, terms=terms)


def _series_error(oracle_lib, rect, nx, ny, terms, n=20000, seed=1):
    """|beta_interp - beta_direct| of lens-free maps: the sheet's series per
    level-2 cell against its closed form, ray by ray; also each ray's
    expansion point (the centre of its cell clipped to the lattice)."""
    gi, gd = _lattice(1, nx, ny, terms), _lattice(0, nx, ny, terms)
    oi = oracle_lib.Oracle(gi, 0.4, 0.1, 0.02, [], [], [], sheet=rect)
    od = oracle_lib.Oracle(gd, 0.4, 0.1, 0.02, [], [], [], sheet=rect)
    rng = np.random.default_rng(seed)
    ii, jj = rng.integers(0, nx, n), rng.integers(0, ny, n)
    bi, _ = oi.trace(ii, jj)
    bd, _ = od.trace(ii, jj)
    th = np.stack([gi.ray_x0 + (ii + 0.5) * gi.ray_dx, gi.ray_y0 + (jj + 0.5) * gi.ray_dy], 1)
    ci, cj = ii // 64, jj // 64
    ex = gi.ray_x0 + 0.5 * (ci * 64 + np.minimum((ci + 1) * 64, nx)) * gi.ray_dx
    ey = gi.ray_y0 + 0.5 * (cj * 64 + np.minimum((cj + 1) * 64, ny)) * gi.ray_dy
    return np.hypot(*(bi - bd).T), th, np.stack([ex, ey], 1)


def _remainder_bound(rect, th, ze, terms, ks=0.02):
    """Truncation bound of a P-term series of the rectangle's holomorphic
    part about z_e: its singularities are the corners, where it behaves as
    (kappa/pi) (z - corner) log(z - corner); with d the distance from z_e to
    the nearest corner and rho = |theta - z_e| / d the tail is below
    (kappa / pi) 4 d rho^P / (1 - rho)."""
    d = np.min([np.hypot(ze[:, 0] - x, ze[:, 1] - y) for x in rect[:2] for y in rect[2:]],
               axis=0)
    rho = np.hypot(*(th - ze).T) / d
    return ks / math.pi * 4.0 * d * rho ** terms / (1.0 - rho)


@pytest.mark.parametrize("terms", [4, 6])
def test_sheet_series_converges_to_the_closed_form(oracle_lib, terms):
    """Lens-free maps in the interpolated scheme carry the rectangle's
    holomorphic part by its P-term series per level-2 cell: against the
    direct scheme's closed form every ray is within the series' remainder
    bound, and two more terms shrink the error by about rho^2."""
    rect = (-40.0, 40.0, -30.0, 30.0)
    err, th, ze = _series_error(oracle_lib, rect, 640, 320, terms)
    bound = _remainder_bound(rect, th, ze, terms)
    assert (err <= bound + 1e-13).all()
    assert err.max() < (3e-7 if terms == 4 else 1e-9)


def test_sheet_series_in_partial_cells_and_at_the_lattice_edge(oracle_lib):
    """The rectangle is the lattice itself (as for lenses drawn in the
    shooting region) and the last column and row of level-2 cells are partial
    (700 x 330 rays, cells of 64): each cell's series is taken about the
    centre of its part of the lattice, so every ray stays within the
    remainder bound about that point, partial cells included."""
    rect = (-8.0, 8.0, -4.0, 4.0)
    err, th, ze = _series_error(oracle_lib, rect, 700, 330, 6, n=40000, seed=2)
    bound = _remainder_bound(rect, th, ze, 6)
    partial = (th[:, 0] > -8.0 + 640 * 16.0 / 700) | (th[:, 1] > -4.0 + 320 * 8.0 / 330)
    assert partial.sum() > 1000
    assert (err <= bound + 1e-13).all()
