"""Workload geometry from the paper's rules, written out plainly in FP64.

TEST INFRASTRUCTURE (part of the oracle): independent of the library's own
derivation, which the tests compare against this one.

Rules followed (Sec. 3.1 and Sec. 3.2):
  * protection zone: the source region s is widened by w = 10 sqrt(kappa_star)
    on every side (Sec. 3.1, the s' formula);
  * shooting (image) region: the preimage of s' under the mean macro map
    beta = diag(1-kappa-gamma, 1-kappa+gamma) theta (Eq. 1), centred on the
    origin: L_ix = L'_sx / |1-kappa-gamma|, L_iy = L'_sy / |1-kappa+gamma|;
  * lens count in the image region N_star = L_ix L_iy kappa_star / (pi <m>)
    (Sec. 3.1; <m> = 1 for unit masses) and L0 = sqrt(L_ix L_iy / N_star);
  * level-1 size L_1x = min(L0, L_ix/10) (Eq. 10), and likewise in y;
  * level-2 size L_2 = L_1 / 20 (Sec. 3.2.2);
  * level-3 (ray) spacing L3 = sqrt(L_ix L_iy / N_rays) (Eq. 11), with rays at
    level-3 pixel centres.

Discretisation choices (our reading, the paper leaves them open): the ray
counts are n_x = round(L_ix/L3), n_y = round(L_iy/L3) and the spacings are then
L_ix/n_x, L_iy/n_y so the lattice covers the region exactly; a level-2 cell is
an R x R block of rays with R a multiple of 64 (nearest to L_2/L3, at least 64)
and a level-1 cell is a Kx x Ky block of level-2 cells with
Kx = max(1, round(L_1x / (R L3x))), Ky likewise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass
class OracleGeometry:
    src_x0: float
    src_y0: float
    src_dx: float
    src_dy: float
    src_nx: int
    src_ny: int
    ray_x0: float
    ray_y0: float
    ray_dx: float
    ray_dy: float
    ray_nx: int
    ray_ny: int
    scheme: int = 0
    coarse: int = 64
    l1_kx: int = 1
    l1_ky: int = 1
    halo: int = 1
    terms: int = 4
    far_order: int = 0  # 0: direct level-2 coefficients; Q: hierarchical, Q terms

    @property
    def n_rays(self) -> int:
        return self.ray_nx * self.ray_ny


def _round_half_away(x: float) -> int:
    return int(math.floor(x + 0.5)) if x >= 0 else -int(math.floor(-x + 0.5))


def derive_geometry(src_lx, src_ly, src_nx, src_ny, kappa, gamma, kappa_star,
                    n_rays=None, ray_nx=None, ray_ny=None, protect=None, mean_mass=1.0,
                    scheme=1, coarse=0, halo=1, terms=4) -> OracleGeometry:
    """Derive the full geometry.  ``protect=None`` uses 10 sqrt(kappa_star);
    ``coarse=0`` applies the L2 = L1/20 rule; give either n_rays or (ray_nx, ray_ny)."""
    lt = 1.0 - kappa - gamma
    lr = 1.0 - kappa + gamma
    if lt == 0.0 or lr == 0.0:
        raise ValueError("the mean macro map is singular")
    w = 10.0 * math.sqrt(kappa_star) if protect is None else float(protect)
    lsx = src_lx + 2.0 * w
    lsy = src_ly + 2.0 * w
    lix = lsx / abs(lt)
    liy = lsy / abs(lr)
    if ray_nx is None:
        l3 = math.sqrt(lix * liy / float(n_rays))
        ray_nx = max(1, _round_half_away(lix / l3))
        ray_ny = max(1, _round_half_away(liy / l3))
    l3x = lix / ray_nx
    l3y = liy / ray_ny
    R, kx, ky = int(coarse), 1, 1
    if scheme == 1:
        if kappa_star > 0.0:
            n_star = lix * liy * kappa_star / (math.pi * mean_mass)
            l0 = math.sqrt(lix * liy / n_star)
        else:
            l0 = math.inf
        l1x = min(l0, lix / 10.0)
        l1y = min(l0, liy / 10.0)
        if R <= 0:
            l2 = min(l1x / 20.0 / l3x, l1y / 20.0 / l3y)
            R = 64 * max(1, _round_half_away(l2 / 64.0))
        kx = max(1, _round_half_away(l1x / (R * l3x)))
        ky = max(1, _round_half_away(l1y / (R * l3y)))
    elif R <= 0:
        R = 64
    return OracleGeometry(
        src_x0=-0.5 * src_lx, src_y0=-0.5 * src_ly,
        src_dx=src_lx / src_nx, src_dy=src_ly / src_ny, src_nx=int(src_nx), src_ny=int(src_ny),
        ray_x0=-0.5 * lix, ray_y0=-0.5 * liy, ray_dx=l3x, ray_dy=l3y,
        ray_nx=int(ray_nx), ray_ny=int(ray_ny),
        scheme=int(scheme), coarse=int(R), l1_kx=int(kx), l1_ky=int(ky), halo=int(halo),
        terms=int(terms))


def derive_fold_geometry(src_lx, src_ly, src_nx, src_ny, kappa0, d_x, kappa_star, n_rays,
                         margin=None, mean_mass=1.0, scheme=1, coarse=0, halo=1, terms=4):
    """Geometry of a map next to a fold caustic (Sec. 2 Eq. 5, Sec. 3.1, Sec. 4.1).

    The source window spans beta_x in [-margin, src_lx] across the caustic (the
    margin, 20 sqrt(kappa_star) by default, lies on the side without macro
    images and is part of the map, as in Fig. 2) and beta_y in
    [-src_ly/2, src_ly/2] along it.  The shooting region is the rectangle
    L_ix = 2 sqrt(2 (src_lx + margin) / d_x) (both images of Eq. 5 with d_y
    neglected), L_iy = src_ly / (2 (1 - kappa_0)), centred on the origin; with
    Table 1 this reproduces N_star = 13745.  Rays and grid levels follow the
    same rules as derive_geometry (Eq. 8, 10, 11)."""
    w = 20.0 * math.sqrt(kappa_star) if margin is None else float(margin)
    lsx = src_lx + w
    lix = 2.0 * math.sqrt(2.0 * lsx / abs(d_x))
    liy = src_ly / abs(2.0 * (1.0 - kappa0))
    l3 = math.sqrt(lix * liy / float(n_rays))
    ray_nx = max(1, _round_half_away(lix / l3))
    ray_ny = max(1, _round_half_away(liy / l3))
    l3x, l3y = lix / ray_nx, liy / ray_ny
    R, kx, ky = int(coarse), 1, 1
    if scheme == 1:
        l0 = math.sqrt(math.pi * mean_mass / kappa_star) if kappa_star > 0 else math.inf
        l1x, l1y = min(l0, lix / 10.0), min(l0, liy / 10.0)
        if R <= 0:
            l2 = min(l1x / 20.0 / l3x, l1y / 20.0 / l3y)
            R = 64 * max(1, _round_half_away(l2 / 64.0))
        kx = max(1, _round_half_away(l1x / (R * l3x)))
        ky = max(1, _round_half_away(l1y / (R * l3y)))
    elif R <= 0:
        R = 64
    return OracleGeometry(
        src_x0=-w, src_y0=-0.5 * src_ly, src_dx=lsx / src_nx, src_dy=src_ly / src_ny,
        src_nx=int(src_nx), src_ny=int(src_ny),
        ray_x0=-0.5 * lix, ray_y0=-0.5 * liy, ray_dx=l3x, ray_dy=l3y,
        ray_nx=int(ray_nx), ray_ny=int(ray_ny),
        scheme=int(scheme), coarse=int(R), l1_kx=int(kx), l1_ky=int(ky), halo=int(halo),
        terms=int(terms))


def fold_n_star(g: OracleGeometry, kappa_star, mean_mass=1.0):
    """Lenses in the shooting region, N_star = L_ix L_iy kappa_star / (pi <m>) (Sec. 3.1)."""
    return g.ray_nx * g.ray_dx * g.ray_ny * g.ray_dy * kappa_star / (math.pi * mean_mass)
