"""Seeded synthetic inputs: lens fields and workload descriptions.

This module is shared by the product path, the oracle-based tests and the
benchmark.  It holds none of the method's arithmetic: it draws lens positions
and masses, and it lists the raw numbers that describe each workload (macro
convergence and shear, star density, source region, pixels, ray budget and
scheme switches).  Geometry derivation, deflection, mapping and counting live
in the library (and, independently, in the oracle).

Recipe (all lengths in Einstein radii of a unit mass):
  * generator: numpy PCG64 seeded with 230814278 + 1000 * workload_id + map_index;
  * positions: uniform in a disk (r = R sqrt(u), phi = 2 pi v) or uniform in an
    axis-aligned rectangle centred on the origin;
  * masses: 1, or a Salpeter power law dN/dm ~ m^-2.35 on [0.08, 1.5] drawn by
    inverse CDF;
  * rectangle fields cover an area pi * N * <m> / kappa_star, so the stars'
    mean convergence equals kappa_star, with aspect ratio
    (1-kappa+gamma)/(1-kappa-gamma), i.e. elongated along the critical line
    like the shooting region;
  * the compensating sheet covers the lenses' rectangle (Workload.sheet).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 230814278
SALPETER = (0.08, 1.5, 2.35)


def seed_for(workload_id: int, map_index: int = 0) -> int:
    return SEED_BASE + 1000 * int(workload_id) + int(map_index)


def rng_for(workload_id: int, map_index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_for(workload_id, map_index)))


def salpeter_mean(lo=SALPETER[0], hi=SALPETER[1], slope=SALPETER[2]) -> float:
    """Mean mass of the truncated power law (closed form)."""
    a, b = 2.0 - slope, 1.0 - slope
    return ((hi ** a - lo ** a) / a) / ((hi ** b - lo ** b) / b)


def salpeter_masses(rng, n, lo=SALPETER[0], hi=SALPETER[1], slope=SALPETER[2]):
    u = rng.random(n)
    e = 1.0 - slope
    return (lo ** e + u * (hi ** e - lo ** e)) ** (1.0 / e)


def uniform_disk(rng, n, radius):
    u = rng.random(n)
    v = rng.random(n)
    r = radius * np.sqrt(u)
    phi = 2.0 * math.pi * v
    return r * np.cos(phi), r * np.sin(phi)


def uniform_rect(rng, n, half_x, half_y):
    x = (2.0 * rng.random(n) - 1.0) * half_x
    y = (2.0 * rng.random(n) - 1.0) * half_y
    return x, y


def field_rect(n, mean_mass, kappa_star, lam_t, lam_r):
    """Half-sides of the lens rectangle: area pi N <m> / kappa_star, aspect lam_r/lam_t."""
    area = math.pi * n * mean_mass / kappa_star
    aspect = abs(lam_r / lam_t)
    return 0.5 * math.sqrt(area * aspect), 0.5 * math.sqrt(area / aspect)


@dataclass
class Workload:
    """Raw description of one map.  Lenses are drawn by :meth:`lenses`."""
    name: str
    workload_id: int
    map_index: int
    kappa: float
    gamma: float
    kappa_star: float
    n_lenses: int
    src_side: float
    src_pixels: int
    n_rays: float | None = None
    ray_nx: int | None = None
    ray_ny: int | None = None
    protect: float | None = None      # None: 10 sqrt(kappa_star)
    scheme: int = 1                   # 0 direct, 1 interpolated
    coarse: int = 0                   # 0: paper rule L2 = L1/20
    masses: str = "salpeter"          # "unit" or "salpeter"
    disk_radius: float | None = None  # disk field instead of the rectangle
    fold: tuple | None = None         # (kappa_0, d_x, d_y) in 1/theta_E: fold macro model
    extra: dict = field(default_factory=dict)

    @property
    def lam_t(self):
        return 1.0 - self.kappa - self.gamma

    @property
    def lam_r(self):
        return 1.0 - self.kappa + self.gamma

    @property
    def mean_mass(self):
        return 1.0 if self.masses == "unit" else salpeter_mean()

    def sheet(self, rect=None):
        """The rectangle (x0, x1, y0, y1) the compensating sheet covers: that of
        the lenses (rect as for lenses()); None for a disk field, whose sheet is
        the infinite one (exact inside the disk)."""
        if self.disk_radius is not None:
            return None
        if rect is not None:
            hx, hy = rect
        else:
            hx, hy = field_rect(self.n_lenses, self.mean_mass, self.kappa_star, self.lam_t,
                                self.lam_r)
        return (-hx, hx, -hy, hy)

    def lenses(self, rect=None):
        """Draw the lens field.  rect = (half_x, half_y) places the lenses in that
        rectangle (e.g. the shooting region, as for the fold workload) instead of
        the area rule."""
        rng = rng_for(self.workload_id, self.map_index)
        n = self.n_lenses
        if self.disk_radius is not None:
            x, y = uniform_disk(rng, n, self.disk_radius)
        else:
            if rect is not None:
                hx, hy = rect
            else:
                hx, hy = field_rect(n, self.mean_mass, self.kappa_star, self.lam_t, self.lam_r)
            x, y = uniform_rect(rng, n, hx, hy)
        m = np.ones(n) if self.masses == "unit" else salpeter_masses(rng, n)
        return np.ascontiguousarray(x), np.ascontiguousarray(y), np.ascontiguousarray(m)


def _kg(lam_t, lam_r):
    """(kappa, gamma) from the two eigenvalues of the macro Jacobian."""
    return 1.0 - 0.5 * (lam_t + lam_r), 0.5 * (lam_r - lam_t)


def plain_small() -> Workload:
    """100 unit lenses in a disk of radius 30; kappa=0.45, gamma=0.5, kappa_star=0.01;
    4096 x 4096 rays over the preimage of a 10 x 10 source square; 256^2 map; direct sum."""
    return Workload("plain-small", 1, 0, 0.45, 0.5, 0.01, 100, 10.0, 256,
                    ray_nx=4096, ray_ny=4096, protect=0.0, scheme=0, coarse=64,
                    masses="unit", disk_radius=30.0)


def near_fold() -> Workload:
    """2000 Salpeter lenses; Jacobian diag(0.01, 0.33); kappa_star=0.005; 1e11 rays;
    2000^2 map over 20 x 20; interpolated, 64 x 64-ray level-2 cells."""
    k, g = _kg(0.01, 0.33)
    return Workload("near-fold", 2, 0, k, g, 0.005, 2000, 20.0, 2000, n_rays=1e11,
                    scheme=1, coarse=64)


def paper_scale() -> Workload:
    """13000 Salpeter lenses; lambda_t=0.005, lambda_r=0.3; kappa_star=0.01; 1e13 rays;
    5000^2 map over 24 x 24 (side chosen so the lens field is ~1.35x the shooting
    region per side, as in near_fold); interpolated with the L2 = L1/20 rule."""
    k, g = _kg(0.005, 0.3)
    return Workload("paper-scale", 3, 0, k, g, 0.01, 13000, 24.0, 5000, n_rays=1e13,
                    scheme=1, coarse=0)


def precision_stress() -> Workload:
    """20000 Salpeter lenses; lambda_t=0.001 (macro mu ~ 3300); kappa_star=0.01;
    4e12 rays; 4000^2 map over 12.5 x 12.5; interpolated, L2 = L1/20 rule."""
    k, g = _kg(0.001, 0.3)
    return Workload("precision-stress", 5, 0, k, g, 0.01, 20000, 12.5, 4000, n_rays=4e12,
                    scheme=1, coarse=0)


def batched_study(n_maps: int = 80, rays_scale: float = 1.0) -> list[Workload]:
    """80 independent maps: N ~ U[2000, 20000], lambda_t ~ logU[0.002, 0.05],
    lambda_r = 0.3, kappa_star ~ U[0.002, 0.02], rays ~ logU[1e11, 1e12] (times
    rays_scale); 2000^2 maps whose side makes the lens field ~1.35x the shooting
    region per side."""
    rng = rng_for(4, 999)
    out = []
    mm = salpeter_mean()
    for m in range(n_maps):
        n = int(rng.integers(2000, 20001))
        lam_t = math.exp(rng.uniform(math.log(0.002), math.log(0.05)))
        lam_r = 0.3
        ks = float(rng.uniform(0.002, 0.02))
        rays = math.exp(rng.uniform(math.log(1e11), math.log(1e12))) * rays_scale
        w = 10.0 * math.sqrt(ks)
        side2 = lam_t * lam_r * math.pi * n * mm / (ks * 1.35 ** 2)
        side = max(1.0, round(math.sqrt(side2) - 2.0 * w, 2))
        k, g = _kg(lam_t, lam_r)
        out.append(Workload("batched-%02d" % m, 4, m, k, g, ks, n, side, 2000, n_rays=rays,
                            scheme=1, coarse=0))
    return out


# Table 1 of the paper: theta_E = 1e-6 arcsec = 1e-6/60 arcmin, d in arcmin^-1.
TABLE1_THETA_E_ARCMIN = 1e-6 / 60.0
TABLE1_D = (3.62 * TABLE1_THETA_E_ARCMIN, -3.41 * TABLE1_THETA_E_ARCMIN)


def paper_table1(n_rays: float = 1000.0 * 363635 * 73877) -> Workload:
    """The paper's own map (Sec. 4.1, Table 1): fold model with kappa_0 = 0.83 and
    d = (3.62, -3.41) arcmin^-1 at theta_E = 1e-6 arcsec, kappa_star = 0.001,
    13745 unit lenses uniform in the shooting region, a 40 x 200 theta_E^2 map
    (across x along the caustic) of 73877 x 363635 pixels, N_av = 1000
    (2.69e13 rays).  Lenses: call lenses(rect=...) with the shooting region."""
    return Workload("paper-table1", 6, 0, 0.83, 0.0, 0.001, 13745, 40.0, 73877,
                    n_rays=n_rays, scheme=1, coarse=0, masses="unit",
                    fold=(0.83, TABLE1_D[0], TABLE1_D[1]),
                    extra={"src_ly": 200.0, "src_ny": 363635})


def fold_study(n_maps: int = 80, pixel: float = 0.011, src_ly: float = 40.0,
               n_av: float = 1000.0) -> list[Workload]:
    """Independent realisations of the paper's lens field near the fold (Table 1
    physics: kappa_0 = 0.83, d = (3.62, -3.41) arcmin^-1 at theta_E = 1e-6
    arcsec, kappa_star = 0.001, unit masses) for the peak statistics of
    Sec. 4.2: each map spans the paper's 40 theta_E across the caustic (plus
    the 20 sqrt(kappa_star) margin) and src_ly along it, in pixels of `pixel`
    theta_E (20x the paper's 5.5e-4 by default), with N_av rays per pixel as in
    the paper.  Lenses: call lenses(rect=...) with the shooting region; their
    number is Table 1's N_star = 13745 for 200 theta_E along the caustic,
    scaled to src_ly (the region's width across the caustic is the paper's)."""
    margin = 20.0 * math.sqrt(0.001)
    nx = int(round((40.0 + margin) / pixel))
    ny = int(round(src_ly / pixel))
    n = int(round(13745 * src_ly / 200.0))
    return [Workload("fold-study-%02d" % m, 7, m, 0.83, 0.0, 0.001, n, 40.0, nx,
                     n_rays=n_av * nx * ny, scheme=1, coarse=0, masses="unit",
                     fold=(0.83, TABLE1_D[0], TABLE1_D[1]),
                     extra={"src_ly": src_ly, "src_ny": ny})
            for m in range(n_maps)]


WORKLOADS = {
    "plain-small": plain_small,
    "near-fold": near_fold,
    "paper-scale": paper_scale,
    "precision-stress": precision_stress,
}
