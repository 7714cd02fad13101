"""Pins of the oracle's geometry rules (Sec. 3.1, Sec. 3.2, Eq. 8, 10, 11) against
numbers the paper prints in Sec. 4.1 and Table 1."""
import json
import math
import os

import pytest

from oracle.geometry import derive_geometry

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_sec4.json")))


def test_protection_zone_width_matches_fig2():
    """s' adds 10 sqrt(kappa_star) per side (Sec. 3.1); with Table 1's kappa_star
    the total widening 20 sqrt(kappa_star) is the 0.632456 of the Fig. 2 range."""
    ks = GOLD["kappa_star"]
    g = derive_geometry(10.0, 10.0, 10, 10, 0.83, 0.16, ks, n_rays=1e6, scheme=0)
    lix = g.ray_nx * g.ray_dx
    widened = lix * abs(1 - 0.83 - 0.16) - 10.0
    assert abs(widened - (-GOLD["fig2_beta_x_low"])) < 1e-6


def test_pixel_size_and_ray_budget():
    """The printed pixel counts give one pixel size in both directions once the
    protection margin is included (5.5e-4 theta_E), and Eq. 8 with N_av = 1000
    gives ~2.7e13 rays, the 'about 1e13' of Sec. 4.1."""
    lx, ly = GOLD["map_theta_E"]
    nx, ny = GOLD["N_pix"]
    margin = -GOLD["fig2_beta_x_low"]
    px, py = lx / nx, (ly + margin) / ny
    assert abs(px / py - 1) < 1e-4
    n_rays = GOLD["N_av"] * nx * ny
    assert 1e13 <= n_rays < 1e14
    assert round(math.log10(n_rays)) == round(math.log10(GOLD["rays_quoted"]))


@pytest.mark.parametrize("lt,lr,ks,side,rays", [(0.005, 0.3, 0.01, 24.0, 1e13),
                                                (0.01, 0.33, 0.005, 20.0, 1e11),
                                                (0.3, 0.5, 0.05, 40.0, 1e7)])
def test_grid_levels_follow_eq10_eq11(lt, lr, ks, side, rays):
    """Level-3 spacing L3 = sqrt(Lix Liy / N_rays) (Eq. 11); level-1 size
    min(L0, Li/10) (Eq. 10); level-2 = level-1 / 20 (Sec. 3.2.2), up to the
    rounding of cells to whole blocks of rays."""
    kappa, gamma = 1 - 0.5 * (lt + lr), 0.5 * (lr - lt)
    mm = 0.2
    g = derive_geometry(side, side, 100, 100, kappa, gamma, ks, n_rays=rays, mean_mass=mm,
                        scheme=1, coarse=0)
    w = 10 * math.sqrt(ks)
    lix, liy = (side + 2 * w) / lt, (side + 2 * w) / lr
    assert abs(g.ray_nx * g.ray_dx / lix - 1) < 1e-12
    assert abs(g.ray_ny * g.ray_dy / liy - 1) < 1e-12
    l3 = math.sqrt(lix * liy / rays)
    assert abs(g.ray_dx / l3 - 1) < 2.0 / min(g.ray_nx, g.ray_ny) + 1e-9
    assert abs(g.ray_nx * g.ray_ny / rays - 1) < 4.0 / min(g.ray_nx, g.ray_ny)
    l0 = math.sqrt(math.pi * mm / ks)          # sqrt(Lix Liy / N_star)
    l1x, l1y = min(l0, lix / 10), min(l0, liy / 10)
    l2 = g.coarse * g.ray_dx
    assert g.coarse % 64 == 0
    assert abs(l2 - min(l1x, l1y) / 20) <= 32 * g.ray_dx + 1e-12 or g.coarse == 64
    assert abs(g.l1_kx - l1x / l2) <= 0.5 + 1e-9 or (g.l1_kx == 1 and l1x / l2 < 1)
    assert abs(g.l1_ky - l1y / (g.coarse * g.ray_dy)) <= 0.5 + 1e-9 or g.l1_ky == 1
