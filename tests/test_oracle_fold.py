"""Pins of the oracle's fold macro model (Sec. 2 Eq. 5/6, Sec. 4.1, Table 1)."""
import json
import math
import os

import numpy as np

from oracle.geometry import derive_fold_geometry, fold_n_star

TABLE1 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table1.json")))
SEC4 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_sec4.json")))


def table1_d_per_theta_e():
    """d of Table 1 in 1/theta_E: arcmin^-1 times theta_E in arcmin."""
    te = TABLE1["theta_E_arcsec"] / 60.0
    return [v * te for v in TABLE1["d_arcmin_inv"]]


def test_table1_lens_count_from_the_fold_geometry():
    """The shooting region of the 200 x 40 theta_E^2 map (Sec. 4.1) with Table 1
    holds N_star = 13745 lenses (Table 1)."""
    dx, dy = table1_d_per_theta_e()
    lx, ly = SEC4["map_theta_E"][1], SEC4["map_theta_E"][0]  # 40 across, 200 along
    g = derive_fold_geometry(lx, ly, SEC4["N_pix"][1], SEC4["N_pix"][0], TABLE1["kappa0"], dx,
                             TABLE1["kappa_star"], n_rays=TABLE1["N_av"] * SEC4["N_pix"][0] *
                             SEC4["N_pix"][1])
    n_star = fold_n_star(g, TABLE1["kappa_star"])
    assert abs(n_star - TABLE1["N_star"]) < 2.0
    # the map pixel is the 5.5e-4 theta_E of Sec. 4.1 in both directions
    assert abs(g.src_dx / 5.5e-4 - 1) < 1e-3 and abs(g.src_dy / 5.5e-4 - 1) < 1e-3
    # Fig. 2: the map starts 20 sqrt(kappa_star) = 0.632456 below the caustic
    assert abs(g.src_x0 - SEC4["fig2_beta_x_low"]) < 1e-6
    # about 2.7e13 rays (Eq. 8), "about 1e13" in Sec. 4.1
    assert 2.6e13 < g.ray_nx * g.ray_ny < 2.8e13


def test_fold_macro_magnification_falls_as_inverse_sqrt(oracle_lib):
    """No lenses, no sheet, d_y = 0: two images at theta_x = +-sqrt(2 beta_x/d_x),
    so mu(beta_x) = 1/((1-kappa_0) sqrt(2 d_x beta_x)) for beta_x > 0 and no rays
    below the caustic; Sec. 4.1: the magnification decreases as 1/sqrt(beta_x)."""
    k0, dx = 0.83, 1.0e-3
    g = derive_fold_geometry(10.0, 10.0, 42, 8, k0, dx, 0.0, n_rays=2.0e7, margin=0.5,
                             scheme=0)
    o = oracle_lib.Oracle(g, 0, 0, 0.0, [], [], [], fold=(k0, dx, 0.0))
    counts, n_out = o.shoot(nthreads=4)
    mu = counts * o.mu_factor()
    a = g.src_x0 + np.arange(g.src_nx) * g.src_dx
    b = a + g.src_dx
    below = b <= 0
    assert np.all(counts[:, below] == 0)
    above = a >= 0
    avg = 2 * (np.sqrt(b[above]) - np.sqrt(a[above])) / (b[above] - a[above])
    expect = avg / ((1 - k0) * math.sqrt(2 * dx))
    inner = slice(1, None)  # the pixel at the caustic diverges; skip it
    rel = mu[:, above][:, inner] / expect[inner] - 1
    assert np.abs(rel).max() < 0.02
    assert abs(rel.mean()) < 2e-3


def test_fold_with_lenses_window_counts(oracle_lib):
    """Counting into a pixel window agrees with the full map."""
    rng = np.random.default_rng(8)
    k0, dx, dy = 0.83, 2.0e-3, -1.5e-3
    g = derive_fold_geometry(4.0, 4.0, 40, 40, k0, dx, 0.01, n_rays=1e6, coarse=64)
    x = rng.uniform(-g.ray_nx * g.ray_dx / 2, g.ray_nx * g.ray_dx / 2, 50)
    y = rng.uniform(-g.ray_ny * g.ray_dy / 2, g.ray_ny * g.ray_dy / 2, 50)
    o = oracle_lib.Oracle(g, 0, 0, 0.01, x, y, np.ones(50), fold=(k0, dx, dy))
    full, nf = o.shoot(nthreads=4)
    win, nw = o.shoot_window(0, 0, g.ray_nx, g.ray_ny, 7, 11, 20, 13, nthreads=4)
    np.testing.assert_array_equal(win, full[11:24, 7:27])
    assert nw == g.ray_nx * g.ray_ny - int(win.sum())


def test_fold_sheet_term_shifts_the_caustic(oracle_lib):
    """No lenses, sheet kappa_star, d_y = 0 (Eq. 6): beta_x = d_x u^2/2 - s with
    u = theta_x + kappa_star/d_x and s = kappa_star^2/(2 d_x), beta_y =
    (2(1-kappa_0) + kappa_star) theta_y, so mu = 2/(c_y sqrt(2 d_x (beta_x + s)))."""
    k0, dx, ks = 0.83, 1.0e-3, 0.01
    g = derive_fold_geometry(10.0, 10.0, 42, 8, k0, dx, ks, n_rays=2.0e7, margin=0.5,
                             scheme=0)
    o = oracle_lib.Oracle(g, 0, 0, ks, [], [], [], fold=(k0, dx, 0.0))
    counts, _ = o.shoot(nthreads=4)
    mu = counts * o.mu_factor()
    s = ks * ks / (2 * dx)
    cy = 2 * (1 - k0) + ks
    a = g.src_x0 + np.arange(g.src_nx) * g.src_dx + s
    b = a + g.src_dx
    assert np.all(counts[:, b <= 0] == 0)
    sel = (a > 0) & (b - s < 8.0)
    sel[np.argmax(sel)] = False  # skip the pixel at the caustic
    avg = 2 * (np.sqrt(b[sel]) - np.sqrt(a[sel])) / (b[sel] - a[sel])
    expect = 2 * avg / (cy * math.sqrt(2 * dx))
    rel = mu[:, sel] / expect - 1
    assert np.abs(rel).max() < 0.02
    assert abs(rel.mean()) < 2e-3
