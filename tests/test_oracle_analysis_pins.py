"""Pins of the oracle's analysis scales (oracle/analysis.py) against things
other than its own formulas: hand-evaluated Table 1 numbers, an identity that
ties Eq. 13, Eq. 14 and the s_f definition together, and the scaling laws the
three formulas imply (each exponent is checked by how the output moves when
one input is scaled)."""
import json
import math
import os

import pytest

from oracle.analysis import fold_scales, mu_peak

HAND = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_scales.json")))
T1 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table1.json")))

CASES = [(1e-6, 3.62, -3.41, 0.83, 0.001, 13745),
         (2e-6, 1.0, 2.0, 0.7, 0.003, 2000),
         (5e-7, -3.0, 0.5, 0.9, 0.0005, 50000),
         (1e-6, 0.4, 4.0, 0.6, 0.02, 800)]


def _t1():
    return fold_scales(T1["theta_E_arcsec"], *T1["d_arcmin_inv"], T1["kappa0"], T1["kappa_star"],
                       T1["N_star"])


@pytest.mark.parametrize("key", ["kappa_c", "sin_a", "s_w", "c_star", "s_f", "n_cf"])
def test_table1_hand_values(key):
    """Every scale at Table 1's parameters equals the hand evaluation."""
    hand_key = {"c_star": "C_star", "n_cf": "N_cf"}.get(key, key)
    want = HAND[hand_key][0]
    assert abs(_t1()[key] / want - 1.0) < 2e-5, (key, _t1()[key], want)


@pytest.mark.parametrize("case", CASES)
def test_ncf_identity(case):
    """N_cf^2 = C_star^2 s_w / s_f: with Eq. 13 (s_w ~ kappa_c^(1/2)
    (kappa_star/kappa_c)^2 / |sin a|), s_f = C_star kappa_star^(1/2) and Eq. 14
    (N_cf^2 = 2 C_star / |sin a| (kappa_star/kappa_c)^(3/2)) the powers of
    kappa_star, kappa_c, C_star and sin a cancel exactly; a slip in any one of
    the three exponents breaks it."""
    s = fold_scales(*case)
    assert math.isclose(s["n_cf"] ** 2, s["c_star"] ** 2 * s["s_w"] / s["s_f"], rel_tol=1e-12)


@pytest.mark.parametrize("case", CASES)
def test_scaling_laws(case):
    """Exponents, one input at a time: kappa_c ~ (theta_E |d|)^(2/3);
    s_w ~ kappa_star^2 at fixed kappa_c and ~ kappa_c^(-3/2) at fixed kappa_star
    (|d| scaled by 8 multiplies kappa_c by 4); s_f ~ kappa_star^(1/2);
    N_cf ~ kappa_star^(3/4); the orientation enters only through |sin a|."""
    th, dx, dy, k0, ks, n = case
    s = fold_scales(*case)
    s_d8 = fold_scales(th, 8 * dx, 8 * dy, k0, ks, n)
    assert math.isclose(s_d8["kappa_c"] / s["kappa_c"], 4.0, rel_tol=1e-12)
    assert math.isclose(s_d8["s_w"] / s["s_w"], 4.0 ** -1.5, rel_tol=1e-12)
    s_th = fold_scales(8 * th, dx, dy, k0, ks, n)
    assert math.isclose(s_th["kappa_c"] / s["kappa_c"], 4.0, rel_tol=1e-12)
    s_k4 = fold_scales(th, dx, dy, k0, 4 * ks, n)
    assert math.isclose(s_k4["s_w"] / s["s_w"], 16.0, rel_tol=1e-12)
    assert math.isclose(s_k4["s_f"] / s["s_f"], 2.0, rel_tol=1e-12)
    assert math.isclose(s_k4["n_cf"] / s["n_cf"], 4.0 ** 0.75, rel_tol=1e-12)
    # rotating d by 90 degrees swaps |sin a| and |cos a|
    s_rot = fold_scales(th, -dy, dx, k0, ks, n)
    ca = abs(dy) / math.hypot(dx, dy)
    assert math.isclose(s_rot["sin_a"], ca, rel_tol=1e-12)
    assert math.isclose(s_rot["s_w"] * ca, s["s_w"] * s["sin_a"], rel_tol=1e-12)
    # C_star depends on N_star alone: C_star^2 = ln 3.05 + ln(N_star)/2
    s_n = fold_scales(th, dx, dy, k0, ks, n * 100)
    assert math.isclose(s_n["c_star"] ** 2 - s["c_star"] ** 2, math.log(10.0), rel_tol=1e-12)
    # kappa_0 plays no part in these scales
    assert fold_scales(th, dx, dy, 0.5 * k0, ks, n) == s


@pytest.mark.parametrize("case", CASES)
def test_mu_peak_prefactor_closed_form(case):
    """Eq. 15's prefactor with |d| per radian: (kappa_c/kappa_star)^(3/4) grows as
    |d|^(1/2) and (D_s/(R |d|))^(1/2) falls as |d|^(-1/2), so the prefactor is
    sqrt((D_s/R) theta_E[rad]) / (|1 - kappa_0| kappa_star^(3/4)), independent
    of d (the familiar 1/sqrt(source size) law of a fold caustic)."""
    th, dx, dy, k0, ks, _ = case
    dsr = 3e9
    th_rad = th / 3600.0 * math.pi / 180.0
    want = math.sqrt(dsr * th_rad) / (abs(1.0 - k0) * ks ** 0.75)
    got = mu_peak(th, dx, dy, k0, ks, dsr, 0.0, 1.0)
    assert math.isclose(got, want, rel_tol=1e-12)
    assert math.isclose(mu_peak(th, 5 * dx, 5 * dy, k0, ks, dsr, 0.0, 1.0), got, rel_tol=1e-12)
    assert math.isclose(mu_peak(th, dx, dy, k0, ks, 4 * dsr, 0.0, 1.0) / got, 2.0, rel_tol=1e-12)


def test_mu_peak_table1_hand_value():
    got = mu_peak(T1["theta_E_arcsec"], *T1["d_arcmin_inv"], T1["kappa0"], T1["kappa_star"],
                  1e10, 0.0, 1.0)
    assert abs(got / HAND["mu_peak0_ds_over_r_1e10"][0] - 1.0) < 2e-5


def test_mu_peak_distance_law():
    """Inside the band the prefactor holds; outside it falls as (s_w/|beta|)^(3/8):
    continuous at s_w, 10x farther -> 10^(-3/8), and symmetric in the sign of beta."""
    args = (1e-6, 3.62, -3.41, 0.83, 0.001, 1e10)
    sw = 33.0
    inner = mu_peak(*args, 0.5 * sw, sw)
    assert inner == mu_peak(*args, 0.0, sw)
    assert math.isclose(mu_peak(*args, sw * (1 + 1e-12), sw), inner, rel_tol=1e-9)
    assert math.isclose(mu_peak(*args, 10 * sw, sw) / inner, 10 ** -0.375, rel_tol=1e-12)
    assert mu_peak(*args, -10 * sw, sw) == mu_peak(*args, 10 * sw, sw)
