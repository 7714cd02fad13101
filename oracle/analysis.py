"""Analysis scales of Sec. 4, written out plainly (oracle side).

TEST INFRASTRUCTURE: independent of the library's lm_fold_scales.

Inputs: Einstein radius theta_E in arcsec, d = -(grad kappa)_0 - (grad gamma)_0 in
arcmin^-1 (Eq. 4 and Table 1), kappa_0, kappa_star, the number of microlenses
N_star, and for the peak magnification the ratio D_s / R (source distance over
source radius, a free input).

  kappa_c = (theta_E |d|)^(2/3)                      (Sec. 4.1, Table 1 note)
  tan a = d_x / d_y                                   (Sec. 4.1, after Eq. 13)
  s_w = 2 theta_E / |sin a| kappa_c^(1/2) (kappa_star/kappa_c)^2          (Eq. 13)
  C_star = [ln(3.05 N_star^(1/2))]^(1/2),  s_f = C_star theta_E kappa_star^(1/2)  (Sec. 4.2)
  N_cf = (2 C_star / |sin a|)^(1/2) (kappa_star/kappa_c)^(3/4)           (Eq. 14)
  mu_peak = 1/|1-kappa_0| (D_s/(R |d|))^(1/2) (kappa_c/kappa_star)^(3/4)
            x (1 if |beta| < s_w else (s_w/|beta|)^(3/8))                (Eq. 15)

Lengths s_w and s_f are returned in units of theta_E (the factor theta_E is
the unit); |d| enters kappa_c as the dimensionless product theta_E |d| with
theta_E converted to arcmin.
"""
from __future__ import annotations

import math

ARCSEC_PER_ARCMIN = 60.0


def fold_scales(theta_e_arcsec, d_x, d_y, kappa0, kappa_star, n_star):
    d = math.hypot(d_x, d_y)
    kappa_c = (theta_e_arcsec / ARCSEC_PER_ARCMIN * d) ** (2.0 / 3.0)
    sin_a = abs(d_x) / d  # tan a = d_x / d_y
    ratio = kappa_star / kappa_c
    s_w = 2.0 / sin_a * math.sqrt(kappa_c) * ratio ** 2
    c_star = math.sqrt(math.log(3.05 * math.sqrt(n_star)))
    s_f = c_star * math.sqrt(kappa_star)
    n_cf = math.sqrt(2.0 * c_star / sin_a) * ratio ** 0.75
    return {"kappa_c": kappa_c, "sin_a": sin_a, "s_w": s_w, "c_star": c_star, "s_f": s_f,
            "n_cf": n_cf}


def mu_peak(theta_e_arcsec, d_x, d_y, kappa0, kappa_star, ds_over_r, beta, s_w):
    """Eq. 15 with |d| in arcmin^-1 and D_s/R dimensionless (|d| converted to
    per radian so that D_s / (R |d|) is dimensionless)."""
    d_per_rad = math.hypot(d_x, d_y) * (180.0 * 60.0 / math.pi)
    kappa_c = (theta_e_arcsec / ARCSEC_PER_ARCMIN * math.hypot(d_x, d_y)) ** (2.0 / 3.0)
    base = 1.0 / abs(1.0 - kappa0) * math.sqrt(ds_over_r / d_per_rad) * (kappa_c / kappa_star) ** 0.75
    b = abs(beta)
    return base if b < s_w else base * (s_w / b) ** 0.375
