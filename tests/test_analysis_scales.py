"""Analysis scales of Sec. 4 (kappa_c, s_w, s_f, N_cf, mu_peak): the library's
host function against the oracle's, and the oracle against Table 1."""
import json
import math
import os

import pytest

import paper_2308_14278_amd.lensmap as lm
from oracle.analysis import fold_scales, mu_peak

TABLE1 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table1.json")))


def test_kappa_c_matches_table1():
    """Table 1 prints kappa_c = 1.9e-5 for theta_E = 1e-6 arcsec and
    d = (3.62, -3.41) arcmin^-1."""
    s = fold_scales(TABLE1["theta_E_arcsec"], *TABLE1["d_arcmin_inv"], TABLE1["kappa0"],
                    TABLE1["kappa_star"], TABLE1["N_star"])
    assert abs(s["kappa_c"] / TABLE1["kappa_c"] - 1) < 0.01
    assert TABLE1["kappa_star"] / s["kappa_c"] > 50  # kappa_star >> kappa_c (Sec. 4.1)


def test_s_w_differs_from_the_printed_value():
    """Eq. 13 with Table 1 gives s_w = 33.1 theta_E; Sec. 4.2 prints 25.5 theta_E.
    The formula is implemented as printed; the stated value is not reproduced."""
    s = fold_scales(TABLE1["theta_E_arcsec"], *TABLE1["d_arcmin_inv"], TABLE1["kappa0"],
                    TABLE1["kappa_star"], TABLE1["N_star"])
    assert abs(s["s_w"] - 33.15) < 0.05
    assert abs(s["s_w"] - TABLE1["s_w_printed"]) > 5


def test_library_matches_oracle():
    for args in [(1e-6, 3.62, -3.41, 0.83, 0.001, 13745, 1e10),
                 (2e-6, 1.0, 2.0, 0.7, 0.003, 2000, 3e9),
                 (1e-6, -3.0, 0.5, 0.9, 0.0005, 50000, 0.0)]:
        o = fold_scales(*args[:6])
        got = lm.lm_fold_scales(*args)
        for k in o:
            assert math.isclose(got[k], o[k], rel_tol=1e-12), k
        if args[6] > 0:
            # Eq. 15 is continuous at |beta| = s_w and falls as |beta|^(-3/8) outside
            mp = mu_peak(*args[:5], args[6], 0.0, o["s_w"])
            assert math.isclose(got["mu_peak0"], mp, rel_tol=1e-12)
            out = mu_peak(*args[:5], args[6], 10 * o["s_w"], o["s_w"])
            assert math.isclose(out / mp, 10 ** (-0.375), rel_tol=1e-12)


def test_rejects_bad_input():
    with pytest.raises(lm.LensmapError):
        lm.lm_fold_scales(0.0, 3.62, -3.41, 0.83, 0.001, 13745)
    with pytest.raises(lm.LensmapError):
        lm.lm_fold_scales(1e-6, 0.0, -3.41, 0.83, 0.001, 13745)
