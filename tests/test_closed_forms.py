"""Pins of the closed-form theories against the paper's printed forms.

The oracle evaluates Jaffe's and Boag's expressions in overflow-free forms;
here each is checked against the expression as printed, evaluated through
scipy's special functions (exponential integral, Hankel and Bessel
functions), and against the limits the paper states."""
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sp

from oracle import closed_forms as cf

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.mark.parametrize("y1,y2", [(0.024, 0.667), (2.4, 0.667), (24.0, 0.667), (1.877, 3.1),
                                   (16.65, 0.9), (63.2, 12.0), (300.0, 0.05)])
def test_jaffe_parallel_matches_printed_ei_form(y1, y2):
    """eq. Jaffe_noangle as printed: (y1/y2) e^{-y1} [Ei(y1 + ln(1+y2)) - Ei(y1)]."""
    printed = y1 / y2 * math.exp(-y1) * (sp.expi(y1 + math.log1p(y2)) - sp.expi(y1))
    assert cf.jaffe_parallel_y(y1, y2) == pytest.approx(printed, rel=1e-11)


def test_jaffe_parallel_limits():
    # weak recombination (y1 -> inf): f -> 1; strong (y1 -> 0): f -> 0
    assert cf.jaffe_parallel_y(1e6, 0.5) == pytest.approx(1.0, abs=1e-6)
    assert cf.jaffe_parallel_y(1e-6, 0.5) < 1e-4
    # monotone in the field: larger E means smaller y2 and larger f
    fs = [cf.jaffe_parallel_y(5.0, y2) for y2 in (10.0, 3.0, 1.0, 0.3)]
    assert all(a < b for a, b in zip(fs[:-1], fs[1:]))


@pytest.mark.parametrize("Z", [1e-4, 0.03, 0.7, 4.0, 40.0, 300.0])
def test_scaled_k0_is_the_papers_hankel_expression(Z):
    """S(Z) = e^Z (i pi/2) H0^(1)(iZ), evaluated with scipy's complex Hankel
    function, equals the quadrature of e^Z K0(Z)."""
    hank = complex(math.exp(Z) * (1j * math.pi / 2) * sp.hankel1(0, 1j * Z))
    assert abs(hank.imag) < 1e-12 * abs(hank.real)
    assert cf.scaled_k0(Z) == pytest.approx(hank.real, rel=1e-11)


@pytest.mark.parametrize("Z", [1e-4, 0.7, 40.0, 700.0, 5e4])
def test_scaled_k0_matches_library(Z):
    # beyond Z ~ 700 the unscaled Hankel function underflows; k0e does not
    assert cf.scaled_k0(Z) == pytest.approx(sp.k0e(Z), rel=1e-11)


def test_jaffe_angle_increases_toward_perpendicular():
    D = 0.5 * (2.82e-2 + 4.35e-2)
    mu = 0.5 * (1.36 + 2.10)
    fs = [cf.jaffe_angle(0.115, 20e-4, 2000.0, th, D, mu, 1.6e-6) for th in
          (math.pi / 6, math.pi / 4, math.pi / 3, math.pi / 2)]
    assert all(a < b for a, b in zip(fs[:-1], fs[1:]))
    assert all(0.99 < f < 1.0 for f in fs)


def test_boag_models_reduce_to_two_voltage_method_at_p0():
    """All three free-electron models converge to f = ln(1+u)/u at p = 0
    (section on Boag's free-electron models)."""
    for u in (1e-3, 0.2, 1.0, 7.0, 40.0):
        fb = math.log(1 + u) / u
        assert cf.boag(u) == pytest.approx(fb, rel=1e-15)
        assert cf.boag_model1(u, 1e-12) == pytest.approx(fb, rel=1e-9)
        assert cf.boag_model2(u, 0.0) == pytest.approx(fb, rel=1e-14)
        assert cf.boag_model3(u, 1e-12) == pytest.approx(fb, rel=1e-9)


def test_boag_models_all_free_electrons_collect_everything():
    for u in (0.3, 3.0, 30.0):
        for m in (cf.boag_model1, cf.boag_model2, cf.boag_model3):
            assert m(u, 1.0) == pytest.approx(1.0, abs=1e-12)


def test_free_electron_fraction():
    assert cf.free_electron_fraction(0.0, 0.2) == 1.0
    assert cf.free_electron_fraction(10.0, 0.2) == pytest.approx((1 - math.exp(-2.0)) / 2.0, rel=1e-15)
    assert cf.free_electron_fraction(1e4, 1.0) == pytest.approx(1e-4, rel=1e-12)


def test_proton_initial_recombination_below_paper_claim():
    """Table I proton track with Table II constants in the 2 mm chamber: the
    paper states initial recombination below 0.1%."""
    t1, t2, claims = GOLDEN["table_I"], GOLDEN["table_II"], GOLDEN["claims"]
    D = 0.5 * (t2["D_pos_cm2_s"] + t2["D_neg_cm2_s"])
    mu = 0.5 * (t2["mu_pos_cm2_Vs"] + t2["mu_neg_cm2_Vs"])
    p = t1["p100"]
    for E in (500.0, 1000.0, 2000.0, 3000.0):
        f = cf.jaffe_parallel(p["let_keV_um"], p["b_um"] * 1e-4, E, claims["jaffe_gap_cm"], D, mu,
                              t2["alpha_cm3_s"])
        assert 1.0 - f < claims["proton_initial_recombination_below"]


def test_heavy_ions_recombine_more_than_protons():
    t1, t2 = GOLDEN["table_I"], GOLDEN["table_II"]
    D = 0.5 * (t2["D_pos_cm2_s"] + t2["D_neg_cm2_s"])
    mu = 0.5 * (t2["mu_pos_cm2_Vs"] + t2["mu_neg_cm2_Vs"])
    fs = {k: cf.jaffe_parallel(v["let_keV_um"], v["b_um"] * 1e-4, 2000.0, 0.2, D, mu, t2["alpha_cm3_s"])
          for k, v in t1.items()}
    assert fs["Fe40"] < fs["Ne60"] < fs["C90"] < fs["p100"]


@pytest.mark.parametrize("p", [0.1, 0.5, 0.9])
def test_boag_models_small_and_large_dose_expansions(p):
    """Expansions of the three free-electron models, worked out by hand from
    their formulas: at small u the loss is linear, 1 - f = k u / 2 with
    k = 1 - p (model 1), (1 - p)^2 (model 2), (1 - p)^(3/2) (model 3, whose
    lambda = 1 - sqrt(1 - p)); at large u only the free electrons survive,
    f -> p, with the first correction -ln(p)/u (model 1), ln((1 - p) u)/u
    (model 2) and -ln(lambda)/u (model 3)."""
    u = 1e-6
    for m, k in ((cf.boag_model1, 1 - p), (cf.boag_model2, (1 - p) ** 2), (cf.boag_model3, (1 - p) ** 1.5)):
        assert (1.0 - m(u, p)) / u == pytest.approx(k / 2, rel=1e-4)
    lam = 1.0 - math.sqrt(1.0 - p)
    u = 400.0 / p  # e^{p u} stays finite
    assert cf.boag_model1(u, p) - p == pytest.approx(-math.log(p) / u, rel=1e-6)
    u2 = 1e8  # model 2 has no exponential: a dose far out on the asymptote
    assert cf.boag_model2(u2, p) - p == pytest.approx(math.log((1 - p) * u2) / u2, rel=1e-6)
    assert cf.boag_model3(u, p) - p == pytest.approx(-math.log(lam) / u, rel=1e-6)
