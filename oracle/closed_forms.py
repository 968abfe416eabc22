"""Analytic recombination theories quoted by the paper -- TEST INFRASTRUCTURE.

These closed forms pin the CPU oracle (they are never used by the product
path).  Each evaluates the paper's expression in a form that stays finite in
FP64 over the whole parameter range; the tests check every rewritten form
against the printed one (through scipy's special functions) where both can be
evaluated.

* ``jaffe_parallel``  -- initial recombination in one Gaussian track parallel
  to the field, eq. Jaffe_noangle.
* ``jaffe_angle``     -- the same for a track at angle theta, eq. angle.
* ``boag``            -- pulsed general recombination, f = ln(1+u)/u, which all
  three free-electron models reduce to at p = 0 (section "Comparison with
  Boag's free-electron models").
* ``boag_model1/2/3`` and ``free_electron_fraction`` -- eqs. model1-3 and
  free_elec.
"""
from __future__ import annotations

import math

import numpy as np

_GL_CACHE = {}


def _gauss_legendre(n):
    if n not in _GL_CACHE:
        _GL_CACHE[n] = np.polynomial.legendre.leggauss(n)
    return _GL_CACHE[n]


def _integrate(fun, a, b, n=64, pieces=16):
    """Composite Gauss-Legendre quadrature of a smooth integrand on [a, b]."""
    x, w = _gauss_legendre(n)
    edges = np.linspace(a, b, pieces + 1)
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        half = 0.5 * (hi - lo)
        mid = 0.5 * (hi + lo)
        total += half * float(np.dot(w, fun(mid + half * x)))
    return total


def jaffe_y(let_keV_um, b_cm, E_V_cm, gap_cm, D, mu, alpha, W_eV=34.0):
    """Jaffe's parameters y1 = 8 pi D/(alpha N0) and y2 = 2 d D/(mu b^2 E),
    with N0 = LET/W the linear ion-pair density (eq. linear_density)."""
    N0 = let_keV_um * 1e7 / W_eV
    y1 = 8.0 * math.pi * D / (alpha * N0)
    y2 = 2.0 * gap_cm * D / (mu * b_cm * b_cm * E_V_cm)
    return y1, y2


def jaffe_parallel_y(y1, y2):
    """f_par = (y1/y2) e^{-y1} [Ei(y1 + ln(1+y2)) - Ei(y1)].

    Ei(b) - Ei(a) = int_a^b e^t/t dt.  With t = y1 + s and then
    s = y1 (e^w - 1) the bracket times e^{-y1} becomes
    int_0^{ln(1 + ln(1+y2)/y1)} exp(y1 (e^w - 1)) dw, whose integrand is
    smooth and bounded by 1 + y2, so no overflow occurs for large y1."""
    L = math.log1p(y2)
    upper = math.log1p(L / y1)
    integral = _integrate(lambda w: np.exp(y1 * np.expm1(w)), 0.0, upper)
    return y1 / y2 * integral


def jaffe_parallel(let_keV_um, b_cm, E_V_cm, gap_cm, D, mu, alpha, W_eV=34.0):
    return jaffe_parallel_y(*jaffe_y(let_keV_um, b_cm, E_V_cm, gap_cm, D, mu, alpha, W_eV))


def scaled_k0(Z):
    """S(Z) = e^Z (i pi/2) H0^(1)(iZ) = e^Z K0(Z) = int_0^inf e^{-Z (cosh t - 1)} dt."""
    if Z <= 0.0:
        return math.inf
    # the integrand is below e^{-745} (FP64 underflow) beyond t_max
    t_max = math.acosh(1.0 + 745.0 / Z)
    return _integrate(lambda t: np.exp(-Z * (np.cosh(t) - 1.0)), 0.0, t_max, n=64, pieces=64)


def jaffe_angle_z(y1, Z):
    return 1.0 / (1.0 + scaled_k0(Z) / y1)


def jaffe_angle(let_keV_um, b_cm, E_V_cm, theta, D, mu, alpha, W_eV=34.0):
    """f_theta = (1 + S(Z)/y1)^{-1}, Z = (mu b E sin(theta) / (2D))^2  (eq. angle)."""
    N0 = let_keV_um * 1e7 / W_eV
    y1 = 8.0 * math.pi * D / (alpha * N0)
    Z = (mu * b_cm * E_V_cm * math.sin(theta) / (2.0 * D)) ** 2
    return jaffe_angle_z(y1, Z)


def boag_u(n0, gap_cm, voltage, mu_pos, mu_neg, alpha):
    """u = alpha/(mu+ + mu-) * n d^2 / V."""
    return alpha / (mu_pos + mu_neg) * n0 * gap_cm * gap_cm / voltage


def boag(u):
    """Two-voltage-method collection efficiency f = ln(1+u)/u."""
    if u == 0.0:
        return 1.0
    return math.log1p(u) / u


def free_electron_fraction(a, d):
    """p = (1 - e^{-a d}) / (a d)  (eq. free_elec)."""
    x = a * d
    return 1.0 if x == 0.0 else -math.expm1(-x) / x


def boag_model1(u, p):
    return math.log1p(math.expm1(p * u) / p) / u


def boag_model2(u, p):
    return p + math.log1p((1.0 - p) * u) / u


def boag_model3(u, p):
    lam = 1.0 - math.sqrt(1.0 - p)
    return lam + math.log1p(math.expm1(lam * (1.0 - lam) * u) / lam) / u
