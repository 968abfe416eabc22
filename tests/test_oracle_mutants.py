"""The oracle's pins catch plausible mistakes in it.

Each case compiles a copy of ``oracle/oracle.c`` with one mistake planted
(a one-line slip: a dropped factor, a flipped sign, a wrong index or
neighbour, a unit slip), loads that copy in place of the oracle for the
length of the case, and requires every pin named for the mistake to fail.
The same pins pass on the oracle itself (the control case, and the pin
files).  Nothing here touches the committed oracle or its built library.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_electron_phase as PE
import test_oracle_pins as P
import test_oracle_pulse_train as PT

SRC = os.path.join(os.path.dirname(os.path.abspath(oracle.__file__)), "oracle.c")


def dense(orc):
    P.test_one_step_matches_dense_matrix_scheme(orc, (4, 4, 5))


def dense_absorbing(orc):
    P.test_absorbing_step_matches_dense_matrix_scheme(orc, (4, 4, 5))


def dense_absorbing_sc(orc):
    P.test_absorbing_step_with_space_charge_matches_dense_matrix_scheme(orc, (4, 4, 5))


def diffusion_moments(orc):
    P.test_pure_diffusion_moments_exact(orc)


def drift_moments(orc):
    P.test_drift_diffusion_moments_exact(orc)


def dt_value(orc):
    P.test_dt_single_track_value(orc)


def released_count(orc):
    P.test_released_count_matches_poisson_summation(orc, 1.0, 0.37)


def released_count_wide(orc):
    # a track as wide as the cell: the lattice sum sees the periodic images
    P.test_released_count_matches_poisson_summation(orc, 5.0, 0.0)


def gaussian_profile(orc):
    P.test_deposit_profile_is_gaussian_in_perpendicular_distance(orc)


def space_charge_map(orc):
    P.test_space_charge_pointwise_map(orc)


def absorbing_balance(orc):
    P.test_absorbing_conservation_and_escape(orc)


def boag(orc):
    P.test_boag_pulsed_general_recombination(orc, 1.0)


def stop_rule(orc):
    P.test_stop_rule_first_step_below_tolerance_after_the_last_deposit(orc)


def reaction_limit(orc):
    P.test_reaction_limit_single_track(orc)


def space_charge_dt(orc):
    P.test_space_charge_dt_bound(orc)


def electron_split(orc):
    P.test_free_electron_initial_split(orc)


def electron_split_field(orc):
    P.test_free_electron_split_field_node_by_node(orc)


def deposit_step(orc):
    P.test_track_deposited_at_floor_of_time_over_dt(orc)


def tilted_profile(orc):
    P.test_deposit_profile_is_gaussian_in_perpendicular_distance(orc)


def separate_radii(orc):
    P.test_separate_radii_conservation_and_released(orc)


def absorbing_deposit(orc):
    P.test_absorbing_deposit_is_the_unwrapped_profile(orc)


def absorbing_eigenmode(orc):
    P.test_absorbing_pure_diffusion_eigenmode(orc)


def electron_dense(orc):
    PE.test_electron_step_matches_dense_matrix_scheme(orc, (4, 4, 5))


def electron_dt_drift(orc):
    PE.test_electron_dt_pure_drift_is_one_cell_per_step(orc)


def electron_dt_diffusion(orc):
    PE.test_electron_dt_pure_diffusion_closed_form(orc)


def train_periods(orc):
    PT.test_train_steps_whole_periods(orc)


def train_superposition(orc):
    PT.test_superposition_without_recombination(orc, 0)


# name: (text in oracle.c, its replacement, occurrence to change, pins that must fail)
MUTANTS = {
    "x diffusion weight halved": (
        "w[1] = D * dt / (p[P_DX] * p[P_DX]);", "w[1] = 0.5 * D * dt / (p[P_DX] * p[P_DX]);", 1,
        [dense, diffusion_moments]),
    "negative ions drift with the positive ones": (
        "const double v = s == 0 ? mu * E : -mu * E;", "const double v = s == 0 ? mu * E : mu * E;", 1,
        [dense, drift_moments]),
    "upwind difference taken on the downwind side": (
        "const double drift = c * (c * (nc - n[IDX(k - 1, j, i)])",
        "const double drift = c * (c * (n[IDX(k + 1, j, i)] - nc)", 1,
        [dense, drift_moments]),
    "z Laplacian reads the upper neighbour twice": (
        "const double lap_z = n[IDX(k + 1, j, i)] - 2.0 * nc + n[IDX(k - 1, j, i)];",
        "const double lap_z = n[IDX(k + 1, j, i)] - 2.0 * nc + n[IDX(k + 1, j, i)];", 1,
        [dense, drift_moments]),
    "recombination sink halved": (
        "const double sink = beta * np_ * nn_;", "const double sink = 0.5 * beta * np_ * nn_;", 1,
        [dense, boag]),
    "anode weight with the drift term's sign flipped": (
        "const double w_up = sz + 0.5 * c * c - 0.5 * c;", "const double w_up = sz + 0.5 * c * c + 0.5 * c;", 1,
        [dense]),
    "von Neumann diffusion term without its factor 2": (
        "const double A = 2.0 * Ds[s] * inv2;", "const double A = Ds[s] * inv2;", 1,
        [dt_value]),
    "LET unit slip (keV/um taken as 0.1 keV/um)": (
        "const double N0 = tr[0] * 1.0e7 / p[P_W]; /* keV/um", "const double N0 = tr[0] * 1.0e6 / p[P_W]; /* keV/um", 1,
        [released_count]),
    "Gaussian exponent with 2 b^2": (
        "return N0 / (M_PI * b * b) * exp(-r2 / (b * b));", "return N0 / (M_PI * b * b) * exp(-r2 / (2.0 * b * b));", 1,
        [released_count, gaussian_profile]),
    "periodic offset wrapped to [0, L) instead of the nearest image": (
        "return d - L * floor(d / L + 0.5);", "return d - L * floor(d / L);", 1,
        [released_count_wide]),
    "space-charge term with the wrong sign": (
        "const double gsc[2] = {-sc_on * p[P_MU_POS]", "const double gsc[2] = {sc_on * p[P_MU_POS]", 1,
        [space_charge_map, dense_absorbing_sc]),
    "escape through the y sides not tallied": (
        "escaped[s] += (sx * miss_x + sy * miss_y) * nc;", "escaped[s] += sx * miss_x * nc;", 1,
        [dense_absorbing, absorbing_balance]),
    "stop test on the signed in-flight sums": (
        "tally[T_POS_ABS] <= p[P_STOP_TOL] * released &&\n        tally[T_NEG_ABS] <= p[P_STOP_TOL] * released_neg)",
        "tally[T_POS_INFLIGHT] <= p[P_STOP_TOL] * released &&\n        tally[T_NEG_INFLIGHT] <= p[P_STOP_TOL] * released_neg)", 1,
        [stop_rule]),
    "stop test before the last deposit": (
        "if (!train && l >= last_deposit && tally[T_POS_ABS]", "if (!train && tally[T_POS_ABS]", 1,
        [stop_rule]),
    "reaction bound twice as loose": (
        "const double dtr = rho / (rate * nref);", "const double dtr = 2.0 * rho / (rate * nref);", 1,
        [reaction_limit]),
    "reaction bound without the screening rate": (
        "rate += mu_max * Q_E / EPS0;", "rate += 0.0 * mu_max * Q_E / EPS0;", 1,
        [space_charge_dt]),
    "attachment measured from the cathode": (
        "const double att = -expm1(-p[P_ATTACH] * (double)k * dz);",
        "const double att = -expm1(-p[P_ATTACH] * (double)(nz - k) * dz);", 1,
        [electron_split_field]),
    "free fraction without its 1/(a d)": (
        "return x == 0.0 ? 1.0 : -expm1(-x) / x;", "return x == 0.0 ? 1.0 : -expm1(-x);", 1,
        [electron_split]),
    "plane of the split one off (z from plane -1)": (
        "const double att = -expm1(-p[P_ATTACH] * (double)k * dz);",
        "const double att = -expm1(-p[P_ATTACH] * (double)(k + 1) * dz);", 1,
        [electron_split, electron_split_field]),
    "track deposited at the nearest step instead of the floor": (
        "const double s = floor(tr[6] / dt);", "const double s = floor(tr[6] / dt + 0.5);", 1,
        [deposit_step]),
    "tilted axis through the anode instead of mid-gap": (
        "const double wz = (double)k * dz - 0.5 * p[P_GAP];", "const double wz = (double)k * dz;", 1,
        [tilted_profile]),
    "separate radius given to the positive ions": (
        "return s == 1 && tr[7] > 0.0 ? tr[7] : tr[1];", "return s == 0 && tr[7] > 0.0 ? tr[7] : tr[1];", 1,
        [separate_radii]),
    "absorbing cell still wraps the track offsets": (
        "return p[P_LATERAL_BC] != 0.0 ? d : wrap(d, L);", "return wrap(d, L);", 1,
        [absorbing_deposit]),
    "absorbing cell reads the wrapped neighbour": (
        "if (jj < 0 || jj >= ny || ii < 0 || ii >= nx) return 0.0;",
        "if (jj < 0 || jj >= ny || ii < 0 || ii >= nx) { jj = (jj + ny) % ny; ii = (ii + nx) % nx; }", 1,
        [dense_absorbing, absorbing_eigenmode]),
    "positive ions spared the electron sink": (
        "const double sinks[3] = {sink_n + sink_e, sink_n, sink_e};",
        "const double sinks[3] = {sink_n, sink_n, sink_e};", 1,
        [electron_dense]),
    "electrons drift with the positive ions": (
        "const double mus[3] = {p[P_MU_POS], -p[P_MU_NEG], -p[P_MU_E]};",
        "const double mus[3] = {p[P_MU_POS], -p[P_MU_NEG], p[P_MU_E]};", 1,
        [electron_dense]),
    "electron step without the diffusion factor 2": (
        "const double A = 2.0 * p[P_D_E] * (1.0 / (p[P_DX] * p[P_DX])",
        "const double A = p[P_D_E] * (1.0 / (p[P_DX] * p[P_DX])", 1,
        [electron_dt_diffusion]),
    "electron step from the ion mobility": (
        "const double v = p[P_MU_E] * E / dz;", "const double v = p[P_MU_NEG] * E / dz;", 1,
        [electron_dt_drift]),
    "train period one step longer than its steps": (
        "dt = period / (double)m;", "dt = period / (double)(m + 1);", 1,
        [train_periods]),
    "train pulses one step late": (
        "if (next_pulse < npulses && next_pulse * m == l) {", "if (next_pulse < npulses && next_pulse * m + 1 == l) {", 1,
        [train_superposition]),
    "last period opened a step after its pulse": (
        "last_pulse = (npulses - 1) * m;", "last_pulse = (npulses - 1) * m + 1;", 1,
        [train_periods]),
}


def _use_mutant(tmp_path, monkeypatch, old, new, nth):
    src = open(SRC).read()
    assert src.count(old) >= nth, old
    at = -1
    for _ in range(nth):
        at = src.index(old, at + 1)
    path = tmp_path / "oracle_mutant.c"
    path.write_text(src[:at] + new + src[at + len(old):])
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", *oracle._CFLAGS, "-o", str(so), str(path), "-lm"])
    monkeypatch.setattr(oracle, "_LIB", str(so))
    monkeypatch.setattr(oracle, "_libs", {})
    monkeypatch.setattr(oracle, "_threaded", False)
    monkeypatch.setattr(oracle, "build", lambda force=False: str(so))
    return oracle


def test_control_every_named_pin_passes_on_the_oracle(orc):
    pins = {pin for *_, named in MUTANTS.values() for pin in named}
    for pin in sorted(pins, key=lambda f: f.__name__):
        pin(orc)


@pytest.mark.parametrize("name", list(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path, monkeypatch):
    old, new, nth, pins = MUTANTS[name]
    orc = _use_mutant(tmp_path, monkeypatch, old, new, nth)
    missed = []
    for pin in pins:
        try:
            pin(orc)
        except Exception:  # an assertion, or an error the mistake provokes
            continue
        missed.append(pin.__name__)
    assert not missed, f"{name}: not caught by {missed}"


# The FP64 reference network (oracle/mlp.py): mistakes that keep its
# forward pass and its analytic gradient consistent with each other, so the
# finite-difference pin cannot see them; the torch-layer pin must.
def _silu_steep(a):
    return a / (1.0 + np.exp(-2.0 * a))


def _dsilu_steep(a):
    s = 1.0 / (1.0 + np.exp(-2.0 * a))
    return s * (1.0 + 2.0 * a * (1.0 - s))


def _summed_loss(original):
    def loss_and_grad(flat, Z, t, cast=True):
        loss, g = original(flat, Z, t, cast)
        return loss * Z.shape[0], g * Z.shape[0]
    return loss_and_grad


@pytest.mark.parametrize("mistake", ["steeper activation", "summed instead of mean loss"])
def test_reference_network_mistakes_fail_the_torch_pin(mistake, monkeypatch):
    import test_oracle_mlp as M
    from oracle import mlp
    if mistake == "steeper activation":
        monkeypatch.setattr(mlp, "silu", _silu_steep)
        monkeypatch.setattr(mlp, "dsilu", _dsilu_steep)
    else:
        monkeypatch.setattr(mlp, "loss_and_grad", _summed_loss(mlp.loss_and_grad))
    M.test_backward_matches_finite_differences()  # still self-consistent
    with pytest.raises(AssertionError):
        M.test_forward_and_gradient_match_a_torch_network()


# The closed forms (oracle/closed_forms.py): a version of Boag's second
# free-electron model that keeps both limits p = 0 (the two-voltage
# formula) and p = 1 (everything collected) yet differs in between; the
# expansion pin sees it.
def _model2_linear(u, p):
    return p + (1.0 - p) * math.log1p(u) / u


@pytest.mark.parametrize("name,fn", [("boag_model2", _model2_linear)])
def test_closed_form_mistakes_fail_the_expansion_pin(name, fn, monkeypatch):
    import test_closed_forms as C
    from oracle import closed_forms
    monkeypatch.setattr(closed_forms, name, fn)
    C.test_boag_models_reduce_to_two_voltage_method_at_p0()  # the old limits still hold
    C.test_boag_models_all_free_electrons_collect_everything()
    with pytest.raises(AssertionError):
        for p in (0.1, 0.5, 0.9):
            C.test_boag_models_small_and_large_dose_expansions(p)
