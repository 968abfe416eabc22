"""Pins of the oracle's pulse train (a beam in time as a periodic train of
identical instantaneous pulses, Distribution of ion tracks): a chamber with
n_pulses = N >= 2 deposits its pulse N times, one period P apart, at a step
shortened so that a period is m = ceil(P / dt1) whole steps, and reports the
last period.

Each check compares the oracle with something it does not compute itself:
the single-pulse run (N = 1, and trains whose pulses never overlap), linear
superposition of separately advanced pulses (no recombination), the charge
balance of a periodic state, and the first-order volume recombination of a
continuous beam, which a fast train approaches.
"""
import math

import numpy as np
import pytest

import workloads as W

AIR = W.AIR


def _small(nz=24, V=40.0, gap=0.05, n0=0.0, **over):
    return W.chamber(6, 5, nz, 2.5e-4, gap, V, uniform_n0=n0, stop_tol=1e-10, **over)


def _train(ch, n, period, max_steps=10**7):
    return dict(ch, n_pulses=int(n), pulse_period_s=float(period), max_steps=int(max_steps))


def _dt1(orc, ch, tr):
    return orc.dt(ch, tr)


def test_one_pulse_is_the_single_pulse_run(orc):
    ch = _small(n0=3e9)
    tr = W.tracks([[40.0, 1e-3, 3 * 2.5e-4, 2.5e-4, 0.4, 0.3, 0.0]])
    ref = orc.solve(ch, tr, with_fields=False)
    for n in (0, 1):
        r = orc.solve(dict(ch, n_pulses=n, pulse_period_s=1e-6), tr, with_fields=False)
        for k in ("f", "ks", "f_R", "n_released", "n_recombined", "steps", "dt", "max_beta_n"):
            assert r[k] == ref[k], k
        assert r["pulses"] == 0 and r["period_released"] == 0.0


def test_train_steps_whole_periods(orc):
    """dt = P / ceil(P / dt1); the run is N m steps; every pulse is counted."""
    ch = _small(n0=1e9)
    dt1 = _dt1(orc, ch, None)
    for mult, n in ((7.3, 3), (1.0, 4), (0.4, 5), (12.0, 2)):
        P = mult * dt1
        m = math.ceil(P / dt1)
        r = orc.solve(_train(ch, n, P), None, with_fields=False)
        assert r["dt"] == P / m
        assert r["dt"] <= dt1 * (1 + 1e-15)
        assert r["steps"] == n * m
        assert r["pulses"] == n
        # n pulses of a uniform n0 at every interior node
        per_pulse = 2 * ch["uniform_n0"] * ch["dx"] * ch["dy"] * (ch["gap"] / ch["nz"]) * \
            ch["nx"] * ch["ny"] * (ch["nz"] - 1)
        assert r["period_released"] == pytest.approx(per_pulse, rel=1e-12)
        assert 2 * r["n_released"] == pytest.approx(n * per_pulse, rel=1e-12)


def test_train_cut_by_max_steps_reports_the_whole_run(orc):
    ch = _small(n0=1e9)
    dt1 = _dt1(orc, ch, None)
    P = 10.5 * dt1  # m = 11
    r = orc.solve(_train(ch, 4, P, max_steps=25), None, with_fields=False)
    assert r["steps"] == 25
    assert r["flags"] & orc.FLAG_MAX_STEPS
    assert r["pulses"] == 3  # at steps 0, 11, 22
    assert r["period_released"] == 0.0  # the last period (from step 33) never began
    collected = r["col_pos_anode"] + r["col_pos_cathode"] + r["col_neg_anode"] + r["col_neg_cathode"]
    assert r["f"] == pytest.approx(collected / (r["n_released"] + r["n_released_neg"]), rel=1e-14)


def test_train_rejects_late_tracks_and_bad_periods(orc):
    ch = _small()
    with pytest.raises(ValueError):
        orc.solve(_train(ch, 3, 1e-6), W.tracks([[10.0, 1e-3, 0.0, 0.0, 0.0, 0.0, 1e-9]]))
    for P in (0.0, -1e-6, float("inf")):
        with pytest.raises(ValueError):
            orc.solve(_train(ch, 3, P), None)


@pytest.mark.parametrize("lateral_bc", [0, 1])
def test_superposition_without_recombination(orc, lateral_bc):
    """alpha = 0 (and no space charge) makes the stepping linear, so the
    train's final fields are the sum over pulses k of the pulse advanced
    alone from its step k m to the end, N m - k m steps; on a periodic
    cell and on an absorbing one."""
    ch = _small(nz=20, n0=2e9, alpha=0.0, lateral_bc=lateral_bc)
    tr = W.tracks([[30.0, 1e-3, 2 * 2.5e-4, 3 * 2.5e-4, 0.5, 1.1, 0.0]])
    dt1 = _dt1(orc, ch, tr)
    n, P = 4, 9.4 * dt1
    r = orc.solve(_train(ch, n, P), tr, with_fields=True)
    m = r["steps"] // n
    dt = r["dt"]
    pos0, neg0, _ = orc.uniform(ch, ch["uniform_n0"])
    pos0, neg0, _ = orc.deposit(ch, tr, 0, dt, pos0, neg0)
    sp = np.zeros_like(pos0)
    sn = np.zeros_like(neg0)
    for k in range(n):
        a, b = orc.advance(ch, dt, pos0, neg0, (n - k) * m)
        sp += a
        sn += b
    scale = float(np.max(np.abs(sp)))
    assert np.max(np.abs(r["pos"] - sp)) <= 1e-12 * scale
    assert np.max(np.abs(r["neg"] - sn)) <= 1e-12 * scale
    assert r["f_R"] == 1.0 and r["period_recombined"] == 0.0


def test_absorbing_train_balances_with_escape(orc):
    """A train on an absorbing cell (the lateral option with pulses): over
    the whole run, what the pulses released is collected, escapes through
    the sides, recombines (one of each sign per pair) or is still in
    flight; the escape is the per-step escaped column summed; the last
    period's f falls below its f_R by what escapes in it, and the same
    train on a periodic cell escapes nothing."""
    ch = _small(nz=24, n0=2e9, V=30.0, gap=0.06, lateral_bc=1)
    tr = W.tracks([[2.0, 1e-3, 0.3e-4, 0.2e-4, 0.0, 0.0, 0.0]])
    T = ch["gap"] ** 2 / (min(AIR["mu_pos"], AIR["mu_neg"]) * ch["voltage"])

    def balance(r):
        col = r["col_pos_anode"] + r["col_pos_cathode"] + r["col_neg_anode"] + r["col_neg_cathode"]
        esc = r["n_escaped_pos"] + r["n_escaped_neg"]
        inflight = r["n_inflight_pos"] + r["n_inflight_neg"]
        released = r["n_released"] + r["n_released_neg"]
        assert col + esc + 2 * r["n_recombined"] + inflight == pytest.approx(released, rel=1e-10)
        return esc / released

    r = orc.solve(_train(ch, 6, T / 3.0), tr, with_trace=True, with_fields=False)
    assert r["flags"] == 0 and r["pulses"] == 6
    assert balance(r) > 1e-3
    assert r["n_escaped_pos"] == pytest.approx(r["trace"][:, 13].sum(), rel=1e-12)
    assert r["n_escaped_neg"] == pytest.approx(r["trace"][:, 14].sum(), rel=1e-12)
    assert r["f"] < r["f_R"] - 1e-3
    rp = orc.solve(_train(dict(ch, lateral_bc=0), 6, T / 3.0), tr, with_fields=False)
    assert rp["flags"] == 0 and rp["pulses"] == 6 and rp["dt"] == r["dt"]
    assert rp["n_escaped_pos"] == 0.0 and rp["n_escaped_neg"] == 0.0
    assert balance(rp) == 0.0


@pytest.mark.parametrize("lateral_bc", [0, 1])
def test_train_with_space_charge_balances_step_by_step(orc, lateral_bc):
    """Every step of a train with the space-charge term (periodic and
    absorbing cells): each species' charge in flight changes by what was
    released before the step (each pulse at the start of its period's
    first step), minus what reached either electrode, recombined or
    escaped, plus the screening term's change; the released column sums
    to the run's release and holds exactly the pulse steps."""
    ch = _small(nz=24, n0=2e9, V=30.0, gap=0.06, lateral_bc=lateral_bc, space_charge=1)
    tr = W.tracks([[2.0, 1e-3, 0.3e-4, 0.2e-4, 0.0, 0.0, 0.0]])
    T = ch["gap"] ** 2 / (min(AIR["mu_pos"], AIR["mu_neg"]) * ch["voltage"])
    n = 5
    r = orc.solve(_train(ch, n, T / 3.0), tr, with_trace=True, with_fields=False)
    assert r["flags"] == 0 and r["pulses"] == n
    t = r["trace"]
    m = r["steps"] // n
    assert np.array_equal(np.flatnonzero(t[:, 9]), np.arange(n) * m)
    assert t[:, 9].sum() == pytest.approx(r["n_released"], rel=1e-14)
    assert t[:, 12].sum() == pytest.approx(r["n_released_neg"], rel=1e-14)
    assert r["n_space_charge_pos"] != 0.0 and r["n_space_charge_neg"] != 0.0
    for a, c, S, Q, rel, X in ((1, 2, 5, 10, 9, 13), (3, 4, 6, 11, 12, 14)):
        prev = np.concatenate([[0.0], t[:-1, S]]) + t[:, rel]
        err = prev - t[:, a] - t[:, c] - t[:, 0] + t[:, Q] - t[:, X] - t[:, S]
        assert np.max(np.abs(err)) <= 1e-12 * r["n_released"]
    assert (r["n_escaped_pos"] > 0.0) == bool(lateral_bc)


def test_pulses_that_never_overlap_match_the_single_pulse(orc):
    """A period several collection times long: each pulse is collected
    before the next arrives, so the last period's f is the single pulse's
    at the same step (dt_safety scaled to give the train's dt)."""
    ch = _small(n0=5e9, V=60.0)
    tr = W.tracks([[80.0, 1e-3, 3 * 2.5e-4, 2.5e-4, 0.0, 0.0, 0.0]])
    dt1 = _dt1(orc, ch, tr)
    single0 = orc.solve(ch, tr, with_fields=False)
    P = 3.0 * single0["steps"] * dt1 + 0.37 * dt1
    r = orc.solve(_train(ch, 2, P), tr, with_fields=False)
    ch1 = dict(ch, dt_safety=ch["dt_safety"] * r["dt"] / dt1)
    single = orc.solve(ch1, tr, with_fields=False)
    assert single["dt"] == pytest.approx(r["dt"], rel=1e-15)
    assert r["f"] == pytest.approx(single["f"], rel=1e-9)
    assert r["f_R"] == pytest.approx(single["f_R"], rel=1e-9)
    assert r["period_released"] == pytest.approx(single["n_released"] + single["n_released_neg"], rel=1e-13)


def test_periodic_state_balances_charge(orc):
    """Once periodic, one period collects or recombines what one pulse
    releases: collected + 2 recombined = released, so f = f_R.  The
    in-flight charge the balance leaves out decays with the pulse count
    (about 2e-5 of a pulse after 13 pulses here, 1e-14 after 40)."""
    ch = _small(nz=32, n0=3e9, V=30.0, gap=0.06)
    T = ch["gap"] ** 2 / (min(AIR["mu_pos"], AIR["mu_neg"]) * ch["voltage"])  # slowest transit
    P = T / 6.0
    r = orc.solve(_train(ch, 40, P), None, with_fields=False)
    assert r["f"] < 0.85  # the pulses overlap and recombine
    rel = r["period_released"]
    assert abs(r["period_collected"] + 2 * r["period_recombined"] - rel) <= 1e-10 * rel
    assert r["f"] == pytest.approx(r["f_R"], abs=1e-10)


@pytest.mark.parametrize("loss", [0.01, 0.003])
def test_fast_train_approaches_continuous_volume_recombination(orc, loss):
    """A train much faster than the ion transit approaches a continuous beam
    producing q = n0 / P pairs per cm^3 and s.  For a continuous beam with
    no diffusion the ions drift at constant speed, n+ = q z / (k+ E) and
    n- = q (d - z) / (k- E), so the loss over the gap is
    int alpha n+ n- dz / (q d) = alpha q d^4 / (6 k+ k- V^2) to first order:
    the small-loss limit of the general-recombination theory the paper
    cites (Introduction: Thomson, Mie, Greening)."""
    d, V = 0.1, 100.0
    kp, km = AIR["mu_pos"], AIR["mu_neg"]
    q = loss * 6 * kp * km * V ** 2 / (AIR["alpha"] * d ** 4)
    rate = 1e6
    ch = W.chamber(2, 2, 64, 1e-3, d, V, uniform_n0=q / rate, D_pos=0.0, D_neg=0.0)
    T = d / (min(kp, km) * V / d)
    r = orc.solve(_train(ch, int(math.ceil(2 * T * rate)) + 1, 1.0 / rate), None, with_fields=False)
    theory = AIR["alpha"] * q * d ** 4 / (6 * kp * km * V ** 2)
    assert (1 - r["f"]) == pytest.approx(theory, rel=0.03)
    assert (1 - r["f_R"]) == pytest.approx(theory, rel=0.03)
