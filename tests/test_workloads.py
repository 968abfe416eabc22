"""Input generators: the shaped pulse's arrival process and placement, and the
surrogate samples (gap resolutions, pulse trains)."""
import math

import numpy as np
import pytest

import workloads as W


def _tri(T):
    # triangular pulse on [0, T], unit integral, peak 2/T at T/2
    return lambda t: (4.0 / T**2) * (t if t < T / 2 else T - t), 2.0 / T


def test_shaped_pulse_counts_and_mean_time():
    """Counts are Poisson with mean fluence * area; arrival times follow
    g(t): the triangular pulse's mean time is T/2 and its variance T^2/24."""
    ch = W.chamber(64, 64, 10, 5e-4, 5e-3, 100.0)
    area = 64 * 5e-4 * 64 * 5e-4
    T = 2e-6
    g, gmax = _tri(T)
    counts, times = [], []
    for seed in range(200):
        tr = W.shaped_pulse(ch, seed, 3e6, g, T, gmax)
        counts.append(len(tr))
        times.extend(tr[:, 6])
    mean = 3e6 * area
    assert np.mean(counts) == pytest.approx(mean, rel=4 * math.sqrt(mean / 200) / mean)
    times = np.asarray(times)
    n = len(times)
    assert times.mean() == pytest.approx(T / 2, abs=4 * T / math.sqrt(24 * n))
    assert times.var() == pytest.approx(T**2 / 24, rel=0.1)
    assert np.all((times >= 0) & (times < T))


def test_shaped_pulse_disc_region_and_values():
    ch = W.chamber(64, 64, 10, 5e-4, 5e-3, 100.0)
    r = 5e-3
    tr = W.shaped_pulse(ch, 3, 2e7, lambda t: 1e6, 1e-6, 1e6, let=lambda rng, n: rng.uniform(1, 2, n),
                        b=8e-4, theta=0.3, region="disc", r_min=r)
    cx, cy = 32 * 5e-4, 32 * 5e-4
    d = np.hypot(tr[:, 2] - cx, tr[:, 3] - cy)
    assert len(tr) > 100 and np.all(d <= r)
    # uniform over the disc: the mean squared radius is r^2/2
    assert np.mean(d**2) == pytest.approx(r * r / 2, rel=0.15)
    assert np.all((tr[:, 0] >= 1) & (tr[:, 0] <= 2)) and np.all(tr[:, 1] == 8e-4) and np.all(tr[:, 4] == 0.3)


def test_surrogate_resolutions_blend_is_continuous(orc):
    """The two gap resolutions around the real plane count: weights sum to
    one, and the blended ln k_s does not jump where the plane count steps
    (a single resolution jumps by a few 1e-4 there)."""
    import math
    for x in W.surrogate_inputs(3, 50):
        res = W.surrogate_resolutions(x)
        assert res[1][0] == res[0][0] + 1 and res[0][0] >= 8
        assert abs(res[0][1] + res[1][1] - 1.0) < 1e-15 and 0.0 <= res[1][1] < 1.0

    def blended(x):
        return sum(w * math.log(orc.solve(*W.surrogate_chamber(x, nz=nz), with_fields=False)["ks"])
                   for nz, w in W.surrogate_resolutions(x))

    def single(x):
        return math.log(orc.solve(*W.surrogate_chamber(x), with_fields=False)["ks"])

    lo = [50.0, 1e-3, 200.0, 0.030 * (1 - 1e-7), 0.1, 100.0]  # 60 planes of 5e-4 cm end at d = 0.03
    hi = [50.0, 1e-3, 200.0, 0.030 * (1 + 1e-7), 0.1, 100.0]
    assert abs(single(hi) - single(lo)) > 2e-4
    assert abs(blended(hi) - blended(lo)) < 1e-5


def test_surrogate_rate_moves_ks_and_is_continuous_at_the_train_threshold(orc):
    """The sixth input: below the train threshold (period at least twice the
    slower ion's gap transit) a sample is one pulse, so k_s is the same at
    10 Hz and just below the threshold.  Just above it the sample becomes a
    pulse train whose last period is the single pulse at the train's step
    (shortened to a whole number of steps per period, which alone moves k_s
    by a few 1e-5 here).  At 100 kHz the pulses overlap and k_s rises well
    above the single pulse's."""
    base = [20.0, 1e-3, 60.0, 0.05, 0.5]
    T = 2 * 0.05 ** 2 / (min(W.AIR["mu_pos"], W.AIR["mu_neg"]) * 60.0)

    def run(rate):
        ch, tr = W.surrogate_chamber(base + [rate])
        return orc.solve(ch, tr, with_fields=False), ch, tr

    r10, ch10, tr = run(10.0)
    r_below, ch_below, _ = run((1 - 1e-6) / T)
    r_above, ch_above, _ = run((1 + 1e-6) / T)
    r_fast, ch_fast, _ = run(1e5)
    assert "n_pulses" not in ch10 and "n_pulses" not in ch_below
    assert ch_above["n_pulses"] == 3 and ch_fast["n_pulses"] == 6
    assert r_below["ks"] == r10["ks"]
    single_at_train_dt = orc.solve(dict(ch10, dt_safety=r_above["dt"] / orc.dt(ch10, tr)), tr, with_fields=False)
    assert r_above["ks"] == pytest.approx(single_at_train_dt["ks"], rel=1e-9)
    assert r_above["ks"] == pytest.approx(r_below["ks"], rel=1e-4)
    assert r_fast["ks"] > 1.05 * r10["ks"]


def test_chamber_refuses_unknown_keywords():
    ch = W.chamber(8, 8, 6, 3e-4, 6 * 3e-4, 10.0, mu_pos=1.5, alpha=0.0)
    assert ch["mu_pos"] == 1.5 and ch["alpha"] == 0.0
    with pytest.raises(TypeError):
        W.chamber(8, 8, 6, 3e-4, 6 * 3e-4, 10.0, n_pulses=3)
