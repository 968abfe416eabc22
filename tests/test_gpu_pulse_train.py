"""Pulse trains on the GPU against the CPU oracle: it_solve with the
stepping kernels (deposits of later pulses between launches) and
it_solve_batch (the pass before each later pulse adds the first pulse's
densities to its outputs), trains and single pulses mixed in one batch.
Same bar as the other parity tests: results, traces and fields to 1e-9
relative, identical step counts and flags; the last-period results too."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-9


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_06749_amd as it
    it.lib()
    return it


def compare(g, o, rtol=RTOL):
    assert g["steps"] == o["steps"], (g["steps"], o["steps"])
    assert g["flags"] == o["flags"], (g["flags"], o["flags"])
    assert g["pulses"] == o["pulses"], (g["pulses"], o["pulses"])
    assert g["dt"] == pytest.approx(o["dt"], rel=1e-14)
    N = max(o["n_released"], 1.0)
    for k in ("f", "ks", "f_R"):
        assert g[k] == pytest.approx(o[k], rel=rtol), k
    for k in ("n_released", "n_released_neg", "n_recombined", "col_pos_anode", "col_pos_cathode", "col_neg_anode",
              "col_neg_cathode", "n_inflight_pos", "n_inflight_neg", "n_escaped_pos", "n_escaped_neg",
              "period_released", "period_collected", "period_recombined"):
        assert abs(g[k] - o[k]) <= rtol * N, (k, g[k], o[k])
    assert g["max_beta_n"] == pytest.approx(o["max_beta_n"], rel=rtol)


def train(ch, n, period, **over):
    return dict(ch, n_pulses=int(n), pulse_period_s=float(period), **over)


def ragged(**over):
    """70 x 13 x 37 nodes (ragged tiles), a parallel and a tilted track and
    a uniform background, all at t = 0."""
    ch = W.chamber(70, 13, 37, 3e-4, 37 * 3e-4, 25.0, dy=2.5e-4, uniform_n0=2e9, **over)
    tr = W.tracks([[10.0, 7e-4, 1.0e-2, 1.5e-3, 0.0, 0.0, 0.0],
                   [12.0, 9e-4, 4.0e-3, 2.0e-3, 0.35, 2.0, 0.0]])
    return ch, tr


EXECS = [dict(kernel=1, tile_y=8), dict(kernel=1, tile_x=32), dict(kernel=1, tile_x=128),
         dict(kernel=2, steps_per_pass=2), dict(kernel=2, steps_per_pass=3), dict(kernel=2, steps_per_pass=4)]
EXEC_IDS = ["plain8", "plain32x16", "pair128x8", "blocked2", "blocked3", "blocked4"]


@pytest.mark.parametrize("ex", EXECS, ids=EXEC_IDS)
def test_train_single_run_matches_oracle(gpu, orc, ex):
    """Five pulses 7.3 single-pulse steps apart (8 steps a period): the
    pulses overlap, and blocked passes are cut at every pulse."""
    ch, tr = ragged()
    ch = train(ch, 5, 7.3 * orc.dt(ch, tr))
    g = gpu.it_solve(ch, tr, exec=ex, trace=True, fields=True)
    o = orc.solve(ch, tr, with_trace=True, with_fields=True)
    compare(g, o)
    assert o["pulses"] == 5 and o["steps"] == 40 and o["period_released"] > 0.0
    err = np.max(np.abs(g["trace"] - o["trace"]))
    assert err <= RTOL * o["n_released"]
    for name in ("pos", "neg"):
        gf = g[name].detach().cpu().numpy()
        assert np.max(np.abs(gf - o[name])) <= RTOL * np.max(np.abs(o[name]))


@pytest.mark.parametrize("variant", ["space_charge", "absorbing"])
@pytest.mark.parametrize("ex", [dict(kernel=1, tile_y=8), dict(kernel=1, tile_x=32)], ids=["plain8", "plain32x16"])
def test_train_single_run_with_options(gpu, orc, variant, ex):
    """The train of the test above with the space-charge term, or with
    absorbing lateral boundaries and a track next to the x = 0 edge."""
    ch, tr = ragged(**({"space_charge": 1} if variant == "space_charge" else {"lateral_bc": 1}))
    if variant == "absorbing":
        tr = tr.copy()
        tr[0, 2] = 3e-4
    ch = train(ch, 5, 7.3 * orc.dt(ch, tr))
    g = gpu.it_solve(ch, tr, exec=ex, trace=True)
    o = orc.solve(ch, tr, with_trace=True, with_fields=False)
    compare(g, o)
    assert o["flags"] == 0 and o["pulses"] == 5
    assert (o["n_space_charge_pos"] != 0.0) == (variant == "space_charge")
    assert (o["n_escaped_pos"] > 0.0) == (variant == "absorbing")
    for k in ("n_space_charge_pos", "n_space_charge_neg"):
        assert abs(g[k] - o[k]) <= RTOL * o["n_released"], k
    assert np.max(np.abs(g["trace"] - o["trace"])) <= RTOL * o["n_released"]


@pytest.mark.parametrize("mult", [0.6, 1.0, 1.7, 2.4], ids=["m1", "m1exact", "m2", "m3"])
def test_short_periods_single_and_batch(gpu, orc, mult):
    """Periods of one to three steps: a pulse at every step (the batch's
    first two passes take theirs from host-set flags)."""
    ch, tr = ragged()
    ch = train(ch, 6, mult * orc.dt(ch, tr))
    o = orc.solve(ch, tr, with_fields=False)
    assert o["steps"] == 6 * math.ceil(mult)
    compare(gpu.it_solve(ch, tr, exec=dict(kernel=1)), o)
    compare(gpu.it_solve_batch([ch], [tr], exec=dict(check_every=4))[0], o)


def single_pulse_dt(ch, tr):
    import oracle
    return oracle.dt(ch, tr)


def mixed_sweep():
    """Single pulses and trains of 1..13-step periods in one batch, uneven
    grids, one train cut by max_steps, one with absorbing lateral
    boundaries, one with space charge, one with no tracks."""
    rng = np.random.default_rng(77)
    chs, trs = [], []
    plan = [(0, 0.0), (4, 5.5), (3, 12.2), (7, 0.8), (0, 0.0), (5, 2.2), (9, 3.0), (4, 1.4)]
    for q, (n, mult) in enumerate(plan):
        nx, ny, nz = int(rng.integers(20, 80)), int(rng.integers(12, 50)), int(rng.integers(8, 36))
        ch = W.chamber(nx, ny, nz, 3e-4, nz * 3e-4, float(rng.uniform(15, 60)),
                       uniform_n0=float(rng.uniform(5e8, 4e9)), lateral_bc=1 if q == 5 else 0,
                       space_charge=1 if q == 6 else 0)
        k = 0 if q == 3 else int(rng.integers(1, 5))
        lx, ly = nx * 3e-4, ny * 3e-4
        tr = W.tracks(np.stack([rng.uniform(2, 20, k), rng.uniform(6e-4, 1.2e-3, k), rng.uniform(0, lx, k),
                                rng.uniform(0, ly, k), rng.uniform(0, 0.6, k), rng.uniform(0, 6.2, k),
                                np.zeros(k)], axis=1))
        if n:
            ch = train(ch, n, mult * single_pulse_dt(ch, tr))
        if q == 7:
            ch["max_steps"] = 3  # cut before the last pulse (m = 2: pulses at 0, 2, 4, 6)
        chs.append(ch)
        trs.append(tr)
    return chs, trs


@pytest.mark.parametrize("shape", [dict(tile_y=8), dict(tile_x=32)], ids=["64x8", "32x16"])
def test_batch_of_trains_and_single_pulses(gpu, orc, shape):
    chs, trs = mixed_sweep()
    res = gpu.it_solve_batch(chs, trs, exec=dict(shape, check_every=6))
    for q, (ch, tr, g) in enumerate(zip(chs, trs, res)):
        o = orc.solve(ch, tr, with_fields=False)
        compare(g, o)
    assert res[7]["flags"] & gpu.IT_FLAG_MAX_STEPS and res[7]["period_released"] == 0.0
    assert res[5]["n_escaped_pos"] > 0.0 and res[6]["n_space_charge_pos"] != 0.0


def test_batch_trains_equal_single_runs(gpu):
    chs, trs = mixed_sweep()
    res = gpu.it_solve_batch(chs, trs)
    for ch, tr, g in zip(chs, trs, res):
        s = gpu.it_solve(ch, tr, exec=dict(kernel=1))
        assert g["steps"] == s["steps"] and g["pulses"] == s["pulses"] and g["flags"] == s["flags"]
        assert g["f"] == pytest.approx(s["f"], rel=1e-12)
        assert g["f_R"] == pytest.approx(s["f_R"], rel=1e-12)


def test_batch_with_short_period_refuses_blocked_passes(gpu):
    """The mixed sweep has periods of one and two steps: a pass of three
    steps would hold two pulses."""
    chs, trs = mixed_sweep()
    with pytest.raises(gpu.ItError) as e:
        gpu.it_solve_batch(chs, trs, exec=dict(kernel=2, steps_per_pass=3))
    assert e.value.code == gpu.IT_ENOTSUP


def blocked_train_sweep(T):
    """Trains whose periods are T, T + 1, 2T + 1 and 13 steps (at most one
    pulse in a pass of T steps; a period of exactly T puts a pulse on the
    same level of every pass), single pulses, a train with space charge, one
    with absorbing lateral boundaries and a track at the x = 0 edge, and one
    cut by max_steps before its last pulse."""
    rng = np.random.default_rng(91)
    chs, trs = [], []
    periods = [T, 0, T + 1, 2 * T + 1, 13, 0, T + 1, T]
    for q, m in enumerate(periods):
        nx, ny, nz = int(rng.integers(24, 90)), int(rng.integers(14, 60)), int(rng.integers(8, 36))
        ch = W.chamber(nx, ny, nz, 3e-4, nz * 3e-4, float(rng.uniform(15, 60)),
                       uniform_n0=float(rng.uniform(5e8, 4e9)), space_charge=1 if q == 6 else 0,
                       lateral_bc=1 if q == 4 else 0)
        k = int(rng.integers(1, 5))
        lx, ly = nx * 3e-4, ny * 3e-4
        tr = W.tracks(np.stack([rng.uniform(2, 20, k), rng.uniform(6e-4, 1.2e-3, k), rng.uniform(0, lx, k),
                                rng.uniform(0, ly, k), rng.uniform(0, 0.6, k), rng.uniform(0, 6.2, k),
                                np.zeros(k)], axis=1))
        if q == 4:
            tr[0, 2] = 3e-4  # next to the absorbing x = 0 edge
        if m:
            ch = train(ch, 6, (m - 0.5) * single_pulse_dt(ch, tr))  # ceil gives m steps a period
        if q == 7:
            ch["max_steps"] = 4 * T + 1  # cut before its last pulse
        chs.append(ch)
        trs.append(tr)
    return chs, trs


@pytest.mark.parametrize("T", [2, 3, 4])
def test_batch_trains_with_blocked_passes(gpu, orc, T):
    """A pass of T steps adds a pulse to the outputs of the level before it
    and its recording block books the release with the pulse's step: every
    instance matches the oracle, max_beta_n and the last period included."""
    chs, trs = blocked_train_sweep(T)
    res = gpu.it_solve_batch(chs, trs, exec=dict(kernel=2, steps_per_pass=T, check_every=4))
    longest = 0
    for ch, tr, g in zip(chs, trs, res):
        o = orc.solve(ch, tr, with_fields=False)
        compare(g, o)
        longest = max(longest, o["steps"])
    # the batch's launches: a priming pass, then graphs of four passes, one
    # more graph in flight when the host sees the last instance stop
    assert res[0]["passes"] <= (longest + T - 1) // T + 9
    assert res[0]["pulses"] == 6 and res[7]["flags"] & gpu.IT_FLAG_MAX_STEPS


def test_batch_trains_take_blocked_passes_by_default(gpu, orc):
    """With every period at least three steps the library's choice is the
    blocked pass of three steps, and the results match the oracle."""
    chs, trs = blocked_train_sweep(3)
    res = gpu.it_solve_batch(chs, trs)
    longest = 0
    for ch, tr, g in zip(chs, trs, res):
        o = orc.solve(ch, tr, with_fields=False)
        compare(g, o)
        longest = max(longest, o["steps"])
    # 78 steps: 26 passes of three steps fit in one graph of 32 passes after
    # the priming pass (65 launches with the next graph in flight); one step
    # per pass would have needed three graphs and 129 launches
    assert res[0]["passes"] <= 65 < longest


def test_train_refuses_late_tracks_and_free_electrons(gpu):
    ch, tr = ragged()
    ch = train(ch, 3, 1e-6)
    late = tr.copy()
    late[1, 6] = 1e-9
    for c, t in ((ch, late), (dict(ch, mu_e=1000.0, D_e=100.0), tr)):
        with pytest.raises(gpu.ItError) as e:
            gpu.it_solve(c, t)
        assert e.value.code == gpu.IT_ENOTSUP
        with pytest.raises(gpu.ItError) as e:
            gpu.it_solve_batch([c], [t])
        assert e.value.code == gpu.IT_ENOTSUP


def test_surrogate_rate_moves_ks_on_the_solver(gpu):
    """The surrogate's sixth input through the batched solver: k_s is the
    single pulse's up to the train threshold (about 21 kHz for this sample),
    barely moves just above it, and rises once the pulses overlap."""
    base = [20.0, 1e-3, 60.0, 0.05, 0.5]
    rates = [10.0, 3e3, 3e4, 1e5]
    chs, trs = zip(*(W.surrogate_chamber(base + [r]) for r in rates))
    res = gpu.it_solve_batch(list(chs), list(trs))
    ks = [r["ks"] for r in res]
    assert [c.get("n_pulses", 0) for c in chs] == [0, 0, 3, 6]
    assert ks[1] == ks[0]
    assert ks[2] == pytest.approx(ks[0], rel=1e-4)
    assert ks[3] > 1.05 * ks[0]
