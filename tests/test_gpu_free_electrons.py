"""Free-electron component on the GPU against the CPU oracle: the
attachment split of the negative charge, the three-carrier electron phase
and the ion phase that follows (eqs. free_elec, ion_elec_distribution)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf

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


def attach_for(p_target, d):
    lo, hi = 1e-9, 1e7
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if cf.free_electron_fraction(mid, d) > p_target:
            lo = mid
        else:
            hi = mid
    return mid


def with_electrons(ch, p, mu_e=1500.0):
    ch = dict(ch)
    ch.update(attach_coeff=attach_for(p, ch["gap"]), mu_e=mu_e, D_e=mu_e * 0.02526)
    return ch


def compare(g, o, keys_extra=()):
    assert g["e_steps"] == o["e_steps"] and g["steps"] == o["steps"] and g["flags"] == o["flags"]
    assert g["f"] == pytest.approx(o["f"], rel=RTOL)
    N = o["n_released"]
    for k in ("n_released", "n_released_neg", "n_recombined", "col_pos_anode", "col_pos_cathode",
              "col_neg_anode", "col_neg_cathode", "e_released", "e_collected_anode", "e_collected_cathode",
              "e_recombined", "released_neg_charge") + tuple(keys_extra):
        assert abs(g[k] - o[k]) <= RTOL * N, (k, g[k], o[k])
    assert g["e_dt"] == pytest.approx(o["e_dt"], rel=1e-14)


@pytest.mark.parametrize("p", [0.1, 0.5])
def test_uniform_pulse_with_free_electrons(gpu, orc, p):
    """Boag's setting: a uniform instantaneous dose in a 1-D chamber."""
    ch = with_electrons(W.chamber(3, 2, 100, 1e-3, 0.1, 100.0, uniform_n0=3e9), p)
    g = gpu.it_solve(ch, W.no_tracks(), trace=True)
    o = orc.solve(ch, W.no_tracks(), with_trace=True, with_fields=False)
    compare(g, o)
    assert np.max(np.abs(g["trace"] - o["trace"])) <= RTOL * o["n_released"]


@pytest.mark.parametrize("ex", [None, dict(kernel=1, tile_y=16), dict(kernel=2, steps_per_pass=3)],
                         ids=["default", "plain16", "blocked3"])
def test_tracks_with_free_electrons(gpu, orc, ex):
    """Tracks parallel and tilted, on a ragged grid, with a background dose:
    the whole run, then the fields after a fixed number of steps (30 into
    the ion phase; a temporally blocked pass may run past the stop step, so
    fields at completion are not comparable)."""
    ch = with_electrons(W.chamber(70, 13, 37, 3e-4, 37 * 3e-4, 25.0, dy=2.5e-4, uniform_n0=2e9), 0.3)
    tr = W.tracks([[10.0, 7e-4, 1.0e-2, 1.5e-3, 0.0, 0.0, 0.0],
                   [12.0, 9e-4, 4.0e-3, 2.0e-3, 0.35, 2.0, 0.0]])
    g = gpu.it_solve(ch, tr, exec=ex)
    o = orc.solve(ch, tr, with_fields=False)
    compare(g, o)
    ch = dict(ch, max_steps=o["e_steps"] + 30)  # ends by the limit, 30 steps into the ion phase
    g = gpu.it_solve(ch, tr, exec=ex, fields=True)
    o = orc.solve(ch, tr, with_fields=True)
    assert o["steps"] == 30 and o["flags"] & gpu.IT_FLAG_MAX_STEPS
    compare(g, o)
    for a, b in ((g["pos"], o["pos"]), (g["neg"], o["neg"])):
        a = a.cpu().numpy()
        assert np.max(np.abs(a - b)) <= RTOL * max(np.abs(b).max(), 1e-300)


def test_step_limit_inside_the_electron_phase(gpu, orc):
    ch = with_electrons(W.chamber(3, 2, 60, 1e-3, 0.06, 50.0, uniform_n0=3e9, max_steps=20), 0.5)
    g = gpu.it_solve(ch, W.no_tracks())
    o = orc.solve(ch, W.no_tracks(), with_fields=False)
    assert o["e_steps"] == 20 and o["steps"] == 0 and o["flags"] & gpu.IT_FLAG_MAX_STEPS
    compare(g, o)


def test_unsupported_combinations(gpu):
    ch = with_electrons(W.chamber(8, 8, 10, 3e-4, 3e-3, 20.0, uniform_n0=1e9), 0.5)
    late = W.tracks([[5.0, 8e-4, 1e-3, 1e-3, 0.0, 0.0, 1e-7]])
    for bad_ch, tr in ((ch, late), (dict(ch, space_charge=1), W.no_tracks())):
        with pytest.raises(gpu.ItError) as e:
            gpu.it_solve(bad_ch, tr)
        assert e.value.code == gpu.IT_ENOTSUP
    with pytest.raises(gpu.ItError) as e:
        gpu.it_solve_batch([ch, ch], [W.no_tracks(), W.no_tracks()])
    assert e.value.code == gpu.IT_ENOTSUP
