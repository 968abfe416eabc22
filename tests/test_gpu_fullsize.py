"""GPU path at the workloads' full sizes, in the launch configuration the
benchmark times, against stored oracle results.

The stored values come from tests/golden/make_golden.py, which runs only the
CPU oracle (the full-size oracle runs take minutes to an hour, too long for a
test).  Fields are compared on sampled nodes (uniform samples plus the 256
largest nodes of each species) and through their 2-norms; tallies step by
step.  Properties that hold at any size (conservation) are checked on the
GPU's own traces.
"""
import glob
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RTOL = 1e-9
# the automatic choice (one step per launch when the fields are asked for),
# the one-step tile shapes, and the blocked kernel at T = 3 (what the
# benchmark times on the continuous-beam window) and T = 4
EXECS = [None, dict(kernel=1, tile_y=16), dict(kernel=1, tile_x=32), dict(kernel=1, tile_x=128),
         dict(kernel=2, steps_per_pass=3), dict(kernel=2, steps_per_pass=4)]
EXEC_IDS = ["default", "plain16", "plain32x16", "pair128x8", "blocked3", "blocked4"]


def load(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{name}.json not generated (run tests/golden/make_golden.py {name})")
    with open(path) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_06749_amd as it
    it.lib()
    return it


def check_result(g, o):
    assert g["steps"] == o["steps"] and g["flags"] == o["flags"]
    assert g["f"] == pytest.approx(o["f"], rel=RTOL)
    N = max(o["n_released"], 1.0)
    for k in ("n_released", "n_recombined", "col_pos_anode", "col_pos_cathode", "col_neg_anode",
              "col_neg_cathode", "n_inflight_pos", "n_inflight_neg"):
        assert abs(g[k] - o[k]) <= RTOL * N, (k, g[k], o[k])


def check_fields(g, summary):
    idx = np.asarray(summary["index"])
    for sp in ("pos", "neg"):
        f = g[sp].cpu().numpy()
        vals = f[idx[:, 0], idx[:, 1], idx[:, 2]]
        ref = np.asarray(summary[sp])
        assert np.max(np.abs(vals - ref)) <= RTOL * summary[f"{sp}_max"]
        assert np.linalg.norm(f) == pytest.approx(summary[f"{sp}_norm2"], rel=RTOL)
        assert np.abs(f).max() == pytest.approx(summary[f"{sp}_max"], rel=RTOL)


def check_conservation(trace, N, tol=1e-12):
    tr = np.asarray(trace)
    for a, c, S, Q, rel in ((1, 2, 5, 10, 9), (3, 4, 6, 11, 12)):
        prev = np.concatenate([[0.0], tr[:-1, S]]) + tr[:, rel]
        err = prev - tr[:, a] - tr[:, c] - tr[:, 0] + tr[:, Q] - tr[:, S]
        assert np.max(np.abs(err)) <= tol * N


def check_trace(got, stored, N):
    # stored traces may hold only the leading ten or thirteen columns
    # (written before the space-charge, negative-release and escaped columns
    # existed): the space-charge and escaped columns must then be zero and
    # the negative-release column equal the positive one (one radius per
    # track)
    ref = np.asarray(stored)
    k = ref.shape[1]
    assert got.shape[0] == ref.shape[0]
    assert np.max(np.abs(got[:, :k] - ref)) <= RTOL * N
    if k == 10:
        assert np.all(got[:, 10:12] == 0.0)
        assert np.array_equal(got[:, 12], got[:, 9])
    if k <= 13:  # written before the escaped columns existed: periodic cells lose nothing
        assert np.all(got[:, 13:15] == 0.0)


def test_single_track_against_stored(gpu):
    gd = load("single_track")
    g = gpu.it_solve(gd["chamber"], np.asarray(gd["tracks"]), trace=True)
    check_result(g, gd["result"])
    check_trace(g["trace"], gd["trace"], gd["result"]["n_released"])


@pytest.mark.parametrize("ex", EXECS, ids=EXEC_IDS)
def test_pulsed_beam_fields_at_full_size(gpu, ex):
    """256 x 256 x 200 nodes, 400 tracks, the first 40 steps."""
    gd = load("pulsed_fields")
    g = gpu.it_solve(gd["chamber"], np.asarray(gd["tracks"]), exec=ex, trace=True, fields=True)
    check_result(g, gd["result"])
    N = gd["result"]["n_released"]
    check_trace(g["trace"], gd["trace"], N)
    check_fields(g, gd["fields"])


@pytest.mark.parametrize("ex", EXECS, ids=EXEC_IDS)
def test_continuous_beam_window_at_full_size(gpu, ex):
    """512 x 512 x 256 nodes, eight tilted tracks, five deposit events in 2000 steps
    (the benchmark's window): results, every per-step record and sampled fields
    at the end."""
    gd = load("continuous_window")
    g = gpu.it_solve(gd["chamber"], np.asarray(gd["tracks"]), exec=ex, trace=True, fields=True)
    check_result(g, gd["result"])
    N = gd["result"]["n_released"]
    check_trace(g["trace"], gd["trace"], N)
    check_fields(g, gd["fields"])
    check_conservation(g["trace"], N)


def test_pulsed_beam_full_run(gpu):
    """The benchmark's workload run to full collection."""
    gd = load("pulsed_full")
    g = gpu.it_solve(gd["chamber"], np.asarray(gd["tracks"]), trace=True)
    check_result(g, gd["result"])
    check_conservation(g["trace"], gd["result"]["n_released"])


# the library's default (blocked passes of three steps, chunks of its choosing) and
# the other executions the autotuner can pick for the timed sweep
SWEEP_EXECS = [None, dict(kernel=2, steps_per_pass=3, z_chunk=48), dict(kernel=2, steps_per_pass=2, z_chunk=16),
               dict(kernel=1)]
SWEEP_IDS = ["default", "blocked3z48", "blocked2z16", "plain"]


@pytest.mark.parametrize("ex", SWEEP_EXECS, ids=SWEEP_IDS)
def test_batched_sweep_against_stored(gpu, ex):
    """The 96-chamber sweep in one batched run; every instance whose oracle
    result is stored is compared."""
    files = sorted(glob.glob(os.path.join(GOLDEN, "sweep_*.json")))
    if not files:
        pytest.skip("no sweep instances generated")
    chs, trs = W.batched_sweep()
    res = gpu.it_solve_batch(chs, trs, exec=ex)
    for fn in files:
        gd = json.load(open(fn))
        check_result(res[gd["instance"]], gd["result"])
