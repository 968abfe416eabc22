"""The launch-shape autotuner: it times real candidates, keeps a valid one,
caches it, skips candidates a chamber does not support, and what it picks
gives the oracle's results."""
import json

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_06749_amd as it
    it.lib()
    return it


@pytest.fixture()
def tuner(gpu):
    from paper_1610_06749_amd import autotune
    autotune._memo.clear()
    yield autotune
    autotune._memo.clear()


def test_tune_picks_a_timed_candidate_and_caches_it(gpu, orc, tuner, tmp_path):
    ch = W.chamber(70, 13, 37, 3e-4, 37 * 3e-4, 25.0, dy=2.5e-4)
    cache = str(tmp_path / "tune.json")
    ex = tuner.tune(ch, steps=16, cache=cache)
    assert ex in tuner.PLAIN + tuner.PAIR + tuner.BLOCKED
    table = json.load(open(cache))
    (key, entry), = table.items()
    assert key.startswith("70x13x37@") and entry["exec"] == ex
    assert len(entry["all"]) == len(tuner.PLAIN + tuner.PAIR + tuner.BLOCKED)  # nx even: pairs included
    assert all(v > 0 for _, v in entry["all"])
    assert entry["voxel_steps_per_s"] == max(v for _, v in entry["all"])
    # a second tuner process would read the file; the memo answers here
    tuner._memo.clear()
    assert tuner.tune(ch, steps=16, cache=cache) == ex
    # the chosen shape computes what the oracle computes
    tr = W.tracks([[10.0, 7e-4, 1.0e-2, 1.5e-3, 0.0, 0.0, 0.0]])
    g = gpu.it_solve(ch, tr, exec=ex)
    o = orc.solve(ch, tr, with_fields=False)
    assert g["steps"] == o["steps"] and g["f"] == pytest.approx(o["f"], rel=1e-9)


def test_tune_skips_unsupported_candidates(gpu, tuner):
    # an odd nx: no tiles of column pairs
    ch = W.chamber(41, 24, 20, 3e-4, 20 * 3e-4, 25.0)
    ex = tuner.tune(ch, steps=8)
    assert ex not in tuner.PAIR
    # absorbing lateral boundaries are tuned apart from the periodic grid of
    # the same size (every candidate takes them)
    tuner._memo.clear()
    ex_a = tuner.tune(dict(ch, lateral_bc=1), steps=8)
    assert len(tuner._memo) == 1 and ex_a in tuner.PLAIN + tuner.BLOCKED


def test_tune_batch_returns_a_working_shape(gpu, tuner, tmp_path):
    chs = [W.chamber(n, n - 7, z, 5e-4, z * 5e-4, 100.0, uniform_n0=1e9) for n, z in ((40, 20), (72, 33), (96, 12))]
    trs = [W.tracks([[20.0, 1e-3, 0.5 * c["nx"] * 5e-4, 0.5 * c["ny"] * 5e-4, 0.0, 0.0, 0.0]]) for c in chs]
    ex = tuner.tune_batch(chs, trs, steps=24, rows=(8, 16), graph_passes=(4, 8), z_chunks=(8,), narrow=True,
                          blocked_T=(2, 3), blocked_z=(8, 16), blocked_graph=(4,), cache=str(tmp_path / "tb.json"))
    if ex["kernel"] == gpu.IT_KERNEL_PLAIN:
        assert (ex["tile_x"], ex["tile_y"]) in ((64, 8), (64, 16), (32, 16))
        assert ex["check_every"] in (4, 8) and ex["z_chunk"] == 8
    else:
        assert ex["steps_per_pass"] in (2, 3) and ex["z_chunk"] in (8, 16) and ex["check_every"] == 4
    table = __import__("json").load(open(str(tmp_path / "tb.json")))
    (entry,) = table.values()
    assert len(entry["all"]) == 3 * 2 + 2 * 2  # one-step shapes x passes per graph, blocked depths x chunks
    a = gpu.it_solve_batch(chs, trs, exec=ex)
    b = gpu.it_solve_batch(chs, trs)
    for ra, rb in zip(a, b):
        assert ra["steps"] == rb["steps"] and ra["flags"] == rb["flags"]
        assert ra["f"] == pytest.approx(rb["f"], rel=1e-11)
