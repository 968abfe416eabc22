"""The stored oracle results (tests/golden/, written by make_golden.py with
the OpenMP build of the oracle) still come out of the current oracle, bit
for bit: the single-track run with its per-step records, and the cheapest
stored instances of the batched sweep.  The GPU parity tests compare the
library against these files, so a change to the oracle's arithmetic must
show up here first."""
import json
import os

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
RESULT_KEYS = ("f", "ks", "f_R", "n_released", "n_recombined", "n_inflight_pos", "n_inflight_neg",
               "col_pos_anode", "col_pos_cathode", "col_neg_anode", "col_neg_cathode", "dt", "steps",
               "flags", "max_beta_n")


def load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        return json.load(fh)


def test_single_track_reproduces(orc):
    g = load("single_track")
    r = orc.solve(g["chamber"], np.asarray(g["tracks"]), with_trace=True, with_fields=False)
    for k in RESULT_KEYS:
        assert r[k] == g["result"][k], k
    assert np.array_equal(r["trace"], np.asarray(g["trace"]))


@pytest.mark.parametrize("q", [94, 18, 91, 93, 86])
def test_sweep_instances_reproduce(orc, q):
    g = load(f"sweep_{q:03d}")
    assert g["instance"] == q
    chs, trs = W.batched_sweep()
    r = orc.solve(chs[q], trs[q], with_fields=False)
    for k in RESULT_KEYS:
        assert r[k] == g["result"][k], k
