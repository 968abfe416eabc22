"""Writes the stored oracle results used by the full-size GPU parity tests.

Calls only the CPU oracle and the seeded input generators; nothing here
touches the GPU library.  Each case writes one JSON file next to this script:

    python tests/golden/make_golden.py single_track pulsed_full pulsed_fields \
        continuous_window sweep:0-95        (or sweep:3,17,40 for a list)

The oracle runs in its OpenMP build, which returns the same bits as the
single-threaded one (tests/test_oracle_threads.py).  Runtime on 8 host
cores: single_track ~1 s, pulsed_fields ~1 min, continuous_window (2000
steps of 512 x 512 x 256) ~30 min, pulsed_full ~30 min, sweep instances from
seconds to twenty minutes each.
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

oracle.use_threads(True)

RESULT_KEYS = ("f", "ks", "f_R", "n_released", "n_recombined", "n_inflight_pos", "n_inflight_neg",
               "col_pos_anode", "col_pos_cathode", "col_neg_anode", "col_neg_cathode", "dt", "steps",
               "flags", "max_beta_n")
N_SAMPLES = 4096


def _result(r):
    return {k: r[k] for k in RESULT_KEYS}


def _samples(shape, seed, n=N_SAMPLES):
    """Sample node indices: half uniform over the interior, half near the
    field maxima is decided by the caller; here uniform (k, j, i)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, shape[0] - 1, n)
    j = rng.integers(0, shape[1], n)
    i = rng.integers(0, shape[2], n)
    return np.stack([k, j, i], axis=1)


def _field_summary(pos, neg, seed):
    idx = _samples(pos.shape, seed)
    # also the 256 largest nodes of each species, where the physics happens
    top = []
    for f in (pos, neg):
        flat = np.argsort(f, axis=None)[-256:]
        top.append(np.stack(np.unravel_index(flat, f.shape), axis=1))
    idx = np.concatenate([idx] + top)
    return {
        "index": idx.tolist(),
        "pos": pos[idx[:, 0], idx[:, 1], idx[:, 2]].tolist(),
        "neg": neg[idx[:, 0], idx[:, 1], idx[:, 2]].tolist(),
        "pos_norm2": float(np.linalg.norm(pos)), "neg_norm2": float(np.linalg.norm(neg)),
        "pos_max": float(np.abs(pos).max()), "neg_max": float(np.abs(neg).max()),
    }


def _write(name, payload):
    payload["generated_by"] = "tests/golden/make_golden.py (CPU oracle only)"
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(payload, fh)
    print(f"wrote {name}.json", flush=True)


def case_single_track():
    ch, tr = W.single_track()
    r = oracle.solve(ch, tr, with_trace=True, with_fields=False)
    _write("single_track", {"chamber": ch, "tracks": tr.tolist(), "result": _result(r),
                            "trace": r["trace"].tolist()})


def case_pulsed_full():
    ch, tr = W.pulsed_beam()
    t0 = time.time()
    r = oracle.solve(ch, tr, with_trace=True, with_fields=False)
    _write("pulsed_full", {"chamber": ch, "tracks": tr.tolist(), "result": _result(r),
                           "trace_every_100": r["trace"][::100].tolist(),
                           "trace_last": r["trace"][-1].tolist(), "seconds": time.time() - t0})


def case_pulsed_fields():
    ch, tr = W.pulsed_beam()
    ch.update(max_steps=40, stop_tol=0.0)
    r = oracle.solve(ch, tr, with_trace=True, with_fields=True)
    _write("pulsed_fields", {"chamber": ch, "tracks": tr.tolist(), "result": _result(r),
                             "trace": r["trace"].tolist(),
                             "fields": _field_summary(r["pos"], r["neg"], seed=11)})


def case_continuous_window():
    """The continuous-beam window (512 x 512 x 256, 2000 steps): four tilted
    tracks at t = 0 and four more arriving inside the window, five deposit
    events in all."""
    ch, tr = W.continuous_window()
    t0 = time.time()
    r = oracle.solve(ch, tr, with_trace=True, with_fields=True)
    assert r["steps"] == W.WINDOW_STEPS
    _write("continuous_window", {"chamber": ch, "tracks": tr.tolist(), "result": _result(r),
                                 "trace": r["trace"].tolist(),
                                 "fields": _field_summary(r["pos"], r["neg"], seed=13),
                                 "seconds": time.time() - t0})


def case_sweep(instances):
    chs, trs = W.batched_sweep()
    for q in instances:
        name = f"sweep_{q:03d}"
        t0 = time.time()
        r = oracle.solve(chs[q], trs[q], with_trace=False, with_fields=False)
        _write(name, {"instance": q, "result": _result(r), "seconds": time.time() - t0})


def main(argv):
    for arg in argv:
        if arg.startswith("sweep:"):
            spec = arg.split(":", 1)[1]
            if "-" in spec:
                lo, hi = (int(v) for v in spec.split("-"))
                case_sweep(range(lo, hi + 1))
            else:
                case_sweep([int(v) for v in spec.split(",")])
        else:
            globals()[f"case_{arg}"]()


if __name__ == "__main__":
    main(sys.argv[1:] or ["single_track"])
