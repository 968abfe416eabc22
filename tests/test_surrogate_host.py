"""Host logic of the surrogate pipeline with the solver call replaced by a
stand-in: rows whose solver run ends non-finite become NaN (and leave the
training data), a run stopped by max_steps is an error, and each row's
reference is the weighted blend over its two gap resolutions."""
import math

import numpy as np
import pytest

import workloads as W


@pytest.fixture
def sur(monkeypatch):
    import torch
    from paper_1610_06749_amd import surrogate
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(surrogate.B, "it_dt", lambda ch, tr=None: 1e-9)
    return surrogate


def fake_solver(bad_voltage=None, limit_voltage=None):
    from paper_1610_06749_amd import binding as B

    def run(chs, trs, exec=None, ws=None, stream=None):
        out = []
        for ch in chs:
            flags, ks = 0, 1.0 + ch["nz"] * 1e-3  # depends on the resolution
            if ch["voltage"] == bad_voltage:
                flags, ks = B.IT_FLAG_NONFINITE, math.nan
            if ch["voltage"] == limit_voltage:
                flags = B.IT_FLAG_MAX_STEPS
            out.append(dict(flags=flags, ks=ks, steps=10))
        return out
    return run


def test_solver_lnks_blends_resolutions_and_marks_nonfinite_rows(sur, monkeypatch):
    X = W.surrogate_inputs(5, 6)
    monkeypatch.setattr(sur.B, "it_solve_batch", fake_solver(bad_voltage=float(X[2, 2])))
    lnks, vs, _ = sur.solver_lnks(X, group=3)
    for q, x in enumerate(X):
        if q == 2:
            assert math.isnan(lnks[q])
            continue
        ref = sum(w * math.log(1.0 + nz * 1e-3) for nz, w in W.surrogate_resolutions(x))
        assert lnks[q] == pytest.approx(ref, rel=1e-14)
    assert vs > 0


def test_solver_lnks_refuses_runs_stopped_by_max_steps(sur, monkeypatch):
    X = W.surrogate_inputs(6, 4)
    monkeypatch.setattr(sur.B, "it_solve_batch", fake_solver(limit_voltage=float(X[1, 2])))
    with pytest.raises(RuntimeError):
        sur.solver_lnks(X)


def test_solver_data_leaves_nonfinite_rows_out(sur, monkeypatch):
    seed = 11
    Xtr = W.surrogate_inputs(seed, 8)
    monkeypatch.setattr(sur.B, "it_solve_batch", fake_solver(bad_voltage=float(Xtr[3, 2])))
    d = sur.solver_data(n_train=8, n_hold=4, seed=seed)
    assert d["train_nonfinite"] == 1 and d["holdout_nonfinite"] == 0
    assert len(d["Xtr"]) == 7 and np.all(np.isfinite(d["ytr"]))
    assert not np.any(np.all(d["Xtr"] == Xtr[3], axis=1))


@pytest.mark.parametrize("n,batch", [(45055, 2048), (32768, 2048), (4097, 512), (300, 512), (300, 0)])
def test_minibatch_order_tiles_every_row(n, batch):
    from paper_1610_06749_amd import surrogate
    order, b = surrogate.minibatch_order(n, batch, 11)
    if batch <= 0 or batch >= n:
        assert b == 0 and np.array_equal(np.sort(order), np.arange(n))
        return
    assert b == batch and len(order) % batch == 0 and len(order) - n < batch
    assert np.array_equal(np.sort(order[:n]), np.arange(n))  # one full shuffle first
    assert np.array_equal(order[n:], order[: len(order) - n])  # then its start again


def test_overlapping_inputs_are_deep_trains_of_the_box():
    X = W.surrogate_inputs_overlapping(7, 500, min_overlap=3.0)
    assert X.shape == (500, 6)
    ov = np.array([W.surrogate_overlap(x) for x in X])
    assert ov.min() >= 3.0
    for j, (lo, hi) in enumerate(W.SURROGATE_RANGES):
        assert X[:, j].min() >= lo and X[:, j].max() <= hi
    # a train of ceil(overlap) + 1 pulses for every row
    for x, o in zip(X[:20], ov[:20]):
        n, P = W.surrogate_train(x)
        assert n == math.ceil(o) + 1 and P == pytest.approx(1.0 / x[5])
    # the same seed, the same rows
    assert np.array_equal(X, W.surrogate_inputs_overlapping(7, 500, min_overlap=3.0))
