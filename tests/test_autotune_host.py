"""Host logic of the batch autotuner with the solver replaced by a
stand-in: choices the batch does not support are skipped, a batch with no
supported choice is an error, and batches of the same grids with other
options (absorbing sides, space charge, pulse trains) are tuned apart."""
import pytest

import workloads as W


@pytest.fixture
def tuner(monkeypatch):
    import torch
    from paper_1610_06749_amd import autotune
    monkeypatch.setattr(autotune, "_memo", {})
    monkeypatch.setattr(autotune, "_device_name", lambda: "host-test")
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(autotune.B, "it_strerror", lambda code: "stand-in")
    return autotune


def stand_in(calls, refuse_blocked=True, refuse_all=False):
    from paper_1610_06749_amd import binding as B

    def run(chs, trs, exec=None, ws=None, stream=None):
        calls.append(dict(exec or {}))
        blocked = (exec or {}).get("kernel") == B.IT_KERNEL_BLOCKED
        if refuse_all or (refuse_blocked and blocked):
            raise B.ItError(B.IT_ENOTSUP, "it_solve_batch")
        return [dict(f=1.0, ks=1.0, flags=0) for _ in chs]
    return run


def _batch(**over):
    chs = [dict(W.chamber(16, 12, 10, 5e-4, 10 * 5e-4, 100.0, uniform_n0=1e9), **over),
           dict(W.chamber(20, 16, 8, 5e-4, 8 * 5e-4, 150.0, uniform_n0=1e9), **over)]
    return chs, [W.no_tracks(), W.no_tracks()]


def test_unsupported_choices_are_skipped(tuner, monkeypatch):
    calls = []
    monkeypatch.setattr(tuner.B, "it_solve_batch", stand_in(calls))
    chs, trs = _batch(n_pulses=3, pulse_period_s=1e-9)
    cands = tuner.batch_candidates(rows=(8,), z_chunks=(8,), blocked_T=(2, 3))
    ex = tuner.tune_batch(chs, trs, steps=4, candidates=cands)
    assert ex["kernel"] == tuner.B.IT_KERNEL_PLAIN
    # every blocked candidate was tried once (refused at its warm-up), every plain one twice
    n_blocked = sum(c["kernel"] == tuner.B.IT_KERNEL_BLOCKED for c in cands)
    assert len(calls) == n_blocked + 2 * (len(cands) - n_blocked)


def test_no_supported_choice_is_an_error(tuner, monkeypatch):
    monkeypatch.setattr(tuner.B, "it_solve_batch", stand_in([], refuse_all=True))
    chs, trs = _batch()
    with pytest.raises(RuntimeError):
        tuner.tune_batch(chs, trs, steps=4, candidates=tuner.batch_candidates(z_chunks=(8,)))


def test_other_errors_pass_through(tuner, monkeypatch):
    from paper_1610_06749_amd import binding as B

    def broken(chs, trs, exec=None, ws=None, stream=None):
        raise B.ItError(B.IT_EINVAL, "it_solve_batch")
    monkeypatch.setattr(tuner.B, "it_solve_batch", broken)
    chs, trs = _batch()
    with pytest.raises(B.ItError):
        tuner.tune_batch(chs, trs, steps=4, candidates=tuner.batch_candidates(z_chunks=(8,)))


def test_batches_with_other_options_are_tuned_apart(tuner, monkeypatch):
    calls = []
    monkeypatch.setattr(tuner.B, "it_solve_batch", stand_in(calls, refuse_blocked=False))
    cands = tuner.batch_candidates(rows=(8,), z_chunks=(8,), blocked_T=(3,), blocked_z=(0,))
    seen = []
    for over in ({}, dict(lateral_bc=1), dict(space_charge=1), dict(n_pulses=3, pulse_period_s=2e-8),
                 dict(n_pulses=3, pulse_period_s=3e-8), {}):
        chs, trs = _batch(**over)
        before = len(calls)
        tuner.tune_batch(chs, trs, steps=4, candidates=cands)
        seen.append(len(calls) - before)
    # five distinct option sets are timed; the repeat of the first is cached
    assert seen[:5] == [2 * len(cands)] * 5 and seen[5] == 0
