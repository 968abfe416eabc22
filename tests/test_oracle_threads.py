"""The oracle's OpenMP timing build returns the same bits as the
single-threaded build: every grid sum is a sum of per-plane partial sums
added in plane order, so the thread count cannot change the order of any
floating-point operation.  CPU only."""
import numpy as np
import pytest

import oracle
import workloads as W


def _cases():
    ch = W.chamber(70, 13, 37, 3e-4, 37 * 3e-4, 40.0, dy=4e-4, uniform_n0=2e9, max_steps=120)
    tr = W.tracks([[30.0, 8e-4, 5e-3, 1.5e-3, 0.0, 0.0, 0.0],
                   [80.0, 6e-4, 1.2e-2, 2e-3, 0.4, 1.1, 0.0],
                   [20.0, 9e-4, 2e-2, 4e-3, 0.2, 4.0, 3e-6]])
    yield "ragged", ch, tr
    yield "absorbing", dict(ch, lateral_bc=1), tr
    yield "space_charge", dict(ch, space_charge=1, uniform_n0=0.0), W.tracks([[5.0, 8e-4, 5e-3, 1.5e-3, 0, 0, 0]])
    fe = dict(ch, mu_e=1500.0, D_e=37.9, attach_coeff=5.0, max_steps=400)
    yield "free_electrons", fe, tr[:2]
    dt1 = oracle.dt(ch, tr[:2])
    train = dict(ch, n_pulses=4, pulse_period_s=17.3 * dt1, max_steps=10**6)
    yield "pulse_train", train, tr[:2]
    yield "absorbing_train_space_charge", dict(train, lateral_bc=1, space_charge=1, uniform_n0=0.0), \
        W.tracks([[5.0, 8e-4, 5e-3, 1.5e-3, 0, 0, 0]])


@pytest.mark.parametrize("name,ch,tr", list(_cases()), ids=[c[0] for c in _cases()])
def test_openmp_build_gives_the_same_bits(name, ch, tr):
    out = {}
    for flag in (False, True):
        oracle.use_threads(flag)
        try:
            out[flag] = oracle.solve(ch, tr, with_trace=True)
        finally:
            oracle.use_threads(False)
    a, b = out[False], out[True]
    if ch.get("n_pulses", 0) >= 2:
        assert a["pulses"] == ch["n_pulses"] and a["flags"] == 0
    assert a.keys() == b.keys()
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k]), k
        else:
            assert a[k] == b[k] or (a[k] != a[k] and b[k] != b[k]), k


def test_openmp_build_uses_several_threads():
    oracle.use_threads(True)
    try:
        n = oracle.threads()
    finally:
        oracle.use_threads(False)
    assert oracle.threads() == 1
    assert n >= 1
