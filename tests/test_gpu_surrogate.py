"""The surrogate pipeline end to end on a small budget: solver-generated
data, GPU training, held-out queries judged by the solver, and fallback
answers that are the solver's own."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sur():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_06749_amd import surrogate
    return surrogate


def test_solver_data_match_single_runs(sur):
    import paper_1610_06749_amd as it
    X = W.surrogate_inputs(31, 24)
    lnks, vs, sec = sur.solver_lnks(X, group=8)
    for x, v in zip(X[:6], lnks[:6]):
        ref = 0.0
        for nz, w in W.surrogate_resolutions(x):
            ch, tr = W.surrogate_chamber(x, nz=nz)
            ref += w * math.log(it.it_solve(ch, tr)["ks"])
        assert v == pytest.approx(ref, rel=1e-12, abs=1e-14)
    assert np.all(lnks > 0) and vs > 0


def test_small_pipeline(sur):
    Xtr = W.surrogate_inputs(41, 512)
    ytr, _, _ = sur.solver_lnks(Xtr)
    s = sur.Surrogate(members=4).fit(Xtr, ytr, steps=800, batch=128, log_every=100)
    assert s.loss_log[-1].max() < 0.5 * s.loss_log[0].max()
    Xq = W.surrogate_inputs(43, 64)
    yq, _, _ = sur.solver_lnks(Xq)
    ans, mask = s.answer(Xq, spread_tol=1e-3)
    # answers of flagged queries are the solver's own
    assert np.allclose(ans[mask], yq[mask], rtol=1e-12, atol=1e-14)
    # the trained ensemble beats the analytic baseline alone on held-out data
    mean, spread, fb, idx, n = s.query(Xq, 1e30)
    import torch
    base = sur.B.it_mlp_baseline(s.model, torch.tensor(Xq, dtype=torch.float32, device="cuda")).cpu().numpy()
    err_net = np.abs(mean.cpu().numpy() - yq)
    err_base = np.abs(base - yq)
    assert np.median(err_net) < np.median(err_base)
