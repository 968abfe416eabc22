"""The allocation-free surrogate query (it_mlp_query_static) against the
query with a workspace, through the C ABI: two calls in a row, the second
with fewer queries, give the same answers, flags and flagged indices bit for
bit (both run the same kernels; only where their scratch lives differs)."""
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


def _model(gpu, members=3, precision=1):
    import torch
    X = W.surrogate_inputs(41, 4096)
    L = np.log(X)
    mu, sd = L.mean(axis=0), L.std(axis=0)
    Z = (L - mu) / sd
    # a narrow training box, so that part of the queries fall outside it
    norm = np.concatenate([mu, sd, 0.6 * Z.min(axis=0), 0.6 * Z.max(axis=0), [0.5, 0.2]]).astype(np.float32)
    params = W.mlp_init(7, members)
    model = torch.empty(gpu.it_mlp_model_bytes(members), dtype=torch.uint8, device="cuda")
    gpu.it_mlp_init(model, members, params, norm, precision=precision)
    return model


def _outputs(n):
    import torch
    return (torch.full((n,), -1.0, dtype=torch.float32, device="cuda"),
            torch.full((n,), -1.0, dtype=torch.float32, device="cuda"),
            torch.full((n,), 7, dtype=torch.uint8, device="cuda"),
            torch.full((n,), -1, dtype=torch.int64, device="cuda"))


@pytest.mark.parametrize("precision", [1, 0], ids=["fp32", "bf16"])
def test_static_query_matches_the_workspace_query(gpu, precision):
    import torch
    model = _model(gpu, precision=precision)
    tol = 1e9  # the box alone decides the fallbacks
    for n in (50_000, 3_001):  # the second call smaller, with a partial last tile
        X = torch.tensor(W.surrogate_inputs(100 + n, n).astype(np.float32), device="cuda")
        mean, spread, fb, idx, cnt = gpu.it_mlp_query(model, X, tol)
        out = _outputs(n)
        cnt_s = gpu.it_mlp_query_static(model, X, tol, out)
        torch.cuda.synchronize()
        assert cnt_s == cnt and 0 < cnt < n
        assert torch.equal(out[0], mean) and torch.equal(out[1], spread) and torch.equal(out[2], fb)
        assert torch.equal(out[3][:cnt], idx)
        assert bool((out[3][cnt:] == -1).all())  # nothing written past the flagged ones


def test_static_query_limits(gpu):
    import torch
    model = _model(gpu)
    X = torch.ones((4, 6), dtype=torch.float32, device="cuda")
    assert gpu.it_mlp_query_static(model, X[:0], 1e-3, _outputs(1)) == 0
    big = gpu.IT_MLP_QUERY_STATIC_MAX + 1
    lib = gpu.lib()
    import ctypes
    cnt = ctypes.c_int64()
    out = _outputs(4)
    # refused before any device work (the buffers are smaller than nq says)
    rc = lib.it_mlp_query_static(ctypes.c_void_p(model.data_ptr()), ctypes.c_void_p(X.data_ptr()), big, 1e-3,
                                 *[ctypes.c_void_p(t.data_ptr()) for t in out], ctypes.byref(cnt), None)
    assert rc == gpu.IT_EINVAL
    torch.cuda.synchronize()
    assert bool((out[0] == -1.0).all()) and bool((out[3] == -1).all())
