"""Surrogate kernels on the GPU against the FP64 reference network.

BF16 models: both sides round weights and hidden activations to BF16 at the
same points.  The FP32 (GPU) and FP64 (reference) pre-activations can land
on opposite sides of a BF16 rounding boundary; such a flip moves one
activation by one BF16 step (2^-8 relative).  So the forward bar is 2e-4 on
the median and 99th percentile sample and 3e-2 on the worst, and gradients
are compared per parameter block in the 2-norm.

FP32 models: the reference runs without casts; the GPU's FP32 arithmetic
(sums of 128 products, expf in SiLU) stays within a few 1e-6 of it, so the
forward bar is 2e-5 on every sample and the gradient bar 1e-4 per block.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_06749_amd as it
    it.lib()
    return it


def make_norm(X, t, margin=1e-3):
    # the box gets a small margin: the GPU standardises in FP32, so a
    # training point on the edge can land a rounding step outside
    L = np.log(X)
    mu, sd = L.mean(axis=0), L.std(axis=0)
    Z = (L - mu) / sd
    return np.concatenate([mu, sd, Z.min(axis=0) - margin, Z.max(axis=0) + margin,
                           [t.mean(), t.std()]]).astype(np.float32)


def setup(gpu, members, n, seed=1, scale=1.0, precision=None):
    import torch
    X = W.surrogate_inputs(seed, n).astype(np.float32)
    t = (np.sin(np.log(X)).sum(axis=1) * 0.3 + 0.1 * np.log(X[:, 0])).astype(np.float32)
    norm = make_norm(X.astype(np.float64), t.astype(np.float64))
    params = W.mlp_init(seed + 10, members) * np.float32(scale)
    model = torch.empty(gpu.it_mlp_model_bytes(members), dtype=torch.uint8, device="cuda")
    gpu.it_mlp_init(model, members, params, norm, precision=precision)
    return model, X, t, norm, params


def ref_forward(params, X, norm, members, cast=True):
    n = dict(mu=norm[0:6].astype(np.float64), sigma=norm[6:12].astype(np.float64))
    Z = mlp.standardise(X.astype(np.float64), n)
    ys = [mlp.forward(params[m].astype(np.float64), Z, cast=cast)[0] * float(norm[25]) + float(norm[24])
          for m in range(members)]
    return np.stack(ys), Z


def test_forward_matches_reference(gpu):
    import torch
    members, n = 3, 4000
    model, X, t, norm, params = setup(gpu, members, n)
    mean, spread, fb, idx, cnt = gpu.it_mlp_query(model, torch.tensor(X, device="cuda"), 1e30)
    ys, _ = ref_forward(params, X, norm, members)
    err = np.abs(mean.cpu().numpy() - ys.mean(axis=0)) / (1 + np.abs(ys.mean(axis=0)))
    assert np.median(err) < 2e-4 and np.quantile(err, 0.99) < 2e-3 and err.max() < 3e-2
    sp = spread.cpu().numpy()
    ref_sp = ys.max(axis=0) - ys.min(axis=0)
    assert np.quantile(np.abs(sp - ref_sp) / (1 + ref_sp), 0.99) < 2e-3
    assert cnt == 0  # every input is inside its own training box


def test_gradient_matches_reference(gpu):
    import torch
    members, n = 2, 2048
    model, X, t, norm, params = setup(gpu, members, n, seed=3)
    grad, loss = gpu.it_mlp_grad(model, members, torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda"))
    g = grad.cpu().numpy()
    _, Z = ref_forward(params, X, norm, members)
    ts = (t.astype(np.float64) - float(norm[24])) / float(norm[25])
    for m in range(members):
        rl, rg = mlp.loss_and_grad(params[m].astype(np.float64), Z, ts, cast=True)
        assert loss[m] == pytest.approx(rl, rel=2e-3)
        off = 0
        for name, shape in mlp.SIZES:
            k = int(np.prod(shape))
            a, b = g[m, off:off + k], rg[off:off + k]
            assert np.linalg.norm(a - b) <= 2e-3 * np.linalg.norm(b) + 1e-7, name
            off += k


def test_fp32_forward_matches_reference(gpu):
    import torch
    members, n = 3, 4000
    model, X, t, norm, params = setup(gpu, members, n, precision=gpu.IT_MLP_FP32)
    mean, spread, fb, idx, cnt = gpu.it_mlp_query(model, torch.tensor(X, device="cuda"), 1e30)
    ys, _ = ref_forward(params, X, norm, members, cast=False)
    err = np.abs(mean.cpu().numpy() - ys.mean(axis=0)) / (1 + np.abs(ys.mean(axis=0)))
    assert err.max() < 2e-5
    ref_sp = ys.max(axis=0) - ys.min(axis=0)
    assert np.max(np.abs(spread.cpu().numpy() - ref_sp) / (1 + ref_sp)) < 2e-5
    # the BF16 model of the same weights is measurably further from the
    # exact network
    model_b, _, _, _, _ = setup(gpu, members, n, precision=gpu.IT_MLP_BF16)
    mean_b = gpu.it_mlp_query(model_b, torch.tensor(X, device="cuda"), 1e30)[0].cpu().numpy()
    err_b = np.abs(mean_b - ys.mean(axis=0)) / (1 + np.abs(ys.mean(axis=0)))
    assert np.median(err_b) > 10 * np.median(err)


def test_fp32_gradient_matches_reference(gpu):
    import torch
    members, n = 2, 2048
    model, X, t, norm, params = setup(gpu, members, n, seed=3, precision=gpu.IT_MLP_FP32)
    grad, loss = gpu.it_mlp_grad(model, members, torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda"))
    g = grad.cpu().numpy()
    _, Z = ref_forward(params, X, norm, members, cast=False)
    ts = (t.astype(np.float64) - float(norm[24])) / float(norm[25])
    for m in range(members):
        rl, rg = mlp.loss_and_grad(params[m].astype(np.float64), Z, ts, cast=False)
        assert loss[m] == pytest.approx(rl, rel=1e-5)
        off = 0
        for name, shape in mlp.SIZES:
            k = int(np.prod(shape))
            a, b = g[m, off:off + k], rg[off:off + k]
            assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-8, name
            off += k


@pytest.mark.parametrize("precision,loss_rel,bar", [("fp32", 1e-5, 1e-4), ("bf16", 2e-3, 2e-3)])
def test_gradient_on_a_ragged_sample_count(gpu, precision, loss_rel, bar):
    """1000 samples (15 full tiles of 64 and one of 40; the weight-gradient
    loop's tail) and an odd member count."""
    import torch
    members, n = 3, 1000
    prec = gpu.IT_MLP_FP32 if precision == "fp32" else gpu.IT_MLP_BF16
    model, X, t, norm, params = setup(gpu, members, n, seed=17, precision=prec)
    grad, loss = gpu.it_mlp_grad(model, members, torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda"))
    g = grad.cpu().numpy()
    cast = precision == "bf16"
    _, Z = ref_forward(params, X, norm, members, cast=cast)
    ts = (t.astype(np.float64) - float(norm[24])) / float(norm[25])
    for m in range(members):
        rl, rg = mlp.loss_and_grad(params[m].astype(np.float64), Z, ts, cast=cast)
        assert loss[m] == pytest.approx(rl, rel=loss_rel)
        off = 0
        for name, shape in mlp.SIZES:
            k = int(np.prod(shape))
            a, b = g[m, off:off + k], rg[off:off + k]
            assert np.linalg.norm(a - b) <= bar * np.linalg.norm(b) + 1e-8, (m, name)
            off += k


def test_fp32_minibatch_training_and_bad_precision(gpu):
    import torch
    members, n = 2, 2048
    model, X, t, norm, params = setup(gpu, members, n, seed=5, precision=gpu.IT_MLP_FP32)
    Xd, td = torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda")
    losses = gpu.it_mlp_train(model, members, Xd, td, steps=300, lr=2e-3, log_every=50, batch=512)
    assert np.all(losses[-1] < 0.2 * losses[0])
    with pytest.raises(gpu.ItError) as e:
        setup(gpu, 1, 64, precision=7)
    assert e.value.code == gpu.IT_EINVAL


def test_training_reduces_loss(gpu):
    import torch
    members, n = 2, 2048
    model, X, t, norm, params = setup(gpu, members, n, seed=5)
    Xd, td = torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda")
    losses = gpu.it_mlp_train(model, members, Xd, td, steps=300, lr=2e-3, log_every=50)
    assert losses.shape == (6, members)
    assert np.all(losses[-1] < 0.2 * losses[0])
    _, loss_after = gpu.it_mlp_grad(model, members, Xd, td)
    assert np.all(loss_after < losses[-1] * 1.5)


def test_minibatch_steps_equal_full_batch_steps_on_each_window(gpu):
    """Minibatch step s uses rows [(s mod n/batch) * batch, ...): two steps
    with batch n/2 equal one full-batch step on each half, bit for bit."""
    import torch
    members, n = 2, 1024
    model_a, X, t, norm, params = setup(gpu, members, n, seed=9)
    model_b = model_a.clone()
    Xd, td = torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda")
    half = n // 2
    gpu.it_mlp_train(model_a, members, Xd, td, steps=2, lr=1e-3, batch=half)
    gpu.it_mlp_train(model_b, members, Xd[:half].contiguous(), td[:half].contiguous(), steps=1, lr=1e-3)
    gpu.it_mlp_train(model_b, members, Xd[half:].contiguous(), td[half:].contiguous(), steps=1, lr=1e-3)
    assert torch.equal(model_a, model_b)
    with pytest.raises(gpu.ItError):  # minibatches must tile the data
        gpu.it_mlp_train(model_a, members, Xd, td, steps=1, lr=1e-3, batch=300)


def test_cosine_schedule_ends_at_final_rate(gpu):
    """A run from lr to lr_final takes the same last step as a constant-rate
    run at lr_final from the same state (the schedule's end point)."""
    import torch
    members, n = 1, 512
    model_a, X, t, norm, params = setup(gpu, members, n, seed=13)
    Xd, td = torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda")
    gpu.it_mlp_train(model_a, members, Xd, td, steps=5, lr=1e-3)
    model_b = model_a.clone()
    gpu.it_mlp_train(model_a, members, Xd, td, steps=1, lr=1e-4, lr_final=1e-4)
    gpu.it_mlp_train(model_b, members, Xd, td, steps=1, lr=1e-4)
    assert torch.equal(model_a, model_b)
    model_c = model_b.clone()
    gpu.it_mlp_train(model_b, members, Xd, td, steps=3, lr=3e-3, lr_final=1e-4)
    # the schedule's midpoint, as the library rounds it (FP64 sum, FP32 rate)
    mid = float(np.float32((float(np.float32(3e-3)) + float(np.float32(1e-4))) / 2))
    gpu.it_mlp_train(model_c, members, Xd, td, steps=2, lr=3e-3, lr_final=mid)
    gpu.it_mlp_train(model_c, members, Xd, td, steps=1, lr=1e-4)
    assert torch.equal(model_b, model_c)


def test_query_fallback_mask_and_indices(gpu):
    import torch
    members, n = 2, 1000
    model, X, t, norm, params = setup(gpu, members, n, seed=7)
    Xq = X.copy()
    Xq[::7, 0] *= 1e3       # LET far outside the training box
    Xq[3::11, 3] *= 0.01    # gap far outside
    mean, spread, fb, idx, cnt = gpu.it_mlp_query(model, torch.tensor(Xq, device="cuda"), 0.5)
    f = fb.cpu().numpy().astype(bool)
    sp = spread.cpu().numpy()
    out_of_box = np.zeros(n, bool)
    out_of_box[::7] = True
    out_of_box[3::11] = True
    assert np.all(f[out_of_box])
    assert np.array_equal(f, out_of_box | (sp > 0.5))
    ix = idx.cpu().numpy()
    assert cnt == f.sum() and np.array_equal(ix, np.nonzero(f)[0])


def test_baseline_matches_closed_forms(gpu):
    """The device baseline -ln f_Jaffe - ln f_Boag against the oracle's
    closed forms (eq. Jaffe_noangle, ln(1+u)/u)."""
    import torch
    from oracle import closed_forms as cf
    from paper_1610_06749_amd import surrogate
    X = W.surrogate_inputs(21, 300)
    model, _, _, norm, params = setup(gpu, 1, 64)
    gpu.it_mlp_init(model, 1, params, norm, surrogate.phys_constants())
    got = gpu.it_mlp_baseline(model, torch.tensor(X, dtype=torch.float32, device="cuda")).cpu().numpy()
    Xf = X.astype(np.float32).astype(np.float64)  # the device sees FP32 inputs
    a = W.AIR
    D, mu = 0.5 * (a["D_pos"] + a["D_neg"]), 0.5 * (a["mu_pos"] + a["mu_neg"])
    for x, g in zip(Xf, got):
        let, b, V, d, dose, _ = x
        fj = cf.jaffe_parallel(let, b, V / d, d, D, mu, a["alpha"], a["W_eV"])
        u = cf.boag_u(dose * W.ion_pairs_per_mGy(), d, V, a["mu_pos"], a["mu_neg"], a["alpha"])
        assert g == pytest.approx(-np.log(fj) - np.log(cf.boag(u)), rel=1e-9, abs=1e-12)
