"""Pins of the FP64 reference network (CPU only): the analytic backward
against central finite differences, the BF16 rounding against torch's
bfloat16 conversion, and one Adam step written out."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp


def _data(n=64, seed=1):
    rng = np.random.default_rng(seed)
    Z = rng.normal(size=(n, 6))
    t = rng.normal(size=n)
    return Z, t


def test_param_count():
    assert mlp.N_PARAMS == W.MLP_PARAMS == 34049


def test_backward_matches_finite_differences():
    Z, t = _data()
    flat = W.mlp_init(3, 1)[0].astype(np.float64) * 0.5
    flat += np.random.default_rng(4).normal(scale=0.05, size=flat.shape)  # nonzero biases
    loss, g = mlp.loss_and_grad(flat, Z, t, cast=False)
    rng = np.random.default_rng(5)
    picks = np.concatenate([rng.integers(0, 768, 6), rng.integers(768, 896, 3), rng.integers(896, 17280, 8),
                            rng.integers(17408, 33792, 8), rng.integers(33792, 34049, 6), [34048]])
    for q in picks:
        h = 1e-6
        fp = flat.copy(); fp[q] += h
        fm = flat.copy(); fm[q] -= h
        num = (mlp.loss_and_grad(fp, Z, t, cast=False)[0] - mlp.loss_and_grad(fm, Z, t, cast=False)[0]) / (2 * h)
        assert g[q] == pytest.approx(num, rel=1e-5, abs=1e-9)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(scale=s, size=2000) for s in (1e-3, 1.0, 1e3)]).astype(np.float32)
    x = np.concatenate([x, np.float32([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0])])
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_adam_one_step():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    m = np.zeros(2)
    v = np.zeros(2)
    p1, m1, v1 = mlp.adam(p, g, m, v, 1, 0.01)
    # first step: m_hat = g, v_hat = g^2, so the update is lr * sign(g) (up to eps)
    assert p1 == pytest.approx(p - 0.01 * np.sign(g), rel=1e-6)
    assert m1 == pytest.approx(0.1 * g) and v1 == pytest.approx(0.001 * g * g)


def test_forward_casts_only_round():
    Z, _ = _data(16)
    flat = W.mlp_init(9, 1)[0].astype(np.float64)
    y0, _ = mlp.forward(flat, Z, cast=False)
    y1, _ = mlp.forward(flat, Z, cast=True)
    # BF16 keeps 8 bits: the two differ, but only at the percent level
    assert np.max(np.abs(y1 - y0)) <= 0.05 * (1 + np.max(np.abs(y0)))
    assert np.max(np.abs(y1 - y0)) > 0


def test_forward_and_gradient_match_a_torch_network():
    """The reference network against the same network assembled from
    torch's own layers (Linear, SiLU, mean squared error) in float64 on the
    CPU, weights taken from the flat vector in the documented order, and
    torch's autograd for the gradient: pins the layer order, the
    activation, the output layer and the loss, which finite differences of
    the reference itself cannot."""
    torch = pytest.importorskip("torch")
    Z, t = _data(48, seed=3)
    flat = W.mlp_init(5, 1)[0].astype(np.float64)
    flat += np.random.default_rng(6).normal(scale=0.05, size=flat.shape)
    P = mlp.unpack(flat)
    net = torch.nn.Sequential(
        torch.nn.Linear(6, 128), torch.nn.SiLU(), torch.nn.Linear(128, 128), torch.nn.SiLU(),
        torch.nn.Linear(128, 128), torch.nn.SiLU(), torch.nn.Linear(128, 1)).double()
    with torch.no_grad():
        for layer, (w, b) in zip((net[0], net[2], net[4], net[6]),
                                 (("W1", "b1"), ("W2", "b2"), ("W3", "b3"), ("w4", "b4"))):
            layer.weight.copy_(torch.tensor(P[w]).reshape(layer.weight.shape))
            layer.bias.copy_(torch.tensor(P[b]))
    y_t = net(torch.tensor(Z))[:, 0]
    loss_t = torch.nn.functional.mse_loss(y_t, torch.tensor(t))
    loss_t.backward()
    y, _ = mlp.forward(flat, Z, cast=False)
    loss, g = mlp.loss_and_grad(flat, Z, t, cast=False)
    assert np.allclose(y, y_t.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert loss == pytest.approx(float(loss_t.detach()), rel=1e-12)
    G = mlp.unpack(g)
    for layer, (w, b) in zip((net[0], net[2], net[4], net[6]),
                             (("W1", "b1"), ("W2", "b2"), ("W3", "b3"), ("w4", "b4"))):
        assert np.allclose(G[w].reshape(layer.weight.shape), layer.weight.grad.numpy(), rtol=1e-10, atol=1e-14)
        assert np.allclose(G[b], layer.bias.grad.numpy(), rtol=1e-10, atol=1e-14)
