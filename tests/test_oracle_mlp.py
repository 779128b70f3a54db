"""Pins for the FP64 proposal-network oracle: library special cases (scipy's
normal CDF, torch's CPU autograd and Adam in float64, torch's bfloat16
rounding), central finite differences, closed forms (first Adam step, masked
MSE), and the packing's inverse map."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import mlp

torch = pytest.importorskip("torch")


def tiny(rng, d_in=7, d_h=5, n_h=3, d_out=4):
    return mlp.init_params(d_in, d_h, n_h, d_out, rng)


def test_gelu_is_x_times_normal_cdf():
    x = np.linspace(-6, 6, 241)
    np.testing.assert_allclose(mlp.gelu(x), x * norm.cdf(x), atol=1e-15)
    t = torch.tensor(x, dtype=torch.float64)
    np.testing.assert_allclose(mlp.gelu(x), torch.nn.functional.gelu(t).numpy(), atol=1e-15)


def test_gelu_grad_finite_difference():
    x = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, atol=1e-9)


def test_forward_backward_match_torch_autograd():
    rng = np.random.default_rng(0)
    params = tiny(rng)
    X = rng.standard_normal((6, 7))
    T = rng.standard_normal((6, 4))
    mask = (rng.uniform(size=(6, 4)) > 0.3).astype(float)
    Y, cache = mlp.forward(params, X)
    L, dY = mlp.mse_loss(Y, T, mask)
    grads = mlp.backward(params, cache, dY)

    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    h = torch.tensor(X)
    for i, (W, b) in enumerate(tp):
        h = h @ W.T + b
        if i < len(tp) - 1:
            h = torch.nn.functional.gelu(h)
    m = torch.tensor(mask)
    Lt = (m * (h - torch.tensor(T)) ** 2).sum() / m.sum()
    Lt.backward()
    np.testing.assert_allclose(Y, h.detach().numpy(), rtol=1e-13, atol=1e-14)
    assert abs(L - Lt.item()) < 1e-13
    for (gW, gb), (W, b) in zip(grads, tp):
        np.testing.assert_allclose(gW, W.grad.numpy(), rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(gb, b.grad.numpy(), rtol=1e-11, atol=1e-13)


def test_backward_central_differences():
    rng = np.random.default_rng(1)
    params = tiny(rng, 4, 3, 2, 2)
    X = rng.standard_normal((5, 4))
    T = rng.standard_normal((5, 2))

    def loss(ps):
        return mlp.mse_loss(mlp.forward(ps, X)[0], T)[0]

    Y, cache = mlp.forward(params, X)
    grads = mlp.backward(params, cache, mlp.mse_loss(Y, T)[1])
    h = 1e-6
    for li in range(len(params)):
        for which in range(2):
            arr = params[li][which]
            g = grads[li][which]
            for idx in np.ndindex(arr.shape):
                p1 = [(W.copy(), b.copy()) for W, b in params]
                p2 = [(W.copy(), b.copy()) for W, b in params]
                p1[li][which][idx] += h
                p2[li][which][idx] -= h
                fd = (loss(p1) - loss(p2)) / (2 * h)
                assert abs(fd - g[idx]) < 1e-7 * max(1.0, abs(fd)), (li, which, idx)


def test_adam_matches_torch_and_first_step_closed_form():
    rng = np.random.default_rng(2)
    params = tiny(rng, 3, 4, 1, 2)
    opt = mlp.Adam(params, lr=1e-2)
    tp = [torch.tensor(a, requires_grad=True) for W, b in params for a in (W, b)]
    topt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    cur = params
    for step in range(5):
        grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in cur]
        new = opt.step(cur, grads)
        if step == 0:      # m_hat = g, v_hat = g^2: the step is -lr g / (|g| + eps)
            for (W0, b0), (W1, b1), (gW, gb) in zip(cur, new, grads):
                np.testing.assert_allclose(W1 - W0, -1e-2 * gW / (np.abs(gW) + 1e-8), rtol=1e-12)
        for t, g in zip(tp, [a for gr in grads for a in gr]):
            t.grad = torch.tensor(g)
        topt.step()
        cur = new
        flat = [a for W, b in cur for a in (W, b)]
        for a, t in zip(flat, tp):
            np.testing.assert_allclose(a, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_masked_mse_hand_value():
    Y = np.array([[1.0, 2.0], [3.0, 5.0]])
    T = np.array([[0.0, 2.0], [1.0, 0.0]])
    m = np.array([[1.0, 1.0], [1.0, 0.0]])
    L, dY = mlp.mse_loss(Y, T, m)
    assert L == (1 + 0 + 4) / 3
    np.testing.assert_array_equal(dY, np.array([[2 / 3, 0.0], [4 / 3, 0.0]]))


def test_pack_covariance_inverse_and_scale():
    rng = np.random.default_rng(3)
    M = 6
    Y = rng.standard_normal((10, M)) + 1j * rng.standard_normal((10, M))
    R = Y.T @ Y.conj() / 10
    x = mlp.pack_covariance(R)
    assert x.size == M * M
    # rebuild R * M / tr(R) from the packed vector
    n_up = M * (M - 1) // 2
    d, re, im = x[:M], x[M:M + n_up], x[M + n_up:]
    Rb = np.diag(d).astype(complex)
    iu = np.triu_indices(M, 1)
    Rb[iu] = re + 1j * im
    Rb[(iu[1], iu[0])] = re - 1j * im
    np.testing.assert_allclose(Rb, R * M / np.trace(R).real, atol=1e-13)
    np.testing.assert_allclose(mlp.pack_covariance(3.7 * R), x, atol=1e-13)
    assert abs(np.sum(d) - M) < 1e-12


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(1000) * 10 ** rng.uniform(-5, 5, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 3.0e38]])
    ref = torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)
