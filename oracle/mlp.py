"""FP64 oracle of the learned proposal network (test infrastructure only).

The paper has no learned component (it names hybrid learned / model-based
processing only as future work, Sec. VII). What is specified here is the
proposal network that predicts coarse directions from the sample covariance,
so that only narrow windows of the Bartlett grid are scanned:

  input   the sample covariance R (Sec. IV-D.2 cost, read for T snapshots),
          packed as M diagonal real parts, then the strict upper triangle's
          real parts, then its imaginary parts (row-major), all divided by
          tr(R) / M  -> M^2 reals;
  network L hidden layers, each an affine map followed by the exact GELU
          x Phi(x); a final affine map to d_out outputs;
  loss    mean squared error over the active outputs (mask),
          L = sum m (y - t)^2 / sum m;
  update  Adam with bias correction.

Weights are W_l [out][in] and b_l [out]; a layer computes Z = H W^T + b.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def pack_covariance(R: np.ndarray) -> np.ndarray:
    """[M][M] Hermitian -> [M^2] reals: diagonal real, strict upper real, strict
    upper imaginary (row-major), scaled by M / tr(R)."""
    R = np.asarray(R, np.complex128)
    M = R.shape[0]
    iu = np.triu_indices(M, 1)
    scale = M / np.trace(R).real
    return np.concatenate([np.diag(R).real, R[iu].real, R[iu].imag]) * scale


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * np.exp(-0.5 * x * x) * INV_SQRT_2PI


def init_params(d_in, d_hidden, n_hidden, d_out, rng):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    dims = [d_in] + [d_hidden] * n_hidden + [d_out]
    params = []
    for i in range(len(dims) - 1):
        bound = 1.0 / math.sqrt(dims[i])
        params.append((rng.uniform(-bound, bound, (dims[i + 1], dims[i])),
                       rng.uniform(-bound, bound, dims[i + 1])))
    return params


def forward(params, X, round_fn=None):
    """Returns (Y, cache). ``round_fn`` (optional) rounds the GEMM operands
    (weights and layer inputs), e.g. to BF16, with everything else in FP64."""
    r = round_fn or (lambda a: a)
    H = np.asarray(X, np.float64)
    cache = []
    for li, (W, b) in enumerate(params):
        Z = r(H) @ r(W).T + b
        cache.append((H, Z))
        H = gelu(Z) if li < len(params) - 1 else Z
    return H, cache


def mse_loss(Y, T, mask=None):
    m = np.ones_like(Y) if mask is None else np.asarray(mask, np.float64)
    n = np.sum(m)
    L = np.sum(m * (Y - T) ** 2) / n
    dY = 2.0 * m * (Y - T) / n
    return L, dY


def backward(params, cache, dY, round_fn=None):
    """Gradients [(dW, db)] for the loss whose gradient wrt the output is dY."""
    r = round_fn or (lambda a: a)
    grads = [None] * len(params)
    dZ = np.asarray(dY, np.float64)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        H, Z = cache[li]
        grads[li] = (dZ.T @ r(H), dZ.sum(axis=0))
        if li > 0:
            dH = dZ @ r(W)
            dZ = dH * gelu_grad(cache[li - 1][1])
    return grads


class Adam:
    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for j, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[i][j] + (1 - self.b1) * g
                v = self.b2 * self.v[i][j] + (1 - self.b2) * g * g
                self.m[i] = tuple(m if k == j else self.m[i][k] for k in range(2))
                self.v[i] = tuple(v if k == j else self.v[i][k] for k in range(2))
                new.append(p - self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append(tuple(new))
        return out


def bf16_round(a):
    """Round float64 values to bfloat16 (round to nearest even, via float32)."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
