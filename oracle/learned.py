"""Reference for the learned warm start (oracle; test infrastructure only).

The paper has no learned component; this is the reference for the
project's own warm start: a proper orthogonal decomposition (POD) of the
method's own unit-amplitude mode solutions and a small multilayer perceptron
mapping frequency features to POD coefficients.

* POD: snapshots X = [x_1 ... x_S] (complex columns). The Gram matrix X^H X
  is diagonalized; with eigenpairs (lambda_i, w_i) in decreasing order the
  basis is phi_i = X w_i / sqrt(lambda_i) (orthonormal in the Euclidean inner
  product), i < r.
* MLP: h_0 = features; z_l = W_l h_l + b_l; h_{l+1} = tanh(z_l) for hidden
  layers; output = z_{L-1}. The device computes each product with weights and
  inputs rounded to bfloat16 (round to nearest even) and accumulates in
  float32; this reference rounds the same operands to bfloat16 and evaluates
  in float64.
* Backward: the same rounding applies to both operands of every product
  (the output-gradient signal and the weights or activations); the bias
  gradient is a plain column sum.
* Loss: mean squared error over all outputs; Adam updates the float32 master
  weights (Kingma & Ba 2015, with bias correction).

Parity status: the backward pass is pinned by central finite differences of
the loss (tests/test_oracle_learned.py); the POD by numpy's SVD of X.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even); returns float64."""
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(f), u, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_forward(params, x, bf16=True):
    """params: list of (W [out,in], b [out]) float32. x [n, in]. Returns output
    [n, out] and the cache of layer inputs/pre-activations for backward."""
    h = np.asarray(x, np.float64)
    cache = []
    L = len(params)
    for l, (W, b) in enumerate(params):
        hin = bf16_round(h.astype(np.float32)) if bf16 else h
        Wr = bf16_round(W) if bf16 else np.asarray(W, np.float64)
        z = hin @ Wr.T + np.asarray(b, np.float64)
        cache.append((hin, Wr, z))
        h = np.tanh(z) if l < L - 1 else z
    return h, cache


def mse_loss_grad(params, x, t, bf16=True):
    """Loss (1/(n*out)) sum (y - t)^2 and gradients w.r.t. every W and b."""
    y, cache = mlp_forward(params, x, bf16)
    n, no = y.shape
    loss = np.sum((y - t) ** 2) / (n * no)
    g = 2.0 * (y - t) / (n * no)
    grads = [None] * len(params)
    L = len(params)
    for l in range(L - 1, -1, -1):
        hin, Wr, z = cache[l]
        if l < L - 1:
            g = g * (1.0 - np.tanh(z) ** 2)
        # every matrix product rounds both operands to bfloat16 on the device
        gq = bf16_round(g.astype(np.float32)) if bf16 else g
        gW = gq.T @ hin
        gb = g.sum(0)
        grads[l] = (gW, gb)
        g = gq @ Wr
    return loss, grads


def adam_step(params, grads, state, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (float32 master weights); state holds (m, v) per array."""
    out = []
    for (W, b), (gW, gb), st in zip(params, grads, state):
        new = []
        for k, (p, gp) in enumerate(((W, gW), (b, gb))):
            m, v = st[k]
            m[:] = b1 * m + (1 - b1) * gp
            v[:] = b2 * v + (1 - b2) * gp * gp
            mh = m / (1 - b1**t)
            vh = v / (1 - b2**t)
            new.append((p - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32))
        out.append(tuple(new))
    return out


def pod(X: np.ndarray, r: int):
    """POD of complex snapshots X [N, S]: basis [N, r] (orthonormal columns)
    and singular values [r], from the eigen-decomposition of X^H X."""
    Gm = X.conj().T @ X
    lam, W = np.linalg.eigh(Gm)
    order = np.argsort(lam)[::-1][:r]
    lam, W = lam[order], W[:, order]
    sig = np.sqrt(np.maximum(lam, 0.0))
    Phi = X @ (W / np.where(sig > 0, sig, 1.0)[None, :])
    return Phi, sig


def frequency_features(omega, omega_max):
    """Inputs of the network for frequency omega: w, sqrt(w), w^2 with w = omega/omega_max."""
    w = np.asarray(omega, np.float64) / omega_max
    return np.stack([w, np.sqrt(np.abs(w)), w * w], -1)
