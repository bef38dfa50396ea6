"""Learned diagonal preconditioner: per-coefficient network, loss and gradients.

Test infrastructure (see the package docstring); plain FP64 NumPy.  There is
no paper passage for this part (the paper only notes that the method suits
coupling with machine learning, Sec. 5); it is the reference the GPU kernels'
forward pass, loss and gradients are checked against.

For residual column j and coefficient i the network sees six features

    g = kappa_i / T_j  (T_j = sum kappa |r|^2 / sum |r|^2, as in the TPA recipe)
    f = [K(g), log g, log kappa_i, (V_ii - lambda_j) / T_j, lambda_j / T_j,
         log(|r_ij| sqrt(L) / ||r_j|| + 1e-30)]

(K the Teter-Payne-Allan factor, V_ii the potential's diagonal in the basis,
lambda_j the current Ritz value) padded with two zeros to eight inputs, and
computes

    h1 = silu(W1 f + b1), h2 = silu(W2 h1 + b2)      (width 64)
    z  = w3 . h2 + b3,    s = K(g) softplus(z) / log 2,

a positive diagonal scale (s = K(g) when the last layer is zero, i.e. the
untrained network is the TPA preconditioner).  The preconditioned residual is
w = s * r.  Training minimises the mean over columns of the direction loss

    loss_j = 1 - |<s r, t>|^2 / (||s r||^2 ||t||^2)

against target corrections t (only the direction of the update matters to a
Rayleigh-Ritz step).  Parameter vector layout (float count 4801): W1 (64 x 8,
row-major), b1 (64), W2 (64 x 64, row-major), b2 (64), w3 (64), b3 (1).
"""
from __future__ import annotations

import math

import numpy as np

NIN = 8
H = 64
NPARAM = H * NIN + H + H * H + H + H + 1
LOG2 = math.log(2.0)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + H * NIN].reshape(H, NIN); o += H * NIN
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]; o += 1
    assert o == NPARAM
    return W1, b1, W2, b2, w3, b3


def init_params(seed: int) -> np.ndarray:
    """He-style initial weights, zero last layer (network = TPA at start)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((H, NIN)) * math.sqrt(2.0 / NIN)
    W2 = rng.standard_normal((H, H)) * math.sqrt(2.0 / H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), np.zeros(H), [0.0]])


def tpa_factor(g):
    num = 27.0 + 18.0 * g + 12.0 * g ** 2 + 8.0 * g ** 3
    return num / (num + 16.0 * g ** 4)


def features(kappa, vdiag, R, lam):
    """Features (L, ncol, 8) and the TPA factors (L, ncol)."""
    R = np.asarray(R)
    L = R.shape[0]
    R2 = np.abs(R) ** 2
    T = (kappa[:, None] * R2).sum(0) / R2.sum(0)
    rn = np.sqrt(R2.sum(0))
    g = kappa[:, None] / T[None, :]
    K = tpa_factor(g)
    F = np.zeros((L, R.shape[1], NIN))
    F[..., 0] = K
    F[..., 1] = np.log(g)
    F[..., 2] = np.log(kappa)[:, None]
    F[..., 3] = (vdiag[:, None] - lam[None, :]) / T[None, :]
    F[..., 4] = (lam / T)[None, :]
    F[..., 5] = np.log(np.abs(R) * math.sqrt(L) / rn[None, :] + 1e-30)
    return F, K


def silu(x):
    return x / (1.0 + np.exp(-x))


def dsilu(x):
    sg = 1.0 / (1.0 + np.exp(-x))
    return sg * (1.0 + x * (1.0 - sg))


def softplus(x):
    return np.logaddexp(0.0, x)


def forward(theta, F, K):
    """Scale s (same shape as K) and the activations needed by backward."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    a1 = F @ W1.T + b1
    h1 = silu(a1)
    a2 = h1 @ W2.T + b2
    h2 = silu(a2)
    z = h2 @ w3 + b3
    s = K * softplus(z) / LOG2
    return s, (a1, h1, a2, h2, z)


def loss_and_grad(theta, F, K, R, Tt):
    """Mean direction loss over columns and its gradient w.r.t. theta."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    s, (a1, h1, a2, h2, z) = forward(theta, F, K)
    ncol = R.shape[1]
    A = (s * np.conj(R) * Tt).sum(0)            # <s r, t>
    B = (s ** 2 * np.abs(R) ** 2).sum(0)        # ||s r||^2
    C = (np.abs(Tt) ** 2).sum(0)                # ||t||^2
    lossj = 1.0 - np.abs(A) ** 2 / (B * C)
    loss = lossj.mean()
    # d loss / d s_i (per column), then through s = K softplus(z) / log 2
    dA = 2.0 * np.real(np.conj(A)[None, :] * np.conj(R) * Tt)
    dB = 2.0 * s * np.abs(R) ** 2
    ds = -(dA * B[None, :] - (np.abs(A) ** 2)[None, :] * dB) / (B ** 2 * C)[None, :] / ncol
    dz = ds * K / LOG2 / (1.0 + np.exp(-z))
    gw3 = np.einsum("ij,ijh->h", dz, h2)
    gb3 = dz.sum()
    da2 = dz[..., None] * w3 * dsilu(a2)
    gW2 = np.einsum("ijh,ijk->hk", da2, h1)
    gb2 = da2.sum((0, 1))
    da1 = (da2 @ W2) * dsilu(a1)
    gW1 = np.einsum("ijh,ijk->hk", da1, F)
    gb1 = da1.sum((0, 1))
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return loss, grad


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new theta, m, v."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad ** 2
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
