"""Electron density on the real-space grid (Sec. 4.2, the density equation).

Test infrastructure (see the package docstring); plain FP64 NumPy.

For one Bloch parameter eta_b and cyclic index nu the equation's summand is
w_b s_j |phi_j|^2 times 2 / N (N the cyclic order); the caller folds these
factors into one weight per state, occ_j = (2 / N) w_b s_j, and sums the
results over (eta_b, nu).  phi_j is the inverse basis transform of the
coefficient column x_j onto the grid (the separated sums of Sec. 3.4, see
transforms.inverse_separable).  Arrays have shape (N_theta1, N_theta2, N_r):
theta1 outermost, r fastest, as the potential.
"""
from __future__ import annotations

import numpy as np

from .basis import Basis
from .transforms import inverse_separable


def density(b: Basis, X: np.ndarray, occ: np.ndarray) -> np.ndarray:
    """rho = sum_j occ_j |Inv(x_j)|^2 on the grid; X of shape (L, nv), occ (nv,)."""
    X = np.asarray(X, dtype=np.complex128)
    if X.ndim == 1:
        X = X[:, None]
    occ = np.asarray(occ, dtype=np.float64)
    g = inverse_separable(b, X)                       # (N1, N2, Nr, nv)
    rho = np.zeros((b.n_t1, b.n_t2, b.n_r))
    for j in range(X.shape[1]):
        rho += occ[j] * (g[..., j].real ** 2 + g[..., j].imag ** 2)
    return rho
