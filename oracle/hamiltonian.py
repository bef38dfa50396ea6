"""The discrete helical-wave Hamiltonian at nu = 0 (Alg. 5 with the 1/r^2
block absent), as a dense matrix and as a matrix-free apply.

Test infrastructure (see the package docstring); plain FP64 NumPy/SciPy.

The operator on coefficient vectors is

    H x = kappa * x + Fwd(V * Inv(x)),

where Inv is the inverse basis transform onto the grid, V the real potential
sampled on the grid, and Fwd the quadrature forward transform (eqs.
Simplify_2, g_mnk; Alg. 5).  ``V`` arrays have shape (N_theta1, N_theta2,
N_r) in the real-space storage order.

Three evaluations of the same operator:
* mode A  ``dense_explicit``: H = diag(kappa) + B^H diag(W V) B with the
  explicit basis matrix B (eq. Naive_Inverse_Transform, eq.
  Fast_fwd_transform_cont);
* mode B  ``dense_dft``: the same matrix from the normalised 2D DFT of V at
  each radius, H_ij = kappa_i delta_ij + (2 pi tau/N) sum_l omega_l
  xi_i(r_l) xi_j(r_l) Vhat_l[(m_i - m_j) mod N_theta1, (n_i - n_j) mod
  N_theta2] (orthogonality of the discrete exponentials);
* mode C  ``apply``: matrix-free, with the separated sums of Sec. 3.4.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .basis import Basis
from .transforms import (basis_matrix, grid_weights, radial_values,
                         inverse_separable, forward_separable)


def dense_explicit(b: Basis, V: np.ndarray, B: np.ndarray | None = None) -> np.ndarray:
    B = basis_matrix(b) if B is None else B
    wv = (grid_weights(b) * V).reshape(-1)
    H = B.conj().T @ (wv[:, None] * B)
    H[np.diag_indices_from(H)] += b.kappa
    return H


def dense_dft(b: Basis, V: np.ndarray) -> np.ndarray:
    rad = radial_values(b)                                      # (nr, L)
    Vhat = np.fft.fft2(V, axes=(0, 1)) / (b.n_t1 * b.n_t2)      # (n1, n2, nr)
    dm = (b.mnk[:, 0][:, None] - b.mnk[:, 0][None, :]) % b.n_t1
    dn = (b.mnk[:, 1][:, None] - b.mnk[:, 1][None, :]) % b.n_t2
    pref = 2.0 * math.pi * b.tau / b.ncyc
    H = np.zeros((b.L, b.L), dtype=np.complex128)
    for l in range(b.n_r):
        H += (pref * b.omega_r[l]) * np.outer(rad[l], rad[l]) * Vhat[dm, dn, l]
    H[np.diag_indices_from(H)] += b.kappa
    return H


def potential_diagonal(b: Basis, V: np.ndarray) -> np.ndarray:
    """V_ii: the diagonal of the potential term, i.e. mode B at m_i = m_j,
    n_i = n_j, where the DFT coefficient is the angular mean of V."""
    rad = radial_values(b)                                      # (nr, L)
    vbar = V.mean(axis=(0, 1))                                  # (nr,)
    pref = 2.0 * math.pi * b.tau / b.ncyc
    return pref * ((b.omega_r * vbar)[:, None] * rad ** 2).sum(0)


def apply(b: Basis, V: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Matrix-free H @ X for X of shape (L,) or (L, nv)."""
    single = X.ndim == 1
    XX = X[:, None] if single else X
    g = inverse_separable(b, XX)
    Y = forward_separable(b, g * V[..., None]) + b.kappa[:, None] * XX
    return Y[:, 0] if single else Y


def lowest(H: np.ndarray, nev: int):
    """Lowest ``nev`` eigenpairs of a Hermitian matrix (LAPACK, subset)."""
    w, v = sla.eigh(H, subset_by_index=[0, nev - 1], driver="evr")
    return w, v
