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

``dense_dft_modes`` evaluates mode B's formula for the whole matrix one pair
of angular modes at a time (each mode's rows are contiguous in the paper's
storage order), so that a mid-size basis (tens of thousands of functions)
fits in memory; ``lowest_values`` returns the lowest eigenvalues only.
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


def dense_dft_modes(b: Basis, V: np.ndarray) -> np.ndarray:
    """Mode B, H_ij = kappa_i delta_ij + (2 pi tau/N) sum_l omega_l xi_i(r_l)
    xi_j(r_l) Vhat_l[(m_i - m_j) mod N_theta1, (n_i - n_j) mod N_theta2],
    filled block by block: for the rows of mode (m_a, n_a) (k = 1..K_a) and
    the columns of mode (m_b, n_b) the block is the matrix product
    Xi_a^T diag(c_l Vhat_l[m_a - m_b, n_a - n_b]) Xi_b over the radial index
    l, with Xi_n[l, k] = xi_{n,k}(r_l) and c_l = (2 pi tau/N) omega_l.  The
    products for all m differences of one pair (n_a, n_b) are taken together.
    Same sum as ``dense_dft``; no arrays of size L^2 besides H."""
    Vhat = np.fft.fft2(V, axes=(0, 1)) / (b.n_t1 * b.n_t2)      # (n1, n2, nr)
    c = (2.0 * math.pi * b.tau / b.ncyc) * b.omega_r             # (nr,)
    m_all, n_all, k_all = b.mnk[:, 0], b.mnk[:, 1], b.mnk[:, 2]
    # modes (m, n) with their first row and K: the rows of one mode are
    # consecutive, k = 1..K (paper storage order, cutoff prefix in k)
    start = np.nonzero((k_all == 1))[0]
    modes_by_n: dict[int, list[tuple[int, int, int]]] = {}
    for r0 in start:
        m, n = int(m_all[r0]), int(n_all[r0])
        K = 1
        while r0 + K < b.L and k_all[r0 + K] == K + 1 and m_all[r0 + K] == m and n_all[r0 + K] == n:
            K += 1
        modes_by_n.setdefault(n, []).append((m, int(r0), K))
    xi = {}
    for n, lst in modes_by_n.items():
        kmax = max(K for _, _, K in lst)
        xi[n] = b.xi(n, np.arange(1, kmax + 1))                   # (nr, Kmax_n)
    H = np.zeros((b.L, b.L), dtype=np.complex128)
    for na, la in modes_by_n.items():
        Xa = xi[na]
        for nb, lb in modes_by_n.items():
            Xb = xi[nb]
            dms = sorted({ma - mb for ma, _, _ in la for mb, _, _ in lb})
            coef = np.stack([c * Vhat[dm % b.n_t1, (na - nb) % b.n_t2, :] for dm in dms])  # (d, nr)
            A = Xa.T[None, :, :] * coef[:, None, :]                # (d, Ka, nr)
            blk = (A.reshape(-1, b.n_r) @ Xb).reshape(len(dms), Xa.shape[1], Xb.shape[1])
            where = {dm: i for i, dm in enumerate(dms)}
            for ma, ra, Ka in la:
                for mb, rb, Kb in lb:
                    H[ra:ra + Ka, rb:rb + Kb] = blk[where[ma - mb], :Ka, :Kb]
    H[np.diag_indices_from(H)] += b.kappa
    return H


def lowest_values(H: np.ndarray, nev: int) -> np.ndarray:
    """Lowest ``nev`` eigenvalues of a Hermitian matrix (LAPACK zheevr on its
    lower triangle, subset by index); H is overwritten."""
    return sla.eigh(H, subset_by_index=[0, nev - 1], driver="evr", eigvals_only=True,
                    overwrite_a=True, check_finite=False)


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
