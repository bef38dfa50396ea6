"""Basis transforms between coefficients and the real-space grid.

Test infrastructure (see the package docstring); plain FP64 NumPy.

Real-space arrays have shape (N_theta1, N_theta2, N_r): theta1 outermost,
then theta2, then r fastest (eq. wavefun_storage_real).  Coefficient vectors
follow the basis' index list ``b.mnk``.

Two independent evaluations of the same discrete transforms are given:

* ``basis_matrix`` -- every basis function at every grid point, so that the
  inverse transform is the naive sum of eq. Naive_Inverse_Transform
  (B @ x) and the forward transform is the quadrature of eq.
  Fast_fwd_transform_cont (B^H @ (W * g));
* ``inverse_separable`` / ``forward_separable`` -- the separated sums of
  Sec. 3.4: G_{m,n}(r) = sum_k g_{m,n,k} xi_{n,k}(r), then the double sum
  over (m, n) of exp(+i 2 pi (m theta1 + n N theta2)) G_{m,n}(r); and for the
  forward direction H_{m,n}(r) = (1/(N_theta1 N_theta2)) sum over the angular
  grid of g exp(-i 2 pi (...)), then (2 pi tau/N) sum_r omega_r xi H
  (eqs. Fast_fwd_transform_cont_3 and _2).  The angular sums are explicit
  exponential matrices, not FFTs.
"""
from __future__ import annotations

import math

import numpy as np

from .basis import Basis


def grid_weights(b: Basis) -> np.ndarray:
    """Quadrature weight of every grid point, shape (N_theta1, N_theta2, N_r)."""
    return np.broadcast_to(b.grid_weight * b.omega_r[None, None, :],
                           (b.n_t1, b.n_t2, b.n_r)).copy()


def radial_values(b: Basis) -> np.ndarray:
    """xi_{n_i,k_i}(r_l) for every index i, shape (N_r, L)."""
    out = np.empty((b.n_r, b.L))
    for n in np.unique(b.mnk[:, 1]):
        sel = np.nonzero(b.mnk[:, 1] == n)[0]
        out[:, sel] = b.xi(int(n), b.mnk[sel, 2])
    return out


def basis_matrix(b: Basis) -> np.ndarray:
    """B[g, i] = F_i(grid point g), g flattened in (theta1, theta2, r) order,
    shape (N_theta1 * N_theta2 * N_r, L)."""
    m = b.mnk[:, 0].astype(np.float64)
    n = b.mnk[:, 1].astype(np.float64)
    e1 = np.exp(2j * math.pi * np.outer(b.theta1, m))               # (n1, L)
    e2 = np.exp(2j * math.pi * b.ncyc * np.outer(b.theta2, n))      # (n2, L)
    rad = radial_values(b)                                          # (nr, L)
    B = e1[:, None, None, :] * e2[None, :, None, :] * rad[None, None, :, :]
    return B.reshape(b.n_t1 * b.n_t2 * b.n_r, b.L)


def inverse_naive(b: Basis, x: np.ndarray, B: np.ndarray | None = None) -> np.ndarray:
    """g = sum_i x_i F_i on the grid; x of shape (L,) or (L, nv)."""
    B = basis_matrix(b) if B is None else B
    g = B @ x
    return g.reshape((b.n_t1, b.n_t2, b.n_r) + x.shape[1:])


def forward_naive(b: Basis, g: np.ndarray, B: np.ndarray | None = None) -> np.ndarray:
    """x_i = sum_g W_g conj(F_i(g)) g(g) (quadrature of <g, F_i>)."""
    B = basis_matrix(b) if B is None else B
    W = grid_weights(b).reshape(-1)
    gg = g.reshape((b.n_t1 * b.n_t2 * b.n_r,) + g.shape[3:])
    Wg = gg * (W if gg.ndim == 1 else W[:, None])
    return B.conj().T @ Wg


def _mode_axes(b: Basis):
    ms = np.arange(b.mnk[:, 0].min(), b.mnk[:, 0].max() + 1)
    ns = np.arange(b.mnk[:, 1].min(), b.mnk[:, 1].max() + 1)
    im = b.mnk[:, 0] - ms[0]
    inn = b.mnk[:, 1] - ns[0]
    return ms, ns, im, inn


def inverse_separable(b: Basis, x: np.ndarray) -> np.ndarray:
    """Inverse transform by the separated sums of Sec. 3.4 (see module doc).
    x of shape (L,) or (L, nv); returns (N_theta1, N_theta2, N_r[, nv])."""
    single = x.ndim == 1
    X = x[:, None] if single else x
    nv = X.shape[1]
    ms, ns, im, inn = _mode_axes(b)
    kmax = int(b.mnk[:, 2].max())
    # coefficient box g[m, n, k] with zeros outside the cutoff mask
    box = np.zeros((ms.size, ns.size, kmax, nv), dtype=np.complex128)
    box[im, inn, b.mnk[:, 2] - 1, :] = X
    # G_{m,n}(r) = sum_k g_{m,n,k} xi_{n,k}(r)
    G = np.zeros((ms.size, ns.size, b.n_r, nv), dtype=np.complex128)
    for j, n in enumerate(ns):
        tab = b.xi(int(n), np.arange(1, kmax + 1))                    # (nr, kmax)
        G[:, j] = np.einsum("lk,mkv->mlv", tab, box[:, j])
    e1 = np.exp(2j * math.pi * np.outer(b.theta1, ms))                # (n1, nm)
    e2 = np.exp(2j * math.pi * b.ncyc * np.outer(b.theta2, ns))       # (n2, nn)
    g = np.einsum("im,mnlv->inlv", e1, G)
    g = np.einsum("jn,inlv->ijlv", e2, g)
    return g[..., 0] if single else g


def forward_separable(b: Basis, g: np.ndarray) -> np.ndarray:
    """Forward transform by the separated sums of Sec. 3.4 (see module doc).
    g of shape (N_theta1, N_theta2, N_r[, nv]); returns (L[, nv])."""
    single = g.ndim == 3
    gg = g[..., None] if single else g
    ms, ns, im, inn = _mode_axes(b)
    kmax = int(b.mnk[:, 2].max())
    e1 = np.exp(-2j * math.pi * np.outer(b.theta1, ms))
    e2 = np.exp(-2j * math.pi * b.ncyc * np.outer(b.theta2, ns))
    # H_{m,n}(r) = 1/(N1 N2) sum_{i,j} g exp(-i 2 pi (m theta1_i + n N theta2_j))
    H = np.einsum("im,ijlv->mjlv", e1, gg)
    H = np.einsum("jn,mjlv->mnlv", e2, H) / (b.n_t1 * b.n_t2)
    out = np.zeros((b.L, gg.shape[3]), dtype=np.complex128)
    pref = 2.0 * math.pi * b.tau / b.ncyc
    for j, n in enumerate(ns):
        sel = np.nonzero(inn == j)[0]
        if sel.size == 0:
            continue
        tab = b.xi(int(n), np.arange(1, kmax + 1)) * b.omega_r[:, None]   # (nr, kmax)
        full = pref * np.einsum("lk,mlv->mkv", tab, H[:, j])             # (nm, kmax, nv)
        out[sel] = full[im[sel], b.mnk[sel, 2] - 1]
    return out[:, 0] if single else out
