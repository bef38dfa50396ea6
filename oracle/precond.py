"""Teter-Payne-Allan diagonal preconditioner (Sec. 3.5).

Test infrastructure (see the package docstring); plain FP64 NumPy.

For a residual column r_j the preconditioned vector is w_ij = K(g_ij) r_ij
with K(g) = (27 + 18 g + 12 g^2 + 8 g^3) / (27 + 18 g + 12 g^2 + 8 g^3 +
16 g^4) and g_ij = (kinetic energy of basis function i) / (kinetic energy of
the residual j).  Reading of the silent part: the kinetic energy of basis
function i is the (Bloch-shifted) kinetic diagonal kappa_i, and that of the
residual is the Rayleigh quotient T_j = sum_i kappa_i |r_ij|^2 / sum_i
|r_ij|^2; a zero residual column is returned unchanged (zero).
"""
from __future__ import annotations

import numpy as np


def tpa_factor(g):
    g = np.asarray(g, dtype=np.float64)
    num = 27.0 + 18.0 * g + 12.0 * g ** 2 + 8.0 * g ** 3
    return num / (num + 16.0 * g ** 4)


def residual_kinetic_energy(kappa, Rres):
    Rres = np.asarray(Rres)
    R2 = np.abs(Rres if Rres.ndim == 2 else Rres[:, None]) ** 2
    den = R2.sum(axis=0)
    num = (np.asarray(kappa)[:, None] * R2).sum(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        T = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    return T


def tpa_apply(kappa, Rres):
    """Preconditioned residual block, same shape as ``Rres``."""
    Rres = np.asarray(Rres)
    single = Rres.ndim == 1
    RR = Rres[:, None] if single else Rres
    T = residual_kinetic_energy(kappa, RR)
    out = np.zeros_like(RR)
    for j in range(RR.shape[1]):
        if T[j] > 0:
            out[:, j] = tpa_factor(np.asarray(kappa) / T[j]) * RR[:, j]
    return out[:, 0] if single else out
