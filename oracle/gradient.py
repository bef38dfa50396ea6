"""Derivatives of a field given by its coefficients (App. C).

Test infrastructure (see the package docstring); plain FP64 NumPy/SciPy.

E(theta1, theta2, r) = sum_i e_i F_i with the helical waves F_i (App. B).
App. C obtains the derivatives in helical coordinates as inverse transforms:
E_theta1 of the coefficients (i 2 pi m) e_i, E_theta2 of (i 2 pi N n) e_i
(eq. Derivative_of_energy_wrt_theta) and E_r with the radial functions
replaced by their r-derivatives (eqs. E_r and B_r); the Cartesian gradient
then follows by the chain rule (eq. Cartesian_Derivatives).  Here the radial
derivative is scipy's Bessel derivative (jvp), not the paper's recurrence, so
that it pins the GPU path's table independently.  Arrays have shape
(N_theta1, N_theta2, N_r[, nv]) as in transforms.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special as sp

from .basis import Basis, bessel_zeros
from .transforms import _mode_axes, inverse_separable


def radial_derivative(b: Basis, n: int, k: np.ndarray, r: np.ndarray | None = None) -> np.ndarray:
    """d xi_{n,k}/dr on the radial grid (or at ``r``), shape (len(r), len(k))."""
    rr = b.r if r is None else np.asarray(r, dtype=np.float64)
    k = np.asarray(k, dtype=np.int64)
    p = b.order(n)
    bz = bessel_zeros(p, int(k.max()))[k - 1]
    c = math.sqrt(b.ncyc / (math.pi * b.tau)) / (b.R * sp.jv(p + 1, bz))
    return sp.jvp(p, np.outer(rr, bz) / b.R) * (c * bz / b.R)[None, :]


def helical_derivatives(b: Basis, X: np.ndarray):
    """(E_theta1, E_theta2, E_r) on the grid for the coefficient block X (L, nv)."""
    X = np.asarray(X, dtype=np.complex128)
    single = X.ndim == 1
    X = X[:, None] if single else X
    m = b.mnk[:, 0].astype(np.float64)[:, None]
    n = b.mnk[:, 1].astype(np.float64)[:, None]
    e1 = inverse_separable(b, (2j * math.pi * m) * X)
    e2 = inverse_separable(b, (2j * math.pi * b.ncyc * n) * X)
    # E_r: the separated sums of Sec. 3.4 with d xi / dr as the radial factor
    nv = X.shape[1]
    ms, ns, im, inn = _mode_axes(b)
    kmax = int(b.mnk[:, 2].max())
    box = np.zeros((ms.size, ns.size, kmax, nv), dtype=np.complex128)
    box[im, inn, b.mnk[:, 2] - 1, :] = X
    G = np.zeros((ms.size, ns.size, b.n_r, nv), dtype=np.complex128)
    for j, nn in enumerate(ns):
        tab = radial_derivative(b, int(nn), np.arange(1, kmax + 1))     # (nr, kmax)
        G[:, j] = np.einsum("lk,mkv->mlv", tab, box[:, j])
    a1 = np.exp(2j * math.pi * np.outer(b.theta1, ms))
    a2 = np.exp(2j * math.pi * b.ncyc * np.outer(b.theta2, ns))
    er = np.einsum("jn,inlv->ijlv", a2, np.einsum("im,mnlv->inlv", a1, G))
    if single:
        return e1[..., 0], e2[..., 0], er[..., 0]
    return e1, e2, er


def cartesian(b: Basis, e1: np.ndarray, e2: np.ndarray, er: np.ndarray):
    """(E_x, E_y, E_z) from the helical derivatives (eq. Cartesian_Derivatives):
    with phi = 2 pi (alpha theta1 + theta2), E_x = -sin(phi) E_theta2 / (2 pi r)
    + cos(phi) E_r, E_y = cos(phi) E_theta2 / (2 pi r) + sin(phi) E_r,
    E_z = (E_theta1 - alpha E_theta2) / tau."""
    shape = (b.n_t1, b.n_t2, b.n_r)
    phi = np.broadcast_to(2.0 * math.pi * (b.alpha * b.theta1[:, None, None] + b.theta2[None, :, None]), shape)
    rr = np.broadcast_to(b.r[None, None, :], shape)
    extra = (slice(None),) * 3 + (None,) * (e1.ndim - 3)
    s, c, rr = np.sin(phi)[extra], np.cos(phi)[extra], rr[extra]
    ex = -s * e2 / (2.0 * math.pi * rr) + c * er
    ey = c * e2 / (2.0 * math.pi * rr) + s * er
    ez = (e1 - b.alpha * e2) / b.tau
    return ex, ey, ez
