"""Seeded random coefficient blocks keyed by (m, n, k).

The value drawn for a given (m, n, k) row does not depend on the order in
which the caller lists its rows, so two codes that store the same index set in
different orders receive the same vectors.
"""
from __future__ import annotations

import numpy as np


def random_block(mnk, nvec: int, seed: int, normalize: bool = True) -> np.ndarray:
    """Complex128 array of shape (len(mnk), nvec): standard normal real and
    imaginary parts, drawn in lexicographic (m, n, k) order from PCG64(seed)
    and returned in the row order of ``mnk``; columns scaled to unit 2-norm
    when ``normalize``."""
    mnk = np.asarray(mnk, dtype=np.int64).reshape(-1, 3)
    L = mnk.shape[0]
    order = np.lexsort((mnk[:, 2], mnk[:, 1], mnk[:, 0]))
    rng = np.random.Generator(np.random.PCG64(seed))
    draws = rng.standard_normal((L, nvec)) + 1j * rng.standard_normal((L, nvec))
    out = np.empty((L, nvec), dtype=np.complex128)
    out[order] = draws
    if normalize and L > 0:
        out /= np.linalg.norm(out, axis=0, keepdims=True)
    return out
