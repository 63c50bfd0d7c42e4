"""Weighted reblocking error analysis (App. C), test infrastructure only.

Samples are the per-step weighted averages (w_i, x_i): w_i = sum of walker
weights, x_i = the mixed estimate at step i.  Blocks of length L give
w'_b = sum w_i and x'_b = sum w_i x_i / w'_b; then
X = sum w'_b x'_b / v1 and S^2 = sum w'_b (x'_b - X)^2 / (v1 - v2/v1) with
v_l = sum (w'_b)^l.  The standard error of the mean is S / sqrt(N_b - 1) and
2 S / sqrt(N_b - 1) is the 95% bound.
"""

from __future__ import annotations

import numpy as np


def reblock(x, w, L: int):
    """Weighted blocked mean, spread S and standard error for block length L."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    nb = x.size // L
    if nb < 2:
        raise ValueError("reblock: need at least two blocks")
    xb = x[: nb * L].reshape(nb, L)
    wb = w[: nb * L].reshape(nb, L)
    wp = wb.sum(axis=1)
    xp = (wb * xb).sum(axis=1) / wp
    v1 = wp.sum()
    v2 = (wp * wp).sum()
    X = (wp * xp).sum() / v1
    S2 = (wp * (xp - X) ** 2).sum() / (v1 - v2 / v1)
    S = float(np.sqrt(S2))
    return float(X), S, S / np.sqrt(nb - 1), nb


def reblock_converged(x, w, discard: int = 200, min_blocks: int = 16, ratio: float = 1.1):
    """Discard the equilibration samples, then double L until the standard error
    stops growing by more than ``ratio`` (saturation of S with L).

    Returns (mean, stderr, L, converged).  With too few samples for two
    sizes with ``min_blocks`` blocks, the last estimate is returned unconverged.
    """
    x = np.asarray(x, dtype=np.float64)[discard:]
    w = np.asarray(w, dtype=np.float64)[discard:]
    L = 1
    prev = None
    while x.size // L >= min_blocks:
        X, S, err, nb = reblock(x, w, L)
        if prev is not None and err <= ratio * prev[1]:
            return X, err, L, True
        prev = (X, err, L)
        L *= 2
    if prev is None:
        X, S, err, nb = reblock(x, w, 1)
        return X, err, 1, False
    return prev[0], prev[1], prev[2], False
