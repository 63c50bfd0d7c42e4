"""Modified Cholesky decomposition of the two-electron tensor (Sec. II.B.2, eq:chol,
eq:chol2) -- test infrastructure only.

The tensor v_pqrs of real orbitals is reshaped into the symmetric positive
semidefinite matrix V_{mu nu} with mu = (p, r) and nu = (q, s), so that
v_pqrs = sum_g L^g_pr L^g_qs once V = sum_g L^g (L^g)^T.  Starting from the
residual Delta = V, each iteration

1. takes the largest residual diagonal element Delta_max = Delta_{nu0 nu0}
   (first index on ties);
2. stops when Delta_max < delta;
3. zeroes the rows and columns mu whose diagonal satisfies
   sqrt(|Delta_mu mu| Delta_max) <= min(1e-9, delta) (damped prescreening);
4. appends L_mu = Delta_{mu nu0} / sqrt(Delta_max) and subtracts L L^T from Delta.

Every residual element is then bounded by delta (Cauchy-Schwarz on the
positive semidefinite residual).  The residual matrix is kept in full here,
as written in the paper; the GPU library keeps only its diagonal.
"""

from __future__ import annotations

import math

import numpy as np


def eri_matrix(eri: np.ndarray) -> np.ndarray:
    """V_{(p r), (q s)} = v_pqrs for v stored as eri[p, q, r, s]."""
    M = eri.shape[0]
    return eri.transpose(0, 2, 1, 3).reshape(M * M, M * M)


def modified_cholesky(eri: np.ndarray, delta: float, max_vectors: int | None = None):
    """Cholesky vectors L (n, M, M) with v_pqrs ~ sum_g L^g_pr L^g_qs, and the list of pivots."""
    M = eri.shape[0]
    V = eri_matrix(np.asarray(eri, dtype=np.float64))
    Delta = V.copy()
    n_max = M * M if max_vectors is None else max_vectors
    vecs, pivots = [], []
    screen = min(1e-9, delta)
    while len(vecs) < n_max:
        diag = np.diag(Delta).copy()
        nu0 = int(np.argmax(diag))
        dmax = float(diag[nu0])
        if dmax < delta:
            break
        dead = np.sqrt(np.abs(diag) * dmax) <= screen
        Delta[dead, :] = 0.0
        Delta[:, dead] = 0.0
        Lvec = Delta[:, nu0] / math.sqrt(dmax)
        Delta = Delta - np.outer(Lvec, Lvec)
        vecs.append(Lvec.reshape(M, M))
        pivots.append(nu0)
    if not vecs:
        return np.zeros((0, M, M)), pivots
    return np.array(vecs), pivots
