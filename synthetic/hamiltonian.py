"""Seeded molecule-shaped model Hamiltonians in Cholesky form.

The paper's workloads are molecules in Gaussian bases (Sec. II, II.B.2 Fig. 2,
Sec. V).  Their integrals need a quantum-chemistry code, so these generators
stand in with the same tensor shapes and structure:

* ``h1``: real symmetric M x M one-body matrix; diagonal ~ N(-2, 0.5^2),
  off-diagonal (upper triangle, mirrored) ~ N(0, s_od^2) with s_od = 0.1 at
  M = 8 and 0.05/sqrt(M) otherwise.
* ``L``: N_g real symmetric M x M Cholesky vectors (Sec. II.B.2, eq:chol),
  L_g = 0.5 exp(-g/M) (Z_g + Z_g^T) / (2 sqrt(M)), Z_g iid N(0,1), drawn in
  order after h1.  N_g = 6M mimics the paper's asymptotic N_g ~ 7M.
* ``phi``: single-determinant real trial (Sec. III.D.1), the lowest N
  eigenvectors of h1 + sum_g L_g L_g, each column signed so that its largest
  entry in modulus is positive; the same orbitals for both spins.
* ``h0`` = 0.

Everything is drawn with ``numpy.random.default_rng(seed)`` (PCG64), on the
host, so every consumer sees identical bytes.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SyntheticSystem:
    M: int
    n_up: int
    n_dn: int
    n_chol: int
    h0: float
    h1: np.ndarray          # (M, M) float64, symmetric
    L: np.ndarray           # (n_chol, M, M) float64, each symmetric
    phi_up: np.ndarray      # (M, n_up) float64
    phi_dn: np.ndarray      # (M, n_dn) float64
    meta: dict = field(default_factory=dict)


# Workload sizes.  "dtau", "n_walkers", "steps" describe the run each one is
# used for; "seed" seeds the Hamiltonian generator; "field_seed" keys the
# counter-based auxiliary-field stream.
CONFIGS = {
    "tiny": dict(M=8, N=2, n_chol=32, n_walkers=16, dtau=0.01, steps=200,
                 qr_period=5, pop_period=5, seed=1001, field_seed=0),
    "medium": dict(M=64, N=16, n_chol=320, n_walkers=512, dtau=0.005, steps=500,
                   qr_period=5, pop_period=5, seed=1002, field_seed=0),
    "large": dict(M=128, N=32, n_chol=800, n_walkers=1024, dtau=0.005, steps=1000,
                  qr_period=5, pop_period=5, seed=1003, field_seed=0),
}


def _offdiag_sigma(M: int) -> float:
    return 0.1 if M == 8 else 0.05 / np.sqrt(M)


def _trial_from(h1: np.ndarray, L: np.ndarray, n: int) -> np.ndarray:
    F = h1 + np.einsum("gpr,grq->pq", L, L)
    F = 0.5 * (F + F.T)
    _, vec = np.linalg.eigh(F)
    phi = vec[:, :n].copy()
    for j in range(n):
        k = int(np.argmax(np.abs(phi[:, j])))
        if phi[k, j] < 0:
            phi[:, j] = -phi[:, j]
    return phi


def gen_system(M: int, N: int, n_chol: int, seed: int, n_dn: int | None = None) -> SyntheticSystem:
    """Random molecule-shaped Hamiltonian with M orbitals, N electrons per spin."""
    n_dn = N if n_dn is None else n_dn
    rng = np.random.default_rng(seed)
    h1 = np.zeros((M, M))
    iu = np.triu_indices(M, k=1)
    h1[iu] = rng.normal(0.0, _offdiag_sigma(M), size=iu[0].size)
    h1 = h1 + h1.T
    h1[np.diag_indices(M)] = rng.normal(-2.0, 0.5, size=M)
    Z = rng.standard_normal((n_chol, M, M))
    scale = 0.5 * np.exp(-np.arange(n_chol) / M) / (2.0 * np.sqrt(M))
    L = (Z + Z.transpose(0, 2, 1)) * scale[:, None, None]
    phi_up = _trial_from(h1, L, N)
    phi_dn = _trial_from(h1, L, n_dn)
    return SyntheticSystem(M=M, n_up=N, n_dn=n_dn, n_chol=n_chol, h0=0.0, h1=h1, L=L,
                           phi_up=phi_up, phi_dn=phi_dn,
                           meta=dict(kind="random", seed=seed))


def config_system(name: str) -> SyntheticSystem:
    c = CONFIGS[name]
    return gen_system(c["M"], c["N"], c["n_chol"], c["seed"])


def diagonal_system(M: int, N: int, n_chol: int, seed: int, occ_up=None, occ_dn=None,
                    mix_trial: bool = False) -> SyntheticSystem:
    """Hamiltonian whose h and every L_g are diagonal in one random orthonormal basis Q.

    h = Q diag(eps) Q^T and L_g = Q diag(l_g) Q^T.  Every Q-occupation determinant is
    then an exact eigenstate, which makes the local energy of that trial a constant
    (zero-variance property, Sec. III.D.1).  ``meta`` carries Q, eps, l and the
    occupations so that tests can write the eigenvalue out in closed form.
    With ``mix_trial`` the trial columns are rotated by a random invertible N x N
    matrix (same determinant, Theorem 1.5), so the trial is not orthonormal.
    """
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((M, M)))
    eps = np.sort(rng.normal(-2.0, 0.5, size=M))
    lvals = rng.normal(0.0, 1.0, size=(n_chol, M)) * (
        0.5 * np.exp(-np.arange(n_chol) / M) / np.sqrt(M))[:, None]
    h1 = (Q * eps) @ Q.T
    h1 = 0.5 * (h1 + h1.T)
    L = np.einsum("pk,gk,qk->gpq", Q, lvals, Q)
    L = 0.5 * (L + L.transpose(0, 2, 1))
    occ_up = list(range(N)) if occ_up is None else list(occ_up)
    occ_dn = list(range(N)) if occ_dn is None else list(occ_dn)
    phi_up = Q[:, occ_up].copy()
    phi_dn = Q[:, occ_dn].copy()
    if mix_trial:
        R_up = rng.standard_normal((len(occ_up), len(occ_up))) + 2.0 * np.eye(len(occ_up))
        R_dn = rng.standard_normal((len(occ_dn), len(occ_dn))) + 2.0 * np.eye(len(occ_dn))
        phi_up = phi_up @ R_up
        phi_dn = phi_dn @ R_dn
    return SyntheticSystem(M=M, n_up=len(occ_up), n_dn=len(occ_dn), n_chol=n_chol, h0=0.0,
                           h1=h1, L=L, phi_up=phi_up, phi_dn=phi_dn,
                           meta=dict(kind="diagonal", seed=seed, Q=Q, eps=eps, lvals=lvals,
                                     occ_up=occ_up, occ_dn=occ_dn))


def random_walkers(sys: SyntheticSystem, n_walkers: int, seed: int, amplitude: float = 0.3):
    """Complex walker determinants U = Phi_T + amplitude * (random complex), per spin.

    Returns (U_up, U_dn) with shapes (n_walkers, M, n_up) and (n_walkers, M, n_dn),
    complex128.  amplitude = 0 gives copies of the trial; large amplitudes give
    determinants far from the trial (overlaps still non-zero with probability 1).
    """
    rng = np.random.default_rng(seed)
    M = sys.M

    def one(phi, n):
        z = rng.standard_normal((n_walkers, M, n)) + 1j * rng.standard_normal((n_walkers, M, n))
        return phi[None].astype(np.complex128) + amplitude * z / np.sqrt(2.0 * M)

    return one(sys.phi_up, sys.n_up), one(sys.phi_dn, sys.n_dn)
