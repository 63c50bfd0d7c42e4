"""Seeded multi-determinant trial expansions Psi_T = sum_d A_d |Psi_d> (Sec. II.B, Sec. III.D.1).

The paper's multi-determinant trials come from CASSCF or selected-CI runs on molecules; these
generators stand in with the same structure (a leading determinant plus determinants that
differ from it), for any ``SyntheticSystem``:

* ``noci_trial``: non-orthogonal determinants; determinant 0 is the lowest N eigenvectors of
  h1, determinant d > 0 rotates them into the virtual space by exp(K) with K antisymmetric,
  K[vir, occ] = angle * Z / sqrt(N), Z iid N(0,1), drawn separately for each spin.
  A_0 = 1, A_d = 0.4 N(0,1) (real).
* ``excitation_trial``: determinant 0 plus single excitations i -> a of h1's eigenvectors
  (shuffled), spin down shifted by three in the shuffled list; A_0 = 1, A_d = 0.3 N(0,1)
  + 0.1 i N(0,1).
* ``occupation_det``: the M x N matrix of unit vectors e_p for the occupied sites ``occ``.
* ``rhf_trial``: a single closed-shell determinant (Sec. III.D.1 names Hartree-Fock as the
  usual trial): the restricted Hartree-Fock orbitals of the system, by level-shifted Roothaan
  iterations from the system's own trial.

Input generation only: none of the AFQMC arithmetic (overlaps, local energies, force bias,
propagation, weights) lives here; ``rhf_trial`` solves the Hartree-Fock equations of the
system, the step that prepares a trial before any AFQMC run.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


def occupation_det(M: int, occ) -> np.ndarray:
    V = np.zeros((M, len(occ)))
    for j, p in enumerate(occ):
        V[p, j] = 1.0
    return V


def _rotation(rng, M: int, N: int, angle: float) -> np.ndarray:
    K = np.zeros((M, M))
    X = angle * rng.standard_normal((M - N, N)) / np.sqrt(N)
    K[N:, :N] = X
    K[:N, N:] = -X.T
    return scipy.linalg.expm(K)


def noci_trial(s, n_det: int, seed: int, angle: float = 0.4):
    """(coeffs (n_det,) complex, ups [n_det x (M, N_up)], dns [n_det x (M, N_dn)])."""
    rng = np.random.default_rng(seed)
    _, C = np.linalg.eigh(s.h1)
    M, nu, nd = s.M, s.n_up, s.n_dn
    ups, dns = [C[:, :nu].copy()], [C[:, :nd].copy()]
    for _ in range(n_det - 1):
        ups.append(C @ _rotation(rng, M, nu, angle)[:, :nu])
        dns.append(C @ _rotation(rng, M, nd, angle)[:, :nd])
    coeffs = np.concatenate([[1.0], 0.4 * rng.standard_normal(n_det - 1)]) + 0j
    return coeffs, ups, dns


def excitation_trial(s, n_det: int, seed: int):
    """Leading determinant plus single excitations (same number of electrons per spin)."""
    rng = np.random.default_rng(seed)
    _, C = np.linalg.eigh(s.h1)
    N = s.n_up
    cands = []
    for i in range(N):
        for a in range(N, s.M):
            occ = list(range(N))
            occ[i] = a
            cands.append(sorted(occ))
    rng.shuffle(cands)
    lead = list(range(N))
    ups, dns = [C[:, lead]], [C[:, lead]]
    for k in range(n_det - 1):
        ups.append(C[:, cands[k]])
        dns.append(C[:, cands[(k + 3) % len(cands)]])
    coeffs = np.concatenate([[1.0], 0.3 * rng.standard_normal(n_det - 1)]) + 0j
    coeffs[1:] += 0.1j * rng.standard_normal(n_det - 1)
    return coeffs, ups, dns


def rhf_trial(s, shift: float = 0.5, tol: float = 1e-12, max_iter: int = 1000):
    """Restricted Hartree-Fock orbitals (M, N) of a closed-shell system (n_up == n_dn = N).

    With the per-spin density P = C C^T the energy is 2 tr(h P) + 2 sum_g (tr L_g P)^2
    - sum_g tr(L_g P L_g P) and its Fock matrix F = h + 2 sum_g tr(L_g P) L_g - sum_g L_g P L_g;
    each iteration takes the N lowest eigenvectors of F + shift (1 - P) (the level shift damps
    the iteration), starting from s.phi_up, until the energy changes by less than tol.  Returns
    (C, energy, iterations)."""
    assert s.n_up == s.n_dn
    M, N = s.M, s.n_up
    C = np.array(s.phi_up, dtype=np.float64)
    C, _ = np.linalg.qr(C)
    e_old = np.inf
    for it in range(1, max_iter + 1):
        P = C @ C.T
        tg = np.einsum("grs,rs->g", s.L, P)
        F = s.h1 + 2.0 * np.einsum("g,gpq->pq", tg, s.L) - np.einsum("gpr,rs,gsq->pq", s.L, P, s.L)
        e = float(s.h0 + np.sum(P * (s.h1 + F)))
        if abs(e - e_old) < tol:
            return C, e, it
        e_old = e
        _, vec = np.linalg.eigh(F + shift * (np.eye(M) - P))
        C = vec[:, :N]
    raise RuntimeError("rhf_trial: no convergence")
