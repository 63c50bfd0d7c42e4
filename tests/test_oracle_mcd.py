"""Modified Cholesky decomposition (Sec. II.B.2) in the oracle: the residual bound, exact rank
recovery, and the cost/accuracy trade-off of the threshold."""

import numpy as np

from oracle import fock as F
from oracle.mcd import eri_matrix, modified_cholesky
from synthetic import gen_system


def _molecule_like_eri(M, seed, n=None):
    """A positive semidefinite tensor with a decaying spectrum, v = sum_k w_k B^k (x) B^k."""
    rng = np.random.default_rng(seed)
    n = n or M * M
    B = rng.standard_normal((n, M, M))
    B = B + B.transpose(0, 2, 1)
    w = np.exp(-np.arange(n) / (0.8 * M)) / M
    return np.einsum("k,kpr,kqs->pqrs", w, B, B)


def test_residual_bounded_by_threshold():
    """After termination every element of V - sum L L^T is at most delta (Cauchy-Schwarz)."""
    eri = _molecule_like_eri(8, 1)
    V = eri_matrix(eri)
    for delta in (1e-2, 1e-4, 1e-6):
        L, piv = modified_cholesky(eri, delta)
        R = V - np.einsum("gm,gn->mn", L.reshape(len(L), -1), L.reshape(len(L), -1))
        assert np.abs(R).max() <= delta * (1 + 1e-9)
        assert len(set(piv)) == len(piv)


def test_fewer_vectors_for_looser_threshold():
    eri = _molecule_like_eri(10, 2)
    n = [len(modified_cholesky(eri, d)[0]) for d in (1e-2, 1e-4, 1e-6, 1e-8)]
    assert n == sorted(n) and n[0] < n[-1] < 100


def test_exact_rank_is_recovered():
    """A tensor built from G Cholesky vectors has rank <= G: at most G vectors are needed, and
    they reproduce v_pqrs and the Fock-space Hamiltonian to the threshold."""
    s = gen_system(6, 2, 7, seed=3)
    eri = F.eri_from_cholesky(s.L)
    L, _ = modified_cholesky(eri, 1e-12)
    assert len(L) <= 7
    assert np.abs(F.eri_from_cholesky(L) - eri).max() < 1e-11
    for g in range(len(L)):
        assert np.abs(L[g] - L[g].T).max() < 1e-12   # symmetric like the input vectors
    fs = F.FockSpace(6, 2, 2)
    H1 = fs.hamiltonian(0.0, s.h1, eri)
    H2 = fs.hamiltonian(0.0, s.h1, F.eri_from_cholesky(L))
    assert np.abs(H1 - H2).max() < 1e-10


def test_prescreening_zeroes_tiny_diagonals():
    """Diagonal entries with sqrt(|D_mu| D_max) <= min(1e-9, delta) are never pivots."""
    s = gen_system(5, 2, 3, seed=4)
    eri = F.eri_from_cholesky(s.L)
    eri[0, 0, 0, 0] += 1e-22     # an (essentially) empty direction stays out
    L, piv = modified_cholesky(eri, 1e-14)
    assert len(L) <= 3
