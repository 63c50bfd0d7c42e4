"""Brute-force second quantization on a tiny Fock sector (test infrastructure only).

Spin orbitals are numbered (p, up) -> p and (p, down) -> M + p.  A basis state
is an occupation bit string n; its vector is a+_{i1} a+_{i2} ... a+_{ik} |0>
with i1 < i2 < ... < ik.  Then a_i |n> = (-1)^{sum_{j<i} n_j} |n - e_i> when
n_i = 1 and zero otherwise, and a+_i is the transpose of a_i.  Everything here
is built from these operator matrices alone -- no determinant formulas -- so
that it can pin the determinant algebra of ``oracle.afqmc`` (Theorem 1,
eq:localenergy2/3) and the Hubbard-Stratonovich / Thouless propagation
(eq:hs, Theorem 1.4) on systems small enough for exact diagonalization.
"""

from __future__ import annotations

from functools import lru_cache
from itertools import combinations

import numpy as np


class FockSpace:
    """All sectors (a, b) with a <= n_up up and b <= n_dn down electrons on M orbitals."""

    def __init__(self, M: int, n_up: int, n_dn: int):
        self.M = M
        self.n_up = n_up
        self.n_dn = n_dn
        self.states = {}
        self.index = {}
        for a in range(n_up + 1):
            for b in range(n_dn + 1):
                sts = []
                for up in combinations(range(M), a):
                    for dn in combinations(range(M), b):
                        bits = 0
                        for p in up:
                            bits |= 1 << p
                        for p in dn:
                            bits |= 1 << (M + p)
                        sts.append(bits)
                sts.sort()
                self.states[(a, b)] = sts
                self.index[(a, b)] = {s: i for i, s in enumerate(sts)}

    def dim(self, sector):
        return len(self.states[sector])

    @lru_cache(maxsize=None)
    def annihilator(self, i: int, sector: tuple) -> np.ndarray:
        """Matrix of a_i from ``sector`` to the sector with one electron fewer of that spin."""
        a, b = sector
        spin_up = i < self.M
        target = (a - 1, b) if spin_up else (a, b - 1)
        src = self.states[sector]
        out = np.zeros((self.dim(target), len(src)))
        if target[0] < 0 or target[1] < 0:
            return out
        tix = self.index[target]
        below = (1 << i) - 1
        for col, n in enumerate(src):
            if n >> i & 1:
                sign = -1.0 if bin(n & below).count("1") % 2 else 1.0
                out[tix[n ^ (1 << i)], col] = sign
        return out

    def creator(self, i: int, sector: tuple) -> np.ndarray:
        """Matrix of a+_i from ``sector`` to the sector with one more electron of that spin."""
        a, b = sector
        up = self.annihilator(i, (a + 1, b) if i < self.M else (a, b + 1))
        return up.T

    # ----- states ---------------------------------------------------------

    def slater(self, U_up: np.ndarray, U_dn: np.ndarray) -> np.ndarray:
        """Vector of a+_{u1} ... a+_{u N_up} a+_{v1} ... a+_{v N_dn} |0> with
        a+_u = sum_p U_pk a+_{p sigma} (Sec. II.A, eq:SDdef), built by applying
        the creation operators one by one to the vacuum."""
        orbs = [(0, U_up[:, k]) for k in range(U_up.shape[1])] + \
               [(1, U_dn[:, k]) for k in range(U_dn.shape[1])]
        vec = np.ones(1, dtype=np.complex128)
        sector = (0, 0)
        for spin, coef in reversed(orbs):
            new_sector = (sector[0] + 1, sector[1]) if spin == 0 else (sector[0], sector[1] + 1)
            new = np.zeros(self.dim(new_sector), dtype=np.complex128)
            for p in range(self.M):
                if coef[p] != 0:
                    new += coef[p] * (self.creator(p + spin * self.M, sector) @ vec)
            vec = new
            sector = new_sector
        return vec

    # ----- operators on the full (n_up, n_dn) sector ------------------------

    @property
    def full(self):
        return (self.n_up, self.n_dn)

    def one_body(self, A_up: np.ndarray, A_dn: np.ndarray | None = None) -> np.ndarray:
        """Matrix of sum_{pq sigma} A^sigma_pq a+_{p sigma} a_{q sigma} on the full sector."""
        A_dn = A_up if A_dn is None else A_dn
        S = self.full
        d = self.dim(S)
        dtype = np.result_type(A_up, A_dn, np.float64)
        out = np.zeros((d, d), dtype=dtype)
        for spin, A in ((0, A_up), (1, A_dn)):
            if (spin == 0 and S[0] == 0) or (spin == 1 and S[1] == 0):
                continue
            ann = [self.annihilator(p + spin * self.M, S) for p in range(self.M)]
            for p in range(self.M):
                for q in range(self.M):
                    if A[p, q] != 0:
                        out += A[p, q] * (ann[p].T @ ann[q])
        return out

    def two_body(self, v: np.ndarray) -> np.ndarray:
        """Matrix of 1/2 sum_{pqrs} v_pqrs sum_{sigma tau} a+_{p s} a+_{q t} a_{s t} a_{r s}
        (eq:bo_ham2) on the full sector, using a+_p a+_q a_s a_r = (a_q a_p)^T (a_s a_r)."""
        S = self.full
        M = self.M
        d = self.dim(S)
        out = np.zeros((d, d))
        vmat = v.reshape(M * M, M * M)           # rows (p, q), columns (r, s)
        for s1 in (0, 1):
            for s2 in (0, 1):
                first = (S[0] - 1, S[1]) if s1 == 0 else (S[0], S[1] - 1)
                if min(first) < 0:
                    continue
                second = (first[0] - 1, first[1]) if s2 == 0 else (first[0], first[1] - 1)
                if min(second) < 0:
                    continue
                # K[(r, s)] = a_{s, s2} a_{r, s1}: S -> second
                K = np.zeros((M, M, self.dim(second), d))
                for r in range(M):
                    ar = self.annihilator(r + s1 * M, S)
                    for s in range(M):
                        K[r, s] = self.annihilator(s + s2 * M, first) @ ar
                Kf = K.reshape(M * M, -1)
                Y = (vmat @ Kf).reshape(M * M, self.dim(second), d)
                Kr = K.reshape(M * M, self.dim(second), d)
                for pq in range(M * M):
                    out += Kr[pq].T @ Y[pq]
        return 0.5 * out

    def hamiltonian(self, h0: float, h1: np.ndarray, v: np.ndarray) -> np.ndarray:
        """H = H0 + sum h_pq a+a + 1/2 sum v_pqrs a+a+aa (eq:bo_ham2) on the full sector."""
        d = self.dim(self.full)
        return h0 * np.eye(d) + self.one_body(h1) + self.two_body(v)


def eri_from_cholesky(L: np.ndarray) -> np.ndarray:
    """v_pqrs = sum_g L^g_pr L^g_qs (Sec. II.B.2), chemist ordering (pr|qs)."""
    return np.einsum("gpr,gqs->pqrs", L, L)
