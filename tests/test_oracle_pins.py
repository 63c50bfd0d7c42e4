"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute-force
second quantization on a 784-state Fock sector, closed forms (Slater-Condon,
zero-variance eigenstates, the non-interacting limit), exact operator
identities (Hubbard-Stratonovich, Thouless), and invariants (Theorem 1.5).
"""

import math

import numpy as np
import pytest
import scipy.linalg

from oracle import afqmc as A
from oracle import fock as F
from synthetic import config_system, diagonal_system, gen_system, random_walkers


@pytest.fixture(scope="module")
def tiny():
    s = config_system("tiny")
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, 0.01)
    fs = F.FockSpace(s.M, s.n_up, s.n_dn)
    H = fs.hamiltonian(s.h0, s.h1, F.eri_from_cholesky(s.L))
    return s, S, fs, H


def _fock_walker(fs, Uu, Ud):
    return fs.slater(Uu, Ud)


# ---------------------------------------------------------------- Theorem 1.1 / 1.2

def test_overlap_matches_fock(tiny):
    """<Phi_T|Psi> = prod det(V^T U) (Theorem 1.1) against the Fock-space inner product."""
    s, S, fs, _ = tiny
    phiT = fs.slater(s.phi_up.astype(complex), s.phi_dn.astype(complex))
    Uu, Ud = random_walkers(s, 6, seed=11, amplitude=1.5)
    for w in range(6):
        ov_fock = np.vdot(phiT, fs.slater(Uu[w], Ud[w]))
        lg = A.overlap_theta(S.V[0], Uu[w])[0] + A.overlap_theta(S.V[1], Ud[w])[0]
        assert abs(np.exp(lg) - ov_fock) <= 1e-12 * abs(ov_fock)


def test_green_function_matches_fock(tiny):
    """G_pq = <a+_p a_q>_m from U (V^T U)^-1 V^T (Theorem 1.2) against Fock space."""
    s, S, fs, _ = tiny
    phiT = fs.slater(s.phi_up.astype(complex), s.phi_dn.astype(complex))
    Uu, Ud = random_walkers(s, 2, seed=12, amplitude=1.0)
    M = s.M
    for w in range(2):
        psi = fs.slater(Uu[w], Ud[w])
        ov = np.vdot(phiT, psi)
        G_up = A.green_function(S.V[0], Uu[w])
        G_dn = A.green_function(S.V[1], Ud[w])
        full = fs.full
        for p in range(M):
            for q in range(M):
                for spin, G in ((0, G_up), (1, G_dn)):
                    op = fs.annihilator(p + spin * M, full).T @ fs.annihilator(q + spin * M, full)
                    ref = np.vdot(phiT, op @ psi) / ov
                    assert abs(G[p, q] - ref) < 1e-12


# ---------------------------------------------------------------- local energy, force bias

@pytest.mark.parametrize("amplitude", [0.0, 0.3, 2.0])
def test_local_energy_and_traces_match_fock(tiny, amplitude):
    """E_L = <Phi_T|H|Psi>/<Phi_T|Psi> with H built from v_pqrs (eq:bo_ham2), and
    <L_g>_m = t_g (eq:precomputing2), for walkers near and far from the trial."""
    s, S, fs, H = tiny
    phiT = fs.slater(s.phi_up.astype(complex), s.phi_dn.astype(complex))
    Uu, Ud = random_walkers(s, 3, seed=13, amplitude=amplitude)
    Lops = [fs.one_body(s.L[g]) for g in (0, 7, 31)]
    for w in range(3):
        psi = fs.slater(Uu[w], Ud[w])
        ov = np.vdot(phiT, psi)
        _, _, e, t = A.measure(S, Uu[w], Ud[w])
        ref = np.vdot(phiT, H @ psi) / ov
        assert abs(e - ref) < 1e-11 * max(1.0, abs(ref))
        for g, Lg in zip((0, 7, 31), Lops):
            assert abs(t[g] - np.vdot(phiT, Lg @ psi) / ov) < 1e-12
        xbar = A.force_bias(t, S.dtau, 1e9)
        vg = 1j * (np.vdot(phiT, Lops[0] @ psi) / ov)         # <v_0>_m, v_g = i L_g
        assert abs(xbar[0] - (-math.sqrt(S.dtau) * vg)) < 1e-12   # eq:fb


def test_local_energy_open_shell_nonorthonormal_trial():
    """Same brute-force check with N_up != N_dn and a non-orthonormal trial (Theorem 1.5)."""
    s = gen_system(6, 2, 10, seed=77, n_dn=1)
    rng = np.random.default_rng(5)
    phi_up = s.phi_up @ (rng.standard_normal((2, 2)) + 2 * np.eye(2))
    phi_dn = 1.7 * s.phi_dn
    S = A.setup(s.h0 + 0.25, s.h1, s.L, phi_up, phi_dn, 0.02)
    fs = F.FockSpace(6, 2, 1)
    H = fs.hamiltonian(s.h0 + 0.25, s.h1, F.eri_from_cholesky(s.L))
    phiT = fs.slater(phi_up.astype(complex), phi_dn.astype(complex))
    Uu = phi_up + 0.5 * (rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2)))
    Ud = phi_dn + 0.5 * (rng.standard_normal((6, 1)) + 1j * rng.standard_normal((6, 1)))
    psi = fs.slater(Uu, Ud)
    ov = np.vdot(phiT, psi)
    _, _, e, _ = A.measure(S, Uu, Ud)
    assert abs(e - np.vdot(phiT, H @ psi) / ov) < 1e-11
    # Trial energy: the Rayleigh quotient of the trial itself.
    assert abs(S.E_T - (np.vdot(phiT, H @ phiT) / np.vdot(phiT, phiT)).real) < 1e-11


# ---------------------------------------------------------------- Slater-Condon closed form

@pytest.mark.parametrize("name", ["tiny", "medium", "large"])
def test_trial_energy_is_slater_condon(name):
    """E_L(Phi_T, Phi_T) = H0 + 2 sum_i h_ii + sum_ij [2 (ii|jj) - (ij|ji)] over the
    occupied orthonormal MOs (closed-shell Slater-Condon rules, Wick with Phi = Psi)."""
    s = config_system(name)
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, 0.005)
    C = s.phi_up                                         # orthonormal columns (eigenvectors)
    h_mo = C.T @ s.h1 @ C
    Lmo = np.einsum("pi,gpq,qj->gij", C, s.L, C)         # (g, i, j)
    J = np.einsum("gii,gjj->ij", Lmo, Lmo)               # (ii|jj)
    K = np.einsum("gij,gji->ij", Lmo, Lmo)               # (ij|ji)
    e_sc = s.h0 + 2 * np.trace(h_mo) + np.sum(2 * J - K)
    assert abs(S.E_T - e_sc) < 1e-10 * abs(e_sc)


# ---------------------------------------------------------------- zero variance (Sec. III.D.1)

@pytest.mark.parametrize("M,N,G,amp", [(8, 2, 16, 1.0), (64, 16, 320, 0.5), (128, 32, 800, 0.3)])
def test_zero_variance_diagonal_hamiltonian(M, N, G, amp):
    """With h and every L_g diagonal in one basis Q, an occupation determinant of Q is an
    exact eigenstate with E(n) = sum eps_p n_p + 1/2 sum_g [(sum_p l_gp n_p)^2 - sum_p l_gp^2 n_p]
    (n_p = n_up + n_dn), so E_L(Psi) = E(n_T) for every walker Psi."""
    s = diagonal_system(M, N, G, seed=M + 3, occ_up=range(1, N + 1), occ_dn=range(N),
                        mix_trial=True)
    eps, lv = s.meta["eps"], s.meta["lvals"]
    n = np.zeros(M)
    n[s.meta["occ_up"]] += 1
    n[s.meta["occ_dn"]] += 1
    e_exact = eps @ n + 0.5 * np.sum((lv @ n) ** 2 - (lv ** 2) @ n)
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, 0.005)
    assert abs(S.E_T - e_exact) < 1e-10 * abs(e_exact)
    Uu, Ud = random_walkers(s, 2, seed=M, amplitude=amp)
    for w in range(2):
        _, _, e, _ = A.measure(S, Uu[w], Ud[w])
        assert abs(e - e_exact) < 1e-9 * abs(e_exact)


# ---------------------------------------------------------------- Cholesky rewrite, HS, Thouless

def test_cholesky_rewrite_operator_identity(tiny):
    """H = H0 + v0 + 1/2 sum_g L_g^2 on the Fock sector (eq:mcd1, eq:hamsum with v_g = i L_g),
    with v0 = h - 1/2 sum_g L_g L_g from the oracle's setup."""
    s, S, fs, H = tiny
    H2 = s.h0 * np.eye(H.shape[0]) + fs.one_body(S.v0)
    for g in range(s.n_chol):
        Lg = fs.one_body(s.L[g])
        H2 += 0.5 * Lg @ Lg
    assert np.abs(H - H2).max() < 1e-12


def test_thouless_propagation(tiny):
    """exp(A-hat)|Psi> is the determinant exp(A) U (Theorem 1.4), and the oracle's Taylor
    series matches exp(A) U to within its truncation tail."""
    s, S, fs, _ = tiny
    rng = np.random.default_rng(3)
    Uu, Ud = random_walkers(s, 1, seed=21, amplitude=0.7)
    x = rng.standard_normal(s.n_chol)
    xbar = 0.05 * (rng.standard_normal(s.n_chol) + 1j * rng.standard_normal(s.n_chol))
    Am = A.propagator_exponent(S, x, xbar)
    lhs = scipy.linalg.expm(fs.one_body(Am)) @ fs.slater(Uu[0], Ud[0])
    E = scipy.linalg.expm(Am)
    rhs = fs.slater(E @ Uu[0], E @ Ud[0])
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max()
    for n_taylor, tol in ((6, 1e-7), (20, 1e-14)):
        T = A.taylor_apply(Am, Uu[0], n_taylor)
        assert np.abs(T - E @ Uu[0]).max() < tol


def test_hubbard_stratonovich_pins_factor_i():
    """Gauss-Hermite average over x of the oracle's propagated determinant (as a Fock
    vector) equals exp(-dt/2 v0) exp(-dt/2 L^2) exp(-dt/2 v0) |Psi> (eq:hs, App. A.2):
    the field term must be exp(i s x L) for the two-body energy to be repulsive.
    The average with a complex shift xbar and the importance factor
    exp(x xbar - xbar^2/2) gives the same operator (App. A.2, shifted contour)."""
    s = gen_system(5, 2, 1, seed=91)
    L = s.L * 6.0
    dt = 0.05
    S = A.setup(0.0, s.h1, L, s.phi_up, s.phi_dn, dt)
    fs = F.FockSpace(5, 2, 2)
    Lhat = fs.one_body(L[0])
    V0 = fs.one_body(S.v0)
    Uu, Ud = random_walkers(s, 1, seed=5, amplitude=0.8)
    psi = fs.slater(Uu[0], Ud[0])
    half = scipy.linalg.expm(-0.5 * dt * V0)
    ref = half @ scipy.linalg.expm(-0.5 * dt * Lhat @ Lhat) @ half @ psi
    nodes, weights = np.polynomial.hermite_e.hermegauss(60)
    weights = weights / math.sqrt(2 * math.pi)
    for xbar0 in (0.0, 0.3 - 0.2j):
        acc = np.zeros_like(psi)
        for xk, wk in zip(nodes, weights):
            Am = A.propagator_exponent(S, np.array([xk]), np.array([xbar0]))
            Ue = [A.propagate(S, Am, U, 40) for U in (Uu[0], Ud[0])]
            imp = np.exp(xk * xbar0 - 0.5 * xbar0 * xbar0)
            acc += wk * imp * fs.slater(*Ue)
        assert np.abs(acc - ref).max() < 1e-10 * np.abs(ref).max()
    # The opposite sign convention (exp(s x L), an attractive interaction) must fail.
    acc = np.zeros_like(psi)
    for xk, wk in zip(nodes, weights):
        Am = -1j * A.propagator_exponent(S, np.array([xk]), np.array([0.0]))
        acc += wk * fs.slater(*[A.propagate(S, Am, U, 40) for U in (Uu[0], Ud[0])])
    assert np.abs(acc - ref).max() > 1e-3 * np.abs(ref).max()


def test_trotter_step_matches_exact_propagator_to_second_order():
    """The split step exp(-dt/2 v0) exp(-dt/2 sum L^2) exp(-dt/2 v0) built from the oracle's
    v0 approaches exp(-dt H) (eq:primitive) with an O(dt^3) error per step."""
    s = config_system("tiny")
    fs = F.FockSpace(8, 2, 2)
    H = fs.hamiltonian(s.h0, s.h1, F.eri_from_cholesky(s.L))
    Uu, Ud = random_walkers(s, 1, seed=8, amplitude=0.5)
    psi = fs.slater(Uu[0], Ud[0])
    Lsq = sum(np.linalg.matrix_power(fs.one_body(s.L[g]), 2) for g in range(s.n_chol))
    errs = []
    for dt in (0.04, 0.02):
        S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, dt)
        half = scipy.linalg.expm(-0.5 * dt * fs.one_body(S.v0))
        split = half @ scipy.linalg.expm(-0.5 * dt * Lsq) @ half @ psi
        errs.append(np.abs(split - scipy.linalg.expm(-dt * H) @ psi).max())
    assert errs[1] < errs[0] / 6.0          # cubic: ratio ~ 8


# ---------------------------------------------------------------- Theorem 1.5, mGS

def test_gram_schmidt_invariance(tiny):
    s, S, _, _ = tiny
    big = gen_system(128, 32, 64, seed=4)
    Sb = A.setup(big.h0, big.h1, big.L, big.phi_up, big.phi_dn, 0.005)
    for sys_, setup_ in ((s, S), (big, Sb)):
        Uu, Ud = random_walkers(sys_, 1, seed=9, amplitude=0.8)
        Qu, ru = A.modified_gram_schmidt(Uu[0])
        Qd, rd = A.modified_gram_schmidt(Ud[0])
        for U, Q, r in ((Uu[0], Qu, ru), (Ud[0], Qd, rd)):
            assert np.abs(Q.conj().T @ Q - np.eye(Q.shape[1])).max() < 1e-13
            R = Q.conj().T @ U
            assert np.abs(np.tril(R, -1)).max() < 1e-12
            assert np.all(r > 0) and np.abs(np.diag(R).real - r).max() < 1e-12
            assert np.abs(np.diag(R).imag).max() < 1e-12
        a0, l0, e0, t0 = A.measure(setup_, Uu[0], Ud[0])
        a1, l1, e1, t1 = A.measure(setup_, Qu, Qd)
        assert abs(e1 - e0) < 1e-11 * abs(e0)
        assert np.abs(t1 - t0).max() < 1e-12
        assert abs(A.wrap_angle(a1 - a0)) < 1e-12
        assert abs((l0 - l1) - np.sum(np.log(ru)) - np.sum(np.log(rd))) < 1e-10


# ---------------------------------------------------------------- non-interacting limit

def test_noninteracting_limit_converges_to_lowest_orbitals():
    """With N_g = 0 the walk is deterministic, U <- exp(-dt h) U, and every walker converges
    to the lowest-N eigenvectors of h: E_L -> 2 sum of the N lowest eigenvalues."""
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((8, 8)))
    eps = np.array([-3.0, -2.6, -1.5, -1.2, -1.0, -0.7, -0.4, 0.1])
    h1 = (Q * eps) @ Q.T
    h1 = 0.5 * (h1 + h1.T)
    trial, _ = np.linalg.qr(rng.standard_normal((8, 2)))
    S = A.setup(0.0, h1, np.zeros((0, 8, 8)), trial, trial, 0.1)
    P = A.Params(dtau=0.1, qr_period=5, pop_period=0)
    wk = A.init_walkers(S, 4)
    for _ in range(400):
        A.step(S, P, wk, np.zeros((4, 0)))
    assert np.abs(wk.e_loc - 2 * eps[:2].sum()).max() < 1e-9


# ---------------------------------------------------------------- weights and caps

def test_phaseless_projection_kills_rotated_walker(tiny):
    """Rotating one orbital by exp(0.75 i pi) before a step makes cos(dtheta) < 0 -> W = 0
    (eq:if_rle), and the dead walker is skipped afterwards (Sec. III.E)."""
    s, S, _, _ = tiny
    P = A.Params(dtau=0.01, pop_period=0)
    wk = A.init_walkers(S, 3)
    wk.U[0][1][:, 0] *= np.exp(0.75j * np.pi)
    x = np.zeros((3, s.n_chol))
    A.step(S, P, wk, x)
    assert wk.W[1] == 0.0 and wk.W[0] > 0 and wk.W[2] > 0
    before = wk.U[0][1].copy()
    A.step(S, P, wk, x)
    assert wk.W[1] == 0.0 and np.array_equal(before, wk.U[0][1])


def test_energy_and_weight_caps():
    E_T, dt, C = -10.0, 0.01, 2.0
    half = math.sqrt(C / dt)
    e = np.array([E_T - 3 * half, E_T, E_T + 0.5 * half, E_T + 9 * half])
    capped = A.capped_energy(e, E_T, dt, C)
    assert np.allclose(capped, [E_T - half, E_T, E_T + 0.5 * half, E_T + half])
    W = A.phaseless_weight(np.array([1.0, 1.0, 50.0]), np.array([E_T - 3 * half, E_T, E_T]),
                           np.zeros(3), np.array([0.0, 0.1, 0.0]), dt, E_T, C, 60.0)
    assert abs(W[0] - math.exp(dt * half)) < 1e-14
    assert abs(W[1] - math.cos(0.1)) < 1e-15
    xb = A.force_bias(np.array([0.0 + 50j, 0.1 + 0.2j]), 0.01, 1.0)
    assert abs(abs(xb[0]) - 1.0) < 1e-15 and abs(xb[1] - (-0.1j) * (0.1 + 0.2j)) < 1e-16


# ---------------------------------------------------------------- comb

def test_comb_invariants():
    rng = np.random.default_rng(4)
    for trial in range(50):
        n = int(rng.integers(1, 300))
        W = rng.exponential(size=n) * (rng.random(n) > 0.3)
        if not W.sum() > 0:
            W[0] = 1.0
        u = float(rng.random())
        parent, Wn = A.comb(W, u)
        total = W.sum()
        assert np.all(np.diff(parent) >= 0)
        assert np.all(W[parent] > 0)
        counts = np.bincount(parent, minlength=n)
        expect = n * W / total
        assert np.all(counts >= np.floor(expect) - 1e-9) and np.all(counts <= np.ceil(expect) + 1e-9)
        assert np.array_equal(Wn, np.ones(n))
    # Equal weights and any u: every walker is kept exactly once.
    parent, _ = A.comb(np.ones(17), 0.999)
    assert np.array_equal(parent, np.arange(17))
