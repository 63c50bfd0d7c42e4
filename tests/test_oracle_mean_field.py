"""Mean-field background subtraction (Sec. II.B.3) in the oracle, pinned in Fock space."""

import math

import numpy as np
import scipy.linalg

from oracle import afqmc as A
from oracle import fock as F
from synthetic import config_system, gaussian_fields, gen_system, random_walkers


def test_mean_field_rewrite_is_an_operator_identity():
    """H = H0' + v0' + 1/2 sum_g (L_g - lbar_g)^2 with H0' = H0 - 1/2 sum lbar^2 and
    v0' = v0 + sum lbar_g L_g, and lbar_g = <Psi_T|L_g|Psi_T> / <Psi_T|Psi_T>."""
    s = config_system("tiny")
    S = A.setup(0.3, s.h1, s.L, s.phi_up, s.phi_dn, 0.01, mean_field=True)
    fs = F.FockSpace(8, 2, 2)
    H = fs.hamiltonian(0.3, s.h1, F.eri_from_cholesky(s.L))
    phiT = fs.slater(s.phi_up.astype(complex), s.phi_dn.astype(complex))
    Hm = S.h0_prop * np.eye(H.shape[0]) + fs.one_body(S.v0)
    for g in range(s.n_chol):
        Lg = fs.one_body(s.L[g])
        assert abs(S.lbar[g] - (np.vdot(phiT, Lg @ phiT) / np.vdot(phiT, phiT)).real) < 1e-12
        D = Lg - S.lbar[g] * np.eye(H.shape[0])
        Hm += 0.5 * D @ D
    assert np.abs(H - Hm).max() < 1e-12
    # the trial energy does not depend on how H is split
    S0 = A.setup(0.3, s.h1, s.L, s.phi_up, s.phi_dn, 0.01)
    assert abs(S.E_T - S0.E_T) < 1e-12


def test_mean_field_hubbard_stratonovich_with_c_number():
    """Gauss-Hermite average of the propagated determinant times the c-number
    exp(-i s (x - xbar) lbar) and the importance factor equals
    exp(-dt/2 v0') exp(-dt/2 (L - lbar)^2) exp(-dt/2 v0') |Psi> for one Cholesky vector."""
    s = gen_system(5, 2, 1, seed=91)
    L = s.L * 6.0
    dt = 0.05
    S = A.setup(0.0, s.h1, L, s.phi_up, s.phi_dn, dt, mean_field=True)
    assert abs(S.lbar[0]) > 0.1
    fs = F.FockSpace(5, 2, 2)
    D = fs.one_body(L[0]) - S.lbar[0] * np.eye(fs.dim(fs.full))
    half = scipy.linalg.expm(-0.5 * dt * fs.one_body(S.v0))
    Uu, Ud = random_walkers(s, 1, seed=5, amplitude=0.8)
    psi = fs.slater(Uu[0], Ud[0])
    ref = half @ scipy.linalg.expm(-0.5 * dt * D @ D) @ half @ psi
    nodes, weights = np.polynomial.hermite_e.hermegauss(60)
    weights = weights / math.sqrt(2 * math.pi)
    for xbar0 in (0.0, 0.2 - 0.1j):
        acc = np.zeros_like(psi)
        for xk, wk in zip(nodes, weights):
            x, xb = np.array([xk]), np.array([xbar0])
            Am = A.propagator_exponent(S, x, xb)
            Ue = [A.propagate(S, Am, U, 40) for U in (Uu[0], Ud[0])]
            c = np.exp(A.mean_field_log_factor(S, x, xb) + xk * xbar0 - 0.5 * xbar0 * xbar0)
            acc += wk * c * fs.slater(*Ue)
        assert np.abs(acc - ref).max() < 1e-10 * np.abs(ref).max()


def test_mean_field_free_projection_matches_exact_finite_beta():
    s = gen_system(8, 2, 1, seed=41)
    L = s.L * 3.0
    dt, nsteps, nw = 0.02, 25, 2000
    S = A.setup(0.0, s.h1, L, s.phi_up, s.phi_dn, dt, mean_field=True)
    fs = F.FockSpace(8, 2, 2)
    H = fs.hamiltonian(0.0, s.h1, F.eri_from_cholesky(L))
    half = scipy.linalg.expm(-0.5 * dt * fs.one_body(S.v0))
    D = fs.one_body(L[0]) - S.lbar[0] * np.eye(fs.dim(fs.full))
    P = half @ scipy.linalg.expm(-0.5 * dt * D @ D) @ half       # the subtracted split
    phiT = fs.slater(s.phi_up.astype(complex), s.phi_dn.astype(complex))
    psi = phiT.copy()
    ref = []
    for k in range(nsteps):
        psi = P @ psi
        ref.append((np.vdot(phiT, H @ psi) / np.vdot(phiT, psi)).real)
    Pa = A.Params(dtau=dt, qr_period=5, pop_period=0, weight_mode=A.WEIGHT_FREE)
    wk = A.init_walkers(S, nw)
    for k in range(nsteps):
        A.step(S, Pa, wk, gaussian_fields(13, 0, wk.walker_id, k, 1))
    c = wk.W * np.exp(1j * wk.theta)
    num = c * wk.e_loc
    g = 20
    idx = np.arange(nw) % g
    full = (num.sum() / c.sum()).real
    jk = np.array([((num.sum() - num[idx == i].sum()) / (c.sum() - c[idx == i].sum())).real
                   for i in range(g)])
    err = np.sqrt((g - 1) / g * np.sum((jk - jk.mean()) ** 2))
    assert err < 0.02 and abs(full - ref[-1]) < 4 * err, (full, err, ref[-1])
