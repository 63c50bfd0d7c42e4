"""Free projection (Sec. II.C) with the hybrid importance function (eq:hybrid-wt) is exact for
the propagator it samples.  With a single Cholesky vector the Hubbard-Stratonovich integral
(eq:hs, App. A.2) is exact, so the walk must reproduce the finite-beta mixed estimate of the
Trotter-split propagator exp(-dt/2 v0) exp(-dt/2 L^2) exp(-dt/2 v0), built here in Fock space,
to within statistical error.  This pins the force bias, the complex weight and phase, and the
QR bookkeeping of |<Phi_T|Psi>| together."""

import numpy as np
import scipy.linalg

from oracle import afqmc as A
from oracle import fock as F
from synthetic import gaussian_fields, gen_system


def test_free_projection_matches_exact_finite_beta():
    s = gen_system(8, 2, 1, seed=41)
    L = s.L * 3.0
    dt, nsteps, nw = 0.02, 25, 2000
    S = A.setup(0.0, s.h1, L, s.phi_up, s.phi_dn, dt)
    fs = F.FockSpace(8, 2, 2)
    H = fs.hamiltonian(0.0, s.h1, F.eri_from_cholesky(L))
    half = scipy.linalg.expm(-0.5 * dt * fs.one_body(S.v0))
    Lhat = fs.one_body(L[0])
    P = half @ scipy.linalg.expm(-0.5 * dt * Lhat @ Lhat) @ half
    phiT = fs.slater(s.phi_up.astype(complex), s.phi_dn.astype(complex))
    psi = phiT.copy()
    ref = []
    for k in range(nsteps):
        psi = P @ psi
        ref.append((np.vdot(phiT, H @ psi) / np.vdot(phiT, psi)).real)
    Pa = A.Params(dtau=dt, qr_period=5, pop_period=0, weight_mode=A.WEIGHT_FREE)
    wk = A.init_walkers(S, nw)
    for k in range(nsteps):
        A.step(S, Pa, wk, gaussian_fields(7, 0, wk.walker_id, k, 1))
        if k in (9, 24):
            c = wk.W * np.exp(1j * wk.theta)
            num = c * wk.e_loc
            g = 20
            idx = np.arange(nw) % g
            full = (num.sum() / c.sum()).real
            jk = np.array([((num.sum() - num[idx == i].sum()) / (c.sum() - c[idx == i].sum())).real
                           for i in range(g)])
            err = np.sqrt((g - 1) / g * np.sum((jk - jk.mean()) ** 2))
            assert err < 0.02
            assert abs(full - ref[k]) < 4 * err, (k, full, err, ref[k])
    # the estimate moved well away from the trial energy: the check is not trivial
    assert ref[24] < S.E_T - 0.3
