"""Pins of the growth phase of the oracle: the local-energy cap centre (App. B.1, eq:cap) and
the trial energy from the growth estimator (App. B.2, eq:corsam).

* Non-interacting limit (N_g = 0): the walk is deterministic and every walker is the same, so
  the total weight grows by exactly exp(-dtau (E_L - E_T)) per step.  The growth estimate must
  then lie between the smallest and largest local energy of its block and, once the walkers
  have converged, equal the exact energy 2 (eps_0 + eps_1); so must the cap centre.  A wrong
  sign or a missing 1/dtau in the estimate fails both.
* Exact diagonalization: with the window E_T +- sqrt(C/dtau) narrowed (C small) so that it
  excludes the exact ground-state energy E0, a cap centred on E_T holds the mixed estimate at
  the window's lower edge, while a cap centred on the growth-phase average of the local
  energy lets it go well below that edge, towards E0.
"""

import math

import numpy as np

from oracle import afqmc as A
from oracle import fock as F
from synthetic import comb_uniform, config_system, gaussian_fields


def _noninteracting(dt):
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((8, 8)))
    eps = np.array([-3.0, -2.6, -1.5, -1.2, -1.0, -0.7, -0.4, 0.1])
    h1 = (Q * eps) @ Q.T
    h1 = 0.5 * (h1 + h1.T)
    trial, _ = np.linalg.qr(rng.standard_normal((8, 2)))
    S = A.setup(0.0, h1, np.zeros((0, 8, 8)), trial, trial, dt)
    return S, 2 * eps[:2].sum()


def test_growth_estimate_noninteracting_limit():
    dt, nw, l = 0.05, 4, 5
    S, e_exact = _noninteracting(dt)
    P = A.Params(dtau=dt, qr_period=5, pop_period=l, n_growth=600)
    wk = A.init_walkers(S, nw)
    assert wk.growth.E_T == S.E_T and wk.growth.e_bar == S.E_T
    block = []
    for k in range(600):
        block.append(wk.e_loc[0].real)      # E_L(Psi_k), the energy in this step's weight
        A.step(S, P, wk, np.zeros((nw, 0)), 0.5)
        if (k + 1) % l == 0:
            lo, hi = min(block), max(block)
            pad = 1e-9 * (1.0 + abs(lo))
            assert lo - pad <= wk.growth.E_T <= hi + pad, (k, wk.growth.E_T, lo, hi)
            block = []
    assert abs(wk.e_loc[0] - e_exact) < 1e-9
    assert abs(wk.growth.E_T - e_exact) < 1e-9
    assert abs(wk.growth.e_bar - e_exact) < 1e-9
    # total weight no longer grows once E_T is the growth estimate
    assert abs(wk.W.sum() / nw - wk.W[0]) < 1e-12


def test_growth_phase_freezes_after_n_growth():
    dt = 0.05
    S, _ = _noninteracting(dt)
    P = A.Params(dtau=dt, qr_period=5, pop_period=5, n_growth=20)
    wk = A.init_walkers(S, 2)
    seen = []
    for k in range(60):
        A.step(S, P, wk, np.zeros((2, 0)), 0.5)
        seen.append((wk.growth.E_T, wk.growth.e_bar))
    assert seen[3] == (S.E_T, S.E_T)          # unchanged until the first block ends
    assert seen[4] != seen[3]                  # the first block end (step 4) updates both
    assert all(v == seen[19] for v in seen[19:])   # last update at step 19 (< 20), then fixed
    assert seen[19] != seen[14]
    # no growth phase: both stay at the trial energy
    P0 = A.Params(dtau=dt, qr_period=5, pop_period=5, n_growth=0)
    wk0 = A.init_walkers(S, 2)
    for k in range(30):
        A.step(S, P0, wk0, np.zeros((2, 0)), 0.5)
    assert (wk0.growth.E_T, wk0.growth.e_bar) == (S.E_T, S.E_T)


def test_cap_centre_from_growth_phase_against_exact_diagonalization():
    s = config_system("tiny")
    dt, nw, steps, C = 0.01, 64, 300, 0.0004
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, dt)
    fs = F.FockSpace(8, 2, 2)
    E0 = float(np.linalg.eigvalsh(fs.hamiltonian(s.h0, s.h1, F.eri_from_cholesky(s.L)))[0])
    half = math.sqrt(C / dt)
    edge = S.E_T - half
    assert E0 < edge - 0.15                    # the window around E_T excludes E0
    out = {}
    for n_growth in (0, steps):
        P = A.Params(dtau=dt, el_cap_C=C, n_growth=n_growth)
        wk = A.init_walkers(S, nw)
        ser, capped = [], []
        for k in range(steps):
            A.step(S, P, wk, gaussian_fields(3, 0, wk.walker_id, k, s.n_chol), comb_uniform(3, 0, k))
            ser.append(A.mixed_energy(S, P, wk)[0])
            live = wk.W > 0
            capped.append(np.mean(np.abs(wk.e_loc.real[live] - wk.growth.e_bar) > half))
        out[n_growth] = (np.array(ser), float(np.mean(capped[steps // 2:])))
    fixed, fixed_cap = out[0]
    grown, grown_cap = out[steps]
    # centred on E_T: never below the edge, and stuck at it, most walkers capped
    assert fixed.min() >= edge - 1e-12
    assert abs(fixed[steps // 2:].mean() - edge) < 0.02
    assert fixed_cap > 0.5
    # centred on the growth-phase average: well below the edge, within 0.1 Ha of E0
    tail = grown[steps // 2:].mean()
    assert tail < edge - 0.08, (tail, edge)
    assert abs(tail - E0) < 0.1, (tail, E0)
    assert grown_cap < 0.3
