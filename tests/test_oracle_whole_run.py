"""The whole-run pin of the oracle (Sec. III.C, App. C): a long phaseless AFQMC run of the tiny
molecule (M=8, 2+2 electrons, N_g=32) against its exact ground-state energy E0 from exact
diagonalization of the 784-state sector.

The estimate is the mean over independent replicas (different field seeds), each reblocked
after its equilibration; its error is taken from the spread of the replicas, which does not
depend on how well a single series' reblocking has converged.

* With a self-consistent restricted Hartree-Fock trial the run agrees with E0 within three
  standard errors.
* With the workload's own trial (the lowest eigenvectors of h1 + sum_g L_g L_g, not
  self-consistent, E_T - E0 = 0.38 Ha) the phaseless constraint leaves a bias of ~30 mHa:
  the slow test shows it is many standard errors wide, that it stays when the time step is
  halved, and that the better trial removes it (the paper notes that the phaseless
  approximation depends on the trial, Sec. III.C).

The default test pools four replicas of 64 walkers x 2000 steps (dtau = 0.01) run in parallel
processes; the slow one (AFQMC_RUN_SLOW=1) eight replicas of 128 walkers x 4000 steps per
trial and time step.
"""

import math
import multiprocessing as mp
import os

import numpy as np
import pytest


def _replica(args):
    """One run: (trial, dtau, walkers, beta, seed) -> reblocked mean of the mixed estimate."""
    trial, dt, nw, beta, seed = args
    from threadpoolctl import threadpool_limits

    from oracle import afqmc as A
    from oracle.reblock import reblock_converged
    from synthetic import comb_uniform, config_system, gaussian_fields, rhf_trial
    with threadpool_limits(limits=1):
        s = config_system("tiny")
        if trial == "rhf":
            C, _, _ = rhf_trial(s)
            S = A.setup(s.h0, s.h1, s.L, C, C, dt)
        else:
            S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, dt)
        steps = int(round(beta / dt))
        equil = int(round(2.0 / dt))
        P = A.Params(dtau=dt, n_growth=equil)
        wk = A.init_walkers(S, nw)
        x, w = [], []
        for k in range(steps):
            A.step(S, P, wk, gaussian_fields(seed, 0, wk.walker_id, k, s.n_chol),
                   comb_uniform(seed, 0, k))
            e = A.mixed_energy(S, P, wk)
            x.append(e[0])
            w.append(e[3])
        mean, err, _, _ = reblock_converged(x, w, discard=equil)
    return mean, err


def _pooled(trial, dt, nw, beta, seeds):
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(len(seeds), max(1, (os.cpu_count() or 1)))) as pool:
        res = pool.map(_replica, [(trial, dt, nw, beta, sd) for sd in seeds])
    means = np.array([m for m, _ in res])
    return float(means.mean()), float(means.std(ddof=1) / math.sqrt(len(means))), means


def _exact():
    from oracle import fock as F
    from synthetic import config_system
    s = config_system("tiny")
    H = F.FockSpace(8, 2, 2).hamiltonian(s.h0, s.h1, F.eri_from_cholesky(s.L))
    return float(np.linalg.eigvalsh(H)[0])


def test_rhf_trial_is_self_consistent():
    """The trial the whole run uses: its energy is E_L(Phi, Phi) (Slater-Condon through the
    oracle), its Fock matrix has no occupied-virtual block, and it lies below the workload's
    own trial."""
    from oracle import afqmc as A
    from synthetic import config_system, rhf_trial
    s = config_system("tiny")
    C, e, _ = rhf_trial(s)
    S = A.setup(s.h0, s.h1, s.L, C, C, 0.01)
    assert abs(S.E_T - e) < 1e-10
    P = C @ C.T
    tg = np.einsum("grs,rs->g", s.L, P)
    F = s.h1 + 2 * np.einsum("g,gpq->pq", tg, s.L) - np.einsum("gpr,rs,gsq->pq", s.L, P, s.L)
    Q = np.eye(8) - P
    assert np.abs(Q @ F @ P).max() < 1e-6
    S0 = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, 0.01)
    assert S.E_T < S0.E_T - 0.2


def test_whole_run_agrees_with_exact_diagonalization():
    E0 = _exact()
    mean, err, means = _pooled("rhf", 0.01, 64, 20.0, [0, 1, 2, 3])
    print(f"whole run (RHF trial, 4 x 64 walkers x 2000 steps): {mean:.5f} +- {err:.5f}, "
          f"replicas {np.round(means, 5)}, exact {E0:.5f}")
    assert err < 0.01
    assert abs(mean - E0) < 3 * err, (mean, err, E0)


@pytest.mark.slow
@pytest.mark.skipif(os.environ.get("AFQMC_RUN_SLOW") != "1",
                    reason="long statistical run; set AFQMC_RUN_SLOW=1")
def test_whole_run_trial_and_time_step_series():
    E0 = _exact()
    seeds = list(range(8))
    out = {}
    for trial, dt in (("rhf", 0.01), ("rhf", 0.005), ("synthetic", 0.01), ("synthetic", 0.005)):
        out[(trial, dt)] = _pooled(trial, dt, 128, 40.0, seeds)[:2]
        m, e = out[(trial, dt)]
        print(f"{trial:9s} dtau={dt}: {m:.5f} +- {e:.5f} (E - E0 = {1e3 * (m - E0):+.1f} mHa)")
    for dt in (0.01, 0.005):
        m, e = out[("rhf", dt)]
        assert abs(m - E0) < 3 * e
        ms, es = out[("synthetic", dt)]
        assert abs(ms - E0) > 5 * es          # the poorer trial's phaseless bias
