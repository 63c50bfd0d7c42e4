"""Multi-determinant trial (Sec. II.B, eq:localenergy2, eq:precomputing2) on the GPU against the
FP64 oracle's ``setup_multi`` / ``measure_multi``: static measurements, random-walk lockstep in
every weight mode and precision, and the full-CI expansion whose local energy is exact."""

import numpy as np
import pytest

from oracle import afqmc as A
from oracle import fock as F
from synthetic import (config_system, excitation_trial, noci_trial, occupation_det,
                       random_walkers)
from tests.parity_helpers import angle_diff, log, oracle_U_to_gpu, run_lockstep

pytestmark = pytest.mark.gpu


def gpu_measure(gs, Uu, Ud):
    """Set the walkers' orbitals, measure on the GPU, return (arg, log|ovlp|, E_L)."""
    import torch
    nw = Uu.shape[0]
    wk = gs.walkers(nw)
    gs.init(wk)
    Ug = oracle_U_to_gpu(Uu, Ud)
    wk.U.copy_(torch.from_numpy(Ug[:, : gs.ntot]))
    gs.measure(wk)
    torch.cuda.synchronize()
    return wk.arg_ovlp.cpu().numpy(), wk.log_ovlp.cpu().numpy(), wk.e_loc.cpu().numpy()


def multi_system(s, trial, **kw):
    import paper_1711_02242_amd as afq
    coeffs, ups, dns = trial
    return afq.System.multidet(s.h0, s.h1, s.L, coeffs, np.array(ups), np.array(dns), **kw)


def oracle_measure(MS, Uu, Ud):
    out = [A.measure_multi(MS, Uu[w], Ud[w]) for w in range(Uu.shape[0])]
    return (np.array([o[0] for o in out]), np.array([o[1] for o in out]),
            np.array([o[2] for o in out]))


EL_TOL = 1e-4   # Ha per walker, mixed-precision contraction


def assert_measure_close(got, ref, rtol, what, e_atol=None):
    """Overlap phase and log-magnitude within rtol (FP64 in every mode); E_L within rtol
    relative, or within e_atol Ha when given (the mixed-precision bar)."""
    ga, gl, ge = got
    ra, rl, re_ = ref
    da = angle_diff(ga, ra).max()
    dl = np.abs(gl - rl).max() / max(1.0, np.abs(rl).max())
    de_abs = np.abs(ge - re_).max()
    de = de_abs / max(1.0, np.abs(re_).max())
    log(f"  {what}: d_arg {da:.2e} d_log {dl:.2e} d_E {de:.2e} ({de_abs:.2e} Ha)")
    assert da <= rtol and dl <= rtol, what
    assert (de_abs <= e_atol) if e_atol is not None else (de <= rtol), what


@pytest.mark.parametrize("kind", ["noci", "excitation"])
@pytest.mark.parametrize("case", ["tiny", "medium"])
def test_multidet_measure_matches_oracle(kind, case):
    s = config_system(case)
    n_det = 5
    trial = (noci_trial if kind == "noci" else excitation_trial)(s, n_det, seed=21)
    log(f"multidet measure {kind} {case} n_det={n_det}")
    MS = A.setup_multi(s.h0, s.h1, s.L, *trial, 0.005)
    gs = multi_system(s, trial, dtau=0.005, precision="fp64")
    assert abs(gs.e_trial - MS.E_T) <= 1e-11 * abs(MS.E_T)
    Uu, Ud = random_walkers(s, 8, seed=4, amplitude=0.6)
    assert_measure_close(gpu_measure(gs, Uu, Ud), oracle_measure(MS, Uu, Ud), 1e-10, "fp64")
    gs.close()


def walkers_near_lead(s, trial, nw, seed, amplitude):
    """Random walkers around the expansion's leading determinant, where the random walk starts
    and stays (walkers nearly orthogonal to the trial give large Theta = U (V^T U)^-1 and
    lose mixed-precision accuracy in proportion)."""
    from dataclasses import replace
    _, ups, dns = trial
    return random_walkers(replace(s, phi_up=np.asarray(ups[0]), phi_dn=np.asarray(dns[0])), nw,
                          seed=seed, amplitude=amplitude)


def cancellation(MS, Uu, Ud):
    """kappa_w = sum_d |r_d| / |sum_d r_d| per walker (r_d = conj(A_d) <Psi_d|Psi_w>): the factor
    by which the combination E_L = sum r_d E_L^d / sum r_d can amplify errors of the E_L^d."""
    out = []
    for w in range(Uu.shape[0]):
        r = []
        for c, S in zip(MS.coeffs, MS.dets):
            lu, _ = A.overlap_theta(S.V[0], Uu[w])
            ld, _ = A.overlap_theta(S.V[1], Ud[w])
            r.append(np.conj(c) * np.exp(lu + ld))
        r = np.array(r)
        out.append(np.abs(r).sum() / abs(r.sum()))
    return np.array(out)


def test_multidet_large_workload_measure():
    """M = 128, N = 32, G = 800 with a three-determinant NOCI trial: sampled walkers.  In the
    mixed-precision modes each determinant's E_L^d keeps the 1e-4 Ha bar; the combination is
    FP64, so the walker's E_L error is bounded by kappa_w * 1e-4 Ha."""
    s = config_system("large")
    trial = noci_trial(s, 3, seed=8, angle=0.3)
    log("multidet measure large n_det=3")
    MS = A.setup_multi(s.h0, s.h1, s.L, *trial, 0.005)
    Uu, Ud = walkers_near_lead(s, trial, 6, seed=5, amplitude=0.3)
    ref = oracle_measure(MS, Uu, Ud)
    kappa = cancellation(MS, Uu, Ud)
    log(f"  kappa {np.round(kappa, 2)}")
    for prec in ("fp64", "fp32", "bf16x3"):
        gs = multi_system(s, trial, dtau=0.005, precision=prec)
        got = gpu_measure(gs, Uu, Ud)
        assert_measure_close(got, ref, 1e-10, prec, None if prec == "fp64" else np.inf)
        if prec != "fp64":
            err = np.abs(got[2] - ref[2])
            log(f"  {prec}: max |dE_L| / kappa = {np.max(err / kappa):.2e} Ha")
            assert np.all(err <= kappa * EL_TOL)
        gs.close()


@pytest.mark.parametrize("mode", ["phaseless", "hybrid", "free"])
def test_multidet_lockstep_fp64(mode):
    s = config_system("tiny")
    trial = noci_trial(s, 4, seed=3)
    log(f"multidet lockstep fp64 {mode}")
    worst, *_ = run_lockstep(s, 16, 30, dtau=0.01, label=f"md-{mode}", weight_mode=mode,
                             trial=trial)
    log(f"  worst {worst}")


def test_multidet_lockstep_medium_excitation():
    s = config_system("medium")
    trial = excitation_trial(s, 6, seed=2)
    log("multidet lockstep medium excitation fp64")
    worst, *_ = run_lockstep(s, 8, 10, dtau=0.005, label="md-medium", trial=trial)
    log(f"  worst {worst}")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_multidet_lockstep_mixed_precision(precision):
    s = config_system("tiny")
    trial = noci_trial(s, 4, seed=3)
    log(f"multidet lockstep {precision}")
    worst, *_ = run_lockstep(s, 16, 30, dtau=0.01, precision=precision, rtol=1e-4,
                             label=f"md-{precision}", trial=trial)
    log(f"  worst {worst}")


def test_multidet_closed_shell_mean_field():
    s = config_system("tiny")
    coeffs, ups, _ = noci_trial(s, 4, seed=6)
    log("multidet closed shell + mean field")
    worst, gs, wk, *_ = run_lockstep(s, 16, 30, dtau=0.01, label="md-cs-mf", mean_field=True,
                                     closed_shell=True, trial=(coeffs, ups, ups))
    assert gs.ntot == s.n_up
    log(f"  worst {worst}")


def test_single_determinant_expansion_equals_single_trial():
    import paper_1711_02242_amd as afq
    s = config_system("medium")
    Uu, Ud = random_walkers(s, 8, seed=3, amplitude=0.5)
    log("multidet n_det=1 vs single")
    g1 = afq.System.from_synthetic(s, dtau=0.005, precision="fp64")
    a1, l1, e1 = gpu_measure(g1, Uu, Ud)
    g2 = multi_system(s, ([2.0 + 0j], [s.phi_up], [s.phi_dn]), dtau=0.005, precision="fp64")
    a2, l2, e2 = gpu_measure(g2, Uu, Ud)
    assert np.abs(e1 - e2).max() <= 1e-12 * np.abs(e1).max()
    assert np.abs(l2 - (l1 + np.log(2.0))).max() <= 1e-12 * max(1.0, np.abs(l1).max())
    assert angle_diff(a1, a2).max() <= 1e-12
    g1.close()
    g2.close()


def fci_expansion(s, fs, evec):
    ups, dns, coeffs = [], [], []
    for n, bits in enumerate(fs.states[fs.full]):
        ups.append(occupation_det(s.M, [p for p in range(s.M) if bits >> p & 1]))
        dns.append(occupation_det(s.M, [p for p in range(s.M) if bits >> (s.M + p) & 1]))
        coeffs.append(evec[n])
    return np.array(coeffs) + 0j, ups, dns


def test_full_ci_expansion_zero_variance():
    """The exact ground state written as its 784 occupation-number determinants (M = 8, 2 + 2
    electrons): every walker non-orthogonal to all of them has E_L = E0."""
    s = config_system("tiny")
    fs = F.FockSpace(s.M, s.n_up, s.n_dn)
    H = fs.hamiltonian(s.h0, s.h1, F.eri_from_cholesky(s.L))
    evals, evecs = np.linalg.eigh(H)
    trial = fci_expansion(s, fs, evecs[:, 0])
    log(f"full-CI expansion n_det={len(trial[0])}")
    gs = multi_system(s, trial, dtau=0.01, precision="fp64")
    Uu, Ud = random_walkers(s, 6, seed=11, amplitude=1.5)
    a, l, e = gpu_measure(gs, Uu, Ud)
    log(f"  max |E_L - E0| = {np.abs(e - evals[0]).max():.2e}")
    assert np.abs(e - evals[0]).max() < 1e-9
    MS = A.setup_multi(s.h0, s.h1, s.L, *trial, 0.01)
    ra, rl, _ = oracle_measure(MS, Uu[:2], Ud[:2])
    assert angle_diff(a[:2], ra).max() < 1e-10 and np.abs(l[:2] - rl).max() < 1e-10
    gs.close()


def test_walkers_orthogonal_to_some_determinants():
    """Walkers started at the leading occupation-number determinant are exactly orthogonal to
    every determinant that differs from it; those terms are skipped on both sides."""
    s = config_system("tiny")
    fs = F.FockSpace(s.M, s.n_up, s.n_dn)
    rng = np.random.default_rng(4)
    coeffs, ups, dns = fci_expansion(s, fs, rng.standard_normal(len(fs.states[fs.full])))
    order = [int(np.argmax(np.abs(coeffs)))]
    order += [d for d in range(len(coeffs)) if d != order[0]]
    trial = (coeffs[order][:60], [ups[d] for d in order][:60], [dns[d] for d in order][:60])
    log("multidet with exactly orthogonal determinants")
    MS = A.setup_multi(s.h0, s.h1, s.L, *trial, 0.01)
    gs = multi_system(s, trial, dtau=0.01, precision="fp64")
    import torch
    wk = gs.walkers(4)
    gs.init(wk)
    torch.cuda.synchronize()
    wo = A.init_walkers(MS, 4)
    assert np.abs(wk.e_loc.cpu().numpy() - wo.e_loc).max() <= 1e-11 * np.abs(wo.e_loc).max()
    assert (wk.weight.cpu().numpy() == 1.0).all()
    gs.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_multidet_wide_shape(precision):
    """A three-determinant NOCI trial at N = 34+30, M = 136 (the wide contraction kernel)."""
    from synthetic import gen_system
    s = gen_system(136, 34, 40, seed=33, n_dn=30)
    trial = noci_trial(s, 3, seed=4, angle=0.3)
    log(f"multidet wide {precision}")
    MS = A.setup_multi(s.h0, s.h1, s.L, *trial, 0.005)
    Uu, Ud = walkers_near_lead(s, trial, 4, seed=6, amplitude=0.4)
    gs = multi_system(s, trial, dtau=0.005, precision=precision)
    ref = oracle_measure(MS, Uu, Ud)
    got = gpu_measure(gs, Uu, Ud)
    assert_measure_close(got, ref, 1e-10, precision, np.inf)
    kappa = cancellation(MS, Uu, Ud)
    assert np.all(np.abs(got[2] - ref[2]) <= kappa * EL_TOL)
    gs.close()
