"""Multi-determinant trial wavefunctions (Sec. III.D.1, eq:usesherman, eq:precomputing2,
eq:localenergy2) in the oracle, pinned in Fock space."""

from itertools import combinations

import numpy as np
import pytest

from oracle import afqmc as A
from oracle import fock as F
from synthetic import config_system, random_walkers
from synthetic import excitation_trial, noci_trial, occupation_det as occ_det


@pytest.fixture(scope="module")
def tiny_fock():
    s = config_system("tiny")
    fs = F.FockSpace(8, 2, 2)
    H = fs.hamiltonian(s.h0, s.h1, F.eri_from_cholesky(s.L))
    return s, fs, H


def test_multidet_overlap_energy_traces_match_fock(tiny_fock):
    s, fs, H = tiny_fock
    coeffs, ups, dns = excitation_trial(s, 5, seed=1)
    MS = A.setup_multi(s.h0, s.h1, s.L, coeffs, ups, dns, 0.01)
    phiT = sum(c * fs.slater(u.astype(complex), d.astype(complex)) for c, u, d in zip(coeffs, ups, dns))
    lead = fs.slater(ups[0].astype(complex), dns[0].astype(complex))
    assert abs(MS.E_T - (np.vdot(lead, H @ lead) / np.vdot(lead, lead)).real) < 1e-11
    Uu, Ud = random_walkers(s, 3, seed=7, amplitude=1.0)
    Lg = fs.one_body(s.L[3])
    for w in range(3):
        psi = fs.slater(Uu[w], Ud[w])
        ov = np.vdot(phiT, psi)
        a, la, e, t = A.measure_multi(MS, Uu[w], Ud[w])
        assert abs(np.exp(la + 1j * a) - ov) < 1e-12 * abs(ov)
        assert abs(e - np.vdot(phiT, H @ psi) / ov) < 1e-11 * abs(e)
        assert abs(t[3] - np.vdot(phiT, Lg @ psi) / ov) < 1e-12


def test_noci_trial_energy_is_rayleigh_quotient(tiny_fock):
    s, fs, H = tiny_fock
    coeffs, ups, dns = noci_trial(s, 4, seed=5)
    MS = A.setup_multi(s.h0, s.h1, s.L, coeffs, ups, dns, 0.01)
    phiT = sum(c * fs.slater(u.astype(complex), d.astype(complex)) for c, u, d in zip(coeffs, ups, dns))
    ref = (np.vdot(phiT, H @ phiT) / np.vdot(phiT, phiT)).real
    assert abs(A.trial_energy_multi(MS) - ref) < 1e-11
    Uu, Ud = random_walkers(s, 2, seed=9, amplitude=0.7)
    for w in range(2):
        psi = fs.slater(Uu[w], Ud[w])
        _, _, e, _ = A.measure_multi(MS, Uu[w], Ud[w])
        assert abs(e - np.vdot(phiT, H @ psi) / np.vdot(phiT, psi)) < 1e-11 * abs(e)


def test_full_ci_trial_has_zero_variance(tiny_fock):
    """With the exact ground state written as a 784-determinant expansion the local energy of
    every walker equals E0 (Sec. III.D.1: E_L = E0 when Psi_T = Phi_0)."""
    s, fs, H = tiny_fock
    evals, evecs = np.linalg.eigh(H)
    gs = evecs[:, 0]
    ups, dns, coeffs = [], [], []
    for n, bits in enumerate(fs.states[fs.full]):
        up = [p for p in range(8) if bits >> p & 1]
        dn = [p for p in range(8) if bits >> (8 + p) & 1]
        ups.append(occ_det(8, up))
        dns.append(occ_det(8, dn))
        coeffs.append(gs[n])
    MS = A.setup_multi(s.h0, s.h1, s.L, np.array(coeffs), ups, dns, 0.01)
    Uu, Ud = random_walkers(s, 2, seed=11, amplitude=1.5)
    for w in range(2):
        _, _, e, _ = A.measure_multi(MS, Uu[w], Ud[w])
        assert abs(e - evals[0]) < 1e-9


def test_single_determinant_expansion_equals_single_setup():
    s = config_system("medium")
    MS = A.setup_multi(s.h0, s.h1, s.L, [2.0 + 0j], [s.phi_up], [s.phi_dn], 0.005)
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, 0.005)
    assert abs(MS.E_T - S.E_T) < 1e-12 * abs(S.E_T)
    Uu, Ud = random_walkers(s, 2, seed=3, amplitude=0.5)
    for w in range(2):
        a1, l1, e1, t1 = A.measure_multi(MS, Uu[w], Ud[w])
        a2, l2, e2, t2 = A.measure(S, Uu[w], Ud[w])
        assert abs(e1 - e2) < 1e-12 * abs(e2) and np.abs(t1 - t2).max() < 1e-12
        assert abs(l1 - (l2 + np.log(2.0))) < 1e-12 and abs(A.wrap_angle(a1 - a2)) < 1e-12


def test_multidet_mean_field_shifts_are_leading_determinant_expectations(tiny_fock):
    s, fs, H = tiny_fock
    coeffs, ups, dns = noci_trial(s, 4, seed=2)
    MS = A.setup_multi(s.h0, s.h1, s.L, coeffs, ups, dns, 0.01, mean_field=True)
    lead = fs.slater(ups[0].astype(complex), dns[0].astype(complex))
    for g in (0, 5, 31):
        Lg = fs.one_body(s.L[g])
        ref = (np.vdot(lead, Lg @ lead) / np.vdot(lead, lead)).real
        assert abs(MS.lbar[g] - ref) < 1e-12
