"""Regression of the oracle against its stored values (tests/golden/make_golden.py): a later
change to the oracle's arithmetic shows up here and must name its justification."""

import json
import os

import numpy as np

from oracle import afqmc as A
from oracle import fock as F
from synthetic import comb_uniform, config_system, gaussian_fields

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_tiny_golden_values():
    g = json.load(open(os.path.join(HERE, "tiny_oracle.json")))
    s = config_system("tiny")
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, 0.01)
    assert abs(S.E_T - g["e_hf"]) < 1e-12
    fs = F.FockSpace(8, 2, 2)
    H = fs.hamiltonian(s.h0, s.h1, F.eri_from_cholesky(s.L))
    assert np.allclose(np.linalg.eigvalsh(H)[:4], g["ed_lowest_four"], atol=1e-11)
    P = A.Params(dtau=0.01)
    wk = A.init_walkers(S, 16)
    series = []
    for k in range(20):
        A.step(S, P, wk, gaussian_fields(0, 0, wk.walker_id, k, s.n_chol), comb_uniform(0, 0, k))
        series.append(A.mixed_energy(S, P, wk)[0])
    assert np.allclose(series, g["mixed_energy_first_20_steps_16_walkers_dtau_0.01_seed_0"],
                       rtol=0, atol=1e-11)
