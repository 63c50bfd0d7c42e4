"""Write the stored expected values of tests/golden/ from the oracle alone.

    python tests/golden/make_golden.py

The paper prints no worked numerical example, so every stored value here is the
oracle's (or the exact diagonalization's) on the seeded synthetic inputs.
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import afqmc as A  # noqa: E402
from oracle import fock as F  # noqa: E402
from synthetic import comb_uniform, config_system, gaussian_fields  # noqa: E402


def main():
    s = config_system("tiny")
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, 0.01)
    fs = F.FockSpace(8, 2, 2)
    H = fs.hamiltonian(s.h0, s.h1, F.eri_from_cholesky(s.L))
    evals = np.linalg.eigvalsh(H)
    P = A.Params(dtau=0.01)
    wk = A.init_walkers(S, 16)
    series = []
    for k in range(20):
        A.step(S, P, wk, gaussian_fields(0, 0, wk.walker_id, k, s.n_chol), comb_uniform(0, 0, k))
        series.append(A.mixed_energy(S, P, wk)[0])
    out = {
        "source": "oracle/ and oracle/fock.py on synthetic 'tiny' (M=8, N=2+2, N_g=32, seed 1001)",
        "e_hf": S.E_T,
        "ed_lowest_four": evals[:4].tolist(),
        "mixed_energy_first_20_steps_16_walkers_dtau_0.01_seed_0": series,
    }
    with open(os.path.join(HERE, "tiny_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
