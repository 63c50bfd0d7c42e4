"""Modified Cholesky decomposition on the GPU against the oracle (same pivots, same vectors)."""

import numpy as np
import pytest

from oracle import fock as F
from oracle.mcd import eri_matrix, modified_cholesky
from synthetic import gen_system
from tests.parity_helpers import log

pytestmark = pytest.mark.gpu


def _eri(M, seed, n):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, M, M))
    B = B + B.transpose(0, 2, 1)
    w = np.exp(-np.arange(n) / (0.8 * M)) / M
    return np.einsum("k,kpr,kqs->pqrs", w, B, B)


@pytest.mark.parametrize("M,delta", [(8, 1e-4), (13, 1e-6), (24, 1e-5)])
def test_gpu_mcd_matches_oracle(M, delta):
    import torch

    import paper_1711_02242_amd as afq
    eri = _eri(M, M, M * M)
    log(f"mcd M={M} delta={delta}")
    Lo, piv = modified_cholesky(eri, delta)
    Lg, conv = afq.modified_cholesky(torch.from_numpy(eri).cuda(), delta)
    Lg = Lg.cpu().numpy()
    assert conv and len(Lg) == len(Lo)
    assert np.abs(Lg - Lo).max() < 1e-10 * np.abs(Lo).max()
    V = eri_matrix(eri)
    R = V - np.einsum("gm,gn->mn", Lg.reshape(len(Lg), -1), Lg.reshape(len(Lg), -1))
    assert np.abs(R).max() <= delta * (1 + 1e-9)
    log(f"  {len(Lg)} vectors")


def test_gpu_mcd_exact_rank_and_max_vectors():
    import torch

    import paper_1711_02242_amd as afq
    s = gen_system(10, 2, 9, seed=3)
    eri = F.eri_from_cholesky(s.L)
    Lg, conv = afq.modified_cholesky(torch.from_numpy(eri).cuda(), 1e-12)
    assert conv and len(Lg) <= 9
    assert np.abs(F.eri_from_cholesky(Lg.cpu().numpy()) - eri).max() < 1e-11
    L4, conv4 = afq.modified_cholesky(torch.from_numpy(eri).cuda(), 1e-12, max_vectors=4)
    assert len(L4) == 4 and not conv4
    assert np.abs(L4.cpu().numpy() - Lg.cpu().numpy()[:4]).max() < 1e-12
