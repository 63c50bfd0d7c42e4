"""Contraction tile variants (walkers per workgroup, wide, flattened, stacked-row, ping-pong and
block-exchange kernels) and the autotuner: every
variant meets the parity bar against the FP64 oracle, and the variants agree with each other."""

import numpy as np
import pytest

from oracle import afqmc as A
from synthetic import config_system, gen_system, random_walkers
from tests.parity_helpers import log, oracle_U_to_gpu

pytestmark = pytest.mark.gpu

EL_TOL = 1e-4   # Ha per walker
SHAPES = {
    "tiny": lambda: (config_system("tiny"), 13),                 # N_P 16: w4, w2
    "n24_m64": lambda: (gen_system(64, 24, 100, seed=51), 9),    # N_P 32: w4, w2, wide
    "medium": lambda: (config_system("medium"), 10),             # N_P 16: w4, w2
}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_every_tile_meets_the_bar(shape, precision):
    import torch

    import paper_1711_02242_amd as afq
    s, nw = SHAPES[shape]()
    Uu, Ud = random_walkers(s, nw, seed=99, amplitude=0.5)
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, 0.005)
    ref = A.init_walkers(S, nw, Uu, Ud).e_loc
    gs = afq.System.from_synthetic(s, dtau=0.005, precision=precision)
    wk = gs.walkers(nw)
    gs.init(wk)
    wk.U.copy_(torch.from_numpy(oracle_U_to_gpu(Uu, Ud)))
    energies = {}
    for tile in ("w4", "w2", "wide", "flat", "stack", "pp", "bx", "bx8"):
        if tile in ("wide", "bx", "bx8") and max(s.n_up, s.n_dn) <= 16:
            with pytest.raises(afq.AfqmcError):
                gs.set_tile(tile)
            continue
        gs.set_tile(tile)
        gs.measure(wk)
        torch.cuda.synchronize()
        e = wk.e_loc.cpu().numpy()
        d = np.abs(e - ref).max()
        log(f"{shape} {precision} {tile}: max |dE_L| = {d:.2e} Ha")
        assert d < EL_TOL
        energies[tile] = e
    for tile, e in energies.items():
        assert np.abs(e - energies["w4"]).max() < 2e-5, tile
    # the same per-wavefront arithmetic in another schedule: identical results
    assert np.array_equal(energies["pp"], energies["w4"])
    if "bx" in energies:
        assert np.array_equal(energies["bx8"], energies["bx"])


def test_autotune_picks_a_valid_tile_and_reuses_it():
    import paper_1711_02242_amd as afq
    s = gen_system(64, 24, 100, seed=51)
    gs = afq.System.from_synthetic(s, dtau=0.005, precision="fp32")
    wk = gs.walkers(64)
    gs.init(wk)
    tile, ms = gs.autotune(wk, reuse=False)
    log(f"autotune: {tile} {ms:.3f} ms")
    assert tile in ("w4", "w2", "wide", "flat", "stack", "pp", "bx", "bx8") and ms > 0 and gs.tile == tile
    gs2 = afq.System.from_synthetic(s, dtau=0.005, precision="fp32")
    wk2 = gs2.walkers(64)
    gs2.init(wk2)
    tile2, ms2 = gs2.autotune(wk2, reuse=True)
    assert tile2 == tile and ms2 == -1.0
    g64 = afq.System.from_synthetic(s, dtau=0.005, precision="fp64")
    w64 = g64.walkers(8)
    g64.init(w64)
    assert g64.autotune(w64, reuse=False)[0] == "default"
