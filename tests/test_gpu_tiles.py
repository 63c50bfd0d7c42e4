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
    "n24_m64": lambda: (gen_system(64, 24, 100, seed=51), 9),    # N_P 32: w4, w2, wide, bx
    "medium": lambda: (config_system("medium"), 10),             # N_P 16: w4, w2
    "n35_m140": lambda: (gen_system(140, 35, 60, seed=53), 5),   # N_P 48: wide, flat, stack
}
TILES = ("w4", "w2", "wide", "flat", "stack", "pp", "bx", "bx8")


def valid_tiles(s, precision):
    """The variants the library accepts for a shape (N_P from max N, wide beyond N = 32 or
    M = 128)."""
    n = max(s.n_up, s.n_dn)
    NP = 16 if n <= 16 else 32 if n <= 32 else 48 if n <= 48 else 64
    KP = (s.M + 31) // 32 * 32
    wide = NP > 32 or s.M > 128
    ok = {"flat", "stack"}
    if not wide:
        ok |= {"w4", "w2", "pp"}
    if not wide and NP == 32:
        ok |= {"bx", "bx8"}
    if NP >= 32 and KP <= 224:
        ok.add("wide")
    return ok


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
    ok = valid_tiles(s, precision)
    for tile in TILES:
        if tile not in ok:
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
    base = "w4" if "w4" in energies else "wide"
    for tile, e in energies.items():
        assert np.abs(e - energies[base]).max() < 2e-5, tile
    # the same per-wavefront arithmetic in another schedule: identical results
    if "pp" in energies:
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
    assert tile in TILES and ms > 0 and gs.tile == tile
    gs2 = afq.System.from_synthetic(s, dtau=0.005, precision="fp32")
    wk2 = gs2.walkers(64)
    gs2.init(wk2)
    tile2, ms2 = gs2.autotune(wk2, reuse=True)
    assert tile2 == tile and ms2 == -1.0
    g64 = afq.System.from_synthetic(s, dtau=0.005, precision="fp64")
    w64 = g64.walkers(8)
    g64.init(w64)
    assert g64.autotune(w64, reuse=False)[0] == "default"
