"""Every compile-time shape of the register-resident contraction and of the fused propagation
against the FP64 oracle.  The contraction kernels are instantiated per K chunk count (K_P = 32,
64, 96, 128) for N_P = 16 and 32, in FP32 and BF16x3 with four or two walkers per workgroup and
in FP64; the propagation per (K_P / 16, row blocks of 16).  Static: per-walker E_L (FP32 /
BF16x3 within 1e-4 Ha, FP64 relative 1e-10).  Dynamic: lockstep FP32 steps, which run the
propagation on the shapes below (K_P / 16 = 2 .. 8, one to four row blocks)."""

import numpy as np
import pytest

from synthetic import gen_system, random_walkers
from tests.parity_helpers import compare_state, gpu_state, log, make_pair, run_lockstep

pytestmark = pytest.mark.gpu

EL_TOL = 1e-4   # Ha per walker

SHAPES = {
    # name: (M, N_up, N_dn, N_g, walkers)   ->  N_P, K_P; propagation K_P / 16, row blocks
    "np32_k32": (32, 24, 20, 30, 6),     # 32, 32;   2, 3
    "np16_k64": (40, 10, 9, 30, 7),      # 16, 64;   3, 2
    "np16_k96": (80, 14, 12, 40, 6),     # 16, 96;   5, 2
    "np32_k96": (90, 30, 22, 40, 5),     # 32, 96;   6, 4
    "np16_k128": (120, 16, 9, 30, 5),    # 16, 128;  8, 2
    "np32_k128": (128, 32, 32, 30, 5),   # 32, 128;  8, 4
    "small_rows": (20, 5, 3, 12, 6),     # 16, 32;   2, 1
}


def _system(name):
    M, nu, nd, G, nw = SHAPES[name]
    return gen_system(M, nu, G, seed=70 + M, n_dn=nd), nw


@pytest.mark.parametrize("tile", ["w4", "w2"])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_contraction_every_k_chunk_count(shape, precision, tile):
    s, nw = _system(shape)
    log(f"k-chunks {shape} {precision} {tile}: M={s.M} N={s.n_up}+{s.n_dn} G={s.n_chol}")
    U = random_walkers(s, nw, seed=5, amplitude=0.5)
    S, P, wo, gs, wk = make_pair(s, nw, dtau=0.005, precision=precision, U=U, tile=tile)
    assert gs.tile == tile
    err = np.abs(gpu_state(wk)["e"] - wo.e_loc).max()
    log(f"  max |dE_L| = {err:.3e} Ha")
    assert err < EL_TOL


@pytest.mark.parametrize("shape", list(SHAPES))
def test_fp64_contraction_every_k_chunk_count(shape):
    s, nw = _system(shape)
    log(f"k-chunks fp64 {shape}: M={s.M} N={s.n_up}+{s.n_dn} G={s.n_chol}")
    U = random_walkers(s, nw, seed=6, amplitude=0.5)
    S, P, wo, gs, wk = make_pair(s, nw, dtau=0.005, precision="fp64", U=U)
    compare_state(S, wo, gpu_state(wk), s.n_up, 1e-10, shape)


@pytest.mark.parametrize("shape", list(SHAPES))
def test_propagation_every_shape_lockstep(shape):
    s, nw = _system(shape)
    log(f"propagation lockstep fp32 {shape}")
    worst, *_ = run_lockstep(s, nw, 3, dtau=0.005, precision="fp32", rtol=1e-4,
                             label=f"kchunks-{shape}", el_abs=1e-4)
    log(f"  worst {worst}")
