"""The stacked-row contraction variants against the FP64 oracle: tile "flat" (the N-row blocks
of q consecutive Cholesky vectors stacked, [Re Theta | Im Theta] side by side in 16-column
blocks) and tile "stack" (the same rows, Re and Im Theta as two 16-column operands), on shapes
that exercise their group boundaries: a tail group shorter than q, unequal spins (different q per
spin), an empty spin, N below and above 16, no Cholesky vectors, the wide shapes, and a
multi-determinant trial.  Static: per-walker E_L within 1e-4 Ha.  Dynamic: lockstep runs, in
which the force-bias traces of every Cholesky vector drive the propagation (a trace written
to the wrong vector leaves sum_g t_g^2, hence E_L, unchanged but not the walk)."""

import numpy as np
import pytest

from oracle import afqmc as A
from synthetic import config_system, gen_system, noci_trial, random_walkers
from tests.parity_helpers import gpu_state, log, make_pair, oracle_U_to_gpu, run_lockstep

pytestmark = pytest.mark.gpu

EL_TOL = 1e-4   # Ha per walker

SHAPES = {
    # name: (system builder, walkers)
    "tiny": (lambda: config_system("tiny"), 12),                        # N 2: q 8
    "ragged_tail": (lambda: gen_system(13, 3, 19, seed=5), 7),          # N 3: q 16, tail of 3
    "open_shell": (lambda: gen_system(40, 11, 150, seed=6, n_dn=7), 9),  # q differs per spin
    "empty_spin": (lambda: gen_system(10, 3, 12, seed=7, n_dn=0), 6),
    "n1": (lambda: gen_system(12, 1, 10, seed=8, n_dn=2), 5),
    "n16": (lambda: gen_system(50, 16, 300, seed=11), 6),
    "n17_m70": (lambda: gen_system(70, 17, 120, seed=12, n_dn=15), 5),
    "n21_m86": (lambda: gen_system(86, 21, 100, seed=13), 5),
    "n34_m136": (lambda: gen_system(136, 34, 40, seed=31, n_dn=30), 5),
    "n40_m160": (lambda: gen_system(160, 40, 60, seed=31), 4),
    "n50_m200": (lambda: gen_system(200, 50, 30, seed=31, n_dn=48), 3),
    "n64_m96": (lambda: gen_system(96, 64, 30, seed=31, n_dn=60), 3),
}


TILES = ["flat", "stack"]


def _supported(tile, precision, s):
    """The stacked-row BF16x3 kernel holds at most 3 row tiles (N <= 48)."""
    return not (tile == "stack" and precision == "bf16x3" and max(s.n_up, s.n_dn) > 48)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("shape", list(SHAPES))
def test_flat_static_local_energy(shape, precision, tile):
    import torch

    import paper_1711_02242_amd as afq
    make, nw = SHAPES[shape]
    s = make()
    log(f"{tile} static {precision} {shape} M={s.M} N={s.n_up}+{s.n_dn} G={s.n_chol}")
    if not _supported(tile, precision, s):
        gs = afq.System.from_synthetic(s, dtau=0.005, precision=precision)
        with pytest.raises(afq.AfqmcError):
            gs.set_tile(tile)
        return
    U = random_walkers(s, nw, seed=99, amplitude=0.4)
    S, P, wo, gs, wk = make_pair(s, nw, dtau=0.005, precision=precision, U=U, tile=tile)
    assert gs.tile == tile
    st = gpu_state(wk)
    err = np.abs(st["e"] - wo.e_loc).max()
    log(f"  max |dE_L| = {err:.3e} Ha")
    assert err < EL_TOL
    # the variant the system would use otherwise agrees closely on the same walkers
    gs.set_tile("default")
    gs.measure(wk)
    torch.cuda.synchronize()
    e_def = wk.e_loc.cpu().numpy()
    assert np.abs(st["e"] - e_def).max() < 2e-5


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["ragged_tail", "open_shell", "empty_spin", "n17_m70",
                                  "n34_m136", "no_cholesky"])
def test_flat_dynamic_drift(case, precision, tile):
    if case == "no_cholesky":
        s, nw = gen_system(9, 2, 0, seed=8), 5
        steps, dt = 10, 0.05
    else:
        make, nw = SHAPES[case]
        s = make()
        steps, dt = (12, 0.01) if s.M <= 40 else (5, 0.005)
    log(f"{tile} dynamic {precision} {case}")
    worst, gs, wk, S, wo = run_lockstep(s, nw, steps, dtau=dt, precision=precision, rtol=1e-4,
                                        label=f"{tile}-{case}-{precision}", tile=tile,
                                        el_abs=EL_TOL)
    st = gpu_state(wk)
    alive = wo.W > 0
    assert np.abs(st["e"][alive] - wo.e_loc[alive]).max() < EL_TOL
    log(f"  worst {worst}")


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_flat_multidet_lockstep(precision, tile):
    s = config_system("tiny")
    trial = noci_trial(s, 4, seed=3)
    log(f"{tile} multidet lockstep {precision}")
    worst, *_ = run_lockstep(s, 16, 30, dtau=0.01, precision=precision, rtol=1e-4,
                             label=f"{tile}-md-{precision}", trial=trial, tile=tile)
    log(f"  worst {worst}")


@pytest.mark.parametrize("tile", TILES)
def test_flat_is_deterministic(tile):
    """No atomics: two launches on the same walkers give the same bits."""
    import torch

    import paper_1711_02242_amd as afq
    s = gen_system(86, 21, 100, seed=13)
    gs = afq.System.from_synthetic(s, dtau=0.005, precision="fp32")
    gs.set_tile(tile)
    wk = gs.walkers(64)
    gs.init(wk)
    Uu, Ud = random_walkers(s, 64, seed=4, amplitude=0.4)
    wk.U.copy_(torch.from_numpy(oracle_U_to_gpu(Uu, Ud)))
    gs.measure(wk)
    torch.cuda.synchronize()
    a = wk.e_loc.cpu().numpy().copy()
    gs.measure(wk)
    torch.cuda.synchronize()
    assert np.array_equal(a, wk.e_loc.cpu().numpy())


def test_flat_refused_in_fp64():
    import paper_1711_02242_amd as afq
    s = config_system("tiny")
    gs = afq.System.from_synthetic(s, dtau=0.01, precision="fp64")
    for tile in TILES:
        with pytest.raises(afq.AfqmcError):
            gs.set_tile(tile)
