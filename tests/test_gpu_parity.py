"""GPU (HIP, through the C ABI) against the CPU oracle on identical seeded inputs.

FP64 bar: relative 1e-10 on E_L, W and U, absolute 1e-10 on the overlap phase.
"""

import numpy as np
import pytest

from oracle import afqmc as A
from synthetic import config_system, gaussian_fields, gen_system, random_walkers
from tests.parity_helpers import (angle_diff, compare_state, gpu_state, gpu_U_to_oracle, log, make_pair,
                                  oracle_U_to_gpu, run_lockstep)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def test_gpu_fields_match_counter_stream(torch_cuda):
    """Philox4x64-10 fields drawn on the device equal the counter stream of synthetic.fields."""
    for G in (32, 37, 800):
        s = gen_system(8, 2, G, seed=3)
        log(f"fields G={G}")
        _, _, wo, gs, wk = make_pair(s, 9, dtau=0.01)
        wk.walker_id.copy_(torch_cuda.tensor([3, 1, 4, 1, 5, 9, 2, 6, 5], dtype=torch_cuda.int64))
        wk.step = 17
        x_gpu = gs.fields_draw(wk, seed=12345, job_id=7).cpu().numpy()
        x_ref = gaussian_fields(12345, 7, [3, 1, 4, 1, 5, 9, 2, 6, 5], 17, G)
        assert np.abs(x_gpu - x_ref).max() < 1e-13


@pytest.mark.parametrize("name", ["tiny", "medium", "large"])
def test_gpu_init_energy_is_trial_energy(torch_cuda, name):
    s = config_system(name)
    log(f"init {name}")
    S, P, wo, gs, wk = make_pair(s, 8, dtau=0.005)
    st = gpu_state(wk)
    assert abs(gs.e_hf - S.E_T) < 1e-11 * abs(S.E_T)
    assert np.abs(st["e"] - S.E_T).max() < 1e-11 * abs(S.E_T)
    assert np.all(st["W"] == 1.0) and np.abs(st["arg"]).max() < 1e-12
    assert np.array_equal(st["ids"], np.arange(8))


@pytest.mark.parametrize("case", ["tiny", "medium", "large", "ragged", "open_shell", "polarized"])
def test_gpu_measure_random_walkers(torch_cuda, case):
    """Overlap phase, log|overlap| and E_L of arbitrary complex walkers (Theorem 1.1-1.2,
    eq:localenergy3) against the oracle."""
    if case in ("tiny", "medium", "large"):
        s = config_system(case)
        nw = {"tiny": 16, "medium": 24, "large": 6}[case]
    elif case == "ragged":
        s = gen_system(13, 3, 19, seed=5)
        nw = 7
    elif case == "open_shell":
        s = gen_system(24, 5, 70, seed=6, n_dn=3)
        nw = 5
    else:
        s = gen_system(10, 3, 12, seed=7, n_dn=0)
        nw = 4
    log(f"measure {case} M={s.M} up={s.n_up} dn={s.n_dn} G={s.n_chol} nw={nw}")
    U = random_walkers(s, nw, seed=99, amplitude=0.8)
    S, P, wo, gs, wk = make_pair(s, nw, dtau=0.005, U=U)
    compare_state(S, wo, gpu_state(wk), s.n_up, 1e-10, case)
    assert np.abs(gpu_state(wk)["logabs"] - wo.logabs).max() < 1e-10


def test_gpu_lockstep_tiny_explicit_fields(torch_cuda):
    """Tiny molecule (M=8, N=2+2, N_g=32), 16 walkers, 200 steps, QR and comb every 5 steps."""
    s = config_system("tiny")
    log("lockstep tiny explicit")
    worst, *_ = run_lockstep(s, 16, 200, dtau=0.01, label="tiny")
    log(f"tiny worst {worst}")


def test_gpu_lockstep_tiny_device_philox(torch_cuda):
    """Same run with the fields drawn on the device from the counter stream."""
    s = config_system("tiny")
    log("lockstep tiny device philox")
    worst, *_ = run_lockstep(s, 16, 60, dtau=0.01, explicit_fields=False, label="tiny-philox",
                             rtol=1e-9)
    log(f"tiny philox worst {worst}")


@pytest.mark.parametrize("case", ["medium", "ragged", "open_shell", "polarized", "no_cholesky"])
def test_gpu_lockstep_shapes(torch_cuda, case):
    if case == "medium":
        s, nw, steps, dt = config_system("medium"), 12, 10, 0.005
    elif case == "ragged":
        s, nw, steps, dt = gen_system(13, 3, 19, seed=5), 7, 12, 0.01
    elif case == "open_shell":
        s, nw, steps, dt = gen_system(24, 5, 70, seed=6, n_dn=3), 9, 10, 0.01
    elif case == "polarized":
        s, nw, steps, dt = gen_system(10, 3, 12, seed=7, n_dn=0), 6, 10, 0.01
    else:
        s, nw, steps, dt = gen_system(9, 2, 0, seed=8), 5, 10, 0.05
    log(f"lockstep {case} M={s.M} up={s.n_up} dn={s.n_dn} G={s.n_chol} nw={nw}")
    worst, *_ = run_lockstep(s, nw, steps, dtau=dt, label=case)
    log(f"{case} worst {worst}")


def test_gpu_lockstep_large_sample(torch_cuda):
    """Full-size Hamiltonian (M=128, N=32+32, N_g=800) on a sample of 4 walkers, 5 steps
    (QR and comb after the fifth)."""
    s = config_system("large")
    log("lockstep large sample")
    worst, *_ = run_lockstep(s, 4, 5, dtau=0.005, label="large", check_every=5)
    log(f"large worst {worst}")


def test_gpu_phaseless_kill_and_comb_replacement(torch_cuda):
    """A walker whose overlap phase jumps by 0.75 pi gets W = 0 (eq:if_rle), stays dead, and
    the comb replaces it; the oracle does the same."""
    import torch
    s = config_system("tiny")
    S, P, wo, gs, wk = make_pair(s, 6, dtau=0.01)
    wo.U[0][2][:, 0] *= np.exp(0.75j * np.pi)
    wk.U[2, 0, :] *= np.exp(0.75j * np.pi)
    for k in range(5):
        x = gaussian_fields(0, 0, wo.walker_id, k, s.n_chol)
        A.step(S, P, wo, x, 0.37)
        gs.step(wk, x=torch.from_numpy(x).cuda(), u_comb=0.37)
        st = gpu_state(wk)
        if k < 4:
            assert st["W"][2] == 0.0 and wo.W[2] == 0.0
        compare_state(S, wo, st, s.n_up, 1e-10, f"kill step {k}")
    assert np.all(gpu_state(wk)["W"] > 0)
    assert gs.status() & 0x20


def test_gpu_run_is_deterministic(torch_cuda):
    """Two identical runs give bitwise-identical walkers (fixed-order reductions, no FP atomics)."""
    s = config_system("medium")
    outs = []
    for rep in range(2):
        _, _, _, gs, wk = make_pair(s, 16, dtau=0.005)
        for k in range(6):
            gs.step(wk, seed=4)
        st = gpu_state(wk)
        outs.append(st)
        gs.close()
    for key in ("U", "W", "arg", "e"):
        assert np.array_equal(outs[0][key], outs[1][key]), key


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gpu_singular_and_nonfinite_walkers_are_killed(torch_cuda, precision):
    """A walker with a zero orbital (singular overlap) or a NaN entry gets W = 0 and sets the
    status word; the other walkers are untouched and the estimator stays finite."""
    s = config_system("medium")
    _, _, wo, gs, wk = make_pair(s, 6, dtau=0.005, precision=precision)
    e_before = gpu_state(wk)["e"].copy()
    wk.U[1, 3, :] = 0.0
    wk.U[4, 20, 7] = float("nan")
    gs.measure(wk)
    st = gpu_state(wk)
    assert st["W"][1] == 0.0 and st["W"][4] == 0.0
    assert np.all(st["W"][[0, 2, 3, 5]] == 1.0)
    assert np.array_equal(st["e"][[0, 2, 3, 5]], e_before[[0, 2, 3, 5]])
    assert gs.status() & 0x2
    a, b, c, n, status = gs.energy(wk)
    assert n == 4 and np.isfinite(a) and c == 4.0
    gs.step(wk, seed=1)
    assert gpu_state(wk)["W"][1] == 0.0


@pytest.mark.parametrize("case", ["n34_m136", "n48_m200", "n20_m232"])
def test_gpu_fp64_beyond_mfma_tile_limits(torch_cuda, case):
    """FP64 sizes outside the register-resident MFMA tiles (N > 32 or M > 128) run the FP64
    VALU contraction, with the overlap on k_overlap_mfma<48> beyond N = 32.  n20_m232 keeps
    N <= 32 at M = 232: the one-wavefront overlap with a ragged K tail (232 = 14.5 x 16) and the
    register Gram-Schmidt with four elements per lane, whose QR runs at the fifth step."""
    if case == "n34_m136":
        s, nw, steps = gen_system(136, 34, 40, seed=21, n_dn=30), 3, 5
    elif case == "n48_m200":
        s, nw, steps = gen_system(200, 48, 24, seed=22, n_dn=40), 2, 5
    else:
        s, nw, steps = gen_system(232, 20, 6, seed=1), 2, 6
    log(f"fp64 large shape {case}")
    worst, *_ = run_lockstep(s, nw, steps, dtau=0.005, label=case)
    log(f"{case} worst {worst}")


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["large", "medium"])
def test_full_size_bench_launch_sampled(torch_cuda, precision, case):
    """Full walker counts: the launch the benchmark times (large: M=128, N=32+32, N_g=800, 1024
    walkers) and the medium workload (M=64, N=16+16, N_g=320, 512 walkers), fields drawn on the
    device, QR and comb every 5 steps.  After three steps the state is copied, the fourth step
    runs on the GPU, and the oracle repeats that step for sampled walkers one by one from the
    copied state (its own Philox fields for the walkers' ids, force bias from their U)."""
    import torch

    import paper_1711_02242_amd as afq
    s = config_system(case)
    nw, seed, dt = (1024, 0, 0.005) if case == "large" else (512, 0, 0.005)
    log(f"full-size launch sampled {case} {precision}")
    gs = afq.System.from_synthetic(s, dtau=dt, precision=precision, qr_period=5, pop_period=5)
    wk = gs.walkers(nw)
    gs.init(wk)
    for _ in range(3):
        gs.step(wk, seed=seed)
    before = gpu_state(wk)
    k = wk.step
    gs.step(wk, seed=seed)
    after = gpu_state(wk)
    gs.close()
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, dt)
    P = A.Params(dtau=dt, qr_period=5, pop_period=5, w_max=max(100.0, nw / 10.0))
    sample = np.array([0, nw // 3, (3 * nw) // 4, nw - 1])
    Uu, Ud = gpu_U_to_oracle(before["U"][sample], s.n_up)
    wo = A.init_walkers(S, len(sample), Uu, Ud)
    wo.W = before["W"][sample].copy()
    wo.walker_id = before["ids"][sample].copy()
    wo.step = k
    # the GPU's cached state stands for the walkers' (arg, log|ovlp|, E_L): the oracle's
    # measurement of the same U agrees to rounding
    assert angle_diff(wo.arg, before["arg"][sample]).max() < 1e-9
    x = gaussian_fields(seed, 0, wo.walker_id, k, s.n_chol)
    A.step(S, P, wo, x, None)
    Ug_u, Ug_d = gpu_U_to_oracle(after["U"][sample], s.n_up)
    tolU, tolE = (1e-10, 1e-10) if precision == "fp64" else (2e-5, 1e-4)
    dU = max(np.abs(Ug_u - wo.U[0]).max(), np.abs(Ug_d - wo.U[1]).max()) / np.abs(wo.U[0]).max()
    dW = np.abs(after["W"][sample] - wo.W).max() / np.abs(wo.W).max()
    dA = angle_diff(after["arg"][sample], wo.arg).max()
    dE = np.abs(after["e"][sample] - wo.e_loc).max()
    log(f"  dU {dU:.2e} dW {dW:.2e} darg {dA:.2e} dE {dE:.2e} Ha")
    assert dU < tolU and dW < max(tolU, 1e-8) and dA < max(tolU, 1e-8)
    assert dE < (tolE * np.abs(wo.e_loc).max() if precision == "fp64" else tolE)
