"""Mixed-precision contraction (FP32 MFMA, BF16x3 MFMA) against the FP64 oracle.

Bar: per-walker local energy within 1e-4 Ha of the FP64 value on identical
walker states; the force-bias traces enter the dynamics, checked through short
lockstep runs whose drift from the oracle is bounded.
"""

import numpy as np
import pytest

from oracle import afqmc as A
from synthetic import config_system, gen_system, random_walkers
from tests.parity_helpers import gpu_state, log, make_pair, oracle_U_to_gpu, run_lockstep

pytestmark = pytest.mark.gpu

EL_TOL = 1e-4   # Ha, per walker


def _static(s, nw, precision, amplitude, seed=99, oracle_sample=None):
    import torch
    U = random_walkers(s, nw, seed=seed, amplitude=amplitude)
    S, P, wo, gs, wk = make_pair(s, nw, dtau=0.005, precision=precision, U=U)
    st = gpu_state(wk)
    n = nw if oracle_sample is None else oracle_sample
    err = np.abs(st["e"][:n] - wo.e_loc[:n]).max()
    arg_err = np.abs(st["arg"][:n] - wo.arg[:n]).max()
    return err, arg_err, gs, wk


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["tiny", "medium", "ragged", "open_shell", "n16"])
def test_static_local_energy(precision, case):
    if case in ("tiny", "medium"):
        s, nw = config_system(case), 24
    elif case == "ragged":
        s, nw = gen_system(13, 3, 19, seed=5), 7
    elif case == "open_shell":
        s, nw = gen_system(40, 11, 150, seed=6, n_dn=7), 9
    else:
        s, nw = gen_system(50, 16, 300, seed=11), 6
    log(f"static {precision} {case} M={s.M} N={s.n_up}+{s.n_dn} G={s.n_chol}")
    err, arg_err, gs, wk = _static(s, nw, precision, amplitude=0.5)
    log(f"  max |dE_L| = {err:.3e} Ha")
    assert err < EL_TOL
    assert arg_err < 1e-12      # overlaps stay FP64 in every mode


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_static_local_energy_large_all_walkers(precision):
    """Full workload (M=128, N=32+32, N_g=800, 1024 walkers, the launch the benchmark
    times): every walker's E_L against the GPU FP64 path, and a sample of 3 against the
    oracle itself."""
    import torch

    import paper_1711_02242_amd as afq
    s = config_system("large")
    nw = 1024
    log(f"static large {precision} all walkers")
    U = random_walkers(s, nw, seed=7, amplitude=0.3)
    Ug = torch.from_numpy(oracle_U_to_gpu(*U)).cuda()
    res = {}
    for prec in ("fp64", precision):
        gs = afq.System.from_synthetic(s, dtau=0.005, precision=prec)
        wk = gs.walkers(nw)
        gs.init(wk)
        wk.U.copy_(Ug)
        gs.measure(wk)
        torch.cuda.synchronize()
        res[prec] = wk.e_loc.cpu().numpy()
        gs.close()
    err = np.abs(res[precision] - res["fp64"]).max()
    log(f"  max |dE_L| vs GPU FP64 over 1024 walkers = {err:.3e} Ha")
    assert err < EL_TOL
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, 0.005)
    for w in (0, 511, 1023):
        _, _, e, _ = A.measure(S, U[0][w], U[1][w])
        assert abs(res["fp64"][w] - e) < 1e-10 * abs(e)
        assert abs(res[precision][w] - e) < EL_TOL


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_dynamic_drift_tiny(precision):
    """40 lockstep steps of the tiny molecule with the same fields: the mixed-precision
    trajectory stays within the stated local-energy tolerance of the oracle's."""
    s = config_system("tiny")
    log(f"dynamic {precision}")
    worst, *_ = run_lockstep(s, 16, 40, dtau=0.01, precision=precision, rtol=5e-5,
                             label=f"tiny-{precision}", el_abs=EL_TOL)
    log(f"  worst {worst}")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["medium", "large", "ragged", "no_cholesky"])
def test_dynamic_drift_shapes(precision, case):
    """Lockstep runs through the mixed-precision A-build, propagation and contraction:
    after every step each walker's E_L stays within 1e-4 Ha of the FP64 oracle's
    (same fields), and weights / orbitals within 1e-4 relative."""
    if case == "medium":
        s, nw, steps, dt = config_system("medium"), 8, 10, 0.005
    elif case == "large":
        s, nw, steps, dt = config_system("large"), 3, 5, 0.005
    elif case == "ragged":
        s, nw, steps, dt = gen_system(13, 3, 19, seed=5), 7, 12, 0.01
    else:
        s, nw, steps, dt = gen_system(9, 2, 0, seed=8), 5, 10, 0.05
    log(f"dynamic {precision} {case}")
    worst, gs, wk, S, wo = run_lockstep(s, nw, steps, dtau=dt, precision=precision, rtol=1e-4,
                                        label=f"{case}-{precision}", check_every=1,
                                        el_abs=EL_TOL)
    st = gpu_state(wk)
    alive = wo.W > 0
    assert np.abs(st["e"][alive] - wo.e_loc[alive]).max() < EL_TOL
    log(f"  worst {worst}")


def test_mixed_precision_refuses_unsupported_sizes():
    """The MFMA kernels cover N <= 64 electrons per spin and M <= 224 orbitals."""
    import paper_1711_02242_amd as afq
    s = gen_system(232, 20, 6, seed=1)
    with pytest.raises(afq.AfqmcError):
        afq.System.from_synthetic(s, dtau=0.005, precision="fp32")
    s = gen_system(70, 65, 4, seed=2)
    for precision in ("fp64", "fp32"):
        with pytest.raises(afq.AfqmcError):
            afq.System.from_synthetic(s, dtau=0.005, precision=precision)


WIDE = {
    # name: (M, N_up, N_dn, N_g, walkers); tile of the wide kernel in brackets
    "n34_m136": (136, 34, 30, 40, 5),    # NP 48, KP 160
    "n20_m150": (150, 20, 20, 50, 5),    # NP 32 (M > 128), KP 160
    "n40_m160": (160, 40, 40, 60, 4),    # NP 48, KP 160 (largest batch draw)
    "n50_m200": (200, 50, 48, 30, 3),    # NP 64, KP 224 (largest serving draw)
    "n64_m96": (96, 64, 60, 30, 3),      # NP 64, KP 96
}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", list(WIDE))
def test_static_local_energy_wide(precision, case):
    """Shapes beyond the register-resident kernels run on the wide MFMA contraction."""
    M, nu, nd, G, nw = WIDE[case]
    s = gen_system(M, nu, G, seed=31, n_dn=nd)
    log(f"static wide {precision} {case}")
    err, arg_err, gs, wk = _static(s, nw, precision, amplitude=0.4)
    log(f"  max |dE_L| = {err:.3e} Ha")
    assert err < EL_TOL
    assert arg_err < 1e-12


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["n34_m136", "n50_m200"])
def test_dynamic_drift_wide(precision, case):
    M, nu, nd, G, nw = WIDE[case]
    s = gen_system(M, nu, G, seed=32, n_dn=nd)
    log(f"dynamic wide {precision} {case}")
    worst, gs, wk, S, wo = run_lockstep(s, nw, 5, dtau=0.005, precision=precision, rtol=1e-4,
                                        label=f"wide-{case}-{precision}", el_abs=EL_TOL)
    st = gpu_state(wk)
    alive = wo.W > 0
    assert np.abs(st["e"][alive] - wo.e_loc[alive]).max() < EL_TOL
    log(f"  worst {worst}")
