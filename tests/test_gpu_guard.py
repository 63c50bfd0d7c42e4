"""The precision guard of the mixed-precision modes (FP32, BF16x3): walkers whose largest
|Theta_pc| exceeds the threshold have their contraction redone on the FP64 MFMA kernel, spin
by spin (a spin below the threshold keeps its low-precision sums, and the overlap kernel writes
the FP64 operand only for the spins above it).

* With a threshold below every walker's, every walker goes through FP64: the mixed modes then
  give the FP64 path's local energies and traces to FP64 rounding (single and multi-determinant
  trials, closed shell).
* The walkers the guard takes each step are exactly those the oracle's propagated
  determinants put above the threshold (integer counts compared step by step).
* Deep in a run of the 128-orbital workload (steps 100 and 500 of GPU FP64), every walker's
  FP32 and BF16x3 local energy with the default thresholds is within 1e-4 Ha of FP64.
"""

import math

import numpy as np
import pytest

from oracle import afqmc as A
from synthetic import config_system, gen_system, noci_trial, random_walkers
from tests.parity_helpers import log, oracle_U_to_gpu, run_lockstep

pytestmark = pytest.mark.gpu

EL_TOL = 1e-4


def _measure(s, U, precision, **kw):
    import torch

    import paper_1711_02242_amd as afq
    gs = afq.System.from_synthetic(s, dtau=0.005, precision=precision, **kw)
    nw = U[0].shape[0]
    wk = gs.walkers(nw)
    gs.init(wk)
    wk.U.copy_(torch.from_numpy(oracle_U_to_gpu(*U)[:, : gs.ntot]))
    gs.measure(wk)
    torch.cuda.synchronize()
    return gs, wk, wk.e_loc.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", ["medium", "closed_shell"])
def test_guard_everywhere_gives_fp64(precision, case):
    s = config_system("medium")
    U = random_walkers(s, 12, seed=5, amplitude=1.5)
    kw = dict(closed_shell=True) if case == "closed_shell" else {}
    if case == "closed_shell":
        U = (U[0], U[0].copy())
    log(f"guard everywhere {precision} {case}")
    _, _, e64 = _measure(s, U, "fp64", **kw)
    _, _, e_off = _measure(s, U, precision, theta_guard=math.inf, **kw)
    _, _, e_all = _measure(s, U, precision, theta_guard=1e-12, **kw)
    d_off = np.abs(e_off - e64).max()
    d_all = np.abs(e_all - e64).max()
    log(f"  max |dE_L|: guard off {d_off:.2e} Ha, guard on every walker {d_all:.2e} Ha")
    assert d_all <= 1e-10 * np.abs(e64).max()
    assert d_off > 100 * d_all


def test_guard_everywhere_multidet():
    s = config_system("tiny")
    trial = noci_trial(s, 3, seed=3)
    import torch

    import paper_1711_02242_amd as afq
    U = random_walkers(s, 8, seed=6, amplitude=1.0)
    out = {}
    for prec, g in (("fp64", None), ("fp32", 1e-12)):
        gs = afq.System.multidet(s.h0, s.h1, s.L, *trial[:1], np.array(trial[1]),
                                 np.array(trial[2]), dtau=0.01, precision=prec, theta_guard=g)
        wk = gs.walkers(8)
        gs.init(wk)
        wk.U.copy_(torch.from_numpy(oracle_U_to_gpu(*U)))
        gs.measure(wk)
        torch.cuda.synchronize()
        out[prec] = wk.e_loc.cpu().numpy()
    assert np.abs(out["fp32"] - out["fp64"]).max() <= 1e-10 * np.abs(out["fp64"]).max()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_guard_takes_the_walkers_the_oracle_predicts(precision):
    """Lockstep from walkers spread around the trial, threshold at the median of their
    max|Theta|: per step, the GPU's count of guarded walkers equals the number of live
    walkers whose propagated determinant has max|Theta| above the threshold in the oracle."""
    s = gen_system(16, 4, 40, seed=23)
    nw, steps, dt = 16, 12, 0.01
    U = random_walkers(s, nw, seed=9, amplitude=1.2)
    S0 = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, dt)

    def tmax(Uu, Ud):
        return max(np.abs(A.overlap_theta(S0.V[0], Uu)[1]).max(),
                   np.abs(A.overlap_theta(S0.V[1], Ud)[1]).max())

    tau = float(np.median([tmax(U[0][w], U[1][w]) for w in range(nw)]))
    log(f"guard count {precision}: threshold {tau:.3f}")
    state = {"expect": [], "got": [], "live": None}

    def record(wo, gs):
        # the step just taken contracted the walkers live before it (the weight update comes
        # after the contraction); Theta is unchanged by the QR (Theorem 1.5)
        state["got"].append(gs.bound_counts(clear=True)[4])
        state["expect"].append(int(sum(tmax(wo.U[0][w], wo.U[1][w]) > tau
                                       for w in np.flatnonzero(state["live"]))))

    def hook(k, S, P, wo, gs):
        if k == 0:
            gs.bound_counts(clear=True)
        else:
            record(wo, gs)
        state["live"] = wo.W > 0

    worst, gs, wk, S, wo = run_lockstep(s, nw, steps, dtau=dt, precision=precision, rtol=1e-4,
                                        el_abs=EL_TOL, U=U, theta_guard=tau, on_step=hook,
                                        label=f"guard-{precision}", pop_period=0)
    record(wo, gs)
    log(f"  guarded per step: GPU {state['got']}, oracle {state['expect']}")
    assert state["got"] == state["expect"]
    assert 0 < sum(state["got"]) < nw * steps


def test_deep_run_mixed_precision_within_bar():
    """Steps 100 and 500 of the 128-orbital workload in GPU FP64 (device fields): all 1024
    walkers' FP32 and BF16x3 local energies (default guards) within 1e-4 Ha of FP64."""
    import torch

    import paper_1711_02242_amd as afq
    s = config_system("large")
    nw, dt = 1024, 0.005
    gs = afq.System.from_synthetic(s, dtau=dt, precision="fp64")
    wk = gs.walkers(nw)
    gs.init(wk)
    others = {p: afq.System.from_synthetic(s, dtau=dt, precision=p) for p in ("fp32", "bf16x3")}
    done = 0
    for target in (100, 500):
        while done < target:
            gs.step(wk, seed=11)
            done += 1
        torch.cuda.synchronize()
        e64 = wk.e_loc.cpu().numpy()
        for p, g2 in others.items():
            w2 = g2.walkers(nw)
            g2.init(w2)
            w2.U.copy_(wk.U)
            g2.measure(w2)
            torch.cuda.synchronize()
            err = np.abs(w2.e_loc.cpu().numpy() - e64).max()
            log(f"  step {target} {p}: max |dE_L| over {nw} walkers = {err:.2e} Ha")
            assert err < EL_TOL
            del w2
