"""Mean-field subtraction (Sec. II.B.3) and the closed-shell one-spin path on the GPU against
the general two-spin FP64 oracle."""

import numpy as np
import pytest

from synthetic import config_system, gen_system, random_walkers
from tests.parity_helpers import gpu_state, log, make_pair, run_lockstep

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["phaseless", "hybrid", "free"])
@pytest.mark.parametrize("case", ["tiny", "medium"])
def test_mean_field_lockstep(mode, case):
    if case == "tiny":
        s, nw, steps, dt = config_system("tiny"), 16, 40, 0.01
    else:
        s, nw, steps, dt = config_system("medium"), 8, 10, 0.005
    log(f"mean field {mode} {case}")
    worst, *_ = run_lockstep(s, nw, steps, dtau=dt, label=f"mf-{mode}-{case}", weight_mode=mode,
                             mean_field=True)
    log(f"  worst {worst}")


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("mean_field", [False, True])
def test_closed_shell_matches_two_spin_oracle(precision, mean_field):
    s = config_system("medium") if precision == "fp64" else config_system("tiny")
    nw, steps, dt = (8, 10, 0.005) if precision == "fp64" else (16, 30, 0.01)
    rtol = 1e-10 if precision == "fp64" else 1e-4
    log(f"closed shell {precision} mf={mean_field}")
    worst, gs, wk, S, wo = run_lockstep(s, nw, steps, dtau=dt, precision=precision, rtol=rtol,
                                        label=f"cs-{precision}", mean_field=mean_field,
                                        closed_shell=True)
    assert gs.ntot == s.n_up and tuple(wk.U.shape) == (nw, s.n_up, s.M)
    log(f"  worst {worst}")


def test_closed_shell_large_static_energy():
    """Full-size closed-shell measure: E_L of random closed-shell walkers equals the two-spin
    GPU FP64 path's."""
    import torch

    import paper_1711_02242_amd as afq
    s = config_system("large")
    nw = 64
    Uu, _ = random_walkers(s, nw, seed=3, amplitude=0.3)
    Ut = torch.from_numpy(np.ascontiguousarray(Uu.transpose(0, 2, 1))).cuda()
    out = {}
    for cs in (False, True):
        gs = afq.System.from_synthetic(s, dtau=0.005, precision="fp64", closed_shell=cs)
        wk = gs.walkers(nw)
        gs.init(wk)
        wk.U.copy_(torch.cat([Ut, Ut], dim=1) if not cs else Ut)
        gs.measure(wk)
        torch.cuda.synchronize()
        out[cs] = (wk.e_loc.cpu().numpy(), wk.arg_ovlp.cpu().numpy(), wk.log_ovlp.cpu().numpy())
        gs.close()
    for a, b in zip(out[False], out[True]):
        assert np.abs(a - b).max() < 1e-10 * max(1.0, np.abs(a).max())


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("nw", [1024, 2048])
def test_closed_shell_large_mixed_precision(precision, nw):
    """Full-size closed-shell measure in the mixed modes, at populations on both sides of the
    default contraction's switch to eight walkers per workgroup (one active spin: 2048 walkers
    take it, 1024 do not; two spins take it at both): E_L equals the two-spin path's in the same
    precision, and both are within 1e-4 Ha of the two-spin FP64 path."""
    import torch

    import paper_1711_02242_amd as afq
    s = config_system("large")
    Uu, _ = random_walkers(s, 64, seed=4, amplitude=0.3)
    Ut = torch.from_numpy(np.ascontiguousarray(Uu.transpose(0, 2, 1))).cuda()
    Ut = Ut.repeat(nw // 64, 1, 1)
    out = {}
    for prec, cs in ((precision, False), (precision, True), ("fp64", False)):
        gs = afq.System.from_synthetic(s, dtau=0.005, precision=prec, closed_shell=cs)
        wk = gs.walkers(nw)
        gs.init(wk)
        wk.U.copy_(torch.cat([Ut, Ut], dim=1) if not cs else Ut)
        gs.measure(wk)
        torch.cuda.synchronize()
        out[(prec, cs)] = wk.e_loc.cpu().numpy()
        del wk
        gs.close()
    two, one, ref = out[(precision, False)], out[(precision, True)], out[("fp64", False)]
    log(f"closed shell {precision} nw={nw}: max |one - two| {np.abs(one - two).max():.2e}, "
        f"max |dE_L| vs FP64 {np.abs(one - ref).max():.2e} Ha")
    assert np.abs(one - two).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(one - ref).max() < 1e-4
    assert np.abs(two - ref).max() < 1e-4


def test_closed_shell_rejects_open_shell_input():
    import paper_1711_02242_amd as afq
    s = gen_system(10, 3, 12, seed=7, n_dn=2)
    with pytest.raises(afq.AfqmcError):
        afq.System.from_synthetic(s, dtau=0.01, closed_shell=True)
