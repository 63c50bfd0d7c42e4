"""The growth phase (App. B.1, B.2) and the rare-event bounds (App. B.1, eq:cap) on the GPU
against the oracle, in lockstep with the same fields.

* E_T and the cap centre of the population match the oracle after every step (compare_state).
* Each bound is made to bind on part of the population -- the local-energy cap (C small), the
  weight cap (w_max small), the force-bias cap (fb_cap small) -- and the GPU's per-step counts
  of capped walkers / components equal the counts read off the oracle's state, exactly; the
  walker states match at the parity bar throughout.
* Deep in the run of the large workload (M=128, N=32+32, N_g=800, 1024 walkers): GPU-FP64
  states after 100 and 500 steps, a sample of walkers against the oracle at 1e-10, every
  walker's FP32 and BF16x3 local energy within 1e-4 Ha of FP64.
"""

import math

import numpy as np
import pytest

from oracle import afqmc as A
from synthetic import config_system, gen_system
from tests.parity_helpers import gpu_U_to_oracle, gpu_state, log, run_lockstep

pytestmark = pytest.mark.gpu

EL_TOL = 1e-4   # Ha per walker


class BoundCounter:
    """Expected per-step bound counts, read off the oracle's state before each step, and
    the GPU's counts of the same step (afqmc_get_bound_counts, cleared every step)."""

    def __init__(self, gs, P, weight_mode):
        self.gs, self.P, self.mode = gs, P, weight_mode
        self.expect, self.got = [], []
        gs.bound_counts(clear=True)

    def before(self, k, S, P, wo):
        live = wo.W > 0
        half = math.sqrt(P.el_cap_C / P.dtau)
        ecap = 0
        if self.mode == "phaseless":
            ecap = int(np.count_nonzero(np.abs(wo.e_loc.real[live] - wo.growth.e_bar) > half))
        mod = math.sqrt(P.dtau) * np.abs(wo.t[live] - S.lbar[None, :])
        fb = int(np.count_nonzero(mod > P.fb_cap))
        pop = P.pop_period > 0 and (k + 1) % P.pop_period == 0
        self.expect.append([ecap, None, fb, int(np.count_nonzero(live)), pop])

    def after(self, wo, wmax):
        c = self.gs.bound_counts(clear=True)
        e = self.expect[-1]
        if not e[4]:     # the comb resets the weights: the capped ones are seen only before it
            e[1] = int(np.count_nonzero(wo.W == wmax))
        self.got.append(list(c))

    def check(self, what):
        for k, (e, g) in enumerate(zip(self.expect, self.got)):
            assert g[0] == e[0] and g[2] == e[2] and g[3] == e[3], (what, k, e, g)
            if e[1] is not None:
                assert g[1] == e[1], (what, k, e, g)
        tot = np.array([[g[0], g[1], g[2], g[3]] for g in self.got]).sum(axis=0)
        return tot


def _lockstep_counted(s, nw, steps, *, dtau, precision="fp64", rtol=1e-10, el_abs=None,
                      weight_mode="phaseless", label="", **kw):
    counter = {}

    def hook(k, S, P, wo, gs):
        if k == 0:
            counter["c"] = BoundCounter(gs, P, weight_mode)
            counter["P"] = P
        else:
            counter["c"].after(wo, P.wmax(nw))
        counter["c"].before(k, S, P, wo)

    worst, gs, wk, S, wo = run_lockstep(s, nw, steps, dtau=dtau, precision=precision, rtol=rtol,
                                        el_abs=el_abs, weight_mode=weight_mode, label=label,
                                        on_step=hook, **kw)
    counter["c"].after(wo, counter["P"].wmax(nw))
    tot = counter["c"].check(label)
    log(f"  {label}: worst {worst}; capped E_L {tot[0]}, W {tot[1]}, xbar {tot[2]} "
        f"of {tot[3]} walker-steps")
    return tot, gs, wk, S, wo


def test_growth_state_follows_oracle_fp64():
    """E_T and the cap centre after every step of a 60-step run (12 block ends)."""
    s = config_system("tiny")
    log("growth state fp64 tiny")
    worst, gs, wk, S, wo = run_lockstep(s, 16, 60, dtau=0.01, label="growth-tiny", n_growth=45)
    e_t, e_bar = gs.growth(wk)
    assert e_t != S.E_T and e_bar != S.E_T        # the block ends moved both
    log(f"  worst {worst}; E_T {e_t:.6f}, centre {e_bar:.6f} (trial {S.E_T:.6f})")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_local_energy_cap_binds_on_part_of_population(precision):
    """C = 1e-5 at dtau = 0.01: a window of +-0.032 Ha around the centre, inside the walkers'
    spread, so the cap binds on some walkers and not on others (148 of 960 walker-steps in
    the oracle)."""
    s = config_system("tiny")
    log(f"E_L cap partial {precision}")
    rtol, el_abs = (1e-10, None) if precision == "fp64" else (1e-4, EL_TOL)
    tot, *_ = _lockstep_counted(s, 24, 40, dtau=0.01, precision=precision, rtol=rtol,
                                el_abs=el_abs, el_cap_C=1e-5, label=f"ecap-{precision}")
    assert 0 < tot[0] < tot[3]


def test_weight_cap_binds_on_part_of_population():
    """The cos projection lowers every weight a little each step, so a cap just below the
    starting weight binds on the walkers that lost least (60 of 960 in the oracle)."""
    s = config_system("tiny")
    log("W cap partial fp64")
    tot, *_ = _lockstep_counted(s, 24, 40, dtau=0.01, w_max=0.99, label="wcap")
    assert 0 < tot[1] < tot[3]


@pytest.mark.parametrize("weight_mode", ["phaseless", "hybrid"])
def test_force_bias_cap_binds_on_part_of_population(weight_mode):
    s = gen_system(12, 3, 30, seed=21)
    log(f"force-bias cap partial {weight_mode}")
    tot, *_ = _lockstep_counted(s, 16, 30, dtau=0.01, fb_cap=0.02, weight_mode=weight_mode,
                                label=f"fbcap-{weight_mode}")
    assert 0 < tot[2] < tot[3] * s.n_chol


def test_all_bounds_binding_medium_fp64():
    s = config_system("medium")
    log("all bounds partial medium fp64")
    tot, *_ = _lockstep_counted(s, 8, 15, dtau=0.005, el_cap_C=0.05, w_max=0.99, fb_cap=0.05,
                                label="all-medium")
    assert 0 < tot[0] < tot[3] and 0 < tot[1] < tot[3] and 0 < tot[2]


def test_large_lockstep_fifty_steps():
    """Eight walkers of the large workload, 50 steps (10 QR, comb and block ends) against the
    oracle at the FP64 bar, the growth state included."""
    s = config_system("large")
    log("large lockstep 8 walkers x 50 steps fp64")
    worst, gs, wk, S, wo = run_lockstep(s, 8, 50, dtau=0.005, label="large-50", check_every=5)
    log(f"  worst {worst}; growth {gs.growth(wk)}")


def test_deep_run_large_states_against_oracle():
    """The benchmark's workload after 100 and 500 GPU-FP64 steps (device fields): a sample of
    walkers against the oracle at 1e-10, and the mixed estimate away from the cap's bound."""
    import paper_1711_02242_amd as afq
    s = config_system("large")
    nw, dt = 1024, 0.005
    gs = afq.System.from_synthetic(s, dtau=dt, precision="fp64")
    wk = gs.walkers(nw)
    gs.init(wk)
    S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, dt)
    half = math.sqrt(2.0 / dt)
    gs.bound_counts(clear=True)
    done = 0
    for target in (100, 500):
        log(f"deep large: stepping to {target}")
        while done < target:
            gs.step(wk, seed=11)
            done += 1
        st = gpu_state(wk)
        e_t, e_bar = st["growth"]
        live = st["W"] > 0
        frac = float(np.mean(np.abs(st["e"].real[live] - e_bar) > half))
        a, _, c, n_alive, _ = gs.energy(wk)
        log(f"  step {target}: E_mix {a / c:.4f}, centre {e_bar:.4f}, E_T {e_t:.4f}, "
            f"alive {n_alive}, outside the cap {frac:.3f}, sum W {c:.4g}")
        assert n_alive == nw                      # both are comb steps
        assert 0.5 * nw <= c <= 2.0 * nw          # weights restart at 1 at every comb
        assert frac < 1.0 and abs(a / c - (e_bar - half)) > 1.0
        Uu, Ud = gpu_U_to_oracle(st["U"], s.n_up)
        idx = np.flatnonzero(live)[[0, 200, 600, -1]]
        for w in idx:
            arg, logabs, e, t = A.measure(S, Uu[w], Ud[w])
            assert abs(st["e"][w] - e) <= 1e-10 * abs(e), (target, w)
            assert abs(((st["arg"][w] - arg + np.pi) % (2 * np.pi)) - np.pi) < 1e-10
    counts = gs.bound_counts()
    log(f"  bound counts over 500 steps: {counts}")
