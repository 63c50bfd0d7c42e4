"""Shared helpers of the GPU parity tests: run the HIP path (through the C ABI) and the
CPU oracle on the same seeded inputs and compare."""

from __future__ import annotations

import math
import sys

import numpy as np

from oracle import afqmc as A
from synthetic import comb_uniform, gaussian_fields


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_U_to_oracle(U: np.ndarray, n_up: int):
    """[nw][ntot][M] orbital-major -> per-spin (nw, M, N_sigma)."""
    return [np.ascontiguousarray(U[:, :n_up, :].transpose(0, 2, 1)),
            np.ascontiguousarray(U[:, n_up:, :].transpose(0, 2, 1))]


def oracle_U_to_gpu(Uu: np.ndarray, Ud: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.concatenate([Uu.transpose(0, 2, 1), Ud.transpose(0, 2, 1)], axis=1))


def make_pair(s, nw: int, *, dtau: float, precision: str = "fp64", qr_period: int = 5,
              pop_period: int = 5, n_taylor: int = 6, U=None, weight_mode: str = "phaseless",
              mean_field: bool = False, closed_shell: bool = False, trial=None, tile=None,
              n_growth: int = 200, el_cap_C: float = 2.0, w_max=None, fb_cap: float = 1.0,
              theta_guard=None):
    """Oracle and GPU system on the same inputs and parameters (``theta_guard``: the GPU's
    precision guard, which the FP64 oracle has no use for).  ``trial`` = (coeffs, ups, dns)
    selects a multi-determinant trial instead of the system's single determinant; ``tile``
    forces a contraction variant."""
    import paper_1711_02242_amd as afq
    P = A.Params(dtau=dtau, n_taylor=n_taylor, qr_period=qr_period, pop_period=pop_period,
                 weight_mode=weight_mode, n_growth=n_growth, el_cap_C=el_cap_C, w_max=w_max,
                 fb_cap=fb_cap)
    kw = dict(dtau=dtau, precision=precision, qr_period=qr_period, pop_period=pop_period,
              n_taylor=n_taylor, weight_mode=weight_mode, mean_field=mean_field,
              closed_shell=closed_shell, n_growth=n_growth, el_cap_C=el_cap_C, w_max=w_max,
              fb_cap=fb_cap, theta_guard=theta_guard)
    if trial is None:
        S = A.setup(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, dtau, mean_field=mean_field)
        gs = afq.System.from_synthetic(s, **kw)
    else:
        coeffs, ups, dns = trial
        S = A.setup_multi(s.h0, s.h1, s.L, coeffs, ups, dns, dtau, mean_field=mean_field)
        gs = afq.System.multidet(s.h0, s.h1, s.L, coeffs, np.array(ups), np.array(dns), **kw)
    if tile is not None:
        gs.set_tile(tile)
    wk = gs.walkers(nw)
    gs.init(wk)
    if U is None:
        wo = A.init_walkers(S, nw)
    else:
        import torch
        Uu, Ud = U
        wo = A.init_walkers(S, nw, Uu, Ud)
        Ug = oracle_U_to_gpu(Uu, Ud)
        wk.U.copy_(torch.from_numpy(Ug[:, : gs.ntot]))
        gs.measure(wk)
    return S, P, wo, gs, wk


def gpu_state(wk):
    import torch
    torch.cuda.synchronize()
    return dict(U=wk.U.cpu().numpy(), W=wk.weight.cpu().numpy(), arg=wk.arg_ovlp.cpu().numpy(),
                logabs=wk.log_ovlp.cpu().numpy(), e=wk.e_loc.cpu().numpy(),
                ids=wk.walker_id.cpu().numpy(), theta=wk.phase.cpu().numpy(),
                growth=wk.system.growth(wk))


def angle_diff(a, b):
    d = np.asarray(a) - np.asarray(b)
    return np.abs(np.mod(d + np.pi, 2 * np.pi) - np.pi)


def compare_state(S, wo, st, n_up: int, rtol: float, what: str = "", el_abs: float | None = None):
    """Largest deviations of the GPU state from the oracle's (returns a dict): relative for U,
    W and (without ``el_abs``) E_L, absolute for the phases; with ``el_abs`` (Ha) every live
    walker's E_L is held to that absolute bound instead.  The population's E_T and cap centre
    (growth phase) are compared too: relative ``rtol`` without ``el_abs``, else within
    ``el_abs`` (centre) and 10 el_abs (E_T)."""
    Uu, Ud = gpu_U_to_oracle(st["U"], n_up)
    if Ud.shape[2] == 0 and wo.U[1].shape[2] == n_up and n_up > 0:
        # closed-shell storage: the up block stands for both spins
        assert np.array_equal(wo.U[0], wo.U[1])
        Ud = Uu
    alive = wo.W > 0
    out = {}
    scaleU = max(np.abs(wo.U[0]).max(), np.abs(wo.U[1]).max() if wo.U[1].size else 0.0)
    dU = np.abs(Uu[alive] - wo.U[0][alive]).max(initial=0.0)
    if wo.U[1].size:
        dU = max(dU, np.abs(Ud[alive] - wo.U[1][alive]).max(initial=0.0))
    out["U"] = dU / scaleU
    out["W"] = np.abs(st["W"] - wo.W).max() / max(1.0, np.abs(wo.W).max())
    de = np.abs(st["e"][alive] - wo.e_loc[alive]).max(initial=0.0)
    if el_abs is None:
        out["e"] = de / max(1.0, np.abs(wo.e_loc[alive]).max(initial=1.0))
    else:
        out["e_abs_ha"] = de
    if st.get("growth") is not None and wo.growth is not None:
        g_et, g_eb = st["growth"]
        if el_abs is None:
            sc = max(1.0, abs(wo.growth.E_T), abs(wo.growth.e_bar))
            out["E_T"] = abs(g_et - wo.growth.E_T) / sc
            out["e_bar"] = abs(g_eb - wo.growth.e_bar) / sc
        else:
            out["E_T_ha"] = abs(g_et - wo.growth.E_T)
            out["e_bar_ha"] = abs(g_eb - wo.growth.e_bar)
    out["arg"] = angle_diff(st["arg"][alive], wo.arg[alive]).max(initial=0.0)
    if wo.theta is not None:
        out["theta"] = angle_diff(st["theta"][alive], wo.theta[alive]).max(initial=0.0)
    out["alive_match"] = bool(np.array_equal(st["W"] > 0, alive))
    lim = {"e_abs_ha": el_abs, "e_bar_ha": 2 * el_abs if el_abs else None,
           "E_T_ha": 10 * el_abs if el_abs else None}
    bad = {k: v for k, v in out.items()
           if k != "alive_match" and not v <= (lim[k] if k in lim else rtol)}
    if bad or not out["alive_match"]:
        raise AssertionError(f"{what}: GPU vs oracle deviation {out} (tol {rtol})")
    return out


def run_lockstep(s, nw: int, steps: int, *, dtau: float, precision: str = "fp64",
                 explicit_fields: bool = True, seed: int = 0, rtol: float = 1e-10,
                 qr_period: int = 5, pop_period: int = 5, check_every: int = 1, U=None,
                 label: str = "", weight_mode: str = "phaseless", mean_field: bool = False,
                 closed_shell: bool = False, trial=None, tile=None, el_abs: float | None = None,
                 n_growth: int = 200, el_cap_C: float = 2.0, w_max=None, fb_cap: float = 1.0,
                 theta_guard=None, on_step=None):
    """Oracle and GPU stepped with the same fields; the states compared after every
    ``check_every`` steps (compare_state).  ``on_step(k, S, P, wo, gs)`` runs before step k."""
    import torch
    S, P, wo, gs, wk = make_pair(s, nw, dtau=dtau, precision=precision, qr_period=qr_period,
                                 pop_period=pop_period, U=U, weight_mode=weight_mode,
                                 mean_field=mean_field, closed_shell=closed_shell, trial=trial,
                                 tile=tile, n_growth=n_growth, el_cap_C=el_cap_C, w_max=w_max,
                                 fb_cap=fb_cap, theta_guard=theta_guard)
    compare_state(S, wo, gpu_state(wk), s.n_up, rtol, f"{label} init", el_abs)
    worst = {}
    for k in range(steps):
        x = gaussian_fields(seed, 0, wo.walker_id, k, s.n_chol)
        u = comb_uniform(seed, 0, k)
        if on_step is not None:
            on_step(k, S, P, wo, gs)
        A.step(S, P, wo, x, u)
        if explicit_fields:
            gs.step(wk, seed=seed, x=torch.from_numpy(x).cuda(), u_comb=u)
        else:
            gs.step(wk, seed=seed)
        if (k + 1) % check_every == 0 or k == steps - 1:
            d = compare_state(S, wo, gpu_state(wk), s.n_up, rtol, f"{label} step {k}", el_abs)
            for key, v in d.items():
                if key != "alive_match":
                    worst[key] = max(worst.get(key, 0.0), v)
    if weight_mode == "free":
        e_fp = gs.free_projection_energy(wk)
        e_ofp = A.free_projection_energy(wo)
        assert abs(e_fp - e_ofp) <= rtol * abs(e_ofp) * 10
    else:
        e_gpu = gs.energy(wk)
        e_or = A.mixed_energy(S, P, wo)
        bar = rtol * abs(e_or[0]) * 10 if el_abs is None else 2 * el_abs
        assert abs(e_gpu[0] / e_gpu[2] - e_or[0]) <= bar
        assert e_gpu[3] == e_or[4]
    return worst, gs, wk, S, wo
