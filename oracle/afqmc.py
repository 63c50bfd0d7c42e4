"""Plain FP64 phaseless AFQMC (test infrastructure only; see package docstring).

Notation follows arXiv:1711.02242.  M orbitals, N_sigma electrons of spin
sigma, N_g Cholesky vectors, s = sqrt(dtau).  A walker of spin sigma is the
M x N_sigma matrix U_sigma (Sec. II.A, eq:SDdef); the trial is the real
M x N_sigma matrix V_sigma (Sec. III.D.1).

Readings taken where the paper leaves a choice (each is listed, with its
reason, in the design notes of the repository):

* two-body energy carries the 1/2 of eq:bo_ham2 (eq:localenergy2/3 print the
  bracket without it);
* v_g = i L_g (Sec. II.B.2) so the force bias is -i s sum_sigma tr(Lh Theta)
  (eq:precomputing2) and the propagator exponent is i s sum (x - xbar) L;
* symmetric Trotter split (eq:primitive) with the one-body halves applied
  exactly, only the field exponent Taylor-expanded (Sec. III.D.2) to
  ``n_taylor`` = 6 terms;
* the weight uses the local energy of the walker before the move (eq:if_rle,
  importance function expanded around the current walker) and
  max(0, cos dtheta) with dtheta the phase of the overlap ratio;
* local-energy cap |E_L - Ebar| <= sqrt(C/dtau), force-bias modulus cap,
  weight cap (eq:cap, App. B.1); the centre Ebar is the weighted average of the
  local energy over the latest population-control block of a growth phase and
  is frozen afterwards;
* the trial energy E_T of the importance function starts at E_L(Phi_T, Phi_T)
  and is reset to the growth estimate (eq:corsam, App. B.2) at the same block
  ends during the growth phase, then frozen;
* comb resampling to a fixed population for the branching step (Sec. III.D.4),
  every copy's weight reset to 1.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# --------------------------------------------------------------------------
# Setup (Sec. II.B.2, eq:mcd1; Sec. III.D.2, eq:precomputing2)
# --------------------------------------------------------------------------

@dataclass
class Setup:
    h0: float
    h1: np.ndarray        # (M, M)
    L: np.ndarray         # (N_g, M, M)
    V: list               # per spin, (M, N_sigma) real trial orbitals
    dtau: float
    v0: np.ndarray        # (M, M)  one-body part after the Cholesky rewrite
    Eh: np.ndarray        # (M, M)  exp(-dtau/2 v0)
    Lh: list              # per spin, (N_g, N_sigma, M) half-rotated Cholesky V^T L_g
    ht: list              # per spin, (N_sigma, M) half-rotated one-body V^T h1
    E_T: float            # trial energy E_L(Phi_T, Phi_T)
    lbar: np.ndarray | None = None   # (N_g,) mean-field shifts <L_g>_T (zeros: no subtraction)
    h0_prop: float = 0.0  # constant of the propagated Hamiltonian (H0, or H0 - 1/2 sum lbar^2)

    @property
    def M(self):
        return self.h1.shape[0]

    @property
    def n_chol(self):
        return self.L.shape[0]


def one_body_v0(h1: np.ndarray, L: np.ndarray) -> np.ndarray:
    """v0_pq = h_pq - 1/2 sum_r v_prrq with v_prrq = sum_g L^g_pr L^g_rq (eq:mcd1)."""
    return h1 - 0.5 * np.einsum("gpr,grq->pq", L, L)


def sym_expm(A: np.ndarray, c: float) -> np.ndarray:
    """exp(c A) for a real symmetric matrix A, by its eigendecomposition."""
    w, Q = np.linalg.eigh(A)
    return (Q * np.exp(c * w)) @ Q.T


def setup(h0, h1, L, phi_up, phi_dn, dtau, e_trial=None, mean_field: bool = False) -> Setup:
    """Precompute everything that does not depend on the walkers.

    With ``mean_field`` the mean-field background is subtracted (Sec. II.B.3): with
    v_g = i L_g and vbar_g = <Psi_T|v_g|Psi_T> = i lbar_g, lbar_g = <L_g>_T real,
    H = H0' + v0' - 1/2 sum_g (v_g - vbar_g)^2 where
    H0' = H0 + 1/2 sum vbar^2 = H0 - 1/2 sum lbar^2 and v0' = v0 - sum vbar_g v_g = v0 + sum lbar_g L_g.
    """
    h1 = np.asarray(h1, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    V = [np.asarray(phi_up, dtype=np.float64), np.asarray(phi_dn, dtype=np.float64)]
    v0 = one_body_v0(h1, L)
    # Half rotation: (Lh_g)_rq = sum_p (V^dagger)_rp L^g_pq, V real (eq:precomputing2).
    Lh = [np.einsum("pr,gpq->grq", Vs, L) for Vs in V]
    ht = [Vs.T @ h1 for Vs in V]
    S = Setup(h0=float(h0), h1=h1, L=L, V=V, dtau=float(dtau), v0=v0, Eh=None, Lh=Lh, ht=ht,
              E_T=0.0, lbar=np.zeros(L.shape[0]), h0_prop=float(h0))
    th = [overlap_theta(V[s], V[s].astype(np.complex128))[1] for s in range(2)]
    e_hf, t_trial = local_energy(S, th)
    if mean_field:
        S.lbar = t_trial.real.copy()
        S.v0 = v0 + np.einsum("g,gpq->pq", S.lbar, L)
        S.h0_prop = float(h0) - 0.5 * float(np.sum(S.lbar ** 2))
    S.Eh = sym_expm(S.v0, -0.5 * dtau)
    S.E_T = float(e_hf.real if e_trial is None else e_trial)
    return S


# --------------------------------------------------------------------------
# Overlap and Green's function (Theorem 1.1-1.2; eq:precomputing)
# --------------------------------------------------------------------------

def overlap_theta(V: np.ndarray, U: np.ndarray):
    """For one spin: (log det T, Theta) with T = V^dagger U and Theta = U T^{-1}.

    <Phi|Psi> = prod_sigma det(V_sigma^dagger U_sigma) (Theorem 1.1) and
    G_pq = (U T^{-1} V^dagger)_qp = (Theta V^dagger)_qp (Theorem 1.2, eq:precomputing).
    The log determinant is returned as a complex number log|det| + i arg det.
    """
    T = V.conj().T @ U
    sign, logabs = np.linalg.slogdet(T)
    Theta = U @ np.linalg.inv(T)
    return complex(logabs + 1j * np.angle(sign)), Theta


def green_function(V: np.ndarray, U: np.ndarray) -> np.ndarray:
    """G_pq = <Phi| a+_p a_q |Psi> / <Phi|Psi> for one spin (Theorem 1.2, thm:1rdm)."""
    T = V.conj().T @ U
    return (U @ np.linalg.inv(T) @ V.conj().T).T


# --------------------------------------------------------------------------
# Local energy and force bias (eq:precomputing2, eq:localenergy2, eq:localenergy3)
# --------------------------------------------------------------------------

def local_energy(S: Setup, Theta: list):
    """Local energy E_L = <Phi_T|H|Psi>/<Phi_T|Psi> and the traces t_g.

    Omega^g_sigma = Lh^g_sigma Theta_sigma (N_sigma x N_sigma) for every g;
    t_g = sum_sigma tr Omega^g_sigma (so <L_g>_m = t_g);
    E_L = h0 + sum_sigma tr(ht_sigma Theta_sigma)
          + 1/2 sum_g [ t_g^2 - sum_sigma tr(Omega^g_sigma Omega^g_sigma) ].
    Returns (E_L complex, t of shape (N_g,) complex).
    """
    t = np.zeros(S.n_chol, dtype=np.complex128)
    exch = 0.0 + 0.0j
    e1 = 0.0 + 0.0j
    for s in range(2):
        if Theta[s].shape[1] == 0:
            continue
        Om = np.matmul(S.Lh[s], Theta[s])                     # (N_g, N, N)
        t += np.trace(Om, axis1=1, axis2=2)
        exch += np.sum(Om * Om.transpose(0, 2, 1))
        e1 += np.trace(S.ht[s] @ Theta[s])
    e2 = 0.5 * (np.sum(t * t) - exch)
    return complex(S.h0 + e1 + e2), t


def force_bias(t: np.ndarray, dtau: float, fb_cap: float) -> np.ndarray:
    """xbar_g = -sqrt(dtau) <v_g>_m = -i sqrt(dtau) t_g (eq:fb, eq:precomputing2),
    with its modulus capped at ``fb_cap`` keeping the phase (App. B.1)."""
    xbar = -1j * math.sqrt(dtau) * t
    mod = np.abs(xbar)
    over = mod > fb_cap
    xbar[over] *= fb_cap / mod[over]
    return xbar


# --------------------------------------------------------------------------
# Propagation (Theorem 1.4; eq:primitive; Sec. III.D.2)
# --------------------------------------------------------------------------

def propagator_exponent(S: Setup, x: np.ndarray, xbar: np.ndarray) -> np.ndarray:
    """A = i sqrt(dtau) sum_g (x_g - xbar_g) L^g, the matrix of sqrt(dtau) sum (x-xbar) v_g."""
    return 1j * math.sqrt(S.dtau) * np.einsum("g,gpq->pq", x - xbar, S.L)


def taylor_apply(A: np.ndarray, X: np.ndarray, n_taylor: int) -> np.ndarray:
    """sum_{n=0}^{n_taylor} A^n X / n!, each term from the previous one as A term / n."""
    Y = X.copy()
    term = X
    for n in range(1, n_taylor + 1):
        term = A @ term / n
        Y = Y + term
    return Y


def propagate(S: Setup, A: np.ndarray, U: np.ndarray, n_taylor: int) -> np.ndarray:
    """U <- exp(-dtau/2 v0) T_n(A) exp(-dtau/2 v0) U for one spin (Thouless, Theorem 1.4)."""
    return S.Eh @ taylor_apply(A, S.Eh @ U, n_taylor)


# --------------------------------------------------------------------------
# Re-orthonormalization (Sec. III.D.5; Theorem 1.5)
# --------------------------------------------------------------------------

def modified_gram_schmidt(U: np.ndarray):
    """Orthonormalize the columns of U in order, subtracting the projection on each
    earlier orthonormal column in turn.  Returns (Q, r) with U = Q R, R upper
    triangular and r = diag(R) > 0, so det R = prod(r) is real and positive."""
    M, N = U.shape
    Q = U.astype(np.complex128).copy()
    r = np.zeros(N)
    for k in range(N):
        v = Q[:, k].copy()
        for j in range(k):
            v = v - np.vdot(Q[:, j], v) * Q[:, j]
        nrm = math.sqrt(float(np.vdot(v, v).real))
        r[k] = nrm
        Q[:, k] = v / nrm
    return Q, r


# --------------------------------------------------------------------------
# Phaseless weight (eq:if_rle, eq:weight_update_2, eq:cap)
# --------------------------------------------------------------------------

def capped_energy(e_re, e_bar: float, dtau: float, C: float):
    """Re E_L bounded to e_bar +- sqrt(C/dtau) (eq:cap); e_bar is the growth-phase average
    of the local energy (App. B.1)."""
    half = math.sqrt(C / dtau)
    return np.clip(e_re, e_bar - half, e_bar + half)


def wrap_angle(a):
    """Angle folded into (-pi, pi]."""
    a = np.asarray(a, dtype=np.float64)
    w = np.mod(a + np.pi, 2.0 * np.pi) - np.pi
    return np.where(w == -np.pi, np.pi, w)


def phaseless_weight(W, e_loc_old, arg_old, arg_new, dtau, E_T, C, w_max, e_bar=None):
    """W' = min(w_max, W exp(-dtau (Re E_L^cap(old) - E_T)) max(0, cos(arg_new - arg_old))),
    the local energy capped around e_bar (eq:cap; E_T when e_bar is not given)."""
    e_cap = capped_energy(np.real(e_loc_old), E_T if e_bar is None else e_bar, dtau, C)
    proj = np.maximum(0.0, np.cos(np.asarray(arg_new) - np.asarray(arg_old)))
    Wn = W * np.exp(-dtau * (e_cap - E_T)) * proj
    return np.minimum(Wn, w_max)


def mean_field_log_factor(S, x, xbar) -> complex:
    """log of the c-number exp(sqrt(dtau) sum_g (x - xbar)_g (-vbar_g)) = exp(-i s sum (x - xbar) lbar)
    that the mean-field-subtracted propagator puts on every walker (zero without subtraction)."""
    return complex(-1j * math.sqrt(S.dtau) * np.sum((x - xbar) * S.lbar))


def hybrid_log_importance(S, x, xbar, log_ovlp_old: complex, log_ovlp_new: complex,
                          E_T: float | None = None) -> complex:
    """log I(x, xbar; Psi) of eq:hybrid-wt:
    log[<Psi_T|B(x - xbar)|Psi>/<Psi_T|Psi>] + x.xbar - xbar.xbar/2, where the overlap ratio is
    that of the propagated and the old determinant (times the mean-field c-number) and B
    carries exp(-dtau (H0' - E_T)) (E_T: the trial energy in use, S.E_T when not given)."""
    e_t = S.E_T if E_T is None else E_T
    return (log_ovlp_new - log_ovlp_old + mean_field_log_factor(S, x, xbar)
            - S.dtau * (S.h0_prop - e_t)
            + complex(np.sum(x * xbar) - 0.5 * np.sum(xbar * xbar)))


# --------------------------------------------------------------------------
# Population control (Sec. III.D.4): comb / systematic resampling
# --------------------------------------------------------------------------

def comb(W: np.ndarray, u: float):
    """Comb resampling to the same population size.

    Positions (u + j) * (sum W / n), j = 0..n-1, fall into the half-open
    cumulative-weight intervals [C_{i-1}, C_i) of the walkers in index order;
    walker j of the new population copies the walker whose interval holds
    position j, and every new weight is 1.  The copies stand for the population
    with equal weights; a common factor of all weights leaves the mixed estimate
    unchanged, and resetting it to 1 keeps the weight cap w_max relative to the
    mean weight however far the total has drifted since the last growth-phase
    update of E_T (App. B.1, B.2).  Returns (parent, W_new).
    """
    n = W.size
    C = np.cumsum(W)
    total = C[-1]
    if not total > 0.0:
        raise ValueError("comb: no walker has positive weight")
    pos = (u + np.arange(n, dtype=np.float64)) * (total / n)
    parent = np.searchsorted(C, pos, side="right")
    last_alive = int(np.nonzero(W > 0)[0][-1])
    parent = np.minimum(parent, last_alive)
    return parent.astype(np.int64), np.ones(n)


# --------------------------------------------------------------------------
# Walker population and the step (Sec. III.E)
# --------------------------------------------------------------------------

WEIGHT_PHASELESS = "phaseless"      # eq:if_rle: local-energy importance function, cos projection
WEIGHT_HYBRID = "hybrid"            # eq:hybrid-wt magnitude with the cos projection
WEIGHT_FREE = "free"                # free projection (Sec. II.C) with the hybrid importance function


@dataclass
class Params:
    dtau: float
    n_taylor: int = 6
    qr_period: int = 5
    pop_period: int = 5
    el_cap_C: float = 2.0
    w_max: float | None = None
    fb_cap: float = 1.0
    weight_mode: str = WEIGHT_PHASELESS
    n_growth: int = 200

    def wmax(self, n_walkers: int) -> float:
        return self.w_max if self.w_max is not None else max(100.0, n_walkers / 10.0)


@dataclass
class Growth:
    """Trial energy and local-energy cap centre of a walker population (App. B.1, B.2).

    Both start at the trial energy.  During the growth phase (steps k < n_growth) the sums
    below are accumulated over the steps of each population-control block; at the block's
    last step (the comb step)
      E_T   <- E_T - (1/dtau) log( sum_k T_{k+1} / sum_k T_k )            (eq:corsam)
      e_bar <- sum_k sum_w W_{k+1} Re E_L(Psi_{k+1}) / sum_k sum_w W_{k+1}
    with T_k the total weight before step k and T_{k+1} after its weight update (before the
    comb), sums over the live walkers.  After the growth phase both stay fixed.  eq:corsam
    prints the logarithm of the growth ratio alone; the expansion of eq:whycorsam,
    log I = -dtau (E_L - E_T), gives it the factor -1/dtau used here."""
    E_T: float
    e_bar: float
    num: float = 0.0      # sum over the block of the total weight after each step
    den: float = 0.0      # sum over the block of the total weight before each step
    swe: float = 0.0      # sum over the block of sum_w W Re E_L (uncapped)
    sw: float = 0.0       # sum over the block of sum_w W


@dataclass
class Walkers:
    U: list               # per spin, (n_w, M, N_sigma) complex128
    W: np.ndarray         # (n_w,)
    arg: np.ndarray       # (n_w,) arg <Phi_T|Psi>, in (-pi, pi]
    logabs: np.ndarray    # (n_w,) log |<Phi_T|Psi>| (diagnostic)
    e_loc: np.ndarray     # (n_w,) complex E_L of the current walker
    t: np.ndarray         # (n_w, N_g) complex traces of the current walker
    walker_id: np.ndarray  # (n_w,) int64
    step: int = 0
    theta: np.ndarray | None = None   # (n_w,) walker phase; stays 0 except in free projection
    growth: "Growth | None" = None    # trial energy and cap centre of the population (App. B)

    @property
    def n(self):
        return self.W.size


def measure(S: Setup, U_up: np.ndarray, U_dn: np.ndarray):
    """Overlap phase, log|overlap|, E_L and t for one walker."""
    lg_up, th_up = overlap_theta(S.V[0], U_up)
    lg_dn, th_dn = overlap_theta(S.V[1], U_dn)
    lg = lg_up + lg_dn
    e, t = local_energy(S, [th_up, th_dn])
    return float(wrap_angle(lg.imag)), float(lg.real), e, t


def _measure_any(S, U_up, U_dn):
    return measure_multi(S, U_up, U_dn) if isinstance(S, MultiSetup) else measure(S, U_up, U_dn)


def _first(S):
    """The single-determinant Setup that carries h, L, E_h and the trial's first determinant."""
    return S.dets[0] if isinstance(S, MultiSetup) else S


def init_walkers(S, n_walkers: int, U_up=None, U_dn=None) -> Walkers:
    """Every walker starts as {Psi_I, W = 1, theta = 0} (Sec. II.C, Sec. III.E) with Psi_I the
    (first) trial determinant unless explicit determinants are given."""
    S = S if isinstance(S, MultiSetup) else S
    S0 = _first(S)
    if U_up is None:
        U_up = np.repeat(S0.V[0][None].astype(np.complex128), n_walkers, axis=0)
    if U_dn is None:
        U_dn = np.repeat(S0.V[1][None].astype(np.complex128), n_walkers, axis=0)
    U_up = np.array(U_up, dtype=np.complex128)
    U_dn = np.array(U_dn, dtype=np.complex128)
    n = U_up.shape[0]
    arg = np.zeros(n)
    logabs = np.zeros(n)
    e = np.zeros(n, dtype=np.complex128)
    t = np.zeros((n, S0.n_chol), dtype=np.complex128)
    for w in range(n):
        arg[w], logabs[w], e[w], t[w] = _measure_any(S, U_up[w], U_dn[w])
    return Walkers(U=[U_up, U_dn], W=np.ones(n), arg=arg, logabs=logabs, e_loc=e, t=t,
                   walker_id=np.arange(n, dtype=np.int64), step=0, theta=np.zeros(n),
                   growth=Growth(E_T=S.E_T, e_bar=S.E_T))


def step(S, P: Params, wk: Walkers, x: np.ndarray, u_comb: float | None = None,
         info: dict | None = None) -> Walkers:
    """One step of the random walk for every walker (Sec. III.E), in place.

    ``x`` (n_w, N_g) are the auxiliary fields drawn for this step; ``u_comb``
    is the comb's uniform, needed when population control is due after it.
    Walkers with zero weight are skipped until population control replaces them.
    """
    Sm, S = S, _first(S)      # Sm measures (single or multi-determinant), S propagates
    k = wk.step
    n = wk.n
    wmax = P.wmax(n)
    do_qr = P.qr_period > 0 and (k + 1) % P.qr_period == 0
    do_pop = P.pop_period > 0 and (k + 1) % P.pop_period == 0
    gr = wk.growth
    in_growth = P.weight_mode != WEIGHT_FREE and P.n_growth > 0 and k < P.n_growth
    if in_growth:
        gr.den += float(np.sum(wk.W[wk.W > 0]))
    for w in range(n):
        if not wk.W[w] > 0.0:
            continue
        xbar = force_bias(wk.t[w] - S.lbar, P.dtau, P.fb_cap)
        A = propagator_exponent(S, x[w], xbar)
        U_up = propagate(S, A, wk.U[0][w], P.n_taylor)
        U_dn = propagate(S, A, wk.U[1][w], P.n_taylor)
        # log|<Phi_T|Psi'>| before any re-orthonormalization: QR divides the overlap by det R.
        log_r = 0.0
        if do_qr:
            U_up, r_up = modified_gram_schmidt(U_up)
            U_dn, r_dn = modified_gram_schmidt(U_dn)
            log_r = float(np.sum(np.log(r_up)) + np.sum(np.log(r_dn)))
        arg_new, logabs_new, e_new, t_new = _measure_any(Sm, U_up, U_dn)
        if P.weight_mode == WEIGHT_PHASELESS:
            dphase = mean_field_log_factor(S, x[w], xbar).imag
            wk.W[w] = phaseless_weight(wk.W[w], wk.e_loc[w], wk.arg[w], arg_new + dphase, P.dtau,
                                       gr.E_T, P.el_cap_C, wmax, gr.e_bar)
        else:
            logI = hybrid_log_importance(S, x[w], xbar, complex(wk.logabs[w], wk.arg[w]),
                                         complex(logabs_new + log_r, arg_new), gr.E_T)
            if P.weight_mode == WEIGHT_HYBRID:
                proj = max(0.0, math.cos(arg_new - wk.arg[w]
                                         + mean_field_log_factor(S, x[w], xbar).imag))
                wk.W[w] = min(wmax, wk.W[w] * math.exp(logI.real) * proj)
            else:   # free projection: complex weight W e^{i theta} times I (eq:weight_update)
                wk.W[w] = wk.W[w] * math.exp(logI.real)
                wk.theta[w] = float(wrap_angle(wk.theta[w] + logI.imag))
        wk.U[0][w] = U_up
        wk.U[1][w] = U_dn
        wk.arg[w] = arg_new
        wk.logabs[w] = logabs_new
        wk.e_loc[w] = e_new
        wk.t[w] = t_new
    if in_growth:
        live = wk.W > 0
        gr.num += float(np.sum(wk.W[live]))
        gr.swe += float(np.sum(wk.W[live] * wk.e_loc.real[live]))
        gr.sw += float(np.sum(wk.W[live]))
        if do_pop:
            if gr.num > 0.0 and gr.den > 0.0:
                gr.E_T = gr.E_T - math.log(gr.num / gr.den) / P.dtau
            if gr.sw > 0.0:
                gr.e_bar = gr.swe / gr.sw
            gr.num = gr.den = gr.swe = gr.sw = 0.0
    if do_pop:
        if u_comb is None:
            raise ValueError("population control is due: u_comb is required")
        parent, Wn = comb(wk.W, u_comb)
        if info is not None:
            info["parent"] = parent
        for arr in (wk.U[0], wk.U[1]):
            arr[:] = arr[parent]
        wk.arg = wk.arg[parent]
        wk.logabs = wk.logabs[parent]
        wk.e_loc = wk.e_loc[parent]
        wk.t = wk.t[parent]
        wk.theta = wk.theta[parent]
        wk.W = Wn
        wk.walker_id = np.arange(n, dtype=np.int64)
    wk.step = k + 1
    return wk


def free_projection_energy(wk: Walkers) -> complex:
    """sum_w W e^{i theta} E_L / sum_w W e^{i theta} (eq:freep, eq:localenergy), uncapped."""
    c = wk.W * np.exp(1j * wk.theta)
    return complex(np.sum(c * wk.e_loc) / np.sum(c))


def mixed_energy(S: Setup, P: Params, wk: Walkers):
    """Mixed estimator sum_w W_w Re E_L^cap(Psi_w) / sum_w W_w (eq:localenergy, theta = 0)
    plus the raw sums: (E_mix, sum W Re E_cap, sum W Im E_L, sum W, n_alive), the local
    energy capped around the population's current centre (eq:cap)."""
    e_cap = capped_energy(wk.e_loc.real, wk.growth.e_bar, P.dtau, P.el_cap_C)
    sw = float(np.sum(wk.W))
    swe = float(np.sum(wk.W * e_cap))
    swi = float(np.sum(wk.W * wk.e_loc.imag))
    alive = int(np.count_nonzero(wk.W > 0))
    return swe / sw, swe, swi, sw, alive


# --------------------------------------------------------------------------
# Multi-determinant trial (Sec. III.D.1, eq:usesherman, eq:precomputing2, eq:localenergy2)
# --------------------------------------------------------------------------

@dataclass
class MultiSetup:
    """Psi_T = sum_d A_d |Psi_d>; one single-determinant Setup per determinant (sharing h, L)."""
    dets: list            # list of Setup, one per determinant
    coeffs: np.ndarray    # (N_d,) complex A_d
    E_T: float
    dtau: float
    lbar: np.ndarray
    h0_prop: float

    @property
    def n_chol(self):
        return self.dets[0].n_chol


def measure_multi(MS: MultiSetup, U_up: np.ndarray, U_dn: np.ndarray):
    """Overlap, local energy and force-bias traces of one walker against a multi-determinant
    trial.  With r_d = A_d^* <Psi_d|Psi>:
      <Psi_T|Psi> = sum_d r_d;   E_L = sum_d r_d E_L^d / sum_d r_d   (linearity of eq:localenergy2);
      t_g = sum_d r_d t^d_g / sum_d r_d                           (eq:precomputing2),
    where E_L^d, t^d are the single-determinant quantities against Psi_d (eq:localenergy3).
    Returns (arg <Psi_T|Psi>, log|<Psi_T|Psi>|, E_L, t)."""
    logs, es, ts, keep = [], [], [], []
    for d, S in enumerate(MS.dets):
        # An exactly singular V_d^T U gives r_d = 0; its energy term A_d^* <Psi_d|H|Psi> is then
        # dropped, which is exact only for walkers non-orthogonal to every determinant
        # (propagated walkers are, with probability one).
        if any(np.linalg.slogdet(S.V[k].T @ U)[0] == 0 for k, U in ((0, U_up), (1, U_dn))
               if U.shape[1] > 0):
            continue
        lg_u, th_u = overlap_theta(S.V[0], U_up)
        lg_d, th_d = overlap_theta(S.V[1], U_dn)
        e, t = local_energy(S, [th_u, th_d])
        logs.append(lg_u + lg_d)
        es.append(e)
        ts.append(t)
        keep.append(d)
    logs = np.array(logs)
    ref = np.max(logs.real)
    r = np.conj(MS.coeffs[keep]) * np.exp(logs - ref)
    R = np.sum(r)
    e = complex(np.sum(r * np.array(es)) / R)
    t = np.sum(r[:, None] * np.array(ts), axis=0) / R
    lg = np.log(R) + ref
    return float(wrap_angle(lg.imag)), float(lg.real), e, t


def setup_multi(h0, h1, L, coeffs, phis_up, phis_dn, dtau, e_trial=None,
                mean_field: bool = False) -> MultiSetup:
    """A_d = coeffs[d], determinant d = (phis_up[d], phis_dn[d]).

    The trial energy E_T and the mean-field shifts lbar are constants of the method (any
    value leaves the estimator exact, Sec. II.B.3, App. B.2); for a multi-determinant trial
    they are taken from the leading determinant d = 0: E_T = E_L(Psi_0; Psi_0) and
    lbar_g = <Psi_0|L_g|Psi_0> / <Psi_0|Psi_0>.  ``trial_energy_multi`` gives the Rayleigh
    quotient of the whole expansion when its determinants are pairwise non-orthogonal."""
    coeffs = np.asarray(coeffs, dtype=np.complex128)
    dets = [setup(h0, h1, L, pu, pd, dtau, mean_field=mean_field) for pu, pd in zip(phis_up, phis_dn)]
    lead = dets[0]
    MS = MultiSetup(dets=dets, coeffs=coeffs, E_T=lead.E_T if e_trial is None else float(e_trial),
                    dtau=float(dtau), lbar=lead.lbar.copy(), h0_prop=lead.h0_prop)
    for S in dets:
        S.E_T = MS.E_T
        if mean_field:
            S.lbar = MS.lbar
            S.v0 = one_body_v0(S.h1, S.L) + np.einsum("g,gpq->pq", MS.lbar, S.L)
            S.h0_prop = MS.h0_prop
            S.Eh = sym_expm(S.v0, -0.5 * dtau)
    return MS


def trial_energy_multi(MS: MultiSetup) -> float:
    """<Psi_T|H|Psi_T>/<Psi_T|Psi_T> = sum_d' A_d' <Psi_T|Psi_d'> E_L(Psi_d') / sum_d' A_d' <Psi_T|Psi_d'>,
    exact when no two determinants of the expansion are orthogonal."""
    num, den = 0.0, 0.0
    for d, S in enumerate(MS.dets):
        a, la, e, _ = measure_multi(MS, S.V[0].astype(complex), S.V[1].astype(complex))
        w = MS.coeffs[d] * np.exp(la + 1j * a)
        num, den = num + w * e, den + w
    return float((num / den).real)
