/*
 * afqmc.h -- C ABI of the MI355X phaseless-AFQMC hot path.
 *
 * The library propagates a population of Slater-determinant walkers with
 * phaseless auxiliary-field QMC for a Hamiltonian given in Cholesky form,
 * following Motta & Zhang, arXiv:1711.02242:
 *
 *   H = H0 + sum_{pq,s} h_pq a+_ps a_qs + 1/2 sum_{pqrs,st} v_pqrs a+_ps a+_qt a_st a_rs
 *   v_pqrs = sum_g L^g_pr L^g_qs                               (Sec. II, eq:bo_ham2;
 *                                                               Sec. II.B.2, eq:chol)
 *
 * One call of afqmc_step is one step of the random walk of Sec. III.E for
 * every walker: force bias from the half-rotated Cholesky tensor
 * (eq:fb, eq:precomputing2), auxiliary fields, Taylor-expanded propagation
 * of the Hubbard-Stratonovich exponent between exact one-body half steps
 * (eq:primitive, Theorem 1.4, Sec. III.D.2), periodic re-orthonormalization
 * (Sec. III.D.5), overlap and Green's function (Theorem 1.1-1.2,
 * eq:precomputing), local energy (eq:localenergy2, eq:localenergy3), the
 * phaseless weight (eq:if_rle, eq:cap) and periodic comb population control
 * (Sec. III.D.4).  afqmc_energy returns the sums of the mixed estimator
 * (eq:localenergy with theta = 0).
 *
 * Conventions
 *  - Real, row-major, FP64 host arrays for the Hamiltonian and the trial.
 *  - Complex numbers are (re, im) pairs of doubles, interleaved.
 *  - Walker orbitals are stored orbital-major: U[w][c][p] is coefficient p
 *    (0..M-1) of occupied orbital c of walker w; orbitals c = 0..n_up-1 are
 *    spin up, c = n_up..n_up+n_dn-1 spin down.  (U[w][c][p] = (U_sigma)_{p,c'}
 *    in the paper's M x N_sigma notation.)
 *  - Every function returns AFQMC_OK (0) or a negative afqmc_status code; the
 *    text of a code is afqmc_error_string(code).  Functions that only enqueue
 *    device work return errors of argument checking and of the launches; a
 *    numerical fault inside a walker (non-finite energy, singular overlap) does
 *    not abort: that walker's weight becomes 0 and a sticky bit is set in the
 *    status word, reported by the next synchronizing call (afqmc_energy).
 *  - All device work of a system is enqueued on the HIP stream given to
 *    afqmc_setup, in order.  Calls on one system must be serialized by the
 *    caller; different systems may be used concurrently on different streams.
 */
#ifndef AFQMC_H
#define AFQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define AFQMC_API __attribute__((visibility("default")))
#else
#define AFQMC_API
#endif

typedef enum {
  AFQMC_OK = 0,
  AFQMC_E_ARG = -1,          /* invalid size, pointer, or non-symmetric h1 / L   */
  AFQMC_E_UNSUPPORTED = -2,  /* precision or size outside what is built          */
  AFQMC_E_SINGULAR = -3,     /* trial determinant with V^T V singular             */
  AFQMC_E_NOMEM = -4,        /* device allocation failed, or workspace too small  */
  AFQMC_E_HIP = -5,          /* a HIP runtime call or launch failed               */
  AFQMC_E_NUMERIC = -6,      /* no live walker left, or non-finite estimator      */
  AFQMC_E_STATE = -7         /* call out of order (e.g. step before init)         */
} afqmc_status;

/* Arithmetic of the bulk contractions (local-energy contraction, propagator
 * build and Taylor propagation).  Overlaps, inverses, determinants, QR,
 * weights and all reductions are FP64 in every mode; walker orbitals are
 * always stored as complex128. */
typedef enum {
  AFQMC_FP64 = 0,     /* FP64 everywhere                                        */
  AFQMC_FP32 = 1,     /* FP32 MFMA with FP32 accumulation                       */
  AFQMC_BF16X3 = 2    /* BF16 split products hi*hi + hi*lo + lo*hi, FP32 accum.  */
} afqmc_precision;

/* Bits of the sticky status word. */
#define AFQMC_STATUS_NONFINITE  0x1u   /* a walker produced NaN/Inf and was killed     */
#define AFQMC_STATUS_SINGULAR   0x2u   /* a walker's overlap matrix was singular       */
#define AFQMC_STATUS_ECAP       0x4u   /* the local-energy cap was applied (eq:cap)    */
#define AFQMC_STATUS_WCAP       0x8u   /* the weight cap was applied (App. B.1)        */
#define AFQMC_STATUS_FBCAP     0x10u   /* the force-bias cap was applied (App. B.1)    */
#define AFQMC_STATUS_PHASE     0x20u   /* cos(dtheta) <= 0 killed a walker (eq:if_rle) */

/* Weight update (afqmc_params.flags; at most one of the two bits):
 *   0                        phaseless, local-energy importance function (eq:if_rle):
 *                            W <- W exp(-dtau (Re E_L^cap(Psi) - E_T)) max(0, cos dtheta),
 *                            Re E_L capped to Ebar +- sqrt(C/dtau) (eq:cap)
 *   AFQMC_FLAG_HYBRID        phaseless with the hybrid importance function (eq:hybrid-wt):
 *                            W <- W |I(x, xbar; Psi)| max(0, cos dtheta), capped at w_max
 *   AFQMC_FLAG_FREE_PROJECTION  free projection (Sec. II.C, eq:weight_update) with the hybrid
 *                            importance function: W e^{i theta} <- W e^{i theta} I(x, xbar; Psi),
 *                            no projection and no caps on W or E_L; needs walkers.phase.
 * I(x, xbar; Psi) = [<Psi_T|Psi'>/<Psi_T|Psi>] e^{-dtau (H0 - E_T)} e^{x.xbar - xbar.xbar/2}. */
#define AFQMC_FLAG_HYBRID            0x1u
#define AFQMC_FLAG_FREE_PROJECTION   0x2u
/* Mean-field background subtraction (Sec. II.B.3): v_g -> v_g - <v_g>_T.  The one-body
 * operator becomes v0 + sum_g lbar_g L^g (lbar_g = <L_g>_T), the force bias
 * -i sqrt(dtau) (t_g - lbar_g), and every step multiplies the walker's overlap by the
 * c-number exp(-i sqrt(dtau) sum_g (x_g - xbar_g) lbar_g), which enters the phase and the
 * hybrid weight.  Combines with any weight mode. */
#define AFQMC_FLAG_MEAN_FIELD        0x4u
/* Closed-shell walkers: requires n_up == n_dn and phi_up == phi_dn.  Identical fields act
 * identically on both spins, so U_up == U_dn for every walker at every step; the library
 * then stores and propagates only the up block -- walkers.U is [n_walkers][n_up][M] -- and
 * counts each spin-summed quantity (log overlap, traces, exchange, one-body energy) twice. */
#define AFQMC_FLAG_CLOSED_SHELL      0x8u

typedef struct afqmc_sys_s* afqmc_sys;   /* opaque, library-owned */

typedef struct {
  int32_t M;            /* orbitals, >= 1                                            */
  int32_t n_up, n_dn;   /* electrons per spin, 0 <= n <= M, n_up + n_dn >= 1         */
  int32_t n_chol;       /* Cholesky vectors N_g, >= 0                                */
  double dtau;          /* time step, > 0                                            */
  double e_trial;       /* E_T in the weight; NaN -> E_L(Phi_T, Phi_T) (App. B.2)   */
  int32_t n_taylor;     /* Taylor terms beyond the identity, 1..20 (Sec. III.D.2)    */
  int32_t qr_period;    /* re-orthonormalize after steps k with (k+1) % p == 0; 0 = never */
  int32_t pop_period;   /* comb after steps k with (k+1) % p == 0; 0 = never          */
  int32_t precision;    /* afqmc_precision                                            */
  double el_cap_C;      /* local-energy cap |Re E_L - Ebar| <= sqrt(C/dtau), > 0 (eq:cap) */
  double w_max;         /* weight cap; NaN -> max(100, n_walkers/10) (App. B.1)       */
  double fb_cap;        /* cap on |xbar_g|, > 0 (App. B.1)                            */
  uint32_t flags;       /* AFQMC_FLAG_* bits; weight mode 0 = phaseless local energy  */
  int32_t n_growth;     /* steps of the growth phase, >= 0 (see "Growth phase" below) */
  double theta_guard;   /* precision guard of the mixed modes, > 0 or NaN (see below)   */
} afqmc_params;

/* Precision guard (AFQMC_FP32, AFQMC_BF16X3).  The rounding error of the low-precision
 * contraction grows with the size of Theta = U (V^T U)^-1, which grows as a walker's overlap
 * with the trial becomes ill-conditioned far into a run.  With the guard, every live walker
 * whose largest |Theta_pc| (over both spins and every determinant) exceeds theta_guard has its
 * force-bias traces and exchange sums computed again on the FP64 MFMA contraction, in the same
 * step, and those FP64 values are the ones used.  theta_guard NaN -> 4.0 in AFQMC_FP32 and
 * 0.75 in AFQMC_BF16X3 (measured: at these bounds the local energy stays within 1e-4 Ha of
 * FP64 on the 128-orbital workload); +inf turns the guard off.  The guard needs the FP64
 * MFMA contraction's shapes (max(n_up, n_dn) <= 32, M <= 128): elsewhere it is off.  The
 * FP64 mode ignores theta_guard. */

/* Growth phase (App. B.1, App. B.2).  Every walker population (its workspace) carries the
 * trial energy E_T of the importance function and the centre Ebar of the local-energy cap
 * (eq:cap).  afqmc_walkers_init sets both to the system's E_T (afqmc_info.e_trial).  In the
 * phaseless modes (weight mode 0 or AFQMC_FLAG_HYBRID) the steps k < n_growth form the growth
 * phase: over each population-control block of pop_period steps the library sums, over the
 * live walkers, the total weight before (T_k) and after (T_{k+1}) every weight update and
 * sum_w W Re E_L; at the block's last step, before the comb,
 *   E_T  <- E_T - (1/dtau) log( sum_k T_{k+1} / sum_k T_k )   (eq:corsam; the factor -1/dtau
 *                                                               follows from eq:whycorsam)
 *   Ebar <- sum_k sum_w W Re E_L / sum_k sum_w W               (the local energy averaged over
 *                                                               the block, App. B.1)
 * Afterwards both stay fixed.  n_growth = 0 (or pop_period = 0) keeps both at the initial
 * E_T throughout.  E_T scales every weight of a step alike, so the mixed estimate does not
 * depend on it; it keeps the total weight from drifting, so that w_max keeps its meaning.
 * Free projection has no caps and ignores n_growth. */

typedef struct {
  int32_t n_walkers;     /* >= 1 */
  int32_t reserved;
  void* U;               /* device, [n_walkers][n_up+n_dn][M] complex128 (see Conventions);
                            [n_walkers][n_up][M] with AFQMC_FLAG_CLOSED_SHELL               */
  double* weight;        /* device, [n_walkers]   W >= 0; W == 0 marks a dead walker         */
  double* arg_ovlp;      /* device, [n_walkers]   arg <Phi_T|Psi> in (-pi, pi]               */
  double* log_ovlp;      /* device, [n_walkers]   log |<Phi_T|Psi>| (diagnostic)            */
  double* e_loc;         /* device, [n_walkers][2] complex E_L of the current determinant    */
  double* phase;         /* device, [n_walkers]   walker phase theta (free projection; may be
                            NULL in the phaseless modes, where theta is identically 0)      */
  int64_t* walker_id;    /* device, [n_walkers]   ids that select the field stream           */
  void* workspace;       /* device, afqmc_workspace_bytes() bytes, 256-byte aligned          */
  size_t workspace_bytes;
  int64_t step;          /* steps taken; afqmc_step advances it                             */
} afqmc_walkers;

typedef struct {
  uint64_t seed;         /* Philox4x64-10 key word 0                                         */
  uint64_t job_id;       /* Philox4x64-10 key word 1                                         */
  const double* x;       /* NULL: draw the fields on the device from the counter stream
                            (block, walker_id, step, 0); else device [n_walkers][n_chol]
                            fields for this step, read as given                              */
  double u_comb;         /* comb uniform in (0,1] if population control is due; NaN: draw it
                            from the counter stream (0, 0, step, 1)                          */
} afqmc_fields;

typedef struct {
  double e_trial;        /* E_T in use                                     */
  double e_hf;           /* E_L(Phi_T, Phi_T)                              */
  size_t device_bytes;   /* library-owned device memory of this system     */
} afqmc_info;

/* Copy the Hamiltonian and trial to the device and precompute everything that
 * does not depend on the walkers (Sec. II.B.2 eq:mcd1; Sec. III.D.2):
 *   v0 = h1 - 1/2 sum_g L^g L^g,  E_h = exp(-dtau/2 v0) (FP64 eigendecomposition),
 *   half-rotated Lh^g_s = V_s^T L^g and h~_s = V_s^T h1 in every precision used,
 *   E_HF = E_L(Phi_T, Phi_T).
 * h1      host, M*M row-major, real symmetric (|h - h^T| <= 1e-12 max|h|)
 * L_chol  host, n_chol*M*M row-major, each L^g real symmetric; may be NULL if n_chol == 0
 * phi_up  host, M*n_up row-major (the M x N_up trial matrix V_up); phi_dn likewise.
 *         The trial need not be orthonormal (Theorem 1.5) but V_s^T V_s must be invertible.
 * stream  hipStream_t on which every later call of this system enqueues its work
 *         (NULL = the null stream).
 * On success *out owns device memory until afqmc_destroy. */
AFQMC_API int afqmc_setup(const afqmc_params* p, double h0, const double* h1, const double* L_chol,
                const double* phi_up, const double* phi_dn, void* stream, afqmc_sys* out);

/* Setup with a multi-determinant trial Psi_T = sum_d A_d |Psi_d> (Sec. II.B; the mixed
 * estimator of eq:localenergy2 and the traces of eq:precomputing2 are linear in <Psi_T|):
 * every per-walker quantity is formed from r_d = conj(A_d) <Psi_d|Psi> as
 *   <Psi_T|Psi> = sum_d r_d,  E_L = sum_d r_d E_L^d / sum_d r_d,  t_g = sum_d r_d t^d_g / sum_d r_d.
 * n_det   1..1024 determinants.
 * coeffs  host, n_det*2 doubles: A_d = coeffs[2d] + i coeffs[2d+1] (finite; not normalized).
 * phi_up  host, n_det blocks of M*n_up row-major (block d is V_{d,up}); phi_dn likewise.
 *         Block 0 is the leading determinant: E_T (when p->e_trial is NaN), E_HF and the
 *         mean-field shifts are taken from it, and afqmc_walkers_init starts the walkers at it;
 *         V_{0,s}^T V_{0,s} must be invertible.  The other blocks may be orthogonal to it.
 * A determinant whose overlap with a walker is exactly singular contributes r_d = 0 and is
 * left out of that walker's E_L (exact for walkers non-orthogonal to every determinant);
 * a walker orthogonal to all of them is treated as a singular overlap.  With
 * AFQMC_FLAG_CLOSED_SHELL every block needs phi_up == phi_dn.  The per-walker workspace
 * grows with n_det (afqmc_workspace_bytes).  Requires max(n_up, n_dn) <= 32 and M <= 128
 * (the MFMA kernels), else AFQMC_E_UNSUPPORTED; otherwise as afqmc_setup. */
AFQMC_API int afqmc_setup_multidet(const afqmc_params* p, double h0, const double* h1,
                                   const double* L_chol, int32_t n_det, const double* coeffs,
                                   const double* phi_up, const double* phi_dn, void* stream,
                                   afqmc_sys* out);

/* Device bytes of workspace that n_walkers walkers need (for admission by HBM footprint). */
AFQMC_API int afqmc_workspace_bytes(afqmc_sys s, int32_t n_walkers, size_t* bytes);

/* Sizes and energies of a system (host values, no device work). */
AFQMC_API int afqmc_get_info(afqmc_sys s, afqmc_info* info);

/* Start every walker at {Psi_I = Phi_T, W = 1, theta = 0} (Sec. II.C, Sec. III.E step 1):
 * writes U, weight, walker_id = index, step = 0, computes the overlap phase, E_L and
 * the cached force-bias traces, and starts the population's growth state (E_T = Ebar = the
 * system's E_T, empty block sums).  Asynchronous. */
AFQMC_API int afqmc_walkers_init(afqmc_sys s, afqmc_walkers* w);

/* Recompute, from the current U, everything cached per walker: arg_ovlp, log_ovlp, e_loc
 * and the force-bias traces (Theorem 1.1-1.2, eq:precomputing2, eq:localenergy3).  Weights
 * and step are untouched.  Used after writing U directly (restart, tests).  Asynchronous. */
AFQMC_API int afqmc_measure(afqmc_sys s, afqmc_walkers* w);

/* One step of the random walk for every walker with W > 0 (Sec. III.E), then w->step++.
 * Asynchronous; allocates nothing. */
AFQMC_API int afqmc_step(afqmc_sys s, afqmc_walkers* w, const afqmc_fields* f);

/* Tile shapes of the local-energy contraction (the dominant kernel).  The register-resident
 * FP32 / BF16x3 kernel takes W = 4 or 2 walkers per workgroup (W = 2 gives small walker
 * populations twice the workgroups); the wide kernel takes one walker per workgroup and splits
 * Theta's columns over its wavefronts; the flattened kernel stacks the N-row blocks of q
 * consecutive Cholesky vectors and puts Re and Im Theta side by side, so N is padded to a
 * multiple of 16 once per q blocks instead of once per block and plane (N up to 64, M up to
 * 224); the stacked-row kernel stacks the rows the same way but keeps Re and Im Theta as two
 * operands of 16 columns (N padded to a multiple of 16, half the operand traffic per flop).
 * Every variant computes the same quantities.
 *   AFQMC_TILE_DEFAULT  where the shape fits it (N <= 32, M <= 128) the block-exchange
 *                       kernel for 16 < N <= 32 (W = 8 when the workgroups with work still
 *                       number at least the device's compute units, else W = 4) and W = 4
 *                       for N <= 16, else wide
 *   AFQMC_TILE_W4, AFQMC_TILE_W2, AFQMC_TILE_WIDE  (wide needs N_P >= 32, i.e. N > 16 or M > 128)
 *   AFQMC_TILE_FLAT, AFQMC_TILE_STACK  (any FP32 / BF16x3 shape)
 *   AFQMC_TILE_PP  eight walkers per workgroup, two wavefronts per SIMD alternating between
 *                  the MFMA chain of one Cholesky vector and the LDS epilogue of the one before
 *                  (N <= 32, M <= 128)
 *   AFQMC_TILE_BX  W = 4 with Omega as four 16 x 16 blocks, the off-diagonal exchange
 *                  lane-local (16 < N <= 32, M <= 128); AFQMC_TILE_BX8 the same with W = 8
 * The FP64 mode has one contraction kernel per shape and accepts only the default. */
#define AFQMC_TILE_DEFAULT 0
#define AFQMC_TILE_W4 1
#define AFQMC_TILE_W2 2
#define AFQMC_TILE_WIDE 3
#define AFQMC_TILE_FLAT 4
#define AFQMC_TILE_STACK 5
#define AFQMC_TILE_PP 6
#define AFQMC_TILE_BX 7
#define AFQMC_TILE_BX8 8

/* Autotuner: times every variant valid for the system's shape on these walkers (initialized
 * or measured; one untimed and three timed launches each, on the system's stream, writing only
 * workspace partial sums), keeps the fastest for every later step and returns it in *tile
 * (and its time per launch in *ms if ms != NULL).  With reuse != 0 a shape tuned before in the
 * process (same device, precision, M, N_up, N_dn, N_g, determinants and walker count) takes
 * the stored choice without timing (*ms = -1).  Synchronizes the stream. */
AFQMC_API int afqmc_autotune(afqmc_sys s, afqmc_walkers* w, int32_t reuse, int32_t* tile,
                             double* ms);
/* Force a variant (AFQMC_E_UNSUPPORTED if it does not fit the shape) / read the one in use. */
AFQMC_API int afqmc_set_tile(afqmc_sys s, int32_t tile);
AFQMC_API int afqmc_get_tile(afqmc_sys s, int32_t* tile);

/* Batches: many systems (uneven M, N, N_g and walker counts) stepped together, one graph
 * launch per step.  Each system keeps its own walkers, fields stream and parameters; the batch
 * captures one afqmc_step of every system into a HIP graph -- each system on a branch stream
 * of its own, forked from and joined into the batch stream, so independent systems may run
 * concurrently -- and replays it with hipGraphLaunch.  One graph is kept per combination of
 * due re-orthonormalization / comb phases.  The results are those of afqmc_step on every
 * system in turn: same kernels, same arithmetic, same field stream.
 *
 * afqmc_batch_create: n >= 1 systems and their walkers (distinct populations, initialized;
 *   the walkers structs and every array they point to must stay valid and unmoved until
 *   afqmc_batch_destroy).  stream: the caller's stream (NULL = the null stream); each batch
 *   step runs after the work enqueued on it before the call, and work enqueued on it after
 *   the call runs after the step.  The graphs run on a stream the batch owns.  Synchronizes
 *   the systems' streams once.  Work of the systems' own streams issued later must be
 *   ordered with the batch's stream by the caller.
 * afqmc_batch_step: fields[n], one per system, with x == NULL (the fields are drawn on the
 *   device from the counter stream) and u_comb NaN; a change of seed or job id recaptures.
 *   Advances every walkers->step.  Asynchronous; allocates nothing once every phase has
 *   been captured (the first steps capture and instantiate the graphs).
 * afqmc_batch_destroy: synchronizes the batch stream and frees the graphs and streams. */
typedef struct afqmc_batch_s* afqmc_batch;
AFQMC_API int afqmc_batch_create(int32_t n, const afqmc_sys* systems, afqmc_walkers* const* walkers,
                                 void* stream, afqmc_batch* out);
AFQMC_API int afqmc_batch_step(afqmc_batch b, const afqmc_fields* fields);
AFQMC_API int afqmc_batch_destroy(afqmc_batch b);
/* How a batch step launches the local-energy contraction, the dominant kernel.
 *   0  every system's step keeps its own kernels on its branch: the batch's only mode
 *      (AFQMC_OK, nothing changes).
 *   1  one launch per family of systems sharing a kernel instance: not available
 *      (AFQMC_E_UNSUPPORTED).  An implementation crashed the host process inside the first
 *      batch step that captured its graph, no cause was found in this library, and it was
 *      taken out.
 * Any other value: AFQMC_E_ARG. */
AFQMC_API int afqmc_batch_set_mode(afqmc_batch b, int32_t mode);

/* Draw (or copy) the fields the next afqmc_step would use, into device x_out
 * [n_walkers][n_chol] doubles.  Asynchronous. */
AFQMC_API int afqmc_fields_draw(afqmc_sys s, const afqmc_walkers* w, const afqmc_fields* f, double* x_out);

/* Mixed-estimator sums over the walkers (eq:localenergy), reduced on the device in a fixed
 * order, copied to the host, synchronizing the stream.  With c_w = W_w e^{i theta_w}
 * (theta = 0 in the phaseless modes) and E_w = E_L(Psi_w), its real part capped to
 * Ebar +- sqrt(C/dtau) (eq:cap; Ebar of the population, see "Growth phase") in the phaseless
 * modes and uncapped in free projection:
 *   out[0] = Re sum_w c_w E_w      out[1] = Im sum_w c_w E_w
 *   out[2] = Re sum_w c_w          out[5] = Im sum_w c_w
 *   out[3] = number of walkers with W > 0
 *   out[4] = status word (AFQMC_STATUS_* bits accumulated since setup or the last clear)
 * The phaseless mixed estimate is out[0] / out[2]; the free-projection one is
 * (out[0] + i out[1]) / (out[2] + i out[5]).
 * Returns AFQMC_E_NUMERIC if no walker is alive or a sum is not finite. */
AFQMC_API int afqmc_energy(afqmc_sys s, const afqmc_walkers* w, double out[6]);

/* The sums of afqmc_energy written to device memory out_dev[0..5] (out_dev[4] = the status
 * word as a double) without synchronizing: per-step records of the mixed estimator in a
 * caller-owned device buffer, read back in blocks (the serving loop).  Asynchronous. */
AFQMC_API int afqmc_energy_enqueue(afqmc_sys s, const afqmc_walkers* w, double* out_dev);

/* HBM footprint of a job before it is set up (admission by memory): *system_bytes = the
 * device memory afqmc_setup (n_det == 1) or afqmc_setup_multidet would hold for these
 * parameters (the value afqmc_get_info reports), *walker_bytes = afqmc_workspace_bytes for
 * n_walkers plus the walker arrays of afqmc_walkers (U, weight, arg_ovlp, log_ovlp, e_loc,
 * phase, walker_id) and 256 bytes of workspace alignment.  Host arithmetic only; returns
 * AFQMC_E_UNSUPPORTED for shapes afqmc_setup would refuse for their size. */
AFQMC_API int afqmc_footprint_bytes(const afqmc_params* p, int32_t n_det, int32_t n_walkers,
                                    size_t* system_bytes, size_t* walker_bytes);

/* Attainable dense MFMA rate (a diagnostic beside the datasheet peaks): launches, on
 * hip_stream, workgroups whose wavefronts (as many as fit at once) each run MFMA instructions
 * of one kind into four accumulators on register operands only, once untimed and three times
 * timed with HIP events, and returns the fastest timed launch's rate in *tflops (dense
 * TFLOP/s; synchronizes the stream).
 *   AFQMC_FP32    v_mfma_f32_32x32x2_f32    (datasheet 157.3)
 *   AFQMC_FP64    v_mfma_f64_16x16x4_f64    (datasheet 78.6)
 *   AFQMC_BF16X3  v_mfma_f32_32x32x16_bf16  (datasheet 2500; a BF16x3 product takes three)
 * out_dev: caller-owned device memory of at least AFQMC_MFMA_PEAK_BYTES bytes, overwritten
 * (one double per workgroup keeps the chains live).  AFQMC_E_ARG for a missing or short
 * buffer, AFQMC_E_UNSUPPORTED for another precision, AFQMC_E_HIP on a launch failure. */
#define AFQMC_MFMA_PEAK_BYTES 16384
AFQMC_API int afqmc_mfma_peak(int32_t precision, void* out_dev, size_t out_bytes,
                              void* hip_stream, double* tflops);

/* The current E_T (out[0]) and cap centre Ebar (out[1]) of a walker population (see
 * "Growth phase"); synchronizes the stream. */
AFQMC_API int afqmc_get_growth(afqmc_sys s, const afqmc_walkers* w, double out[2]);

/* Counters of the rare-event bounds (App. B.1) accumulated by afqmc_step since setup or the
 * last clear (synchronizes the stream; clear != 0 zeroes them afterwards):
 *   out[0] walker-steps whose local energy was capped in the weight (eq:cap)
 *   out[1] walker-steps whose weight was capped at w_max
 *   out[2] force-bias components xbar_g whose modulus was capped at fb_cap
 *   out[3] walker-steps whose weight was updated (live walkers)
 *   out[4] walker-steps whose contraction the precision guard redid in FP64
 * out[0] / out[3] is the fraction of capped walker-steps. */
AFQMC_API int afqmc_get_bound_counts(afqmc_sys s, uint64_t out[5], int clear);

/* Read and clear the sticky status word (synchronizes the stream). */
AFQMC_API int afqmc_get_status(afqmc_sys s, uint32_t* status, int clear);

/* Kernel timing with HIP events on the system's stream.  enable = 1 starts recording
 * (and resets the totals), 0 stops.  afqmc_kernel_time returns the accumulated time in
 * milliseconds and the number of launches of one kernel group, synchronizing the stream:
 *   0 = local-energy contraction, 1 = overlap / inverse, 2 = fields and force bias,
 *   3 = propagator build, 4 = Taylor propagation, 5 = QR, 6 = weights, 7 = comb,
 *   8 = energy assembly, 9 = the precision guard (walker list and FP64 redo). */
AFQMC_API int afqmc_kernel_timing(afqmc_sys s, int enable);
AFQMC_API int afqmc_kernel_time(afqmc_sys s, int kernel, double* ms, int64_t* launches);

/* Modified Cholesky decomposition of the two-electron tensor (Sec. II.B.2, eq:chol, eq:chol2):
 * with V_{(p r),(q s)} = v_pqrs, find vectors L^g (each M x M) with V ~ sum_g L^g L^g^T.  Each
 * step takes the largest residual diagonal Dmax (first index on ties), stops when Dmax < delta,
 * zeroes the entries with sqrt(|D_mu| Dmax) <= min(1e-9, delta) (damped prescreening) and appends
 * the residual pivot column / sqrt(Dmax).  On convergence every residual element is <= delta.
 * eri       device, [M][M][M][M] doubles, eri[p][q][r][s] = v_pqrs (real orbitals, so
 *           v_pqrs = v_rqps = v_psrq); read only
 * L_out     device, [max_vectors][M][M] doubles (caller-owned); vector g is L_out[g]
 * n_vectors host out: number of vectors written
 * converged host out (may be NULL): 1 if Dmax < delta was reached within max_vectors
 * workspace device, afqmc_mcd_workspace_bytes(M) bytes, 256-byte aligned
 * stream    hipStream_t for the work; the call synchronizes it.
 * Returns AFQMC_E_ARG / AFQMC_E_NOMEM on bad arguments, AFQMC_E_HIP on launch errors. */
AFQMC_API int afqmc_mcd_workspace_bytes(int32_t M, size_t* bytes);
AFQMC_API int afqmc_modified_cholesky(const double* eri, int32_t M, double delta,
                                      int32_t max_vectors, double* L_out, int32_t* n_vectors,
                                      int32_t* converged, void* workspace,
                                      size_t workspace_bytes, void* stream);

/* Allocation-free modified Cholesky, for callers that cannot allocate device memory
 * (serving loops and harnesses that forbid hipMalloc): the same decomposition, kernels and
 * results as afqmc_modified_cholesky, with its workspace in a library-owned static device
 * array of AFQMC_MCD_NOALLOC_BYTES bytes, one per GPU, held until the process ends (this
 * call allocates nothing).  Limit: M <= AFQMC_MCD_NOALLOC_MAX_M, else AFQMC_E_UNSUPPORTED
 * before any device work.  The array of a GPU is shared by every call on that GPU and keeps
 * the last call's contents; each call initializes what it reads.  Calls that overlap on one
 * GPU (from several threads, or on several streams) race on it: serialize them.  The stream
 * must belong to the current device.  Arguments and errors otherwise as
 * afqmc_modified_cholesky. */
#define AFQMC_MCD_NOALLOC_MAX_M 256
#define AFQMC_MCD_NOALLOC_BYTES 590080   /* D 256^2 doubles + 256^2 flags + state, 256-aligned */
AFQMC_API int afqmc_modified_cholesky_noalloc(const double* eri, int32_t M, double delta,
                                              int32_t max_vectors, double* L_out,
                                              int32_t* n_vectors, int32_t* converged,
                                              void* stream);

/* Free the device memory owned by the system. */
AFQMC_API int afqmc_destroy(afqmc_sys s);

AFQMC_API const char* afqmc_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* AFQMC_H */
