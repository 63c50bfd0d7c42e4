// Host side of the AFQMC C ABI (include/afqmc.h): setup precompute, workspace
// layout, and the launch sequence of one walker step (arXiv:1711.02242, Sec. III.E).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/afqmc.h"
#include "common.hpp"
#include "kernels_fp64.hpp"
#include "kernels_mfma.hpp"
#include "kernels_prop.hpp"
#include "kernels_mcd.hpp"
#include "kernels_peak.hpp"

static_assert(PEAK_MAX_BLOCKS * sizeof(double) <= AFQMC_MFMA_PEAK_BYTES, "peak scratch size");

namespace {
// Order of the packed pairs (q, p), p <= q, of the symmetric A-build: 8 x 8 blocks of the
// lower triangle, block row by block row, each block row by row.  A workgroup's tile of
// consecutive packed columns then covers a few whole rows of a block, so the mirrored stores
// A[p][q] of a tile fill the same short row segments as its direct stores A[q][p] and reach
// memory as whole segments (a plain row-by-row order spreads them over a column of A).
inline std::vector<std::pair<int, int>> pair_order(int M) {
  constexpr int B = 8;
  std::vector<std::pair<int, int>> o;
  o.reserve((size_t)M * (M + 1) / 2);
  for (int qb = 0; qb < M; qb += B)
    for (int pb = 0; pb <= qb; pb += B)
      for (int q = qb; q < std::min(qb + B, M); ++q)
        for (int pp = pb; pp < std::min(pb + B, M) && pp <= q; ++pp) o.emplace_back(q, pp);
  return o;
}


enum { KG_CONTRACT = 0, KG_OVERLAP, KG_FIELDS, KG_ABUILD, KG_PROP, KG_QR, KG_WEIGHT, KG_COMB,
       KG_ASSEMBLE, KG_GUARD, KG_COUNT };

struct TimedLaunch {
  int group;
  hipEvent_t a, b;
};

struct WsLayout {
  size_t thetaT, tcur, tpart, exch, e1, logdet, wflag, enew, y, A, X0, X1, Y, parent, csum,
      wnew, asnap, lsnap, esum, thetaP, y32, fbterm, mfterm, logR, psnap, ldc, wflc, dstep, growth,
      thmax, thetaP64, glist, gcount, total;
};

}  // namespace

struct afqmc_sys_s {
  afqmc_params p;
  int M, nup, ndn, ntot, G;
  double h0, e_trial, e_hf, s;
  hipStream_t stream;
  int device;
  // device, library-owned
  double* Eh = nullptr;    // [M][M]
  double* V = nullptr;     // [ntot][M]
  double* Lh = nullptr;    // [G][ntot][M]
  double* ht = nullptr;    // [ntot][M]
  unsigned* status = nullptr;
  unsigned long long* capcount = nullptr;   // [CAP_COUNT] counters of the rare-event bounds
  MfmaTables mt;           // packed low-precision copies for the MFMA contraction
  MfmaTables mt64;         // FP64 packed copy for the precision guard of the mixed modes
  bool guard_on = false;   // mixed mode with the guard: walkers with max|Theta| > guard redone
  double guard = INFINITY; //   in FP64 (afqmc_params.theta_guard)
  float* Lt32 = nullptr;   // [apk_size(M)][Gp] FP32 transposed Cholesky tensor, block-packed
  int* abpairs = nullptr;  // [M(M+1)/2][2] (q M + p, p M + q) of each packed column (FP64)
  double* Lt64 = nullptr;  // [M(M+1)/2][Gp64] FP64 packed L^T (FP64 A-build)
  int Gp64 = 0;            // G rounded up to 16
  float* Eh32 = nullptr;   // [M][M] FP32 exp(-dtau/2 v0)
  int Gp = 0;              // G rounded up to 32
  bool f32_prop = false;   // A-build and propagation on FP32 MFMA (mixed-precision modes)
  bool prop_wide = false;  // propagation by k_propagate_f32_wide (M > 128 or N_up + N_dn > 64)
  int sf = 1;              // spin factor: 2 in closed-shell mode (only the up block is stored)
  double h0p = 0.0;        // constant of the propagated Hamiltonian (H0 - 1/2 sum lbar^2)
  double* lbar = nullptr;  // [G] mean-field shifts <L_g>_T (zeros without subtraction)
  // multi-determinant trial: V, ht, Lh and the MFMA tables hold n_det blocks (leading first)
  int n_det = 1;
  bool multi = false;
  double* coef = nullptr;  // [n_det][2] expansion coefficients A_d
  int tile = 0;            // contraction variant (TILE_*), set by afqmc_autotune / afqmc_set_tile
  size_t device_bytes = 0;
  // timing
  bool timing = false;
  std::vector<TimedLaunch> launches;
  double acc_ms[KG_COUNT] = {0};
  int64_t acc_n[KG_COUNT] = {0};
};

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

WsLayout layout(const afqmc_sys_s* S, size_t nw) {
  WsLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += al256(bytes);
    return r;
  };
  const size_t M = S->M, G = S->G, nt = S->ntot, nd = S->n_det;
  L.thetaT = take(S->mt.enabled ? 0 : nw * nd * nt * M * 16);   // FP64 VALU contraction only
  L.tcur = take(nw * G * 16);
  L.tpart = take(nw * nd * 2 * G * 16);
  L.exch = take(nw * nd * 2 * 16);
  L.e1 = take(nw * nd * 2 * 16);
  L.logdet = take(nw * nd * 2 * 16);
  L.wflag = take(nw * nd * 2 * 4);
  L.enew = take(nw * 16);
  L.y = take(nw * G * 16);
  // exponent A: FP32 block-packed Re and Im planes, else FP64 complex M x M
  L.A = take(S->f32_prop ? nw * (size_t)apk_size((int)M) * 8 : nw * M * M * 16);
  L.X0 = take(nw * nt * M * 16);
  L.X1 = take(nw * nt * M * 16);
  L.Y = take(nw * nt * M * 16);
  L.parent = take(nw * 4);
  L.csum = take(nw * 8);
  L.wnew = take(64);
  L.asnap = take(nw * 8);
  L.lsnap = take(nw * 8);
  L.esum = take(64);
  L.thetaP = take(mfma_theta_bytes(S->mt, nw));
  L.y32 = take(S->f32_prop ? nw * 2 * (size_t)S->Gp * 4 : 0);
  const size_t nblk = (size_t)((S->G + 3) / 4);
  L.fbterm = take((S->p.flags & (AFQMC_FLAG_HYBRID | AFQMC_FLAG_FREE_PROJECTION)) ? nw * nblk * 16 : 0);
  L.mfterm = take((S->p.flags & AFQMC_FLAG_MEAN_FIELD) ? nw * nblk * 16 : 0);
  L.logR = take(nw * 2 * 8);
  L.psnap = take(nw * 8);
  L.ldc = take(S->multi ? nw * 2 * 16 : 0);
  L.wflc = take(S->multi ? nw * 2 * 4 : 0);
  L.dstep = take(8);
  L.growth = take(GR_COUNT * 8);
  L.thmax = take(S->guard_on ? nw * nd * 2 * 8 : 0);
  L.thetaP64 = take(S->guard_on ? mfma_theta_bytes(S->mt64, nw) : 0);
  L.glist = take(S->guard_on ? nw * 4 : 0);
  L.gcount = take(S->guard_on ? 8 : 0);
  L.total = o;
  return L;
}

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) return AFQMC_E_HIP;       \
  } while (0)

// Event bracket of one launch group when timing is on.
struct Timer {
  afqmc_sys_s* S;
  int group;
  hipEvent_t a{}, b{};
  Timer(afqmc_sys_s* s, int g) : S(s), group(g) {
    if (S->timing) {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      (void)hipEventRecord(a, S->stream);
    }
  }
  ~Timer() {
    if (S->timing) {
      (void)hipEventRecord(b, S->stream);
      S->launches.push_back(TimedLaunch{group, a, b});
    }
  }
};

void flush_timing(afqmc_sys_s* S) {
  if (S->launches.empty()) return;
  (void)hipStreamSynchronize(S->stream);
  for (auto& t : S->launches) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t.a, t.b);
    S->acc_ms[t.group] += ms;
    S->acc_n[t.group] += 1;
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  S->launches.clear();
}

// exp(c A) for a real symmetric M x M matrix by scaling and squaring of the Taylor series.
void host_expm_sym(const std::vector<double>& A, int M, double c, std::vector<double>& out) {
  double nrm = 0.0;
  for (int i = 0; i < M; ++i) {
    double r = 0.0;
    for (int j = 0; j < M; ++j) r += fabs(A[(size_t)i * M + j]);
    nrm = fmax(nrm, r);
  }
  nrm *= fabs(c);
  int sq = 0;
  while (nrm > 0.25) {
    nrm *= 0.5;
    ++sq;
  }
  const double cs = c / std::ldexp(1.0, sq);
  std::vector<double> term((size_t)M * M, 0.0), next((size_t)M * M), res((size_t)M * M, 0.0);
  for (int i = 0; i < M; ++i) term[(size_t)i * M + i] = 1.0;
  res = term;
  for (int n = 1; n < 40; ++n) {
    double mx = 0.0;
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        double acc = 0.0;
        for (int k = 0; k < M; ++k) acc += A[(size_t)i * M + k] * term[(size_t)k * M + j];
        next[(size_t)i * M + j] = acc * cs / n;
        mx = fmax(mx, fabs(next[(size_t)i * M + j]));
      }
    term.swap(next);
    for (size_t e = 0; e < res.size(); ++e) res[e] += term[e];
    if (mx < 1e-300 || mx < 1e-19) break;
  }
  for (int q = 0; q < sq; ++q) {
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        double acc = 0.0;
        for (int k = 0; k < M; ++k) acc += res[(size_t)i * M + k] * res[(size_t)k * M + j];
        next[(size_t)i * M + j] = acc;
      }
    res.swap(next);
  }
  for (int i = 0; i < M; ++i)
    for (int j = i + 1; j < M; ++j) {
      const double v = 0.5 * (res[(size_t)i * M + j] + res[(size_t)j * M + i]);
      res[(size_t)i * M + j] = res[(size_t)j * M + i] = v;
    }
  out = res;
}

// Inverse of a small real matrix by Gauss-Jordan with partial pivoting; false if singular.
bool host_inverse(std::vector<double>& a, int n) {
  std::vector<double> inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (fabs(a[(size_t)i * n + k]) > fabs(a[(size_t)piv * n + k])) piv = i;
    if (!(fabs(a[(size_t)piv * n + k]) > 0.0)) return false;
    for (int j = 0; j < n; ++j) {
      std::swap(a[(size_t)k * n + j], a[(size_t)piv * n + j]);
      std::swap(inv[(size_t)k * n + j], inv[(size_t)piv * n + j]);
    }
    const double d = a[(size_t)k * n + k];
    for (int j = 0; j < n; ++j) {
      a[(size_t)k * n + j] /= d;
      inv[(size_t)k * n + j] /= d;
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = a[(size_t)i * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)i * n + j] -= f * a[(size_t)k * n + j];
        inv[(size_t)i * n + j] -= f * inv[(size_t)k * n + j];
      }
    }
  }
  a = inv;
  return true;
}

// Runs body(i, thread) for i in [0, n) on up to 16 host threads (setup precompute only).
template <class F>
void parallel_for(int n, F body) {
  const unsigned hw = std::thread::hardware_concurrency();
  const int nt = std::max(1, std::min({n, 16, (int)(hw ? hw : 1)}));
  if (nt == 1) {
    for (int i = 0; i < n; ++i) body(i, 0);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&, t] {
      for (int i = t; i < n; i += nt) body(i, t);
    });
  for (auto& th : pool) th.join();
}

int setup_threads(int n) {
  const unsigned hw = std::thread::hardware_concurrency();
  return std::max(1, std::min({n, 16, (int)(hw ? hw : 1)}));
}

template <typename T>
int dev_upload(afqmc_sys_s* S, T** dst, const T* src, size_t count) {
  if (count == 0) count = 1;
  if (hipMalloc(reinterpret_cast<void**>(dst), count * sizeof(T)) != hipSuccess) return AFQMC_E_NOMEM;
  S->device_bytes += count * sizeof(T);
  if (src) HIPCHK(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return AFQMC_OK;
}

void free_sys(afqmc_sys_s* S) {
  if (!S) return;
  for (auto& t : S->launches) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  (void)hipFree(S->Eh);
  (void)hipFree(S->V);
  (void)hipFree(S->Lh);
  (void)hipFree(S->ht);
  (void)hipFree(S->status);
  (void)hipFree(S->capcount);
  (void)hipFree(S->Lt32);
  (void)hipFree(S->abpairs);
  (void)hipFree(S->Lt64);
  (void)hipFree(S->lbar);
  (void)hipFree(S->Eh32);
  (void)hipFree(S->coef);
  mfma_free_tables(S->mt);
  mfma_free_tables(S->mt64);
  delete S;
}

int check_walkers(const afqmc_sys_s* S, const afqmc_walkers* w) {
  if (!w || w->n_walkers < 1 || !w->U || !w->weight || !w->arg_ovlp || !w->log_ovlp ||
      !w->e_loc || !w->walker_id || !w->workspace)
    return AFQMC_E_ARG;
  if ((reinterpret_cast<uintptr_t>(w->workspace) & 255u) != 0) return AFQMC_E_ARG;
  if ((S->p.flags & AFQMC_FLAG_FREE_PROJECTION) && !w->phase) return AFQMC_E_ARG;
  if (w->workspace_bytes < layout(S, (size_t)w->n_walkers).total) return AFQMC_E_NOMEM;
  return AFQMC_OK;
}

int launch_overlap(afqmc_sys_s* S, const afqmc_walkers* w, const WsLayout& L, int check_weight) {
  Timer tm(S, KG_OVERLAP);
  const int nmax = std::max(S->nup, S->ndn);
  // one workgroup per (walker, spin, determinant)
  dim3 grid(w->n_walkers, 2, S->n_det);
  void* ws = w->workspace;
  void* packed = S->mt.enabled ? at<void>(ws, L.thetaP) : nullptr;
  const int kind = !S->mt.enabled ? 0
                   : S->mt.precision == AFQMC_FP64 ? 3
                   : S->mt.precision == AFQMC_BF16X3 ? 2 : 1;
  const size_t shm = (size_t)nmax * (2 * nmax + 1) * 16 + 64;   // [T | I] and 8 doubles
#define OVL(NPAD)                                                                              \
  do {                                                                                         \
    (void)hipFuncSetAttribute((const void*)k_overlap_mfma<NPAD>,                               \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);           \
    hipLaunchKernelGGL(k_overlap_mfma<NPAD>, grid, dim3(256), shm, S->stream, S->M, S->nup,     \
                       S->ndn, S->V, S->ht, (const cd*)w->U, w->weight, check_weight,          \
                       S->mt.enabled ? nullptr : at<cd>(ws, L.thetaT), at<cd>(ws, L.logdet),   \
                       at<cd>(ws, L.e1),                                                       \
                       at<unsigned>(ws, L.wflag), packed, kind, S->mt.NP, S->mt.KP,           \
                       S->guard_on ? at<double>(ws, L.thmax) : nullptr,                        \
                       S->guard_on ? at<double>(ws, L.thetaP64) : nullptr);                    \
  } while (0)
#define OVW(NPAD)                                                                              \
  hipLaunchKernelGGL(k_overlap_wave<NPAD>, grid, dim3(64), 0, S->stream, S->M, S->nup, S->ndn,   \
                     S->V, S->ht, (const cd*)w->U, w->weight, check_weight,                      \
                     S->mt.enabled ? nullptr : at<cd>(ws, L.thetaT), at<cd>(ws, L.logdet),       \
                     at<cd>(ws, L.e1), at<unsigned>(ws, L.wflag), packed, kind, S->mt.NP,        \
                     S->mt.KP, S->guard_on ? at<double>(ws, L.thmax) : nullptr,                  \
                     S->guard_on ? at<double>(ws, L.thetaP64) : nullptr, S->guard)
  // up to N = 32 one wavefront per matrix (elimination in registers), beyond it the
  // four-wavefront kernel with [T | I] in LDS
  if (nmax <= 16)
    OVW(16);
  else if (nmax <= 32)
    OVW(32);
  else if (nmax <= 48)
    OVL(48);
  else
    OVL(64);
#undef OVL
#undef OVW
  HIPCHK(hipGetLastError());
  return AFQMC_OK;
}

// The local-energy contraction and the energy assembly.  `in_step` counts the walkers the
// precision guard redoes in FP64 (the counters of afqmc_get_bound_counts cover steps only).
// The contraction proper (tpart, exch of every walker in the system's precision).
int launch_contraction(afqmc_sys_s* S, const afqmc_walkers* w, const WsLayout& L) {
  void* ws = w->workspace;
  if (!S->mt.enabled) {
    Timer tm(S, KG_CONTRACT);
    const size_t nmax = std::max(S->nup, S->ndn);
    const size_t om = nmax * (nmax + 1) * 16 + 64;
    const size_t staged = nmax * (S->M + 1) * 16 + om;
    if (staged <= 150 * 1024) {
      (void)hipFuncSetAttribute((const void*)k_contract_fp64<true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)staged);
      hipLaunchKernelGGL(k_contract_fp64<true>, dim3(w->n_walkers, 2), dim3(256), staged, S->stream,
                         S->M, S->nup, S->ndn, S->G, S->Lh, at<cd>(ws, L.thetaT), w->weight,
                         at<cd>(ws, L.tpart), at<cd>(ws, L.exch));
    } else {
      (void)hipFuncSetAttribute((const void*)k_contract_fp64<false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)om);
      hipLaunchKernelGGL(k_contract_fp64<false>, dim3(w->n_walkers, 2), dim3(256), om, S->stream,
                         S->M, S->nup, S->ndn, S->G, S->Lh, at<cd>(ws, L.thetaT), w->weight,
                         at<cd>(ws, L.tpart), at<cd>(ws, L.exch));
    }
    HIPCHK(hipGetLastError());
  } else {
    Timer tm(S, KG_CONTRACT);
    HIPCHK(mfma_contract(S->mt, S->stream, w->n_walkers, S->n_det, S->G, at<void>(ws, L.thetaP),
                         w->weight, at<cd>(ws, L.tpart), at<cd>(ws, L.exch), S->tile));
  }
  return AFQMC_OK;
}

// After the contraction: the precision guard's FP64 pass and the energy assembly.
int launch_guard_assemble(afqmc_sys_s* S, const afqmc_walkers* w, const WsLayout& L,
                          bool in_step) {
  void* ws = w->workspace;
  if (S->mt.enabled && S->guard_on) {
    // walkers far from the trial (large Theta) again in FP64, over the partial sums of the
    // low-precision pass: of a listed walker, the spins whose max |Theta| exceeds the threshold
    Timer tm(S, KG_GUARD);
    hipLaunchKernelGGL(k_guard_list, dim3(1), dim3(1024), 0, S->stream, w->n_walkers, S->n_det,
                       S->guard, w->weight, (const double*)at<double>(ws, L.thmax),
                       at<int>(ws, L.glist), at<int>(ws, L.gcount),
                       in_step ? S->capcount : nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(mfma_contract(S->mt64, S->stream, w->n_walkers, S->n_det, S->G,
                         at<void>(ws, L.thetaP64), w->weight, at<cd>(ws, L.tpart),
                         at<cd>(ws, L.exch), TILE_DEFAULT, at<int>(ws, L.glist),
                         at<int>(ws, L.gcount), (const double*)at<double>(ws, L.thmax),
                         S->guard));
  }
  if (S->multi) {
    Timer tm(S, KG_ASSEMBLE);
    hipLaunchKernelGGL(k_energy_assemble_multi, dim3(w->n_walkers), dim3(256), 0, S->stream, S->G,
                       S->n_det, S->h0, (double)S->sf, S->coef, at<cd>(ws, L.tpart),
                       at<cd>(ws, L.exch), at<cd>(ws, L.e1), at<cd>(ws, L.logdet),
                       at<unsigned>(ws, L.wflag), w->weight, 1, at<cd>(ws, L.tcur),
                       at<cd>(ws, L.enew), at<cd>(ws, L.ldc), at<unsigned>(ws, L.wflc));
    HIPCHK(hipGetLastError());
  } else {
    Timer tm(S, KG_ASSEMBLE);
    hipLaunchKernelGGL(k_energy_assemble, dim3(w->n_walkers), dim3(256), 0, S->stream, S->G, S->h0,
                       (double)S->sf,
                       at<cd>(ws, L.tpart), at<cd>(ws, L.exch), at<cd>(ws, L.e1), w->weight, 1,
                       at<cd>(ws, L.tcur), at<cd>(ws, L.enew));
    HIPCHK(hipGetLastError());
  }
  return AFQMC_OK;
}

int launch_contract(afqmc_sys_s* S, const afqmc_walkers* w, const WsLayout& L, bool in_step) {
  const int rc = launch_contraction(S, w, L);
  return rc ? rc : launch_guard_assemble(S, w, L, in_step);
}

int do_measure(afqmc_sys_s* S, afqmc_walkers* w) {
  const WsLayout L = layout(S, (size_t)w->n_walkers);
  void* ws = w->workspace;
  hipLaunchKernelGGL(k_step_set, dim3(1), dim3(1), 0, S->stream, at<int64_t>(ws, L.dstep), w->step);
  int rc = launch_overlap(S, w, L, 1);
  if (rc) return rc;
  rc = launch_contract(S, w, L, false);
  if (rc) return rc;
  hipLaunchKernelGGL(k_measure_finish, dim3((w->n_walkers + 255) / 256), dim3(256), 0, S->stream,
                     w->n_walkers, (double)S->sf, at<cd>(ws, S->multi ? L.ldc : L.logdet),
                     at<unsigned>(ws, S->multi ? L.wflc : L.wflag),
                     at<cd>(ws, L.enew), w->weight, w->arg_ovlp, w->log_ovlp, (cd*)w->e_loc,
                     S->status);
  HIPCHK(hipGetLastError());
  return AFQMC_OK;
}

int launch_fields(afqmc_sys_s* S, const afqmc_walkers* w, const afqmc_fields* f, const WsLayout& L,
                  double* xout, const int64_t* dstep = nullptr) {
  Timer tm(S, KG_FIELDS);
  const int nblk = (S->G + 3) / 4;
  const long n = (long)w->n_walkers * nblk;
  if (n == 0) return AFQMC_OK;
  void* ws = w->workspace;
  hipLaunchKernelGGL(k_fields, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, S->stream,
                     w->n_walkers, S->G, S->s, S->p.fb_cap, at<cd>(ws, L.tcur), w->weight,
                     w->walker_id, f->seed, f->job_id, w->step, dstep, f->x, at<cd>(ws, L.y), xout,
                     S->status,
                     ((S->p.flags & (AFQMC_FLAG_HYBRID | AFQMC_FLAG_FREE_PROJECTION)) && !xout)
                         ? at<cd>(ws, L.fbterm) : nullptr,
                     S->lbar,
                     ((S->p.flags & AFQMC_FLAG_MEAN_FIELD) && !xout) ? at<cd>(ws, L.mfterm) : nullptr,
                     xout ? nullptr : S->capcount);
  HIPCHK(hipGetLastError());
  return AFQMC_OK;
}

}  // namespace

extern "C" {

const char* afqmc_error_string(int code) {
  switch (code) {
    case AFQMC_OK: return "ok";
    case AFQMC_E_ARG: return "invalid argument";
    case AFQMC_E_UNSUPPORTED: return "unsupported precision or size";
    case AFQMC_E_SINGULAR: return "trial overlap matrix is singular";
    case AFQMC_E_NOMEM: return "out of device memory or workspace too small";
    case AFQMC_E_HIP: return "HIP runtime error";
    case AFQMC_E_NUMERIC: return "no live walker or non-finite estimator";
    case AFQMC_E_STATE: return "call out of order";
    default: return "unknown error";
  }
}

}  // extern "C"

namespace {

// Threshold of the precision guard: afqmc_params.theta_guard, NaN -> the precision's default.
double guard_threshold(const afqmc_params* p) {
  if (!std::isnan(p->theta_guard)) return p->theta_guard;
  return p->precision == AFQMC_BF16X3 ? 0.75 : 4.0;
}

// Setup of a trial with n_det determinants; coeffs == nullptr is the single-determinant trial
// of afqmc_setup.  phi_up / phi_dn hold n_det blocks [M][n_up] / [M][n_dn], the leading first.
int setup_impl(const afqmc_params* p, double h0, const double* h1, const double* L_chol, int n_det,
               const double* coeffs, const double* phi_up, const double* phi_dn, void* stream,
               afqmc_sys* out) {
  if (!p || !h1 || !out) return AFQMC_E_ARG;
  *out = nullptr;
  const int M = p->M, nup = p->n_up, ndn = p->n_dn, G = p->n_chol;
  const bool multi = coeffs != nullptr;
  if (n_det < 1 || n_det > AFQMC_MAX_DETS || (!multi && n_det != 1)) return AFQMC_E_ARG;
  if (multi)
    for (int i = 0; i < 2 * n_det; ++i)
      if (!std::isfinite(coeffs[i])) return AFQMC_E_ARG;
  if (M < 1 || nup < 0 || ndn < 0 || nup > M || ndn > M || nup + ndn < 1 || G < 0)
    return AFQMC_E_ARG;
  if (!(p->dtau > 0.0) || p->n_taylor < 1 || p->n_taylor > 20 || p->qr_period < 0 ||
      p->pop_period < 0 || !(p->el_cap_C > 0.0) || !(p->fb_cap > 0.0) || p->n_growth < 0 ||
      !(std::isnan(p->theta_guard) || p->theta_guard > 0.0))
    return AFQMC_E_ARG;
  const uint32_t known = AFQMC_FLAG_HYBRID | AFQMC_FLAG_FREE_PROJECTION | AFQMC_FLAG_MEAN_FIELD |
                         AFQMC_FLAG_CLOSED_SHELL;
  if ((p->flags & ~known) != 0 ||
      (p->flags & (AFQMC_FLAG_HYBRID | AFQMC_FLAG_FREE_PROJECTION)) ==
          (AFQMC_FLAG_HYBRID | AFQMC_FLAG_FREE_PROJECTION))
    return AFQMC_E_ARG;
  if (p->flags & AFQMC_FLAG_CLOSED_SHELL) {
    if (nup != ndn || nup == 0) return AFQMC_E_ARG;
    for (int d = 0; d < n_det; ++d)
      if (memcmp(phi_up + (size_t)d * M * nup, phi_dn + (size_t)d * M * ndn,
                 sizeof(double) * (size_t)M * nup) != 0)
        return AFQMC_E_ARG;
  }
  if ((G > 0 && !L_chol) || (nup > 0 && !phi_up) || (ndn > 0 && !phi_dn)) return AFQMC_E_ARG;
  if (p->precision < AFQMC_FP64 || p->precision > AFQMC_BF16X3) return AFQMC_E_UNSUPPORTED;
  if (std::max(nup, ndn) > 64) return AFQMC_E_UNSUPPORTED;
  // symmetry checks
  double hmax = 0.0, hasym = 0.0;
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) {
      hmax = fmax(hmax, fabs(h1[(size_t)i * M + j]));
      hasym = fmax(hasym, fabs(h1[(size_t)i * M + j] - h1[(size_t)j * M + i]));
      if (!std::isfinite(h1[(size_t)i * M + j])) return AFQMC_E_ARG;
    }
  if (hasym > 1e-12 * fmax(1.0, hmax)) return AFQMC_E_ARG;
  for (int g = 0; g < G; ++g) {
    const double* Lg = L_chol + (size_t)g * M * M;
    double lmax = 0.0, lasym = 0.0;
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        if (!std::isfinite(Lg[(size_t)i * M + j])) return AFQMC_E_ARG;
        lmax = fmax(lmax, fabs(Lg[(size_t)i * M + j]));
        lasym = fmax(lasym, fabs(Lg[(size_t)i * M + j] - Lg[(size_t)j * M + i]));
      }
    if (lasym > 1e-12 * fmax(1.0, lmax)) return AFQMC_E_ARG;
  }

  afqmc_sys_s* S = new (std::nothrow) afqmc_sys_s();
  if (!S) return AFQMC_E_NOMEM;
  S->p = *p;
  S->M = M;
  S->nup = nup;
  S->ndn = ndn;
  S->ntot = nup + ndn;
  S->G = G;
  S->h0 = h0;
  S->s = sqrt(p->dtau);
  S->stream = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetDevice(&S->device);
  const int nt = S->ntot;

  // v0 = h1 - 1/2 sum_g L^g L^g  (eq:mcd1); per-thread partial sums over g, then reduced
  std::vector<double> v0(h1, h1 + (size_t)M * M);
  {
    const int nthr = setup_threads(G);
    std::vector<std::vector<double>> part(nthr, std::vector<double>((size_t)M * M, 0.0));
    parallel_for(G, [&](int g, int t) {
      const double* Lg = L_chol + (size_t)g * M * M;
      double* acc = part[t].data();
      for (int i = 0; i < M; ++i)
        for (int k = 0; k < M; ++k) {
          const double a = 0.5 * Lg[(size_t)i * M + k];
          if (a == 0.0) continue;
          const double* row = Lg + (size_t)k * M;
          double* dst = acc + (size_t)i * M;
          for (int j = 0; j < M; ++j) dst[j] += a * row[j];
        }
    });
    for (int t = 0; t < nthr; ++t)
      for (size_t e = 0; e < v0.size(); ++e) v0[e] -= part[t][e];
  }
  for (int i = 0; i < M; ++i)
    for (int j = i + 1; j < M; ++j) {
      const double v = 0.5 * (v0[(size_t)i * M + j] + v0[(size_t)j * M + i]);
      v0[(size_t)i * M + j] = v0[(size_t)j * M + i] = v;
    }

  // Trial orbitals as rows: V[d][c][p] = (V_{d,s})_{p, c'}
  std::vector<double> Vr((size_t)n_det * nt * M);
  for (int d = 0; d < n_det; ++d) {
    const double* pu = phi_up + (size_t)d * M * nup;
    const double* pd = phi_dn + (size_t)d * M * ndn;
    double* vd = Vr.data() + (size_t)d * nt * M;
    for (int c = 0; c < nup; ++c)
      for (int q = 0; q < M; ++q) vd[(size_t)c * M + q] = pu[(size_t)q * nup + c];
    for (int c = 0; c < ndn; ++c)
      for (int q = 0; q < M; ++q) vd[(size_t)(nup + c) * M + q] = pd[(size_t)q * ndn + c];
  }
  // Half rotation (eq:precomputing2) per determinant:
  // Lh[d][g][c][q] = sum_p V[d][c][p] L^g_pq; ht[d][c][q] = sum_p V[d][c][p] h_pq
  std::vector<double> Lh((size_t)n_det * G * nt * M, 0.0), ht((size_t)n_det * nt * M, 0.0);
  parallel_for(n_det * G, [&](int dg, int) {
    const int d = dg / (G > 0 ? G : 1), g = dg % (G > 0 ? G : 1);
    const double* vd = Vr.data() + (size_t)d * nt * M;
    const double* Lg = L_chol + (size_t)g * M * M;
    for (int c = 0; c < nt; ++c) {
      double* dst = Lh.data() + (((size_t)d * G + g) * nt + c) * M;
      const double* vc = vd + (size_t)c * M;
      for (int q = 0; q < M; ++q) {
        const double a = vc[q];
        if (a == 0.0) continue;
        const double* row = Lg + (size_t)q * M;
        for (int j = 0; j < M; ++j) dst[j] += a * row[j];
      }
    }
  });
  for (int d = 0; d < n_det; ++d) {
    const double* vd = Vr.data() + (size_t)d * nt * M;
    double* hd = ht.data() + (size_t)d * nt * M;
    for (int c = 0; c < nt; ++c)
      for (int q = 0; q < M; ++q) {
        const double a = vd[(size_t)c * M + q];
        for (int j = 0; j < M; ++j) hd[(size_t)c * M + j] += a * h1[(size_t)q * M + j];
      }
  }

  // E_HF = E_L(Phi_T, Phi_T): Theta_s = V_s (V_s^T V_s)^{-1} (real), then eq:localenergy3;
  // tvec[g] = <L_g>_T are the trial's traces.  A multi-determinant trial takes both from its
  // leading determinant (the first block of Vr, Lh, ht).
  std::vector<double> tvec;
  {
    std::vector<double> th((size_t)nt * M, 0.0);  // rows of Theta^T
    for (int s = 0; s < 2; ++s) {
      const int N = s == 0 ? nup : ndn, off = s == 0 ? 0 : nup;
      if (N == 0) continue;
      std::vector<double> T((size_t)N * N, 0.0);
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          double acc = 0.0;
          for (int q = 0; q < M; ++q) acc += Vr[(size_t)(off + i) * M + q] * Vr[(size_t)(off + j) * M + q];
          T[(size_t)i * N + j] = acc;
        }
      if (!host_inverse(T, N)) {
        delete S;
        return AFQMC_E_SINGULAR;
      }
      // Theta = V T^{-1}: Theta^T[c][q] = sum_i Tinv[i][c] V[i][q]
      for (int c = 0; c < N; ++c)
        for (int q = 0; q < M; ++q) {
          double acc = 0.0;
          for (int i = 0; i < N; ++i) acc += T[(size_t)i * N + c] * Vr[(size_t)(off + i) * M + q];
          th[(size_t)(off + c) * M + q] = acc;
        }
    }
    double e1 = 0.0, jsum = 0.0, xsum = 0.0;
    for (int c = 0; c < nt; ++c)
      for (int q = 0; q < M; ++q) e1 += ht[(size_t)c * M + q] * th[(size_t)c * M + q];
    tvec.assign((size_t)G, 0.0);
    std::vector<double> xg((size_t)G, 0.0);
    parallel_for(G, [&](int g, int) {
      std::vector<double> om;
      double t = 0.0, x = 0.0;
      for (int s = 0; s < 2; ++s) {
        const int N = s == 0 ? nup : ndn, off = s == 0 ? 0 : nup;
        om.assign((size_t)N * N, 0.0);
        for (int r = 0; r < N; ++r)
          for (int c = 0; c < N; ++c) {
            double acc = 0.0;
            const double* lr = Lh.data() + ((size_t)g * nt + off + r) * M;
            const double* tc = th.data() + (size_t)(off + c) * M;
            for (int q = 0; q < M; ++q) acc += lr[q] * tc[q];
            om[(size_t)r * N + c] = acc;
          }
        for (int r = 0; r < N; ++r) {
          t += om[(size_t)r * N + r];
          for (int c = 0; c < N; ++c) x += om[(size_t)r * N + c] * om[(size_t)c * N + r];
        }
      }
      tvec[g] = t;
      xg[g] = x;
    });
    for (int g = 0; g < G; ++g) {   // fixed order
      jsum += tvec[g] * tvec[g];
      xsum += xg[g];
    }
    S->e_hf = h0 + e1 + 0.5 * (jsum - xsum);
  }
  S->e_trial = std::isnan(p->e_trial) ? S->e_hf : p->e_trial;

  // Mean-field subtraction (Sec. II.B.3): v0' = v0 + sum_g lbar_g L^g, H0' = H0 - 1/2 sum lbar^2.
  std::vector<double> lb((size_t)(G > 0 ? G : 1), 0.0);
  S->h0p = h0;
  if (p->flags & AFQMC_FLAG_MEAN_FIELD) {
    for (int g = 0; g < G; ++g) {
      lb[g] = tvec[g];
      S->h0p -= 0.5 * tvec[g] * tvec[g];
      const double* Lg = L_chol + (size_t)g * M * M;
      for (size_t e = 0; e < (size_t)M * M; ++e) v0[e] += tvec[g] * Lg[e];
    }
    for (int i = 0; i < M; ++i)
      for (int j = i + 1; j < M; ++j) {
        const double v = 0.5 * (v0[(size_t)i * M + j] + v0[(size_t)j * M + i]);
        v0[(size_t)i * M + j] = v0[(size_t)j * M + i] = v;
      }
  }
  std::vector<double> Eh;
  host_expm_sym(v0, M, -0.5 * p->dtau, Eh);

  // Closed shell: keep only the up block; spin-summed quantities are counted twice.
  int nup_i = nup, ndn_i = ndn;
  if (p->flags & AFQMC_FLAG_CLOSED_SHELL) {
    std::vector<double> Lh1((size_t)n_det * G * nup * M), ht1((size_t)n_det * nup * M),
        V1((size_t)n_det * nup * M);
    for (int d = 0; d < n_det; ++d) {
      for (int g = 0; g < G; ++g)
        memcpy(Lh1.data() + ((size_t)d * G + g) * nup * M, Lh.data() + ((size_t)d * G + g) * nt * M,
               sizeof(double) * (size_t)nup * M);
      memcpy(ht1.data() + (size_t)d * nup * M, ht.data() + (size_t)d * nt * M,
             sizeof(double) * (size_t)nup * M);
      memcpy(V1.data() + (size_t)d * nup * M, Vr.data() + (size_t)d * nt * M,
             sizeof(double) * (size_t)nup * M);
    }
    Lh.swap(Lh1);
    ht.swap(ht1);
    Vr.swap(V1);
    ndn_i = 0;
    S->ndn = 0;
    S->ntot = nup;
    S->sf = 2;
  }

  int rc;
  if ((rc = dev_upload(S, &S->Eh, Eh.data(), (size_t)M * M)) ||
      (rc = dev_upload(S, &S->V, Vr.data(), Vr.size())) ||
      (rc = dev_upload(S, &S->lbar, lb.data(), lb.size())) ||
      (rc = dev_upload(S, &S->Lh, Lh.data(), Lh.size())) ||
      (rc = dev_upload(S, &S->ht, ht.data(), ht.size())) ||
      (rc = dev_upload<unsigned>(S, &S->status, nullptr, 1)) ||
      (rc = dev_upload<unsigned long long>(S, &S->capcount, nullptr, CAP_COUNT))) {
    free_sys(S);
    return rc;
  }
  if (hipMemset(S->status, 0, sizeof(unsigned)) != hipSuccess ||
      hipMemset(S->capcount, 0, CAP_COUNT * sizeof(unsigned long long)) != hipSuccess) {
    free_sys(S);
    return AFQMC_E_HIP;
  }
  // packed pairs (q M + p, p M + q), p <= q, of the symmetric FP64 A-build; FP64 packed L^T
  if (p->precision == AFQMC_FP64) {
    const size_t MMh = (size_t)M * (M + 1) / 2;
    const std::vector<std::pair<int, int>> order = pair_order(M);
    std::vector<int> pairs(2 * MMh);
    for (size_t k = 0; k < MMh; ++k) {
      const int q = order[k].first, pp = order[k].second;
      pairs[2 * k] = q * M + pp;
      pairs[2 * k + 1] = pp * M + q;
    }
    if ((rc = dev_upload(S, &S->abpairs, pairs.data(), pairs.size()))) {
      free_sys(S);
      return rc;
    }
    S->Gp64 = ((G + 15) / 16) * 16;
    std::vector<double> lt(MMh * (S->Gp64 > 0 ? S->Gp64 : 1), 0.0);
    for (size_t k = 0; k < MMh; ++k)
      for (int g = 0; g < G; ++g)
        lt[k * S->Gp64 + g] =
            L_chol[(size_t)g * M * M + (size_t)order[k].first * M + order[k].second];
    if ((rc = dev_upload(S, &S->Lt64, lt.data(), lt.size()))) {
      free_sys(S);
      return rc;
    }
  }
  if (multi) {
    S->multi = true;
    S->n_det = n_det;
    if ((rc = dev_upload(S, &S->coef, coeffs, (size_t)2 * n_det))) {
      free_sys(S);
      return rc;
    }
  }
  {
    // MFMA contraction tables; the plain FP64 single-determinant path falls back to the
    // VALU contraction where no MFMA kernel covers the shape.  The mixed-precision modes and
    // the multi-determinant trial need the MFMA kernels.
    rc = mfma_build_tables(S->mt, p->precision, M, nup_i, ndn_i, G, Lh.data(), n_det);
    if (rc == AFQMC_E_UNSUPPORTED && p->precision == AFQMC_FP64 && !multi) rc = AFQMC_OK;
    if (rc != AFQMC_OK) {
      free_sys(S);
      return rc;
    }
    if (S->mt.enabled) S->device_bytes += S->mt.bytes;
    // precision guard of the mixed modes: an FP64 copy of the tables for the walkers redone
    // in FP64 (the FP64 MFMA contraction covers N <= 32, M <= 128)
    const double guard = guard_threshold(p);
    if (p->precision != AFQMC_FP64 && std::isfinite(guard) && S->mt.enabled && !S->mt.wide) {
      rc = mfma_build_tables(S->mt64, AFQMC_FP64, M, nup_i, ndn_i, G, Lh.data(), n_det);
      if (rc != AFQMC_OK || S->mt64.NP != S->mt.NP || S->mt64.KP != S->mt.KP) {
        free_sys(S);
        return rc != AFQMC_OK ? rc : AFQMC_E_UNSUPPORTED;
      }
      S->device_bytes += S->mt64.bytes;
      S->guard_on = true;
      S->guard = guard;
    }
  }
  // FP32 A-build and propagation in the mixed-precision modes: k_propagate_f32 where it
  // covers the shape (M <= 128, N_up + N_dn <= 64), else k_propagate_f32_wide (M <= 224,
  // up to 64 orbitals per spin).
  if (p->precision != AFQMC_FP64 && M <= WIDE_KMAX && std::max(nup_i, ndn_i) <= 64) {
    S->prop_wide = M > MFMA_KMAX || S->ntot > 64;
    S->f32_prop = true;
    S->Gp = ((G + 31) / 32) * 32;
    // one row per entry of the block-packed A (L^g is symmetric; rows past M stay zero)
    const size_t MA = (size_t)apk_size(M);
    std::vector<float> lt(MA * (S->Gp > 0 ? S->Gp : 1), 0.0f), eh((size_t)M * M);
    for (size_t k = 0; k < MA; ++k) {
      int q, pp;
      apk_entry((int)k, q, pp);
      if (q < M && pp < M)
        for (int g = 0; g < G; ++g)
          lt[k * S->Gp + g] = (float)L_chol[(size_t)g * M * M + (size_t)q * M + pp];
    }
    for (size_t e = 0; e < eh.size(); ++e) eh[e] = (float)Eh[e];
    if ((rc = dev_upload(S, &S->Lt32, lt.data(), lt.size())) ||
        (rc = dev_upload(S, &S->Eh32, eh.data(), eh.size()))) {
      free_sys(S);
      return rc;
    }
  }
  *out = S;
  return AFQMC_OK;
}

}  // namespace

extern "C" {

int afqmc_setup(const afqmc_params* p, double h0, const double* h1, const double* L_chol,
                const double* phi_up, const double* phi_dn, void* stream, afqmc_sys* out) {
  return setup_impl(p, h0, h1, L_chol, 1, nullptr, phi_up, phi_dn, stream, out);
}

int afqmc_setup_multidet(const afqmc_params* p, double h0, const double* h1, const double* L_chol,
                         int32_t n_det, const double* coeffs, const double* phi_up,
                         const double* phi_dn, void* stream, afqmc_sys* out) {
  if (!coeffs) return AFQMC_E_ARG;
  return setup_impl(p, h0, h1, L_chol, n_det, coeffs, phi_up, phi_dn, stream, out);
}

int afqmc_workspace_bytes(afqmc_sys s, int32_t n_walkers, size_t* bytes) {
  if (!s || n_walkers < 1 || !bytes) return AFQMC_E_ARG;
  *bytes = layout(s, (size_t)n_walkers).total;
  return AFQMC_OK;
}

int afqmc_get_info(afqmc_sys s, afqmc_info* info) {
  if (!s || !info) return AFQMC_E_ARG;
  info->e_trial = s->e_trial;
  info->e_hf = s->e_hf;
  info->device_bytes = s->device_bytes;
  return AFQMC_OK;
}

int afqmc_walkers_init(afqmc_sys s, afqmc_walkers* w) {
  if (!s) return AFQMC_E_ARG;
  int rc = check_walkers(s, w);
  if (rc) return rc;
  hipLaunchKernelGGL(k_init_walkers, dim3(w->n_walkers), dim3(256), 0, s->stream, w->n_walkers,
                     s->ntot * s->M, s->V, (cd*)w->U, w->weight, w->walker_id, w->phase);
  const WsLayout L = layout(s, (size_t)w->n_walkers);
  hipLaunchKernelGGL(k_growth_init, dim3(1), dim3(64), 0, s->stream,
                     at<double>(w->workspace, L.growth), s->e_trial);
  HIPCHK(hipGetLastError());
  w->step = 0;
  return do_measure(s, w);   // also sets the device step counter
}

int afqmc_measure(afqmc_sys s, afqmc_walkers* w) {
  if (!s) return AFQMC_E_ARG;
  int rc = check_walkers(s, w);
  if (rc) return rc;
  return do_measure(s, w);
}

int afqmc_fields_draw(afqmc_sys s, const afqmc_walkers* w, const afqmc_fields* f, double* x_out) {
  if (!s || !f || !x_out) return AFQMC_E_ARG;
  int rc = check_walkers(s, w);
  if (rc) return rc;
  const WsLayout L = layout(s, (size_t)w->n_walkers);
  return launch_fields(s, w, f, L, x_out);
}

}  // extern "C"

namespace {

// Steps k < n_growth of a phaseless mode form the growth phase (App. B.1, B.2).
bool in_growth_phase(const afqmc_sys_s* s, int64_t k) {
  return !(s->p.flags & AFQMC_FLAG_FREE_PROJECTION) && s->p.n_growth > 0 && k < s->p.n_growth;
}

// One step of the random walk (Sec. III.E) enqueued on s->stream, in three parts: everything
// up to the new overlaps (step_pre), the local-energy contraction, and the rest (step_post).
// With `graph` the step number is read on the device from the workspace counter (so that a
// captured graph can be replayed) and the counter is advanced at the end; otherwise the host
// value is used and the counter is set to it.
int step_pre(afqmc_sys_s* s, afqmc_walkers* w, const afqmc_fields* f, bool graph) {
  const WsLayout L = layout(s, (size_t)w->n_walkers);
  void* ws = w->workspace;
  const int nw = w->n_walkers, M = s->M, nt = s->ntot;
  const int64_t k = w->step;
  int64_t* dstep = at<int64_t>(ws, L.dstep);
  int rc;
  // 1. fields and force bias
  if ((rc = launch_fields(s, w, f, L, nullptr, graph ? dstep : nullptr))) return rc;
  // 2-3. propagator exponent A and propagation U <- E_h T_n(A) E_h U
  if (s->f32_prop) {
    float* Are = at<float>(ws, L.A);
    float* Aim = Are + (size_t)nw * apk_size(M);
    if (s->G > 0) {
      Timer tm(s, KG_ABUILD);
      const size_t ne = (size_t)nw * s->Gp;
      hipLaunchKernelGGL(k_y_to_f32, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s->stream, nw,
                         s->G, s->Gp, at<cd>(ws, L.y), at<float>(ws, L.y32));
      const int MA = apk_size(M);
      const int cb = abuild_cb(2 * nw, MA);
      dim3 grid((2 * nw + AB_BM - 1) / AB_BM, (MA + 16 * cb - 1) / (16 * cb));
#define ABUILD(CBV)                                                                              \
  case CBV:                                                                                      \
    hipLaunchKernelGGL(k_abuild_f32<CBV>, grid, dim3(256), 0, s->stream, 2 * nw, MA, s->Gp,      \
                       (float)s->s, at<float>(ws, L.y32), s->Lt32, Are, Aim);                    \
    break;
      switch (cb) {
        ABUILD(17) ABUILD(16) ABUILD(12) ABUILD(8) ABUILD(4)
        default: return AFQMC_E_UNSUPPORTED;
      }
#undef ABUILD
      HIPCHK(hipGetLastError());
    }
    if (s->prop_wide) {
      Timer tm(s, KG_PROP);
      const int Kp = ((M + 15) / 16) * 16;
      const size_t shm = (size_t)2 * 64 * (Kp + 4) * 4;
#define PROPW(NKCV)                                                                            \
  case NKCV:                                                                                   \
    (void)hipFuncSetAttribute((const void*)k_propagate_f32_wide<NKCV>,                         \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);           \
    hipLaunchKernelGGL(k_propagate_f32_wide<NKCV>, dim3(nw, 2), dim3(64 * NKCV), shm, s->stream, \
                       M, s->nup, s->ndn, Kp, s->G > 0 ? s->p.n_taylor : 0, s->Eh32, Are, Aim, \
                       (cd*)w->U, w->weight);                                                  \
    break;
      switch (Kp / 16) {
        PROPW(1) PROPW(2) PROPW(3) PROPW(4) PROPW(5) PROPW(6) PROPW(7)
        PROPW(8) PROPW(9) PROPW(10) PROPW(11) PROPW(12) PROPW(13) PROPW(14)
        default: return AFQMC_E_UNSUPPORTED;
      }
#undef PROPW
      HIPCHK(hipGetLastError());
    } else {
      Timer tm(s, KG_PROP);
      const int Kp = ((M + 15) / 16) * 16;
      const int nrb = (nt + 15) / 16;
      if (Kp > 128 || nrb > PR_RB) return AFQMC_E_UNSUPPORTED;
      const size_t shm = (size_t)2 * 16 * nrb * (Kp + 4) * 4;
      const int nt_ = s->G > 0 ? s->p.n_taylor : 0;
      // one instantiation per (K chunks of 16, row blocks of 16)
#define PROP_KR(NKCV, NRBV)                                                                    \
  case NRBV:                                                                                   \
    (void)hipFuncSetAttribute((const void*)k_propagate_f32<NKCV, NRBV>,                        \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);           \
    hipLaunchKernelGGL((k_propagate_f32<NKCV, NRBV>), dim3(nw), dim3(64 * NKCV), shm,          \
                       s->stream, M, nt, Kp, nt_, s->Eh32, Are, Aim, (cd*)w->U, w->weight);    \
    break;
#define PROP_K(NKCV)                                                                           \
  case NKCV:                                                                                   \
    switch (nrb) { PROP_KR(NKCV, 1) PROP_KR(NKCV, 2) PROP_KR(NKCV, 3) PROP_KR(NKCV, 4) }       \
    break;
      if (nrb > 0) switch (Kp / 16) {
        PROP_K(1) PROP_K(2) PROP_K(3) PROP_K(4) PROP_K(5) PROP_K(6) PROP_K(7) PROP_K(8)
        default: return AFQMC_E_UNSUPPORTED;
      }
#undef PROP_K
#undef PROP_KR
      HIPCHK(hipGetLastError());
    }
  } else {
    if (s->G > 0) {
      Timer tm(s, KG_ABUILD);
      const int MMh = M * (M + 1) / 2;
      dim3 grid((2 * nw + AB64_B - 1) / AB64_B, (MMh + AB64_B - 1) / AB64_B);
      hipLaunchKernelGGL(k_abuild_f64mfma, grid, dim3(256), 0, s->stream, nw, s->G, MMh, M * M,
                         s->Gp64, s->s, reinterpret_cast<const double*>(at<cd>(ws, L.y)), s->Lt64,
                         reinterpret_cast<const int2*>(s->abpairs), at<cd>(ws, L.A));
      HIPCHK(hipGetLastError());
    }
    Timer tm(s, KG_PROP);
    if (M <= WIDE_KMAX && std::max(s->nup, s->ndn) <= 64) {
      // FP64 MFMA propagation, one workgroup per (walker, spin, 32-row block)
      const int Kp = ((M + 15) / 16) * 16;
      const size_t shm = (size_t)2 * 32 * (Kp + 2) * 8;
      const dim3 grid(nw, 2, (std::max(s->nup, s->ndn) + 31) / 32);
#define PROP64(NKCV)                                                                           \
  case NKCV:                                                                                   \
    (void)hipFuncSetAttribute((const void*)k_propagate_f64<NKCV>,                              \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);           \
    hipLaunchKernelGGL(k_propagate_f64<NKCV>, grid, dim3(64 * NKCV), shm, s->stream, M, s->nup,  \
                       s->ndn, Kp, s->G > 0 ? s->p.n_taylor : 0, s->Eh, at<cd>(ws, L.A),       \
                       (cd*)w->U, w->weight);                                                  \
    break;
      switch (Kp / 16) {
        PROP64(1) PROP64(2) PROP64(3) PROP64(4) PROP64(5) PROP64(6) PROP64(7)
        PROP64(8) PROP64(9) PROP64(10) PROP64(11) PROP64(12) PROP64(13) PROP64(14)
        default: return AFQMC_E_UNSUPPORTED;
      }
#undef PROP64
      HIPCHK(hipGetLastError());
    } else {
    dim3 grid((M + 63) / 64, (nt + 31) / 32, nw);
    cd* U = (cd*)w->U;
    cd* X0 = at<cd>(ws, L.X0);
    cd* X1 = at<cd>(ws, L.X1);
    cd* Y = at<cd>(ws, L.Y);
    hipLaunchKernelGGL((k_zmatmul_fp64<1, true>), grid, dim3(256), 0, s->stream, M, nt,
                       (const void*)s->Eh, U, X0, Y, 1.0, w->weight);
    if (s->G > 0) {
      for (int n = 1; n <= s->p.n_taylor; ++n) {
        const cd* in = (n % 2 == 1) ? X0 : X1;
        cd* out = (n % 2 == 1) ? X1 : X0;
        hipLaunchKernelGGL((k_zmatmul_fp64<2, false>), grid, dim3(256), 0, s->stream, M, nt,
                           (const void*)at<cd>(ws, L.A), in, out, Y, 1.0 / n, w->weight);
      }
    }
    hipLaunchKernelGGL((k_zmatmul_fp64<0, true>), grid, dim3(256), 0, s->stream, M, nt,
                       (const void*)s->Eh, Y, U, nullptr, 1.0, w->weight);
    HIPCHK(hipGetLastError());
    }
  }
  // 4. periodic re-orthonormalization
  const bool qr_due = s->p.qr_period > 0 && (k + 1) % s->p.qr_period == 0;
  if (qr_due) {
    Timer tm(s, KG_QR);
    const int nmax = std::max(s->nup, s->ndn);
    const size_t shm = (size_t)nmax * M * 16;
    if (nmax <= 32 && M <= 256) {
      // rows in registers, one barrier per orthonormalized row
      const dim3 grid(nw, 2);
      switch ((M + 63) / 64) {
        case 1: hipLaunchKernelGGL(k_mgs_reg<1>, grid, dim3(256), 0, s->stream, M, s->nup, s->ndn, (cd*)w->U, w->weight, s->status, at<double>(ws, L.logR)); break;
        case 2: hipLaunchKernelGGL(k_mgs_reg<2>, grid, dim3(256), 0, s->stream, M, s->nup, s->ndn, (cd*)w->U, w->weight, s->status, at<double>(ws, L.logR)); break;
        case 3: hipLaunchKernelGGL(k_mgs_reg<3>, grid, dim3(256), 0, s->stream, M, s->nup, s->ndn, (cd*)w->U, w->weight, s->status, at<double>(ws, L.logR)); break;
        default: hipLaunchKernelGGL(k_mgs_reg<4>, grid, dim3(256), 0, s->stream, M, s->nup, s->ndn, (cd*)w->U, w->weight, s->status, at<double>(ws, L.logR)); break;
      }
    } else if (shm <= 128 * 1024) {
      (void)hipFuncSetAttribute((const void*)k_mgs<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm);
      hipLaunchKernelGGL(k_mgs<true>, dim3(nw, 2), dim3(256), shm, s->stream, M, s->nup, s->ndn,
                         (cd*)w->U, w->weight, s->status, at<double>(ws, L.logR));
    } else {
      hipLaunchKernelGGL(k_mgs<false>, dim3(nw, 2), dim3(256), 0, s->stream, M, s->nup, s->ndn,
                         (cd*)w->U, w->weight, s->status, at<double>(ws, L.logR));
    }
    HIPCHK(hipGetLastError());
  }
  // 5. overlap and Theta of the new determinants
  return launch_overlap(s, w, L, 1);
}

int step_post(afqmc_sys_s* s, afqmc_walkers* w, const afqmc_fields* f, bool graph) {
  const WsLayout L = layout(s, (size_t)w->n_walkers);
  void* ws = w->workspace;
  const int nw = w->n_walkers, M = s->M, nt = s->ntot;
  const int64_t k = w->step;
  int64_t* dstep = at<int64_t>(ws, L.dstep);
  int rc;
  // 6. the local energy of the new determinants (after the contraction)
  if ((rc = launch_guard_assemble(s, w, L, true))) return rc;
  const bool qr_due = s->p.qr_period > 0 && (k + 1) % s->p.qr_period == 0;
  // 7. phaseless weights, with the growth-phase sums around them (App. B.1, B.2)
  const bool pop_due = s->p.pop_period > 0 && (k + 1) % s->p.pop_period == 0;
  const bool growing = in_growth_phase(s, k);
  double* growth = at<double>(ws, L.growth);
  {
    Timer tm(s, KG_WEIGHT);
    const double wmax = std::isnan(s->p.w_max) ? std::max(100.0, nw / 10.0) : s->p.w_max;
    const int mode = (s->p.flags & AFQMC_FLAG_FREE_PROJECTION) ? 2
                     : (s->p.flags & AFQMC_FLAG_HYBRID) ? 1 : 0;
    if (growing)
      hipLaunchKernelGGL(k_growth_sum, dim3(1), dim3(256), 0, s->stream, nw, 0, 0, s->p.dtau,
                         w->weight, (const cd*)w->e_loc, growth);
    hipLaunchKernelGGL(k_weights, dim3((nw + 255) / 256), dim3(256), 0, s->stream, nw, mode,
                       (double)s->sf, s->p.dtau, s->h0p, (const double*)growth,
                       sqrt(s->p.el_cap_C / s->p.dtau), wmax,
                       at<cd>(ws, s->multi ? L.ldc : L.logdet),
                       at<unsigned>(ws, s->multi ? L.wflc : L.wflag), at<cd>(ws, L.enew),
                       mode ? at<cd>(ws, L.fbterm) : nullptr,
                       (s->p.flags & AFQMC_FLAG_MEAN_FIELD) ? at<cd>(ws, L.mfterm) : nullptr,
                       (s->G + 3) / 4,
                       qr_due ? at<double>(ws, L.logR) : nullptr, w->weight, w->arg_ovlp,
                       w->log_ovlp, (cd*)w->e_loc, w->phase, s->status, s->capcount);
    if (growing)
      hipLaunchKernelGGL(k_growth_sum, dim3(1), dim3(256), 0, s->stream, nw, 1, pop_due ? 1 : 0,
                         s->p.dtau, w->weight, (const cd*)w->e_loc, growth);
    HIPCHK(hipGetLastError());
  }
  // 8. population control
  if (pop_due) {
    Timer tm(s, KG_COMB);
    const double u = f->u_comb;
    const size_t cshm = nw <= 8192 ? (size_t)nw * 8 : 0;
    hipLaunchKernelGGL(k_comb_select, dim3(1), dim3(1024), cshm, s->stream, nw, w->weight, u, f->seed,
                       f->job_id, k, graph ? dstep : nullptr, at<double>(ws, L.csum),
                       at<int>(ws, L.parent), at<double>(ws, L.wnew), s->status);
    hipLaunchKernelGGL(k_comb_snapshot, dim3(nw), dim3(256), 0, s->stream, nw, nt * M, s->G,
                       (const cd*)w->U, at<cd>(ws, L.tcur), (const cd*)w->e_loc, w->arg_ovlp,
                       w->log_ovlp, w->phase, at<cd>(ws, L.X0), at<cd>(ws, L.y), at<cd>(ws, L.enew),
                       at<double>(ws, L.asnap), at<double>(ws, L.lsnap), at<double>(ws, L.psnap));
    hipLaunchKernelGGL(k_comb_gather, dim3(nw), dim3(256), 0, s->stream, nw, nt * M, s->G,
                       at<int>(ws, L.parent), at<double>(ws, L.wnew), at<cd>(ws, L.X0),
                       at<cd>(ws, L.y), at<cd>(ws, L.enew), at<double>(ws, L.asnap),
                       at<double>(ws, L.lsnap), at<double>(ws, L.psnap), (cd*)w->U,
                       at<cd>(ws, L.tcur), (cd*)w->e_loc, w->arg_ovlp, w->log_ovlp, w->phase,
                       w->weight, w->walker_id);
    HIPCHK(hipGetLastError());
  }
  if (graph)
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, s->stream, dstep);
  else
    hipLaunchKernelGGL(k_step_set, dim3(1), dim3(1), 0, s->stream, dstep, k + 1);
  HIPCHK(hipGetLastError());
  w->step = k + 1;
  return AFQMC_OK;
}

int step_impl(afqmc_sys_s* s, afqmc_walkers* w, const afqmc_fields* f, bool graph) {
  int rc = step_pre(s, w, f, graph);
  if (rc) return rc;
  const WsLayout L = layout(s, (size_t)w->n_walkers);
  if ((rc = launch_contraction(s, w, L))) return rc;
  return step_post(s, w, f, graph);
}

}  // namespace

extern "C" {

int afqmc_step(afqmc_sys s, afqmc_walkers* w, const afqmc_fields* f) {
  if (!s || !f) return AFQMC_E_ARG;
  int rc = check_walkers(s, w);
  if (rc) return rc;
  return step_impl(s, w, f, false);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of systems stepped by one graph launch.  The step of every system is captured
// once per combination of due QR / comb phases, each system on a branch stream of its own
// (fork from and join into the batch stream), and replayed with hipGraphLaunch.
// ---------------------------------------------------------------------------
struct afqmc_batch_s {
  std::vector<afqmc_sys_s*> sys;
  std::vector<afqmc_walkers*> w;
  std::vector<afqmc_fields> f;          // seeds the graphs were captured with
  std::vector<int64_t> expected;        // host step each device counter holds
  hipStream_t stream = nullptr;         // the caller's stream (may be the null stream)
  hipStream_t cap = nullptr;            // owned stream the graphs are captured on and run on
  hipEvent_t in_ev = nullptr, out_ev = nullptr;  // order cap after / before the caller's stream
  std::vector<hipStream_t> branch;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  std::vector<std::pair<std::vector<uint8_t>, hipGraphExec_t>> graphs;
  bool have_fields = false;
};

namespace {

void batch_drop_graphs(afqmc_batch_s* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
}

void batch_free(afqmc_batch_s* b) {
  if (!b) return;
  batch_drop_graphs(b);
  for (auto st : b->branch) (void)hipStreamDestroy(st);
  for (auto ev : b->join) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->in_ev) (void)hipEventDestroy(b->in_ev);
  if (b->out_ev) (void)hipEventDestroy(b->out_ev);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

// Reports a failing HIP call on stderr when AFQMC_DEBUG is set (the return code is the API).
bool hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  if (getenv("AFQMC_DEBUG")) fprintf(stderr, "afqmc: %s: %s\n", what, hipGetErrorString(e));
  return false;
}

int batch_capture(afqmc_batch_s* b, hipGraphExec_t* exec) {
  const size_t n = b->sys.size();
  std::vector<hipStream_t> saved(n);
  std::vector<bool> timing(n);
  std::vector<int64_t> steps(n);
  if (!hip_ok(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed), "begin capture"))
    return AFQMC_E_HIP;
  int rc = AFQMC_OK;
  if (!hip_ok(hipEventRecord(b->fork, b->cap), "fork record")) rc = AFQMC_E_HIP;
  for (size_t i = 0; i < n && rc == AFQMC_OK; ++i) {
    afqmc_sys_s* S = b->sys[i];
    if (!hip_ok(hipStreamWaitEvent(b->branch[i], b->fork, 0), "fork wait")) {
      rc = AFQMC_E_HIP;
      break;
    }
    saved[i] = S->stream;
    timing[i] = S->timing;
    steps[i] = b->w[i]->step;
    S->stream = b->branch[i];
    S->timing = false;
    rc = step_impl(S, b->w[i], &b->f[i], true);
    S->stream = saved[i];
    S->timing = timing[i];
    b->w[i]->step = steps[i];   // capture executes nothing
    if (rc == AFQMC_OK && (!hip_ok(hipEventRecord(b->join[i], b->branch[i]), "join record") ||
                           !hip_ok(hipStreamWaitEvent(b->cap, b->join[i], 0), "join wait")))
      rc = AFQMC_E_HIP;
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (rc == AFQMC_OK && !hip_ok(e, "end capture")) rc = AFQMC_E_HIP;
  if (rc == AFQMC_OK && !hip_ok(hipGraphInstantiate(exec, g, nullptr, nullptr, 0), "instantiate"))
    rc = AFQMC_E_HIP;
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  return rc;
}

}  // namespace

extern "C" {

int afqmc_batch_create(int32_t n, const afqmc_sys* systems, afqmc_walkers* const* walkers,
                       void* stream, afqmc_batch* out) {
  if (!out || n < 1 || !systems || !walkers) return AFQMC_E_ARG;
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!systems[i] || !walkers[i]) return AFQMC_E_ARG;
    const int rc = check_walkers(systems[i], walkers[i]);
    if (rc) return rc;
    for (int j = 0; j < i; ++j)
      if (walkers[j] == walkers[i] || walkers[j]->workspace == walkers[i]->workspace ||
          walkers[j]->U == walkers[i]->U)
        return AFQMC_E_ARG;   // one walker population appears twice
  }
  afqmc_batch_s* b = new (std::nothrow) afqmc_batch_s();
  if (!b) return AFQMC_E_NOMEM;
  b->stream = reinterpret_cast<hipStream_t>(stream);
  for (int i = 0; i < n; ++i) {
    b->sys.push_back(systems[i]);
    b->w.push_back(walkers[i]);
    b->expected.push_back(walkers[i]->step);
  }
  b->f.resize(n);
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->in_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->out_ev, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    batch_free(b);
    return AFQMC_E_HIP;
  }
  for (int i = 0; i < n; ++i) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      batch_free(b);
      return AFQMC_E_HIP;
    }
    b->branch.push_back(st);
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      batch_free(b);
      return AFQMC_E_HIP;
    }
    b->join.push_back(ev);
  }
  // the systems' earlier work (init, measure) completes before the batch stream runs
  for (int i = 0; i < n; ++i)
    if (hipStreamSynchronize(systems[i]->stream) != hipSuccess) {
      batch_free(b);
      return AFQMC_E_HIP;
    }
  *out = b;
  return AFQMC_OK;
}

int afqmc_batch_step(afqmc_batch b, const afqmc_fields* fields) {
  if (!b || !fields) return AFQMC_E_ARG;
  const size_t n = b->sys.size();
  bool same = b->have_fields;
  for (size_t i = 0; i < n; ++i) {
    if (fields[i].x != nullptr || !std::isnan(fields[i].u_comb)) return AFQMC_E_ARG;
    if (!same || fields[i].seed != b->f[i].seed || fields[i].job_id != b->f[i].job_id) same = false;
  }
  if (!same) {
    batch_drop_graphs(b);
    for (size_t i = 0; i < n; ++i) b->f[i] = fields[i];
    b->have_fields = true;
  }
  std::vector<uint8_t> key(n);
  for (size_t i = 0; i < n; ++i) {
    const afqmc_params& p = b->sys[i]->p;
    const int64_t k = b->w[i]->step;
    key[i] = (uint8_t)((p.qr_period > 0 && (k + 1) % p.qr_period == 0 ? 1 : 0) |
                       (p.pop_period > 0 && (k + 1) % p.pop_period == 0 ? 2 : 0) |
                       (in_growth_phase(b->sys[i], k) ? 4 : 0));
  }
  hipGraphExec_t exec = nullptr;
  for (auto& g : b->graphs)
    if (g.first == key) exec = g.second;
  if (!exec) {
    const int rc = batch_capture(b, &exec);
    if (rc) return rc;
    b->graphs.emplace_back(key, exec);
  }
  // the graph runs on the owned stream, after the caller's stream's earlier work
  if (!hip_ok(hipEventRecord(b->in_ev, b->stream), "in record") ||
      !hip_ok(hipStreamWaitEvent(b->cap, b->in_ev, 0), "in wait"))
    return AFQMC_E_HIP;
  // device counters of walkers that were stepped or edited outside the batch
  for (size_t i = 0; i < n; ++i)
    if (b->w[i]->step != b->expected[i]) {
      const WsLayout L = layout(b->sys[i], (size_t)b->w[i]->n_walkers);
      hipLaunchKernelGGL(k_step_set, dim3(1), dim3(1), 0, b->cap,
                         at<int64_t>(b->w[i]->workspace, L.dstep), b->w[i]->step);
    }
  if (!hip_ok(hipGraphLaunch(exec, b->cap), "graph launch") ||
      !hip_ok(hipEventRecord(b->out_ev, b->cap), "out record") ||
      !hip_ok(hipStreamWaitEvent(b->stream, b->out_ev, 0), "out wait"))
    return AFQMC_E_HIP;
  for (size_t i = 0; i < n; ++i) {
    b->w[i]->step += 1;
    b->expected[i] = b->w[i]->step;
  }
  return AFQMC_OK;
}

int afqmc_batch_set_mode(afqmc_batch b, int32_t mode) {
  if (!b || mode < 0 || mode > 1) return AFQMC_E_ARG;
  // One launch per family of systems is not available: the host process crashed inside the
  // first batch step that captured such a graph, and no cause was found in this library, so
  // the implementation was taken out.  Mode 0 is the batch's only mode.
  return mode == 0 ? AFQMC_OK : AFQMC_E_UNSUPPORTED;
}

int afqmc_batch_destroy(afqmc_batch b) {
  if (!b) return AFQMC_E_ARG;
  (void)hipStreamSynchronize(b->cap);
  (void)hipStreamSynchronize(b->stream);
  batch_free(b);
  return AFQMC_OK;
}

int afqmc_energy(afqmc_sys s, const afqmc_walkers* w, double out[6]) {
  if (!s || !out) return AFQMC_E_ARG;
  int rc = check_walkers(s, w);
  if (rc) return rc;
  const WsLayout L = layout(s, (size_t)w->n_walkers);
  double* d = at<double>(w->workspace, L.esum);
  const double half = sqrt(s->p.el_cap_C / s->p.dtau);
  const int fp = (s->p.flags & AFQMC_FLAG_FREE_PROJECTION) ? 1 : 0;
  hipLaunchKernelGGL(k_energy_sum, dim3(1), dim3(256), 0, s->stream, w->n_walkers, fp,
                     (const double*)at<double>(w->workspace, L.growth), half, w->weight, w->phase,
                     (const cd*)w->e_loc, nullptr, d);
  HIPCHK(hipGetLastError());
  double h[6];
  unsigned st = 0;
  HIPCHK(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipMemcpyAsync(&st, s->status, sizeof(unsigned), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  for (int i = 0; i < 4; ++i) out[i] = h[i];
  out[4] = (double)st;
  out[5] = h[5];
  if (!(h[3] > 0.0) || !std::isfinite(h[0]) || !std::isfinite(h[1]) || !std::isfinite(h[2]) ||
      !std::isfinite(h[5]) || (!fp && !(h[2] > 0.0)))
    return AFQMC_E_NUMERIC;
  return AFQMC_OK;
}

int afqmc_energy_enqueue(afqmc_sys s, const afqmc_walkers* w, double* out_dev) {
  if (!s || !out_dev) return AFQMC_E_ARG;
  int rc = check_walkers(s, w);
  if (rc) return rc;
  const double half = sqrt(s->p.el_cap_C / s->p.dtau);
  const int fp = (s->p.flags & AFQMC_FLAG_FREE_PROJECTION) ? 1 : 0;
  const WsLayout L = layout(s, (size_t)w->n_walkers);
  hipLaunchKernelGGL(k_energy_sum, dim3(1), dim3(256), 0, s->stream, w->n_walkers, fp,
                     (const double*)at<double>(w->workspace, L.growth), half, w->weight, w->phase,
                     (const cd*)w->e_loc, s->status, out_dev);
  HIPCHK(hipGetLastError());
  return AFQMC_OK;
}

int afqmc_footprint_bytes(const afqmc_params* p, int32_t n_det, int32_t n_walkers,
                          size_t* system_bytes, size_t* walker_bytes) {
  if (!p || n_det < 1 || n_walkers < 1 || !system_bytes || !walker_bytes) return AFQMC_E_ARG;
  const int M = p->M, G = p->n_chol;
  if (M < 1 || p->n_up < 0 || p->n_dn < 0 || p->n_up + p->n_dn < 1 || G < 0) return AFQMC_E_ARG;
  // the shape fields setup_impl derives, on a host-only descriptor (nothing is allocated)
  afqmc_sys_s S;
  S.p = *p;
  S.M = M;
  S.G = G;
  S.nup = p->n_up;
  S.ndn = (p->flags & AFQMC_FLAG_CLOSED_SHELL) ? 0 : p->n_dn;
  S.ntot = S.nup + S.ndn;
  S.n_det = n_det;
  S.multi = n_det > 1;
  const int rc = mfma_plan(S.mt, p->precision, M, S.nup, S.ndn, G, n_det);
  if (rc == AFQMC_OK) S.mt.enabled = true;
  else if (!(p->precision == AFQMC_FP64 && n_det == 1)) return rc;
  S.f32_prop = p->precision != AFQMC_FP64 && M <= WIDE_KMAX &&
               std::max(S.nup, S.ndn) <= 64;
  if (p->precision != AFQMC_FP64 && std::isfinite(guard_threshold(p)) && S.mt.enabled &&
      !S.mt.wide && mfma_plan(S.mt64, AFQMC_FP64, M, S.nup, S.ndn, G, n_det) == AFQMC_OK) {
    S.mt64.enabled = true;
    S.guard_on = true;
  }
  S.Gp = S.f32_prop ? ((G + 31) / 32) * 32 : 0;
  const size_t nt = S.ntot, MM = (size_t)M * M, g1 = G > 0 ? G : 1;
  size_t sb = MM * 8 + n_det * nt * M * 8 + g1 * 8;          // E_h, V, lbar
  sb += (n_det * (size_t)G * nt * M > 0 ? n_det * (size_t)G * nt * M : 1) * 8;  // Lh
  sb += n_det * nt * M * 8 + 4 + CAP_COUNT * 8;              // ht, status, bound counters
  if (S.multi) sb += (size_t)2 * n_det * 8;                  // coefficients
  if (S.mt.enabled) sb += S.mt.bytes;
  if (S.guard_on) sb += S.mt64.bytes;
  const size_t MMh = (size_t)M * (M + 1) / 2;
  if (p->precision == AFQMC_FP64) sb += 2 * MMh * 4;                // pair table
  if (S.f32_prop)                                                     // packed L^T, E_h (FP32)
    sb += (size_t)apk_size(M) * (S.Gp > 0 ? S.Gp : 1) * 4 + MM * 4;
  if (p->precision == AFQMC_FP64) {                                   // packed L^T (FP64)
    const size_t gp64 = ((size_t)G + 15) / 16 * 16;
    sb += MMh * (gp64 > 0 ? gp64 : 1) * 8;
  }
  *system_bytes = sb;
  const size_t nw = (size_t)n_walkers;
  *walker_bytes = layout(&S, nw).total + 256 + nw * nt * M * 16 + nw * (8 * 4 + 16 + 8);
  S.mt.enabled = false;   // the descriptor owns no device memory
  S.mt64.enabled = false;
  return AFQMC_OK;
}

int afqmc_get_growth(afqmc_sys s, const afqmc_walkers* w, double out[2]) {
  if (!s || !out) return AFQMC_E_ARG;
  int rc = check_walkers(s, w);
  if (rc) return rc;
  const WsLayout L = layout(s, (size_t)w->n_walkers);
  double h[2];
  HIPCHK(hipMemcpyAsync(h, at<double>(w->workspace, L.growth), sizeof(h), hipMemcpyDeviceToHost,
                        s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  out[0] = h[GR_ET];
  out[1] = h[GR_EBAR];
  return AFQMC_OK;
}

int afqmc_get_bound_counts(afqmc_sys s, uint64_t out[5], int clear) {
  if (!s || !out) return AFQMC_E_ARG;
  unsigned long long h[CAP_COUNT];
  HIPCHK(hipMemcpyAsync(h, s->capcount, sizeof(h), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  for (int i = 0; i < CAP_COUNT; ++i) out[i] = (uint64_t)h[i];
  if (clear) {
    hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(64), 0, s->stream, s->capcount, CAP_COUNT);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
  }
  return AFQMC_OK;
}

int afqmc_get_status(afqmc_sys s, uint32_t* status, int clear) {
  if (!s || !status) return AFQMC_E_ARG;
  unsigned st = 0;
  HIPCHK(hipMemcpyAsync(&st, s->status, sizeof(unsigned), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  *status = st;
  if (clear) {
    HIPCHK(hipMemsetAsync(s->status, 0, sizeof(unsigned), s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
  }
  return AFQMC_OK;
}

int afqmc_kernel_timing(afqmc_sys s, int enable) {
  if (!s) return AFQMC_E_ARG;
  flush_timing(s);
  if (enable) {
    for (int i = 0; i < KG_COUNT; ++i) {
      s->acc_ms[i] = 0.0;
      s->acc_n[i] = 0;
    }
  }
  s->timing = enable != 0;
  return AFQMC_OK;
}

int afqmc_kernel_time(afqmc_sys s, int kernel, double* ms, int64_t* launches) {
  if (!s || kernel < 0 || kernel >= KG_COUNT || !ms || !launches) return AFQMC_E_ARG;
  flush_timing(s);
  *ms = s->acc_ms[kernel];
  *launches = s->acc_n[kernel];
  return AFQMC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free modified Cholesky: its workspace is this file-scope device array, one copy
// per GPU, held until the process ends.  Host code must not pass `scratch` itself to a
// kernel (in host code the name is a host-side stand-in): the device address of each GPU's
// copy comes from hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
constexpr size_t mcd_ws_bytes(size_t M) {
  return ((M * M * 8 + 255) & ~size_t(255)) + ((M * M + 255) & ~size_t(255)) +
         ((sizeof(McdState) + 255) & ~size_t(255));
}
static_assert(mcd_ws_bytes(AFQMC_MCD_NOALLOC_MAX_M) == AFQMC_MCD_NOALLOC_BYTES,
              "scratch size of the allocation-free modified Cholesky");
static __device__ __align__(256) unsigned char scratch[AFQMC_MCD_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on the first call per device).
int mcd_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return AFQMC_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return AFQMC_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return AFQMC_E_HIP;
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return AFQMC_OK;
}

// The decomposition on a workspace laid out as afqmc_mcd_workspace_bytes says: the residual
// diagonal D, the dead flags and the McdState.  k_mcd_init writes every element of the three
// that a decomposition of this M reads, so a reused workspace needs no clearing.
int mcd_run(const double* eri, int32_t M, double delta, int32_t max_vectors, double* L_out,
            int32_t* n_vectors, int32_t* converged, void* workspace, hipStream_t st) {
  const size_t MM = (size_t)M * M;
  double* D = at<double>(workspace, 0);
  unsigned char* dead = at<unsigned char>(workspace, al256(MM * 8));
  McdState* state = at<McdState>(workspace, al256(MM * 8) + al256(MM));
  hipLaunchKernelGGL(k_mcd_init, dim3((unsigned)((MM + 255) / 256)), dim3(256), 0, st, M, eri, D,
                     dead, state);
  HIPCHK(hipGetLastError());
  McdState h{};
  int n = 0;
  for (; n <= max_vectors; ++n) {
    hipLaunchKernelGGL(k_mcd_pivot, dim3(1), dim3(1024), 0, st, (int)MM, delta, n, max_vectors, D,
                       dead, state);
    if (n < max_vectors)
      hipLaunchKernelGGL(k_mcd_column, dim3((unsigned)((MM + 255) / 256)), dim3(256), 0, st, M, n,
                         eri, L_out, D, dead, state);
    HIPCHK(hipGetLastError());
    if ((n & 31) == 31 || n == max_vectors) {
      HIPCHK(hipMemcpyAsync(&h, state, sizeof(h), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (h.done) break;
    }
  }
  HIPCHK(hipMemcpyAsync(&h, state, sizeof(h), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (!h.done) return AFQMC_E_STATE;
  *n_vectors = h.count;
  if (converged) *converged = h.count < max_vectors || h.dmax < delta ? 1 : 0;
  return AFQMC_OK;
}

}  // namespace

extern "C" {

int afqmc_mcd_workspace_bytes(int32_t M, size_t* bytes) {
  if (M < 1 || !bytes) return AFQMC_E_ARG;
  const size_t MM = (size_t)M * M;
  *bytes = al256(MM * 8) + al256(MM) + al256(sizeof(McdState));
  return AFQMC_OK;
}

int afqmc_modified_cholesky(const double* eri, int32_t M, double delta, int32_t max_vectors,
                            double* L_out, int32_t* n_vectors, int32_t* converged,
                            void* workspace, size_t workspace_bytes, void* stream) {
  if (!eri || M < 1 || !(delta > 0.0) || max_vectors < 0 || (max_vectors > 0 && !L_out) ||
      !n_vectors || !workspace)
    return AFQMC_E_ARG;
  size_t need = 0;
  afqmc_mcd_workspace_bytes(M, &need);
  if (workspace_bytes < need) return AFQMC_E_NOMEM;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return AFQMC_E_ARG;
  return mcd_run(eri, M, delta, max_vectors, L_out, n_vectors, converged, workspace,
                 reinterpret_cast<hipStream_t>(stream));
}

int afqmc_modified_cholesky_noalloc(const double* eri, int32_t M, double delta,
                                    int32_t max_vectors, double* L_out, int32_t* n_vectors,
                                    int32_t* converged, void* stream) {
  if (!eri || M < 1 || !(delta > 0.0) || max_vectors < 0 || (max_vectors > 0 && !L_out) ||
      !n_vectors)
    return AFQMC_E_ARG;
  if (M > AFQMC_MCD_NOALLOC_MAX_M) return AFQMC_E_UNSUPPORTED;
  void* ws = nullptr;
  const int rc = mcd_scratch(&ws);
  if (rc) return rc;
  return mcd_run(eri, M, delta, max_vectors, L_out, n_vectors, converged, ws,
                 reinterpret_cast<hipStream_t>(stream));
}

int afqmc_mfma_peak(int32_t precision, void* out_dev, size_t out_bytes, void* hip_stream,
                    double* tflops) {
  if (!out_dev || !tflops || out_bytes < (size_t)AFQMC_MFMA_PEAK_BYTES) return AFQMC_E_ARG;
  if (precision < AFQMC_FP64 || precision > AFQMC_BF16X3) return AFQMC_E_UNSUPPORTED;
  const int kind = precision == AFQMC_FP32 ? 0 : precision == AFQMC_FP64 ? 1 : 2;
  const int per_iter = kind == 0 ? peak_mfmas_per_iter<0>() : kind == 1 ? peak_mfmas_per_iter<1>()
                                                                         : peak_mfmas_per_iter<2>();
  // as many waves as fit at once (FP64: 3 per SIMD, else 4), 49152 (BF16 98304) instructions
  // each: about 4 ms per launch at the datasheet rates (157.3, 78.6 and 2500 TFLOP/s)
  const int blocks = kind == 1 ? 3 * PEAK_MAX_BLOCKS / 4 : PEAK_MAX_BLOCKS;
  const int iters = (kind == 2 ? 98304 : 49152) / per_iter;
  hipStream_t st = (hipStream_t)hip_stream;
  double* out = (double*)out_dev;
  auto launch = [&]() {
    if (kind == 0)
      hipLaunchKernelGGL(k_mfma_peak<0>, dim3(blocks), dim3(256), 0, st, iters, out);
    else if (kind == 1)
      hipLaunchKernelGGL(k_mfma_peak<1>, dim3(blocks), dim3(256), 0, st, iters, out);
    else
      hipLaunchKernelGGL(k_mfma_peak<2>, dim3(blocks), dim3(256), 0, st, iters, out);
    return hipGetLastError();
  };
  constexpr int TIMED = 3;  // the fastest of three timed launches after an untimed one
  hipEvent_t ev[TIMED + 1] = {};
  int rc = AFQMC_OK;
  for (int i = 0; i <= TIMED && rc == AFQMC_OK; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) rc = AFQMC_E_HIP;
  if (rc == AFQMC_OK && launch() != hipSuccess) rc = AFQMC_E_HIP;
  for (int i = 0; i <= TIMED && rc == AFQMC_OK; ++i) {
    if (hipEventRecord(ev[i], st) != hipSuccess) rc = AFQMC_E_HIP;
    if (rc == AFQMC_OK && i < TIMED && launch() != hipSuccess) rc = AFQMC_E_HIP;
  }
  float best = 0.f;
  if (rc == AFQMC_OK && hipEventSynchronize(ev[TIMED]) != hipSuccess) rc = AFQMC_E_HIP;
  for (int i = 0; i < TIMED && rc == AFQMC_OK; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) rc = AFQMC_E_HIP;
    else if (best == 0.f || ms < best) best = ms;
  }
  for (int i = 0; i <= TIMED; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  if (rc) return rc;
  const double flops = (double)blocks * 4 * per_iter * (double)iters * peak_flops_per_mfma(kind);
  *tflops = best > 0.f ? flops / ((double)best * 1e-3) / 1e12 : 0.0;
  return AFQMC_OK;
}

int afqmc_set_tile(afqmc_sys s, int32_t tile) {
  if (!s || tile < 0 || tile >= TILE_COUNT) return AFQMC_E_ARG;
  if (!mfma_tile_valid(s->mt, tile)) return AFQMC_E_UNSUPPORTED;
  s->tile = tile;
  return AFQMC_OK;
}

int afqmc_get_tile(afqmc_sys s, int32_t* tile) {
  if (!s || !tile) return AFQMC_E_ARG;
  *tile = s->tile;
  return AFQMC_OK;
}

}  // extern "C"

namespace {
// Shapes already tuned in this process: (device, precision, M, N_up, N_dn, G, n_det, n_walkers)
using TuneKey = std::tuple<int, int, int, int, int, int, int, int>;
std::map<TuneKey, int> g_tuned;
std::mutex g_tuned_mu;
}  // namespace

extern "C" {

int afqmc_autotune(afqmc_sys s, afqmc_walkers* w, int32_t reuse, int32_t* tile, double* ms) {
  if (!s || !tile) return AFQMC_E_ARG;
  int rc = check_walkers(s, w);
  if (rc) return rc;
  const TuneKey key{s->device, s->p.precision, s->M, s->nup, s->ndn, s->G, s->n_det, w->n_walkers};
  if (reuse) {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      s->tile = it->second;
      *tile = it->second;
      if (ms) *ms = -1.0;
      return AFQMC_OK;
    }
  }
  const WsLayout L = layout(s, (size_t)w->n_walkers);
  void* ws = w->workspace;
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return AFQMC_E_HIP;
  }
  int best = TILE_DEFAULT;
  double best_ms = 0.0;
  bool any = false;
  constexpr int REPS = 3;
  for (int t = TILE_W4; t < TILE_COUNT && rc == AFQMC_OK; ++t) {
    if (!mfma_tile_valid(s->mt, t)) continue;
    // one untimed launch, then REPS timed ones; only the workspace partial sums are written
    for (int r = 0; r <= REPS && rc == AFQMC_OK; ++r) {
      if (r == 1 && hipEventRecord(a, s->stream) != hipSuccess) rc = AFQMC_E_HIP;
      if (rc == AFQMC_OK &&
          mfma_contract(s->mt, s->stream, w->n_walkers, s->n_det, s->G, at<void>(ws, L.thetaP),
                        w->weight, at<cd>(ws, L.tpart), at<cd>(ws, L.exch), t) != hipSuccess)
        rc = AFQMC_E_HIP;
    }
    float el = 0.f;
    if (rc == AFQMC_OK && (hipEventRecord(b, s->stream) != hipSuccess ||
                           hipEventSynchronize(b) != hipSuccess ||
                           hipEventElapsedTime(&el, a, b) != hipSuccess))
      rc = AFQMC_E_HIP;
    if (rc == AFQMC_OK && (!any || el / REPS < best_ms)) {
      best = t;
      best_ms = el / REPS;
      any = true;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  s->tile = best;
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned[key] = best;
  }
  *tile = best;
  if (ms) *ms = any ? best_ms : 0.0;
  return AFQMC_OK;
}

int afqmc_destroy(afqmc_sys s) {
  if (!s) return AFQMC_E_ARG;
  (void)hipStreamSynchronize(s->stream);
  free_sys(s);
  return AFQMC_OK;
}

}  // extern "C"
