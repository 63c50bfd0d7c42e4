// MFMA form of the local-energy contraction (arXiv:1711.02242, Sec. III.D.3,
// eq:localenergy3; force-bias traces of eq:precomputing2).
//
// For every walker w, spin s and Cholesky index g:
//   Omega = Lh^g_s Theta_s     (N x N complex = real N x M times complex M x N)
//   tpart[w][s][g] = tr Omega,  exch[w][s] = sum_g tr(Omega Omega).
// Omega is never stored: it lives in MFMA accumulators for one g at a time.
//
// Mapping to CDNA4 (gfx950): one wavefront owns one walker-spin and keeps
// [Re Theta | Im Theta] (M x 2N) in registers for the whole kernel; the four
// wavefronts of a workgroup (four walkers of the same spin) stream the shared
// tiles Lh^g_s (N x M) through double-buffered LDS.  Per g the wave runs the
// MFMA chain over K = M for the Re and Im halves, then an LDS transpose gives
// every lane the partner element Omega_ji of each Omega_ij it holds.
// Per-g partial products are summed in FP32 and accumulated across g in FP64.
//
// Padding: N is padded to NP (16 or 32) and M to KP (a multiple of 32, at most
// 128) with zeros in both operands, which leaves traces and products unchanged.
//
// Precisions: FP32 operands with FP32 accumulation (v_mfma_f32_32x32x2_f32,
// v_mfma_f32_16x16x4_f32), or BF16x3: x = hi + lo with hi = bf16(x),
// lo = bf16(x - hi), and a b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b with FP32
// accumulation (v_mfma_f32_32x32x16_bf16, v_mfma_f32_16x16x32_bf16).
#pragma once

#include <stdint.h>
#include <string.h>

#include <type_traits>
#include <vector>

#include "common.hpp"

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int MFMA_KMAX = 128;   // K limit of the register-resident contraction kernels
constexpr int WIDE_KMAX = 224;   // K limit of the wide (workgroup-per-walker) kernel
// Contraction kernel variants (tile shapes) the autotuner chooses among.
enum {
  TILE_DEFAULT = 0, TILE_W4 = 1, TILE_W2 = 2, TILE_WIDE = 3, TILE_FLAT = 4, TILE_STACK = 5,
  TILE_PP = 6, TILE_BX = 7, TILE_BX8 = 8, TILE_COUNT = 9
};

struct MfmaTables {
  bool enabled = false;
  int precision = 0;  // AFQMC_FP64, AFQMC_FP32 or AFQMC_BF16X3
  int NP = 0, KP = 0, M = 0, G = 0, nup = 0, ndn = 0, n_det = 1;
  bool wide = false;   // N > 32 or M > 128 (up to 64, 224): the kernel of contract_wide.hpp
  void* Lp = nullptr;  // fp64 / fp32: [n_det][2][G][NP][KP]; bf16x3: [n_det][2][G][2 (hi, lo)][NP][KP]
  size_t bytes = 0;
};

// Round-to-nearest-even float -> bf16 bits (identical on host and device).
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan kept
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_bits_to_f32(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

inline size_t mfma_theta_bytes(const MfmaTables& t, size_t nw) {
  if (!t.enabled) return 0;
  // fp32 re/im, or bf16 re/im x hi/lo (same bytes); fp64 re/im
  return nw * (size_t)t.n_det * 2 * 2 * (size_t)t.NP * t.KP * (t.precision == AFQMC_FP64 ? 8 : 4);
}

// Shape of the tables (no allocation): NP, KP, kernel family and device bytes.
inline int mfma_plan(MfmaTables& t, int precision, int M, int nup, int ndn, int G, int n_det) {
  const int nmax = nup > ndn ? nup : ndn;
  // register-resident kernels up to N = 32, M = 128 (all precisions); beyond, up to N = 64,
  // M = 224, the wide FP32 / BF16x3 kernel
  const bool fast = nmax <= 32 && M <= MFMA_KMAX;
  const bool wide = !fast && precision != AFQMC_FP64 && nmax <= 64 && M <= WIDE_KMAX;
  if (!fast && !wide) return AFQMC_E_UNSUPPORTED;
  if (precision < AFQMC_FP64 || precision > AFQMC_BF16X3) return AFQMC_E_UNSUPPORTED;
  t.precision = precision;
  t.wide = wide;
  t.NP = nmax <= 16 ? 16 : nmax <= 32 ? 32 : nmax <= 48 ? 48 : 64;
  if (wide && t.NP < 32) t.NP = 32;
  t.KP = ((M + 31) / 32) * 32;
  t.M = M;
  t.G = G;
  t.nup = nup;
  t.ndn = ndn;
  t.n_det = n_det;
  const size_t per = (size_t)t.NP * t.KP;
  if (precision == AFQMC_FP64) t.bytes = ((size_t)n_det * 2 * G * per + 2) * sizeof(double);
  else if (precision == AFQMC_FP32) t.bytes = ((size_t)n_det * 2 * G * per + 1) * sizeof(float);
  else t.bytes = ((size_t)n_det * 2 * G * 2 * per + 2) * sizeof(uint16_t);
  return AFQMC_OK;
}

inline int mfma_build_tables(MfmaTables& t, int precision, int M, int nup, int ndn, int G,
                             const double* Lh /* host [n_det][G][nup+ndn][M] */, int n_det = 1) {
  const int prc = mfma_plan(t, precision, M, nup, ndn, G, n_det);
  if (prc != AFQMC_OK) return prc;
  const int nt = nup + ndn;
  const size_t per = (size_t)t.NP * t.KP;
  if (precision == AFQMC_FP64) {
    std::vector<double> h((size_t)n_det * 2 * G * per + 2, 0.0);
    for (int d = 0; d < n_det; ++d)
    for (int s = 0; s < 2; ++s) {
      const int N = s ? ndn : nup, off = s ? nup : 0;
      for (int g = 0; g < G; ++g)
        for (int r = 0; r < N; ++r)
          for (int p = 0; p < M; ++p)
            h[(((size_t)d * 2 + s) * G + g) * per + (size_t)r * t.KP + p] =
                Lh[(((size_t)d * G + g) * nt + off + r) * M + p];
    }
    t.bytes = h.size() * sizeof(double);
    if (hipMalloc(&t.Lp, t.bytes) != hipSuccess) return AFQMC_E_NOMEM;
    if (hipMemcpy(t.Lp, h.data(), t.bytes, hipMemcpyHostToDevice) != hipSuccess) return AFQMC_E_HIP;
  } else if (precision == AFQMC_FP32) {
    std::vector<float> h((size_t)n_det * 2 * G * per + 1, 0.0f);
    for (int d = 0; d < n_det; ++d)
    for (int s = 0; s < 2; ++s) {
      const int N = s ? ndn : nup, off = s ? nup : 0;
      for (int g = 0; g < G; ++g)
        for (int r = 0; r < N; ++r)
          for (int p = 0; p < M; ++p)
            h[(((size_t)d * 2 + s) * G + g) * per + (size_t)r * t.KP + p] =
                (float)Lh[(((size_t)d * G + g) * nt + off + r) * M + p];
    }
    t.bytes = h.size() * sizeof(float);
    if (hipMalloc(&t.Lp, t.bytes) != hipSuccess) return AFQMC_E_NOMEM;
    if (hipMemcpy(t.Lp, h.data(), t.bytes, hipMemcpyHostToDevice) != hipSuccess) return AFQMC_E_HIP;
  } else if (precision == AFQMC_BF16X3) {
    std::vector<uint16_t> h((size_t)n_det * 2 * G * 2 * per + 2, 0);
    for (int d = 0; d < n_det; ++d)
    for (int s = 0; s < 2; ++s) {
      const int N = s ? ndn : nup, off = s ? nup : 0;
      for (int g = 0; g < G; ++g)
        for (int r = 0; r < N; ++r)
          for (int p = 0; p < M; ++p) {
            const float x = (float)Lh[(((size_t)d * G + g) * nt + off + r) * M + p];
            const uint16_t hi = f32_to_bf16_bits(x);
            const uint16_t lo = f32_to_bf16_bits(x - bf16_bits_to_f32(hi));
            const size_t base = ((((size_t)d * 2 + s) * G + g) * 2) * per + (size_t)r * t.KP + p;
            h[base] = hi;
            h[base + per] = lo;
          }
    }
    t.bytes = h.size() * sizeof(uint16_t);
    if (hipMalloc(&t.Lp, t.bytes) != hipSuccess) return AFQMC_E_NOMEM;
    if (hipMemcpy(t.Lp, h.data(), t.bytes, hipMemcpyHostToDevice) != hipSuccess) return AFQMC_E_HIP;
  } else {
    return AFQMC_E_UNSUPPORTED;
  }
  t.enabled = true;
  return AFQMC_OK;
}

inline void mfma_free_tables(MfmaTables& t) {
  if (t.Lp) (void)hipFree(t.Lp);
  t.Lp = nullptr;
  t.enabled = false;
}

#include "contract_mfma.hpp"
#include "contract_wide.hpp"
#include "contract_flat.hpp"
#include "contract_pp.hpp"
#include "contract_bx.hpp"

inline size_t mfma_contract_lds_bytes(const MfmaTables& t, int wpb) {
  const bool bf = t.precision == AFQMC_BF16X3;
  const int esz = bf ? 2 : 4, planes = bf ? 2 : 1;
  const int lda = t.KP + (bf ? 8 : 4);
  const size_t tile = (size_t)t.NP * lda * esz * planes;
  return 2 * tile + (size_t)wpb * 2 * t.NP * (t.NP + 4) * 4;
}

// Compute units of the current device (queried once per device).
inline int device_cu_count() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] <= 0) {
    int n = 0;
    cus[dev] = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                       n > 0
                   ? n
                   : 256;
  }
  return cus[dev];
}

// Whether a contraction variant can run on these tables.
inline bool mfma_tile_valid(const MfmaTables& t, int tile) {
  if (!t.enabled) return false;
  if (t.precision == AFQMC_FP64) return tile == TILE_DEFAULT;
  switch (tile) {
    case TILE_DEFAULT: return true;
    case TILE_W4:
    case TILE_W2:
    case TILE_PP: return !t.wide;
    case TILE_BX:
    case TILE_BX8: return !t.wide && t.NP == 32;
    case TILE_WIDE: return t.NP >= 32 && t.KP <= WIDE_KMAX;
    case TILE_FLAT:
    case TILE_STACK: {
      if (t.KP > WIDE_KMAX || t.NP > 64) return false;
      const FlatLaunch f =
          flat_launch(t.nup, t.ndn, t.G, t.precision == AFQMC_BF16X3, tile == TILE_STACK);
      return f.ok && f.lds <= FLAT_LDS_CAP;
    }
    default: return false;
  }
}

// ---------------------------------------------------------------------------
// FP64 form of the contraction on v_mfma_f64_16x16x4_f64.
// Operand lanes: A[i][k] at lane i + 16k, B[k][j] at lane j + 16k.  Output: lane l,
// item v holds D[l/16 + 4v][l%16] (rows strided by 4 -- not the FP32 16x16 layout).
// Two wavefronts share one walker-spin: one holds Re Theta, the other Im Theta
// (M x N each, 128 VGPRs at M = 128) as the B operand for the whole kernel.  A
// workgroup of 4 waves covers two walkers of one spin.  The Lh^g tile is single-
// buffered in LDS with a register prefetch two g ahead, which keeps two
// workgroups per CU.  Per g each wave writes its Omega plane (Re or Im) to LDS;
// the Re wave then accumulates sum_ij (R_ij R_ji - I_ij I_ji) and the Im wave
// 2 sum_ij I_ij R_ji, both in FP64.  NK = K_P / 8 register chunks of K (compile time: no
// per-chunk branches); tr Omega is summed over the lanes by DPP row shifts.
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <int NP, int NK>
__global__ void __launch_bounds__(256, 2) k_contract_f64mfma(
    int nw, int G, int nup, int ndn, int KP_arg, const double* __restrict__ Lp,
    const double* __restrict__ thp, const double* __restrict__ weight, cd* __restrict__ tpart,
    cd* __restrict__ exch, const int* __restrict__ wlist, const int* __restrict__ wcount,
    const double* __restrict__ gthmax, double guard) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int NB = NP / 16;
  constexpr int NCH = NK;                     // K chunks of 8 held per lane as 4 x f64x2
  constexpr int KP = 8 * NK;                  // K_P (the launcher passes it as KP_arg)
  (void)KP_arg;
  constexpr int LDE = NP + 1;
  const int s = blockIdx.y & 1, d = blockIdx.y >> 1, n_det = gridDim.y >> 1;
  const int N = s ? ndn : nup;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int pair = wave >> 1, part = wave & 1;  // part 0: Re Theta, 1: Im Theta
  int w = blockIdx.x * 2 + pair;
  if (wlist) {
    // only the listed walkers (the precision guard): slot -> walker, workgroups past the
    // count exit at once (the count is the same for every thread of the workgroup)
    const int cnt = *wcount;
    if ((int)blockIdx.x * 2 >= cnt) return;
    w = w < cnt ? wlist[w] : -1;
  }
  const int wd = w * n_det + d;                 // (walker, determinant) slot of the outputs
  Lp += (size_t)d * 2 * G * NP * KP;
  if (N == 0) {
    if (w >= 0 && w < nw && part == 0) {
      for (int g = lane; g < G; g += 64) tpart[((size_t)wd * 2 + s) * G + g] = mkc(0.0, 0.0);
      if (lane == 0) exch[2 * wd + s] = mkc(0.0, 0.0);
    }
    return;
  }
  bool active = (w >= 0) && (w < nw) && (weight[w] > 0.0);
  // with the precision guard's per-spin maxima, of a listed walker only the spins above the
  // threshold (those whose FP64 operand the overlap kernel wrote); the others keep their sums
  if (active && wlist && gthmax) active = gthmax[2 * wd + s] > guard;
  constexpr int lda = KP + 2;
  double* At = reinterpret_cast<double*>(smem);                       // [NP][KP + 2]
  double* ep = At + (size_t)NP * lda + (size_t)pair * 2 * NP * LDE;   // this pair's planes
  double* epR = ep;
  double* epI = ep + NP * LDE;
  const int j16 = lane & 15, q = lane >> 4;

  // B operand: lane holds Theta_part[16 b + j16][8 c + 2 q + {0, 1}]
  f64x2 breg[NB][NCH];
  if (active) {
    const double* tb = thp + (((size_t)wd * 2 + s) * 2 + part) * NP * KP;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int c = 0; c < NCH; ++c)
        breg[b][c] = *reinterpret_cast<const f64x2*>(tb + (size_t)(16 * b + j16) * KP + 8 * c + 2 * q);
  }

  // tile staging: NP * KP doubles as 16-byte chunks
  constexpr int chunks_per_row = KP / 2;
  constexpr int nchunks = NP * chunks_per_row;
  constexpr int MAXCH = (nchunks + 255) / 256;   // 16-byte chunks per thread
  u32x4 pre[MAXCH];
  const double* Lbase = Lp + (size_t)s * G * NP * KP;
#define F64_GLOAD(G_)                                                                          \
  do {                                                                                         \
    const u32x4* src_ = reinterpret_cast<const u32x4*>(Lbase + (size_t)(G_) * NP * KP);        \
    _Pragma("unroll") for (int c_ = 0; c_ < MAXCH; ++c_) {                                     \
      const int ch_ = tid + c_ * 256;                                                          \
      pre[c_] = src_[ch_ < nchunks ? ch_ : 0];                                                 \
    }                                                                                          \
  } while (0)
#define F64_LSTORE()                                                                           \
  do {                                                                                         \
    _Pragma("unroll") for (int c_ = 0; c_ < MAXCH; ++c_) {                                     \
      const int ch_ = tid + c_ * 256;                                                          \
      if ((c_ + 1) * 256 <= nchunks || ch_ < nchunks) {                                        \
        const int row_ = ch_ / chunks_per_row, col_ = (ch_ % chunks_per_row) * 2;              \
        *reinterpret_cast<u32x4*>(At + (size_t)row_ * lda + col_) = pre[c_];                   \
      }                                                                                        \
    }                                                                                          \
  } while (0)

  double xacc = 0.0;
  if (G > 0) {
    F64_GLOAD(0);
    F64_LSTORE();
  }
  // every global load so far (Theta, the first tile) complete here: otherwise the waits for
  // the Theta registers land inside the g loop, where they also wait for the prefetched tiles
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  __syncthreads();
  if (G > 1) F64_GLOAD(1);
  for (int g = 0; g < G; ++g) {
    f64x4 acc[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    if (active) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        f64x2 af[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a)
          af[a] = *reinterpret_cast<const f64x2*>(At + (size_t)(16 * a + j16) * lda + 8 * c + 2 * q);
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
          for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a][e], breg[b][c][e], acc[a][b], 0, 0, 0);
      }
      // this wave's plane, column-major: element (row r, col c) at [c * LDE + r]
      double* pl = part ? epI : epR;
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            pl[(16 * b + j16) * LDE + 16 * a + q + 4 * v] = acc[a][b][v];
    }
    __syncthreads();
    if (g + 1 < G) F64_LSTORE();
    if (active) {
      double pr = 0.0;
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 16 * a + q + 4 * v, j = 16 * b + j16;
            const double mine = acc[a][b][v];
            const double Rji = epR[i * LDE + j];
            if (part == 0) {
              const double Iij = epI[j * LDE + i], Iji = epI[i * LDE + j];
              pr += mine * Rji - Iij * Iji;
            } else {
              pr += 2.0 * mine * Rji;
            }
          }
      xacc += pr;
      const int dl = lane < NP ? lane : NP - 1;
      double dg = part ? epI[dl * LDE + dl] : epR[dl * LDE + dl];
      if (lane >= NP) dg = 0.0;
      dg = NP == 32 ? dpp_half_sum(dg) : dpp_row_sum(dg);   // lane NP - 1
      if (lane == NP - 1) reinterpret_cast<double*>(tpart + ((size_t)wd * 2 + s) * G + g)[part] = dg;
    }
    F64_GLOAD(g + 2 < G ? g + 2 : G - 1);   // unconditional: the waits stay exact
    __syncthreads();
  }
#undef F64_GLOAD
#undef F64_LSTORE
  if (active) {
    xacc = wave_sum(xacc);
    if (lane == 0) reinterpret_cast<double*>(exch + 2 * wd + s)[part] = xacc;
  }
}

inline size_t mfma_f64_contract_lds_bytes(const MfmaTables& t) {
  return ((size_t)t.NP * (t.KP + 2) + (size_t)2 * 2 * t.NP * (t.NP + 1)) * 8;
}

inline hipError_t mfma_contract(const MfmaTables& t, hipStream_t st, int nw, int n_det, int G,
                                const void* thetaP, const double* weight, cd* tpart, cd* exch,
                                int tile = TILE_DEFAULT, const int* wlist = nullptr,
                                const int* wcount = nullptr, const double* gthmax = nullptr,
                                double guard = 0.0) {
  if (t.precision == AFQMC_FP64) {
    const size_t shm = mfma_f64_contract_lds_bytes(t);
    dim3 grid((nw + 1) / 2, 2 * n_det);
    // one instantiation per K chunk count (K_P = 32 .. 128 in steps of 32)
    if (t.KP % 32 != 0 || t.KP < 32 || t.KP > MFMA_KMAX) return hipErrorInvalidValue;
#define LAUNCH_F64(NPV, NKV)                                                                   \
  do {                                                                                         \
    (void)hipFuncSetAttribute((const void*)k_contract_f64mfma<NPV, NKV>,                       \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);           \
    hipLaunchKernelGGL((k_contract_f64mfma<NPV, NKV>), grid, dim3(256), shm, st, nw, G, t.nup, \
                       t.ndn, t.KP, (const double*)t.Lp, (const double*)thetaP, weight, tpart, \
                       exch, wlist, wcount, gthmax, guard);                                    \
  } while (0)
#define LAUNCH_F64_NP(NPV)                                                                     \
  do {                                                                                         \
    switch (t.KP / 8) {                                                                        \
      case 4: LAUNCH_F64(NPV, 4); break;                                                       \
      case 8: LAUNCH_F64(NPV, 8); break;                                                       \
      case 12: LAUNCH_F64(NPV, 12); break;                                                     \
      default: LAUNCH_F64(NPV, 16); break;                                                     \
    }                                                                                          \
  } while (0)
    if (t.NP == 32) LAUNCH_F64_NP(32);
    else LAUNCH_F64_NP(16);
#undef LAUNCH_F64_NP
#undef LAUNCH_F64
    return hipGetLastError();
  }
  const bool bf = t.precision == AFQMC_BF16X3;
  if (!mfma_tile_valid(t, tile)) tile = TILE_DEFAULT;
  // default at N_P = 32: the block-exchange kernel (fewest LDS and vector instructions per g),
  // eight walkers per workgroup when the workgroups with work (walkers, active spins,
  // determinants) still cover every CU
  if (tile == TILE_DEFAULT && !t.wide && t.NP == 32) {
    const int spins = (t.nup > 0 ? 1 : 0) + (t.ndn > 0 ? 1 : 0);
    tile = (size_t)((nw + 7) / 8) * spins * n_det >= (size_t)device_cu_count() ? TILE_BX8
                                                                                 : TILE_BX;
  }
  if (tile == TILE_FLAT || tile == TILE_STACK) {
    const bool stk = tile == TILE_STACK;
    const FlatLaunch f = flat_launch(t.nup, t.ndn, G, bf, stk);
    dim3 grid(nw, 2 * n_det);
#define LAUNCH_FLAT_KR(BFV, KM, RTV)                                                              \
  do {                                                                                            \
    if (stk)                                                                                      \
      hipLaunchKernelGGL((k_contract_mfma_stack<KM, BFV, ((RTV) > (BFV ? 3 : STACK_MAX_RT)        \
                                                              ? (BFV ? 3 : STACK_MAX_RT)          \
                                                              : (RTV))>),                         \
                         grid, dim3(64 * f.waves), f.lds, st, nw, G, t.nup, t.ndn, t.NP, t.KP,    \
                         f.qup, f.qdn, f.LDR, (const void*)t.Lp, thetaP, weight, tpart, exch);    \
    else                                                                                          \
      hipLaunchKernelGGL((k_contract_mfma_flat<KM, BFV, (RTV)>), grid, dim3(64 * f.waves), f.lds, \
                         st, nw, G, t.nup, t.ndn, t.NP, t.KP, f.qup, f.qdn, f.LDR,                \
                         (const void*)t.Lp, thetaP, weight, tpart, exch);                         \
  } while (0)
  // one instantiation per row-tile count (flat 1 .. 7, BF16x3 1 .. 4; stack 1 .. 7, BF16x3
  // 1 .. 3)
#define LAUNCH_FLAT_K(BFV, KM)                                                                    \
  do {                                                                                            \
    switch (f.RT) {                                                                               \
      case 1: LAUNCH_FLAT_KR(BFV, KM, 1); break;                                                  \
      case 2: LAUNCH_FLAT_KR(BFV, KM, 2); break;                                                  \
      case 3: LAUNCH_FLAT_KR(BFV, KM, 3); break;                                                  \
      case 4: LAUNCH_FLAT_KR(BFV, KM, 4); break;                                                  \
      case 5: LAUNCH_FLAT_KR(BFV, KM, BFV ? 4 : 5); break;                                        \
      case 6: LAUNCH_FLAT_KR(BFV, KM, BFV ? 4 : 6); break;                                        \
      default: LAUNCH_FLAT_KR(BFV, KM, BFV ? 4 : 7); break;                                       \
    }                                                                                             \
  } while (0)
  // and per K chunk count (K_P = 32 .. 224 in steps of 32)
#define LAUNCH_FLAT(BFV)                                                                          \
  do {                                                                                            \
    constexpr int KCH_ = BFV ? 32 : 16;                                                           \
    switch (t.KP / KCH_) {                                                                        \
      case 32 / KCH_: LAUNCH_FLAT_K(BFV, 32 / KCH_); break;                                       \
      case 64 / KCH_: LAUNCH_FLAT_K(BFV, 64 / KCH_); break;                                       \
      case 96 / KCH_: LAUNCH_FLAT_K(BFV, 96 / KCH_); break;                                       \
      case 128 / KCH_: LAUNCH_FLAT_K(BFV, 128 / KCH_); break;                                     \
      case 160 / KCH_: LAUNCH_FLAT_K(BFV, 160 / KCH_); break;                                     \
      case 192 / KCH_: LAUNCH_FLAT_K(BFV, 192 / KCH_); break;                                     \
      default: LAUNCH_FLAT_K(BFV, 224 / KCH_); break;                                             \
    }                                                                                             \
  } while (0)
    if (bf) LAUNCH_FLAT(true);
    else LAUNCH_FLAT(false);
#undef LAUNCH_FLAT
#undef LAUNCH_FLAT_K
#undef LAUNCH_FLAT_KR
    return hipGetLastError();
  }
  if (t.wide || tile == TILE_WIDE) {
    dim3 grid(nw, 2 * n_det);
#define LAUNCH_WIDE_K(NPV, BFV, KM)                                                             \
  do {                                                                                          \
    const size_t shm_ = wide_contract_lds_bytes_t<NPV, BFV>(t.KP);                              \
    hipLaunchKernelGGL((k_contract_mfma_wide<NPV, BFV, KM>), grid, dim3(4 * NPV), shm_, st, nw, \
                       G, t.nup, t.ndn, t.KP, (const void*)t.Lp, thetaP, weight, tpart, exch);  \
  } while (0)
  // one instantiation per K chunk count (K_P = 32 .. 224 in steps of 32)
#define LAUNCH_WIDE(NPV, BFV)                                                                   \
  do {                                                                                          \
    constexpr int KCH_ = BFV ? 32 : 16;                                                         \
    switch (t.KP / KCH_) {                                                                      \
      case 32 / KCH_: LAUNCH_WIDE_K(NPV, BFV, 32 / KCH_); break;                                \
      case 64 / KCH_: LAUNCH_WIDE_K(NPV, BFV, 64 / KCH_); break;                                \
      case 96 / KCH_: LAUNCH_WIDE_K(NPV, BFV, 96 / KCH_); break;                                \
      case 128 / KCH_: LAUNCH_WIDE_K(NPV, BFV, 128 / KCH_); break;                              \
      case 160 / KCH_: LAUNCH_WIDE_K(NPV, BFV, 160 / KCH_); break;                              \
      case 192 / KCH_: LAUNCH_WIDE_K(NPV, BFV, 192 / KCH_); break;                              \
      default: LAUNCH_WIDE_K(NPV, BFV, 224 / KCH_); break;                                      \
    }                                                                                           \
  } while (0)
    if (t.NP == 64) {
      if (bf) LAUNCH_WIDE(64, true);
      else LAUNCH_WIDE(64, false);
    } else if (t.NP == 48) {
      if (bf) LAUNCH_WIDE(48, true);
      else LAUNCH_WIDE(48, false);
    } else {
      if (bf) LAUNCH_WIDE(32, true);
      else LAUNCH_WIDE(32, false);
    }
#undef LAUNCH_WIDE
#undef LAUNCH_WIDE_K
    return hipGetLastError();
  }
  const int wpb = tile == TILE_W2 ? 2 : 4;
  // the kernels are instantiated for K_P = 32, 64, 96, 128
  if (t.KP % 32 != 0 || t.KP < 32 || t.KP > MFMA_KMAX) return hipErrorInvalidValue;
  if (tile == TILE_BX || tile == TILE_BX8) {
    const int wb = tile == TILE_BX8 ? 8 : 4;
    const size_t shm = bx_contract_lds_bytes(t.KP, bf, wb);
    dim3 grid((nw + wb - 1) / wb, 2 * n_det);
#define LAUNCH_BX(BFV, NKV, WBV)                                                               \
  do {                                                                                         \
    (void)hipFuncSetAttribute((const void*)k_contract_mfma_bx<BFV, NKV, WBV>,                  \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);           \
    hipLaunchKernelGGL((k_contract_mfma_bx<BFV, NKV, WBV>), grid, dim3(64 * WBV), shm, st, nw, \
                       G, t.nup, t.ndn, (const void*)t.Lp, thetaP, weight, tpart, exch);       \
  } while (0)
#define LAUNCH_BX_W(BFV, NKV)                                                                  \
  case NKV:                                                                                    \
    if (wb == 8) LAUNCH_BX(BFV, NKV, 8);                                                       \
    else LAUNCH_BX(BFV, NKV, 4);                                                               \
    break;
    // one instantiation per K chunk count (K_P = 32 .. 128 in steps of 32)
    if (bf) {
      switch (t.KP / 32) { LAUNCH_BX_W(true, 1) LAUNCH_BX_W(true, 2) LAUNCH_BX_W(true, 3)
                           default: LAUNCH_BX_W(true, 4) }
    } else {
      switch (t.KP / 16) { LAUNCH_BX_W(false, 2) LAUNCH_BX_W(false, 4) LAUNCH_BX_W(false, 6)
                           default: LAUNCH_BX_W(false, 8) }
    }
#undef LAUNCH_BX_W
#undef LAUNCH_BX
    return hipGetLastError();
  }
  if (tile == TILE_PP) {
    const size_t shm = pp_contract_lds_bytes(t.NP, t.KP, bf);
    dim3 grid((nw + 7) / 8, 2 * n_det);
#define LAUNCH_PP_K(NPV, BFV, NKV)                                                             \
  do {                                                                                         \
    (void)hipFuncSetAttribute((const void*)k_contract_mfma_pp<NPV, BFV, NKV>,                  \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);           \
    hipLaunchKernelGGL((k_contract_mfma_pp<NPV, BFV, NKV>), grid, dim3(512), shm, st, nw, G,   \
                       t.nup, t.ndn, (const void*)t.Lp, thetaP, weight, tpart, exch);          \
  } while (0)
#define LAUNCH_PP(NPV, BFV)                                                                    \
  do {                                                                                         \
    constexpr int KCH_ = contract_kch<NPV, BFV>();                                             \
    switch (t.KP / KCH_) {                                                                     \
      case 32 / KCH_: LAUNCH_PP_K(NPV, BFV, 32 / KCH_); break;                                 \
      case 64 / KCH_: LAUNCH_PP_K(NPV, BFV, 64 / KCH_); break;                                 \
      case 96 / KCH_: LAUNCH_PP_K(NPV, BFV, 96 / KCH_); break;                                 \
      default: LAUNCH_PP_K(NPV, BFV, 128 / KCH_); break;                                       \
    }                                                                                          \
  } while (0)
    if (t.NP == 32) {
      if (bf) LAUNCH_PP(32, true);
      else LAUNCH_PP(32, false);
    } else {
      if (bf) LAUNCH_PP(16, true);
      else LAUNCH_PP(16, false);
    }
#undef LAUNCH_PP
#undef LAUNCH_PP_K
    return hipGetLastError();
  }
  const size_t shm = mfma_contract_lds_bytes(t, wpb);
  dim3 grid((nw + wpb - 1) / wpb, 2 * n_det);
#define LAUNCH_CONTRACT_K(NPV, BFV, WPBV, NKV)                                                  \
  do {                                                                                          \
    (void)hipFuncSetAttribute((const void*)k_contract_mfma<NPV, BFV, WPBV, NKV>,                \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);            \
    hipLaunchKernelGGL((k_contract_mfma<NPV, BFV, WPBV, NKV>), grid, dim3(64 * WPBV), shm, st,  \
                       nw, G, t.nup, t.ndn, t.KP, (const void*)t.Lp, thetaP, weight, tpart,     \
                       exch);                                                                   \
  } while (0)
  // one instantiation per K chunk count (K_P = 32 .. 128 in steps of 32)
#define LAUNCH_CONTRACT(NPV, BFV, WPBV)                                                         \
  do {                                                                                          \
    constexpr int KCH_ = contract_kch<NPV, BFV>();                                              \
    switch (t.KP / KCH_) {                                                                      \
      case 32 / KCH_: LAUNCH_CONTRACT_K(NPV, BFV, WPBV, 32 / KCH_); break;                      \
      case 64 / KCH_: LAUNCH_CONTRACT_K(NPV, BFV, WPBV, 64 / KCH_); break;                      \
      case 96 / KCH_: LAUNCH_CONTRACT_K(NPV, BFV, WPBV, 96 / KCH_); break;                      \
      default: LAUNCH_CONTRACT_K(NPV, BFV, WPBV, 128 / KCH_); break;                            \
    }                                                                                           \
  } while (0)
  if (wpb == 4) {
    if (t.NP == 32) {
      if (bf) LAUNCH_CONTRACT(32, true, 4);
      else LAUNCH_CONTRACT(32, false, 4);
    } else {
      if (bf) LAUNCH_CONTRACT(16, true, 4);
      else LAUNCH_CONTRACT(16, false, 4);
    }
  } else {
    if (t.NP == 32) {
      if (bf) LAUNCH_CONTRACT(32, true, 2);
      else LAUNCH_CONTRACT(32, false, 2);
    } else {
      if (bf) LAUNCH_CONTRACT(16, true, 2);
      else LAUNCH_CONTRACT(16, false, 2);
    }
  }
#undef LAUNCH_CONTRACT
#undef LAUNCH_CONTRACT_K
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Overlap, determinant and Theta with the two small products on FP64 MFMA
// (Theorem 1.1-1.2, eq:precomputing), for N <= 64.  One block (4 waves) per
// (walker, spin, determinant); only the Gauss-Jordan matrix [T | I] lives in LDS, which keeps
// several blocks per CU.
//   T = V^T U             (16x16 blocks, K = M, U read from global as complex)
//   [T | I] -> [I | T^-1] (Gauss-Jordan, partial pivoting, log det from the pivots)
//   Theta^T = (T^-1)^T U^T  (16x16 blocks, K = N, complex product as four real ones)
// Outputs: e1 = tr(ht Theta), log det T (complex), singular flags, and the packed MFMA
// operand of the contraction or (thetaT != NULL, for the FP64 VALU contraction) Theta^T in FP64.
// For the precision guard of the mixed modes (thmax != NULL): max |Theta_pc| of the block's
// walker-spin in thmax and the FP64 packed operand (the layout of packed_kind 3) in packed64.
// ---------------------------------------------------------------------------
template <int NPAD>
__global__ void __launch_bounds__(256) k_overlap_mfma(
    int M, int nup, int ndn, const double* __restrict__ V, const double* __restrict__ ht,
    const cd* __restrict__ U, const double* __restrict__ weight, int check_weight,
    cd* __restrict__ thetaT, cd* __restrict__ logdet, cd* __restrict__ e1,
    unsigned* __restrict__ wflag, void* __restrict__ packed, int packed_kind, int NP, int KP,
    double* __restrict__ thmax, double* __restrict__ packed64) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  constexpr int NB = NPAD / 16;
  // determinant d of the trial (blockIdx.z); per-determinant outputs are indexed by
  // wd = w * n_det + d, and the trial arrays V, ht are offset to determinant d.
  const int d = blockIdx.z, n_det = gridDim.z;
  const int wd_ = blockIdx.x * n_det + d;
  V += (size_t)d * (nup + ndn) * M;
  ht += (size_t)d * (nup + ndn) * M;
  const int w = blockIdx.x, s = blockIdx.y;
  const int N = s == 0 ? nup : ndn;
  const int off = s == 0 ? 0 : nup;
  const int ntot = nup + ndn;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (N == 0) {
    if (tid == 0) {
      logdet[2 * wd_ + s] = mkc(0.0, 0.0);
      e1[2 * wd_ + s] = mkc(0.0, 0.0);
      wflag[2 * wd_ + s] = 0u;
      if (thmax) thmax[2 * wd_ + s] = 0.0;
    }
    return;
  }
  if (check_weight && !(weight[w] > 0.0)) return;
  const int lda = 2 * N + 1;
  cd* Ag = reinterpret_cast<cd*>(smem_raw);          // [N][2N+1]
  double* red = reinterpret_cast<double*>(Ag + (size_t)N * lda);  // [8]
  __shared__ int s_piv, s_sing, s_nswap;
  __shared__ cd s_pk;
  __shared__ cd s_pv[NPAD];  // pivot of every step: log det is taken after the elimination
  const int l16 = lane & 15, q = lane >> 4;
  const cd* Uw = U + ((size_t)w * ntot + off) * M;
  const double* Vs = V + (size_t)off * M;

  // ---- T = V^T U on MFMA: wave t handles block (t / NB, t % NB)
  for (int t = wave; t < NB * NB; t += 4) {
    const int a = t / NB, b = t % NB;
    f64x4 tr = {0.0, 0.0, 0.0, 0.0}, ti = {0.0, 0.0, 0.0, 0.0};
    const int ri = 16 * a + l16, cj = 16 * b + l16;
    // rows / columns past N read row 0 (their outputs are never stored); K past M reads the
    // last column and is zeroed on the V side.  Four K steps of loads go out before their
    // MFMAs, so the global latency is paid once per four steps (eight cost a wave per SIMD).
    const int rr = ri < N ? ri : 0, cc = cj < N ? cj : 0;
    for (int k0 = 0; k0 < M; k0 += 16) {
      double va[4];
      cd ub[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 4 * u + q, kk = k < M ? k : M - 1;
        va[u] = Vs[(size_t)rr * M + kk];
        ub[u] = Uw[(size_t)cc * M + kk];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double av = k0 + 4 * u + q < M ? va[u] : 0.0;
        tr = __builtin_amdgcn_mfma_f64_16x16x4f64(av, ub[u].re, tr, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f64_16x16x4f64(av, ub[u].im, ti, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * a + q + 4 * v, c = 16 * b + l16;
      if (r < N && c < N) Ag[r * lda + c] = mkc(tr[v], ti[v]);
    }
  }
  for (int e = tid; e < N * N; e += blockDim.x) {
    const int i = e / N, j = e % N;
    Ag[i * lda + N + j] = mkc(i == j ? 1.0 : 0.0, 0.0);
  }
  if (tid == 0) {
    s_sing = 0;
    s_nswap = 0;
  }
  __syncthreads();
  // ---- Gauss-Jordan with partial pivoting, three barriers per pivot k:
  //   (1) wave 0 finds the pivot row and records the pivot value;
  //   (2) rows k and piv are exchanged and the new row k is divided by the pivot;
  //   (3) every other row i loses A[i][k] times row k.
  // Columns left of k are never read again, so (2) starts at column k and (3) at k + 1;
  // column k itself is not eliminated, which lets (3) read its multipliers A[i][k] in place.
  for (int k = 0; k < N; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      for (int i = k + lane; i < N; i += 64) {
        const cd v = Ag[i * lda + k];
        const double m = v.re * v.re + v.im * v.im;
        if (m > best) {
          best = m;
          bi = i;
        }
      }
      wave_argmax(best, bi);
      if (lane == 0) {
        s_piv = bi;
        s_pk = Ag[bi * lda + k];
        s_pv[k] = s_pk;
        if (!(best > 0.0)) s_sing = 1;
        if (bi != k) s_nswap += 1;
      }
    }
    __syncthreads();
    if (s_sing) break;
    const int piv = s_piv;
    const cd pk = s_pk;
    for (int j = k + tid; j < 2 * N; j += blockDim.x) {
      const cd rk = Ag[k * lda + j], rp = Ag[piv * lda + j];
      Ag[k * lda + j] = cdiv(rp, pk);
      if (piv != k) Ag[piv * lda + j] = rk;
    }
    __syncthreads();
    const int ncol = 2 * N - (k + 1);
    for (int e = tid; e < N * ncol; e += blockDim.x) {
      const int i = e / ncol, j = k + 1 + e % ncol;
      if (i != k) cfms(Ag[i * lda + j], Ag[i * lda + k], Ag[k * lda + j]);
    }
    __syncthreads();
  }
  if (s_sing) {
    if (tid == 0) {
      wflag[2 * wd_ + s] = WFLAG_SINGULAR;
      logdet[2 * wd_ + s] = mkc(-INFINITY, 0.0);
      e1[2 * wd_ + s] = mkc(0.0, 0.0);
    }
    return;
  }
  if (tid < 64) {
    // log det T = sum_k log pivot_k (+ i pi per row exchange): the logarithms of all pivots
    // at once, off the elimination's critical path (0.36 -> 0.32 ms at 2048 walker-spins)
    double la = 0.0, ar = 0.0;
    for (int k = lane; k < N; k += 64) {
      const cd pv = s_pv[k];
      la += log(hypot(pv.re, pv.im));
      ar += atan2(pv.im, pv.re);
    }
    la = wave_sum(la);
    ar = wave_sum(ar);
    if (lane == 0) {
      logdet[2 * wd_ + s] = mkc(la, ar + M_PI * (double)(s_nswap & 1));
      wflag[2 * wd_ + s] = 0u;
    }
  }
  // ---- Theta^T[c][p] = sum_j Tinv[j][c] U^T[j][p] on MFMA (K = j, padded to NPAD)
  const int CB = (M + 15) / 16;
  const size_t per = (size_t)NP * KP;
  cd* Tw = thetaT ? thetaT + ((size_t)wd_ * ntot + off) * M : nullptr;
  const double* hts = ht + (size_t)off * M;
  double e1re = 0.0, e1im = 0.0;
  double th2max = 0.0;   // largest |Theta_pc|^2 this thread stored
  for (int t = wave; t < NB * CB; t += 4) {
    const int a = t / CB, b = t % CB;
    f64x4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
    const int c_in = 16 * a + l16;   // A row (output row c)
    const int p_in = 16 * b + l16;   // B column (output column p)
    // U loads four K steps at a time ahead of their MFMAs; rows j past N and columns past M
    // read valid elements (T^-1 is zero there on the A side, such outputs are never stored)
    const int pp = p_in < M ? p_in : M - 1;
    // h~ entries of the tile's outputs, loaded ahead as well up to N_P = 32 (beyond, the
    // registers would cost a wave per SIMD)
    constexpr bool HPRE = NPAD <= 32;
    double hvv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 16 * a + q + 4 * v;
      hvv[v] = HPRE ? hts[(size_t)(c < N ? c : N - 1) * M + pp] : 0.0;
    }
#pragma unroll
    for (int k0 = 0; k0 < NPAD; k0 += 16) {
      cd uvv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = k0 + 4 * u + q;
        uvv[u] = Uw[(size_t)(j < N ? j : N - 1) * M + pp];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = k0 + 4 * u + q;
        const cd tv = (j < N && c_in < N) ? Ag[j * lda + N + c_in] : mkc(0.0, 0.0);
        const cd uv = uvv[u];
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.re, uv.re, cr, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-tv.im, uv.im, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.re, uv.im, ci, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.im, uv.re, ci, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 16 * a + q + 4 * v, p = 16 * b + l16;
      if (c >= N || p >= M) continue;
      const cd th = mkc(cr[v], ci[v]);
      if (thetaT) Tw[(size_t)c * M + p] = th;   // FP64 copy only for the VALU contraction
      if (thmax) {
        th2max = fmax(th2max, th.re * th.re + th.im * th.im);
        double* o = packed64 + ((size_t)wd_ * 2 + s) * 2 * per + (size_t)c * KP + p;
        o[0] = th.re;
        o[per] = th.im;
      }
      const double hv = HPRE ? hvv[v] : hts[(size_t)c * M + p];
      e1re = fma(hv, th.re, e1re);
      e1im = fma(hv, th.im, e1im);
      if (packed_kind == 3) {
        double* o = reinterpret_cast<double*>(packed) + ((size_t)wd_ * 2 + s) * 2 * per + (size_t)c * KP + p;
        o[0] = th.re;
        o[per] = th.im;
      } else if (packed_kind == 1) {
        float* o = reinterpret_cast<float*>(packed) + ((size_t)wd_ * 2 + s) * 2 * per + (size_t)c * KP + p;
        o[0] = (float)th.re;
        o[per] = (float)th.im;
      } else if (packed_kind == 2) {
        uint16_t* o = reinterpret_cast<uint16_t*>(packed) + ((size_t)wd_ * 2 + s) * 4 * per + (size_t)c * KP + p;
        const float xr = (float)th.re, xi = (float)th.im;
        const uint16_t hr = f32_to_bf16_bits(xr), hi = f32_to_bf16_bits(xi);
        o[0] = hr;
        o[per] = f32_to_bf16_bits(xr - bf16_bits_to_f32(hr));
        o[2 * per] = hi;
        o[3 * per] = f32_to_bf16_bits(xi - bf16_bits_to_f32(hi));
      }
    }
  }
  if (packed_kind) {
    const int planes = packed_kind == 2 ? 4 : 2;
    for (size_t e = tid; e < (size_t)planes * per; e += blockDim.x) {
      const int pl = (int)(e / per);
      const int c = (int)((e % per) / KP), p = (int)(e % KP);
      if (c < N && p < M) continue;
      const size_t o = ((size_t)wd_ * 2 + s) * planes * per + (size_t)pl * per + (size_t)c * KP + p;
      if (packed_kind == 3) reinterpret_cast<double*>(packed)[o] = 0.0;
      else if (packed_kind == 1) reinterpret_cast<float*>(packed)[o] = 0.f;
      else reinterpret_cast<uint16_t*>(packed)[o] = 0;
    }
  }
  if (thmax) {
    for (size_t e = tid; e < (size_t)2 * per; e += blockDim.x) {
      const int c = (int)((e % per) / KP), p = (int)(e % KP);
      if (c < N && p < M) continue;
      packed64[((size_t)wd_ * 2 + s) * 2 * per + e] = 0.0;
    }
    const double m2 = block_max(th2max, red);
    if (tid == 0) thmax[2 * wd_ + s] = sqrt(m2);
  }
  e1re = block_sum(e1re, red);
  e1im = block_sum(e1im, red);
  if (tid == 0) e1[2 * wd_ + s] = mkc(e1re, e1im);
}

// A double of lane l (l wave-uniform) in every lane.
__device__ __forceinline__ double readlane_d(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint64_t r = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  return __builtin_bit_cast(double, r);
}

// Zero the padding of one walker-spin's packed operand planes (rows c >= N of every column,
// columns p >= M of rows c < N), one wavefront.
template <typename E>
__device__ inline void zero_packed_pad(E* base, int planes, size_t per, int N, int M, int NP, int KP,
                                       int lane) {
  for (int pl = 0; pl < planes; ++pl) {
    E* o = base + (size_t)pl * per;
    for (int c = N; c < NP; ++c)
      for (int p = lane; p < KP; p += 64) o[(size_t)c * KP + p] = E(0);
    if (M < KP)
      for (int c = 0; c < N; ++c)
        for (int p = M + lane; p < KP; p += 64) o[(size_t)c * KP + p] = E(0);
  }
}

// ---------------------------------------------------------------------------
// The outputs of k_overlap_mfma for N <= 32 (Theorem 1.1-1.2, eq:precomputing) with one
// wavefront per (walker, spin, determinant) and no workgroup barrier:
//   T = V^T U on FP64 MFMA (16 x 16 blocks, K = M; each lane loads four consecutive k and
//     MFMA u takes the u-th of them, the same permutation of k in both operands);
//   T^-1 by Gauss-Jordan in place in registers: lane i + 32 h holds row i, columns
//     16 h .. 16 h + 15, with the identity in rows and columns past N.  Pivoting is implicit:
//     rows stay in their lanes and step k takes as pivot the unused row p_k with the largest
//     |T_ik|.  The result X satisfies (T^-1)_ij = X[p_i][q_j], q the inverse of p, so
//     det T = prod_k pivot_k times the sign of the permutation p, and
//   Theta^T[c][m] = sum_j (T^-1)_jc U_jm = sum_r X[r][q_c] U[q_r][m] on FP64 MFMA (K = r).
// Step k of the elimination: the two lanes of row p_k put its raw entries in LDS and every
// lane reads those of its own half of the columns; row i loses f_i times that row, with
// f_i = T_ik / T_pk and f_p = 1 - 1 / T_pk (which leaves the pivot row divided by the pivot);
// column k then holds -f_i, and 1 / T_pk in row p_k.
// With the precision guard (thmax != NULL) the FP64 operand is written only for a walker-spin
// whose max |Theta| exceeds the guard's threshold: the guard redoes exactly those spins.
// ---------------------------------------------------------------------------
template <int NPAD>
__global__ void __launch_bounds__(64, 2) k_overlap_wave(
    int M, int nup, int ndn, const double* __restrict__ V, const double* __restrict__ ht,
    const cd* __restrict__ U, const double* __restrict__ weight, int check_weight,
    cd* __restrict__ thetaT, cd* __restrict__ logdet, cd* __restrict__ e1,
    unsigned* __restrict__ wflag, void* __restrict__ packed, int packed_kind, int NP, int KP,
    double* __restrict__ thmax, double* __restrict__ packed64, double guard) {
  static_assert(NPAD == 16 || NPAD == 32, "one wavefront inverts at most 32 x 32");
  constexpr int NB = NPAD / 16, NKC = NPAD / 16, XL = 33;
  __shared__ __attribute__((aligned(16))) cd Xs[32 * XL];   // T, then X
  __shared__ __attribute__((aligned(16))) cd Rb[2][16];     // pivot row, by column half
  __shared__ cd s_pv[32];
  __shared__ int s_p[32], s_q[32];
  const int d = blockIdx.z, n_det = gridDim.z;
  const int wd_ = blockIdx.x * n_det + d;
  V += (size_t)d * (nup + ndn) * M;
  ht += (size_t)d * (nup + ndn) * M;
  const int w = blockIdx.x, s = blockIdx.y;
  const int N = s == 0 ? nup : ndn;
  const int off = s == 0 ? 0 : nup;
  const int ntot = nup + ndn;
  const int lane = threadIdx.x;
  if (N == 0) {
    if (lane == 0) {
      logdet[2 * wd_ + s] = mkc(0.0, 0.0);
      e1[2 * wd_ + s] = mkc(0.0, 0.0);
      wflag[2 * wd_ + s] = 0u;
      if (thmax) thmax[2 * wd_ + s] = 0.0;
    }
    return;
  }
  if (check_weight && !(weight[w] > 0.0)) return;
  const int l16 = lane & 15, q = lane >> 4;
  const cd* Uw = U + ((size_t)w * ntot + off) * M;
  const double* Vs = V + (size_t)off * M;

  // ---- T = V^T U: block (a, b) rows 16 a + l16 of V, columns 16 b + l16 (rows of U); rows
  // past N read row 0 (never stored), k past M reads column M - 1 with V zeroed there.  The
  // loads of the next 16 k go out before the MFMAs of these.
  {
    f64x4 tr[NB][NB], ti[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) tr[a][b] = ti[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    const double* vrow[NB];
    const cd* urow[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int r = 16 * a + l16;
      vrow[a] = Vs + (size_t)(r < N ? r : 0) * M;
      urow[a] = Uw + (size_t)(r < N ? r : 0) * M;
    }
    double va[NB][4], vn[NB][4];
    cd ub[NB][4], un[NB][4];
    auto load = [&](int k0, double (&vv)[NB][4], cd (&uu)[NB][4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 4 * q + u, kk = k < M ? k : M - 1;
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          const double x = vrow[a][kk];
          vv[a][u] = k < M ? x : 0.0;
          uu[a][u] = urow[a][kk];
        }
      }
    };
    load(0, va, ub);
    for (int k0 = 0; k0 < M; k0 += 16) {
      if (k0 + 16 < M) load(k0 + 16, vn, un);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            tr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[a][u], ub[b][u].re, tr[a][b], 0, 0, 0);
            ti[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[a][u], ub[b][u].im, ti[a][b], 0, 0, 0);
          }
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          va[a][u] = vn[a][u];
          ub[a][u] = un[a][u];
        }
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * a + q + 4 * v, c = 16 * b + l16;
          if (r < N && c < N) Xs[r * XL + c] = mkc(tr[a][b][v], ti[a][b][v]);
        }
  }
  wave_lds_fence();

  // ---- Gauss-Jordan in registers
  const int gi = lane & 31, gh = lane >> 5;
  cd x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int j = 16 * gh + c;
    x[c] = gi < N && j < N ? Xs[gi * XL + j] : mkc(gi == j ? 1.0 : 0.0, 0.0);
  }
  bool used = false;
  int sing = 0;
  // a fixed trip count keeps the loop unrolled, so x[ck] is a register; the body is skipped
  // (uniformly) past N or after a zero pivot
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    if (k >= N || sing) continue;
    const int hk = k >> 4, ck = k & 15;
    const cd xk = x[ck];   // column k in the lanes of half hk
    double best = gh == hk && !used && gi < N ? xk.re * xk.re + xk.im * xk.im : -1.0;
    int bi = gi;
    wave_argmax(best, bi);
    const int p = __builtin_amdgcn_readfirstlane(bi);
    best = readlane_d(best, 0);
    if (!(best > 0.0)) {
      sing = 1;
      continue;
    }
    const int pl = p + 32 * hk;
    const cd pk = mkc(readlane_d(xk.re, pl), readlane_d(xk.im, pl));
    const double rb = 1.0 / best;
    const cd inv = mkc(pk.re * rb, -pk.im * rb);
    if (gi == p) {
#pragma unroll
      for (int c = 0; c < 16; ++c) Rb[gh][c] = x[c];
    }
    if (lane == 0) {
      s_p[k] = p;
      s_pv[k] = pk;
    }
    // this lane's T_ik: its own register in half hk, the partner lane's (lane ^ 32) otherwise
    const cd xo = mkc(__shfl_xor(xk.re, 32), __shfl_xor(xk.im, 32));
    const cd aik = gh == hk ? xk : xo;
    cd f = mkc(aik.re * inv.re - aik.im * inv.im, aik.re * inv.im + aik.im * inv.re);
    if (gi == p) f = mkc(1.0 - inv.re, -inv.im);
    wave_lds_fence();
#pragma unroll
    for (int c = 0; c < 16; ++c) cfms(x[c], f, Rb[gh][c]);
    if (gh == hk) x[ck] = gi == p ? inv : mkc(-f.re, -f.im);
    used = used || gi == p;
    wave_lds_fence();   // the next step's pivot row overwrites Rb
  }
  if (sing) {
    if (lane == 0) {
      wflag[2 * wd_ + s] = WFLAG_SINGULAR;
      logdet[2 * wd_ + s] = mkc(-INFINITY, 0.0);
      e1[2 * wd_ + s] = mkc(0.0, 0.0);
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < 16; ++c) Xs[gi * XL + 16 * gh + c] = x[c];
  if (lane < N) s_q[s_p[lane]] = lane;
  wave_lds_fence();
  {
    // log det T = sum_k log pivot_k, plus i pi when the permutation p is odd
    double la = 0.0, ar = 0.0;
    if (lane < N) {
      const cd pv = s_pv[lane];
      la = log(hypot(pv.re, pv.im));
      ar = atan2(pv.im, pv.re);
    }
    la = wave_sum(la);
    ar = wave_sum(ar);
    if (lane == 0) {
      unsigned seen = 0u;
      int cycles = 0;
      for (int i0 = 0; i0 < N; ++i0) {
        if ((seen >> i0) & 1u) continue;
        ++cycles;
        for (int j = i0; !((seen >> j) & 1u); j = s_p[j]) seen |= 1u << j;
      }
      logdet[2 * wd_ + s] = mkc(la, ar + M_PI * (double)((N - cycles) & 1));
      wflag[2 * wd_ + s] = 0u;
    }
  }

  // ---- Theta^T[c][m] = sum_r X[r][q_c] U[q_r][m]: the X operand read from LDS at
  // immediate offsets from one address per row block a (rows r past N of X are identity rows,
  // zero in the columns q_c < N; columns c past N read column 0 and are never stored), U rows
  // by q, 16 columns m per block, the next block's U loads ahead of this block's MFMAs
  int xb[NB];
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    const int c = 16 * a + l16;
    xb[a] = 4 * q * XL + (c < N ? s_q[c] : 0);
  }
  int uro[NKC][4];   // U row q_r, as an element offset
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = 16 * kc + 4 * q + u;
      uro[kc][u] = (r < N ? s_q[r] : 0) * M;
    }
  const int CBn = (M + 15) / 16;
  const size_t per = (size_t)NP * KP;
  cd* Tw = thetaT ? thetaT + ((size_t)wd_ * ntot + off) * M : nullptr;
  const double* hts = ht + (size_t)off * M;
  double e1re = 0.0, e1im = 0.0, th2max = 0.0;
  bool guarded = false;   // the precision guard takes this walker-spin
  cd uv[NKC][4], un2[NKC][4];
  auto loadu = [&](int b, cd (&dst)[NKC][4]) {
    const int pp = 16 * b + l16, pc = pp < M ? pp : M - 1;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
      for (int u = 0; u < 4; ++u) dst[kc][u] = Uw[uro[kc][u] + pc];
  };
  // pass 0 writes the outputs and finds max |Theta|; pass 1, only for a walker-spin the
  // precision guard takes (max |Theta| above its threshold, the test the guard applies to the
  // stored value), computes Theta again for its FP64 operand
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      if (!thmax) break;
      for (int o = 32; o > 0; o >>= 1) th2max = fmax(th2max, __shfl_xor(th2max, o));
      const double m = sqrt(th2max);
      if (lane == 0) thmax[2 * wd_ + s] = m;
      guarded = m > guard;
      if (!guarded) break;
    }
    loadu(0, uv);
    for (int b0 = 0; b0 < CBn; ++b0) {
      // an opaque block index keeps the compiler from turning every store address of the
      // epilogue into a 64-bit induction variable held across the loop
      int b = b0;
      asm volatile("" : "+s"(b));
      if (b + 1 < CBn) loadu(b + 1, un2);
      const int pp = 16 * b + l16, pc = pp < M ? pp : M - 1;
      double hvv[NB][4];   // h~ at this block's outputs, loaded ahead of the MFMAs
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * a + q + 4 * v;
          hvv[a][v] = hts[(size_t)(c < N ? c : N - 1) * M + pc];
        }
      f64x4 cr[NB], ci[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) cr[a] = ci[a] = f64x4{0.0, 0.0, 0.0, 0.0};
      // the X reads stay in the loop (hoisted they would hold 64 registers across it)
      int xo[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        xo[a] = xb[a];
        asm volatile("" : "+v"(xo[a]));
      }
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int a = 0; a < NB; ++a) {
            const cd tv = Xs[xo[a] + (16 * kc + u) * XL], uw = uv[kc][u];
            cr[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.re, uw.re, cr[a], 0, 0, 0);
            cr[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(-tv.im, uw.im, cr[a], 0, 0, 0);
            ci[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.re, uw.im, ci[a], 0, 0, 0);
            ci[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(tv.im, uw.re, ci[a], 0, 0, 0);
          }
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * a + q + 4 * v, p = pp;
          if (c >= N || p >= M) continue;
          const cd th = mkc(cr[a][v], ci[a][v]);
          if (pass == 1) {
            double* o = packed64 + ((size_t)wd_ * 2 + s) * 2 * per + (size_t)c * KP + p;
            o[0] = th.re;
            o[per] = th.im;
            continue;
          }
          if (thetaT) Tw[(size_t)c * M + p] = th;
          if (thmax) th2max = fmax(th2max, th.re * th.re + th.im * th.im);
          e1re = fma(hvv[a][v], th.re, e1re);
          e1im = fma(hvv[a][v], th.im, e1im);
          if (packed_kind == 3) {
            double* o = reinterpret_cast<double*>(packed) + ((size_t)wd_ * 2 + s) * 2 * per + (size_t)c * KP + p;
            o[0] = th.re;
            o[per] = th.im;
          } else if (packed_kind == 1) {
            float* o = reinterpret_cast<float*>(packed) + ((size_t)wd_ * 2 + s) * 2 * per + (size_t)c * KP + p;
            o[0] = (float)th.re;
            o[per] = (float)th.im;
          } else if (packed_kind == 2) {
            uint16_t* o = reinterpret_cast<uint16_t*>(packed) + ((size_t)wd_ * 2 + s) * 4 * per + (size_t)c * KP + p;
            const float xr = (float)th.re, xi = (float)th.im;
            const uint16_t hr = f32_to_bf16_bits(xr), hi = f32_to_bf16_bits(xi);
            o[0] = hr;
            o[per] = f32_to_bf16_bits(xr - bf16_bits_to_f32(hr));
            o[2 * per] = hi;
            o[3 * per] = f32_to_bf16_bits(xi - bf16_bits_to_f32(hi));
          }
        }
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
        for (int u = 0; u < 4; ++u) uv[kc][u] = un2[kc][u];
    }
  }
  const size_t ws_ = (size_t)wd_ * 2 + s;
  if (packed_kind == 3)
    zero_packed_pad(reinterpret_cast<double*>(packed) + ws_ * 2 * per, 2, per, N, M, NP, KP, lane);
  else if (packed_kind == 1)
    zero_packed_pad(reinterpret_cast<float*>(packed) + ws_ * 2 * per, 2, per, N, M, NP, KP, lane);
  else if (packed_kind == 2)
    zero_packed_pad(reinterpret_cast<uint16_t*>(packed) + ws_ * 4 * per, 4, per, N, M, NP, KP, lane);
  if (guarded) zero_packed_pad(packed64 + ws_ * 2 * per, 2, per, N, M, NP, KP, lane);
  e1re = wave_sum(e1re);
  e1im = wave_sum(e1im);
  if (lane == 0) e1[2 * wd_ + s] = mkc(e1re, e1im);
}
