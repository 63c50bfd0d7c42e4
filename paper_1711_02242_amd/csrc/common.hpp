// Shared device helpers of the AFQMC library: complex FP64 arithmetic, the
// counter-based Philox4x64-10 stream (Salmon, Moraes, Dror, Shaw, SC'11) and
// wavefront reductions for CDNA (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef __HIP_DEVICE_COMPILE__
#include <cmath>
#endif

#define AFQMC_WAVE 64

struct cd {
  double re, im;
};

__host__ __device__ inline cd mkc(double re, double im) { return cd{re, im}; }
__host__ __device__ inline cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cd csub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cd cmul(cd a, cd b) {
  return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cd cscale(cd a, double s) { return cd{a.re * s, a.im * s}; }
__host__ __device__ inline cd cconjmul(cd a, cd b) {  // conj(a) * b
  return cd{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__host__ __device__ inline cd cdiv(cd a, cd b) {
  // Smith's algorithm keeps the intermediate magnitudes bounded.
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, den = b.re + b.im * r;
    return cd{(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  } else {
    double r = b.re / b.im, den = b.re * r + b.im;
    return cd{(a.re * r + a.im) / den, (a.im * r - a.re) / den};
  }
}
// a += b * c
__host__ __device__ inline void cfma(cd& a, cd b, cd c) {
  a.re = fma(b.re, c.re, fma(-b.im, c.im, a.re));
  a.im = fma(b.re, c.im, fma(b.im, c.re, a.im));
}
// a -= b * c
__host__ __device__ inline void cfms(cd& a, cd b, cd c) {
  a.re = fma(-b.re, c.re, fma(b.im, c.im, a.re));
  a.im = fma(-b.re, c.im, fma(-b.im, c.re, a.im));
}
// a += b * r (r real)
__host__ __device__ inline void cfmar(cd& a, cd b, double r) {
  a.re = fma(b.re, r, a.re);
  a.im = fma(b.im, r, a.im);
}

__host__ __device__ inline bool cfinite(cd a) { return isfinite(a.re) && isfinite(a.im); }

// ---------------------------------------------------------------------------
// Philox4x64-10.  Round: (hi0, lo0) = M0 * x0, (hi1, lo1) = M1 * x2 (full 128-bit
// products); x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0); the key is bumped by
// the Weyl constants (W0, W1) before every round after the first.
// ---------------------------------------------------------------------------
struct u64x4 {
  uint64_t v[4];
};

__device__ inline u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                      uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * x0, hi0 = __umul64hi(M0, x0);
    const uint64_t lo1 = M1 * x2, hi1 = __umul64hi(M1, x2);
    const uint64_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
    x0 = n0;
    x1 = lo1;
    x2 = n2;
    x3 = lo0;
  }
  u64x4 o;
  o.v[0] = x0;
  o.v[1] = x1;
  o.v[2] = x2;
  o.v[3] = x3;
  return o;
}

// uint64 -> double in (0, 1]: ((r >> 11) + 0.5) * 2^-53 (equal to 1 only where the sum rounds up).
__device__ inline double u64_unit(uint64_t r) {
  return ((double)(r >> 11) + 0.5) * 0x1p-53;
}

// ---------------------------------------------------------------------------
// Wavefront / block reductions (fixed order -> deterministic results).
// ---------------------------------------------------------------------------

// DPP sums over lanes (fixed order, deterministic).  dpp_row_sum: the sum over each 16-lane row,
// left in the row's last lane (lanes 15, 31, 47, 63): four shifts within the row, out-of-row
// sources read as zero.  dpp_half_sum: then the last lane of rows 0 and 2 added into rows 1
// and 3 (row_bcast:15), so lane 31 holds the sum over lanes 0..31 and lane 63 over 32..63.
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                               ROW_MASK, 0xF, BOUND));
}
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ double dpp_f(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK,
                                                            0xF, BOUND);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL,
                                                            ROW_MASK, 0xF, BOUND);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T dpp_row_sum(T v) {
  v += dpp_f<0x111, 0xF, true>(v);   // row_shr:1
  v += dpp_f<0x112, 0xF, true>(v);   // row_shr:2
  v += dpp_f<0x114, 0xF, true>(v);   // row_shr:4
  v += dpp_f<0x118, 0xF, true>(v);   // row_shr:8
  return v;
}
template <typename T>
__device__ __forceinline__ T dpp_half_sum(T v) {
  v = dpp_row_sum(v);
  v += dpp_f<0x142, 0xA, false>(v);  // row_bcast:15 into rows 1 and 3
  return v;
}

// Sum over all 64 lanes, returned to every lane: the two half sums of dpp_half_sum read from
// lanes 31 and 63.
__device__ __forceinline__ float dpp_wave_sum(float v) {
  v = dpp_half_sum(v);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 31)) +
         __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Sum over the 64 lanes of a wavefront (every lane active), the same value in every lane:
// DPP row sums, then the two half sums read from lanes 31 and 63.
__device__ inline double wave_sum(double v) {
  v = dpp_half_sum(v);
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
  const uint64_t a = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, 31) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane(lo, 31);
  const uint64_t b = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, 63) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane(lo, 63);
  return __builtin_bit_cast(double, a) + __builtin_bit_cast(double, b);
}

// Largest value over the 64 lanes (every lane active), ties to the smallest index; the result
// in every lane.  The order (value descending, index ascending) is total, so the outcome does
// not depend on the combination order: DPP row shifts, row_bcast:15, then lanes 31 and 63.
// Sources outside the row (or rows left out by the mask) read as (-inf, INT_MAX).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_argmax_step(double& best, int& idx) {
  const uint64_t u = __builtin_bit_cast(uint64_t, best);
  const uint64_t ninf = __builtin_bit_cast(uint64_t, -__builtin_inf());
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)ninf, (int)(uint32_t)u,
                                                            CTRL, ROW_MASK, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(
      (int)(uint32_t)(ninf >> 32), (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xF, false);
  const int oi = __builtin_amdgcn_update_dpp(0x7fffffff, idx, CTRL, ROW_MASK, 0xF, false);
  const double ob = __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  if (ob > best || (ob == best && oi < idx)) {
    best = ob;
    idx = oi;
  }
}
__device__ inline void wave_argmax(double& best, int& idx) {
  dpp_argmax_step<0x111, 0xF>(best, idx);   // row_shr:1
  dpp_argmax_step<0x112, 0xF>(best, idx);   // row_shr:2
  dpp_argmax_step<0x114, 0xF>(best, idx);   // row_shr:4
  dpp_argmax_step<0x118, 0xF>(best, idx);   // row_shr:8
  dpp_argmax_step<0x142, 0xA>(best, idx);   // row_bcast:15 into rows 1 and 3
  const uint64_t u = __builtin_bit_cast(uint64_t, best);
  const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
  const double b31 = __builtin_bit_cast(
      double, ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, 31) << 32) |
                  (uint32_t)__builtin_amdgcn_readlane(lo, 31));
  const double b63 = __builtin_bit_cast(
      double, ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, 63) << 32) |
                  (uint32_t)__builtin_amdgcn_readlane(lo, 63));
  const int i31 = __builtin_amdgcn_readlane(idx, 31), i63 = __builtin_amdgcn_readlane(idx, 63);
  const bool hi_wins = b63 > b31 || (b63 == b31 && i63 < i31);
  best = hi_wins ? b63 : b31;
  idx = hi_wins ? i63 : i31;
}

// Growth-phase state of a walker population (k_growth_sum), doubles in the workspace.
enum { GR_ET = 0, GR_EBAR, GR_NUM, GR_DEN, GR_SWE, GR_SW, GR_COUNT = 8 };
// Counters of the rare-event bounds (App. B.1), 64-bit, library-owned per system:
// walker-steps with the local energy capped in the weight, with the weight capped,
// force-bias components capped, and walker-steps whose weight was updated.
// The fifth counts walker-steps whose contraction the precision guard redid in FP64.
enum { CAP_E = 0, CAP_W, CAP_FB, CAP_LIVE, CAP_GUARD, CAP_COUNT = 5 };

// Adds the number of active lanes of the wavefront with `pred` true to *c: one atomic per
// wavefront, from its lowest active lane (integer sums: the total is order independent).
__device__ inline void wave_count(unsigned long long* c, bool pred) {
  const unsigned long long m = __ballot(pred);
  const unsigned long long act = __ballot(true);
  if (m && __lane_id() == __builtin_ctzll(act)) atomicAdd(c, (unsigned long long)__popcll(m));
}

// Largest value over the block of one double per thread; every thread gets the result.
// `red` must hold blockDim.x / 64 doubles.  Contains __syncthreads().
__device__ inline double block_max(double v, double* red) {
  const int lane = threadIdx.x % AFQMC_WAVE, wid = threadIdx.x / AFQMC_WAVE;
  const int nw = (blockDim.x + AFQMC_WAVE - 1) / AFQMC_WAVE;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, AFQMC_WAVE));
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = red[0];
  for (int i = 1; i < nw; ++i) t = fmax(t, red[i]);
  return t;
}

// Sum over the block of one double per thread; every thread gets the result.
// `red` must hold blockDim.x / 64 doubles.  Contains __syncthreads().
__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x % AFQMC_WAVE, wid = threadIdx.x / AFQMC_WAVE;
  const int nw = (blockDim.x + AFQMC_WAVE - 1) / AFQMC_WAVE;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}
