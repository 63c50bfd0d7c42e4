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

#include <vector>

#include "common.hpp"

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int MFMA_KMAX = 128;
constexpr int MFMA_WAVES = 4;

struct MfmaTables {
  bool enabled = false;
  int precision = 0;  // AFQMC_FP32 or AFQMC_BF16X3
  int NP = 0, KP = 0, M = 0, G = 0, nup = 0, ndn = 0;
  void* Lp = nullptr;  // fp32: [2][G][NP][KP]; bf16x3: [2][G][2 (hi, lo)][NP][KP] bf16 bits
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
  return nw * 2 * 2 * (size_t)t.NP * t.KP * 4;  // fp32 re/im, or bf16 re/im x hi/lo
}

inline int mfma_build_tables(MfmaTables& t, int precision, int M, int nup, int ndn, int G,
                             const double* Lh /* host [G][nup+ndn][M] */) {
  const int nmax = nup > ndn ? nup : ndn;
  if (nmax > 32 || M > MFMA_KMAX) return AFQMC_E_UNSUPPORTED;
  t.precision = precision;
  t.NP = nmax <= 16 ? 16 : 32;
  t.KP = ((M + 31) / 32) * 32;
  t.M = M;
  t.G = G;
  t.nup = nup;
  t.ndn = ndn;
  const int nt = nup + ndn;
  const size_t per = (size_t)t.NP * t.KP;
  if (precision == AFQMC_FP32) {
    std::vector<float> h((size_t)2 * G * per + 1, 0.0f);
    for (int s = 0; s < 2; ++s) {
      const int N = s ? ndn : nup, off = s ? nup : 0;
      for (int g = 0; g < G; ++g)
        for (int r = 0; r < N; ++r)
          for (int p = 0; p < M; ++p)
            h[((size_t)s * G + g) * per + (size_t)r * t.KP + p] =
                (float)Lh[((size_t)g * nt + off + r) * M + p];
    }
    t.bytes = h.size() * sizeof(float);
    if (hipMalloc(&t.Lp, t.bytes) != hipSuccess) return AFQMC_E_NOMEM;
    if (hipMemcpy(t.Lp, h.data(), t.bytes, hipMemcpyHostToDevice) != hipSuccess) return AFQMC_E_HIP;
  } else if (precision == AFQMC_BF16X3) {
    std::vector<uint16_t> h((size_t)2 * G * 2 * per + 2, 0);
    for (int s = 0; s < 2; ++s) {
      const int N = s ? ndn : nup, off = s ? nup : 0;
      for (int g = 0; g < G; ++g)
        for (int r = 0; r < N; ++r)
          for (int p = 0; p < M; ++p) {
            const float x = (float)Lh[((size_t)g * nt + off + r) * M + p];
            const uint16_t hi = f32_to_bf16_bits(x);
            const uint16_t lo = f32_to_bf16_bits(x - bf16_bits_to_f32(hi));
            const size_t base = (((size_t)s * G + g) * 2) * per + (size_t)r * t.KP + p;
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

// ---------------------------------------------------------------------------
// Theta (FP64, rows of Theta^T) -> packed operand of the contraction.
// fp32:   [w][s][re/im][NP][KP] float
// bf16x3: [w][s][re/im][hi/lo][NP][KP] bf16 bits
// ---------------------------------------------------------------------------
template <bool BF16>
__global__ void __launch_bounds__(256) k_pack_theta(int nw, int M, int nup, int ndn, int NP, int KP,
                                                    const cd* __restrict__ thetaT,
                                                    const double* __restrict__ weight,
                                                    void* __restrict__ out) {
  const int ntot = nup + ndn;
  const size_t per = (size_t)NP * KP;
  const size_t total = (size_t)nw * 2 * per;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int p = (int)(e % KP);
  const int j = (int)((e / KP) % NP);
  const int s = (int)((e / per) % 2);
  const int w = (int)(e / (2 * per));
  if (!(weight[w] > 0.0)) return;
  const int N = s ? ndn : nup, off = s ? nup : 0;
  cd v = mkc(0.0, 0.0);
  if (j < N && p < M) v = thetaT[((size_t)w * ntot + off + j) * M + p];
  const size_t base = ((size_t)w * 2 + s) * 2 * (BF16 ? 2 : 1) * per + (size_t)j * KP + p;
  if (!BF16) {
    float* o = reinterpret_cast<float*>(out);
    o[base] = (float)v.re;
    o[base + per] = (float)v.im;
  } else {
    uint16_t* o = reinterpret_cast<uint16_t*>(out);
    const float xr = (float)v.re, xi = (float)v.im;
    const uint16_t hr = f32_to_bf16_bits(xr), hi = f32_to_bf16_bits(xi);
    o[base] = hr;
    o[base + per] = f32_to_bf16_bits(xr - bf16_bits_to_f32(hr));
    o[base + 2 * per] = hi;
    o[base + 3 * per] = f32_to_bf16_bits(xi - bf16_bits_to_f32(hi));
  }
}

// ---------------------------------------------------------------------------
// The contraction kernel.  Grid: (ceil(nw / 4), 2 spins); 256 threads.
// ---------------------------------------------------------------------------
template <int NP, bool BF16>
__global__ void __launch_bounds__(256, 2) k_contract_mfma(
    int nw, int G, int nup, int ndn, int KP, const void* __restrict__ Lp_,
    const void* __restrict__ thp_, const double* __restrict__ weight, cd* __restrict__ tpart,
    cd* __restrict__ exch) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int s = blockIdx.y;
  const int N = s ? ndn : nup;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int w = blockIdx.x * MFMA_WAVES + wave;
  const bool active = (w < nw) && (N > 0) && (weight[w] > 0.0);
  if (N == 0) {
    if (w < nw) {
      for (int g = lane; g < G; g += 64) tpart[((size_t)w * 2 + s) * G + g] = mkc(0.0, 0.0);
      if (lane == 0) exch[2 * w + s] = mkc(0.0, 0.0);
    }
    return;
  }
  // element sizes: fp32 tiles are floats; bf16 tiles are 2-byte values, hi and lo planes.
  constexpr int ESZ = BF16 ? 2 : 4;
  constexpr int PLANES = BF16 ? 2 : 1;
  const int lda = KP + (BF16 ? 8 : 4);                 // LDS row stride in elements (16 B pad)
  const size_t tile_elems = (size_t)NP * KP * PLANES;  // one g in global memory
  const int tile_lds_bytes = NP * lda * ESZ * PLANES;
  unsigned char* Abuf0 = smem;
  unsigned char* Abuf1 = smem + tile_lds_bytes;
  constexpr int LDE = NP + 4;
  float* ep = reinterpret_cast<float*>(smem + 2 * tile_lds_bytes) + (size_t)wave * 2 * NP * LDE;
  float* ep_re = ep;
  float* ep_im = ep + NP * LDE;

  const unsigned char* Lbase =
      reinterpret_cast<const unsigned char*>(Lp_) + (size_t)s * G * tile_elems * ESZ;

  // ---- copy of one g-tile global -> LDS, 16 bytes per thread per chunk
  const int chunks_per_row = KP * ESZ / 16;
  const int nchunks = NP * PLANES * chunks_per_row;
  constexpr int MAXCH = (32 * MFMA_KMAX * 4 + 255 * 16) / (256 * 16);  // 4
  u32x4 pre[MAXCH];
#define AFQMC_GLOAD(G_)                                                                        \
  do {                                                                                         \
    const u32x4* src_ = reinterpret_cast<const u32x4*>(Lbase + (size_t)(G_) * tile_elems * ESZ); \
    _Pragma("unroll") for (int c_ = 0; c_ < MAXCH; ++c_) {                                     \
      const int ch_ = tid + c_ * 256;                                                          \
      pre[c_] = src_[ch_ < nchunks ? ch_ : 0];                                                 \
    }                                                                                          \
  } while (0)
#define AFQMC_LSTORE(DST_)                                                                     \
  do {                                                                                         \
    _Pragma("unroll") for (int c_ = 0; c_ < MAXCH; ++c_) {                                     \
      const int ch_ = tid + c_ * 256;                                                          \
      if (ch_ < nchunks) {                                                                     \
        const int row_ = ch_ / chunks_per_row;                                                 \
        const int col_ = (ch_ % chunks_per_row) * (16 / ESZ);                                  \
        *reinterpret_cast<u32x4*>((DST_) + ((size_t)row_ * lda + col_) * ESZ) = pre[c_];       \
      }                                                                                        \
    }                                                                                          \
  } while (0)

  // ---- Theta operand into registers
  const int KCH = BF16 ? (NP == 32 ? 16 : 32) : (NP == 32 ? 8 : 16);  // K per register chunk
  const int nk = KP / KCH;
  constexpr int MAXK = BF16 ? (NP == 32 ? 8 : 4) : (NP == 32 ? 16 : 8);
  constexpr int LGRP = NP == 32 ? 32 : 16;  // lanes per K group
  const int col = lane % LGRP;              // row i of A / column j of B
  const int kg = lane / LGRP;               // K group of the lane
  const int kofs = BF16 ? 8 * kg : 4 * kg;  // element offset of the lane inside a K chunk

  u32x4 bre[MAXK], bim[MAXK];   // fp32: 4 floats;  bf16: 8 bf16 (hi)
  u32x4 bre_lo[BF16 ? MAXK : 1], bim_lo[BF16 ? MAXK : 1];
  if (active) {
    const size_t per = (size_t)NP * KP;
    const unsigned char* tb = reinterpret_cast<const unsigned char*>(thp_) +
                              ((size_t)w * 2 + s) * 2 * PLANES * per * ESZ;
#pragma unroll
    for (int c = 0; c < MAXK; ++c) {
      if (c < nk) {
        const size_t off = ((size_t)col * KP + c * KCH + kofs) * ESZ;
        bre[c] = *reinterpret_cast<const u32x4*>(tb + off);
        if (BF16) {
          bre_lo[BF16 ? c : 0] = *reinterpret_cast<const u32x4*>(tb + per * ESZ + off);
          bim[c] = *reinterpret_cast<const u32x4*>(tb + 2 * per * ESZ + off);
          bim_lo[BF16 ? c : 0] = *reinterpret_cast<const u32x4*>(tb + 3 * per * ESZ + off);
        } else {
          bim[c] = *reinterpret_cast<const u32x4*>(tb + per * ESZ + off);
        }
      }
    }
  }

  double xr = 0.0, xi = 0.0;
  if (G > 0) {
    AFQMC_GLOAD(0);
    AFQMC_LSTORE(Abuf0);
  }
  __syncthreads();
  for (int g = 0; g < G; ++g) {
    unsigned char* Acur = (g & 1) ? Abuf1 : Abuf0;
    unsigned char* Anext = (g & 1) ? Abuf0 : Abuf1;
    if (g + 1 < G) AFQMC_GLOAD(g + 1);
    const unsigned char* arow = Acur + ((size_t)col * lda + kofs) * ESZ;
    if constexpr (NP == 32) {
      f32x16 cre = {}, cim = {};
      if (active) {
#pragma unroll
        for (int c = 0; c < MAXK; ++c) {
          if (c < nk) {
            if constexpr (!BF16) {
              const f32x4 a = *reinterpret_cast<const f32x4*>(arow + (size_t)c * KCH * ESZ);
              const f32x4 br = __builtin_bit_cast(f32x4, bre[c]);
              const f32x4 bi = __builtin_bit_cast(f32x4, bim[c]);
              cre = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, br.x, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, bi.x, cim, 0, 0, 0);
              cre = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, br.y, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, bi.y, cim, 0, 0, 0);
              cre = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, br.z, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, bi.z, cim, 0, 0, 0);
              cre = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, br.w, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, bi.w, cim, 0, 0, 0);
            } else {
              const bf16x8 ah = __builtin_bit_cast(
                  bf16x8, *reinterpret_cast<const u32x4*>(arow + (size_t)c * KCH * ESZ));
              const bf16x8 al = __builtin_bit_cast(
                  bf16x8, *reinterpret_cast<const u32x4*>(arow + ((size_t)NP * lda + c * KCH) * ESZ));
              const bf16x8 brh = __builtin_bit_cast(bf16x8, bre[c]);
              const bf16x8 brl = __builtin_bit_cast(bf16x8, bre_lo[BF16 ? c : 0]);
              const bf16x8 bih = __builtin_bit_cast(bf16x8, bim[c]);
              const bf16x8 bil = __builtin_bit_cast(bf16x8, bim_lo[BF16 ? c : 0]);
              cre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, brh, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bih, cim, 0, 0, 0);
              cre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, brl, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bil, cim, 0, 0, 0);
              cre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, brh, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bih, cim, 0, 0, 0);
            }
          }
        }
        // column-major store of Omega: lane holds column j = col, rows 8*(v/4) + 4*kg + v%4
#pragma unroll
        for (int v4 = 0; v4 < 4; ++v4) {
          const int r0 = 8 * v4 + 4 * kg;
          *reinterpret_cast<float4*>(ep_re + col * LDE + r0) =
              make_float4(cre[4 * v4], cre[4 * v4 + 1], cre[4 * v4 + 2], cre[4 * v4 + 3]);
          *reinterpret_cast<float4*>(ep_im + col * LDE + r0) =
              make_float4(cim[4 * v4], cim[4 * v4 + 1], cim[4 * v4 + 2], cim[4 * v4 + 3]);
        }
      }
      __syncthreads();
      if (active) {
        float pr = 0.f, pi = 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int i = 8 * (v / 4) + 4 * kg + (v % 4);
          const float R = cre[v], I = cim[v];
          const float Rt = ep_re[i * LDE + col], It = ep_im[i * LDE + col];
          pr += R * Rt - I * It;
          pi += R * It + I * Rt;
        }
        xr += (double)pr;
        xi += (double)pi;
      }
    } else {
      f32x4 cre = {}, cim = {};
      if (active) {
#pragma unroll
        for (int c = 0; c < MAXK; ++c) {
          if (c < nk) {
            if constexpr (!BF16) {
              const f32x4 a = *reinterpret_cast<const f32x4*>(arow + (size_t)c * KCH * ESZ);
              const f32x4 br = __builtin_bit_cast(f32x4, bre[c]);
              const f32x4 bi = __builtin_bit_cast(f32x4, bim[c]);
              cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, br.x, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bi.x, cim, 0, 0, 0);
              cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, br.y, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bi.y, cim, 0, 0, 0);
              cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, br.z, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, bi.z, cim, 0, 0, 0);
              cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, br.w, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, bi.w, cim, 0, 0, 0);
            } else {
              const bf16x8 ah = __builtin_bit_cast(
                  bf16x8, *reinterpret_cast<const u32x4*>(arow + (size_t)c * KCH * ESZ));
              const bf16x8 al = __builtin_bit_cast(
                  bf16x8, *reinterpret_cast<const u32x4*>(arow + ((size_t)NP * lda + c * KCH) * ESZ));
              const bf16x8 brh = __builtin_bit_cast(bf16x8, bre[c]);
              const bf16x8 brl = __builtin_bit_cast(bf16x8, bre_lo[BF16 ? c : 0]);
              const bf16x8 bih = __builtin_bit_cast(bf16x8, bim[c]);
              const bf16x8 bil = __builtin_bit_cast(bf16x8, bim_lo[BF16 ? c : 0]);
              cre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, brh, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bih, cim, 0, 0, 0);
              cre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, brl, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bil, cim, 0, 0, 0);
              cre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, brh, cre, 0, 0, 0);
              cim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bih, cim, 0, 0, 0);
            }
          }
        }
        // lane holds column j = col, rows 4*kg + v
        *reinterpret_cast<float4*>(ep_re + col * LDE + 4 * kg) =
            make_float4(cre[0], cre[1], cre[2], cre[3]);
        *reinterpret_cast<float4*>(ep_im + col * LDE + 4 * kg) =
            make_float4(cim[0], cim[1], cim[2], cim[3]);
      }
      __syncthreads();
      if (active) {
        float pr = 0.f, pi = 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 4 * kg + v;
          const float R = cre[v], I = cim[v];
          const float Rt = ep_re[i * LDE + col], It = ep_im[i * LDE + col];
          pr += R * Rt - I * It;
          pi += R * It + I * Rt;
        }
        xr += (double)pr;
        xi += (double)pi;
      }
    }
    if (active) {
      // trace: lanes [0, NP) read Re Omega_jj, lanes [NP, 2NP) read Im Omega_jj
      float d = 0.f;
      if (lane < NP) d = ep_re[lane * LDE + lane];
      else if (lane < 2 * NP) d = ep_im[(lane - NP) * LDE + (lane - NP)];
#pragma unroll
      for (int o = NP / 2; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
      double* tp = reinterpret_cast<double*>(tpart + ((size_t)w * 2 + s) * G + g);
      if (lane == 0) tp[0] = (double)d;
      if (lane == NP) tp[1] = (double)d;
    }
    if (g + 1 < G) AFQMC_LSTORE(Anext);
    __syncthreads();
  }
  if (active) {
    xr = wave_sum(xr);
    xi = wave_sum(xi);
    if (lane == 0) exch[2 * w + s] = mkc(xr, xi);
  }
#undef AFQMC_GLOAD
#undef AFQMC_LSTORE
}

inline size_t mfma_contract_lds_bytes(const MfmaTables& t) {
  const bool bf = t.precision == AFQMC_BF16X3;
  const int esz = bf ? 2 : 4, planes = bf ? 2 : 1;
  const int lda = t.KP + (bf ? 8 : 4);
  const size_t tile = (size_t)t.NP * lda * esz * planes;
  return 2 * tile + (size_t)MFMA_WAVES * 2 * t.NP * (t.NP + 4) * 4;
}

inline hipError_t mfma_pack_theta(const MfmaTables& t, hipStream_t st, int nw, int M, int nup,
                                  int ndn, const cd* thetaT, const double* weight, void* out) {
  const size_t total = (size_t)nw * 2 * t.NP * t.KP;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (t.precision == AFQMC_BF16X3)
    hipLaunchKernelGGL(k_pack_theta<true>, dim3(blocks), dim3(256), 0, st, nw, M, nup, ndn, t.NP,
                       t.KP, thetaT, weight, out);
  else
    hipLaunchKernelGGL(k_pack_theta<false>, dim3(blocks), dim3(256), 0, st, nw, M, nup, ndn, t.NP,
                       t.KP, thetaT, weight, out);
  return hipGetLastError();
}

inline hipError_t mfma_contract(const MfmaTables& t, hipStream_t st, int nw, int G,
                                const void* thetaP, const double* weight, cd* tpart, cd* exch) {
  const size_t shm = mfma_contract_lds_bytes(t);
  dim3 grid((nw + MFMA_WAVES - 1) / MFMA_WAVES, 2);
  const bool bf = t.precision == AFQMC_BF16X3;
#define LAUNCH_CONTRACT(NPV, BFV)                                                               \
  do {                                                                                          \
    (void)hipFuncSetAttribute((const void*)k_contract_mfma<NPV, BFV>,                           \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);            \
    hipLaunchKernelGGL((k_contract_mfma<NPV, BFV>), grid, dim3(256), shm, st, nw, G, t.nup,     \
                       t.ndn, t.KP, (const void*)t.Lp, thetaP, weight, tpart, exch);            \
  } while (0)
  if (t.NP == 32) {
    if (bf) LAUNCH_CONTRACT(32, true);
    else LAUNCH_CONTRACT(32, false);
  } else {
    if (bf) LAUNCH_CONTRACT(16, true);
    else LAUNCH_CONTRACT(16, false);
  }
#undef LAUNCH_CONTRACT
  return hipGetLastError();
}
