// The FP32 / BF16x3 MFMA local-energy contraction kernel (arXiv:1711.02242,
// Sec. III.D.3, eq:localenergy3; force-bias traces of eq:precomputing2).
// Types, tables and launchers are in kernels_mfma.hpp, which includes this file;
// the kernel sits in a file of its own so that its source can be identified
// exactly by the hardware-counter measurements taken on it.
//
// For every walker w, spin s and Cholesky index g:
//   Omega = Lh^g_s Theta_s     (N x N complex = real N x M times complex M x N)
//   tpart[w][s][g] = tr Omega,  exch[w][s] = sum_g tr(Omega Omega).
// One wavefront owns one walker-spin and keeps [Re Theta | Im Theta] (M x 2N)
// in registers for the whole kernel; the WPB wavefronts of a workgroup (WPB
// walkers of the same spin, WPB = 4 or 2) stream the shared tiles Lh^g_s (N x M)
// through double-buffered LDS.  Per g the wave runs the MFMA chain over K = M for the
// Re and Im halves, then an LDS transpose through the wave's own planes gives every
// lane the partner element Omega_ji of each Omega_ij it holds (a wavefront fence, not a
// workgroup barrier, orders it; one barrier per g guards the shared tile buffers).  Per-g partial products are summed in
// FP32 and accumulated across g in FP64.
#pragma once

// Orders a wave's LDS stores before its later LDS loads of other lanes' elements (the
// per-wave Omega planes): wavefront-scope release / acquire, no workgroup barrier.
__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// The contraction kernel.  Grid: (ceil(nw / WPB), 2 n_det); 64 WPB threads.
// ---------------------------------------------------------------------------
template <int NP, bool BF16, int WPB>
__global__ void __launch_bounds__(64 * WPB, 2) k_contract_mfma(
    int nw, int G, int nup, int ndn, int KP, const void* __restrict__ Lp_,
    const void* __restrict__ thp_, const double* __restrict__ weight, cd* __restrict__ tpart,
    cd* __restrict__ exch) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  // blockIdx.y = 2 d + s: determinant d of the trial, spin s
  const int s = blockIdx.y & 1, dd = blockIdx.y >> 1, n_det = gridDim.y >> 1;
  const int N = s ? ndn : nup;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int NT = 64 * WPB;
  const int w = blockIdx.x * WPB + wave;
  const int wd = w * n_det + dd;   // (walker, determinant) slot of the outputs
  const bool active = (w < nw) && (N > 0) && (weight[w] > 0.0);
  if (N == 0) {
    if (w < nw) {
      for (int g = lane; g < G; g += 64) tpart[((size_t)wd * 2 + s) * G + g] = mkc(0.0, 0.0);
      if (lane == 0) exch[2 * wd + s] = mkc(0.0, 0.0);
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
      reinterpret_cast<const unsigned char*>(Lp_) + ((size_t)dd * 2 + s) * G * tile_elems * ESZ;

  // ---- copy of one g-tile global -> LDS, 16 bytes per thread per chunk
  const int chunks_per_row = KP * ESZ / 16;
  const int nchunks = NP * PLANES * chunks_per_row;
  constexpr int MAXCH = (32 * MFMA_KMAX * 4 / 16 + NT - 1) / NT;  // 4 (WPB 4), 8 (WPB 2)
  u32x4 pre[MAXCH];
#define AFQMC_GLOAD(G_)                                                                        \
  do {                                                                                         \
    const u32x4* src_ = reinterpret_cast<const u32x4*>(Lbase + (size_t)(G_) * tile_elems * ESZ); \
    _Pragma("unroll") for (int c_ = 0; c_ < MAXCH; ++c_) {                                     \
      const int ch_ = tid + c_ * NT;                                                           \
      pre[c_] = src_[ch_ < nchunks ? ch_ : 0];                                                 \
    }                                                                                          \
  } while (0)
#define AFQMC_LSTORE(DST_)                                                                     \
  do {                                                                                         \
    _Pragma("unroll") for (int c_ = 0; c_ < MAXCH; ++c_) {                                     \
      const int ch_ = tid + c_ * NT;                                                           \
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
                              ((size_t)wd * 2 + s) * 2 * PLANES * per * ESZ;
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
    // FP32: the next tile's loads are unconditional (the last g re-reads its own tile), so
    // the waits placed before the MFMAs do not stall on them (3 % faster); BF16x3 keeps the
    // conditional form, which measures 3 % faster there
    if constexpr (BF16) {
      if (g + 1 < G) AFQMC_GLOAD(g + 1);
    } else {
      AFQMC_GLOAD(g + 1 < G ? g + 1 : g);
    }
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
      wave_lds_fence();   // each wave reads back only its own Omega planes
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
      wave_lds_fence();   // each wave reads back only its own Omega planes
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
      double* tp = reinterpret_cast<double*>(tpart + ((size_t)wd * 2 + s) * G + g);
      if (lane == 0) tp[0] = (double)d;
      if (lane == NP) tp[1] = (double)d;
    }
    if (g + 1 < G) AFQMC_LSTORE(Anext);
    __syncthreads();
  }
  if (active) {
    xr = wave_sum(xr);
    xi = wave_sum(xi);
    if (lane == 0) exch[2 * wd + s] = mkc(xr, xi);
  }
#undef AFQMC_GLOAD
#undef AFQMC_LSTORE
}

