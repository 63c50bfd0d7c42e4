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
// workgroup barrier, orders it; one barrier per g guards the shared tile buffers).
// Per-g partial products are summed in FP32 and accumulated across g in FP64; tr Omega
// is summed over the lanes by DPP row shifts (no LDS round trips).
#pragma once

// Orders a wave's LDS stores before its later LDS loads of other lanes' elements (the
// per-wave Omega planes): wavefront-scope release / acquire, no workgroup barrier.
__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One term of tr(Omega Omega): the lane's Omega_ij = R + i I times its partner
// Omega_ji = Rt + i It, accumulated into (pr, pi) by four FMAs (the fewest vector
// instructions: on the matrix-core SIMDs vector work adds to the MFMA time).  The FMAs are
// explicit so that the rounding is the same in every kernel that uses them.
__device__ __forceinline__ void exch_term(float R, float I, float Rt, float It, float& pr,
                                          float& pi) {
  pr = __builtin_fmaf(R, Rt, pr);
  pr = __builtin_fmaf(-I, It, pr);
  pi = __builtin_fmaf(R, It, pi);
  pi = __builtin_fmaf(I, Rt, pi);
}

// One K chunk of Omega = Lh Theta for the Re and Im halves.  FP32: a holds four K values of
// one row of Lh (one per MFMA step), br / bi four K values of one column of Re / Im Theta.
// BF16x3: a / al the hi / lo bf16 of eight K values, br / brl and bi / bil likewise; the
// three products hi.hi + hi.lo + lo.hi.
// FIRST: the chunk starts Omega, so its first products take a zero accumulator (an inline
// constant of the MFMA instead of clearing the accumulator registers with vector moves).
template <int NP, bool BF16, bool FIRST = false, typename Acc>
__device__ __forceinline__ void contract_chunk(u32x4 ah, u32x4 al, u32x4 brh, u32x4 brl,
                                               u32x4 bih, u32x4 bil, Acc& cre, Acc& cim) {
  if constexpr (!BF16) {
    const f32x4 a = __builtin_bit_cast(f32x4, ah);
    const f32x4 br = __builtin_bit_cast(f32x4, brh);
    const f32x4 bi = __builtin_bit_cast(f32x4, bih);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const Acc cr = FIRST && k == 0 ? Acc{} : cre, ci = FIRST && k == 0 ? Acc{} : cim;
      if constexpr (NP == 32) {
        cre = __builtin_amdgcn_mfma_f32_32x32x2f32(a[k], br[k], cr, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_32x32x2f32(a[k], bi[k], ci, 0, 0, 0);
      } else {
        cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], br[k], cr, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], bi[k], ci, 0, 0, 0);
      }
    }
  } else {
    const bf16x8 h = __builtin_bit_cast(bf16x8, ah), l = __builtin_bit_cast(bf16x8, al);
    const bf16x8 rh = __builtin_bit_cast(bf16x8, brh), rl = __builtin_bit_cast(bf16x8, brl);
    const bf16x8 ih = __builtin_bit_cast(bf16x8, bih), il = __builtin_bit_cast(bf16x8, bil);
    if constexpr (FIRST) {
      cre = Acc{};
      cim = Acc{};
    }
    if constexpr (NP == 32) {
      cre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(l, rh, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(l, ih, cim, 0, 0, 0);
      cre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h, rl, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h, il, cim, 0, 0, 0);
      cre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h, rh, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h, ih, cim, 0, 0, 0);
    } else {
      cre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l, rh, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l, ih, cim, 0, 0, 0);
      cre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, rl, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, il, cim, 0, 0, 0);
      cre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, rh, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, ih, cim, 0, 0, 0);
    }
  }
}

// K values per register chunk of the contraction kernel: FP32 4 MFMA steps (2 or 4 K each),
// BF16x3 one step (16 or 32 K).
template <int NP, bool BF16>
constexpr int contract_kch() {
  return BF16 ? (NP == 32 ? 16 : 32) : (NP == 32 ? 8 : 16);
}

// ---------------------------------------------------------------------------
// The contraction kernel.  Grid: (ceil(nw / WPB), 2 n_det); 64 WPB threads.  NK = K_P / KCH
// register chunks of K (compile time: no per-chunk branches, and the A fragment of chunk
// c + 1 is read from LDS while the MFMAs of chunk c run).
// ---------------------------------------------------------------------------
template <int NP, bool BF16, int WPB, int NK>
__global__ void __launch_bounds__(64 * WPB, 2) k_contract_mfma(
    int nw, int G, int nup, int ndn, int KP_arg, const void* __restrict__ Lp_,
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
  constexpr int KCH = contract_kch<NP, BF16>();
  constexpr int KP = NK * KCH;                          // K_P (the launcher passes it as KP_arg)
  (void)KP_arg;
  constexpr int lda = KP + (BF16 ? 8 : 4);              // LDS row stride in elements (16 B pad)
  constexpr size_t tile_elems = (size_t)NP * KP * PLANES;  // one g in global memory
  constexpr int tile_lds_bytes = NP * lda * ESZ * PLANES;
  unsigned char* Abuf0 = smem;
  unsigned char* Abuf1 = smem + tile_lds_bytes;
  constexpr int LDE = NP + 4;
  float* ep = reinterpret_cast<float*>(smem + 2 * tile_lds_bytes) + (size_t)wave * 2 * NP * LDE;
  float* ep_re = ep;
  float* ep_im = ep + NP * LDE;

  const unsigned char* Lbase =
      reinterpret_cast<const unsigned char*>(Lp_) + ((size_t)dd * 2 + s) * G * tile_elems * ESZ;

  // ---- copy of one g-tile global -> LDS, 16 bytes per thread per chunk
  constexpr int chunks_per_row = KP * ESZ / 16;
  constexpr int nchunks = NP * PLANES * chunks_per_row;
  constexpr int MAXCH = (nchunks + NT - 1) / NT;   // 16-byte chunks per thread
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
      if ((c_ + 1) * NT <= nchunks || ch_ < nchunks) {                                         \
        const int row_ = ch_ / chunks_per_row;                                                 \
        const int col_ = (ch_ % chunks_per_row) * (16 / ESZ);                                  \
        *reinterpret_cast<u32x4*>((DST_) + ((size_t)row_ * lda + col_) * ESZ) = pre[c_];       \
      }                                                                                        \
    }                                                                                          \
  } while (0)

  // ---- Theta operand into registers
  constexpr int LGRP = NP == 32 ? 32 : 16;  // lanes per K group
  const int col = lane % LGRP;              // row i of A / column j of B
  const int kg = lane / LGRP;               // K group of the lane
  const int kofs = BF16 ? 8 * kg : 4 * kg;  // element offset of the lane inside a K chunk

  u32x4 bre[NK], bim[NK];   // fp32: 4 floats;  bf16: 8 bf16 (hi)
  u32x4 bre_lo[BF16 ? NK : 1], bim_lo[BF16 ? NK : 1];
  if (active) {
    const size_t per = (size_t)NP * KP;
    const unsigned char* tb = reinterpret_cast<const unsigned char*>(thp_) +
                              ((size_t)wd * 2 + s) * 2 * PLANES * per * ESZ;
#pragma unroll
    for (int c = 0; c < NK; ++c) {
      const size_t off = ((size_t)col * KP + c * KCH + kofs) * ESZ;
      bre[c] = *reinterpret_cast<const u32x4*>(tb + off);
      if constexpr (BF16) {
        bre_lo[c] = *reinterpret_cast<const u32x4*>(tb + per * ESZ + off);
        bim[c] = *reinterpret_cast<const u32x4*>(tb + 2 * per * ESZ + off);
        bim_lo[c] = *reinterpret_cast<const u32x4*>(tb + 3 * per * ESZ + off);
      } else {
        bim[c] = *reinterpret_cast<const u32x4*>(tb + per * ESZ + off);
      }
    }
  }

  using Acc = typename std::conditional<NP == 32, f32x16, f32x4>::type;
  constexpr int NV = NP == 32 ? 16 : 4;   // accumulator elements per lane
  double xr = 0.0, xi = 0.0;
  if (G > 0) {
    AFQMC_GLOAD(0);
    AFQMC_LSTORE(Abuf0);
  }
  // every global load so far (Theta, the first tile) complete here: otherwise the waits for
  // the Theta registers land inside the g loop, where they also wait for the next tile
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  __syncthreads();
  for (int g = 0; g < G; ++g) {
    unsigned char* Acur = (g & 1) ? Abuf1 : Abuf0;
    unsigned char* Anext = (g & 1) ? Abuf0 : Abuf1;
    // FP32: the next tile's loads are unconditional (the last g re-reads its own tile), so
    // the waits placed before the MFMAs do not stall on them; BF16x3 keeps the conditional
    // form, which measures faster there
    if constexpr (BF16) {
      if (g + 1 < G) AFQMC_GLOAD(g + 1);
    } else {
      AFQMC_GLOAD(g + 1 < G ? g + 1 : g);
    }
    const unsigned char* arow = Acur + ((size_t)col * lda + kofs) * ESZ;
    const size_t lo_ofs = (size_t)NP * lda * ESZ;   // bf16: lo plane of the tile
    Acc cre, cim;   // set by the first chunk (read only by active waves)
    if (active) {
      if constexpr (WPB == 4) {
        // A fragment of chunk c + 1 read while chunk c's MFMAs run; the scheduling barrier
        // keeps the compiler from regrouping the reads (it pairs chunks and waits at once)
        u32x4 ah = *reinterpret_cast<const u32x4*>(arow);
        u32x4 al = BF16 ? *reinterpret_cast<const u32x4*>(arow + lo_ofs) : ah;
#pragma unroll
        for (int c = 0; c < NK; ++c) {
          u32x4 nh = ah, nl = al;
          if (c + 1 < NK) {
            nh = *reinterpret_cast<const u32x4*>(arow + (size_t)(c + 1) * KCH * ESZ);
            if constexpr (BF16)
              nl = *reinterpret_cast<const u32x4*>(arow + lo_ofs + (size_t)(c + 1) * KCH * ESZ);
          }
          if (c == 0)
            contract_chunk<NP, BF16, true>(ah, al, bre[c], bre_lo[BF16 ? c : 0], bim[c],
                                           bim_lo[BF16 ? c : 0], cre, cim);
          else
            contract_chunk<NP, BF16>(ah, al, bre[c], bre_lo[BF16 ? c : 0], bim[c],
                                     bim_lo[BF16 ? c : 0], cre, cim);
          __builtin_amdgcn_sched_barrier(0);
          ah = nh;
          al = nl;
        }
      } else {
        // two walkers per workgroup hold twice the tile-copy registers: no room for a
        // second A fragment
#pragma unroll
        for (int c = 0; c < NK; ++c) {
          const u32x4 ah = *reinterpret_cast<const u32x4*>(arow + (size_t)c * KCH * ESZ);
          const u32x4 al =
              BF16 ? *reinterpret_cast<const u32x4*>(arow + lo_ofs + (size_t)c * KCH * ESZ) : ah;
          if (c == 0)
            contract_chunk<NP, BF16, true>(ah, al, bre[c], bre_lo[BF16 ? c : 0], bim[c],
                                           bim_lo[BF16 ? c : 0], cre, cim);
          else
            contract_chunk<NP, BF16>(ah, al, bre[c], bre_lo[BF16 ? c : 0], bim[c],
                                     bim_lo[BF16 ? c : 0], cre, cim);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      // column-major store of Omega: lane holds column j = col, rows
      // 8*(v/4) + 4*kg + v%4 (32 x 32) or 4*kg + v (16 x 16)
#pragma unroll
      for (int v4 = 0; v4 < NV / 4; ++v4) {
        const int r0 = (NP == 32 ? 8 * v4 : 0) + 4 * kg;
        *reinterpret_cast<float4*>(ep_re + col * LDE + r0) =
            make_float4(cre[4 * v4], cre[4 * v4 + 1], cre[4 * v4 + 2], cre[4 * v4 + 3]);
        *reinterpret_cast<float4*>(ep_im + col * LDE + r0) =
            make_float4(cim[4 * v4], cim[4 * v4 + 1], cim[4 * v4 + 2], cim[4 * v4 + 3]);
      }
    }
    wave_lds_fence();   // each wave reads back only its own Omega planes
    if (active) {
      // the diagonal (lanes [0, NP): Re Omega_jj, lanes [NP, 2NP): Im) and the partner
      // element Omega_ji of every Omega_ij the lane holds; with four walkers per workgroup
      // all are read before any is used (two per workgroup leave no registers for that)
      const int dl = lane < 2 * NP ? lane : 2 * NP - 1;
      float d = dl < NP ? ep_re[dl * (LDE + 1)] : ep_im[(dl - NP) * (LDE + 1)];
      float pr = 0.f, pi = 0.f;
      if constexpr (WPB == 4) {
        float Rt[NV], It[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int i = (NP == 32 ? 8 * (v / 4) : 0) + 4 * kg + (v % 4);
          Rt[v] = ep_re[i * LDE + col];
          It[v] = ep_im[i * LDE + col];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int v = 0; v < NV; ++v) exch_term(cre[v], cim[v], Rt[v], It[v], pr, pi);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int i = (NP == 32 ? 8 * (v / 4) : 0) + 4 * kg + (v % 4);
          exch_term(cre[v], cim[v], ep_re[i * LDE + col], ep_im[i * LDE + col], pr, pi);
        }
      }
      xr += (double)pr;
      xi += (double)pi;
      // trace: Re in lane NP - 1, Im in lane 2 NP - 1
      d = NP == 32 ? dpp_half_sum(d) : dpp_row_sum(d);
      double* tp = reinterpret_cast<double*>(tpart + ((size_t)wd * 2 + s) * G + g);
      if (lane == NP - 1) tp[0] = (double)d;
      if (lane == 2 * NP - 1) tp[1] = (double)d;
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
