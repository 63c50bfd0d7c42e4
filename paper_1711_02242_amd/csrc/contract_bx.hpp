// FP32 / BF16x3 MFMA local-energy contraction with the exchange split by 16 x 16 blocks
// (arXiv:1711.02242, Sec. III.D.3, eq:localenergy3; force-bias traces of eq:precomputing2), for
// N_P = 32.
// Included by kernels_mfma.hpp after contract_mfma.hpp.
//
// As in k_contract_mfma, one wavefront owns one walker-spin and keeps Theta in registers, and
// the four wavefronts of a workgroup stream the tiles Lh^g (N_P x K_P) through double-buffered
// LDS.  Omega = Lh^g Theta is computed as four 16 x 16 blocks on v_mfma_f32_16x16x4_f32
// (BF16x3: v_mfma_f32_16x16x32_bf16, three products lo.hi + hi.lo + hi.hi per block),
//     Omega = [[A, B], [C, D]],   tr(Omega Omega) = tr(A A) + tr(D D) + 2 tr(B C),
// with C produced transposed: C^T = Theta_L^T Lh_low^T is the same MFMA with its two operand
// registers swapped, so it costs nothing extra and lands in B's lane layout.  tr(B C) =
// sum_ij B_ij (C^T)_ij is then a lane-local product; only the diagonal blocks go through LDS for
// their transposes, as one float4 per element (Re A, Im A, Re D, Im D interleaved), four
// 16-byte stores and four 16-byte loads per g at immediate offsets from one base address.
// That is about half the LDS instructions and a quarter fewer vector FMAs than the 32 x 32
// form, and on the matrix-core SIMDs both add to the MFMA time.
#pragma once

// WPB walkers per workgroup (4 or 8; two wavefronts per SIMD either way): eight share each
// tile copy and barrier among twice the walkers.
template <bool BF16, int NK, int WPB>
__global__ void __launch_bounds__(64 * WPB, 8 / WPB) k_contract_mfma_bx(
    int nw, int G, int nup, int ndn, const void* __restrict__ Lp_, const void* __restrict__ thp_,
    const double* __restrict__ weight, cd* __restrict__ tpart, cd* __restrict__ exch) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int NP = 32, NT = 64 * WPB;
  constexpr int ESZ = BF16 ? 2 : 4, PLANES = BF16 ? 2 : 1;
  constexpr int KCH = BF16 ? 32 : 16;     // K per chunk: FP32 4 MFMA steps of 4, BF16 one of 32
  constexpr int KP = NK * KCH;
  constexpr int lda = KP + (BF16 ? 8 : 4);   // LDS row stride of the tile (elements)
  constexpr size_t tile_elems = (size_t)NP * KP * PLANES;
  constexpr int tile_lds_bytes = NP * lda * ESZ * PLANES;
  constexpr int LDX = 17;                 // row stride of the transpose planes, in float4
  const int s = blockIdx.y & 1, dd = blockIdx.y >> 1, n_det = gridDim.y >> 1;
  const int N = s ? ndn : nup;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int w = blockIdx.x * WPB + wave;
  const int wd = w * n_det + dd;
  const bool active = (w < nw) && (N > 0) && (weight[w] > 0.0);
  if (N == 0) {
    if (w < nw) {
      for (int g = lane; g < G; g += 64) tpart[((size_t)wd * 2 + s) * G + g] = mkc(0.0, 0.0);
      if (lane == 0) exch[2 * wd + s] = mkc(0.0, 0.0);
    }
    return;
  }
  unsigned char* Abuf0 = smem;
  unsigned char* Abuf1 = smem + tile_lds_bytes;
  // [16 rows][LDX][Re A, Im A, Re D, Im D] per wave
  float* ep = reinterpret_cast<float*>(smem + 2 * tile_lds_bytes) + (size_t)wave * 16 * LDX * 4;
  const unsigned char* Lbase =
      reinterpret_cast<const unsigned char*>(Lp_) + ((size_t)dd * 2 + s) * G * tile_elems * ESZ;

  // ---- copy of one g-tile global -> LDS, 16 bytes per thread per chunk
  constexpr int chunks_per_row = KP * ESZ / 16;
  constexpr int nchunks = NP * PLANES * chunks_per_row;
  constexpr int MAXCH = (nchunks + NT - 1) / NT;
  u32x4 pre[MAXCH];
  auto gload = [&](int g_) {
    const u32x4* src = reinterpret_cast<const u32x4*>(Lbase + (size_t)g_ * tile_elems * ESZ);
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) {
      const int ch = tid + c * NT;
      pre[c] = src[ch < nchunks ? ch : 0];
    }
  };
  auto lstore = [&](unsigned char* dst) {
#pragma unroll
    for (int c = 0; c < MAXCH; ++c) {
      const int ch = tid + c * NT;
      if ((c + 1) * NT <= nchunks || ch < nchunks) {
        const int row = ch / chunks_per_row;
        const int cl = (ch % chunks_per_row) * (16 / ESZ);
        *reinterpret_cast<u32x4*>(dst + ((size_t)row * lda + cl) * ESZ) = pre[c];
      }
    }
  };

  // ---- Theta: columns j (left block) and 16 + j (right block), the lane's K values of each
  // chunk (FP32 16 c + 4 kq .. + 3, BF16 32 c + 8 kq .. + 7; BF16x3: hi and lo planes)
  const int j = lane & 15, kq = lane >> 4;
  const int kofs = BF16 ? 8 * kq : 4 * kq;
  u32x4 tLr[NK], tLi[NK], tRr[NK], tRi[NK];
  u32x4 tLr_lo[BF16 ? NK : 1], tLi_lo[BF16 ? NK : 1], tRr_lo[BF16 ? NK : 1], tRi_lo[BF16 ? NK : 1];
  if (active) {
    const size_t per = (size_t)NP * KP * ESZ;   // bytes of one plane
    const unsigned char* tb = reinterpret_cast<const unsigned char*>(thp_) +
                              ((size_t)wd * 2 + s) * 2 * PLANES * per;
    // planes: FP32 Re, Im; BF16x3 Re hi, Re lo, Im hi, Im lo
    constexpr int IM = BF16 ? 2 : 1;
#pragma unroll
    for (int c = 0; c < NK; ++c) {
      const size_t oL = ((size_t)j * KP + c * KCH + kofs) * ESZ;
      const size_t oR = ((size_t)(16 + j) * KP + c * KCH + kofs) * ESZ;
      tLr[c] = *reinterpret_cast<const u32x4*>(tb + oL);
      tLi[c] = *reinterpret_cast<const u32x4*>(tb + IM * per + oL);
      tRr[c] = *reinterpret_cast<const u32x4*>(tb + oR);
      tRi[c] = *reinterpret_cast<const u32x4*>(tb + IM * per + oR);
      if constexpr (BF16) {
        tLr_lo[c] = *reinterpret_cast<const u32x4*>(tb + per + oL);
        tLi_lo[c] = *reinterpret_cast<const u32x4*>(tb + 3 * per + oL);
        tRr_lo[c] = *reinterpret_cast<const u32x4*>(tb + per + oR);
        tRi_lo[c] = *reinterpret_cast<const u32x4*>(tb + 3 * per + oR);
      }
    }
  }

  double xr = 0.0, xi = 0.0;
  if (G > 0) {
    gload(0);
    lstore(Abuf0);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): Theta and the first tile
  __syncthreads();
  for (int g = 0; g < G; ++g) {
    unsigned char* Acur = (g & 1) ? Abuf1 : Abuf0;
    unsigned char* Anext = (g & 1) ? Abuf0 : Abuf1;
    gload(g + 1 < G ? g + 1 : g);   // unconditional: the waits before the MFMAs skip it
    if (active) {
      // A fragments: rows j (upper block) and 16 + j (lower block) of Lh^g
      const unsigned char* up = Acur + ((size_t)j * lda + kofs) * ESZ;
      const unsigned char* lo = up + (size_t)16 * lda * ESZ;
      const size_t lo_ofs = (size_t)NP * lda * ESZ;   // BF16x3: lo plane of the tile
      f32x4 Ar, Ai, Br, Bi, Cr, Ci, Dr, Di;   // C holds C^T
      u32x4 au = *reinterpret_cast<const u32x4*>(up);
      u32x4 al = *reinterpret_cast<const u32x4*>(lo);
      u32x4 au_lo = BF16 ? *reinterpret_cast<const u32x4*>(up + lo_ofs) : au;
      u32x4 al_lo = BF16 ? *reinterpret_cast<const u32x4*>(lo + lo_ofs) : al;
#pragma unroll
      for (int c = 0; c < NK; ++c) {
        u32x4 nu = au, nl = al, nu_lo = au_lo, nl_lo = al_lo;
        if (c + 1 < NK) {
          const size_t o = (size_t)(c + 1) * KCH * ESZ;
          nu = *reinterpret_cast<const u32x4*>(up + o);
          nl = *reinterpret_cast<const u32x4*>(lo + o);
          if constexpr (BF16) {
            nu_lo = *reinterpret_cast<const u32x4*>(up + lo_ofs + o);
            nl_lo = *reinterpret_cast<const u32x4*>(lo + lo_ofs + o);
          }
        }
        if constexpr (!BF16) {
          const f32x4 u = __builtin_bit_cast(f32x4, au), l = __builtin_bit_cast(f32x4, al);
          const f32x4 lr = __builtin_bit_cast(f32x4, tLr[c]), li = __builtin_bit_cast(f32x4, tLi[c]);
          const f32x4 rr = __builtin_bit_cast(f32x4, tRr[c]), ri = __builtin_bit_cast(f32x4, tRi[c]);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const bool z = c == 0 && t == 0;   // the first products start from zero
            Ar = __builtin_amdgcn_mfma_f32_16x16x4f32(u[t], lr[t], z ? f32x4{} : Ar, 0, 0, 0);
            Ai = __builtin_amdgcn_mfma_f32_16x16x4f32(u[t], li[t], z ? f32x4{} : Ai, 0, 0, 0);
            Br = __builtin_amdgcn_mfma_f32_16x16x4f32(u[t], rr[t], z ? f32x4{} : Br, 0, 0, 0);
            Bi = __builtin_amdgcn_mfma_f32_16x16x4f32(u[t], ri[t], z ? f32x4{} : Bi, 0, 0, 0);
            Cr = __builtin_amdgcn_mfma_f32_16x16x4f32(lr[t], l[t], z ? f32x4{} : Cr, 0, 0, 0);
            Ci = __builtin_amdgcn_mfma_f32_16x16x4f32(li[t], l[t], z ? f32x4{} : Ci, 0, 0, 0);
            Dr = __builtin_amdgcn_mfma_f32_16x16x4f32(l[t], rr[t], z ? f32x4{} : Dr, 0, 0, 0);
            Di = __builtin_amdgcn_mfma_f32_16x16x4f32(l[t], ri[t], z ? f32x4{} : Di, 0, 0, 0);
          }
        } else {
          // three products per block, the two small cross terms first: X += a_lo b_hi +
          // a_hi b_lo + a_hi b_hi (C^T: Theta as the first operand, Lh as the second)
          const bf16x8 uh = __builtin_bit_cast(bf16x8, au), ul = __builtin_bit_cast(bf16x8, au_lo);
          const bf16x8 lh = __builtin_bit_cast(bf16x8, al), ll = __builtin_bit_cast(bf16x8, al_lo);
          auto prod3 = [&](bf16x8 ah, bf16x8 al_, u32x4 bh, u32x4 bl, f32x4& x) {
            const bf16x8 h = __builtin_bit_cast(bf16x8, bh), l_ = __builtin_bit_cast(bf16x8, bl);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al_, h, c == 0 ? f32x4{} : x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, l_, x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, h, x, 0, 0, 0);
          };
          auto prod3t = [&](u32x4 th, u32x4 tl, bf16x8 bh, bf16x8 bl, f32x4& x) {
            const bf16x8 h = __builtin_bit_cast(bf16x8, th), l_ = __builtin_bit_cast(bf16x8, tl);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bl, c == 0 ? f32x4{} : x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l_, bh, x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bh, x, 0, 0, 0);
          };
          prod3(uh, ul, tLr[c], tLr_lo[c], Ar);
          prod3(uh, ul, tLi[c], tLi_lo[c], Ai);
          prod3(uh, ul, tRr[c], tRr_lo[c], Br);
          prod3(uh, ul, tRi[c], tRi_lo[c], Bi);
          prod3t(tLr[c], tLr_lo[c], lh, ll, Cr);
          prod3t(tLi[c], tLi_lo[c], lh, ll, Ci);
          prod3(lh, ll, tRr[c], tRr_lo[c], Dr);
          prod3(lh, ll, tRi[c], tRi_lo[c], Di);
        }
        __builtin_amdgcn_sched_barrier(0);
        au = nu;
        al = nl;
        au_lo = nu_lo;
        al_lo = nl_lo;
      }
      // the lane holds block column j, rows 4 kq + v; element (i, j) of A and D goes to
      // ep[i][j][0..3] and its partner (j, i) comes back from ep[j][i][0..3]
      float* mine = ep + ((size_t)(4 * kq) * LDX + j) * 4;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        *reinterpret_cast<float4*>(mine + (size_t)v * LDX * 4) = make_float4(Ar[v], Ai[v], Dr[v], Di[v]);
      wave_lds_fence();   // the wave reads back only its own planes
      const float* part = ep + ((size_t)j * LDX + 4 * kq) * 4;
      float4 P[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) P[v] = *reinterpret_cast<const float4*>(part + v * 4);
      // diagonals: lanes 0-15 Re A, 16-31 Re D, 32-47 Im A, 48-63 Im D
      const int dp = ((lane >> 4) & 1) * 2 + (lane >> 5);
      float d = ep[((size_t)j * LDX + j) * 4 + dp];
      __builtin_amdgcn_sched_barrier(0);
      float pr = 0.f, pi = 0.f, qr = 0.f, qi = 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        exch_term(Ar[v], Ai[v], P[v].x, P[v].y, pr, pi);
        exch_term(Dr[v], Di[v], P[v].z, P[v].w, pr, pi);
        exch_term(Br[v], Bi[v], Cr[v], Ci[v], qr, qi);
      }
      xr += (double)__builtin_fmaf(2.f, qr, pr);
      xi += (double)__builtin_fmaf(2.f, qi, pi);
      // trace: Re in lane 31 (A + D), Im in lane 63
      d = dpp_half_sum(d);
      double* tp = reinterpret_cast<double*>(tpart + ((size_t)wd * 2 + s) * G + g);
      if (lane == 31) tp[0] = (double)d;
      if (lane == 63) tp[1] = (double)d;
      // the next g's stores to the planes come after every lane's loads of this g
      wave_lds_fence();
    }
    if (g + 1 < G) lstore(Anext);
    __syncthreads();
  }
  if (active) {
    xr = wave_sum(xr);
    xi = wave_sum(xi);
    if (lane == 0) exch[2 * wd + s] = mkc(xr, xi);
  }
}

// Dynamic LDS of the block-exchange kernel: two tile buffers and the wavefronts' planes.
inline size_t bx_contract_lds_bytes(int KP, bool bf, int wpb) {
  const size_t tile = bf ? (size_t)32 * (KP + 8) * 2 * 2 : (size_t)32 * (KP + 4) * 4;
  return 2 * tile + (size_t)wpb * 16 * 17 * 4 * 4;
}
