// FP32 / BF16x3 MFMA local-energy contraction in ping-pong form (arXiv:1711.02242,
// Sec. III.D.3, eq:localenergy3; force-bias traces of eq:precomputing2).  Included by
// kernels_mfma.hpp after contract_mfma.hpp, whose per-wavefront arithmetic it shares: one
// wavefront owns one walker-spin, keeps [Re Theta | Im Theta] in registers, computes
// Omega^g = Lh^g Theta per g on the matrix cores and pairs every Omega_ij with Omega_ji through
// its own LDS planes.
//
// The difference is the schedule.  A workgroup holds eight walkers of one spin, two wavefronts
// per SIMD: wavefronts 0-3 (group 0) and 4-7 (group 1).  Time is cut into phases separated by
// workgroup barriers; in phase p a wavefront of group k does step p - k of its own sequence
// chain(0), epilogue(0), chain(1), epilogue(1), ...  So on every SIMD one wavefront issues the
// MFMA chain of g while its partner runs the epilogue (LDS transpose, partner products, trace)
// of the g before: the matrix core is fed by one wavefront at a time and the epilogue runs
// beside it instead of between two chains.  The chain wavefront raises its issue priority.
// Tile g of Lh is read in phases 2g (group 0) and 2g + 1 (group 1); tile g + 1 is fetched
// during phase 2g and stored to the other LDS buffer at its end, so two buffers suffice.
#pragma once

template <int NP, bool BF16, int NK>
__global__ void __launch_bounds__(512, 1) k_contract_mfma_pp(
    int nw, int G, int nup, int ndn, const void* __restrict__ Lp_,
    const void* __restrict__ thp_, const double* __restrict__ weight, cd* __restrict__ tpart,
    cd* __restrict__ exch) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int WPB = 8, NT = 512;
  const int bx = blockIdx.x;
  const int s = blockIdx.y & 1, dd = blockIdx.y >> 1, n_det = gridDim.y >> 1;
  const int N = s ? ndn : nup;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int grp = wave >> 2;
  const int w = bx * WPB + wave;
  const int wd = w * n_det + dd;
  const bool active = (w < nw) && (N > 0) && (weight[w] > 0.0);
  if (N == 0) {   // uniform over the workgroup (N depends on the spin only)
    if (w < nw) {
      for (int g = lane; g < G; g += 64) tpart[((size_t)wd * 2 + s) * G + g] = mkc(0.0, 0.0);
      if (lane == 0) exch[2 * wd + s] = mkc(0.0, 0.0);
    }
    return;
  }
  constexpr int ESZ = BF16 ? 2 : 4;
  constexpr int PLANES = BF16 ? 2 : 1;
  constexpr int KCH = contract_kch<NP, BF16>();
  constexpr int KP = NK * KCH;
  constexpr int lda = KP + (BF16 ? 8 : 4);
  constexpr size_t tile_elems = (size_t)NP * KP * PLANES;
  constexpr int tile_lds_bytes = NP * lda * ESZ * PLANES;
  constexpr int LDE = NP + 4;
  float* ep_re = reinterpret_cast<float*>(smem + 2 * tile_lds_bytes) + (size_t)wave * 2 * NP * LDE;
  float* ep_im = ep_re + NP * LDE;
  const unsigned char* Lbase =
      reinterpret_cast<const unsigned char*>(Lp_) + ((size_t)dd * 2 + s) * G * tile_elems * ESZ;

  // ---- copy of one g-tile global -> LDS by all 512 threads, 16 bytes per thread per chunk
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

  // ---- Theta operand into registers (the packed layout of k_contract_mfma)
  constexpr int LGRP = NP == 32 ? 32 : 16;
  const int col = lane % LGRP;
  const int kg = lane / LGRP;
  const int kofs = BF16 ? 8 * kg : 4 * kg;
  u32x4 bre[NK], bim[NK];
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
  constexpr int NV = NP == 32 ? 16 : 4;
  Acc cre, cim;   // Omega of the wave's last chain, kept for its epilogue
  double xr = 0.0, xi = 0.0;
  if (G > 0) {
    gload(0);
    lstore(smem);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): Theta and the first tile
  __syncthreads();
  const int nph = 2 * G + 1;
  for (int ph = 0; ph < nph; ++ph) {
    // tile g + 1 is fetched during phase 2g and stored at its end
    const int gt = ph >> 1;
    const bool fetch = (ph & 1) == 0 && gt + 1 < G;
    if (fetch) gload(gt + 1);
    const int mine = ph - grp;   // this wave's step: 2g chain of g, 2g + 1 epilogue of g
    if (active && mine >= 0 && mine < 2 * G) {
      const int g = mine >> 1;
      if ((mine & 1) == 0) {
        __builtin_amdgcn_s_setprio(1);
        const unsigned char* arow =
            smem + (g & 1) * tile_lds_bytes + ((size_t)col * lda + kofs) * ESZ;
        const size_t lo_ofs = (size_t)NP * lda * ESZ;
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
        __builtin_amdgcn_s_setprio(0);
      } else {
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
        wave_lds_fence();   // the wave reads back only its own planes
        const int dl = lane < 2 * NP ? lane : 2 * NP - 1;
        float d = dl < NP ? ep_re[dl * (LDE + 1)] : ep_im[(dl - NP) * (LDE + 1)];
        float Rt[NV], It[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int i = (NP == 32 ? 8 * (v / 4) : 0) + 4 * kg + (v % 4);
          Rt[v] = ep_re[i * LDE + col];
          It[v] = ep_im[i * LDE + col];
        }
        __builtin_amdgcn_sched_barrier(0);
        float pr = 0.f, pi = 0.f;
#pragma unroll
        for (int v = 0; v < NV; ++v) exch_term(cre[v], cim[v], Rt[v], It[v], pr, pi);
        xr += (double)pr;
        xi += (double)pi;
        // trace: Re in lane NP - 1, Im in lane 2 NP - 1
        d = NP == 32 ? dpp_half_sum(d) : dpp_row_sum(d);
        double* tp = reinterpret_cast<double*>(tpart + ((size_t)wd * 2 + s) * G + g);
        if (lane == NP - 1) tp[0] = (double)d;
        if (lane == 2 * NP - 1) tp[1] = (double)d;
        // the planes are written again two phases later, after two barriers
      }
    }
    if (fetch) lstore(smem + ((gt + 1) & 1) * tile_lds_bytes);
    __syncthreads();
  }
  if (active) {
    xr = wave_sum(xr);
    xi = wave_sum(xi);
    if (lane == 0) exch[2 * wd + s] = mkc(xr, xi);
  }
}

// Dynamic LDS of the ping-pong kernel: two tile buffers and eight wavefronts' Omega planes.
inline size_t pp_contract_lds_bytes(int NP, int KP, bool bf) {
  const int esz = bf ? 2 : 4, planes = bf ? 2 : 1, lda = KP + (bf ? 8 : 4);
  return 2 * (size_t)NP * lda * esz * planes + (size_t)8 * 2 * NP * (NP + 4) * 4;
}
