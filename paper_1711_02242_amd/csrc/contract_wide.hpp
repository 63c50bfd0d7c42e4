// Wide form of the FP32 / BF16x3 MFMA local-energy contraction (arXiv:1711.02242,
// Sec. III.D.3, eq:localenergy3; force-bias traces of eq:precomputing2), for the
// shapes the register-resident kernel of contract_mfma.hpp cannot hold: N up to 64
// electrons per spin and M up to 224 orbitals.
//
// One workgroup owns one (walker, determinant, spin).  Its NPW / 16 wavefronts
// split the columns of Theta: wave j keeps [Re | Im] Theta[:, 16 j .. 16 j + 15]
// (K up to 224) in registers for the whole kernel and computes the column block
// Omega[:, 16 j .. 16 j + 15] = Lh^g Theta[:, block] for every g on
// v_mfma_f32_16x16x4_f32 (BF16x3: v_mfma_f32_16x16x32_bf16, three products
// hi*hi + hi*lo + lo*hi).  The A operand (rows of Lh^g) is read by every wave
// straight from the cache hierarchy, one K chunk ahead in registers; the waves of a
// workgroup read the same rows at nearly the same time, so L1 serves the sharing and
// LDS holds only Omega.  That keeps several workgroups per CU at these shapes.
// Omega is written column-major to LDS so that each lane reads the partner
// Omega_ji of every Omega_ij it holds; tr(Omega Omega) is summed per g in FP32 and
// across g in FP64, and wave 0 / wave 1 form Re / Im tr Omega.
#pragma once

template <int NPW, bool BF16, int NK>
__global__ void __launch_bounds__(256, 2) k_contract_mfma_wide(
    int nw, int G, int nup, int ndn, int KP, const void* __restrict__ Lp_,
    const void* __restrict__ thp_, const double* __restrict__ weight, cd* __restrict__ tpart,
    cd* __restrict__ exch) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int NW = NPW / 16;   // wavefronts = 16-column blocks of Theta
  constexpr int NR = NPW / 16;   // 16-row tiles of Omega
  constexpr int NT = 64 * NW;    // threads
  const int s = blockIdx.y & 1, dd = blockIdx.y >> 1, n_det = gridDim.y >> 1;
  const int N = s ? ndn : nup;
  const int w = blockIdx.x;
  const int wd = w * n_det + dd;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (w >= nw) return;
  if (N == 0) {
    for (int g = tid; g < G; g += NT) tpart[((size_t)wd * 2 + s) * G + g] = mkc(0.0, 0.0);
    if (tid == 0) exch[2 * wd + s] = mkc(0.0, 0.0);
    return;
  }
  if (!(weight[w] > 0.0)) return;  // the whole workgroup is one walker

  constexpr int ESZ = BF16 ? 2 : 4;
  constexpr int PLANES = BF16 ? 2 : 1;
  const size_t tile_elems = (size_t)NPW * KP * PLANES;  // one g in global memory
  constexpr int LDE = NPW + 4;
  float* ep_re = reinterpret_cast<float*>(smem);        // Omega column-major
  float* ep_im = ep_re + NPW * LDE;
  double* red = reinterpret_cast<double*>(ep_im + NPW * LDE);  // [2][NW]

  const unsigned char* Lbase =
      reinterpret_cast<const unsigned char*>(Lp_) + ((size_t)dd * 2 + s) * G * tile_elems * ESZ;

  // ---- Theta column block into registers (B operand: rows k, column 16 wave + col)
  constexpr int KCH = BF16 ? 32 : 16;      // K per register chunk (4 lane groups)
  constexpr int MAXK = NK;                 // K chunks held: KP = NK * KCH exactly
  constexpr int nk = NK;
  const int col = lane & 15, kg = lane >> 4;
  const int kofs = BF16 ? 8 * kg : 4 * kg;
  const int bcol = 16 * wave + col;        // Theta column of this lane
  u32x4 bre[MAXK], bim[MAXK];
  u32x4 bre_lo[BF16 ? MAXK : 1], bim_lo[BF16 ? MAXK : 1];
  {
    const size_t per = (size_t)NPW * KP;
    const unsigned char* tb = reinterpret_cast<const unsigned char*>(thp_) +
                              ((size_t)wd * 2 + s) * 2 * PLANES * per * ESZ;
#pragma unroll
    for (int c = 0; c < MAXK; ++c) {
      if (c < nk) {
        const size_t off = ((size_t)bcol * KP + c * KCH + kofs) * ESZ;
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
  // A operand of row tile r, K chunk c of a tile: this lane's 16 bytes (and the lo plane) at
  // tile base (wave-uniform) + row offset (per lane) + c KCH ESZ (immediate)
  const size_t plane_bytes = (size_t)NPW * KP * ESZ;
  const size_t tile_bytes = tile_elems * ESZ;
  uint32_t roff[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) roff[r] = (uint32_t)(((16 * r + col) * KP + kofs) * ESZ);
  auto a_ld = [&](const unsigned char* tg, int r, int c) {
    return *reinterpret_cast<const u32x4*>(tg + roff[r] + c * KCH * ESZ);
  };

  double xr = 0.0, xi = 0.0;
  u32x4 acur[NR], acur_lo[BF16 ? NR : 1];
  if (G > 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      acur[r] = a_ld(Lbase, r, 0);
      if (BF16) acur_lo[BF16 ? r : 0] = a_ld(Lbase + plane_bytes, r, 0);
    }
  }
  for (int g = 0; g < G; ++g) {
    const unsigned char* tg = Lbase + (size_t)g * tile_bytes;
    f32x4 cre[NR], cim[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      cre[r] = f32x4{0.f, 0.f, 0.f, 0.f};
      cim[r] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int c = 0; c < MAXK; ++c) {
      if (c < nk) {
        // next chunk (or the first chunk of the next g) one step ahead
        const bool more = c + 1 < nk || g + 1 < G;
        const unsigned char* tn = c + 1 < nk ? tg : tg + tile_bytes;
        const int cn = c + 1 < nk ? c + 1 : 0;
        u32x4 anx[NR], anx_lo[BF16 ? NR : 1];
        if (more) {
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            anx[r] = a_ld(tn, r, cn);
            if (BF16) anx_lo[BF16 ? r : 0] = a_ld(tn + plane_bytes, r, cn);
          }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if constexpr (!BF16) {
            const f32x4 a = __builtin_bit_cast(f32x4, acur[r]);
            const f32x4 br = __builtin_bit_cast(f32x4, bre[c]);
            const f32x4 bi = __builtin_bit_cast(f32x4, bim[c]);
            cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, br.x, cre[r], 0, 0, 0);
            cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bi.x, cim[r], 0, 0, 0);
            cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, br.y, cre[r], 0, 0, 0);
            cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bi.y, cim[r], 0, 0, 0);
            cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, br.z, cre[r], 0, 0, 0);
            cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, bi.z, cim[r], 0, 0, 0);
            cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, br.w, cre[r], 0, 0, 0);
            cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, bi.w, cim[r], 0, 0, 0);
          } else {
            const bf16x8 ah = __builtin_bit_cast(bf16x8, acur[r]);
            const bf16x8 al = __builtin_bit_cast(bf16x8, acur_lo[BF16 ? r : 0]);
            const bf16x8 brh = __builtin_bit_cast(bf16x8, bre[c]);
            const bf16x8 brl = __builtin_bit_cast(bf16x8, bre_lo[BF16 ? c : 0]);
            const bf16x8 bih = __builtin_bit_cast(bf16x8, bim[c]);
            const bf16x8 bil = __builtin_bit_cast(bf16x8, bim_lo[BF16 ? c : 0]);
            cre[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, brh, cre[r], 0, 0, 0);
            cim[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bih, cim[r], 0, 0, 0);
            cre[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, brl, cre[r], 0, 0, 0);
            cim[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bil, cim[r], 0, 0, 0);
            cre[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, brh, cre[r], 0, 0, 0);
            cim[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bih, cim[r], 0, 0, 0);
          }
        }
        if (more) {
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            acur[r] = anx[r];
            if (BF16) acur_lo[BF16 ? r : 0] = anx_lo[BF16 ? r : 0];
          }
        }
      }
      // keep each chunk's loads one chunk ahead instead of hoisting them all
      __builtin_amdgcn_sched_barrier(0);
    }
    // lane holds Omega[16 r + 4 kg + v][bcol], v = 0..3: column-major store
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      *reinterpret_cast<float4*>(ep_re + bcol * LDE + 16 * r + 4 * kg) =
          make_float4(cre[r][0], cre[r][1], cre[r][2], cre[r][3]);
      *reinterpret_cast<float4*>(ep_im + bcol * LDE + 16 * r + 4 * kg) =
          make_float4(cim[r][0], cim[r][1], cim[r][2], cim[r][3]);
    }
    __syncthreads();  // Omega complete
    {
      float pr = 0.f, pi = 0.f;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * r + 4 * kg + v;
          const float R = cre[r][v], I = cim[r][v];
          const float Rt = ep_re[i * LDE + bcol], It = ep_im[i * LDE + bcol];
          pr += R * Rt - I * It;
          pi += R * It + I * Rt;
        }
      }
      xr += (double)pr;
      xi += (double)pi;
    }
    if (wave < 2) {
      // trace: wave 0 sums Re Omega_jj, wave 1 Im Omega_jj
      const float* epp = wave == 0 ? ep_re : ep_im;
      float d = lane < NPW ? epp[lane * LDE + lane] : 0.f;
      d = dpp_wave_sum(d);
      if (lane == 0) reinterpret_cast<double*>(tpart + ((size_t)wd * 2 + s) * G + g)[wave] = (double)d;
    }
    __syncthreads();  // Omega reads done before the next g writes it
  }
  xr = wave_sum(xr);
  xi = wave_sum(xi);
  if (lane == 0) {
    red[wave] = xr;
    red[NW + wave] = xi;
  }
  __syncthreads();
  if (tid == 0) {
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < NW; ++k) {
      sr += red[k];
      si += red[NW + k];
    }
    exch[2 * wd + s] = mkc(sr, si);
  }
}

template <int NPW, bool BF16>
constexpr size_t wide_contract_lds_bytes_t(int) {
  return (size_t)2 * NPW * (NPW + 4) * 4 + 2 * (NPW / 16) * 8;
}
