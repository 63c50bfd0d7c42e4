// Flattened form of the FP32 / BF16x3 MFMA local-energy contraction (arXiv:1711.02242,
// Sec. III.D.3, eq:localenergy3; force-bias traces of eq:precomputing2) for electron counts
// that are not multiples of 16.  The padded kernels compute every Omega^g = Lh^g Theta as an
// N_P x N_P block (N_P = 16, 32, 48 or 64) for Re and Im each, so at N = 35 they spend
// (48 / 35)^2 = 1.9 times the work on padding.  Here the padding is paid once per group
// instead of once per g and per plane:
//   rows    q consecutive blocks Lh^g (q N rows) form one group of RT row tiles of 16
//           (q = floor(16 RT / N); RT <= 7 is chosen per shape for the least total work);
//   columns [Re Theta | Im Theta] side by side, 2N columns padded to a multiple of 16.
// At N = 35 that is 112 rows for 105 and 80 columns for 70 (1.22 instead of 1.9).
//
// One workgroup owns one (walker, determinant, spin); wavefront j keeps the 16 columns
// 16 j .. 16 j + 15 of [Re Theta | Im Theta] (all K) in registers as the B operand.  For a
// group, each wave accumulates all RT row tiles of its column block at once, walking K in
// chunks: the A operand of the RT tiles for chunk c + 1 is loaded straight from the cache
// hierarchy while the 4 RT MFMAs of chunk c run.  The waves of a workgroup walk the same
// chunks at nearly the same time, so L1 serves the sharing and LDS holds only Omega'.  The
// finished group Omega' = [Re Omega | Im Omega] goes to LDS (column-major); every lane then
// takes the elements it computed and reads their partners:
//   own Re Omega_ij:  Re += R_ij R_ji,  Im += R_ij I_ji
//   own Im Omega_ij:  Re -= I_ij I_ji,  Im += I_ij R_ji
// which sums tr(Omega Omega) over the group in FP32 (accumulated across groups in FP64);
// the waves reduce the diagonals tr Omega^g by DPP lane sums into an LDS row of traces that
// is written out once at the end (no atomics: the result is the same on every run).  Rows
// are read in place from the padded [g][N_P][K_P] table of the other kernels; rows past a
// group's end read a valid row and are never used.
#pragma once

constexpr int FLAT_MAX_RT = 7;              // row tiles of a group (FP32; BF16x3 4: its A
                                            // operand takes twice the registers)
constexpr size_t FLAT_LDS_CAP = 65536;      // LDS bytes of one workgroup

template <int NK, bool BF16, int RT>
__global__ void __launch_bounds__(512) k_contract_mfma_flat(
    int nw, int G, int nup, int ndn, int NP, int KP, int qup, int qdn, int LDR,
    const void* __restrict__ Lp_, const void* __restrict__ thp_,
    const double* __restrict__ weight, cd* __restrict__ tpart, cd* __restrict__ exch) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int s = blockIdx.y & 1, dd = blockIdx.y >> 1, n_det = gridDim.y >> 1;
  const int N = s ? ndn : nup;
  const int q = s ? qdn : qup;
  const int w = blockIdx.x;
  const int wd = w * n_det + dd;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int NWV = blockDim.x >> 6;
  if (w >= nw) return;
  if (N == 0) {
    for (int g = tid; g < G; g += blockDim.x) tpart[((size_t)wd * 2 + s) * G + g] = mkc(0.0, 0.0);
    if (tid == 0) exch[2 * wd + s] = mkc(0.0, 0.0);
    return;
  }
  if (!(weight[w] > 0.0)) return;  // the whole workgroup is one walker

  constexpr int ESZ = BF16 ? 2 : 4;
  constexpr int PLANES = BF16 ? 2 : 1;
  constexpr int KCH = BF16 ? 32 : 16;           // K per register chunk; K_P = NK KCH
  const size_t per = (size_t)NP * KP;           // elements of one plane of one g
  const size_t gstride = per * PLANES * ESZ;    // bytes of one g in the table
  float* ep = reinterpret_cast<float*>(smem);   // Omega' column-major [16 NWV][LDR]
  float* tr = ep + (size_t)16 * NWV * LDR;      // traces [G][2]
  double* red = reinterpret_cast<double*>(tr + 2 * ((G + 1) & ~1));  // [2][NWV]
  const unsigned char* Lbase =
      reinterpret_cast<const unsigned char*>(Lp_) + ((size_t)dd * 2 + s) * G * gstride;

  const int col = lane & 15, kg = lane >> 4;
  const int kofs = (BF16 ? 8 : 4) * kg;
  const int cc = 16 * wave + col;          // column of [Re Theta | Im Theta] held by the lane
  const bool col_ok = cc < 2 * N;
  const bool im_col = cc >= N;
  const int j = im_col ? cc - N : cc;      // column of Theta (Re or Im plane)

  // ---- B operand: 16 columns of [Re | Im] Theta, all K (zero in padded columns)
  u32x4 bh[NK], bl[BF16 ? NK : 1];
  {
    const unsigned char* tb = reinterpret_cast<const unsigned char*>(thp_) +
                              ((size_t)wd * 2 + s) * 2 * PLANES * per * ESZ +
                              (im_col ? (size_t)PLANES * per * ESZ : 0) +
                              ((size_t)(col_ok ? j : 0) * KP + kofs) * ESZ;
    const u32x4 z = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int c = 0; c < NK; ++c) {
      bh[c] = col_ok ? *reinterpret_cast<const u32x4*>(tb + c * KCH * ESZ) : z;
      if (BF16)
        bl[BF16 ? c : 0] = col_ok ? *reinterpret_cast<const u32x4*>(tb + per * ESZ + c * KCH * ESZ) : z;
    }
  }

  const int ngroups = (G + q - 1) / q;
  // Byte offset, from a group's first block, of this lane's A row (row `col`) in each row
  // tile of a full group.  In a group of qk blocks the rows at offsets >= qk gstride lie past
  // its end and read the group's first row instead (clamp()).
  uint32_t ro[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int rho = 16 * r + col;
    const int gl = rho / N, i = rho - gl * N;
    ro[r] = (uint32_t)((size_t)gl * gstride + ((size_t)i * KP + kofs) * ESZ);
  }
  auto clamp = [&](uint32_t o, uint32_t lim) { return o < lim ? o : (uint32_t)(kofs * ESZ); };
  auto ld = [&](const unsigned char* p) { return *reinterpret_cast<const u32x4*>(p); };
  auto qlim = [&](int k) { return (uint32_t)((size_t)min(q, G - k * q) * gstride); };

  u32x4 acur[RT], acur_l[BF16 ? RT : 1];
  {
    const uint32_t lim = qlim(0);
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const unsigned char* p = Lbase + clamp(ro[r], lim);
      acur[r] = ld(p);
      if (BF16) acur_l[BF16 ? r : 0] = ld(p + per * ESZ);
    }
  }

  double xr = 0.0, xi = 0.0;
  for (int k = 0; k < ngroups; ++k) {
    const unsigned char* gb = Lbase + (size_t)k * q * gstride;
    const uint32_t lim = qlim(k);
    // the next group (this one again after the last, so that the loads never depend on a
    // branch and the wait before each chunk's MFMAs covers only that chunk)
    const int kn = k + 1 < ngroups ? k + 1 : k;
    const unsigned char* gbn = Lbase + (size_t)kn * q * gstride;
    const uint32_t limn = qlim(kn);
    f32x4 acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NK; ++c) {
      u32x4 anx[RT], anx_l[BF16 ? RT : 1];
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const unsigned char* p = c + 1 < NK ? gb + clamp(ro[r], lim) + (c + 1) * KCH * ESZ
                                            : gbn + clamp(ro[r], limn);
        anx[r] = ld(p);
        if (BF16) anx_l[BF16 ? r : 0] = ld(p + per * ESZ);
      }
      __builtin_amdgcn_sched_barrier(0);  // the next chunk's loads go out before this chunk's MFMAs
      // the RT row tiles interleaved, so consecutive MFMAs accumulate into different tiles
      if constexpr (!BF16) {
        const f32x4 b = __builtin_bit_cast(f32x4, bh[c]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            const f32x4 a = __builtin_bit_cast(f32x4, acur[r]);
            acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b[m], acc[r], 0, 0, 0);
          }
      } else {
        // per chunk: lo x hi, hi x lo, then hi x hi (small terms first)
        const bf16x8 b_h = __builtin_bit_cast(bf16x8, bh[c]);
        const bf16x8 b_l = __builtin_bit_cast(bf16x8, bl[BF16 ? c : 0]);
#pragma unroll
        for (int r = 0; r < RT; ++r)
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf16x8, acur_l[BF16 ? r : 0]), b_h, acc[r], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < RT; ++r)
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, acur[r]),
                                                           b_l, acc[r], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < RT; ++r)
          acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, acur[r]),
                                                           b_h, acc[r], 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        acur[r] = anx[r];
        if (BF16) acur_l[BF16 ? r : 0] = anx_l[BF16 ? r : 0];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // lane holds Omega'[16 r + 4 kg + v][cc], v = 0..3: column-major store
#pragma unroll
    for (int r = 0; r < RT; ++r)
      *reinterpret_cast<float4*>(ep + cc * LDR + 16 * r + 4 * kg) =
          make_float4(acc[r][0], acc[r][1], acc[r][2], acc[r][3]);
    __syncthreads();  // Omega' of the group complete
    const int qk = min(q, G - k * q);
    float pr = 0.f, pi = 0.f;
    if (col_ok) {
      // element (rho, cc) of the group, rho = 16 r + 4 kg + v: block gl, row i
      auto pair = [&](float own, int gl, int i) {
        const int rp = gl * N + j;  // row of the partner block row j
        const float p_re = ep[i * LDR + rp], p_im = ep[(N + i) * LDR + rp];
        if (!im_col) {
          pr += own * p_re;
          pi += own * p_im;
        } else {
          pr -= own * p_im;
          pi += own * p_re;
        }
      };
      if constexpr (RT <= 4) {
        // own elements from the accumulators
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const int rho0 = 16 * r + 4 * kg;
          int gl = rho0 / N, i = rho0 - gl * N;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (gl < qk) pair(acc[r][v], gl, i);
            if (++i == N) {
              i = 0;
              ++gl;
            }
          }
        }
      } else {
        // not unrolled, own elements from LDS: hoisting every load of a large group would
        // cost ~13 VGPRs per row tile and with them a wave per SIMD of occupancy
#pragma unroll 1
        for (int r = 0; r < RT; ++r) {
          const int rho0 = 16 * r + 4 * kg;
          int gl = rho0 / N, i = rho0 - gl * N;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (gl < qk) pair(ep[cc * LDR + rho0 + v], gl, i);
            if (++i == N) {
              i = 0;
              ++gl;
            }
          }
        }
      }
    }
    xr += (double)pr;
    xi += (double)pi;
    for (int gl = wave; gl < qk; gl += NWV) {
      float dr = 0.f, di = 0.f;
      if (lane < N) {
        dr = ep[lane * LDR + gl * N + lane];
        di = ep[(N + lane) * LDR + gl * N + lane];
      }
      dr = dpp_wave_sum(dr);
      di = dpp_wave_sum(di);
      if (lane == 0) {
        tr[2 * (k * q + gl)] = dr;
        tr[2 * (k * q + gl) + 1] = di;
      }
    }
    __syncthreads();  // reads done before the next group's stores
  }

  for (int g = tid; g < G; g += blockDim.x)
    tpart[((size_t)wd * 2 + s) * G + g] = mkc((double)tr[2 * g], (double)tr[2 * g + 1]);
  xr = wave_sum(xr);
  xi = wave_sum(xi);
  if (lane == 0) {
    red[wave] = xr;
    red[NWV + wave] = xi;
  }
  __syncthreads();
  if (tid == 0) {
    double sr = 0.0, si = 0.0;
    for (int kk = 0; kk < NWV; ++kk) {
      sr += red[kk];
      si += red[NWV + kk];
    }
    exch[2 * wd + s] = mkc(sr, si);
  }
}

// ---------------------------------------------------------------------------
// Stacked-row form: the rows of q consecutive blocks Lh^g are stacked as above, but each
// wavefront keeps Re and Im of 16 Theta columns (j = 16 w .. 16 w + 15) as two B operands,
// like the wide kernel, so every A fragment feeds 8 MFMAs instead of 4 (half the A traffic
// per flop) at the cost of padding N, not 2N, to a multiple of 16.  Omega is kept as Re and
// Im planes in LDS; a lane's partner of Omega_ij is Omega_ji in the same two planes.
// ---------------------------------------------------------------------------
template <int NK, bool BF16, int RT>
__global__ void __launch_bounds__(256) k_contract_mfma_stack(
    int nw, int G, int nup, int ndn, int NP, int KP, int qup, int qdn, int LDR,
    const void* __restrict__ Lp_, const void* __restrict__ thp_,
    const double* __restrict__ weight, cd* __restrict__ tpart, cd* __restrict__ exch) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int s = blockIdx.y & 1, dd = blockIdx.y >> 1, n_det = gridDim.y >> 1;
  const int N = s ? ndn : nup;
  const int q = s ? qdn : qup;
  const int w = blockIdx.x;
  const int wd = w * n_det + dd;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int NWV = blockDim.x >> 6;
  if (w >= nw) return;
  if (N == 0) {
    for (int g = tid; g < G; g += blockDim.x) tpart[((size_t)wd * 2 + s) * G + g] = mkc(0.0, 0.0);
    if (tid == 0) exch[2 * wd + s] = mkc(0.0, 0.0);
    return;
  }
  if (!(weight[w] > 0.0)) return;  // the whole workgroup is one walker

  constexpr int ESZ = BF16 ? 2 : 4;
  constexpr int PLANES = BF16 ? 2 : 1;
  constexpr int KCH = BF16 ? 32 : 16;
  const size_t per = (size_t)NP * KP;
  const size_t gstride = per * PLANES * ESZ;
  float* ep_re = reinterpret_cast<float*>(smem);          // Re Omega column-major [16 NWV][LDR]
  float* ep_im = ep_re + (size_t)16 * NWV * LDR;          // Im Omega
  float* tr = ep_im + (size_t)16 * NWV * LDR;             // traces [G][2]
  double* red = reinterpret_cast<double*>(tr + 2 * ((G + 1) & ~1));  // [2][NWV]
  const unsigned char* Lbase =
      reinterpret_cast<const unsigned char*>(Lp_) + ((size_t)dd * 2 + s) * G * gstride;

  const int col = lane & 15, kg = lane >> 4;
  const int kofs = (BF16 ? 8 : 4) * kg;
  const int j = 16 * wave + col;     // Theta column of the lane
  const bool col_ok = j < N;

  // ---- B operands: Re and Im of 16 Theta columns, all K (zero in padded columns)
  u32x4 br[NK], bi[NK], brl[BF16 ? NK : 1], bil[BF16 ? NK : 1];
  {
    const unsigned char* tb = reinterpret_cast<const unsigned char*>(thp_) +
                              ((size_t)wd * 2 + s) * 2 * PLANES * per * ESZ +
                              ((size_t)(col_ok ? j : 0) * KP + kofs) * ESZ;
    const size_t im_ofs = (size_t)PLANES * per * ESZ;
    const u32x4 z = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int c = 0; c < NK; ++c) {
      const unsigned char* p = tb + c * KCH * ESZ;
      br[c] = col_ok ? *reinterpret_cast<const u32x4*>(p) : z;
      bi[c] = col_ok ? *reinterpret_cast<const u32x4*>(p + im_ofs) : z;
      if (BF16) {
        brl[BF16 ? c : 0] = col_ok ? *reinterpret_cast<const u32x4*>(p + per * ESZ) : z;
        bil[BF16 ? c : 0] = col_ok ? *reinterpret_cast<const u32x4*>(p + im_ofs + per * ESZ) : z;
      }
    }
  }

  const int ngroups = (G + q - 1) / q;
  uint32_t ro[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int rho = 16 * r + col;
    const int gl = rho / N, i = rho - gl * N;
    ro[r] = (uint32_t)((size_t)gl * gstride + ((size_t)i * KP + kofs) * ESZ);
  }
  auto clamp = [&](uint32_t o, uint32_t lim) { return o < lim ? o : (uint32_t)(kofs * ESZ); };
  auto ld = [&](const unsigned char* p) { return *reinterpret_cast<const u32x4*>(p); };
  auto qlim = [&](int k) { return (uint32_t)((size_t)min(q, G - k * q) * gstride); };

  u32x4 acur[RT], acur_l[BF16 ? RT : 1];
  {
    const uint32_t lim = qlim(0);
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const unsigned char* p = Lbase + clamp(ro[r], lim);
      acur[r] = ld(p);
      if (BF16) acur_l[BF16 ? r : 0] = ld(p + per * ESZ);
    }
  }

  double xr = 0.0, xi = 0.0;
  for (int k = 0; k < ngroups; ++k) {
    const unsigned char* gb = Lbase + (size_t)k * q * gstride;
    const uint32_t lim = qlim(k);
    const int kn = k + 1 < ngroups ? k + 1 : k;
    const unsigned char* gbn = Lbase + (size_t)kn * q * gstride;
    const uint32_t limn = qlim(kn);
    f32x4 cre[RT], cim[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      cre[r] = f32x4{0.f, 0.f, 0.f, 0.f};
      cim[r] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int c = 0; c < NK; ++c) {
      u32x4 anx[RT], anx_l[BF16 ? RT : 1];
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const unsigned char* p = c + 1 < NK ? gb + clamp(ro[r], lim) + (c + 1) * KCH * ESZ
                                            : gbn + clamp(ro[r], limn);
        anx[r] = ld(p);
        if (BF16) anx_l[BF16 ? r : 0] = ld(p + per * ESZ);
      }
      __builtin_amdgcn_sched_barrier(0);  // the next chunk's loads go out before this chunk's MFMAs
      if constexpr (!BF16) {
        const f32x4 b_r = __builtin_bit_cast(f32x4, br[c]);
        const f32x4 b_i = __builtin_bit_cast(f32x4, bi[c]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            const f32x4 a = __builtin_bit_cast(f32x4, acur[r]);
            cre[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b_r[m], cre[r], 0, 0, 0);
            cim[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m], b_i[m], cim[r], 0, 0, 0);
          }
      } else {
        const bf16x8 rh = __builtin_bit_cast(bf16x8, br[c]);
        const bf16x8 rl = __builtin_bit_cast(bf16x8, brl[BF16 ? c : 0]);
        const bf16x8 ih = __builtin_bit_cast(bf16x8, bi[c]);
        const bf16x8 il = __builtin_bit_cast(bf16x8, bil[BF16 ? c : 0]);
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const bf16x8 ah = __builtin_bit_cast(bf16x8, acur[r]);
          const bf16x8 al = __builtin_bit_cast(bf16x8, acur_l[BF16 ? r : 0]);
          cre[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, rh, cre[r], 0, 0, 0);
          cim[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, ih, cim[r], 0, 0, 0);
          cre[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, rl, cre[r], 0, 0, 0);
          cim[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, il, cim[r], 0, 0, 0);
          cre[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, rh, cre[r], 0, 0, 0);
          cim[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, ih, cim[r], 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        acur[r] = anx[r];
        if (BF16) acur_l[BF16 ? r : 0] = anx_l[BF16 ? r : 0];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // lane holds Omega[16 r + 4 kg + v][j], v = 0..3: column-major stores
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      *reinterpret_cast<float4*>(ep_re + j * LDR + 16 * r + 4 * kg) =
          make_float4(cre[r][0], cre[r][1], cre[r][2], cre[r][3]);
      *reinterpret_cast<float4*>(ep_im + j * LDR + 16 * r + 4 * kg) =
          make_float4(cim[r][0], cim[r][1], cim[r][2], cim[r][3]);
    }
    __syncthreads();  // Omega of the group complete
    const int qk = min(q, G - k * q);
    float pr = 0.f, pi = 0.f;
    if (col_ok) {
      // element (rho, j), rho = 16 r + 4 kg + v: block gl, row i; partner Omega_ji
      auto pair = [&](float R, float I, int gl, int i) {
        const int rp = gl * N + j;
        const float Rt = ep_re[i * LDR + rp], It = ep_im[i * LDR + rp];
        pr += R * Rt - I * It;
        pi += R * It + I * Rt;
      };
      {
        // not unrolled, own elements from LDS: the registers stay with the MFMA loop
#pragma unroll 1
        for (int r = 0; r < RT; ++r) {
          const int rho0 = 16 * r + 4 * kg;
          int gl = rho0 / N, i = rho0 - gl * N;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (gl < qk) pair(ep_re[j * LDR + rho0 + v], ep_im[j * LDR + rho0 + v], gl, i);
            if (++i == N) {
              i = 0;
              ++gl;
            }
          }
        }
      }
    }
    xr += (double)pr;
    xi += (double)pi;
    for (int gl = wave; gl < qk; gl += NWV) {
      float dr = 0.f, di = 0.f;
      if (lane < N) {
        dr = ep_re[lane * LDR + gl * N + lane];
        di = ep_im[lane * LDR + gl * N + lane];
      }
      dr = dpp_wave_sum(dr);
      di = dpp_wave_sum(di);
      if (lane == 0) {
        tr[2 * (k * q + gl)] = dr;
        tr[2 * (k * q + gl) + 1] = di;
      }
    }
    __syncthreads();  // reads done before the next group's stores
  }

  for (int g = tid; g < G; g += blockDim.x)
    tpart[((size_t)wd * 2 + s) * G + g] = mkc((double)tr[2 * g], (double)tr[2 * g + 1]);
  xr = wave_sum(xr);
  xi = wave_sum(xi);
  if (lane == 0) {
    red[wave] = xr;
    red[NWV + wave] = xi;
  }
  __syncthreads();
  if (tid == 0) {
    double sr = 0.0, si = 0.0;
    for (int kk = 0; kk < NWV; ++kk) {
      sr += red[kk];
      si += red[NWV + kk];
    }
    exch[2 * wd + s] = mkc(sr, si);
  }
}

// Launch geometry of the flattened (stack = false) and stacked-row (stack = true) kernels:
// wavefronts per workgroup (16 columns each: of [Re | Im] Theta, or Re and Im of Theta),
// row tiles per group (one RT for both spins: the least total row-tile work
// sum_s ceil(G / q_s) RT over RT = ceil(N_max / 16) .. the register cap, smaller RT within
// 1 %), blocks per group of each spin, LDS row stride and bytes.
struct FlatLaunch {
  bool ok = false;  // a row-tile count within the register cap holds N_max rows
  int waves = 1, RT = 1, qup = 1, qdn = 1, LDR = 20;
  size_t lds = 0;
};

constexpr int STACK_MAX_RT = 7;             // FP32; BF16x3 3 (four B operands)

inline size_t flat_lds_bytes(int waves, int LDR, int G, bool stack) {
  return (size_t)(stack ? 2 : 1) * 16 * waves * LDR * 4 + (size_t)2 * ((G + 1) & ~1) * 4 +
         (size_t)2 * waves * 8;
}

inline FlatLaunch flat_launch(int nup, int ndn, int G, bool bf16, bool stack = false) {
  FlatLaunch f;
  const int nmax = nup > ndn ? nup : ndn;
  f.waves = stack ? (nmax + 15) / 16 : (2 * nmax + 15) / 16;
  if (f.waves < 1) f.waves = 1;
  const int rt_min = nmax > 0 ? (nmax + 15) / 16 : 1;
  const int g1 = G > 1 ? G : 1;
  const int rt_max = stack ? (bf16 ? 3 : STACK_MAX_RT) : (bf16 ? 4 : FLAT_MAX_RT);
  double best = 1e300;
  for (int rt = rt_min; rt <= rt_max; ++rt) {
    if (rt > rt_min && flat_lds_bytes(f.waves, 16 * rt + 4, G, stack) > FLAT_LDS_CAP) break;
    const int qu = nup > 0 ? std::min(g1, 16 * rt / nup) : 1;
    const int qd = ndn > 0 ? std::min(g1, 16 * rt / ndn) : 1;
    const double work = (double)rt * ((nup > 0 ? (g1 + qu - 1) / qu : 0) +
                                      (ndn > 0 ? (g1 + qd - 1) / qd : 0));
    if (work < best * 0.99) {
      best = work;
      f.ok = true;
      f.RT = rt;
      f.qup = qu;
      f.qdn = qd;
    }
  }
  f.LDR = 16 * f.RT + 4;
  f.lds = flat_lds_bytes(f.waves, f.LDR, G, stack);
  return f;
}
