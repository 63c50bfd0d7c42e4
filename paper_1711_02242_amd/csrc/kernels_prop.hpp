// FP32 MFMA kernels of the propagation (arXiv:1711.02242, Sec. III.D.2, Theorem 1.4,
// eq:primitive):
//
//   A_w = i s sum_g y_wg L^g                       (propagator exponent, y = x - xbar)
//   U_w <- E_h T_n(A_w) E_h U_w,   T_n(A) = sum_{k<=n} A^k / k!,   E_h = exp(-dtau/2 v0)
//
// Walker orbitals are rows (U^T, orbital-major), so the propagation multiplies
// the rows from the right: u' = u E_h T_n(A) E_h, using E_h^T = E_h and
// A^T = A (every L^g is symmetric).  Both MFMA operands are then contiguous
// along the contraction index.
#pragma once

#include "common.hpp"
#include "kernels_mfma.hpp"

// ---------------------------------------------------------------------------
// Block-packed storage of the FP32 exponent A_w (symmetric, one Re and one Im plane per
// walker): the 8 x 8 blocks (QB, PB), PB <= QB, of the lower block triangle, block row by
// block row, each block whole and row-major (a diagonal block holds both of its halves).
// A_w[q][p] for p in the upper block triangle is read as A_w[p][q].  Entries past M (the last
// block row and column when 8 does not divide M) hold zero.
// ---------------------------------------------------------------------------
__host__ __device__ inline int apk_size(int M) {
  const int nb = (M + 7) / 8;
  return 32 * nb * (nb + 1);   // 64 entries per block, nb (nb + 1) / 2 blocks
}
__host__ __device__ inline int apk_index(int q, int p) {
  int QB = q >> 3, PB = p >> 3, qi = q & 7, pi = p & 7;
  if (PB > QB) {
    const int t = QB, ti = qi;
    QB = PB, qi = pi;
    PB = t, pi = ti;
  }
  return 64 * (QB * (QB + 1) / 2 + PB) + 8 * qi + pi;
}
// The (q, p) of packed entry k (inverse of apk_index on the lower block triangle).
inline void apk_entry(int k, int& q, int& p) {
  const int blk = k >> 6, e = k & 63;
  int QB = 0;
  while ((QB + 1) * (QB + 2) / 2 <= blk) ++QB;
  const int PB = blk - QB * (QB + 1) / 2;
  q = 8 * QB + (e >> 3);
  p = 8 * PB + (e & 7);
}

// Workgroup tile of a gx x gy grid renumbered for the 8 XCDs (workgroups go to them
// round-robin by linear id, each XCD with an L2 of its own).  Where gx is even and 4 divides
// gy, XCD x takes the block of half the rows (x & 1) and a quarter of the columns (x >> 1),
// rows fastest: its share of the row operand stays small enough for its L2 while the column
// operand streams through once.  Otherwise each XCD takes a contiguous run of tiles in
// x-fastest order.
__device__ __forceinline__ int2 xcd_tile(int gx, int gy) {
  const int n = gx * gy, L = blockIdx.x + gx * blockIdx.y;
  const int x = L & 7, j = L >> 3;
  if ((gx & 1) == 0 && (gy & 3) == 0) {
    const int hx = gx >> 1, qy = gy >> 2;   // block of hx x qy tiles = n / 8
    return make_int2((x & 1) * hx + j % hx, (x >> 1) * qy + j / hx);
  }
  const int q = n >> 3, r = n & 7;
  const int t = x * q + (x < r ? x : r) + j;
  return make_int2(t % gx, t / gx);
}

// Four consecutive entries A[q][p0 .. p0 + 3] (p0 a multiple of 4, q < M) of a block-packed
// plane, zero past M: one 16-byte load inside the lower block triangle, four loads of a
// column of the block (p0, q) above it.
__device__ __forceinline__ f32x4 apk_load4(const float* __restrict__ Ap, int M, int q, int p0) {
  if ((p0 >> 3) <= (q >> 3)) return *reinterpret_cast<const f32x4*>(Ap + apk_index(q, p0));
  f32x4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (p0 + e < M) v[e] = Ap[apk_index(q, p0 + e)];
  return v;
}

// ---------------------------------------------------------------------------
// A-build as a tiled MFMA GEMM:  C[r][col] = sum_k Y[r][k] Lt[col][k]
//   r = 2w + (0: Re y, 1: Im y),  col = block-packed entry of A (apk_index; MA = apk_size(M)
//   columns, about half of M^2 since A is symmetric),  k = g (padded to Gp, zeros).
//   Re A_w[col] = -s C[2w+1][col],  Im = s C[2w][col]: planar FP32 output of MA entries per
//   walker, each written once (a tile's columns are whole block rows: contiguous stores).
// Tile 128 rows x 16 CB columns per workgroup, two workgroups per CU; four wavefronts of
// 32 rows x 16 CB columns (2 x CB blocks of v_mfma_f32_16x16x4_f32); K chunks of 16
// double-buffered in LDS, Y rows first, then the Lt rows of the tile's columns.  The host
// picks CB (abuild_cb) so that the workgroups fill whole rounds of the device's slots: at
// M = 128 the 8704 packed columns make 32 tiles of 272 (CB = 17), and 1024 walkers 16 row
// tiles, 512 workgroups in all, one round on 256 CUs.  A lane holds four consecutive k of
// its row in each operand and MFMA e takes the e-th of them: a permutation of the k of the
// chunk, the same in both operands.
// ---------------------------------------------------------------------------
constexpr int AB_BM = 128, AB_BK = 16, AB_LD = AB_BK + 4;

template <int CB>
__global__ void __launch_bounds__(256, 2) k_abuild_f32(int rows /*2 nw*/, int MA, int Gp, float s,
                                                       const float* __restrict__ Y,
                                                       const float* __restrict__ Lt,
                                                       float* __restrict__ Are,
                                                       float* __restrict__ Aim) {
  constexpr int BN = 16 * CB, TR = AB_BM + BN;
  constexpr int NLD = TR * (AB_BK / 4);           // 16-byte pieces of one K chunk
  constexpr int PER = (NLD + 255) / 256;
  static_assert(2 * TR * AB_LD * 4 <= 65536, "tile exceeds the static LDS of a workgroup");
  __shared__ __attribute__((aligned(16))) float Ls[2][TR * AB_LD];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int2 tile = xcd_tile(gridDim.x, gridDim.y);
  const int r0 = tile.x * AB_BM, c0 = tile.y * BN;
  const int wr = wave * 32;
  const int col = lane & 15, kg = lane >> 4;
  // piece e of a chunk: tile row e / 4 (rows below AB_BM are Y rows, the rest Lt rows), k
  // offset 4 (e % 4); with 256 threads, pass c covers rows 64 c .. 64 c + 63, so the Y / Lt
  // choice is uniform per pass.  Rows past the walkers and columns past the packed triangle
  // re-read row / column 0: they only feed accumulator rows / columns that are never stored.
  f32x4 stg[PER];
  auto gload = [&](int k0) {
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int e = tid + c * 256;
      if ((c + 1) * 256 <= NLD || e < NLD) {
        const int rr = e >> 2, kk = (e & 3) * 4;
        const float* src;
        if (c * 64 + 63 < AB_BM) {
          const int gr = r0 + rr;
          src = Y + (size_t)(gr < rows ? gr : 0) * Gp;
        } else {
          const int gc = c0 + rr - AB_BM;
          src = Lt + (size_t)(gc < MA ? gc : 0) * Gp;
        }
        stg[c] = *reinterpret_cast<const f32x4*>(src + k0 + kk);
      }
    }
  };
  auto lstore = [&](float* dst) {
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int e = tid + c * 256;
      if ((c + 1) * 256 <= NLD || e < NLD)
        *reinterpret_cast<f32x4*>(dst + (e >> 2) * AB_LD + (e & 3) * 4) = stg[c];
    }
  };
  f32x4 acc[2][CB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nk = Gp / AB_BK;
  gload(0);
  lstore(Ls[0]);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const float* Lb = Ls[kc & 1];
    if (kc + 1 < nk) gload((kc + 1) * AB_BK);
    const f32x4 fa0 = *reinterpret_cast<const f32x4*>(Lb + (wr + col) * AB_LD + 4 * kg);
    const f32x4 fa1 = *reinterpret_cast<const f32x4*>(Lb + (wr + 16 + col) * AB_LD + 4 * kg);
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const f32x4 fb = *reinterpret_cast<const f32x4*>(Lb + (AB_BM + 16 * b + col) * AB_LD + 4 * kg);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc[0][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa0[e], fb[e], acc[0][b], 0, 0, 0);
        acc[1][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa1[e], fb[e], acc[1][b], 0, 0, 0);
      }
    }
    if (kc + 1 < nk) lstore(Ls[(kc + 1) & 1]);
    __syncthreads();
  }
  // epilogue: lane holds column 16 b + col, rows 16 a + 4 kg + v of the wave's 32; v = 0, 1
  // are the Re and Im rows of one walker, v = 2, 3 of the next
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int cc = c0 + 16 * b + col;
      if (cc >= MA) continue;
#pragma unroll
      for (int v = 0; v < 4; v += 2) {
        const int r = r0 + wr + 16 * a + 4 * kg + v;   // even
        if (r >= rows) continue;
        const size_t o = (size_t)(r >> 1) * MA + cc;
        Are[o] = -s * acc[a][b][v + 1];
        Aim[o] = s * acc[a][b][v];
      }
    }
}

// Column blocks of 16 per A-build tile, from those compiled: the least MFMA time, counted as
// (rounds of the device's workgroup slots) x (workgroups per CU) x CB, with the workgroups
// per CU of each instance from the runtime's occupancy (queried once per device); ties go to
// the wider tile.
constexpr int AB_CBS[] = {17, 16, 12, 8, 4};
constexpr int AB_NCB = sizeof(AB_CBS) / sizeof(AB_CBS[0]);
template <int I>
inline const void* abuild_fn() {
  return reinterpret_cast<const void*>(k_abuild_f32<AB_CBS[I]>);
}
inline int abuild_cb(int rows, int MA) {
  static int per_cu[64][AB_NCB] = {};
  static const void* const fns[AB_NCB] = {abuild_fn<0>(), abuild_fn<1>(), abuild_fn<2>(),
                                          abuild_fn<3>(), abuild_fn<4>()};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  const long long cus = device_cu_count(), nrow = (rows + AB_BM - 1) / AB_BM;
  int best = AB_CBS[0];
  long long best_cost = -1;
  for (int i = 0; i < AB_NCB; ++i) {
    if (per_cu[dev][i] <= 0) {
      int n = 0;
      per_cu[dev][i] =
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fns[i], 256, 0) == hipSuccess && n > 0
              ? n
              : 1;
    }
    const long long cb = AB_CBS[i], n = per_cu[dev][i];
    const long long wgs = nrow * ((MA + 16 * cb - 1) / (16 * cb));
    const long long cost = (wgs + n * cus - 1) / (n * cus) * n * cb;
    if (best_cost < 0 || cost < best_cost) best = (int)cb, best_cost = cost;
  }
  return best;
}

// ---------------------------------------------------------------------------
// Fused propagation of one walker per workgroup: u' = u E_h T_n(A) E_h for all
// its orbitals u (rows).  One wavefront per 16 output columns q; the wave keeps
// its columns of A (Re, Im) and of E_h in registers as the MFMA B operand for
// the whole Taylor series, while the current term (rows c, FP32 Re/Im planes)
// lives in LDS as the A operand.  Sum Y of the series accumulates in registers.
// v_mfma_f32_16x16x4_f32; output lane layout: column j = lane % 16, rows 4*(lane/16) + v.
// Requirements: M <= 128, ntot <= 64.
// ---------------------------------------------------------------------------
constexpr int PR_RB = 4;  // row blocks of 16 (ntot <= 64)

// NKC = K_P / 16 wavefronts (K chunks of 16), NRB = ceil(ntot / 16) row blocks: both compile
// time, so the chunk loops carry no branches and the LDS reads can run ahead of the MFMAs.
template <int NKC, int NRB>
__global__ void __launch_bounds__(64 * NKC, 1) k_propagate_f32(
    int M, int ntot, int Kp_arg, int n_taylor, const float* __restrict__ Eh32 /*[M][M]*/,
    const float* __restrict__ Are, const float* __restrict__ Aim, cd* __restrict__ U,
    const double* __restrict__ weight) {
  extern __shared__ __attribute__((aligned(16))) float tsm[];
  const int w = blockIdx.x;
  if (!(weight[w] > 0.0)) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int Kp = 16 * NKC;
  (void)Kp_arg;
  constexpr int ldt = Kp + 4;
  constexpr int RP = 16 * NRB;   // term rows held in LDS
  float* Tr = tsm;             // [RP][ldt]
  float* Ti = tsm + RP * ldt;  // [RP][ldt]
  const int j = lane & 15, q4 = lane >> 4;
  const int qcol = 16 * wave + j;  // output column owned by the lane
  const size_t MA = (size_t)apk_size(M);

  // load U rows (FP64 complex) into the term planes, zero padding: all loads of a thread go
  // out before the first store (padding positions read a valid element and store zero)
  const cd* Uw = U + (size_t)w * ntot * M;
  {
    constexpr int NT = 64 * NKC, NIT = RP * Kp / NT;   // = 4 NRB
    cd uv[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = tid + it * NT, c = e / Kp, p = e % Kp;
      uv[it] = Uw[(size_t)(c < ntot ? c : 0) * M + (p < M ? p : 0)];
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = tid + it * NT, c = e / Kp, p = e % Kp;
      const bool ok = c < ntot && p < M;
      Tr[c * ldt + p] = ok ? (float)uv[it].re : 0.f;
      Ti[c * ldt + p] = ok ? (float)uv[it].im : 0.f;
    }
  }
  // B operands: lane holds rows q = qcol, k = 16*kc + 4*q4 .. +3 (16-byte loads where the
  // four are inside the row and aligned)
  f32x4 be[NKC], bar_[NKC], bai[NKC], bas[NKC];
  const bool colok = qcol < M;
  auto load_eh = [&]() {
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      be[kc] = f32x4{0.f, 0.f, 0.f, 0.f};
      const int p0 = 16 * kc + 4 * q4;
      if (colok) {
        if ((M & 3) == 0 && p0 + 4 <= M) {
          be[kc] = *reinterpret_cast<const f32x4*>(Eh32 + (size_t)qcol * M + p0);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (p0 + e < M) be[kc][e] = Eh32[(size_t)qcol * M + p0 + e];
        }
      }
    }
  };
  load_eh();
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
    bar_[kc] = f32x4{0.f, 0.f, 0.f, 0.f};
    bai[kc] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int p0 = 16 * kc + 4 * q4;
    if (colok) {
      bar_[kc] = apk_load4(Are + (size_t)w * MA, M, qcol, p0);
      bai[kc] = apk_load4(Aim + (size_t)w * MA, M, qcol, p0);
    }
    bas[kc] = bar_[kc] + bai[kc];
  }
  __syncthreads();

  f32x4 yre[NRB], yim[NRB], cre[NRB], cim[NRB];
  // X = U E_h  (real B operand)
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    cre[rb] = f32x4{};
    cim[rb] = f32x4{};
  }
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      const f32x4 ar = *reinterpret_cast<const f32x4*>(&Tr[(16 * rb + j) * ldt + 16 * kc + 4 * q4]);
      const f32x4 ai = *reinterpret_cast<const f32x4*>(&Ti[(16 * rb + j) * ldt + 16 * kc + 4 * q4]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        cre[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[e], be[kc][e], cre[rb], 0, 0, 0);
        cim[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[e], be[kc][e], cim[rb], 0, 0, 0);
      }
    }
  }
  __syncthreads();
  // write X back as the first term, Y = X
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    yre[rb] = cre[rb];
    yim[rb] = cim[rb];
    if (qcol < Kp) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Tr[(16 * rb + 4 * q4 + v) * ldt + qcol] = cre[rb][v];
        Ti[(16 * rb + 4 * q4 + v) * ldt + qcol] = cim[rb][v];
      }
    }
  }
  __syncthreads();
  // Taylor terms: T <- T A / n, Y += T.  The complex product takes three real ones,
  // P1 = Tr Ar, P2 = Ti Ai, P3 = (Tr + Ti)(Ar + Ai): Re = P1 - P2, Im = P3 - P1 - P2.
  for (int n = 1; n <= n_taylor; ++n) {
    f32x4 p1[NRB], p2[NRB], p3[NRB];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        const f32x4 ar = *reinterpret_cast<const f32x4*>(&Tr[(16 * rb + j) * ldt + 16 * kc + 4 * q4]);
        const f32x4 ai = *reinterpret_cast<const f32x4*>(&Ti[(16 * rb + j) * ldt + 16 * kc + 4 * q4]);
        const f32x4 as = ar + ai;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool first = kc == 0 && e == 0;
          p1[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[e], bar_[kc][e], first ? f32x4{} : p1[rb], 0, 0, 0);
          p2[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[e], bai[kc][e], first ? f32x4{} : p2[rb], 0, 0, 0);
          p3[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[e], bas[kc][e], first ? f32x4{} : p3[rb], 0, 0, 0);
        }
      }
    }
    const float inv = 1.0f / (float)n;
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      cre[rb] = (p1[rb] - p2[rb]) * inv;
      cim[rb] = (p3[rb] - p1[rb] - p2[rb]) * inv;
      yre[rb] += cre[rb];
      yim[rb] += cim[rb];
      if (qcol < Kp) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Tr[(16 * rb + 4 * q4 + v) * ldt + qcol] = cre[rb][v];
          Ti[(16 * rb + 4 * q4 + v) * ldt + qcol] = cim[rb][v];
        }
      }
    }
    __syncthreads();
  }
  // Y into the planes, then U' = Y E_h (E_h read again: the Taylor loop does not hold it)
  load_eh();
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    if (qcol < Kp) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Tr[(16 * rb + 4 * q4 + v) * ldt + qcol] = yre[rb][v];
        Ti[(16 * rb + 4 * q4 + v) * ldt + qcol] = yim[rb][v];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    cre[rb] = f32x4{};
    cim[rb] = f32x4{};
  }
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      const f32x4 ar = *reinterpret_cast<const f32x4*>(&Tr[(16 * rb + j) * ldt + 16 * kc + 4 * q4]);
      const f32x4 ai = *reinterpret_cast<const f32x4*>(&Ti[(16 * rb + j) * ldt + 16 * kc + 4 * q4]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        cre[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[e], be[kc][e], cre[rb], 0, 0, 0);
        cim[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[e], be[kc][e], cim[rb], 0, 0, 0);
      }
    }
  }
  cd* Uo = U + (size_t)w * ntot * M;
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    if (!colok) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 16 * rb + 4 * q4 + v;
      if (c < ntot) Uo[(size_t)c * M + qcol] = mkc((double)cre[rb][v], (double)cim[rb][v]);
    }
  }
}

// Fields for the FP32 A-build: Y[2w][g] = Re y, Y[2w+1][g] = Im y, zero for g >= G (< Gp).
__global__ void __launch_bounds__(256) k_y_to_f32(int nw, int G, int Gp, const cd* __restrict__ y,
                                                  float* __restrict__ Y) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)nw * Gp) return;
  const int w = (int)(e / Gp), g = (int)(e % Gp);
  cd v = mkc(0.0, 0.0);
  if (g < G) v = y[(size_t)w * G + g];
  Y[(size_t)(2 * w) * Gp + g] = (float)v.re;
  Y[(size_t)(2 * w + 1) * Gp + g] = (float)v.im;
}

// ---------------------------------------------------------------------------
// Fused propagation for the wide shapes (M up to 224, up to 64 orbitals per spin):
// u' = u E_h T_n(A) E_h for the orbitals of one spin of one walker per workgroup
// (grid: walkers x 2 spins).  As in k_propagate_f32, one wavefront per 16 output
// columns q and the current term (rows c, FP32 Re/Im planes) in LDS as the A operand;
// the B operands (columns q of E_h and of A, read as rows since both are symmetric)
// are streamed from memory one 16-wide K chunk ahead instead of being held in
// registers; a workgroup of NKC wavefronts gets 512 / ceil(NKC / 4) VGPRs per wave.
// ---------------------------------------------------------------------------
template <int NKC>
__global__ void __launch_bounds__(64 * NKC) k_propagate_f32_wide(
    int M, int nup, int ndn, int Kp, int n_taylor, const float* __restrict__ Eh32 /*[M][M]*/,
    const float* __restrict__ Are, const float* __restrict__ Aim, cd* __restrict__ U,
    const double* __restrict__ weight) {
  extern __shared__ __attribute__((aligned(16))) float tsm[];
  constexpr int RB = 4;                         // row blocks of 16 (N_s <= 64)
  const int w = blockIdx.x, s = blockIdx.y;
  const int N = s ? ndn : nup, off = s ? nup : 0, ntot = nup + ndn;
  if (N == 0 || !(weight[w] > 0.0)) return;     // uniform over the workgroup
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ldt = Kp + 4;
  float* Tr = tsm;                  // [64][ldt]
  float* Ti = tsm + 16 * RB * ldt;  // [64][ldt]
  const int j = lane & 15, q4 = lane >> 4;
  const int qcol = 16 * wave + j;   // output column owned by the lane
  const bool colok = qcol < M;
  const size_t MA = (size_t)apk_size(M);
  const int nrb = (N + 15) / 16;
  const float* Eq = Eh32 + (size_t)(colok ? qcol : 0) * M;
  const float* Aw_re = Are + (size_t)w * MA;
  const float* Aw_im = Aim + (size_t)w * MA;
  // B operand of K chunk kc: rows p = 16 kc + 4 q4 + e of column qcol (zero beyond M), of
  // E_h (full) and of A (block-packed)
  auto lda4 = [&](const float* Ap, int kc) {
    return colok ? apk_load4(Ap, M, qcol, 16 * kc + 4 * q4) : f32x4{0.f, 0.f, 0.f, 0.f};
  };
  auto ld4 = [&](const float* row, int kc) {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    const int p0 = 16 * kc + 4 * q4;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (colok && p0 + e < M) v[e] = row[p0 + e];
    return v;
  };

  const cd* Uw = U + ((size_t)w * ntot + off) * M;
  for (int e = tid; e < 16 * RB * Kp; e += blockDim.x) {
    const int c = e / Kp, p = e % Kp;
    cd v = mkc(0.0, 0.0);
    if (c < N && p < M) v = Uw[(size_t)c * M + p];
    Tr[c * ldt + p] = (float)v.re;
    Ti[c * ldt + p] = (float)v.im;
  }
  __syncthreads();

  f32x4 yre[RB], yim[RB], cre[RB], cim[RB];
  // real B (E_h): C = T E_h
  auto mul_real = [&](const float* Bq) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      cre[rb] = f32x4{};
      cim[rb] = f32x4{};
    }
    f32x4 b = ld4(Bq, 0);
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      const f32x4 bn = kc + 1 < NKC ? ld4(Bq, kc + 1) : b;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb >= nrb) break;
        const f32x4 ar = *reinterpret_cast<const f32x4*>(&Tr[(16 * rb + j) * ldt + 16 * kc + 4 * q4]);
        const f32x4 ai = *reinterpret_cast<const f32x4*>(&Ti[(16 * rb + j) * ldt + 16 * kc + 4 * q4]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          cre[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[e], b[e], cre[rb], 0, 0, 0);
          cim[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[e], b[e], cim[rb], 0, 0, 0);
        }
      }
      b = bn;
    }
  };
  auto store_planes = [&](const f32x4* pr, const f32x4* pi) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if (rb < nrb && qcol < Kp) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Tr[(16 * rb + 4 * q4 + v) * ldt + qcol] = pr[rb][v];
          Ti[(16 * rb + 4 * q4 + v) * ldt + qcol] = pi[rb][v];
        }
      }
    }
  };

  // X = U E_h; the first term and Y = X
  mul_real(Eq);
  __syncthreads();
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    yre[rb] = cre[rb];
    yim[rb] = cim[rb];
  }
  store_planes(cre, cim);
  __syncthreads();
  // Taylor terms: T <- T A / n, Y += T
  for (int n = 1; n <= n_taylor; ++n) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      cre[rb] = f32x4{};
      cim[rb] = f32x4{};
    }
    f32x4 br = lda4(Aw_re, 0), bi = lda4(Aw_im, 0);
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      const f32x4 brn = kc + 1 < NKC ? lda4(Aw_re, kc + 1) : br;
      const f32x4 bin = kc + 1 < NKC ? lda4(Aw_im, kc + 1) : bi;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb >= nrb) break;
        const f32x4 ar = *reinterpret_cast<const f32x4*>(&Tr[(16 * rb + j) * ldt + 16 * kc + 4 * q4]);
        const f32x4 ai = *reinterpret_cast<const f32x4*>(&Ti[(16 * rb + j) * ldt + 16 * kc + 4 * q4]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          cre[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[e], br[e], cre[rb], 0, 0, 0);
          cre[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[e], bi[e], cre[rb], 0, 0, 0);
          cim[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[e], bi[e], cim[rb], 0, 0, 0);
          cim[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[e], br[e], cim[rb], 0, 0, 0);
        }
      }
      br = brn;
      bi = bin;
    }
    const float inv = 1.0f / (float)n;
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      cre[rb] *= inv;
      cim[rb] *= inv;
      yre[rb] += cre[rb];
      yim[rb] += cim[rb];
    }
    store_planes(cre, cim);
    __syncthreads();
  }
  // Y into the planes, then U' = Y E_h
  store_planes(yre, yim);
  __syncthreads();
  mul_real(Eq);
  cd* Uo = U + ((size_t)w * ntot + off) * M;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    if (rb >= nrb || !colok) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 16 * rb + 4 * q4 + v;
      if (c < N) Uo[(size_t)c * M + qcol] = mkc((double)cre[rb][v], (double)cim[rb][v]);
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 A-build on v_mfma_f64_16x16x4_f64, lower triangle only (A_w is symmetric):
//   C[r][col] = sum_g Y[r][g] Lt[col][g],  r = 2w + (0: Re y, 1: Im y) read straight from the
//   interleaved complex y [nw][G],  col = packed pair p <= q,  Lt FP64 [MMh][Gp] (zero beyond G).
//   A_w[q][p] = A_w[p][q] = (-s C[2w+1][col], s C[2w][col])  (complex128 [nw][M][M]).
// Tile 64 x 64 per workgroup, K chunks of 16 double-buffered in LDS, 4 waves of 32 x 32
// (2 x 2 blocks).  Operand lanes: A[i][k] at lane i + 16k, B[k][j] at lane j + 16k;
// output lane l, item v holds D[l/16 + 4v][l%16], so rows 2w and 2w + 1 of a walker sit in
// lanes l and l + 16 (same v) and meet through one shuffle.
// ---------------------------------------------------------------------------
constexpr int AB64_B = 64, AB64_K = 16, AB64_LD = AB64_K + 2;

__global__ void __launch_bounds__(256) k_abuild_f64mfma(int nw, int G, int MMh, int MA, int Gp,
                                                        double s, const double* __restrict__ y,
                                                        const double* __restrict__ Lt,
                                                        const int2* __restrict__ pairs,
                                                        cd* __restrict__ A) {
  __shared__ __attribute__((aligned(16))) double As[2][AB64_B * AB64_LD];
  __shared__ __attribute__((aligned(16))) double Bs[2][AB64_B * AB64_LD];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rows = 2 * nw;
  const int r0 = blockIdx.x * AB64_B, c0 = blockIdx.y * AB64_B;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int l16 = lane & 15, q = lane >> 4;
  // each thread moves 4 doubles of A and 4 of B per K chunk: element e = tid + 256 i
  double pa[4], pb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 256 * i;
      const int rr = e >> 4, kk = e & 15;
      const int r = r0 + rr, c = c0 + rr, g = k0 + kk;
      pa[i] = (r < rows && g < G) ? y[((size_t)(r >> 1) * G + g) * 2 + (r & 1)] : 0.0;
      pb[i] = (c < MMh && g < Gp) ? Lt[(size_t)c * Gp + g] : 0.0;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 256 * i;
      const int rr = e >> 4, kk = e & 15;
      As[buf][rr * AB64_LD + kk] = pa[i];
      Bs[buf][rr * AB64_LD + kk] = pb[i];
    }
  };
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int nk = (G + AB64_K - 1) / AB64_K;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((kc + 1) * AB64_K);
#pragma unroll
    for (int ks = 0; ks < AB64_K / 4; ++ks) {
      double fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) fa[a] = As[buf][(wr + 16 * a + l16) * AB64_LD + 4 * ks + q];
#pragma unroll
      for (int b = 0; b < 2; ++b) fb[b] = Bs[buf][(wc + 16 * b + l16) * AB64_LD + 4 * ks + q];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    if (kc + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }
  // epilogue: lane (q even) holds row 2w's value, lane + 16 row 2w + 1's
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int cc = c0 + wc + 16 * b + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double mine = acc[a][b][v];
        const double odd = __shfl_down(mine, 16, 64);
        const int r = r0 + wr + 16 * a + q + 4 * v;   // even for even q
        if ((q & 1) || cc >= MMh || r >= rows) continue;
        const int2 pq = pairs[cc];
        const int w = r >> 1;
        const cd val = mkc(-s * odd, s * mine);
        A[(size_t)w * MA + pq.x] = val;
        if (pq.y != pq.x) A[(size_t)w * MA + pq.y] = val;
      }
    }
}

// ---------------------------------------------------------------------------
// FP64 propagation on v_mfma_f64_16x16x4_f64: u' = u E_h T_n(A) E_h for up to 32 orbitals
// (one row block) of one spin of one walker per workgroup (grid: walkers x 2 spins x row
// blocks), one wavefront per 16 output columns q.  The current term (Re / Im planes) sits
// in LDS as the A operand; the B operands (rows q of the symmetric A_w, complex128, and of
// E_h) are streamed per 16-wide K chunk.  Inside a chunk lane group q4 = lane / 16 takes
// k = 16 kc + 4 q4 + e for its four MFMAs e, on both operands, so each lane's operands are
// contiguous (the sum over k is unchanged).  Output lane l, item v: row l/16 + 4v, column l%16.
// ---------------------------------------------------------------------------
template <int NKC>
__global__ void __launch_bounds__(64 * NKC) k_propagate_f64(
    int M, int nup, int ndn, int Kp, int n_taylor, const double* __restrict__ Eh /*[M][M]*/,
    const cd* __restrict__ A /*[nw][M][M]*/, cd* __restrict__ U,
    const double* __restrict__ weight) {
  extern __shared__ __attribute__((aligned(16))) double dsm[];
  constexpr int RB = 2;                          // 16-row blocks per workgroup (32 rows)
  const int w = blockIdx.x, s = blockIdx.y, rblk = blockIdx.z;
  const int N = s ? ndn : nup, off = (s ? nup : 0) + 32 * rblk, ntot = nup + ndn;
  const int nrows = min(32, N - 32 * rblk);
  if (nrows <= 0 || !(weight[w] > 0.0)) return;  // uniform over the workgroup
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ldt = Kp + 2;
  double* Tr = dsm;                 // [32][ldt]
  double* Ti = dsm + 32 * ldt;      // [32][ldt]
  const int j = lane & 15, q4 = lane >> 4;
  const int qcol = 16 * wave + j;
  const bool colok = qcol < M;
  const size_t MM = (size_t)M * M;
  const int nrb = (nrows + 15) / 16;
  const double* Ehq = Eh + (size_t)(colok ? qcol : 0) * M;
  const cd* Aq = A + (size_t)w * MM + (size_t)(colok ? qcol : 0) * M;

  const cd* Uw = U + ((size_t)w * ntot + off) * M;
  for (int e = tid; e < 32 * Kp; e += blockDim.x) {
    const int c = e / Kp, p = e % Kp;
    cd v = mkc(0.0, 0.0);
    if (c < nrows && p < M) v = Uw[(size_t)c * M + p];
    Tr[c * ldt + p] = v.re;
    Ti[c * ldt + p] = v.im;
  }
  __syncthreads();

  f64x4 yre[RB], yim[RB], cre[RB], cim[RB];
  auto zero = [&](f64x4* a) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) a[rb] = f64x4{0.0, 0.0, 0.0, 0.0};
  };
  // real B (E_h): C = T E_h
  auto mul_real = [&]() {
    zero(cre);
    zero(cim);
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      double b[4];
      const int p0 = 16 * kc + 4 * q4;
#pragma unroll
      for (int e = 0; e < 4; ++e) b[e] = (colok && p0 + e < M) ? Ehq[p0 + e] : 0.0;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb >= nrb) break;
        const double* tr = &Tr[(16 * rb + j) * ldt + p0];
        const double* ti = &Ti[(16 * rb + j) * ldt + p0];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          cre[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(tr[e], b[e], cre[rb], 0, 0, 0);
          cim[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ti[e], b[e], cim[rb], 0, 0, 0);
        }
      }
    }
  };
  auto store_planes = [&](const f64x4* pr, const f64x4* pi) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if (rb < nrb && qcol < Kp) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Tr[(16 * rb + q4 + 4 * v) * ldt + qcol] = pr[rb][v];
          Ti[(16 * rb + q4 + 4 * v) * ldt + qcol] = pi[rb][v];
        }
      }
    }
  };

  mul_real();   // X = U E_h: the first term and Y = X
  __syncthreads();
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    yre[rb] = cre[rb];
    yim[rb] = cim[rb];
  }
  store_planes(cre, cim);
  __syncthreads();
  for (int n = 1; n <= n_taylor; ++n) {
    zero(cre);
    zero(cim);
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      double br[4], bi[4];
      const int p0 = 16 * kc + 4 * q4;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const cd a = (colok && p0 + e < M) ? Aq[p0 + e] : mkc(0.0, 0.0);
        br[e] = a.re;
        bi[e] = a.im;
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb >= nrb) break;
        const double* tr = &Tr[(16 * rb + j) * ldt + p0];
        const double* ti = &Ti[(16 * rb + j) * ldt + p0];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          cre[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(tr[e], br[e], cre[rb], 0, 0, 0);
          cre[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ti[e], bi[e], cre[rb], 0, 0, 0);
          cim[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(tr[e], bi[e], cim[rb], 0, 0, 0);
          cim[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ti[e], br[e], cim[rb], 0, 0, 0);
        }
      }
    }
    const double inv = 1.0 / (double)n;
    __syncthreads();
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      cre[rb] *= inv;
      cim[rb] *= inv;
      yre[rb] += cre[rb];
      yim[rb] += cim[rb];
    }
    store_planes(cre, cim);
    __syncthreads();
  }
  store_planes(yre, yim);   // U' = Y E_h
  __syncthreads();
  mul_real();
  cd* Uo = U + ((size_t)w * ntot + off) * M;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    if (rb >= nrb || !colok) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 16 * rb + q4 + 4 * v;
      if (c < nrows) Uo[(size_t)c * M + qcol] = mkc(cre[rb][v], cim[rb][v]);
    }
  }
}
