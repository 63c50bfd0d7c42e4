// FP64 kernels of the walker step (arXiv:1711.02242, Sec. III.D-E).
//
// Layouts (w = walker, c = occupied orbital, spin-up orbitals first,
// p, q = basis index, g = Cholesky index):
//   U, ThetaT, Taylor buffers : cd [nw][ntot][M]   (row c = orbital c)
//   L                         : double [G][M][M]
//   Lh (half-rotated V^T L^g) : double [G][ntot][M]  (rows of spin s at off_s)
//   ht (V^T h1)               : double [ntot][M]
//   V  (trial orbitals)       : double [ntot][M]
//   A  (propagator exponent)  : cd [nw][M][M]
#pragma once

#include "common.hpp"

// Per-walker fault flags written by the overlap kernel.
#define WFLAG_SINGULAR 1u

// ---------------------------------------------------------------------------
// Local-energy contraction in FP64 (eq:localenergy3): for every g,
// Omega = Lh^g_s Theta_s (N x N), tpart[w][s][g] = tr Omega and
// exch[w][s] = sum_g tr(Omega Omega).  One block per (walker, spin).
// ---------------------------------------------------------------------------
template <bool THETA_IN_LDS>
__global__ void __launch_bounds__(256) k_contract_fp64(
    int M, int nup, int ndn, int G, const double* __restrict__ Lh, const cd* __restrict__ thetaT,
    const double* __restrict__ weight, cd* __restrict__ tpart /*[nw][2][G]*/,
    cd* __restrict__ exch /*[nw][2]*/) {
  extern __shared__ unsigned char smem_raw[];
  const int w = blockIdx.x, s = blockIdx.y;
  const int N = s == 0 ? nup : ndn;
  const int off = s == 0 ? 0 : nup;
  const int ntot = nup + ndn;
  const int tid = threadIdx.x;
  if (N == 0) {
    for (int g = tid; g < G; g += blockDim.x) tpart[((size_t)w * 2 + s) * G + g] = mkc(0.0, 0.0);
    if (tid == 0) exch[2 * w + s] = mkc(0.0, 0.0);
    return;
  }
  if (!(weight[w] > 0.0)) return;
  // Theta rows staged in LDS when they fit ([N][M+1]); otherwise read from global memory.
  const int ldt = THETA_IN_LDS ? M + 1 : M;
  cd* Ts = reinterpret_cast<cd*>(smem_raw);
  cd* Om = THETA_IN_LDS ? Ts + (size_t)N * ldt : Ts;   // [N][N+1]
  double* red = reinterpret_cast<double*>(Om + (size_t)N * (N + 1));
  const cd* Tw = thetaT + ((size_t)w * ntot + off) * M;
  if (THETA_IN_LDS)
    for (int e = tid; e < N * M; e += blockDim.x) Ts[(e / M) * ldt + e % M] = Tw[e];
  const cd* Th = THETA_IN_LDS ? Ts : Tw;
  __syncthreads();
  double xr = 0.0, xi = 0.0;
  for (int g = 0; g < G; ++g) {
    const double* Lg = Lh + ((size_t)g * ntot + off) * M;
    for (int e = tid; e < N * N; e += blockDim.x) {
      const int r = e / N, c = e % N;
      cd acc = mkc(0.0, 0.0);
      const double* lr = Lg + (size_t)r * M;
      const cd* tc = Th + (size_t)c * ldt;
      for (int p = 0; p < M; ++p) cfmar(acc, tc[p], lr[p]);
      Om[r * (N + 1) + c] = acc;
    }
    __syncthreads();
    for (int e = tid; e < N * N; e += blockDim.x) {
      const int r = e / N, c = e % N;
      const cd a = Om[r * (N + 1) + c], b = Om[c * (N + 1) + r];
      xr += a.re * b.re - a.im * b.im;
      xi += a.re * b.im + a.im * b.re;
    }
    if (tid < AFQMC_WAVE) {
      double tr = 0.0, ti = 0.0;
      for (int r = tid; r < N; r += AFQMC_WAVE) {
        tr += Om[r * (N + 1) + r].re;
        ti += Om[r * (N + 1) + r].im;
      }
      tr = wave_sum(tr);
      ti = wave_sum(ti);
      if (tid == 0) tpart[((size_t)w * 2 + s) * G + g] = mkc(tr, ti);
    }
    __syncthreads();
  }
  xr = block_sum(xr, red);
  xi = block_sum(xi, red);
  if (tid == 0) exch[2 * w + s] = mkc(xr, xi);
}

// ---------------------------------------------------------------------------
// Local-energy assembly: t_g = sum_s tpart, E_L = h0 + e1 + 1/2 (sum_g t_g^2 - exch)
// (eq:localenergy2-3 with the 1/2 of eq:bo_ham2).  One block per walker.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_energy_assemble(
    int G, double h0, double sf, const cd* __restrict__ tpart, const cd* __restrict__ exch,
    const cd* __restrict__ e1, const double* __restrict__ weight, int check_weight,
    cd* __restrict__ tcur /*[nw][G]*/, cd* __restrict__ enew /*[nw]*/) {
  __shared__ double red[8];
  const int w = blockIdx.x, tid = threadIdx.x;
  if (check_weight && !(weight[w] > 0.0)) return;
  double jr = 0.0, ji = 0.0;
  for (int g = tid; g < G; g += blockDim.x) {
    const cd t = cadd(cscale(tpart[((size_t)w * 2) * G + g], sf), tpart[((size_t)w * 2 + 1) * G + g]);
    tcur[(size_t)w * G + g] = t;
    jr += t.re * t.re - t.im * t.im;
    ji += 2.0 * t.re * t.im;
  }
  jr = block_sum(jr, red);
  ji = block_sum(ji, red);
  if (tid == 0) {
    const cd x = cadd(cscale(exch[2 * w], sf), exch[2 * w + 1]);
    const cd e = cadd(cscale(e1[2 * w], sf), e1[2 * w + 1]);
    enew[w] = mkc(h0 + e.re + 0.5 * (jr - x.re), e.im + 0.5 * (ji - x.im));
  }
}

// Multi-determinant trial Psi_T = sum_d A_d Psi_d (Sec. II.B, eq:localenergy2, eq:precomputing2).
// Per (walker, determinant) slot wd = w * n_det + d the overlap and contraction kernels have
// left logdet, wflag, e1, tpart and exch of determinant d.  With
//   r_d = conj(A_d) <Psi_d|Psi> / e^{ref},  ref = max_d log|<Psi_d|Psi>|,  R = sum_d r_d,
// this kernel forms the mixed local energy E_L = sum_d r_d E_L^d / R, the force-bias traces
// t_g = sum_d r_d t^d_g / R and log <Psi_T|Psi> = log R + ref.  Determinants with an exactly
// singular overlap matrix have r_d = 0 and are skipped (their energy term is dropped, exact only
// for walkers non-orthogonal to every determinant).  The combined log-overlap is written as a
// spin pair (log/sf, 0) so that sf * first + second reproduces it in the weight kernels; a walker
// with no usable determinant (or R = 0) is flagged singular.  One block per walker.
constexpr int AFQMC_MAX_DETS = 1024;
__global__ void __launch_bounds__(256) k_energy_assemble_multi(
    int G, int n_det, double h0, double sf, const double* __restrict__ coef /*[n_det][2]*/,
    const cd* __restrict__ tpart, const cd* __restrict__ exch, const cd* __restrict__ e1,
    const cd* __restrict__ logdet, const unsigned* __restrict__ wflag,
    const double* __restrict__ weight, int check_weight, cd* __restrict__ tcur /*[nw][G]*/,
    cd* __restrict__ enew /*[nw]*/, cd* __restrict__ ldc /*[nw][2]*/,
    unsigned* __restrict__ wflc /*[nw][2]*/) {
  __shared__ double red[8];
  __shared__ cd s_r[AFQMC_MAX_DETS];    // r_d / R
  __shared__ cd s_lg[AFQMC_MAX_DETS];   // log <Psi_d|Psi>
  __shared__ int s_ok[AFQMC_MAX_DETS];
  __shared__ cd s_esum;
  __shared__ int s_bad, s_first;
  const int w = blockIdx.x, tid = threadIdx.x;
  if (check_weight && !(weight[w] > 0.0)) return;
  for (int d = tid; d < n_det; d += blockDim.x) {
    const size_t wd = (size_t)w * n_det + d;
    const cd l0 = logdet[2 * wd], l1 = logdet[2 * wd + 1];
    const unsigned fl = wflag[2 * wd] | wflag[2 * wd + 1];
    s_lg[d] = mkc(sf * l0.re + l1.re, sf * l0.im + l1.im);
    s_ok[d] = (fl & WFLAG_SINGULAR) ? 0 : 1;
  }
  __syncthreads();
  if (tid == 0) {
    double ref = -INFINITY;
    int first = -1;
    for (int d = 0; d < n_det; ++d)
      if (s_ok[d]) {
        ref = fmax(ref, s_lg[d].re);
        if (first < 0) first = d;
      }
    s_first = first;
    cd R = mkc(0.0, 0.0);
    for (int d = 0; d < n_det; ++d) {
      cd r = mkc(0.0, 0.0);
      if (s_ok[d]) {
        const double m = exp(s_lg[d].re - ref);
        // conj(A_d) * e^{lg - ref}
        r = cconjmul(mkc(coef[2 * d], coef[2 * d + 1]), mkc(m * cos(s_lg[d].im), m * sin(s_lg[d].im)));
      }
      s_r[d] = r;
      R = cadd(R, r);
    }
    const bool bad = !(ref > -INFINITY) || !(R.re != 0.0 || R.im != 0.0) || !cfinite(R);
    s_bad = bad ? 1 : 0;
    if (!bad) {
      for (int d = 0; d < n_det; ++d) s_r[d] = cdiv(s_r[d], R);
      const double lre = log(sqrt(R.re * R.re + R.im * R.im)) + ref;
      const double lim = atan2(R.im, R.re);
      ldc[2 * w] = mkc(lre / sf, lim / sf);
    } else {
      ldc[2 * w] = mkc(-INFINITY, 0.0);
    }
    ldc[2 * w + 1] = mkc(0.0, 0.0);
    wflc[2 * w] = bad ? WFLAG_SINGULAR : 0u;
    wflc[2 * w + 1] = 0u;
    s_esum = mkc(0.0, 0.0);
  }
  __syncthreads();
  if (s_bad) return;
  for (int d = 0; d < n_det; ++d) {
    if (!s_ok[d]) continue;  // uniform over the block
    const size_t wd = (size_t)w * n_det + d;
    const cd rd = s_r[d];
    double jr = 0.0, ji = 0.0;
    for (int g = tid; g < G; g += blockDim.x) {
      const cd t = cadd(cscale(tpart[(wd * 2) * G + g], sf), tpart[(wd * 2 + 1) * G + g]);
      const cd c = cmul(rd, t);
      // the first usable determinant writes, later ones accumulate (same thread owns g)
      tcur[(size_t)w * G + g] = (d == s_first) ? c : cadd(tcur[(size_t)w * G + g], c);
      jr += t.re * t.re - t.im * t.im;
      ji += 2.0 * t.re * t.im;
    }
    jr = block_sum(jr, red);
    ji = block_sum(ji, red);
    if (tid == 0) {
      const cd x = cadd(cscale(exch[2 * wd], sf), exch[2 * wd + 1]);
      const cd e = cadd(cscale(e1[2 * wd], sf), e1[2 * wd + 1]);
      const cd ed = mkc(h0 + e.re + 0.5 * (jr - x.re), e.im + 0.5 * (ji - x.im));
      s_esum = cadd(s_esum, cmul(rd, ed));
    }
  }
  if (tid == 0) enew[w] = s_esum;
}

// ---------------------------------------------------------------------------
// Auxiliary fields and force bias (eq:hs2, eq:fb, eq:precomputing2, App. B.1):
// x from the Philox stream (or given), xbar = -i s t capped in modulus,
// y = x - xbar.  One thread per (walker, block of 4 fields).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fields(
    int nw, int G, double s, double fb_cap, const cd* __restrict__ tcur,
    const double* __restrict__ weight, const int64_t* __restrict__ walker_id, uint64_t seed,
    uint64_t job, int64_t step_arg, const int64_t* __restrict__ dstep,
    const double* __restrict__ xin, cd* __restrict__ y,
    double* __restrict__ xout, unsigned* __restrict__ status, cd* __restrict__ fbterm,
    const double* __restrict__ lbar, cd* __restrict__ mfterm,
    unsigned long long* __restrict__ counts) {
  // the step number comes from the device counter when one is given (graph replays)
  const int64_t step = dstep ? *dstep : step_arg;
  const int nblk = (G + 3) / 4;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nw * nblk) return;
  const int w = (int)(idx / nblk), b = (int)(idx % nblk);
  double x[4];
  if (xin) {
    for (int j = 0; j < 4; ++j) x[j] = (4 * b + j < G) ? xin[(size_t)w * G + 4 * b + j] : 0.0;
  } else {
    const u64x4 r = philox4x64_10((uint64_t)b, (uint64_t)walker_id[w], (uint64_t)step, 0ull,
                                  seed, job);
    const double u0 = u64_unit(r.v[0]), u1 = u64_unit(r.v[1]);
    const double u2 = u64_unit(r.v[2]), u3 = u64_unit(r.v[3]);
    const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
    const double a1 = 2.0 * M_PI * u1, a3 = 2.0 * M_PI * u3;
    x[0] = r0 * cos(a1);
    x[1] = r0 * sin(a1);
    x[2] = r1 * cos(a3);
    x[3] = r1 * sin(a3);
  }
  if (xout) {
    for (int j = 0; j < 4; ++j)
      if (4 * b + j < G) xout[(size_t)w * G + 4 * b + j] = x[j];
    return;
  }
  const bool alive = weight[w] > 0.0;
  bool capped = false;
  unsigned ncap = 0;
  double fr = 0.0, fi = 0.0;  // sum over the block of x xbar - xbar^2 / 2 (eq:hybrid-wt)
  double mr = 0.0, mi = 0.0;  // sum over the block of y_g lbar_g (mean-field c-number)
  for (int j = 0; j < 4; ++j) {
    const int g = 4 * b + j;
    if (g >= G) break;
    cd yv = mkc(0.0, 0.0);
    if (alive) {
      const cd t = tcur[(size_t)w * G + g];
      const double lb = lbar[g];
      // xbar = -i s (t - lbar) = (s t.im, -s (t.re - lbar))
      double br = s * t.im, bi = -s * (t.re - lb);
      const double mod = hypot(br, bi);
      if (mod > fb_cap) {
        br *= fb_cap / mod;
        bi *= fb_cap / mod;
        capped = true;
        ++ncap;
      }
      yv = mkc(x[j] - br, -bi);
      fr += x[j] * br - 0.5 * (br * br - bi * bi);
      fi += x[j] * bi - br * bi;
      mr += yv.re * lb;
      mi += yv.im * lb;
    }
    y[(size_t)w * G + g] = yv;
  }
  if (fbterm) fbterm[(size_t)w * nblk + b] = mkc(fr, fi);
  // log of exp(-i s sum y lbar) = (s Im(sum y lbar), -s Re(sum y lbar))
  if (mfterm) mfterm[(size_t)w * nblk + b] = mkc(s * mi, -s * mr);
  if (capped) atomicOr(status, 0x10u);
  if (counts)
    for (unsigned j = 1; j <= 4; ++j) wave_count(&counts[CAP_FB], ncap >= j);
}


// ---------------------------------------------------------------------------
// Batched complex product out^T[c][i] = scale * sum_k Mat[i][k] in^T[c][k] for one
// walker per blockIdx.z (Theorem 1.4: applying exp(A) to the orbitals).
// MODE 0: out = r.  MODE 1: out = r, Y = r.  MODE 2: out = r, Y += r.
// REALMAT: Mat is one real M x M matrix shared by all walkers (exp(-dtau/2 v0)).
// Tile: 64 rows i x 32 orbitals c per block, K chunks of 16.
// ---------------------------------------------------------------------------
template <int MODE, bool REALMAT>
__global__ void __launch_bounds__(256) k_zmatmul_fp64(int M, int ntot, const void* __restrict__ Mat,
                                                      const cd* __restrict__ in, cd* __restrict__ out,
                                                      cd* __restrict__ Y, double scale,
                                                      const double* __restrict__ weight) {
  constexpr int TI = 64, TC = 32, TK = 16;
  __shared__ cd sA[TK][TI + 1];
  __shared__ cd sB[TK][TC + 1];
  const int w = blockIdx.z;
  if (!(weight[w] > 0.0)) return;
  const int i0 = blockIdx.x * TI, c0 = blockIdx.y * TC;
  const int tid = threadIdx.x;
  const int ti = tid % 16, tc = tid / 16;   // thread owns rows ti + 16*a (a<4), cols tc + 16*b (b<2)
  const cd* inw = in + (size_t)w * ntot * M;
  const cd* Aw = REALMAT ? nullptr : reinterpret_cast<const cd*>(Mat) + (size_t)w * M * M;
  const double* Ar = REALMAT ? reinterpret_cast<const double*>(Mat) : nullptr;
  cd acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = mkc(0.0, 0.0);
  for (int k0 = 0; k0 < M; k0 += TK) {
    for (int e = tid; e < TI * TK; e += 256) {
      const int ii = e / TK, kk = e % TK;
      const int i = i0 + ii, k = k0 + kk;
      cd v = mkc(0.0, 0.0);
      if (i < M && k < M) v = REALMAT ? mkc(Ar[(size_t)i * M + k], 0.0) : Aw[(size_t)i * M + k];
      sA[kk][ii] = v;
    }
    for (int e = tid; e < TC * TK; e += 256) {
      const int cc = e / TK, kk = e % TK;
      const int c = c0 + cc, k = k0 + kk;
      sB[kk][cc] = (c < ntot && k < M) ? inw[(size_t)c * M + k] : mkc(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      cd av[4], bv[2];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sA[kk][ti + 16 * a];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = sB[kk][tc + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) cfma(acc[a][b], av[a], bv[b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + ti + 16 * a;
    if (i >= M) continue;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int c = c0 + tc + 16 * b;
      if (c >= ntot) continue;
      const size_t o = ((size_t)w * ntot + c) * M + i;
      const cd r = cscale(acc[a][b], scale);
      out[o] = r;
      if (MODE == 1) Y[o] = r;
      if (MODE == 2) Y[o] = cadd(Y[o], r);
    }
  }
}

// ---------------------------------------------------------------------------
// Modified Gram-Schmidt on the orbitals of one (walker, spin) (Sec. III.D.5):
// column k is normalized, then its projection is removed from every later
// column.  Rows of U (orbital-major) are updated in place in global memory.
// ---------------------------------------------------------------------------
template <bool IN_LDS>
__global__ void __launch_bounds__(256) k_mgs(int M, int nup, int ndn, cd* __restrict__ U,
                                             const double* __restrict__ weight,
                                             unsigned* __restrict__ status,
                                             double* __restrict__ logR /*[nw][2]*/) {
  // IN_LDS: the N x M block is staged in LDS (dynamic, N M complex), orthonormalized there and
  // written back once; otherwise it is processed in place in global memory.
  extern __shared__ __attribute__((aligned(16))) unsigned char mgs_smem[];
  __shared__ cd dots[64];
  __shared__ double s_norm;
  const int w = blockIdx.x, s = blockIdx.y;
  const int N = s == 0 ? nup : ndn;
  const int off = s == 0 ? 0 : nup;
  const int ntot = nup + ndn;
  if (N == 0) {
    if (threadIdx.x == 0) logR[2 * w + s] = 0.0;
    return;
  }
  if (!(weight[w] > 0.0)) return;
  cd* Ug = U + ((size_t)w * ntot + off) * M;
  const int tid = threadIdx.x, lane = tid % AFQMC_WAVE, wid = tid / AFQMC_WAVE;
  cd* Uw = IN_LDS ? reinterpret_cast<cd*>(mgs_smem) : Ug;
  if (IN_LDS) {
    for (int e = tid; e < N * M; e += blockDim.x) Uw[e] = Ug[e];
    __syncthreads();
  }
  double lr = 0.0;  // sum_k log r_kk: QR divides <Phi_T|Psi> by det R (Theorem 1.5)
  const int nwave = blockDim.x / AFQMC_WAVE;
  for (int k = 0; k < N; ++k) {
    cd* qk = Uw + (size_t)k * M;
    if (wid == 0) {
      double nn = 0.0;
      for (int p = lane; p < M; p += AFQMC_WAVE) nn += qk[p].re * qk[p].re + qk[p].im * qk[p].im;
      nn = wave_sum(nn);
      if (lane == 0) s_norm = sqrt(nn);
    }
    __syncthreads();
    const double nrm = s_norm;
    if (!(nrm > 0.0) && tid == 0) atomicOr(status, 0x2u);
    lr += log(nrm);
    const double inv = 1.0 / nrm;
    for (int p = tid; p < M; p += blockDim.x) qk[p] = cscale(qk[p], inv);
    __syncthreads();
    // dots for the later columns, one wavefront per column
    for (int j0 = k + 1; j0 < N; j0 += 64) {
      for (int j = j0 + wid; j < min(N, j0 + 64); j += nwave) {
        const cd* uj = Uw + (size_t)j * M;
        double dr = 0.0, di = 0.0;
        for (int p = lane; p < M; p += AFQMC_WAVE) {
          const cd v = cconjmul(qk[p], uj[p]);
          dr += v.re;
          di += v.im;
        }
        dr = wave_sum(dr);
        di = wave_sum(di);
        if (lane == 0) dots[j - j0] = mkc(dr, di);
      }
      __syncthreads();
      const int nj = min(N, j0 + 64) - j0;
      for (int e = tid; e < nj * M; e += blockDim.x) {
        const int j = j0 + e / M, p = e % M;
        cfms(Uw[(size_t)j * M + p], dots[j - j0], qk[p]);
      }
      __syncthreads();
    }
  }
  if (IN_LDS)
    for (int e = tid; e < N * M; e += blockDim.x) Ug[e] = Uw[e];
  if (tid == 0) logR[2 * w + s] = lr;
}

// ---------------------------------------------------------------------------
// The same modified Gram-Schmidt (Sec. III.D.5) for N <= 32 and M <= 64 NE with the rows in
// registers: wavefront t of the four holds rows j = 4 s + t (s < 8), elements p = lane + 64 e
// (e < NE) of each.  Step k: the wavefront of row k normalizes it and puts it in LDS (two
// buffers, so one barrier per step suffices); every wavefront then removes its projection
// from its own rows j > k.  log det R is summed per wavefront, then over the four.
// ---------------------------------------------------------------------------
template <int NE>
__global__ void __launch_bounds__(256) k_mgs_reg(int M, int nup, int ndn, cd* __restrict__ U,
                                                 const double* __restrict__ weight,
                                                 unsigned* __restrict__ status,
                                                 double* __restrict__ logR) {
  __shared__ __attribute__((aligned(16))) cd qb[2][64 * NE];
  __shared__ double lrs[4];
  const int w = blockIdx.x, s = blockIdx.y;
  const int N = s == 0 ? nup : ndn;
  const int off = s == 0 ? 0 : nup;
  const int ntot = nup + ndn;
  const int tid = threadIdx.x, lane = tid & 63;
  if (N == 0) {
    if (tid == 0) logR[2 * w + s] = 0.0;
    return;
  }
  if (!(weight[w] > 0.0)) return;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  cd* Ug = U + ((size_t)w * ntot + off) * M;
  cd r[8][NE];
#pragma unroll
  for (int s8 = 0; s8 < 8; ++s8) {
    const int j = 4 * s8 + wave;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int p = lane + 64 * e;
      r[s8][e] = j < N && p < M ? Ug[(size_t)j * M + p] : mkc(0.0, 0.0);
    }
  }
  double lr = 0.0;   // sum of log r_kk over this wavefront's rows
  for (int k = 0; k < N; ++k) {
    if (wave == (k & 3)) {
      // row k is slot k / 4: selected by a compile-time slot index, so r stays in registers
#pragma unroll
      for (int s8 = 0; s8 < 8; ++s8) {
        if (s8 != (k >> 2)) continue;
        double nn = 0.0;
#pragma unroll
        for (int e = 0; e < NE; ++e) nn += r[s8][e].re * r[s8][e].re + r[s8][e].im * r[s8][e].im;
        nn = wave_sum(nn);
        const double nrm = sqrt(nn);
        if (!(nrm > 0.0) && lane == 0) atomicOr(status, 0x2u);
        lr += log(nrm);
        const double inv = 1.0 / nrm;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          r[s8][e] = cscale(r[s8][e], inv);
          qb[k & 1][lane + 64 * e] = r[s8][e];
        }
      }
    }
    __syncthreads();
    cd q[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) q[e] = qb[k & 1][lane + 64 * e];
#pragma unroll
    for (int s8 = 0; s8 < 8; ++s8) {
      const int j = 4 * s8 + wave;
      if (j <= k || j >= N) continue;
      double dr = 0.0, di = 0.0;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const cd v = cconjmul(q[e], r[s8][e]);
        dr += v.re;
        di += v.im;
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
#pragma unroll
      for (int e = 0; e < NE; ++e) cfms(r[s8][e], mkc(dr, di), q[e]);
    }
  }
#pragma unroll
  for (int s8 = 0; s8 < 8; ++s8) {
    const int j = 4 * s8 + wave;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int p = lane + 64 * e;
      if (j < N && p < M) Ug[(size_t)j * M + p] = r[s8][e];
    }
  }
  if (lane == 0) lrs[wave] = lr;
  __syncthreads();
  if (tid == 0) logR[2 * w + s] = lrs[0] + lrs[1] + lrs[2] + lrs[3];
}

// ---------------------------------------------------------------------------
// Weight update, one thread per walker.
//   mode 0 phaseless local energy (eq:if_rle, eq:cap):
//          W <- min(w_max, W exp(-dtau (Re E_L^cap(old) - E_T)) max(0, cos dtheta)),
//          Re E_L capped to the centre +- ecap_half; E_T and the centre come from the
//          population's growth state (k_growth_sum)
//   mode 1 phaseless hybrid (eq:hybrid-wt): W <- min(w_max, W |I| max(0, cos dtheta))
//   mode 2 free projection (Sec. II.C): W e^{i theta} <- W e^{i theta} I
// with log I = log(<Phi_T|Psi'>/<Phi_T|Psi>) - dtau (h0 - E_T) + sum_g (x xbar - xbar^2/2),
// where <Phi_T|Psi'> is taken before this step's QR (log det R added back).
// ---------------------------------------------------------------------------
__global__ void k_weights(int nw, int mode, double sf, double dtau, double h0,
                          const double* __restrict__ growth, double ecap_half, double w_max,
                          const cd* __restrict__ logdet,
                          const unsigned* __restrict__ wflag, const cd* __restrict__ enew,
                          const cd* __restrict__ fbterm, const cd* __restrict__ mfterm, int nblk,
                          const double* __restrict__ logR,
                          double* __restrict__ weight, double* __restrict__ arg_ovlp,
                          double* __restrict__ log_ovlp, cd* __restrict__ e_loc,
                          double* __restrict__ phase, unsigned* __restrict__ status,
                          unsigned long long* __restrict__ counts) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const double W = weight[w];
  if (!(W > 0.0)) return;
  const double e_trial = growth[GR_ET];
  const double e_bar = growth[GR_EBAR];
  unsigned st = 0u;
  const cd l0 = logdet[2 * w], l1 = logdet[2 * w + 1];
  double a = sf * l0.im + l1.im;
  a = a - 2.0 * M_PI * floor((a + M_PI) / (2.0 * M_PI));   // (-pi, pi]
  if (a <= -M_PI) a += 2.0 * M_PI;
  const double la = sf * l0.re + l1.re;
  const cd en = enew[w];
  const unsigned fl = wflag[2 * w] | wflag[2 * w + 1];
  // mean-field c-number on the overlap ratio (zero without subtraction)
  double mre = 0.0, mim = 0.0;
  if (mfterm)
    for (int b = 0; b < nblk; ++b) {
      const cd f = mfterm[(size_t)w * nblk + b];
      mre += f.re;
      mim += f.im;
    }
  double Wn;
  if (fl & WFLAG_SINGULAR) {
    Wn = 0.0;
    st |= 0x2u;
  } else if (!cfinite(en) || !isfinite(a) || !isfinite(la)) {
    Wn = 0.0;
    st |= 0x1u;
  } else if (mode == 0) {
    const cd eo = e_loc[w];
    double ec = eo.re;
    if (ec < e_bar - ecap_half) {
      ec = e_bar - ecap_half;
      st |= 0x4u;
    } else if (ec > e_bar + ecap_half) {
      ec = e_bar + ecap_half;
      st |= 0x4u;
    }
    const double proj = fmax(0.0, cos(a - arg_ovlp[w] + mim));
    if (!(proj > 0.0)) st |= 0x20u;
    Wn = W * exp(-dtau * (ec - e_trial)) * proj;
    if (Wn > w_max) {
      Wn = w_max;
      st |= 0x8u;
    }
  } else {
    double fr = 0.0, fi = 0.0;
    for (int b = 0; b < nblk; ++b) {
      const cd f = fbterm[(size_t)w * nblk + b];
      fr += f.re;
      fi += f.im;
    }
    const double lr = logR ? sf * logR[2 * w] + logR[2 * w + 1] : 0.0;
    const double lre = (la + lr - log_ovlp[w]) + mre - dtau * (h0 - e_trial) + fr;
    const double lim = (a - arg_ovlp[w]) + mim + fi;
    if (mode == 1) {
      const double proj = fmax(0.0, cos(a - arg_ovlp[w] + mim));
      if (!(proj > 0.0)) st |= 0x20u;
      Wn = W * exp(lre) * proj;
      if (Wn > w_max) {
        Wn = w_max;
        st |= 0x8u;
      }
    } else {
      Wn = W * exp(lre);
      double th = phase[w] + lim;
      th = th - 2.0 * M_PI * floor((th + M_PI) / (2.0 * M_PI));
      if (th <= -M_PI) th += 2.0 * M_PI;
      phase[w] = th;
      if (!isfinite(Wn)) {
        Wn = 0.0;
        st |= 0x1u;
      }
    }
  }
  weight[w] = Wn;
  arg_ovlp[w] = a;
  log_ovlp[w] = la;
  e_loc[w] = en;
  if (st) atomicOr(status, st);
  if (counts) {
    wave_count(&counts[CAP_E], (st & 0x4u) != 0u);
    wave_count(&counts[CAP_W], (st & 0x8u) != 0u);
    wave_count(&counts[CAP_LIVE], true);
  }
}

// ---------------------------------------------------------------------------
// Growth phase (App. B.1, B.2): the trial energy E_T of the importance function and the
// centre of the local-energy cap (eq:cap) of one walker population, in the workspace:
//   g[GR_ET] E_T, g[GR_EBAR] cap centre, and the sums over the current population-control
//   block: g[GR_NUM] of the total weight after each step, g[GR_DEN] of the total weight
//   before it, g[GR_SWE] of sum_w W Re E_L (uncapped), g[GR_SW] of sum_w W (live walkers).
// At the block's last step (the comb step) of the growth phase
//   E_T <- E_T - log(num / den) / dtau       (eq:corsam, with the -1/dtau of eq:whycorsam)
//   centre <- swe / sw                       (the local energy averaged over the block)
// and the sums restart.  Both values stay fixed outside the growth phase.
// ---------------------------------------------------------------------------
// Precision guard of the mixed modes: the live walkers whose largest |Theta_pc| over spins
// and determinants exceeds `limit`, listed in walker order in wlist, and their number in
// *wcount (added to counts[CAP_GUARD] when counts != NULL).  One workgroup of 1024 threads,
// each taking a contiguous range of walkers; the list offsets come from one sequential scan.
__global__ void __launch_bounds__(1024) k_guard_list(int nw, int nd, double limit,
                                                     const double* __restrict__ weight,
                                                     const double* __restrict__ thmax,
                                                     int* __restrict__ wlist,
                                                     int* __restrict__ wcount,
                                                     unsigned long long* __restrict__ counts) {
  __shared__ int part[1024];
  const int T = blockDim.x, t = threadIdx.x;
  const int per = (nw + T - 1) / T;
  const int lo = min(nw, t * per), hi = min(nw, lo + per);
  auto flagged = [&](int w) {
    if (!(weight[w] > 0.0)) return false;
    double m = 0.0;
    for (int i = 0; i < 2 * nd; ++i) m = fmax(m, thmax[(size_t)w * 2 * nd + i]);
    return m > limit;
  };
  int c = 0;
  for (int w = lo; w < hi; ++w) c += flagged(w) ? 1 : 0;
  part[t] = c;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int i = 0; i < T; ++i) {
      const int v = part[i];
      part[i] = acc;
      acc += v;
    }
    *wcount = acc;
    if (counts && acc > 0) atomicAdd(&counts[CAP_GUARD], (unsigned long long)acc);
  }
  __syncthreads();
  int o = part[t];
  for (int w = lo; w < hi; ++w)
    if (flagged(w)) wlist[o++] = w;
}

__global__ void k_clear_u64(unsigned long long* __restrict__ c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0ull;
}

__global__ void k_growth_init(double* __restrict__ g, double e_trial) {
  if (threadIdx.x < GR_COUNT) g[threadIdx.x] = threadIdx.x <= GR_EBAR ? e_trial : 0.0;
}

// after == 0: before the weight update, den += sum W.  after == 1: num += sum W,
// swe += sum W Re E_L, sw += sum W, then the update at a block end.  One block of 256.
__global__ void __launch_bounds__(256) k_growth_sum(int nw, int after, int block_end, double dtau,
                                                    const double* __restrict__ weight,
                                                    const cd* __restrict__ e_loc,
                                                    double* __restrict__ g) {
  __shared__ double red[4];
  double a = 0.0, b = 0.0;
  for (int w = threadIdx.x; w < nw; w += blockDim.x) {
    const double W = weight[w];
    if (W > 0.0) {
      a += W;
      if (after) b += W * e_loc[w].re;
    }
  }
  a = block_sum(a, red);
  if (after) b = block_sum(b, red);
  if (threadIdx.x != 0) return;
  if (!after) {
    g[GR_DEN] += a;
    return;
  }
  g[GR_NUM] += a;
  g[GR_SWE] += b;
  g[GR_SW] += a;
  if (block_end) {
    if (g[GR_NUM] > 0.0 && g[GR_DEN] > 0.0) g[GR_ET] = g[GR_ET] - log(g[GR_NUM] / g[GR_DEN]) / dtau;
    if (g[GR_SW] > 0.0) g[GR_EBAR] = g[GR_SWE] / g[GR_SW];
    g[GR_NUM] = g[GR_DEN] = g[GR_SWE] = g[GR_SW] = 0.0;
  }
}

// Initialization / measurement: phase and log of the overlap, E_L, from logdet and enew.
__global__ void k_measure_finish(int nw, double sf, const cd* __restrict__ logdet,
                                 const unsigned* __restrict__ wflag, const cd* __restrict__ enew,
                                 double* __restrict__ weight, double* __restrict__ arg_ovlp,
                                 double* __restrict__ log_ovlp, cd* __restrict__ e_loc,
                                 unsigned* __restrict__ status) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const cd l0 = logdet[2 * w], l1 = logdet[2 * w + 1];
  double a = sf * l0.im + l1.im;
  a = a - 2.0 * M_PI * floor((a + M_PI) / (2.0 * M_PI));
  if (a <= -M_PI) a += 2.0 * M_PI;
  const unsigned fl = wflag[2 * w] | wflag[2 * w + 1];
  arg_ovlp[w] = a;
  log_ovlp[w] = sf * l0.re + l1.re;
  e_loc[w] = enew[w];
  if ((fl & WFLAG_SINGULAR) || !cfinite(enew[w])) {
    weight[w] = 0.0;
    atomicOr(status, (fl & WFLAG_SINGULAR) ? 0x2u : 0x1u);
  }
}

// ---------------------------------------------------------------------------
// Comb population control (Sec. III.D.4): sequential cumulative weights in walker
// order, positions (u + j) * (sum W / n), parent = walker whose half-open interval
// holds the position; every copy gets weight 1.  One thread does the scan so the
// arithmetic order is fixed.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_comb_select(int nw, const double* __restrict__ weight,
                                                      double u_given, uint64_t seed, uint64_t job,
                                                      int64_t step_arg,
                                                      const int64_t* __restrict__ dstep,
                                                      double* __restrict__ csum,
                                                      int* __restrict__ parent,
                                                      double* __restrict__ wnew,
                                                      unsigned* __restrict__ status) {
  // Cumulative weights are summed by one thread in walker order (the arithmetic order of a
  // sequential cumulative sum); the weights are staged in LDS first when they fit.  The
  // parent of each position is then found by an independent binary search.
  extern __shared__ double cs[];
  __shared__ double s_total, s_u;
  __shared__ int s_last;
  const bool in_lds = nw <= 8192;
  double* C = in_lds ? cs : csum;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) C[i] = weight[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    double u = u_given;
    if (isnan(u)) {
      const int64_t step = dstep ? *dstep : step_arg;
      const u64x4 r = philox4x64_10(0ull, 0ull, (uint64_t)step, 1ull, seed, job);
      u = u64_unit(r.v[0]);
    }
    double acc = 0.0;
    int last_alive = -1;
    for (int i = 0; i < nw; ++i) {
      const double wi = C[i];
      acc += wi;
      C[i] = acc;
      if (wi > 0.0) last_alive = i;
    }
    s_total = acc;
    s_u = u;
    s_last = last_alive;
  }
  __syncthreads();
  const double total = s_total;
  const int last_alive = s_last;
  if (!(total > 0.0) || last_alive < 0) {
    for (int j = threadIdx.x; j < nw; j += blockDim.x) parent[j] = j;
    if (threadIdx.x == 0) {
      *wnew = -1.0;
      atomicOr(status, 0x1u);
    }
    return;
  }
  const double step_w = total / (double)nw;
  const double u = s_u;
  for (int j = threadIdx.x; j < nw; j += blockDim.x) {
    const double pos = (u + (double)j) * step_w;
    // first i with C[i] > pos (half-open intervals [C_{i-1}, C_i))
    int lo = 0, hi = nw;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (C[mid] <= pos) lo = mid + 1;
      else hi = mid;
    }
    parent[j] = lo < last_alive ? lo : last_alive;
  }
  // every copy restarts at weight 1: a factor common to all weights leaves the mixed estimate
  // unchanged, and the weight cap stays relative to the mean weight (App. B.1, B.2)
  if (threadIdx.x == 0) *wnew = 1.0;
}

// Gather walker state from a snapshot by parent index.  One block per walker.
// Snapshot of every walker's state before the comb overwrites it (one block per walker).
__global__ void __launch_bounds__(256) k_comb_snapshot(
    int nw, int rowlen /*ntot*M*/, int G, const cd* __restrict__ U, const cd* __restrict__ tcur,
    const cd* __restrict__ e_loc, const double* __restrict__ arg_ovlp,
    const double* __restrict__ log_ovlp, const double* __restrict__ phase, cd* __restrict__ Usnap,
    cd* __restrict__ tsnap, cd* __restrict__ esnap, double* __restrict__ asnap,
    double* __restrict__ lsnap, double* __restrict__ psnap) {
  const int j = blockIdx.x;
  for (int e = threadIdx.x; e < rowlen; e += blockDim.x)
    Usnap[(size_t)j * rowlen + e] = U[(size_t)j * rowlen + e];
  for (int e = threadIdx.x; e < G; e += blockDim.x) tsnap[(size_t)j * G + e] = tcur[(size_t)j * G + e];
  if (threadIdx.x == 0) {
    esnap[j] = e_loc[j];
    asnap[j] = arg_ovlp[j];
    lsnap[j] = log_ovlp[j];
    if (phase) psnap[j] = phase[j];
  }
}

// Device copy of the walkers' step counter: set from the host value, or advanced by one at
// the end of a replayed step.
__global__ void k_step_set(int64_t* __restrict__ dstep, int64_t v) { *dstep = v; }
__global__ void k_step_advance(int64_t* __restrict__ dstep) { *dstep += 1; }

__global__ void __launch_bounds__(256) k_comb_gather(
    int nw, int rowlen /*ntot*M*/, int G, const int* __restrict__ parent,
    const double* __restrict__ wnew, const cd* __restrict__ Usnap, const cd* __restrict__ tsnap,
    const cd* __restrict__ esnap, const double* __restrict__ asnap,
    const double* __restrict__ lsnap, const double* __restrict__ psnap, cd* __restrict__ U,
    cd* __restrict__ tcur, cd* __restrict__ e_loc, double* __restrict__ arg_ovlp,
    double* __restrict__ log_ovlp, double* __restrict__ phase, double* __restrict__ weight,
    int64_t* __restrict__ walker_id) {
  const int j = blockIdx.x;
  const double wv = *wnew;
  if (!(wv > 0.0)) return;
  const int pj = parent[j];
  for (int e = threadIdx.x; e < rowlen; e += blockDim.x)
    U[(size_t)j * rowlen + e] = Usnap[(size_t)pj * rowlen + e];
  for (int e = threadIdx.x; e < G; e += blockDim.x)
    tcur[(size_t)j * G + e] = tsnap[(size_t)pj * G + e];
  if (threadIdx.x == 0) {
    e_loc[j] = esnap[pj];
    arg_ovlp[j] = asnap[pj];
    log_ovlp[j] = lsnap[pj];
    if (phase) phase[j] = psnap[pj];
    weight[j] = wv;
    walker_id[j] = j;
  }
}

// ---------------------------------------------------------------------------
// Mixed-estimator sums (eq:localenergy, theta = 0) in a fixed reduction order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_energy_sum(int nw, int free_proj,
                                                    const double* __restrict__ growth,
                                                    double ecap_half,
                                                    const double* __restrict__ weight,
                                                    const double* __restrict__ phase,
                                                    const cd* __restrict__ e_loc,
                                                    const unsigned* __restrict__ status,
                                                    double* __restrict__ out) {
  // c = W e^{i theta}: sums of c E (Re, Im), of c (Re, Im) and the live count.  The local
  // energy is capped (eq:cap) around the population's cap centre in the phaseless modes and
  // taken as is in free projection.
  __shared__ double red[8];
  const double e_bar = growth[GR_EBAR];
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0, f = 0.0;
  for (int w = threadIdx.x; w < nw; w += blockDim.x) {
    const double W = weight[w];
    if (W > 0.0) {
      const cd e = e_loc[w];
      double cr = W, ci = 0.0;
      double er = e.re;
      if (free_proj) {
        cr = W * cos(phase[w]);
        ci = W * sin(phase[w]);
      } else {
        er = fmin(fmax(e.re, e_bar - ecap_half), e_bar + ecap_half);
      }
      a += cr * er - ci * e.im;
      b += cr * e.im + ci * er;
      c += cr;
      f += ci;
      d += 1.0;
    }
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  c = block_sum(c, red);
  d = block_sum(d, red);
  f = block_sum(f, red);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
    out[2] = c;
    out[3] = d;
    out[4] = status ? (double)*status : 0.0;
    out[5] = f;
  }
}

// Walkers start as the trial: U[w] = V (as complex), W = 1, id = w.
__global__ void k_init_walkers(int nw, int rowlen, const double* __restrict__ V,
                               cd* __restrict__ U, double* __restrict__ weight,
                               int64_t* __restrict__ walker_id, double* __restrict__ phase) {
  const int w = blockIdx.x;
  for (int e = threadIdx.x; e < rowlen; e += blockDim.x)
    U[(size_t)w * rowlen + e] = mkc(V[e], 0.0);
  if (threadIdx.x == 0) {
    weight[w] = 1.0;
    walker_id[w] = w;
    if (phase) phase[w] = 0.0;
  }
}
