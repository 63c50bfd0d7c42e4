// Modified Cholesky decomposition of the two-electron tensor on the GPU
// (arXiv:1711.02242, Sec. II.B.2, eq:chol, eq:chol2).
//
// V_{mu nu} = v_pqrs with mu = p M + r, nu = q M + s, v stored as eri[p][q][r][s].
// Only the diagonal of the residual, D_mu = (V - sum_g L^g L^g^T)_{mu mu}, is kept:
// the pivot column of the residual is rebuilt from the tensor and the previous
// vectors, c_mu = V_{mu nu0} - sum_g L^g_mu L^g_nu0.  Per vector:
//   k_mcd_pivot : nu0 = argmax D (first index on ties), Dmax; stop when Dmax < delta;
//                 damped prescreening sqrt(|D_mu| Dmax) <= min(1e-9, delta) -> mu dead;
//   k_mcd_column: L_mu = c_mu / sqrt(Dmax) (0 for dead mu), D_mu -= L_mu^2.
#pragma once

#include "common.hpp"

struct McdState {
  int done;       // 1 once converged or out of vectors
  int count;      // number of vectors when done
  int piv;        // current pivot
  int pad;
  double dmax;    // current Dmax
};

__global__ void k_mcd_init(int M, const double* __restrict__ eri, double* __restrict__ D,
                           unsigned char* __restrict__ dead, McdState* __restrict__ st) {
  const int MM = M * M;
  const int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu < MM) {
    const int p = mu / M, r = mu % M;
    D[mu] = eri[(((size_t)p * M + p) * M + r) * M + r];
    dead[mu] = 0;
  }
  if (mu == 0) {
    st->done = 0;
    st->count = 0;
    st->piv = -1;
    st->dmax = 0.0;
  }
}

__global__ void __launch_bounds__(1024) k_mcd_pivot(int MM, double delta, int n, int max_vectors,
                                                    double* __restrict__ D,
                                                    unsigned char* __restrict__ dead,
                                                    McdState* __restrict__ st) {
  __shared__ double bv[16];
  __shared__ int bi[16];
  __shared__ double s_dmax;
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = st->done;
  __syncthreads();
  if (s_stop) return;
  double best = -INFINITY;
  int idx = MM;
  for (int mu = threadIdx.x; mu < MM; mu += blockDim.x) {
    const double v = D[mu];
    if (v > best) {  // strict: the first (smallest) index wins within a thread's stride
      best = v;
      idx = mu;
    }
  }
  // wave then block argmax, ties -> smallest index
  wave_argmax(best, idx);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    bv[wid] = best;
    bi[wid] = idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = -INFINITY;
    int i = MM;
    const int nwv = (blockDim.x + 63) / 64;
    for (int k = 0; k < nwv; ++k)
      if (bv[k] > b || (bv[k] == b && bi[k] < i)) {
        b = bv[k];
        i = bi[k];
      }
    s_dmax = b;
    if (!(b >= delta) || n >= max_vectors) {
      st->done = 1;
      st->count = n;
      st->dmax = b;
      s_stop = 1;
    } else {
      st->piv = i;
      st->dmax = b;
    }
  }
  __syncthreads();
  if (s_stop) return;
  const double dmax = s_dmax;
  const double screen = fmin(1e-9, delta);
  for (int mu = threadIdx.x; mu < MM; mu += blockDim.x)
    if (!dead[mu] && sqrt(fabs(D[mu]) * dmax) <= screen) {
      dead[mu] = 1;
      D[mu] = 0.0;
    }
}

__global__ void __launch_bounds__(256) k_mcd_column(int M, int n, const double* __restrict__ eri,
                                                    double* __restrict__ L /*[..][MM]*/,
                                                    double* __restrict__ D,
                                                    const unsigned char* __restrict__ dead,
                                                    const McdState* __restrict__ st) {
  if (st->done) return;
  const int MM = M * M;
  const int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu >= MM) return;
  const int nu0 = st->piv;
  const double dmax = st->dmax;
  double* Ln = L + (size_t)n * MM;
  if (dead[mu]) {
    Ln[mu] = 0.0;
    return;
  }
  const int p = mu / M, r = mu % M, q = nu0 / M, s = nu0 % M;
  double c = eri[(((size_t)p * M + q) * M + r) * M + s];
  for (int g = 0; g < n; ++g) c -= L[(size_t)g * MM + mu] * L[(size_t)g * MM + nu0];
  const double l = c / sqrt(dmax);
  Ln[mu] = l;
  D[mu] = (mu == nu0) ? 0.0 : D[mu] - l * l;
}
