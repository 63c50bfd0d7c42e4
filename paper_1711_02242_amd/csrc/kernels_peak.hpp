// Attainable dense MFMA rate of the device: every wavefront runs MFMA instructions of one
// kind on register operands only (no memory traffic) into four accumulators, each
// instruction reading a different pair of operand registers, 8 (BF16: 2) such groups per
// loop iteration so that the loop overhead stays small.  The time is the matrix cores'
// sustained issue rate at the clock the device holds under that load; the local-energy
// contraction is compared with it as well as with the datasheet peak.
#pragma once

constexpr int PEAK_MAX_BLOCKS = 1024;  // workgroups of 256 threads (4 waves per SIMD on 256 CUs)

// KIND: 0 = v_mfma_f32_32x32x2_f32, 1 = v_mfma_f64_16x16x4_f64, 2 = v_mfma_f32_32x32x16_bf16
template <int KIND> struct PeakOps;
template <> struct PeakOps<0> {
  typedef float op;
  typedef f32x16 acc;
  static constexpr int NB = 8;
  static __device__ acc mfma(op a, op b, acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  static __device__ op make(int x) { return 1.0f + 1e-7f * (float)x; }
};
template <> struct PeakOps<1> {
  typedef double op;
  typedef double acc __attribute__((ext_vector_type(4)));
  static constexpr int NB = 8;
  static __device__ acc mfma(op a, op b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ op make(int x) { return 1.0 + 1e-9 * (double)x; }
};
template <> struct PeakOps<2> {
  typedef bf16x8 op;
  typedef f32x16 acc;
  static constexpr int NB = 2;
  static __device__ acc mfma(op a, op b, acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ op make(int x) {
    op v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)(1.0f + 0.0078125f * (float)((x + e) & 127));
    return v;
  }
};

// MFMA instructions per wavefront and loop iteration, and FLOP of one instruction.
template <int KIND> constexpr int peak_mfmas_per_iter() { return PeakOps<KIND>::NB * 8; }
constexpr double peak_flops_per_mfma(int kind) {
  return kind == 0 ? 2.0 * 32 * 32 * 2 : kind == 1 ? 2.0 * 16 * 16 * 4 : 2.0 * 32 * 32 * 16;
}

template <int KIND>
__global__ void __launch_bounds__(256) k_mfma_peak(int iters, double* __restrict__ out) {
  using O = PeakOps<KIND>;
  constexpr int NB = O::NB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  typename O::op A[2][2], B[NB][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int e = 0; e < 2; ++e) A[a][e] = O::make(lane + 64 * a + 128 * e);
#pragma unroll
  for (int c = 0; c < NB; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 2; ++e) B[c][b][e] = O::make(wave + 4 * c + 32 * b + 64 * e + 128);
  typename O::acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename O::acc{};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = O::mfma(A[a][e], B[c][b][e], acc[a][b]);
  }
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) s += (double)acc[a][b][0] + (double)acc[a][b][3];
  // one value per workgroup keeps every chain live
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}
