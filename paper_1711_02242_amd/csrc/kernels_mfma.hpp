// MFMA form of the local-energy contraction (placeholder: FP32 / BF16x3 not built yet).
#pragma once

#include "common.hpp"

struct MfmaTables {
  bool enabled = false;
  int precision = 0;
  size_t bytes = 0;
};

inline size_t mfma_theta_bytes(const MfmaTables&, size_t) { return 0; }
inline int mfma_build_tables(MfmaTables&, int, int, int, int, int, const double*) {
  return AFQMC_E_UNSUPPORTED;
}
inline void mfma_free_tables(MfmaTables&) {}
inline hipError_t mfma_pack_theta(const MfmaTables&, hipStream_t, int, int, int, int, const cd*,
                                  const double*, void*) {
  return hipErrorInvalidValue;
}
inline hipError_t mfma_contract(const MfmaTables&, hipStream_t, int, int, const void*, const double*,
                                cd*, cd*) {
  return hipErrorInvalidValue;
}
