// Dispatch of the Wilson hopping term by storage precision; the kernels
// live in dslash_kernels.h, instantiated by dslash_f64.hip, dslash_f32.hip,
// dslash_f16.hip and dslash_bf16.hip (compiled in parallel).
#include "internal.h"

namespace hmc {

#define HMC_DSLASH_DECL(P)                                                                                    \
  hipError_t launch_dslash_##P(int dagger, int epi, const LatArg& g, int out_par, const DslashArgs* table, \
                               int nbatch, const DslashArgs& one, hipStream_t st, int j);
HMC_DSLASH_DECL(f64)
HMC_DSLASH_DECL(f32)
HMC_DSLASH_DECL(f16)
HMC_DSLASH_DECL(bf16)
#undef HMC_DSLASH_DECL

hipError_t launch_dslash(hmc_prec prec, int dagger, int epi, const LatArg& g, int out_par, const DslashArgs* table,
                         int nbatch, const DslashArgs& one, hipStream_t st, int j) {
  switch (prec) {
    case HMC_F64: return launch_dslash_f64(dagger, epi, g, out_par, table, nbatch, one, st, j);
    case HMC_F32: return launch_dslash_f32(dagger, epi, g, out_par, table, nbatch, one, st, j);
    case HMC_F16: return launch_dslash_f16(dagger, epi, g, out_par, table, nbatch, one, st, j);
    case HMC_BF16: return launch_dslash_bf16(dagger, epi, g, out_par, table, nbatch, one, st, j);
  }
  return hipErrorInvalidValue;
}

}  // namespace hmc
