// Wilson hopping term with SpF32 spinors and LkF32 links (all link forms,
// shapes and epilogues).
#include "dslash_kernels.h"

namespace hmc {

hipError_t launch_dslash_f32(int dagger, int epi, const LatArg& g, int out_par, const DslashArgs* table, int nbatch,
                        const DslashArgs& one, hipStream_t st, int j) {
  return launch_links<SpF32, LkF32>(HMC_F32, dagger, epi, g, out_par, table, nbatch, one, st, j);
}

}  // namespace hmc
