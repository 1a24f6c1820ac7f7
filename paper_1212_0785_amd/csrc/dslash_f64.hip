// Wilson hopping term with SpF64 spinors and LkF64 links (all link forms,
// shapes and epilogues).
#include "dslash_kernels.h"

namespace hmc {

hipError_t launch_dslash_f64(int dagger, int epi, const LatArg& g, int out_par, const DslashArgs* table, int nbatch,
                        const DslashArgs& one, hipStream_t st, int j) {
  return launch_links<SpF64, LkF64>(HMC_F64, dagger, epi, g, out_par, table, nbatch, one, st, j);
}

}  // namespace hmc
