// y-pass kernels of the demag refresh for one layer count, MMC_NZ (set by the
// build: this unit is compiled once per nz in 1..8).
#include "demag_fft.h"

#ifndef MMC_NZ
#error "compile with -DMMC_NZ=<layers>"
#endif

namespace mmc {
template hipError_t launch_ypass_nz<MMC_NZ>(const Chains&, const DemagPlan&, const float2*, hipStream_t);
}
