// Lane-per-translation kernels (placeholder until the specialised path lands).
#include "kernels.hpp"

namespace shfmm {

bool lpt_available(int, bool, int, int) { return false; }

hipError_t launch_lpt(const DevTables &, const TransArgs &, bool, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace shfmm
