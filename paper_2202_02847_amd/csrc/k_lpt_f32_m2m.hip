// Fixed-order lane-per-translation kernels: float, M2M, orders 2..16.
#include "lpt_impl.hpp"

namespace shfmm {
namespace lpt {
template hipError_t launch_fixed<float, float, OP_M2M>(int, const DevTables &, const TransArgs &, hipStream_t);
}  // namespace lpt
}  // namespace shfmm
