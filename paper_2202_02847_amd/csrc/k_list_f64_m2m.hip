// Work-list lane-per-translation kernels: double, M2M, order buckets 4..16.
#include "list_impl.hpp"

namespace shfmm {
namespace lpt {
template hipError_t launch_list_fixed<double, double, OP_M2M>(int, const DevTables &, const ListArgs &, hipStream_t);
}  // namespace lpt
}  // namespace shfmm
