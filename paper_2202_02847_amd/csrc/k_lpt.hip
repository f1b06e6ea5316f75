// Lane-per-translation kernels: dispatch.  The kernel template is in lpt_impl.hpp; its
// instantiations are spread over the k_lpt_<dtype>_<op>.hip units.
#include <map>
#include <mutex>
#include <utility>

#include "list_impl.hpp"

namespace shfmm {

namespace lpt {

// Persistent grid: as many workgroups as are resident at once on the device (CU count x
// occupancy of this kernel), each looping over blocks of 64 translations.  Cached per
// kernel and device.
int resident_workgroups(const void *fn)
{
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({fn, dev});
    if (it != cache.end()) return it->second;
    int cu = 0, occ = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 256, 0) != hipSuccess || occ <= 0) occ = 1;
    const int n = cu * occ;
    cache[{fn, dev}] = n;
    return n;
}

}  // namespace lpt

bool lpt_available(int op, bool f32, int p_in, int p_out)
{
    (void)op;
    (void)f32;
    return p_in == p_out && p_in >= 2 && p_in <= kLptMaxOrder;
}

hipError_t launch_lpt(const DevTables &tab, const TransArgs &a, bool f32, hipStream_t s)
{
    using namespace lpt;
    if (a.count <= 0) return hipSuccess;
    const int P = a.p_in;
    if (f32) {
        if (a.op == OP_M2M) return launch_fixed<float, float, OP_M2M>(P, tab, a, s);
        if (a.op == OP_M2L) return launch_fixed<float, float, OP_M2L>(P, tab, a, s);
        return launch_fixed<float, float, OP_L2L>(P, tab, a, s);
    }
    if (a.op == OP_M2M) return launch_fixed<double, double, OP_M2M>(P, tab, a, s);
    if (a.op == OP_M2L) return launch_fixed<double, double, OP_M2L>(P, tab, a, s);
    return launch_fixed<double, double, OP_L2L>(P, tab, a, s);
}

}  // namespace shfmm

namespace shfmm {

const int *list_buckets(int *n)
{
    if (n) *n = (int)(sizeof(lpt::kListBuckets) / sizeof(lpt::kListBuckets[0]));
    return lpt::kListBuckets;
}

hipError_t launch_list_lpt(const DevTables &tab, const ListArgs &la, int op, bool f32, int bucket, hipStream_t s)
{
    using namespace lpt;
    if (la.ntasks <= 0) return hipSuccess;
    if (f32) {
        if (op == OP_M2M) return launch_list_fixed<float, float, OP_M2M>(bucket, tab, la, s);
        if (op == OP_M2L) return launch_list_fixed<float, float, OP_M2L>(bucket, tab, la, s);
        return launch_list_fixed<float, float, OP_L2L>(bucket, tab, la, s);
    }
    if (op == OP_M2M) return launch_list_fixed<double, double, OP_M2M>(bucket, tab, la, s);
    if (op == OP_M2L) return launch_list_fixed<double, double, OP_M2L>(bucket, tab, la, s);
    return launch_list_fixed<double, double, OP_L2L>(bucket, tab, la, s);
}

}  // namespace shfmm
