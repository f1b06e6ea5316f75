// Binning of mixed work lists (host side), shared by the plans (plan.cpp) and the serving
// runtime (server.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <vector>

#include "context.hpp"
#include "kernels.hpp"

namespace shfmm {

// Kernel mapping of a bin: lane-per-translation with 64- or 32-item tasks, one wavefront per
// translation, or the matrix-core block kernel with 16-item tasks (orders 17..31) in
// workgroups of 4 wavefronts, two per CU (MAP_BLOCK, where two blocks' LDS fit) or one
// workgroup of 8 per CU (MAP_BLOCK8).
enum ListMapping { MAP_LPT64 = 0, MAP_LPT32 = 1, MAP_GENERAL = 2, MAP_BLOCK = 3, MAP_BLOCK8 = 4 };
inline bool is_block(int m) { return m == MAP_BLOCK || m == MAP_BLOCK8; }
inline int task_size(int m) { return m == MAP_LPT32 ? 32 : is_block(m) ? 16 : 64; }

struct ListBin {
    int mapping = MAP_LPT64;
    int op = -1;        // lane-per-translation bins: the operation (general bins mix them)
    int bucket = 0;     // order bucket (lane-per-translation) or order class (general)
    bool wide = false;  // FP32 I/O with FP64 arithmetic (orders >= 20)
    int pmax = 0;       // largest order in the bin
    bool tuned = false;
    int64_t item_first = 0, item_count = 0;
    int64_t task_first = 0, task_count = 0;
};

// Chooses the mapping of a group (may time candidates; the bin arrives with its default
// mapping: MAP_LPT64 for orders up to 16, a block mapping for 17..31); returns a
// ListMapping, or < 0 on a device error.
using MappingChoice = std::function<int(ListBin &bin, const std::vector<ListItem> &group)>;

// Groups validated items by operation and order (lane-per-translation bins per (op, bucket),
// block-kernel bins per (op, order class) for orders 17..31, wavefront bins per (order class,
// width) above), reorders `items` bin by bin (largest orders
// first inside a bin), cuts the lane-per-translation bins into tasks (appended to `tasks`)
// and orders the bins largest first.  Returns SH_OK or SH_EDEVICE (from `choose`).
sh_status bin_items(int dtype, std::vector<ListItem> &items, std::vector<ListTask> &tasks,
                    std::vector<ListBin> &bins, const MappingChoice &choose);

// The mapping the tuning cache holds for a bin of `count` items, else `dflt`.
int cached_mapping(int dtype, int op, int bucket, int64_t count, bool *tuned, int dflt = MAP_LPT64);

// Launches one bin (device item / task arrays as laid out by bin_items).
hipError_t launch_list_bin(const sh_ctx *ctx, bool f32, const ListBin &b, const ListItem *d_items,
                           const ListTask *d_tasks, const void *in, void *out, unsigned flags, hipStream_t s);

}  // namespace shfmm
