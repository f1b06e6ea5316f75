// Library-internal definition of the context handle and a scoped device switch, shared by
// the translation entry points (api.cpp) and the work-list planner (plan.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/shfmm.h"
#include "device_common.hpp"

struct sh_ctx {
    int device = -1;
    int max_order = 0;
    void *dev_mem = nullptr;  // one allocation holding every table
    int *err_flag = nullptr;  // device int
    shfmm::DevTables tabs{};
};

namespace shfmm {

// Makes `dev` current for the lifetime of the guard and restores the previous device.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = (hipSetDevice(dev) == hipSuccess);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard &) = delete;
    DeviceGuard &operator=(const DeviceGuard &) = delete;
};

// Batched translation on device pointers (the dispatch behind sh_translate_batch /
// sh_translate_indexed, for use inside the library).
sh_status translate_device(const sh_ctx *ctx, int op, int dtype, int p_in, int p_out, int64_t count,
                           const void *r, const int64_t *src, const void *in, int64_t ld_in,
                           const int64_t *dst, void *out, int64_t ld_out, unsigned flags, void *stream);

// Normalisation weight w_n^m = sqrt((n+m)! (n-m)!) in extended precision.
long double norm_weight(int n, int m);

}  // namespace shfmm
