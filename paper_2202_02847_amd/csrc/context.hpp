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

}  // namespace shfmm
