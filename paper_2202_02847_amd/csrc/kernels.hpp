// Host-side launchers of the translation kernels (implemented in the .hip files).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.hpp"

namespace shfmm {

// Arguments of one batched translation call (device pointers).
struct TransArgs {
    int op;      // OP_M2M / OP_M2L / OP_L2L
    int p_in, p_out;
    int64_t count;
    const void *r;   // count x 3 reals
    const void *in;  // input solids (pool when src != nullptr)
    int64_t ld_in;
    void *out;       // output solids (pool when dst != nullptr)
    int64_t ld_out;
    const int64_t *src;  // optional gather indices
    const int64_t *dst;  // optional scatter indices
    unsigned flags;      // bit 0: accumulate
    int *err;            // device error flag
};

// General rotation kernel: any orders up to the table order, one wavefront per translation.
hipError_t launch_general(const DevTables &tab, const TransArgs &a, bool f32, hipStream_t s);

// Highest order with a fixed-order (lane-per-translation) kernel.
constexpr int kLptMaxOrder = 16;

// Lane-per-translation rotation kernel for common equal orders; returns false when no
// specialisation exists for (op, dtype, p_in, p_out) (the caller falls back).
bool lpt_available(int op, bool f32, int p_in, int p_out);
hipError_t launch_lpt(const DevTables &tab, const TransArgs &a, bool f32, hipStream_t s);

// Direct O(P^4) double-height M2L (FP64).
hipError_t launch_m2l_naive(const TransArgs &a, hipStream_t s);

// Device P2M (FP64).
hipError_t launch_p2m(int P, int64_t count, const double *centres, int64_t npts,
                      const double *pts, const double *q, double *M, int64_t ldM, hipStream_t s);

}  // namespace shfmm
