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
    unsigned flags;      // bit 0: accumulate; bit 1: single-height M2L (p_in = p_out)
    int *err;            // device error flag
};
constexpr unsigned kSingleHeightFlag = 2u;

// One item of a mixed work list (same layout as the public sh_item): operation, orders,
// input / output offsets (in reals) into the caller's arena, shift.
struct ListItem {
    int32_t op, p_in, p_out, reserved;
    int64_t in_off, out_off;
    double r[3];
};
static_assert(sizeof(ListItem) == 56, "ListItem layout");

// A task of the lane-per-translation list kernel: up to 64 consecutive items (of one op)
// sharing (p_in, p_out).
struct ListTask {
    int32_t p_in, p_out;
    int32_t count;
    int32_t reserved;
    int64_t first;
};

struct ListArgs {
    const ListItem *items;
    int64_t count;        // items (wavefront-per-item kernel)
    const ListTask *tasks;
    int64_t ntasks;       // tasks (lane-per-translation kernel)
    const void *arena_in;
    void *arena_out;
    unsigned flags;
    int *err;
};

// General rotation kernel: any orders up to the table order, one wavefront per translation.
hipError_t launch_general(const DevTables &tab, const TransArgs &a, bool f32, hipStream_t s);

// Work-list forms.  General: one wavefront per item, any op / orders (pmax = largest order
// in the list, sizes the LDS).  Lane-per-translation: tasks of one op whose orders are at
// most `bucket`; bucket must be one of list_buckets().
hipError_t launch_list_general(const DevTables &tab, const ListArgs &la, bool f32, bool wide, int pmax,
                               hipStream_t s);
hipError_t launch_list_lpt(const DevTables &tab, const ListArgs &la, int op, bool f32, int bucket,
                           hipStream_t s);
// Order buckets of the lane-per-translation list kernel (ascending).
const int *list_buckets(int *n);

// Shared-shift grouped GEMM (k_shared.hip): translations grouped by class, class c owning
// rows [class_start[c], class_start[c+1]) of the FP32 input / output arrays.
struct SharedArgs {
    int64_t count;
    int nclass;
    int K, Kp, N, NT, KS;           // input reals, K padded to 32, output reals, output tiles, K steps
    const int64_t *class_start;     // device, nclass + 1
    const float *in;
    int64_t ld_in;
    float *out;
    int64_t ld_out;
    const void *frag;               // operator fragments (BF16 pieces, or FP32 values)
    int64_t frag_class_stride;      // elements per (class, piece)
    const unsigned char *live_in;   // Kp flags: input real used (not Im C_n^0, not padding)
    const unsigned char *live_out;  // N flags: output real not Im C_n^0
    unsigned flags;                 // bit 0: accumulate
};
hipError_t launch_shared_prep(const double *traw, int64_t nclass, int K, int N, int KS, int NT, int npieces,
                              const double *s_in, const double *s_out, unsigned short *frag, hipStream_t s);
hipError_t launch_shared_prep_f32(const double *traw, int64_t nclass, int K, int N, int KS, int NT,
                                  const double *s_in, const double *s_out, float *frag, hipStream_t s);
// prec: 6 / 3 (BF16 split, frag = BF16 pieces) or 1 (FP32, frag = floats)
hipError_t launch_shared_gemm(const SharedArgs &a, int prec, hipStream_t s);
int shared_max_classes();

namespace lpt {
// Workgroups resident at once on the current device for kernel fn (CU count x occupancy).
int resident_workgroups(const void *fn);
}

// Block kernel on the FP64 matrix cores (k_big.hip): 16 translations per workgroup pass, any
// p_in, p_out up to 31 (FP32 I/O in the normalised basis, FP64 arithmetic).
bool big_available(int p_in, int p_out);
size_t big_lds_bytes(int PM);
hipError_t launch_big(const DevTables &tab, const TransArgs &a, bool f32, hipStream_t s);
// Work-list form: tasks of up to 16 items of operation op sharing (p_in, p_out); pmax = the
// largest order of the launch's tasks (sizes the LDS), below 32.
// nw: 4 for workgroups of 4 wavefronts, two per CU (used only where two blocks' LDS fit,
// big_list_two_per_cu), else one workgroup of 8 per CU
hipError_t launch_list_big(const DevTables &tab, const ListArgs &la, int op, bool f32, int pmax, int nw, hipStream_t s);
bool big_list_two_per_cu(int pmax);

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
// L2P: potential and gradient of the local expansions of `count` boxes at their `npts`
// targets each; out holds 4 doubles per target (flags bit 0: accumulate).
hipError_t launch_l2p(int P, int64_t count, const double *centres, int64_t npts, const double *pts,
                      const double *L, int64_t ldL, double *out, unsigned flags, hipStream_t s);

}  // namespace shfmm
