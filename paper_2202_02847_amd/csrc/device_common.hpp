// Device-side definitions shared by the translation kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.hpp"

namespace shfmm {

// Constant tables resident in device memory (built and uploaded once per context).
// Swap matrices: dense (n+1)x(n+1) row-major per degree n at offset n(n+1)(2n+1)/6,
// kinds F, G (M side), FL, GL (L side).  z coefficients: column m block at
// sum_{j<m} (P-j)^2, entry [out-m][in-m] with row length P-m, P = table order.
// Three table sets: paper basis in FP64 (FP64 path), normalised basis in FP32 (FP32 path)
// and normalised basis in FP64 (FP32 path with FP64 arithmetic at high order).
struct DevTables {
    const double *swap64[4];
    const float *swap32[4];
    const double *swap64n[4];
    const double *z64[3];
    const float *z32[3];
    const double *z64n[3];
    const double *pk64[2];   // packed swap tables, [0] M side (F, G), [1] L side (FL, GL)
    const float *pk32[2];
    const double *pk64n[2];
    const double *bsw[2][2];  // block-kernel swap fragments [basis: 0 paper, 1 normalised][side: 0 M, 1 L]
    const double *bz[2][3];   // block-kernel z fragments [basis][op]
    int P;
};

// Table set for I/O type Real and arithmetic type Acc: Real = double uses the paper basis,
// Real = float uses the normalised basis in the arithmetic type.
template <typename Real, typename Acc>
struct Tab;
template <>
struct Tab<double, double> {
    __device__ static const double *swap(const DevTables &t, int k) { return t.swap64[k]; }
    __device__ static const double *z(const DevTables &t, int k) { return t.z64[k]; }
    __device__ static const double *packed(const DevTables &t, int side) { return t.pk64[side]; }
};
template <>
struct Tab<float, float> {
    __device__ static const float *swap(const DevTables &t, int k) { return t.swap32[k]; }
    __device__ static const float *z(const DevTables &t, int k) { return t.z32[k]; }
    __device__ static const float *packed(const DevTables &t, int side) { return t.pk32[side]; }
};
template <>
struct Tab<float, double> {
    __device__ static const double *swap(const DevTables &t, int k) { return t.swap64n[k]; }
    __device__ static const double *z(const DevTables &t, int k) { return t.z64n[k]; }
    __device__ static const double *packed(const DevTables &t, int side) { return t.pk64n[side]; }
};

// The FP32 path switches its arithmetic to FP64 from this order on (gfx950 runs
// non-packed FP32 and FP64 FMA at the same rate; HBM traffic stays FP32).
constexpr int kF32WideOrder = 20;

enum { OP_M2M = 0, OP_M2L = 1, OP_L2L = 2 };

// Order the device tables are laid out for (every context builds them up to this order),
// so that kernels with compile-time orders address table entries at fixed offsets.
constexpr int kZTableOrder = 64;
enum { SW_F = 0, SW_G = 1, SW_FL = 2, SW_GL = 3 };


// Geometry of a shift (Section 3.4, step 1): |r|, rho = sqrt(x^2+y^2) and the two
// z-rotation angles, without trigonometric functions:
//   cos a = y/rho, sin a = x/rho  (cos a = 1, sin a = 0 when x = y = 0)
//   cos b = z/|r|, sin b = -rho/|r|
// Rotating by a, swapping x<->z, rotating by b and swapping again sends r to (0,0,|r|).
struct Geometry {
    double R, s;  // |r| and 1/|r|
    double ca, sa, cb, sb;
    int valid;    // 0: r = 0; -1: not finite; 1: ok
};

__device__ __forceinline__ Geometry shift_geometry(double x, double y, double z)
{
    Geometry g;
    const double rho2 = x * x + y * y;
    const double r2 = rho2 + z * z;
    const bool finite = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(r2);
    g.valid = !finite ? -1 : (r2 > 0.0 ? 1 : 0);
    const double R = sqrt(r2);
    const double rho = sqrt(rho2);
    g.R = R;
    g.s = (g.valid == 1) ? 1.0 / R : 0.0;
    if (rho > 0.0) {
        const double ir = 1.0 / rho;
        g.ca = y * ir;
        g.sa = x * ir;
    } else {
        g.ca = 1.0;
        g.sa = 0.0;
    }
    g.cb = (g.valid == 1) ? z * g.s : 1.0;
    g.sb = (g.valid == 1) ? -rho * g.s : 0.0;
    return g;
}

// Vector (not scalar-cache) atomic raise of the context's device error flag.
__device__ __forceinline__ void raise_device_error(int *flag, int code)
{
    if (flag) atomicCAS(flag, 0, code);
}

}  // namespace shfmm
