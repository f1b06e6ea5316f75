// Memory layouts shared by the host table builder and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace shfmm {

// dense (n+1)x(n+1) swap block of degree n starts at n(n+1)(2n+1)/6
__host__ __device__ constexpr int swap_off(int n) { return n * (n + 1) * (2 * n + 1) / 6; }
// Re C_n^m of a solid
__host__ __device__ constexpr int solid_pos(int n, int m) { return n * (n + 1) + 2 * m; }
// start of column block m of a z-coefficient table of order P: sum_{j<m} (P-j)^2
__host__ __device__ constexpr int64_t z_col_off(int P, int m)
{
    return ((int64_t)P * (P + 1) * (2 * P + 1) - (int64_t)(P - m) * (P - m + 1) * (2 * (P - m) + 1)) / 6;
}

// Packed swap tables (the paper's packing, Section 3.2, Fig. 3, for scalar loads): for each
// degree n and output order m = 0..n, first the non-zero entries of the real-part matrix
// (F or FL: l = 0..n with m + l + n even), then those of the imaginary-part matrix (G or
// GL: m >= 1, l = 1..n with m + l + n odd), l ascending.  The kernels read them in exactly
// this order, so consecutive entries are contiguous in memory.
__host__ __device__ constexpr int packed_re_count(int n, int m)
{
    int c = 0;
    for (int l = 0; l <= n; ++l) c += ((m + l + n) % 2 == 0);
    return c;
}
__host__ __device__ constexpr int packed_im_count(int n, int m)
{
    int c = 0;
    if (m == 0) return 0;
    for (int l = 1; l <= n; ++l) c += ((m + l + n) % 2 == 1);
    return c;
}
__host__ __device__ constexpr int packed_row_count(int n)
{
    int c = 0;
    for (int m = 0; m <= n; ++m) c += packed_re_count(n, m) + packed_im_count(n, m);
    return c;
}
__host__ __device__ constexpr int packed_off(int n)
{
    int c = 0;
    for (int j = 0; j < n; ++j) c += packed_row_count(j);
    return c;
}

// MFMA fragment tables of the block kernel for orders up to kBigOrder (FP64 16x16x4 A operands,
// 64 doubles per fragment, lane l holding row l % 16 and K index l / 16 of the 16 x 4 block).
// Every degree and every column has a slot of the same size, zero-padded past the K steps and
// tiles it uses, so a wavefront can fetch any slot with unconditional loads.
//  * swap: degree n's slot holds, for output-order parity pm, part q (0: real-part matrix,
//    1: imaginary) and K step ks < 4, fragment (pm * 2 + q) * 4 + ks with entry
//    (m = 2 (l % 16) + pm, l' = 2 (4 ks + l / 16) + ((n + pm + q) & 1)) of the (n+1) x (n+1)
//    swap matrix (zero outside the degree and, for q = 1, in row or column 0): the
//    chequerboard splits every swap into two dense blocks by parity.  Only the first
//    big_ks(n) K steps can be nonzero.
//  * z: column m's slot holds, for output tile mt < 2 and K step ks < 8, fragment mt * 8 + ks
//    with entry (out = m + 16 mt + l % 16, in = m + 4 ks + l / 16) of the column's z matrix.
constexpr int kBigOrder = 32;
constexpr int kBigSlot = 16 * 64;  // doubles per degree or column slot
__host__ __device__ constexpr int big_ks(int n) { return (n / 2 + 4) / 4; }
__host__ __device__ constexpr int big_swap_off(int n) { return n * kBigSlot; }
__host__ __device__ constexpr int big_z_off(int m) { return m * kBigSlot; }

}  // namespace shfmm
