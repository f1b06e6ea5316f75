// Lane-per-translation rotation kernels for fixed orders (compile-time P_in, P_out).
//
// Mapping (the paper's nu-solid blocking, Section 3.2-3.4, with nu = 64 = one wavefront):
//   * a workgroup of 4 wavefronts owns a block of 64 translations; lane t of every
//     wavefront works on translation t of the block;
//   * the 64 solids are loaded from HBM with coalesced 16-byte (FP64) / 8-byte (FP32)
//     accesses into LDS (one padded row of P(P+1) reals per translation);
//   * rows (degrees) of the forward rotation, columns (orders) of the z-axis step and rows
//     of the backward rotation are shared out between the 4 wavefronts by a static
//     greedy schedule; each row or column is held in registers while it is transformed;
//   * because every lane applies the same swap matrix or z coefficient at the same time,
//     table entries are wave-uniform: they come through scalar loads at compile-time
//     offsets, and the chequerboard zeros of F_n, G_n are skipped at compile time;
//   * the block is written back from LDS with coalesced stores.
// Only the shift geometry differs between lanes (the powers e^{im a}, e^{im b}, |r|^n).
#pragma once
#include <type_traits>

#include "kernels.hpp"

namespace shfmm {
namespace lpt {


template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Greedy static schedule: items (rows or columns) sorted by cost, each given to the
// least-loaded of the NW wavefronts.  cost(i) ~ (i+1)^2 for rows, (P-m)^2 for columns.
constexpr int row_owner(int P, int n, int NW = 4)
{
    long load[16] = {};
    int own = 0;
    for (int k = P - 1; k >= 0; --k) {
        int w = 0;
        for (int j = 1; j < NW; ++j)
            if (load[j] < load[w]) w = j;
        load[w] += (long)(k + 1) * (k + 1);
        if (k == n) own = w;
    }
    return own;
}

constexpr int col_owner(int PIN, int POUT, int m, int NW = 4)
{
    long load[16] = {};
    int own = 0;
    const int PM = PIN > POUT ? PIN : POUT;
    for (int k = 0; k < PM; ++k) {
        int w = 0;
        for (int j = 1; j < NW; ++j)
            if (load[j] < load[w]) w = j;
        const long ci = PIN - k > 0 ? PIN - k : 1;
        load[w] += ci * (POUT - k > 0 ? POUT - k : 1);
        if (k == m) own = w;
    }
    return own;
}

// Tables are read through the constant address space: their addresses are wave-uniform,
// so the loads become scalar loads into SGPRs (the kernel never writes the tables).
template <typename Acc>
using cptr = const __attribute__((address_space(4))) Acc *;

template <typename Acc>
__device__ __forceinline__ cptr<Acc> as_const(const Acc *p)
{
    return (cptr<Acc>)(p);
}

// Returns p unchanged, but opaque to the optimizer: the table loads inside the per-block
// loop then depend on a loop-variant value and are not hoisted out of it (hoisting every
// table entry of every row out of the loop overflows the SGPR file).  Emits no instruction.
template <typename Acc>
__device__ __forceinline__ cptr<Acc> launder(cptr<Acc> p)
{
    uint64_t v = (uint64_t)(p);
    asm volatile("" : "+s"(v));
    return (cptr<Acc>)(v);
}

// Workgroup barrier that orders LDS accesses only.  The kernels communicate between
// wavefronts through LDS alone, so global loads issued for the next block stay in flight
// across it (a full __syncthreads would wait for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename Acc>
struct Pair;
template <>
struct Pair<double> {
    using T = double2;
};
template <>
struct Pair<float> {
    using T = float2;
};

// Powers e^{im a}, e^{im b} of one translation (lane).  With HOLD they are tabulated once
// (m = 0..PM-1, held in registers); otherwise only e^{ia}, e^{ib} are kept and every row
// regenerates its powers by complex multiplication (trading VALU work for registers at
// the higher orders).
template <typename Acc, int PM, bool HOLD>
struct Powers;
template <typename Acc, int PM>
struct Powers<Acc, PM, true> {
    Acc ca[PM], sa[PM], cb[PM], sb[PM];
    __device__ __forceinline__ void init(const Geometry &g)
    {
        double c1 = 1.0, s1 = 0.0, c2 = 1.0, s2 = 0.0;
#pragma unroll
        for (int m = 0; m < PM; ++m) {
            ca[m] = (Acc)c1;
            sa[m] = (Acc)s1;
            cb[m] = (Acc)c2;
            sb[m] = (Acc)s2;
            const double t1 = c1 * g.ca - s1 * g.sa;
            s1 = c1 * g.sa + s1 * g.ca;
            c1 = t1;
            const double t2 = c2 * g.cb - s2 * g.sb;
            s2 = c2 * g.sb + s2 * g.cb;
            c2 = t2;
        }
    }
    // x <- x * e^{+-i m angle}  (which: 0 = a, 1 = b)
    template <int N>
    __device__ __forceinline__ void rot(Acc (&xr)[N + 1], Acc (&xi)[N + 1], int which, Acc sgn) const
    {
#pragma unroll
        for (int m = 1; m <= N; ++m) {
            const Acc cs = which ? cb[m] : ca[m];
            const Acc sn = sgn * (which ? sb[m] : sa[m]);
            const Acc a = xr[m], b = xi[m];
            xr[m] = a * cs - b * sn;
            xi[m] = a * sn + b * cs;
        }
    }
};
template <typename Acc, int PM>
struct Powers<Acc, PM, false> {
    Acc ca1, sa1, cb1, sb1;
    __device__ __forceinline__ void init(const Geometry &g)
    {
        ca1 = (Acc)g.ca;
        sa1 = (Acc)g.sa;
        cb1 = (Acc)g.cb;
        sb1 = (Acc)g.sb;
    }
    template <int N>
    __device__ __forceinline__ void rot(Acc (&xr)[N + 1], Acc (&xi)[N + 1], int which, Acc sgn) const
    {
        const Acc c1 = which ? cb1 : ca1, s1 = sgn * (which ? sb1 : sa1);
        Acc cs = 1, sn = 0;
#pragma unroll
        for (int m = 1; m <= N; ++m) {
            const Acc t = cs * c1 - sn * s1;
            sn = cs * s1 + sn * c1;
            cs = t;
            const Acc a = xr[m], b = xi[m];
            xr[m] = a * cs - b * sn;
            xi[m] = a * sn + b * cs;
        }
    }
};

// Number of packed entries for output order m of degree n, and where they start.
template <int N>
constexpr int packed_m_count(int m)
{
    return packed_re_count(N, m) + packed_im_count(N, m);
}
template <int N>
constexpr int packed_m_off(int m)
{
    int c = packed_off(N);
    for (int j = 0; j < m; ++j) c += packed_m_count<N>(j);
    return c;
}

// y = swap(x) for degree n, reading the packed non-zeros (layout.hpp) in storage order:
// for each output order m, the real-part entries (l with m + l + n even), then the
// imaginary-part entries (m, l >= 1, m + l + n odd).  Offsets are compile-time, so the
// entries of one output are a contiguous run fetched by wide scalar loads.  The loads of
// output m+1 are issued before the arithmetic of output m, and a scheduling barrier per
// output stops the scheduler from hoisting more: at most two outputs' entries are live in
// SGPRs (hoisting whole rows overflows the SGPR file and spills to VGPR lanes).
template <typename Acc, int N, int M>
__device__ __forceinline__ void swap_fetch(cptr<Acc> T, Acc (&t)[N + 1])
{
    if constexpr (M <= N) {
        constexpr int c = packed_m_count<N>(M), o = packed_m_off<N>(M);
#pragma unroll
        for (int j = 0; j < c; ++j) t[j] = T[o + j];
    }
}

template <typename Acc, int N, int M>
__device__ __forceinline__ void swap_out(const Acc (&t)[N + 1], const Acc (&xr)[N + 1], const Acc (&xi)[N + 1],
                                         Acc (&yr)[N + 1], Acc (&yi)[N + 1])
{
    int at = 0;
    Acc ar = 0, ai = 0;
#pragma unroll
    for (int l = 0; l <= N; ++l)
        if ((M + l + N) % 2 == 0) ar += t[at++] * xr[l];
    if (M > 0) {
#pragma unroll
        for (int l = 1; l <= N; ++l)
            if ((M + l + N) % 2 == 1) ai += t[at++] * xi[l];
    }
    yr[M] = ar;
    yi[M] = ai;
}

template <typename Acc, int N, int M>
__device__ __forceinline__ void swap_pipe(cptr<Acc> T, Acc (&cur)[N + 1], const Acc (&xr)[N + 1],
                                          const Acc (&xi)[N + 1], Acc (&yr)[N + 1], Acc (&yi)[N + 1])
{
    if constexpr (M <= N) {
        Acc nxt[N + 1];
        swap_fetch<Acc, N, M + 1>(T, nxt);
        swap_out<Acc, N, M>(cur, xr, xi, yr, yi);
        __builtin_amdgcn_sched_barrier(0);
        swap_pipe<Acc, N, M + 1>(T, nxt, xr, xi, yr, yi);
    }
}

template <typename Acc, int N>
__device__ __forceinline__ void swap_row(cptr<Acc> T, const Acc (&xr)[N + 1], const Acc (&xi)[N + 1],
                                         Acc (&yr)[N + 1], Acc (&yi)[N + 1])
{
    Acc cur[N + 1];
    swap_fetch<Acc, N, 0>(T, cur);
    swap_pipe<Acc, N, 0>(T, cur, xr, xi, yr, yi);
}

// Coefficients c(o, k), k = m..PIN-1, of output degree o in column m of the unit z-shift.
// In the paper basis (the FP64 tables) a coefficient depends on o + k alone (M2L:
// (-1)^{o+m} (o+k)!, a Hankel matrix) or on o - k (M2M: (-1)^{o-k}/(o-k)!, L2L: 1/(k-o)!,
// Toeplitz), so one short sequence serves every column: row 0 (M2L, L2L) or the last row
// (M2M) of column 0 of the order-64 table holds it, and the few scalar-cache lines it spans
// stay resident instead of one block of lines per column.  The normalised tables (FP32) are
// read per column.  Entries outside the triangle of M2M / L2L are returned as 0 (unused).
// single (M2L only): the single-height kernel (eq. m2lkernels, left) keeps the terms with
// o + k <= PIN - 1; the others are returned as 0.  The fixed-order kernel passes it as a
// compile-time constant (a kernel form of its own), so neither form carries the selection.
template <typename Real, typename Acc, int OP, int PIN, int M>
__device__ __forceinline__ void z_fetch(cptr<Acc> Z0, int o, Acc (&c)[PIN - M], bool single = false)
{
    constexpr bool SEQ = std::is_same<Real, double>::value && std::is_same<Acc, double>::value;
    constexpr int K = kZTableOrder;
    const cptr<Acc> Z = launder(Z0);  // reloaded per output: only two outputs' entries live
#pragma unroll
    for (int k = M; k < PIN; ++k) {
        if ((OP == OP_M2M && k > o) || (OP == OP_L2L && k < o)) {
            c[k - M] = (Acc)0;
        } else if constexpr (SEQ) {
            if constexpr (OP == OP_M2L) {
                const Acc v = Z[o + k];
                c[k - M] = ((o + M) & 1) ? -v : v;
            } else if constexpr (OP == OP_M2M) {
                c[k - M] = Z[(K - 1) * K + (K - 1) - (o - k)];
            } else {
                c[k - M] = Z[k - o];
            }
        } else {
            c[k - M] = Z[z_col_off(K, M) + (int64_t)(o - M) * (K - M) + (k - M)];
        }
        if (OP == OP_M2L && o + k > PIN - 1) c[k - M] = single ? (Acc)0 : c[k - M];
    }
}

// The L-side swap of degree N from the M-side table.  The L-side real-part matrix is
// F_L = D F^T D^{-1} (D = diag(2, 1, ..., 1), the corrected reading of the transposed matrices
// of Section 3.4) and the imaginary-part matrix is G^T, so
//   Re y = D F^T D^{-1} Re x,   Im y = G^T Im x,
// computed as updates y += x_L * (packed row L of F, G) over L = 0..N: every output sums its
// terms in the same (ascending) order as the product with the L-side table would, and the
// factors 2 and 1/2 are exact, so the result is that product's (with the accumulators pinned
// per step, see pin_all: 2^20 M2L outputs at orders 13 and 14 equal the L-side table's bit
// for bit).  One table then serves both sides, halving the scalar-cache footprint of M2L
// (forward F, backward F_L).
template <typename Acc, int N, int L>
__device__ __forceinline__ void swapT_in(const Acc (&t)[N + 1], Acc xl_r, Acc xl_i, Acc (&yr)[N + 1],
                                         Acc (&yi)[N + 1])
{
    int at = 0;
#pragma unroll
    for (int l = 0; l <= N; ++l)
        if ((L + l + N) % 2 == 0) yr[l] += t[at++] * xl_r;
    if (L > 0) {
#pragma unroll
        for (int l = 1; l <= N; ++l)
            if ((L + l + N) % 2 == 1) yi[l] += t[at++] * xl_i;
    }
}

// Makes every accumulator of a row opaque at this point.  Without it the optimiser sinks some
// outputs' sums of the transposed update past the later steps (the sums are pure arithmetic,
// the scalar table loads are not), so the table entries those sums need stay live across the
// whole row and spill to vector-register lanes (at P = 16 about 1,900 lane moves per block),
// and the sunk sums come out in another association.
template <typename Acc, int N>
__device__ __forceinline__ void pin_all(Acc (&y)[N + 1])
{
#pragma unroll
    for (int l = 0; l <= N; ++l) asm volatile("" : "+v"(y[l]));
}

template <typename Acc, int N, int L>
__device__ __forceinline__ void swapT_pipe(cptr<Acc> T, Acc (&cur)[N + 1], const Acc (&xr)[N + 1],
                                           const Acc (&xi)[N + 1], Acc (&yr)[N + 1], Acc (&yi)[N + 1])
{
    if constexpr (L <= N) {
        Acc nxt[N + 1];
        swap_fetch<Acc, N, L + 1>(T, nxt);
        swapT_in<Acc, N, L>(cur, L == 0 ? xr[0] * (Acc)0.5 : xr[L], xi[L], yr, yi);
        pin_all<Acc, N>(yr);
        pin_all<Acc, N>(yi);
        __builtin_amdgcn_sched_barrier(0);
        swapT_pipe<Acc, N, L + 1>(T, nxt, xr, xi, yr, yi);
    }
}

// TR = false: y = (F, G) x from the packed M-side table; TR = true: the L-side swap from the
// same table (see swapT_in).
template <typename Acc, int N, bool TR>
__device__ __forceinline__ void swap_row_x(cptr<Acc> T, const Acc (&xr)[N + 1], const Acc (&xi)[N + 1],
                                           Acc (&yr)[N + 1], Acc (&yi)[N + 1])
{
    if constexpr (!TR) {
        swap_row<Acc, N>(T, xr, xi, yr, yi);
    } else {
#pragma unroll
        for (int m = 0; m <= N; ++m) {
            yr[m] = (Acc)0;
            yi[m] = (Acc)0;
        }
        Acc cur[N + 1];
        swap_fetch<Acc, N, 0>(T, cur);
        swapT_pipe<Acc, N, 0>(T, cur, xr, xi, yr, yi);
        yr[0] *= (Acc)2;
    }
}

// Calls f(std::integral_constant<int, W>) for the wavefront index W = wave, so that each
// wavefront runs straight-line code for its own share of rows / columns.
template <int NW, int W, typename F>
__device__ __forceinline__ void per_wave_from(int wave, F &&f)
{
    if constexpr (W == NW - 1) {
        f(std::integral_constant<int, W>{});
    } else {
        if (wave == W)
            f(std::integral_constant<int, W>{});
        else
            per_wave_from<NW, W + 1>(wave, f);
    }
}
template <int NW = 4, typename F>
__device__ __forceinline__ void per_wave(int wave, F &&f)
{
    per_wave_from<NW, 0>(wave, f);
}

template <typename Acc>
__device__ __forceinline__ Acc ipow(Acc x, int e)
{
    Acc r = 1;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// LDS row stride (reals) of one translation: P(P+1) padded so that (Re, Im) pair accesses
// by consecutive lanes fall in distinct banks (stride = 2 mod 4).
template <int PM>
constexpr int lpt_stride()
{
    return (PM * (PM + 1)) % 4 == 2 ? PM * (PM + 1) : PM * (PM + 1) + 2;
}
// workgroups (of 4 wavefronts) that fit on one CU by LDS: 160 KiB per CU on gfx950
template <typename Acc, int PM>
constexpr int lpt_blocks_per_cu()
{
    const int bytes = 64 * lpt_stride<PM>() * (int)sizeof(Acc) + 256;
    const int b = 163840 / bytes;
    return b < 1 ? 1 : (b > 8 ? 8 : b);
}
// minimum waves per SIMD requested from the register allocator: 2 while two workgroups
// fit in LDS (the allocator then stays within 256 VGPRs), else 1
template <typename Acc, int PM>
constexpr int lpt_min_waves()
{
    return lpt_blocks_per_cu<Acc, PM>() >= 2 ? 2 : 1;
}
// wavefronts per workgroup: where LDS allows only one workgroup per CU, 12 (three per SIMD,
// to hide each other's latency) up to order 14 and 8 (two per SIMD) above, where three per
// SIMD leave too few registers (2^20 FP64 M2L on one MI355X, 12 against 8 wavefronts:
// P = 13 0.851 vs 0.889 ms, P = 14 1.050 vs 1.107 ms, P = 15 1.344 vs 1.232 ms, P = 16 1.606
// vs 1.487 ms); else 4
template <typename Acc, int PM>
constexpr int lpt_waves()
{
    return lpt_blocks_per_cu<Acc, PM>() >= 2 ? 4 : (PM <= 14 ? 12 : 8);
}
template <typename Acc, int PM>
constexpr int lpt_min_waves_nw()
{
    return lpt_waves<Acc, PM>() == 12 ? 3 : (lpt_blocks_per_cu<Acc, PM>() >= 2 || lpt_waves<Acc, PM>() == 8 ? 2 : 1);
}
// Powers held in registers (tabulated once per block) up to this order, regenerated per row
// above.  FP32 from order 9 on regenerates them: with the next block's prefetch also off
// (lpt_prefetch_ok) the kernel fits in 159 VGPRs at order 10, three wavefronts per SIMD instead
// of two (FP32 M2L, 2^20 translations at P = 10: 0.258 -> 0.237 ms on one MI355X).
template <typename Acc, int PM>
constexpr bool lpt_hold_powers()
{
    return sizeof(Acc) == 4 ? PM <= 8 : PM <= 6;
}
// Whether a block's input may be prefetched into registers during the previous block (when it
// fits in 64 VGPRs): not for FP32 from order 9 on, where the registers buy a third wavefront
// per SIMD instead (lpt_hold_powers).  Below order 9 the prefetch wins (P = 6: 0.079 ms with it,
// 0.094 ms without).
template <typename Real, int PM>
constexpr bool lpt_prefetch_ok()
{
    return !(sizeof(Real) == 4 && PM >= 9);
}

// Whether the L-side swaps read the M-side table transposed (swap_row_x) instead of the
// L-side table.  Measured on MI355X (FP64 M2L, 2^20 translations): at order 10 the L-side
// table is faster (0.385 vs 0.468 ms); from order 12 one table in the scalar cache wins
// (P = 12: 0.675 vs 0.690 ms, P = 16: 1.41 vs 1.48 ms; with the accumulators pinned, 1.391 ms
// against 1.527 for the L-side table and 1.445 for the unpinned transposed read).  The FP32
// tables (normalised basis) satisfy the same identity, and with the accumulators pinned the FP32
// kernel gains as well (P = 14: 0.512 vs 0.633 ms, P = 16: 0.915 vs 1.043 ms, P = 12 equal;
// outputs bit-identical to the L-side table's).
template <typename Acc, int PM>
constexpr bool lpt_transposed_l()
{
    return PM >= 12;
}

// IDX: translations gather their input from the index array src and scatter to dst
// (indexed pools); otherwise translation i of the call uses solid i of in / out.
// SGL (M2L only): the single-height z-step, a compile-time choice so that the double-height
// kernel carries no per-coefficient selection (2^20 FP64 M2L, one MI355X: a run-time flag
// cost 3% at P = 13, 15 and 16 and 7% at P = 14, in scalar selects on the z-step's path).
template <typename Real, typename Acc, int OP, int PIN, int POUT, bool IDX, bool SGL>
__global__ __launch_bounds__((64 * lpt_waves<Acc, (PIN > POUT ? PIN : POUT)>()),
                             (lpt_min_waves_nw<Acc, (PIN > POUT ? PIN : POUT)>()))
void k_lpt(DevTables tab, TransArgs a)
{
    constexpr int PM = PIN > POUT ? PIN : POUT;
    constexpr int SIN = PIN * (PIN + 1), SOUT = POUT * (POUT + 1);
    constexpr int SP = lpt_stride<PM>();
    constexpr bool HOLD = lpt_hold_powers<Acc, PM>();
    constexpr int NW = lpt_waves<Acc, PM>();  // wavefronts of the workgroup
    constexpr int NT = 64 * NW;               // its threads
    using P2 = typename Pair<Acc>::T;
    using R2 = typename Pair<Real>::T;
    __shared__ Acc X[64 * SP];
    __shared__ int bad[64];
    __shared__ int bad_flag;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    using T = Tab<Real, Acc>;
    // L-side swaps (forward for L2L, backward for M2L and L2L): from the L-side table, or
    // from the M-side table read transposed (lpt_transposed_l)
    constexpr bool TL = lpt_transposed_l<Acc, PM>();
    constexpr bool FT = TL && OP == OP_L2L, BT = TL && OP != OP_M2M;
    const cptr<Acc> Pfw0 = as_const(T::packed(tab, (OP == OP_L2L && !TL) ? 1 : 0));
    const cptr<Acc> Pbw0 = as_const(T::packed(tab, (OP != OP_M2M && !TL) ? 1 : 0));
    const cptr<Acc> Z0 = as_const(T::z(tab, OP));
    static_assert(!SGL || OP == OP_M2L, "single height is an M2L form");
    constexpr bool single = SGL;
    const Real *__restrict__ rr = reinterpret_cast<const Real *>(a.r);
    const Real *__restrict__ gin = reinterpret_cast<const Real *>(a.in);
    Real *__restrict__ gout = reinterpret_cast<Real *>(a.out);
    const bool acc = (a.flags & 1u) != 0;
    const int64_t nblk = (a.count + 63) / 64;

    // Input of a block: NP (Re, Im) pairs, LIT per thread.  When they fit in <= 64 VGPRs
    // the next block's pairs and shifts are fetched into registers while the current block
    // is transformed (software pipelining across the persistent loop); otherwise each block
    // is loaded in chunks when it starts.  Every load is unconditional -- lanes past the
    // end of a partial block re-read a valid solid of the block -- so no load waits on
    // another (a guarded load splits the code and the wait-count pass then serialises).
    constexpr int NP = 64 * (SIN / 2);
    constexpr int LIT = (NP + NT - 1) / NT;
    // Where the 64 solids leave LDS room for one workgroup per CU (FP64 orders 13..16),
    // every lane reads the rows of its own translation straight into registers in the
    // forward rotation: no load phase through LDS, and the loads of one wavefront overlap
    // the other wavefronts' arithmetic.  (Storing the output rows straight from the
    // backward rotation as well measured no faster than the coalesced store phase, and
    // non-temporal per-lane row stores were 2.5x slower: partial-line writes.)
    constexpr bool DIRECT = NW >= 8;
    constexpr bool PREFETCH = !DIRECT && LIT * 2 * (int)sizeof(Real) / 4 <= 64 && lpt_prefetch_ok<Real, PM>();
    constexpr int CH = PREFETCH ? LIT : 16 * 4 / (int)sizeof(Real);  // loads per batch
    R2 pre[CH];
    Real prx = 0, pry = 0, prz = 1;
    const int64_t *__restrict__ gsrc = a.src;
    const int64_t *__restrict__ gdst = a.dst;
    // issue the loads of pairs c0 + tid + NT i (i < CH) of the block at bb (ntb translations)
    // IDX: each lane loads the source index of translation `lane` of the block once, and the
    // loads of a pair take their translation's index from that lane by a cross-lane read (one
    // global load per lane instead of one per pair; with the destination indices read the same
    // way, 2^20 FP64 M2L with sorted indices at P = 10: 0.439 ms, from 0.457)
    auto load_batch = [&](int64_t bb, int ntb, int c0) {
        int64_t row[IDX ? CH : 1];
        if constexpr (IDX) {
            const long mine = gsrc[bb + (lane < ntb ? lane : ntb - 1)];
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int t = (c0 + tid + NT * i) / (SIN / 2);
                row[i] = __shfl(mine, t < ntb ? t : ntb - 1, 64);
            }
        }
        // block base (wave-uniform, 64-bit) + 32-bit per-lane offsets (ld_in < 2^24)
        const Real *__restrict__ bin = gin + bb * a.ld_in;
        const int ldi = (int)a.ld_in;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int p = c0 + tid + NT * i;
            const int t = p / (SIN / 2);
            const int k = 2 * (p - t * (SIN / 2));
            if constexpr (IDX)
                pre[i] = *reinterpret_cast<const R2 *>(gin + row[i] * a.ld_in + k);
            else
                pre[i] = *reinterpret_cast<const R2 *>(bin + ((t < ntb ? t : ntb - 1) * ldi + k));
        }
    };
    // write the batch to LDS (rows of translations >= ntb are written but never used)
    auto store_batch_lds = [&](int c0) {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int p = c0 + tid + NT * i;
            if (c0 + NT * i + NT <= NP || p < NP) {
                const int t = p / (SIN / 2);
                const int k = 2 * (p - t * (SIN / 2));
                *reinterpret_cast<P2 *>(&X[t * SP + k]) = P2{(Acc)pre[i].x, (Acc)pre[i].y};
            }
        }
    };
    auto load_shift = [&](int64_t bb, int ntb) {
        const int tc = lane < ntb ? lane : ntb - 1;
        prx = rr[3 * (bb + tc)];
        pry = rr[3 * (bb + tc) + 1];
        prz = rr[3 * (bb + tc) + 2];
    };
    auto block_count = [&](int64_t b) { return (int)((a.count - b * 64) < 64 ? (a.count - b * 64) : 64); };
    if (PREFETCH && (int64_t)blockIdx.x < nblk) {
        load_batch((int64_t)blockIdx.x * 64, block_count(blockIdx.x), 0);
        load_shift((int64_t)blockIdx.x * 64, block_count(blockIdx.x));
    }

    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t base = blk * 64;
        const int nt = block_count(blk);
        // IDX: destination index of translation `lane` of this block, loaded now so that the
        // store phase reads it from this lane without waiting on memory
        long dmine = 0;
        if constexpr (IDX) dmine = gdst[base + (lane < nt ? lane : nt - 1)];
        const cptr<Acc> Pfw = launder(Pfw0), Pbw = launder(Pbw0), Z = launder(Z0);
        if constexpr (PREFETCH) {
            store_batch_lds(0);
        } else if constexpr (DIRECT) {
            load_shift(base, nt);
        } else {
#pragma unroll 1
            for (int c0 = 0; c0 < NP; c0 += NT * CH) {
                load_batch(base, nt, c0);
                store_batch_lds(c0);
            }
            load_shift(base, nt);
        }
        // DIRECT: this lane's input solid (lanes past a partial block re-read the last one)
        const Real *__restrict__ lin = gin;
        if constexpr (DIRECT) {
            const int tc = lane < nt ? lane : nt - 1;
            lin = gin + (IDX ? gsrc[base + tc] : base + tc) * a.ld_in;
        }
        double x = (double)prx, y = (double)pry, z = (double)prz;
        if (lane >= nt) {
            x = 0.0;
            y = 0.0;
            z = 1.0;
        }

        // ---- per-lane shift geometry (every wavefront, redundantly) ----
        const Geometry g = shift_geometry(x, y, z);
        if (wave == 0) {
            bad[lane] = (g.valid == 1) ? 0 : (g.valid == 0 ? 1 : 2);
            const bool any = __any(g.valid != 1 && lane < nt);
            if (lane == 0) bad_flag = any ? 1 : 0;
        }
        Powers<Acc, PM, HOLD> pw;
        pw.init(g);
        const Acc s = (Acc)(g.valid == 1 ? g.s : 1.0);
        const Acc R = (Acc)(g.valid == 1 ? g.R : 1.0);
        Acc *Xt = X + lane * SP;
        bool bad_any;
        if constexpr (DIRECT) {
            // every wavefront holds all 64 shifts: the block-wide test needs no LDS round trip,
            // and nothing else of this block is in LDS yet (the previous block ended with a
            // barrier after its store phase)
            bad_any = __any(g.valid != 1 && lane < nt);
        } else {
            lds_barrier();
            bad_any = bad_flag != 0;
        }
        if constexpr (PREFETCH) {
            const int64_t nb = blk + gridDim.x;
            if (nb < nblk) {  // in flight during the transform of this block
                load_batch(nb * 64, block_count(nb), 0);
                load_shift(nb * 64, block_count(nb));
            }
        }

        // ---- forward rotation of the input rows ----
        per_wave<NW>(wave, [&](auto wc) {
        static_for<0, PIN>([&](auto nc) {
            constexpr int n = decltype(nc)::value;
            if constexpr (row_owner(PIN, n, NW) == decltype(wc)::value) {
            Acc xr[n + 1], xi[n + 1], yr[n + 1], yi[n + 1];
            if constexpr (DIRECT) {
                __builtin_amdgcn_sched_barrier(0);  // one row's loads in flight at a time
                R2 v[n + 1];
#pragma unroll
                for (int m = 0; m <= n; ++m) v[m] = *reinterpret_cast<const R2 *>(lin + solid_pos(n, m));
#pragma unroll
                for (int m = 0; m <= n; ++m) {
                    xr[m] = (Acc)v[m].x;
                    xi[m] = m ? (Acc)v[m].y : (Acc)0;
                }
            } else {
#pragma unroll
                for (int m = 0; m <= n; ++m) {
                    const P2 v = *reinterpret_cast<const P2 *>(&Xt[solid_pos(n, m)]);
                    xr[m] = v.x;
                    xi[m] = m ? v.y : (Acc)0;
                }
            }
            // scale: M2L/M2M  M_n / |r|^{n+1};  L2L  L_n |r|^n   (eq. scaling)
            const Acc f = (OP == OP_L2L) ? ipow(R, n) : ipow(s, n + 1);
#pragma unroll
            for (int m = 0; m <= n; ++m) {
                xr[m] *= f;
                xi[m] *= f;
            }
            pw.template rot<n>(xr, xi, 0, (Acc)1);
            swap_row_x<Acc, n, FT>(Pfw, xr, xi, yr, yi);
            pw.template rot<n>(yr, yi, 1, (Acc)1);
            swap_row_x<Acc, n, FT>(launder(Pfw), yr, yi, xr, xi);
#pragma unroll
            for (int m = 0; m <= n; ++m) *reinterpret_cast<P2 *>(&Xt[solid_pos(n, m)]) = P2{xr[m], xi[m]};
            }
        });
        });
        lds_barrier();

        // ---- z-axis step, one column (order m) at a time, unit shift ----
        per_wave<NW>(wave, [&](auto wc) {
        static_for<0, POUT>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            if constexpr (col_owner(PIN, POUT, m, NW) != decltype(wc)::value) {
            } else if constexpr (m >= PIN) {
#pragma unroll
                for (int o = m; o < POUT; ++o) *reinterpret_cast<P2 *>(&Xt[solid_pos(o, m)]) = P2{(Acc)0, (Acc)0};
            } else {
                Acc ir[PIN], ii[PIN];
#pragma unroll
                for (int k = m; k < PIN; ++k) {
                    const P2 v = *reinterpret_cast<const P2 *>(&Xt[solid_pos(k, m)]);
                    ir[k] = v.x;
                    ii[k] = v.y;
                }
                // coefficients of output o + 1 are fetched while output o is summed
                Acc cz[PIN - m];
                z_fetch<Real, Acc, OP, PIN, m>(Z, m, cz, single);
#pragma unroll
                for (int o = m; o < POUT; ++o) {
                    Acc nz[PIN - m];
                    if (o + 1 < POUT) z_fetch<Real, Acc, OP, PIN, m>(Z, o + 1, nz, single);
                    Acc orr = 0, oi = 0;
#pragma unroll
                    for (int k = m; k < PIN; ++k) {
                        if (OP == OP_M2M && k > o) continue;
                        if (OP == OP_L2L && k < o) continue;
                        orr += cz[k - m] * ir[k];
                        oi += cz[k - m] * ii[k];
                    }
                    *reinterpret_cast<P2 *>(&Xt[solid_pos(o, m)]) = P2{orr, oi};
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int k = 0; k < PIN - m; ++k) cz[k] = nz[k];
                }
            }
        });
        });
        lds_barrier();

        // ---- backward rotation of the output rows ----
        per_wave<NW>(wave, [&](auto wc) {
        static_for<0, POUT>([&](auto nc) {
            constexpr int n = decltype(nc)::value;
            if constexpr (row_owner(POUT, n, NW) == decltype(wc)::value) {
            Acc xr[n + 1], xi[n + 1], yr[n + 1], yi[n + 1];
#pragma unroll
            for (int m = 0; m <= n; ++m) {
                const P2 v = *reinterpret_cast<const P2 *>(&Xt[solid_pos(n, m)]);
                xr[m] = v.x;
                xi[m] = m ? v.y : (Acc)0;
            }
            swap_row_x<Acc, n, BT>(Pbw, xr, xi, yr, yi);
            pw.template rot<n>(yr, yi, 1, (Acc)-1);
            swap_row_x<Acc, n, BT>(launder(Pbw), yr, yi, xr, xi);
            pw.template rot<n>(xr, xi, 0, (Acc)-1);
            // unscale: M2L/L2L  L_n / |r|^n;  M2M  M_n |r|^{n+1}
            const Acc f = (OP == OP_M2M) ? ipow(R, n + 1) : ipow(s, n);
#pragma unroll
            for (int m = 0; m <= n; ++m)
                *reinterpret_cast<P2 *>(&Xt[solid_pos(n, m)]) = P2{xr[m] * f, m ? xi[m] * f : (Acc)0};
            }
        });
        });
        lds_barrier();

        // ---- coalesced store.  Common case (overwrite, every shift valid): destination
        //      rows first, then every store back to back.  Accumulation and invalid
        //      shifts take the per-element path below. ----
        if (!acc && !bad_any) {
            constexpr int NQ = 64 * (SOUT / 2);
            constexpr int SIT = (NQ + NT - 1) / NT;
            const int nq = nt * (SOUT / 2);
            int64_t drow[IDX ? SIT : 1];
            Real *__restrict__ bout = gout + base * a.ld_out;  // block base + 32-bit offsets
            const int ldo = (int)a.ld_out;
            if constexpr (IDX) {
                // destination indices from the lanes that loaded them at the block's start
#pragma unroll
                for (int i = 0; i < SIT; ++i) {
                    const int t = (tid + NT * i) / (SOUT / 2);
                    drow[i] = __shfl(dmine, t < nt ? t : nt - 1, 64);
                }
            }
            if (nt == 64) {
#pragma unroll
                for (int i = 0; i < SIT; ++i) {
                    const int p = tid + NT * i;
                    if (NT * i + NT <= NQ || p < NQ) {
                        const int t = p / (SOUT / 2);
                        const int k = 2 * (p - t * (SOUT / 2));
                        const P2 v = *reinterpret_cast<const P2 *>(&X[t * SP + k]);
                        Real *d = IDX ? gout + drow[i] * a.ld_out + k : bout + (t * ldo + k);
                        *reinterpret_cast<R2 *>(d) = R2{(Real)v.x, (Real)v.y};
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < SIT; ++i) {
                    const int p = tid + NT * i;
                    if (p < nq) {
                        const int t = p / (SOUT / 2);
                        const int k = 2 * (p - t * (SOUT / 2));
                        const P2 v = *reinterpret_cast<const P2 *>(&X[t * SP + k]);
                        Real *d = IDX ? gout + drow[i] * a.ld_out + k : bout + (t * ldo + k);
                        *reinterpret_cast<R2 *>(d) = R2{(Real)v.x, (Real)v.y};
                    }
                }
            }
        } else
        for (int p = tid; p < nt * (SOUT / 2); p += NT) {
            const int t = p / (SOUT / 2);
            const int k = 2 * (p - t * (SOUT / 2));
            const int64_t di = IDX ? gdst[base + t] : base + t;
            R2 *dstp = reinterpret_cast<R2 *>(gout + di * a.ld_out + k);
            const P2 v = *reinterpret_cast<const P2 *>(&X[t * SP + k]);
            R2 w{(Real)v.x, (Real)v.y};
            const int b = bad[t];
            if (b != 0 || acc) {
                int n = (int)((sqrtf(4.0f * (float)k + 1.0f) - 1.0f) * 0.5f);
                while ((n + 1) * (n + 2) <= k) ++n;
                while (n * (n + 1) > k) --n;
                const bool m0 = (k == n * (n + 1));
                if (b != 0) {
                    if (b == 1 && OP != OP_M2L) {
                        // zero shift of M2M / L2L: identity, truncated / zero-padded
                        const int64_t si = IDX ? gsrc[base + t] : base + t;
                        const bool keep = n < PIN && n < POUT;
                        w.x = keep ? gin[si * a.ld_in + k] : (Real)0;
                        w.y = (keep && !m0) ? gin[si * a.ld_in + k + 1] : (Real)0;
                    } else {
                        w.x = w.y = (Real)NAN;
                        if (k == 0) raise_device_error(a.err, -3);
                    }
                }
                if (acc && !(b != 0 && !(b == 1 && OP != OP_M2L))) {
                    const R2 old = *dstp;
                    w.x += old.x;
                    if (!m0) w.y += old.y;
                }
            }
            *dstp = w;
        }
        lds_barrier();
    }
}

// Workgroups resident at once on the current device for kernel fn (CU count x occupancy).
int resident_workgroups(const void *fn);

template <typename Real, typename Acc, int OP, int PV, bool IDX, bool SGL>
hipError_t launch_one_form(const DevTables &tab, const TransArgs &a, hipStream_t s)
{
    const void *fn = reinterpret_cast<const void *>(&k_lpt<Real, Acc, OP, PV, PV, IDX, SGL>);
    const int64_t nblk = (a.count + 63) / 64;
    const int64_t res = resident_workgroups(fn);
    const dim3 grid((unsigned)(nblk < res ? nblk : res)), block(64 * lpt_waves<Acc, PV>());
    hipLaunchKernelGGL((k_lpt<Real, Acc, OP, PV, PV, IDX, SGL>), grid, block, 0, s, tab, a);
    return hipGetLastError();
}

template <typename Real, typename Acc, int OP, int PV, bool IDX>
hipError_t launch_one(const DevTables &tab, const TransArgs &a, hipStream_t s)
{
    if constexpr (OP == OP_M2L) {
        if ((a.flags & kSingleHeightFlag) != 0) return launch_one_form<Real, Acc, OP, PV, IDX, true>(tab, a, s);
    }
    return launch_one_form<Real, Acc, OP, PV, IDX, false>(tab, a, s);
}

// Launcher for one (dtype, op); instantiated in the k_lpt_<dtype>_<op>.hip units.
template <typename Real, typename Acc, int OP>
hipError_t launch_fixed(int P, const DevTables &tab, const TransArgs &a, hipStream_t s)
{
    const bool idx = a.src != nullptr;
    switch (P) {
#define SH_CASE(PV)                                                                       \
    case PV:                                                                              \
        return idx ? launch_one<Real, Acc, OP, PV, true>(tab, a, s)                       \
                   : launch_one<Real, Acc, OP, PV, false>(tab, a, s);
        SH_CASE(2)
        SH_CASE(3)
        SH_CASE(4)
        SH_CASE(5)
        SH_CASE(6)
        SH_CASE(7)
        SH_CASE(8)
        SH_CASE(9)
        SH_CASE(10)
        SH_CASE(11)
        SH_CASE(12)
        SH_CASE(13)
        SH_CASE(14)
        SH_CASE(15)
        SH_CASE(16)
#undef SH_CASE
    default:
        return hipErrorInvalidValue;
    }
}

extern template hipError_t launch_fixed<double, double, OP_M2M>(int, const DevTables &, const TransArgs &, hipStream_t);
extern template hipError_t launch_fixed<double, double, OP_M2L>(int, const DevTables &, const TransArgs &, hipStream_t);
extern template hipError_t launch_fixed<double, double, OP_L2L>(int, const DevTables &, const TransArgs &, hipStream_t);
extern template hipError_t launch_fixed<float, float, OP_M2M>(int, const DevTables &, const TransArgs &, hipStream_t);
extern template hipError_t launch_fixed<float, float, OP_M2L>(int, const DevTables &, const TransArgs &, hipStream_t);
extern template hipError_t launch_fixed<float, float, OP_L2L>(int, const DevTables &, const TransArgs &, hipStream_t);

}  // namespace lpt
}  // namespace shfmm
