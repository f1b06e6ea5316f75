// Block kernel for large orders (up to 31): the rotation scheme of Section 3.4 on the FP64
// matrix cores, 16 translations at a time.
//
// A lane-per-translation kernel needs 64 solids in LDS, which no longer fits above order 16.
// Here a workgroup holds 16 solids in LDS, coefficient-major (X[c][t], t = translation), and
// every O(P^3) step becomes a small GEMM whose N dimension is the 16 translations:
//   * swaps: the chequerboard of F / G splits each row's swap into two dense blocks by the
//     parity of the output order m (m + l + n even for the real part, odd for the imaginary
//     part), each at most 16 x 16 up to degree 31: one 16 x 16 x 4 FP64 MFMA per K step, with
//     A = table fragments (prepared on the host in operand order, read from L2) and
//     B = the row's coefficients of the 16 translations (LDS);
//   * z-translation: per column m, the column's Hankel / Toeplitz matrix times the column of
//     the 16 rotated solids, real and imaginary parts as two GEMMs sharing the fragments.
// The O(P^2) steps (scaling, z-rotations) run on the VALU between the GEMMs, on the MFMA
// output registers.  Rows (forward and backward rotations) and columns (z-step) are spread
// over the 8 wavefronts (two per SIMD) in snake order; LDS barriers separate the phases.
// FP64 16x16x4 MFMA operand layout (checked on the device): A[l % 16][l / 16],
// B[l / 16][l % 16], D[4 j + l / 16][l % 16] for lane l and output register j.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "layout.hpp"

namespace shfmm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kBT = 16;     // translations per block
// Wavefronts per workgroup: 8 (two per SIMD, hiding each other's latency) where a block's LDS
// leaves room for one workgroup per CU; 4 where two workgroups fit (orders up to 21), so that two
// blocks are in flight per CU and one's z-step overlaps the other's memory streams.
constexpr int kLdsPerCu = 160 * 1024;

template <typename Real>
struct Pair2;
template <>
struct Pair2<double> {
    using T = double2;
};
template <>
struct Pair2<float> {
    using T = float2;
};

// LDS carve-up (in doubles): (n, m) of pair p[528] | X[S][16] | powers[4][32][16] | scale_in[32][16]
// | scale_out[32][16] | in offsets[16] | out offsets[16] | shifts[16][3] | bad flags[16].  The pair
// table comes first so that its place does not depend on the orders of a task.
constexpr int kBigPairs = kBigOrder * (kBigOrder + 1) / 2;
static_assert(kBigPairs % 4 == 0, "the pair table fills whole doubles");
struct BigLds {
    int pm;  // order stride of the power and scale tables (the block's largest order)
    double *X, *pw, *scin, *scout, *r;
    int64_t *ioff, *ooff;
    int *bad;
    unsigned short *nm;  // 32 n + m of pair index p = n (n + 1) / 2 + m
};

// Offsets (in doubles) of the LDS carve-up; big_lds and the launch size both come from here.
struct BigLdsOffsets {
    size_t X, pw, scin, scout, ioff, ooff, r, bad, end;
};
__host__ __device__ constexpr BigLdsOffsets big_lds_offsets(int PM)
{
    BigLdsOffsets o{};
    o.X = kBigPairs / 4;
    o.pw = o.X + (size_t)PM * (PM + 1) * kBT;
    o.scin = o.pw + 4 * (size_t)PM * kBT;
    o.scout = o.scin + (size_t)PM * kBT;
    o.ioff = o.scout + (size_t)PM * kBT;
    o.ooff = o.ioff + kBT;
    o.r = o.ooff + kBT;
    o.bad = o.r + 3 * kBT;
    o.end = o.bad + kBT / 2;
    return o;
}
__host__ __device__ constexpr size_t big_lds_doubles(int PM) { return big_lds_offsets(PM).end; }

__device__ __forceinline__ BigLds big_lds(double *sm, int PM)
{
    const BigLdsOffsets o = big_lds_offsets(PM);
    BigLds L;
    L.pm = PM;
    L.nm = reinterpret_cast<unsigned short *>(sm);
    L.X = sm + o.X;
    L.pw = sm + o.pw;
    L.scin = sm + o.scin;
    L.scout = sm + o.scout;
    L.ioff = reinterpret_cast<int64_t *>(sm + o.ioff);
    L.ooff = reinterpret_cast<int64_t *>(sm + o.ooff);
    L.r = sm + o.r;
    L.bad = reinterpret_cast<int *>(sm + o.bad);
    return L;
}

// degree n of pair index p (p = n(n+1)/2 + m)
__device__ __forceinline__ int pair_degree(int p)
{
    int n = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
    while ((n + 1) * (n + 2) / 2 <= p) ++n;
    while (n * (n + 1) / 2 > p) --n;
    return n;
}

// Fills the (n, m) table of every pair index below kBigPairs; it depends on nothing else, so a
// workgroup fills it once, before its first barrier.
__device__ __forceinline__ void fill_pair_table(const BigLds &L)
{
    for (int p = threadIdx.x; p < kBigPairs; p += blockDim.x) {
        const int n = pair_degree(p);
        L.nm[p] = (unsigned short)(32 * n + (p - n * (n + 1) / 2));
    }
}

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Index (in doubles) of element (pair p, translation t) in X: the real part, followed by the
// imaginary part, so one 16-byte LDS access moves both.
__device__ __forceinline__ int xe(int p, int t) { return (p * kBT + t) * 2; }
// Index of (cos, sin) of m times angle k (0: alpha, 1: beta) of translation t in the power table.
__device__ __forceinline__ int pwi(const BigLds &L, int k, int m, int t) { return ((k * L.pm + m) * kBT + t) * 2; }
__device__ __forceinline__ double2 lds2(const double *p) { return *reinterpret_cast<const double2 *>(p); }
__device__ __forceinline__ void sts2(double *p, double a, double b) { *reinterpret_cast<double2 *>(p) = double2{a, b}; }
// Waits until every vector memory operation this wavefront has issued is complete (the
// compiler does not track LDS written by direct loads).
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Operator fragments of row n (both parities and parts, every K step; K steps past the
// row's count are zero in the table and never used).  Both swaps of a row use the same table.
// The loads are unconditional (every degree's slot has the same size), so a fetch issued for
// the next row stays in flight while the current row is transformed.
struct RowFrag {
    double a[2][2][4];
};
__device__ __forceinline__ void load_row_frag(const double *__restrict__ frag, int n, int lane, RowFrag &f)
{
    const double *F = frag + big_swap_off(n < kBigOrder ? n : kBigOrder - 1) + lane;
#pragma unroll
    for (int pm = 0; pm < 2; ++pm)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) f.a[pm][q][ks] = F[((pm * 2 + q) * 4 + ks) * 64];
}

// Swap of row n of the 16 solids: D[pm][q] = (output parity pm, part q) blocks; NP = n & 1 (so
// that the input parity each block takes is known at compile time).  Each lane reads (re, im)
// of the two input orders of its K index and step (one per parity) before the first product.
// Orders past the degree read order n instead: the operator fragments are zero there (and zero
// in the imaginary part at order 0), so those products add exact zeros.  With RAW the row holds
// the input as loaded: Im C_n^0 is dropped, and the scale and the rotation by e^{i m alpha} are
// applied here.
template <bool RAW, int NP>
__device__ __forceinline__ void swap_row(const RowFrag &f, const double *X, const BigLds &L, int n, int lane,
                                         d4 (&D)[2][2])
{
    const int ks_n = big_ks(n);
    const int t = lane & 15, kg = lane >> 4;
    const double *Xn = X + xe(n * (n + 1) / 2, t);
    const double sc = RAW ? L.scin[n * kBT + t] : 1.0;
    double b[2][2][4];  // [input parity][part][K step]
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        if (ks >= ks_n) break;
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            const int lc = 2 * (4 * ks + kg) + par;
            const int l = lc <= n ? lc : n;
            const double2 v = lds2(Xn + l * 2 * kBT);
            double re = v.x, im = v.y;
            if (RAW) {
                const double2 cs = lds2(L.pw + pwi(L, 0, l, t));
                const double a = re * sc, c = l ? im * sc : 0.0;
                re = a * cs.x - c * cs.y;
                im = a * cs.y + c * cs.x;
            }
            b[par][0][ks] = re;
            b[par][1][ks] = im;
        }
    }
#pragma unroll
    for (int pm = 0; pm < 2; ++pm)
#pragma unroll
        for (int q = 0; q < 2; ++q) D[pm][q] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        if (ks >= ks_n) break;
#pragma unroll
        for (int pm = 0; pm < 2; ++pm)
#pragma unroll
            for (int q = 0; q < 2; ++q) D[pm][q] = mfma64(f.a[pm][q][ks], b[(NP + pm + q) & 1][q][ks], D[pm][q]);
    }
}

// Second swap of a row straight from the first swap's output registers: in the D layout,
// element j of lane group g holds order m = 2 (4 j + g) + p of parity block p, which is exactly
// the B operand of K step j, K index g, for the input-parity p = (n + pm + q) & 1 blocks.
template <int NP>
__device__ __forceinline__ void swap_row_regs(const RowFrag &f, int n, const d4 (&Din)[2][2], d4 (&D)[2][2])
{
    const int ks_n = big_ks(n);
#pragma unroll
    for (int pm = 0; pm < 2; ++pm)
#pragma unroll
        for (int q = 0; q < 2; ++q) D[pm][q] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        if (ks >= ks_n) break;
#pragma unroll
        for (int pm = 0; pm < 2; ++pm)
#pragma unroll
            for (int q = 0; q < 2; ++q) D[pm][q] = mfma64(f.a[pm][q][ks], Din[(NP + pm + q) & 1][q][ks], D[pm][q]);
    }
}

// Rotates the D blocks of row n in place by e^{+-i m beta}.  Orders m > n are zero in D.
__device__ __forceinline__ void rotate_beta(const BigLds &L, int n, int lane, d4 (&D)[2][2], double sgn)
{
    const int t = lane & 15, g = lane >> 4;
#pragma unroll
    for (int pm = 0; pm < 2; ++pm)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = 2 * (4 * j + g) + pm;
            if (m > n) continue;
            const double2 cs = lds2(L.pw + pwi(L, 1, m, t));
            const double s = sgn * cs.y;
            const double re = D[pm][0][j], im = D[pm][1][j];
            D[pm][0][j] = re * cs.x - im * s;
            D[pm][1][j] = re * s + im * cs.x;
        }
}

// Writes the D blocks of row n back to X, after an optional rotation by e^{-i m alpha} and
// scale per translation.
__device__ __forceinline__ void write_row(double *X, const BigLds &L, int n, int lane, const d4 (&D)[2][2], bool unrotate)
{
    const int t = lane & 15, g = lane >> 4;
    double *Xn = X + xe(n * (n + 1) / 2, t);
    const double f = unrotate ? L.scout[n * kBT + t] : 1.0;
#pragma unroll
    for (int pm = 0; pm < 2; ++pm)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = 2 * (4 * j + g) + pm;
            if (m > n) continue;
            double re = D[pm][0][j], im = D[pm][1][j];
            if (unrotate) {
                const double2 cs = lds2(L.pw + pwi(L, 0, m, t));
                const double a = re;
                re = (a * cs.x + im * cs.y) * f;
                im = (im * cs.x - a * cs.y) * f;
            }
            sts2(Xn + m * 2 * kBT, re, m ? im : 0.0);
        }
}

// Final form of row n straight to memory: rotation by e^{-i m alpha}, the output scale, and
// the store of every order m <= n of translations t < nt.
template <typename Real>
__device__ __forceinline__ void store_row(Real *__restrict__ aout, const BigLds &L, int n, int lane, const d4 (&D)[2][2],
                                          int nt)
{
    using R2 = typename Pair2<Real>::T;
    const int t = lane & 15, g = lane >> 4;
    if (t >= nt) return;
    R2 *row = reinterpret_cast<R2 *>(aout + L.ooff[t]) + n * (n + 1) / 2;
    const double f = L.scout[n * kBT + t];
#pragma unroll
    for (int pm = 0; pm < 2; ++pm)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = 2 * (4 * j + g) + pm;
            if (m > n) continue;
            const double2 cs = lds2(L.pw + pwi(L, 0, m, t));
            const double re = D[pm][0][j], im = D[pm][1][j];
            R2 w;
            w.x = (Real)((re * cs.x + im * cs.y) * f);
            w.y = m ? (Real)((im * cs.x - re * cs.y) * f) : (Real)0;
            row[m] = w;
        }
}

// Issues the direct-to-LDS loads of input row n (pairs n(n+1)/2 .. n(n+1)/2 + n of every
// translation) into its place in X: each instruction moves 4 pairs of the 16 translations,
// lane l taking pair 4 i + l / 16 of translation l % 16, which is X's own order.
__device__ __forceinline__ void dma_row(const double *__restrict__ ain, const BigLds &L, int n, int lane)
{
    const int t = lane & 15, pl = lane >> 4;
    const int p0 = n * (n + 1) / 2;
    const double *src = ain + L.ioff[t] + 2 * (p0 + pl);
    for (int i = 0; 4 * i <= n; ++i) {
        if (4 * i + pl <= n)
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src + 8 * i),
                                             (__attribute__((address_space(3))) void *)(L.X + xe(p0 + 4 * i, 0)), 16,
                                             0, 0);
    }
}

// One block of up to 16 translations whose offsets and shifts are in L (t >= nt repeat the
// last valid translation and are not stored).
template <typename Real, int OP, int NW>
__device__ void big_block(const DevTables &tab, const BigLds &L, int p_in, int p_out, int nt, const Real *__restrict__ ain,
                          Real *__restrict__ aout, bool acc_out, int *err)
{
    using R2 = typename Pair2<Real>::T;
    constexpr int basis = sizeof(Real) == 4 ? 1 : 0;
    // FP64 inputs go from memory to LDS as they are, one row ahead of the forward rotation
    // that uses them; FP32 inputs pass through registers (to widen them) in a load phase.
    constexpr bool direct = sizeof(Real) == 8;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int kWaves = NW, kThreads = 64 * NW;
    double *X = L.X;
    auto row_of = [&](int n0) { return n0 + (((n0 / kWaves) & 1) ? kWaves - 1 - wave : wave); };

    if constexpr (direct) {
        if (row_of(0) < p_in) dma_row(reinterpret_cast<const double *>(ain), L, row_of(0), lane);
    }

    // ---- geometry, powers and scales: thread (m, t) fills order m of translation t, every
    // order below the block's largest (powers by repeated squaring) ----
    for (int mt = tid; mt < L.pm * kBT; mt += kThreads) {
        const int t = mt & 15, m = mt >> 4;
        const Geometry g = shift_geometry(L.r[3 * t], L.r[3 * t + 1], L.r[3 * t + 2]);
        const bool ok = g.valid == 1;
        if (m == 0) L.bad[t] = ok ? 0 : (g.valid == 0 ? 1 : 2);
        double ca = ok ? g.ca : 1.0, sa = ok ? g.sa : 0.0, cb = ok ? g.cb : 1.0, sb = ok ? g.sb : 0.0;
        double R = ok ? g.R : 1.0, sr = ok ? g.s : 1.0;
        const double R1 = R, s1 = sr;
        double c1 = 1.0, s1m = 0.0, c2 = 1.0, s2m = 0.0, rn = 1.0, sn = 1.0;
        for (int k = m; k; k >>= 1) {
            if (k & 1) {
                const double u1 = c1 * ca - s1m * sa;
                s1m = c1 * sa + s1m * ca;
                c1 = u1;
                const double u2 = c2 * cb - s2m * sb;
                s2m = c2 * sb + s2m * cb;
                c2 = u2;
                rn *= R;
                sn *= sr;
            }
            const double v1 = ca * ca - sa * sa;
            sa = 2.0 * ca * sa;
            ca = v1;
            const double v2 = cb * cb - sb * sb;
            sb = 2.0 * cb * sb;
            cb = v2;
            R *= R;
            sr *= sr;
        }
        sts2(L.pw + pwi(L, 0, m, t), c1, s1m);
        sts2(L.pw + pwi(L, 1, m, t), c2, s2m);
        // rn = R^m, sn = s^m
        L.scin[m * kBT + t] = (OP == OP_L2L) ? rn : sn * s1;
        L.scout[m * kBT + t] = (OP == OP_M2M) ? rn * R1 : sn;
    }
    __syncthreads();
    // outputs go straight from the backward rotation to memory unless the call accumulates
    // or a translation of the block has a zero or non-finite shift
    const bool fused = !acc_out && __ballot(lane < kBT && L.bad[lane & 15] != 0) == 0;

    // ---- FP32 load: widen, scale and rotate by alpha.  Thread (s, t) takes pairs p = s + 32 u
    // of translation t, so its source row and the immediate offsets of its loads and LDS stores
    // are fixed; each thread has all of its loads in flight before it uses one ----
    if constexpr (!direct) {
        constexpr int U = 16, TS = kThreads / 16;  // threads per translation
        const int t = tid & 15, s0 = tid >> 4;
        const int npin = p_in * (p_in + 1) / 2;
        const R2 *src = reinterpret_cast<const R2 *>(ain + L.ioff[t]);
        for (int base = 0; base < npin; base += TS * U) {
            R2 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = base + s0 + TS * u;
                v[u] = p < npin ? src[p] : R2{};
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = base + s0 + TS * u;
                if (p >= npin) break;
                const int nm = L.nm[p], n = nm >> 5, m = nm & 31;
                const double f = L.scin[n * kBT + t];
                const double a = (double)v[u].x * f, b = m ? (double)v[u].y * f : 0.0;
                const double2 cs = lds2(L.pw + pwi(L, 0, m, t));
                sts2(X + xe(p, t), a * cs.x - b * cs.y, m ? a * cs.y + b * cs.x : 0.0);
            }
        }
        __syncthreads();
    }

    const int fw = (OP == OP_L2L) ? 1 : 0, bw = (OP == OP_M2M) ? 0 : 1;
    const double *Ffw = tab.bsw[basis][fw], *Fbw = tab.bsw[basis][bw];

    // ---- forward rotation, rows in snake order over the wavefronts; the next row's
    // fragments (and, for FP64, its input) are fetched while the current row is transformed ----
    {
        auto row = [&](const RowFrag &f, int n) {
            d4 D[2][2], E[2][2];
            if (n & 1) {
                swap_row<direct, 1>(f, X, L, n, lane, D);
                rotate_beta(L, n, lane, D, 1.0);
                swap_row_regs<1>(f, n, D, E);
            } else {
                swap_row<direct, 0>(f, X, L, n, lane, D);
                rotate_beta(L, n, lane, D, 1.0);
                swap_row_regs<0>(f, n, D, E);
            }
            write_row(X, L, n, lane, E, false);
        };
        auto fetch = [&](int n, RowFrag &f) {
            if constexpr (direct) {
                wait_vm_all();  // the current row's input and fragments have landed
                if (n < p_in) dma_row(reinterpret_cast<const double *>(ain), L, n, lane);
            }
            load_row_frag(Ffw, n, lane, f);
        };
        RowFrag fa, fb;
        load_row_frag(Ffw, row_of(0), lane, fa);
        for (int n0 = 0; n0 < p_in; n0 += 2 * kWaves) {
            if (row_of(n0) >= p_in) break;
            fetch(row_of(n0 + kWaves), fb);
            row(fa, row_of(n0));
            if (row_of(n0 + kWaves) >= p_in) break;
            fetch(row_of(n0 + 2 * kWaves), fa);
            row(fb, row_of(n0 + kWaves));
        }
    }
    __syncthreads();

    // ---- z-translation, columns in snake order; the next column's fragments are fetched
    // (unconditionally, from fixed-size slots) while the current column is multiplied ----
    {
        const double *Zt = tab.bz[basis][OP];
        const int t = lane & 15, kg = lane >> 4;
        auto load_z = [&](int m, double (&za)[2][8]) {
            const double *Z = Zt + big_z_off(m < kBigOrder ? m : kBigOrder - 1) + lane;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) za[mt][ks] = Z[(mt * 8 + ks) * 64];
        };
        auto column = [&](const double (&za)[2][8], int m) {
            const int mto = (p_out - m + 15) / 16;
            const int ki = m < p_in ? (p_in - m + 3) / 4 : 0;
            double b[2][8];
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
                if (ks >= ki) break;
                const int i = m + 4 * ks + kg;
                const bool ok = i < p_in;
                const int r = ok ? i : m;
                const double2 v = lds2(X + xe(r * (r + 1) / 2 + m, t));
                b[0][ks] = ok ? v.x : 0.0;
                b[1][ks] = ok ? v.y : 0.0;
            }
            d4 res[2][2];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                d4 a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
                if (mt < mto) {
#pragma unroll
                    for (int ks = 0; ks < 8; ++ks) {
                        if (ks >= ki) break;
                        a0 = mfma64(za[mt][ks], b[0][ks], a0);
                        a1 = mfma64(za[mt][ks], b[1][ks], a1);
                    }
                }
                res[0][mt] = a0;
                res[1][mt] = a1;
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                if (mt >= mto) continue;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int o = m + 16 * mt + 4 * j + kg;
                    if (o >= p_out) continue;
                    sts2(X + xe(o * (o + 1) / 2 + m, t), res[0][mt][j], m ? res[1][mt][j] : 0.0);
                }
            }
        };
        double za[2][8], zb[2][8];
        load_z(row_of(0), za);
        for (int m0 = 0; m0 < p_out; m0 += 2 * kWaves) {
            if (row_of(m0) >= p_out) break;
            load_z(row_of(m0 + kWaves), zb);
            column(za, row_of(m0));
            if (row_of(m0 + kWaves) >= p_out) break;
            load_z(row_of(m0 + 2 * kWaves), za);
            column(zb, row_of(m0 + kWaves));
        }
    }
    __syncthreads();

    // ---- backward rotation, unscale ----
    {
        auto row = [&](const RowFrag &f, int n) {
            d4 D[2][2], E[2][2];
            if (n & 1) {
                swap_row<false, 1>(f, X, L, n, lane, D);
                rotate_beta(L, n, lane, D, -1.0);
                swap_row_regs<1>(f, n, D, E);
            } else {
                swap_row<false, 0>(f, X, L, n, lane, D);
                rotate_beta(L, n, lane, D, -1.0);
                swap_row_regs<0>(f, n, D, E);
            }
            if (fused)
                store_row<Real>(aout, L, n, lane, E, nt);  // rotate by -alpha, unscale, store
            else
                write_row(X, L, n, lane, E, true);  // rotate by -alpha, unscale
        };
        RowFrag fa, fb;
        load_row_frag(Fbw, row_of(0), lane, fa);
        for (int n0 = 0; n0 < p_out; n0 += 2 * kWaves) {
            if (row_of(n0) >= p_out) break;
            load_row_frag(Fbw, row_of(n0 + kWaves), lane, fb);
            row(fa, row_of(n0));
            if (row_of(n0 + kWaves) >= p_out) break;
            load_row_frag(Fbw, row_of(n0 + 2 * kWaves), lane, fa);
            row(fb, row_of(n0 + kWaves));
        }
    }
    __syncthreads();

    // ---- store (when the backward rotation did not store already) ----
    if (!fused) {
        const int npair = p_out * (p_out + 1) / 2;
        for (int idx = tid; idx < npair * kBT; idx += kThreads) {
            const int t = idx & 15, p = idx >> 4;
            if (t >= nt) continue;
            const int nm = L.nm[p], n = nm >> 5, m = nm & 31;
            R2 *dp = reinterpret_cast<R2 *>(aout + L.ooff[t] + 2 * p);
            const double2 v = lds2(X + xe(p, t));
            double re = v.x, im = m ? v.y : 0.0;
            const int bad = L.bad[t];
            const bool ident = bad == 1 && OP != OP_M2L;
            if (bad) {
                if (ident) {  // zero shift of M2M / L2L: identity, truncated / zero-padded
                    const bool keep = n < p_in;
                    re = keep ? (double)ain[L.ioff[t] + 2 * p] : 0.0;
                    im = (keep && m) ? (double)ain[L.ioff[t] + 2 * p + 1] : 0.0;
                } else {
                    re = im = __builtin_nan("");
                    if (p == 0) raise_device_error(err, -3);
                }
            }
            if (acc_out && (!bad || ident)) {
                const R2 old = *dp;
                re += (double)old.x;
                if (m) im += (double)old.y;
            }
            R2 w;
            w.x = (Real)re;
            w.y = (Real)im;
            *dp = w;
        }
    }
    __syncthreads();
}

// Batched form: translation i = 16 b + t of the call.
template <typename Real, int OP, bool IDX, int NW>
__global__ __launch_bounds__(64 * NW, 2) void k_big(DevTables tab, TransArgs a)
{
    extern __shared__ double sm[];
    const int PM = a.p_in > a.p_out ? a.p_in : a.p_out;
    const BigLds L = big_lds(sm, PM);
    const Real *ain = reinterpret_cast<const Real *>(a.in);
    Real *aout = reinterpret_cast<Real *>(a.out);
    const Real *rr = reinterpret_cast<const Real *>(a.r);
    fill_pair_table(L);
    const int64_t nblk = (a.count + kBT - 1) / kBT;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t first = blk * kBT;
        const int nt = (int)((a.count - first) < kBT ? (a.count - first) : kBT);
        if (threadIdx.x < kBT) {
            const int t = threadIdx.x;
            const int64_t i = first + (t < nt ? t : nt - 1);
            const int64_t si = IDX ? a.src[i] : i, di = IDX ? a.dst[i] : i;
            L.ioff[t] = si * a.ld_in;
            L.ooff[t] = di * a.ld_out;
            L.r[3 * t] = (double)rr[3 * i];
            L.r[3 * t + 1] = (double)rr[3 * i + 1];
            L.r[3 * t + 2] = (double)rr[3 * i + 2];
        }
        __syncthreads();
        big_block<Real, OP, NW>(tab, L, a.p_in, a.p_out, nt, ain, aout, (a.flags & 1u) != 0, a.err);
    }
}

template <typename Real, int OP, bool IDX, int NW>
hipError_t launch_big_nw(const DevTables &tab, const TransArgs &a, hipStream_t s)
{
    constexpr int kThreads = 64 * NW;
    const int PM = a.p_in > a.p_out ? a.p_in : a.p_out;
    const size_t smem = big_lds_doubles(PM) * sizeof(double);
    const void *fn = reinterpret_cast<const void *>(&k_big<Real, OP, IDX, NW>);
    int dev = 0, cu = 256, occ = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kThreads, smem) != hipSuccess || occ < 1) occ = 1;
    const int64_t nblk = (a.count + kBT - 1) / kBT;
    const int64_t res = (int64_t)cu * occ;
    const dim3 grid((unsigned)(nblk < res ? nblk : res)), block(kThreads);
    hipLaunchKernelGGL((k_big<Real, OP, IDX, NW>), grid, block, smem, s, tab, a);
    return hipGetLastError();
}

// Two workgroups of 4 wavefronts per CU where two blocks' LDS fit, else one of 8.
__host__ __device__ constexpr bool big_two_per_cu(int PM) { return 2 * big_lds_doubles(PM) * sizeof(double) <= kLdsPerCu; }

template <typename Real, int OP, bool IDX>
hipError_t launch_big_one(const DevTables &tab, const TransArgs &a, hipStream_t s)
{
    const int PM = a.p_in > a.p_out ? a.p_in : a.p_out;
    return big_two_per_cu(PM) ? launch_big_nw<Real, OP, IDX, 4>(tab, a, s) : launch_big_nw<Real, OP, IDX, 8>(tab, a, s);
}

template <typename Real, bool IDX>
hipError_t launch_big_op(const DevTables &tab, const TransArgs &a, hipStream_t s)
{
    if (a.op == OP_M2M) return launch_big_one<Real, OP_M2M, IDX>(tab, a, s);
    if (a.op == OP_M2L) return launch_big_one<Real, OP_M2L, IDX>(tab, a, s);
    return launch_big_one<Real, OP_L2L, IDX>(tab, a, s);
}

// Work-list form: one task (up to 16 items of one operation sharing (p_in, p_out)) per
// workgroup pass; the LDS is sized for the bin's largest order.
template <typename Real, int OP, int NW>
__global__ __launch_bounds__(64 * NW, 2) void k_big_list(DevTables tab, ListArgs la)
{
    extern __shared__ double sm[];
    const Real *ain = reinterpret_cast<const Real *>(la.arena_in);
    Real *aout = reinterpret_cast<Real *>(la.arena_out);
    fill_pair_table(big_lds(sm, 2));
    for (int64_t task = blockIdx.x; task < la.ntasks; task += gridDim.x) {
        const ListTask tk = la.tasks[task];
        const int p_in = tk.p_in, p_out = tk.p_out, nt = tk.count;
        const BigLds L = big_lds(sm, p_in > p_out ? p_in : p_out);
        if (threadIdx.x < kBT) {
            const int t = threadIdx.x;
            const ListItem &it = la.items[tk.first + (t < nt ? t : nt - 1)];
            L.ioff[t] = it.in_off;
            L.ooff[t] = it.out_off;
            L.r[3 * t] = it.r[0];
            L.r[3 * t + 1] = it.r[1];
            L.r[3 * t + 2] = it.r[2];
        }
        __syncthreads();
        big_block<Real, OP, NW>(tab, L, p_in, p_out, nt, ain, aout, (la.flags & 1u) != 0, la.err);
    }
}

template <typename Real, int OP, int NW>
hipError_t launch_big_list_nw(const DevTables &tab, const ListArgs &la, int pmax, hipStream_t s)
{
    constexpr int kThreads = 64 * NW;
    const size_t smem = big_lds_doubles(pmax) * sizeof(double);
    const void *fn = reinterpret_cast<const void *>(&k_big_list<Real, OP, NW>);
    int dev = 0, cu = 256, occ = 1;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kThreads, smem) != hipSuccess || occ < 1) occ = 1;
    const int64_t res = (int64_t)cu * occ;
    const dim3 grid((unsigned)(la.ntasks < res ? la.ntasks : res)), block(kThreads);
    hipLaunchKernelGGL((k_big_list<Real, OP, NW>), grid, block, smem, s, tab, la);
    return hipGetLastError();
}

// workgroups of 4 wavefronts (two per CU) where asked for and two blocks' LDS fit, else of 8
template <typename Real, int OP>
hipError_t launch_big_list_one(const DevTables &tab, const ListArgs &la, int pmax, int nw, hipStream_t s)
{
    return nw == 4 && big_two_per_cu(pmax) ? launch_big_list_nw<Real, OP, 4>(tab, la, pmax, s)
                                           : launch_big_list_nw<Real, OP, 8>(tab, la, pmax, s);
}

template <typename Real>
hipError_t launch_big_list_op(const DevTables &tab, const ListArgs &la, int op, int pmax, int nw, hipStream_t s)
{
    if (op == OP_M2M) return launch_big_list_one<Real, OP_M2M>(tab, la, pmax, nw, s);
    if (op == OP_M2L) return launch_big_list_one<Real, OP_M2L>(tab, la, pmax, nw, s);
    return launch_big_list_one<Real, OP_L2L>(tab, la, pmax, nw, s);
}

}  // namespace

hipError_t launch_list_big(const DevTables &tab, const ListArgs &la, int op, bool f32, int pmax, int nw, hipStream_t s)
{
    if (la.ntasks <= 0) return hipSuccess;
    if (pmax < 1 || pmax >= kBigOrder) return hipErrorInvalidValue;
    return f32 ? launch_big_list_op<float>(tab, la, op, pmax, nw, s)
               : launch_big_list_op<double>(tab, la, op, pmax, nw, s);
}

bool big_list_two_per_cu(int pmax) { return pmax >= 1 && pmax < kBigOrder && big_two_per_cu(pmax); }

bool big_available(int p_in, int p_out)
{
    const int PM = p_in > p_out ? p_in : p_out;
    return PM >= 2 && PM < kBigOrder && big_lds_doubles(PM) * sizeof(double) <= 160 * 1024;
}

size_t big_lds_bytes(int PM) { return big_lds_doubles(PM) * sizeof(double); }

hipError_t launch_big(const DevTables &tab, const TransArgs &a, bool f32, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    const bool idx = a.src != nullptr;
    if (f32) return idx ? launch_big_op<float, true>(tab, a, s) : launch_big_op<float, false>(tab, a, s);
    return idx ? launch_big_op<double, true>(tab, a, s) : launch_big_op<double, false>(tab, a, s);
}

}  // namespace shfmm
