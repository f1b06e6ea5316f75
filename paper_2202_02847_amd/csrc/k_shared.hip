// Shared-shift translations on the matrix cores.
//
// For translations that share one shift vector (the fixed offsets of a uniform octree level:
// 316 M2L offsets, 8 parent/child offsets) every step of the rotation scheme of Section 3.4
// (scalings, z-rotations, swaps, z-translation) is the same linear map, so the translation
// of the whole class is one real matrix T_c (p_out(p_out+1) x p_in(p_in+1)) in the
// normalised basis, applied to every solid of the class: a dense contraction.  The
// operators are generated on the device in FP64 (the rotation kernels applied to unit
// solids), split into BF16 pieces, and applied by a grouped GEMM on MFMA with FP32
// accumulation:
//   x3: a_hi b_hi + a_hi b_mid + a_mid b_hi          (about 16 significant bits)
//   x6: x3 + a_hi b_lo + a_mid b_mid + a_lo b_hi       (about FP32 accuracy)
// where a = a_hi + a_mid + a_lo is the FP32 input and b the FP64 operator entry, each piece
// a BF16 number (8 significant bits).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace shfmm {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest even; Inf and NaN stay Inf and NaN
__device__ __forceinline__ unsigned short bf16_bits(float x)
{
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

constexpr int kTM = 64;    // translations per work item (4 MFMA row tiles)
constexpr int kKC = 128;   // K (input reals) per LDS chunk
constexpr int kNTW = 5;    // output tiles of 16 per wavefront and work item
constexpr int kNTC = 4 * kNTW;
constexpr int kMaxClasses = 4096;
constexpr int kMaxK = 64 * 65 + 32;  // input reals of order 64, padded
constexpr int kMaxN = 64 * 65;       // output reals of order 64

// ---------------------------------------------------------------------------------------
// Operator preparation: T_raw[c][k][n] (FP64, paper basis, row k = image of unit solid k)
// -> normalised entries split into BF16 pieces, stored in B-operand fragment order:
// frag[c][piece][nt][ks][lane][j] holds B[k][n] with k = 32 ks + 8 (lane / 16) + j and
// n = 16 nt + lane % 16 (zero outside k < K, n < N).
// ---------------------------------------------------------------------------------------
__global__ void k_shared_prep(const double *__restrict__ traw, int64_t nclass, int K, int N, int KS, int NT,
                              int npieces, const double *__restrict__ s_in, const double *__restrict__ s_out,
                              unsigned short *__restrict__ frag)
{
    const int64_t per_class = (int64_t)NT * KS * 64 * 8;
    const int64_t total = nclass * per_class;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / per_class;
        int64_t rest = e - c * per_class;
        const int j = (int)(rest & 7);
        const int lane = (int)((rest >> 3) & 63);
        rest >>= 9;
        const int ks = (int)(rest % KS);
        const int nt = (int)(rest / KS);
        const int k = 32 * ks + 8 * (lane >> 4) + j;
        const int n = 16 * nt + (lane & 15);
        double t = 0.0;
        if (k < K && n < N) t = traw[(c * K + k) * N + n] * s_out[n] / s_in[k];
        unsigned short p[3];
        double rem = t;
        for (int q = 0; q < 3; ++q) {
            p[q] = bf16_bits((float)rem);
            rem -= (double)bf16_value(p[q]);
        }
        const int64_t slot = ((int64_t)nt * KS + ks) * 512 + lane * 8 + j;
        for (int q = 0; q < npieces; ++q) frag[(c * npieces + q) * per_class + slot] = p[q];
    }
}

// FP32 operator fragments for the 16x16x4 FP32 MFMA: frag[c][nt][ks][lane][j] holds B[k][n]
// with k = 32 ks + 4 j + lane / 16 and n = 16 nt + lane % 16 (a lane's 8 values of a 32-wide K
// block are contiguous), rounded once from the FP64 image.
__global__ void k_shared_prep_f32(const double *__restrict__ traw, int64_t nclass, int K, int N, int KS, int NT,
                                  const double *__restrict__ s_in, const double *__restrict__ s_out,
                                  float *__restrict__ frag)
{
    const int64_t per_class = (int64_t)NT * KS * 512;
    const int64_t total = nclass * per_class;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / per_class;
        int64_t rest = e - c * per_class;
        const int j = (int)(rest & 7);
        const int lane = (int)((rest >> 3) & 63);
        rest >>= 9;
        const int ks = (int)(rest % KS);
        const int nt = (int)(rest / KS);
        const int k = 32 * ks + 4 * j + (lane >> 4);
        const int n = 16 * nt + (lane & 15);
        double t = 0.0;
        if (k < K && n < N) t = traw[(c * K + k) * N + n] * s_out[n] / s_in[k];
        frag[e] = (float)t;
    }
}

// ---------------------------------------------------------------------------------------
// Grouped GEMM.  Work item = (class c, 64 consecutive translations of c, a chunk of up to
// 20 output tiles of 16).  The FP32 input rows of the 64 translations are split into BF16
// pieces once per K chunk of 128 and staged in LDS; wavefront w owns output tiles
// w, w + 4, ..., w + 16 of the chunk and multiplies them with the operator fragments, read
// from global memory (L2-resident: shared by every work item of the class) one K step ahead.
// The MFMAs are issued product by product over 20 independent accumulators.
// ---------------------------------------------------------------------------------------
template <int PREC>
__global__ __launch_bounds__(256, 2) void k_shared_gemm(SharedArgs a)
{
    constexpr int NPB = PREC == 6 ? 3 : 2;   // operator pieces
    constexpr int NPA = PREC == 6 ? 3 : 2;   // input pieces
    __shared__ s16x8 Ap[NPA][kTM][kKC / 8 + 1];   // BF16 pieces, rows padded by one 16-byte slot
    __shared__ int tiles_before[kMaxClasses + 1];
    __shared__ unsigned char live[kMaxK];
    __shared__ unsigned char live_o[kMaxN];
    const int tid = threadIdx.x, lane = tid & 63;
    for (int k = tid; k < a.Kp; k += 256) live[k] = a.live_in[k];
    for (int n = tid; n < a.N; n += 256) live_o[n] = a.live_out[n];
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nclass = a.nclass;
    const int64_t count = a.count;

    // work items per class: ceil(rows / 64) x N chunks (prefix sum in LDS)
    const int nchunks = (a.NT + kNTC - 1) / kNTC;
    if (wave == 0) {
        int carry = 0;
        for (int c0 = 0; c0 < nclass; c0 += 64) {
            const int c = c0 + lane;
            int v = 0;
            if (c < nclass) {
                int64_t s0 = a.class_start[c], s1 = a.class_start[c + 1];
                s0 = s0 < 0 ? 0 : (s0 > count ? count : s0);
                s1 = s1 < s0 ? s0 : (s1 > count ? count : s1);
                v = (int)((s1 - s0 + kTM - 1) / kTM) * nchunks;
            }
            for (int d = 1; d < 64; d <<= 1) {
                const int u = __shfl_up(v, d);
                if (lane >= d) v += u;
            }
            if (c < nclass) tiles_before[c + 1] = carry + v;
            carry += __shfl(v, 63);
        }
        if (lane == 0) tiles_before[0] = 0;
    }
    __syncthreads();
    const int total = tiles_before[nclass];

    // XCD-aware walk: workgroups are dealt to the 8 XCDs in turn (blockIdx % 8), and each
    // XCD takes a contiguous eighth of the work items, so that the few classes it works on at
    // a time keep their operators in its own L2 (the grid is a multiple of 8)
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, per_xcd = gridDim.x >> 3;
    const int w_end = (int)(((int64_t)total * (xcd + 1)) >> 3);
    for (int w = (int)(((int64_t)total * xcd) >> 3) + slot; w < w_end; w += per_xcd) {
        int lo = 0, hi = nclass - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tiles_before[mid] <= w) lo = mid; else hi = mid - 1;
        }
        const int c = lo;
        const int local = w - tiles_before[c];
        const int mtile = local / nchunks, chunk = local - mtile * nchunks;
        int64_t s0 = a.class_start[c], s1 = a.class_start[c + 1];
        s0 = s0 < 0 ? 0 : (s0 > count ? count : s0);
        s1 = s1 < s0 ? s0 : (s1 > count ? count : s1);
        const int64_t first = s0 + (int64_t)mtile * kTM;
        const int rows = (int)((s1 - first) < kTM ? (s1 - first) : kTM);
        const int nt0 = chunk * kNTC;
        // this wave's output tiles (tiles past the end re-read the last one; not stored)
        const unsigned short *bbase =
            reinterpret_cast<const unsigned short *>(a.frag) + (int64_t)c * NPB * a.frag_class_stride + lane * 8;
        int toff[kNTW];  // wave-uniform offsets of this wave's output tiles
#pragma unroll
        for (int i = 0; i < kNTW; ++i) {
            const int nt = nt0 + wave + 4 * i;
            const int ntc = nt < a.NT ? nt : a.NT - 1;
            toff[i] = __builtin_amdgcn_readfirstlane(ntc * a.KS * 512);
        }
        const bool last_tile = nt0 + wave + 4 * (kNTW - 1) < a.NT;

        f32x4 acc[4][kNTW];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int t = 0; t < kNTW; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};

        // operator fragments of K step 0
        s16x8 bcur[kNTW][NPB];
#pragma unroll
        for (int i = 0; i < kNTW; ++i)
#pragma unroll
            for (int q = 0; q < NPB; ++q)
                bcur[i][q] = *reinterpret_cast<const s16x8 *>(bbase + toff[i] + q * a.frag_class_stride);

        for (int kc = 0; kc < a.Kp; kc += kKC) {
            const int kw = (a.Kp - kc) < kKC ? (a.Kp - kc) : kKC;  // multiple of 32
            // split 64 input rows x kw reals into BF16 pieces in LDS (8 reals per thread step;
            // rows past the class re-read its last row)
            __syncthreads();
            // every load of the chunk is issued before the first is used (one memory latency
            // per chunk); addresses are clamped into the solid, and the padding and Im C_n^0
            // entries are zeroed by the live flags
            constexpr int IT = kTM * (kKC / 8) / 256;
            const int lim = kTM * (kw / 8);
            float x[IT][8];
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int p0 = tid + 256 * it;
                const int p = p0 < lim ? p0 : lim - 1;
                const int t = p / (kw / 8);
                const int k = kc + 8 * (p - t * (kw / 8));
                const int64_t row = first + (t < rows ? t : rows - 1);
#pragma unroll
                for (int j = 0; j < 8; j += 2) {
                    const int kk = k + j < a.K ? k + j : a.K - 2;
                    const float2 v = *reinterpret_cast<const float2 *>(a.in + row * a.ld_in + kk);
                    x[it][j] = v.x;
                    x[it][j + 1] = v.y;
                }
            }
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int p = tid + 256 * it;
                if (p >= lim) break;
                const int t = p / (kw / 8);
                const int k8 = p - t * (kw / 8);
                const int k = kc + 8 * k8;
#pragma unroll
                for (int j = 0; j < 8; ++j) x[it][j] = live[k + j] ? x[it][j] : 0.f;
                s16x8 h, m, l;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const __bf16 hb = (__bf16)x[it][j];  // v_cvt_pk_bf16_f32: round to nearest even
                    const float r1 = x[it][j] - (float)hb;
                    const __bf16 mb = (__bf16)r1;
                    h[j] = __builtin_bit_cast(short, hb);
                    m[j] = __builtin_bit_cast(short, mb);
                    if (NPA == 3) l[j] = __builtin_bit_cast(short, (__bf16)(r1 - (float)mb));
                }
                Ap[0][t][k8] = h;
                Ap[1][t][k8] = m;
                if (NPA == 3) Ap[NPA - 1][t][k8] = l;
            }
            __syncthreads();
            for (int ks = 0; ks < kw / 32; ++ks) {
                const int kglob = (kc >> 5) + ks;
                const int knext = kglob + 1 < a.KS ? kglob + 1 : kglob;
                // input fragments: row 16 mt + lane % 16, k = 32 ks + 8 (lane / 16) + j; the high
                // piece stays in registers for the step, the others pass through one slot
                auto load_a = [&](int q, s16x8 (&f)[4]) {
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt) f[mt] = Ap[q][mt * 16 + (lane & 15)][4 * ks + (lane >> 4)];
                };
                s16x8 ahi[4], ax[4];
                load_a(0, ahi);
                load_a(1, ax);
                // one product (input fragments f x operator piece pb) over the 4 x 5 output blocks
                auto mma = [&](const s16x8 (&f)[4], int pb) {
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                        for (int i = 0; i < kNTW - 1; ++i)
                            acc[mt][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf16x8, f[mt]), __builtin_bit_cast(bf16x8, bcur[i][pb]),
                                acc[mt][i], 0, 0, 0);
                    if (last_tile) {  // wave-uniform: this wave's fifth output tile exists
#pragma unroll
                        for (int mt = 0; mt < 4; ++mt)
                            acc[mt][kNTW - 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf16x8, f[mt]), __builtin_bit_cast(bf16x8, bcur[kNTW - 1][pb]),
                                acc[mt][kNTW - 1], 0, 0, 0);
                    }
                };
                // the next K step's operator piece q is loaded right after its last use here, so
                // the loads fly during the remaining products
                auto fetch = [&](int q) {
#pragma unroll
                    for (int i = 0; i < kNTW; ++i)
                        bcur[i][q] = *reinterpret_cast<const s16x8 *>(bbase + toff[i] + q * a.frag_class_stride +
                                                                      knext * 512);
                };
                if (PREC == 6) {
                    mma(ahi, 2);  // a_hi b_lo
                    fetch(2);
                }
                mma(ahi, 1);      // a_hi b_mid
                mma(ahi, 0);      // a_hi b_hi
                if (PREC == 6) mma(ax, 1);  // a_mid b_mid
                fetch(1);
                mma(ax, 0);       // a_mid b_hi
                if (PREC == 6) {
                    load_a(2, ax);
                    mma(ax, 0);   // a_lo b_hi
                }
                fetch(0);
            }
        }
        // store: D row (translation) 16 mt + 4 (lane / 16) + j, column (output) 16 nt + lane % 16
        const bool accumulate = (a.flags & 1u) != 0;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
            for (int i = 0; i < kNTW; ++i) {
                const int n = (nt0 + wave + 4 * i) * 16 + (lane & 15);
                if (n >= a.N) continue;
                const bool live = live_o[n] != 0;  // from LDS: a global load here would wait
                                                   // for every store issued before it
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int t = mt * 16 + 4 * (lane >> 4) + j;
                    if (t >= rows) continue;
                    float *o = a.out + (first + t) * a.ld_out + n;
                    float v = live ? acc[mt][i][j] : 0.f;
                    if (accumulate && live) v += *o;
                    *o = v;
                }
            }
        }
    }
}

// FP32 form of the grouped GEMM (v_mfma_f32_16x16x4f32, FP32 operands and accumulation): the
// same work items and walk as above; inputs staged in LDS as FP32 with each lane's 8 values of
// a 32-wide K block contiguous (As[t][ks][g][j], k = 32 ks + 4 j + g).
__global__ __launch_bounds__(256, 2) void k_shared_gemm_f32(SharedArgs a)
{
    constexpr int KB = kKC / 32;  // 32-wide K blocks per LDS chunk
    __shared__ float As[kTM][KB][4][8 + 1];  // row padded so that lanes of one row avoid a bank
    __shared__ int tiles_before[kMaxClasses + 1];
    __shared__ unsigned char live[kMaxK];
    __shared__ unsigned char live_o[kMaxN];
    typedef float f8 __attribute__((ext_vector_type(8)));
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nclass = a.nclass;
    const int64_t count = a.count;
    const float *frag = reinterpret_cast<const float *>(a.frag);
    for (int k = tid; k < a.Kp; k += 256) live[k] = a.live_in[k];
    for (int n = tid; n < a.N; n += 256) live_o[n] = a.live_out[n];
    const int nchunks = (a.NT + kNTC - 1) / kNTC;
    if (wave == 0) {
        int carry = 0;
        for (int c0 = 0; c0 < nclass; c0 += 64) {
            const int c = c0 + lane;
            int v = 0;
            if (c < nclass) {
                int64_t s0 = a.class_start[c], s1 = a.class_start[c + 1];
                s0 = s0 < 0 ? 0 : (s0 > count ? count : s0);
                s1 = s1 < s0 ? s0 : (s1 > count ? count : s1);
                v = (int)((s1 - s0 + kTM - 1) / kTM) * nchunks;
            }
            for (int d = 1; d < 64; d <<= 1) {
                const int u = __shfl_up(v, d);
                if (lane >= d) v += u;
            }
            if (c < nclass) tiles_before[c + 1] = carry + v;
            carry += __shfl(v, 63);
        }
        if (lane == 0) tiles_before[0] = 0;
    }
    __syncthreads();
    const int total = tiles_before[nclass];
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, per_xcd = gridDim.x >> 3;
    const int w_end = (int)(((int64_t)total * (xcd + 1)) >> 3);
    for (int w = (int)(((int64_t)total * xcd) >> 3) + slot; w < w_end; w += per_xcd) {
        int lo = 0, hi = nclass - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tiles_before[mid] <= w) lo = mid; else hi = mid - 1;
        }
        const int c = lo;
        const int local = w - tiles_before[c];
        const int mtile = local / nchunks, chunk = local - mtile * nchunks;
        int64_t s0 = a.class_start[c], s1 = a.class_start[c + 1];
        s0 = s0 < 0 ? 0 : (s0 > count ? count : s0);
        s1 = s1 < s0 ? s0 : (s1 > count ? count : s1);
        const int64_t first = s0 + (int64_t)mtile * kTM;
        const int rows = (int)((s1 - first) < kTM ? (s1 - first) : kTM);
        const int nt0 = chunk * kNTC;
        const float *bbase = frag + (int64_t)c * a.frag_class_stride + lane * 8;
        int toff[kNTW];
#pragma unroll
        for (int i = 0; i < kNTW; ++i) {
            const int nt = nt0 + wave + 4 * i;
            const int ntc = nt < a.NT ? nt : a.NT - 1;
            toff[i] = __builtin_amdgcn_readfirstlane(ntc * a.KS * 512);
        }
        const bool last_tile = nt0 + wave + 4 * (kNTW - 1) < a.NT;
        f32x4 acc[4][kNTW];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int t = 0; t < kNTW; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int kc = 0; kc < a.Kp; kc += kKC) {
            const int kw = (a.Kp - kc) < kKC ? (a.Kp - kc) : kKC;
            __syncthreads();
            // every load of the chunk first (one memory latency per chunk), addresses clamped
            // into the solid, padding and Im C_n^0 zeroed by the live flags
            constexpr int IT = kTM * (kKC / 2) / 256;
            const int lim = kTM * (kw / 2);
            float2 xv[IT];
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int p0 = tid + 256 * it;
                const int p = p0 < lim ? p0 : lim - 1;
                const int t = p / (kw / 2);
                const int k = kc + 2 * (p - t * (kw / 2));
                const int64_t row = first + (t < rows ? t : rows - 1);
                xv[it] = *reinterpret_cast<const float2 *>(a.in + row * a.ld_in + (k < a.K ? k : a.K - 2));
            }
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int p = tid + 256 * it;
                if (p >= lim) break;
                const int t = p / (kw / 2);
                const int k = kc + 2 * (p - t * (kw / 2));
                const int r0 = k - kc, r1 = r0 + 1;
                As[t][r0 >> 5][r0 & 3][(r0 & 31) >> 2] = live[k] ? xv[it].x : 0.f;
                As[t][r1 >> 5][r1 & 3][(r1 & 31) >> 2] = live[k + 1] ? xv[it].y : 0.f;
            }
            __syncthreads();
            for (int kb = 0; kb < kw / 32; ++kb) {
                const int kglob = (kc >> 5) + kb;
                f8 b[kNTW];
#pragma unroll
                for (int i = 0; i < kNTW; ++i) b[i] = *reinterpret_cast<const f8 *>(bbase + toff[i] + kglob * 512);
                float av[4][8];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int j = 0; j < 8; ++j) av[mt][j] = As[mt * 16 + (lane & 15)][kb][lane >> 4][j];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                        for (int i = 0; i < kNTW - 1; ++i)
                            acc[mt][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt][j], b[i][j], acc[mt][i], 0, 0, 0);
                    if (last_tile) {
#pragma unroll
                        for (int mt = 0; mt < 4; ++mt)
                            acc[mt][kNTW - 1] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt][j], b[kNTW - 1][j], acc[mt][kNTW - 1], 0, 0, 0);
                    }
                }
            }
        }
        const bool accumulate = (a.flags & 1u) != 0;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
            for (int i = 0; i < kNTW; ++i) {
                const int n = (nt0 + wave + 4 * i) * 16 + (lane & 15);
                if (n >= a.N) continue;
                const bool live_n = live_o[n] != 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int t = mt * 16 + 4 * (lane >> 4) + j;
                    if (t >= rows) continue;
                    float *o = a.out + (first + t) * a.ld_out + n;
                    float v = live_n ? acc[mt][i][j] : 0.f;
                    if (accumulate && live_n) v += *o;
                    *o = v;
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_shared_prep_f32(const double *traw, int64_t nclass, int K, int N, int KS, int NT,
                                  const double *s_in, const double *s_out, float *frag, hipStream_t s)
{
    const int64_t total = nclass * (int64_t)NT * KS * 512;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_shared_prep_f32, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, traw,
                       nclass, K, N, KS, NT, s_in, s_out, frag);
    return hipGetLastError();
}

hipError_t launch_shared_prep(const double *traw, int64_t nclass, int K, int N, int KS, int NT, int npieces,
                              const double *s_in, const double *s_out, unsigned short *frag, hipStream_t s)
{
    const int64_t total = nclass * (int64_t)NT * KS * 512;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_shared_prep, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, traw,
                       nclass, K, N, KS, NT, npieces, s_in, s_out, frag);
    return hipGetLastError();
}

int shared_max_classes() { return kMaxClasses; }

hipError_t launch_shared_gemm(const SharedArgs &a, int prec, hipStream_t s)
{
    if (a.count <= 0 || a.nclass <= 0) return hipSuccess;
    const void *fn = prec == 6   ? reinterpret_cast<const void *>(&k_shared_gemm<6>)
                     : prec == 3 ? reinterpret_cast<const void *>(&k_shared_gemm<3>)
                                 : reinterpret_cast<const void *>(&k_shared_gemm_f32);
    const int res = lpt::resident_workgroups(fn);
    // enough work items for the whole batch, capped at the resident count (persistent loop)
    const int nchunks = (a.NT + kNTC - 1) / kNTC;
    const int64_t upper = ((a.count + kTM - 1) / kTM + a.nclass) * nchunks;
    int64_t g = upper < res ? upper : res;
    g = (g + 7) / 8 * 8;  // a multiple of the XCD count (the kernel's walk assumes it)
    const dim3 grid((unsigned)g), block(256);
    if (prec == 6)
        hipLaunchKernelGGL(k_shared_gemm<6>, grid, block, 0, s, a);
    else if (prec == 3)
        hipLaunchKernelGGL(k_shared_gemm<3>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(k_shared_gemm_f32, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace shfmm
