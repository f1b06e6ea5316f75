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
#include <type_traits>

#include "kernels.hpp"

namespace shfmm {

namespace {

constexpr int kLptMaxOrder = 16;

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Greedy static schedule: items (rows or columns) sorted by cost, each given to the
// least-loaded of the 4 wavefronts.  cost(i) ~ (i+1)^2 for rows, (P-m)^2 for columns.
constexpr int row_owner(int P, int n)
{
    long load[4] = {0, 0, 0, 0};
    int own = 0;
    for (int k = P - 1; k >= 0; --k) {
        int w = 0;
        for (int j = 1; j < 4; ++j)
            if (load[j] < load[w]) w = j;
        load[w] += (long)(k + 1) * (k + 1);
        if (k == n) own = w;
    }
    return own;
}

constexpr int col_owner(int PIN, int POUT, int m)
{
    long load[4] = {0, 0, 0, 0};
    int own = 0;
    const int PM = PIN > POUT ? PIN : POUT;
    for (int k = 0; k < PM; ++k) {
        int w = 0;
        for (int j = 1; j < 4; ++j)
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

// Powers of the two rotations for one translation (lane), m = 0..PM-1.
template <typename Acc, int PM>
struct Powers {
    Acc ca[PM], sa[PM], cb[PM], sb[PM];
};

// y = T x for row n of the swap tables (F/G or FL/GL): Re by T_re, Im by T_im.
// Entries with m + l + n odd (Re) / even (Im) are zero and skipped at compile time.
template <typename Acc, int N>
__device__ __forceinline__ void swap_row(cptr<Acc> Tre, cptr<Acc> Tim,
                                         const Acc (&xr)[N + 1], const Acc (&xi)[N + 1],
                                         Acc (&yr)[N + 1], Acc (&yi)[N + 1])
{
    constexpr int off = swap_off(N);
#pragma unroll
    for (int m = 0; m <= N; ++m) {
        Acc ar = 0, ai = 0;
#pragma unroll
        for (int l = 0; l <= N; ++l) {
            if ((m + l + N) % 2 == 0)
                ar += Tre[off + m * (N + 1) + l] * xr[l];
            else if (m > 0 && l > 0)
                ai += Tim[off + m * (N + 1) + l] * xi[l];
        }
        yr[m] = ar;
        yi[m] = ai;
    }
}

// x <- x * (c + i sgn s)
template <typename Acc, int N, int PM>
__device__ __forceinline__ void zrot_row(Acc (&xr)[N + 1], Acc (&xi)[N + 1], const Acc (&c)[PM],
                                         const Acc (&s)[PM], Acc sgn)
{
#pragma unroll
    for (int m = 1; m <= N; ++m) {
        const Acc a = xr[m], b = xi[m], cs = c[m], sn = sgn * s[m];
        xr[m] = a * cs - b * sn;
        xi[m] = a * sn + b * cs;
    }
}

template <typename Acc>
__device__ __forceinline__ Acc ipow(Acc x, int e)
{
    Acc r = 1;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

template <typename Real, typename Acc, int OP, int PIN, int POUT>
__global__ __launch_bounds__(256, 2) void k_lpt(DevTables tab, TransArgs a)
{
    constexpr int PM = PIN > POUT ? PIN : POUT;
    constexpr int SIN = PIN * (PIN + 1), SOUT = POUT * (POUT + 1);
    constexpr int S = PM * (PM + 1);
    constexpr int SP = (S % 4 == 2) ? S : S + 2;  // padded row: conflict-free pair access
    using P2 = typename Pair<Acc>::T;
    using R2 = typename Pair<Real>::T;
    __shared__ Acc X[64 * SP];
    __shared__ int bad[64];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    using T = Tab<Real, Acc>;
    constexpr int fw = (OP == OP_L2L) ? SW_FL : SW_F;
    constexpr int bw = (OP == OP_M2M) ? SW_F : SW_FL;
    const cptr<Acc> Ffw = as_const(T::swap(tab, fw));
    const cptr<Acc> Gfw = as_const(T::swap(tab, fw + 1));
    const cptr<Acc> Fbw = as_const(T::swap(tab, bw));
    const cptr<Acc> Gbw = as_const(T::swap(tab, bw + 1));
    const cptr<Acc> Z = as_const(T::z(tab, OP));
    const Real *__restrict__ rr = reinterpret_cast<const Real *>(a.r);
    const Real *__restrict__ gin = reinterpret_cast<const Real *>(a.in);
    Real *__restrict__ gout = reinterpret_cast<Real *>(a.out);
    const bool acc = (a.flags & 1u) != 0;
    const int64_t nblk = (a.count + 63) / 64;

    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t base = blk * 64;
        const int nt = (int)((a.count - base) < 64 ? (a.count - base) : 64);

        // ---- coalesced load of the block's input solids into LDS ----
        for (int p = tid; p < nt * (SIN / 2); p += 256) {
            const int t = p / (SIN / 2);
            const int k = 2 * (p - t * (SIN / 2));
            const int64_t si = a.src ? a.src[base + t] : base + t;
            const R2 v = *reinterpret_cast<const R2 *>(gin + si * a.ld_in + k);
            *reinterpret_cast<P2 *>(&X[t * SP + k]) = P2{(Acc)v.x, (Acc)v.y};
        }

        // ---- per-lane shift geometry (every wavefront, redundantly) ----
        double x = 0.0, y = 0.0, z = 1.0;
        if (lane < nt) {
            x = (double)rr[3 * (base + lane)];
            y = (double)rr[3 * (base + lane) + 1];
            z = (double)rr[3 * (base + lane) + 2];
        }
        const Geometry g = shift_geometry(x, y, z);
        if (wave == 0) bad[lane] = (g.valid == 1) ? 0 : (g.valid == 0 ? 1 : 2);
        Powers<Acc, PM> pw;
        {
            double c1 = 1.0, s1 = 0.0, c2 = 1.0, s2 = 0.0;
#pragma unroll
            for (int m = 0; m < PM; ++m) {
                pw.ca[m] = (Acc)c1;
                pw.sa[m] = (Acc)s1;
                pw.cb[m] = (Acc)c2;
                pw.sb[m] = (Acc)s2;
                const double t1 = c1 * g.ca - s1 * g.sa;
                s1 = c1 * g.sa + s1 * g.ca;
                c1 = t1;
                const double t2 = c2 * g.cb - s2 * g.sb;
                s2 = c2 * g.sb + s2 * g.cb;
                c2 = t2;
            }
        }
        const Acc s = (Acc)(g.valid == 1 ? g.s : 1.0);
        const Acc R = (Acc)(g.valid == 1 ? g.R : 1.0);
        Acc *Xt = X + lane * SP;
        __syncthreads();

        // ---- forward rotation of the input rows ----
        static_for<0, PIN>([&](auto nc) {
            constexpr int n = decltype(nc)::value;
            if (row_owner(PIN, n) != wave) return;
            Acc xr[n + 1], xi[n + 1], yr[n + 1], yi[n + 1];
#pragma unroll
            for (int m = 0; m <= n; ++m) {
                const P2 v = *reinterpret_cast<const P2 *>(&Xt[solid_pos(n, m)]);
                xr[m] = v.x;
                xi[m] = m ? v.y : (Acc)0;
            }
            // scale: M2L/M2M  M_n / |r|^{n+1};  L2L  L_n |r|^n   (eq. scaling)
            const Acc f = (OP == OP_L2L) ? ipow(R, n) : ipow(s, n + 1);
#pragma unroll
            for (int m = 0; m <= n; ++m) {
                xr[m] *= f;
                xi[m] *= f;
            }
            zrot_row<Acc, n, PM>(xr, xi, pw.ca, pw.sa, (Acc)1);
            swap_row<Acc, n>(Ffw, Gfw, xr, xi, yr, yi);
            zrot_row<Acc, n, PM>(yr, yi, pw.cb, pw.sb, (Acc)1);
            swap_row<Acc, n>(Ffw, Gfw, yr, yi, xr, xi);
#pragma unroll
            for (int m = 0; m <= n; ++m) *reinterpret_cast<P2 *>(&Xt[solid_pos(n, m)]) = P2{xr[m], xi[m]};
        });
        __syncthreads();

        // ---- z-axis step, one column (order m) at a time, unit shift ----
        static_for<0, POUT>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            if (col_owner(PIN, POUT, m) != wave) return;
            if constexpr (m >= PIN) {
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
                constexpr int64_t zb = z_col_off(kZTableOrder, m);
#pragma unroll
                for (int o = m; o < POUT; ++o) {
                    Acc orr = 0, oi = 0;
#pragma unroll
                    for (int k = m; k < PIN; ++k) {
                        if (OP == OP_M2M && k > o) continue;
                        if (OP == OP_L2L && k < o) continue;
                        const Acc c = Z[zb + (int64_t)(o - m) * (kZTableOrder - m) + (k - m)];
                        orr += c * ir[k];
                        oi += c * ii[k];
                    }
                    *reinterpret_cast<P2 *>(&Xt[solid_pos(o, m)]) = P2{orr, oi};
                }
            }
        });
        __syncthreads();

        // ---- backward rotation of the output rows ----
        static_for<0, POUT>([&](auto nc) {
            constexpr int n = decltype(nc)::value;
            if (row_owner(POUT, n) != wave) return;
            Acc xr[n + 1], xi[n + 1], yr[n + 1], yi[n + 1];
#pragma unroll
            for (int m = 0; m <= n; ++m) {
                const P2 v = *reinterpret_cast<const P2 *>(&Xt[solid_pos(n, m)]);
                xr[m] = v.x;
                xi[m] = m ? v.y : (Acc)0;
            }
            swap_row<Acc, n>(Fbw, Gbw, xr, xi, yr, yi);
            zrot_row<Acc, n, PM>(yr, yi, pw.cb, pw.sb, (Acc)-1);
            swap_row<Acc, n>(Fbw, Gbw, yr, yi, xr, xi);
            zrot_row<Acc, n, PM>(xr, xi, pw.ca, pw.sa, (Acc)-1);
            // unscale: M2L/L2L  L_n / |r|^n;  M2M  M_n |r|^{n+1}
            const Acc f = (OP == OP_M2M) ? ipow(R, n + 1) : ipow(s, n);
#pragma unroll
            for (int m = 0; m <= n; ++m)
                *reinterpret_cast<P2 *>(&Xt[solid_pos(n, m)]) = P2{xr[m] * f, m ? xi[m] * f : (Acc)0};
        });
        __syncthreads();

        // ---- coalesced store (overwrite / accumulate); invalid shifts fixed up here ----
        for (int p = tid; p < nt * (SOUT / 2); p += 256) {
            const int t = p / (SOUT / 2);
            const int k = 2 * (p - t * (SOUT / 2));
            const int64_t di = a.dst ? a.dst[base + t] : base + t;
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
                        const int64_t si = a.src ? a.src[base + t] : base + t;
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
        __syncthreads();
    }
}

template <typename Real, typename Acc, int OP>
hipError_t launch_fixed(int P, const DevTables &tab, const TransArgs &a, hipStream_t s)
{
    const int64_t nblk = (a.count + 63) / 64;
    const dim3 grid((unsigned)(nblk < (1 << 20) ? nblk : (1 << 20))), block(256);
    switch (P) {
#define SH_CASE(PV)                                                                        \
    case PV:                                                                               \
        hipLaunchKernelGGL((k_lpt<Real, Acc, OP, PV, PV>), grid, block, 0, s, tab, a);     \
        break;
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
#undef SH_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool lpt_available(int op, bool f32, int p_in, int p_out)
{
    (void)op;
    (void)f32;
    return p_in == p_out && p_in >= 2 && p_in <= 12;
}

hipError_t launch_lpt(const DevTables &tab, const TransArgs &a, bool f32, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    const int P = a.p_in;
    if (f32) {
        if (a.op == OP_M2M) return launch_fixed<float, float, OP_M2M>(P, tab, a, s);
        if (a.op == OP_M2L) return launch_fixed<float, float, OP_M2L>(P, tab, a, s);
        return launch_fixed<float, float, OP_L2L>(P, tab, a, s);
    }
    if (a.op == OP_M2M) return launch_fixed<double, double, OP_M2M>(P, tab, a, s);
    if (a.op == OP_M2L) return launch_fixed<double, double, OP_M2L>(P, tab, a, s);
    return launch_fixed<double, double, OP_L2L>(P, tab, a, s);
}

}  // namespace shfmm
