// General rotation-based translation kernel: one wavefront per translation, any
// input/output orders up to the table order, FP64 (paper basis) or FP32 (normalised
// basis).  Lanes own output coefficients (n, m); the solid lives in LDS.
//
// Steps (Section 3.4, "Summary: The Entire Algorithm"; M2M/L2L by the same skeleton):
//   1. geometry of the shift, powers e^{im a}, e^{im b}, |r|^{+-n} (no trigonometry)
//   2. rows of the input: scale, rotate by a, swap x<->z, rotate by b, swap again
//   3. columns: the z-axis step with unit shift (M2L: Hankel of factorials, eq. zm2l-matrix;
//      M2M/L2L: Toeplitz of 1/j!), signs folded into the coefficient table
//   4. rows of the output: swap, rotate by -b, swap, rotate by -a, unscale, store
// The M-side swap uses F, G; the L-side uses FL, GL (L -> B L of eq. swaptransform).
#include "kernels.hpp"

namespace shfmm {

namespace {

__device__ __forceinline__ int tri_row(int c)
{
    int n = (int)((sqrtf(8.0f * (float)c + 1.0f) - 1.0f) * 0.5f);
    while ((n + 1) * (n + 2) / 2 <= c) ++n;
    while (n * (n + 1) / 2 > c) --n;
    return n;
}

// degree n of the real at index i of a solid (row n occupies [n(n+1), (n+1)(n+2)))
__device__ __forceinline__ int solid_row(int i)
{
    int n = (int)((sqrtf(4.0f * (float)i + 1.0f) - 1.0f) * 0.5f);
    while ((n + 1) * (n + 2) <= i) ++n;
    while (n * (n + 1) > i) --n;
    return n;
}

// y <- swap(x) on rows [0, rows): Re by Tre, Im by Tim (chequerboard: only every other l).
template <typename Real>
__device__ __forceinline__ void swap_rows(const Real *__restrict__ Tre, const Real *__restrict__ Tim,
                                          const Real *x, Real *y, int rows, int lane)
{
    const int tri = rows * (rows + 1) / 2;
    for (int c = lane; c < tri; c += 64) {
        const int n = tri_row(c);
        const int m = c - n * (n + 1) / 2;
        const Real *fr = Tre + swap_off(n) + m * (n + 1);
        const Real *gr = Tim + swap_off(n) + m * (n + 1);
        const Real *xr = x + solid_pos(n, 0);
        Real yre = 0, yim = 0;
        for (int l = (m + n) & 1; l <= n; l += 2) yre += fr[l] * xr[2 * l];
        for (int l = ((m + n) & 1) ^ 1; l <= n; l += 2) yim += gr[l] * xr[2 * l + 1];
        y[solid_pos(n, m)] = yre;
        y[solid_pos(n, m) + 1] = yim;
    }
}

// x <- x * (er + i*sgn*ei)[m] on rows [0, rows)
template <typename Real>
__device__ __forceinline__ void zrot_rows(Real *x, const Real *er, const Real *ei, Real sgn, int rows, int lane)
{
    const int tri = rows * (rows + 1) / 2;
    for (int c = lane; c < tri; c += 64) {
        const int n = tri_row(c);
        const int m = c - n * (n + 1) / 2;
        const Real a = x[solid_pos(n, m)], b = x[solid_pos(n, m) + 1];
        const Real cr = er[m], ci = sgn * ei[m];
        x[solid_pos(n, m)] = a * cr - b * ci;
        x[solid_pos(n, m) + 1] = a * ci + b * cr;
    }
}

// One translation by one wavefront (lanes own output coefficients, the solid in LDS).
// smem: 2 P(P+1) + 6 P reals of type Acc, P = max(p_in, p_out).
// Real: type of the solids and shifts in memory; Acc: arithmetic type (LDS state, tables).
template <typename Real, typename Acc, int OP>
__device__ void general_one(const DevTables &tab, int p_in, int p_out, double rx, double ry, double rz,
                            const Real *in, Real *out, bool acc, int *err, unsigned char *smem_raw,
                            bool single = false)
{
    const int Pm = p_in > p_out ? p_in : p_out;
    const int S = Pm * (Pm + 1);
    Acc *A = reinterpret_cast<Acc *>(smem_raw);
    Acc *B = A + S;
    Acc *ear = B + S;
    Acc *eai = ear + Pm;
    Acc *ebr = eai + Pm;
    Acc *ebi = ebr + Pm;
    Acc *sc_in = ebi + Pm;
    Acc *sc_out = sc_in + Pm;
    const int lane = threadIdx.x;

    const int fw = (OP == OP_L2L) ? SW_FL : SW_F;
    const int bw = (OP == OP_M2M) ? SW_F : SW_FL;
    using T = Tab<Real, Acc>;
    const Acc *Ffw = T::swap(tab, fw), *Gfw = T::swap(tab, fw + 1);
    const Acc *Fbw = T::swap(tab, bw), *Gbw = T::swap(tab, bw + 1);
    const Acc *Z = T::z(tab, OP);  // ZM2M = 0, ZM2L = 1, ZL2L = 2 match OP
    const int TP = tab.P;
    const Geometry g = shift_geometry(rx, ry, rz);

    if (g.valid != 1) {
        // M2M / L2L with r = 0: identity (truncated / zero-padded); otherwise NaN + flag
        const bool ident = (g.valid == 0) && (OP != OP_M2L);
        const int rows_copy = ident ? (p_in < p_out ? p_in : p_out) : 0;
        for (int i = lane; i < p_out * (p_out + 1); i += 64) {
            const int nn = solid_row(i);
            const bool im0 = (i == nn * (nn + 1) + 1);
            Real v;
            if (!ident)
                v = (Real)NAN;
            else
                v = (nn < rows_copy && !im0) ? in[i] : (Real)0;
            out[i] = im0 ? (Real)0 : ((acc && ident) ? out[i] + v : v);
        }
        if (!ident && lane == 0) raise_device_error(err, -3);
        return;
    }

    // ---- step 1: powers (FP64, rounded once to Real) ----
    if (lane == 0) {
        double cr = 1.0, ci = 0.0, dr = 1.0, dI = 0.0;
        for (int j = 0; j < Pm; ++j) {
            ear[j] = (Acc)cr;
            eai[j] = (Acc)ci;
            ebr[j] = (Acc)dr;
            ebi[j] = (Acc)dI;
            double t1 = cr * g.ca - ci * g.sa;
            ci = cr * g.sa + ci * g.ca;
            cr = t1;
            t1 = dr * g.cb - dI * g.sb;
            dI = dr * g.sb + dI * g.cb;
            dr = t1;
        }
        // s^j and |r|^j
        double sp = 1.0, rp = 1.0;
        for (int n = 0; n < Pm; ++n) {
            // scale in:  M2L/M2M  M_n -> M_n / |r|^{n+1};  L2L  L_n -> L_n |r|^n
            // scale out: M2L/L2L  L_n -> L_n / |r|^n;      M2M  M_n -> M_n |r|^{n+1}
            if (OP == OP_L2L) {
                sc_in[n] = (Acc)rp;
                sc_out[n] = (Acc)sp;
            } else if (OP == OP_M2L) {
                sc_in[n] = (Acc)(sp * g.s);
                sc_out[n] = (Acc)sp;
            } else {
                sc_in[n] = (Acc)(sp * g.s);
                sc_out[n] = (Acc)(rp * g.R);
            }
            sp *= g.s;
            rp *= g.R;
        }
    }
    // ---- load input rows [0, p_in) ----
    for (int i = lane; i < p_in * (p_in + 1); i += 64) A[i] = (Acc)in[i];
    __syncthreads();
    // ---- step 2: scale + rotate a (Im C_n^0 of the input is ignored) ----
    {
        const int tri = p_in * (p_in + 1) / 2;
        for (int c = lane; c < tri; c += 64) {
            const int n = tri_row(c);
            const int m = c - n * (n + 1) / 2;
            const Acc f = sc_in[n];
            const Acc x = A[solid_pos(n, m)] * f;
            const Acc y = (m == 0) ? (Acc)0 : A[solid_pos(n, m) + 1] * f;
            A[solid_pos(n, m)] = x * ear[m] - y * eai[m];
            A[solid_pos(n, m) + 1] = x * eai[m] + y * ear[m];
        }
    }
    __syncthreads();
    swap_rows<Acc>(Ffw, Gfw, A, B, p_in, lane);
    __syncthreads();
    zrot_rows<Acc>(B, ebr, ebi, (Acc)1, p_in, lane);
    __syncthreads();
    swap_rows<Acc>(Ffw, Gfw, B, A, p_in, lane);
    __syncthreads();
    // ---- step 3: z-axis step, columns m, unit shift ----
    {
        const int tri = p_out * (p_out + 1) / 2;
        for (int c = lane; c < tri; c += 64) {
            const int o = tri_row(c);
            const int m = c - o * (o + 1) / 2;
            Acc yr = 0, yi = 0;
            if (m < p_in) {
                int lo = m, hi = p_in - 1;
                if (OP == OP_M2M) hi = (o < hi) ? o : hi;
                if (OP == OP_L2L) lo = o;
                // single-height M2L (eq. m2lkernels, left): terms with o + i <= p_in - 1
                if (OP == OP_M2L && single) hi = (p_in - 1 - o < hi) ? p_in - 1 - o : hi;
                const Acc *zrow = Z + z_col_off(TP, m) + (int64_t)(o - m) * (TP - m) - m;
                for (int i = lo; i <= hi; ++i) {
                    yr += zrow[i] * A[solid_pos(i, m)];
                    yi += zrow[i] * A[solid_pos(i, m) + 1];
                }
            }
            B[solid_pos(o, m)] = yr;
            B[solid_pos(o, m) + 1] = yi;
        }
    }
    __syncthreads();
    // ---- step 4: back rotation of the output rows ----
    swap_rows<Acc>(Fbw, Gbw, B, A, p_out, lane);
    __syncthreads();
    zrot_rows<Acc>(A, ebr, ebi, (Acc)-1, p_out, lane);
    __syncthreads();
    swap_rows<Acc>(Fbw, Gbw, A, B, p_out, lane);
    __syncthreads();
    {
        const int tri = p_out * (p_out + 1) / 2;
        for (int c = lane; c < tri; c += 64) {
            const int n = tri_row(c);
            const int m = c - n * (n + 1) / 2;
            const Acc f = sc_out[n];
            const Acc x = B[solid_pos(n, m)] * f;
            const Acc y = B[solid_pos(n, m) + 1] * f;
            // multiply by e^{-im a}
            Acc vr = x * ear[m] + y * eai[m];
            Acc vi = (m == 0) ? (Acc)0 : (y * ear[m] - x * eai[m]);
            if (acc) {
                vr += (Acc)out[solid_pos(n, m)];
                if (m) vi += (Acc)out[solid_pos(n, m) + 1];
            }
            out[solid_pos(n, m)] = (Real)vr;
            out[solid_pos(n, m) + 1] = (Real)vi;
        }
    }
    __syncthreads();
}

template <typename Real, typename Acc, int OP>
__global__ __launch_bounds__(64) void k_general(DevTables tab, TransArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    const Real *rr = reinterpret_cast<const Real *>(a.r);
    const bool acc = (a.flags & 1u) != 0;
    for (int64_t t = blockIdx.x; t < a.count; t += gridDim.x) {
        const int64_t si = a.src ? a.src[t] : t;
        const int64_t di = a.dst ? a.dst[t] : t;
        general_one<Real, Acc, OP>(tab, a.p_in, a.p_out, (double)rr[3 * t], (double)rr[3 * t + 1],
                                   (double)rr[3 * t + 2], reinterpret_cast<const Real *>(a.in) + si * a.ld_in,
                                   reinterpret_cast<Real *>(a.out) + di * a.ld_out, acc, a.err, smem_raw,
                                   (a.flags & kSingleHeightFlag) != 0);
    }
}

// Work-list form: wavefront-per-item over items[0, count), any op and orders per item.
template <typename Real, typename Acc>
__global__ __launch_bounds__(64) void k_list_general(DevTables tab, ListArgs la)
{
    extern __shared__ unsigned char smem_raw[];
    const bool acc = (la.flags & 1u) != 0;
    const Real *ain = reinterpret_cast<const Real *>(la.arena_in);
    Real *aout = reinterpret_cast<Real *>(la.arena_out);
    for (int64_t t = blockIdx.x; t < la.count; t += gridDim.x) {
        const ListItem it = la.items[t];
        const Real *in = ain + it.in_off;
        Real *out = aout + it.out_off;
        if (it.op == OP_M2M)
            general_one<Real, Acc, OP_M2M>(tab, it.p_in, it.p_out, it.r[0], it.r[1], it.r[2], in, out, acc, la.err, smem_raw);
        else if (it.op == OP_M2L)
            general_one<Real, Acc, OP_M2L>(tab, it.p_in, it.p_out, it.r[0], it.r[1], it.r[2], in, out, acc, la.err, smem_raw);
        else
            general_one<Real, Acc, OP_L2L>(tab, it.p_in, it.p_out, it.r[0], it.r[1], it.r[2], in, out, acc, la.err, smem_raw);
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_list_general(const DevTables &tab, const ListArgs &la, bool f32, bool wide, int pmax,
                               hipStream_t s)
{
    if (la.count <= 0) return hipSuccess;
    const size_t elem = (f32 && !wide) ? sizeof(float) : sizeof(double);
    const size_t smem = (size_t)(2 * pmax * (pmax + 1) + 6 * pmax) * elem;
    const int64_t grid64 = la.count < (1 << 20) ? la.count : (1 << 20);
    if (wide)
        hipLaunchKernelGGL((k_list_general<float, double>), dim3((unsigned)grid64), dim3(64), smem, s, tab, la);
    else if (f32)
        hipLaunchKernelGGL((k_list_general<float, float>), dim3((unsigned)grid64), dim3(64), smem, s, tab, la);
    else
        hipLaunchKernelGGL((k_list_general<double, double>), dim3((unsigned)grid64), dim3(64), smem, s, tab, la);
    return hipGetLastError();
}

hipError_t launch_general(const DevTables &tab, const TransArgs &a, bool f32, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    const int Pm = a.p_in > a.p_out ? a.p_in : a.p_out;
    const bool wide = f32 && Pm >= kF32WideOrder;  // FP32 I/O, FP64 arithmetic
    const size_t elem = (f32 && !wide) ? sizeof(float) : sizeof(double);
    const size_t smem = (size_t)(2 * Pm * (Pm + 1) + 6 * Pm) * elem;
    const int64_t grid64 = a.count < (1 << 20) ? a.count : (1 << 20);
    const dim3 grid((unsigned)grid64), block(64);
#define SH_LAUNCH(T, A, OPV) hipLaunchKernelGGL((k_general<T, A, OPV>), grid, block, smem, s, tab, a)
    if (wide) {
        if (a.op == OP_M2M) SH_LAUNCH(float, double, OP_M2M);
        else if (a.op == OP_M2L) SH_LAUNCH(float, double, OP_M2L);
        else SH_LAUNCH(float, double, OP_L2L);
    } else if (f32) {
        if (a.op == OP_M2M) SH_LAUNCH(float, float, OP_M2M);
        else if (a.op == OP_M2L) SH_LAUNCH(float, float, OP_M2L);
        else SH_LAUNCH(float, float, OP_L2L);
    } else {
        if (a.op == OP_M2M) SH_LAUNCH(double, double, OP_M2M);
        else if (a.op == OP_M2L) SH_LAUNCH(double, double, OP_M2L);
        else SH_LAUNCH(double, double, OP_L2L);
    }
#undef SH_LAUNCH
    return hipGetLastError();
}

}  // namespace shfmm
