// Lane-per-translation kernel over a mixed work list (orders and offsets per item).
//
// The list is cut (on the host) into tasks of up to 64 items of one operation sharing
// (p_in, p_out); a kernel instantiation serves one operation and one order bucket PB
// (p_in, p_out <= PB).  The structure is the fixed-order kernel's (lpt_impl.hpp): a
// workgroup of 4 wavefronts holds 64 solids in LDS, lane t works on item t of the task,
// rows / columns are shared out among the wavefronts, and tables are wave-uniform scalar
// loads; the orders are runtime values, so rows and columns beyond them are skipped by
// uniform branches.  Solids are gathered from / scattered to the caller's arena at the
// items' offsets.
#pragma once

#include "lpt_impl.hpp"

namespace shfmm {
namespace lpt {

// q = p / d for 0 <= p < 2^24, 1 <= d < 2^12, through a float reciprocal plus one correction
__device__ __forceinline__ int fast_div(int p, int d, float inv)
{
    int q = (int)((float)p * inv);
    if (q * d > p)
        --q;
    else if ((q + 1) * d <= p)
        ++q;
    return q;
}

template <typename Real, typename Acc, int OP, int PB>
__global__ __launch_bounds__(256, (lpt_min_waves<Acc, PB>()))
void k_list_lpt(DevTables tab, ListArgs la)
{
    constexpr int SP = lpt_stride<PB>();
    // powers held per lane up to bucket 12 in FP32 (the list kernel keeps its own register
    // budget; its buckets were tuned with this choice)
    constexpr bool HOLD = sizeof(Acc) == 4 ? PB <= 12 : lpt_hold_powers<Acc, PB>();
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
    constexpr bool TL = lpt_transposed_l<Acc, PB>();
    constexpr bool FT = TL && OP == OP_L2L, BT = TL && OP != OP_M2M;
    const cptr<Acc> Pfw0 = as_const(T::packed(tab, (OP == OP_L2L && !TL) ? 1 : 0));
    const cptr<Acc> Pbw0 = as_const(T::packed(tab, (OP != OP_M2M && !TL) ? 1 : 0));
    const cptr<Acc> Z0 = as_const(T::z(tab, OP));
    const Real *__restrict__ ain = reinterpret_cast<const Real *>(la.arena_in);
    Real *__restrict__ aout = reinterpret_cast<Real *>(la.arena_out);
    const bool acc = (la.flags & 1u) != 0;
    constexpr int CH = 16 * 4 / (int)sizeof(Real);  // loads in flight per thread (32 VGPRs)

    for (int64_t task = blockIdx.x; task < la.ntasks; task += gridDim.x) {
        const ListTask tk = la.tasks[task];
        const int p_in = __builtin_amdgcn_readfirstlane(tk.p_in);
        const int p_out = __builtin_amdgcn_readfirstlane(tk.p_out);
        const int nt = __builtin_amdgcn_readfirstlane(tk.count);
        const int sinp = p_in * (p_in + 1) / 2, soutp = p_out * (p_out + 1) / 2;
        const float inv_in = 1.0f / (float)sinp, inv_out = 1.0f / (float)soutp;
        const cptr<Acc> Pfw = launder(Pfw0), Pbw = launder(Pbw0), Z = launder(Z0);

        // this lane's item (lanes past the task re-read its last item)
        const ListItem *itp = la.items + tk.first + (lane < nt ? lane : nt - 1);
        const int64_t my_in = itp->in_off, my_out = itp->out_off;
        double x = itp->r[0], y = itp->r[1], z = itp->r[2];
        if (lane >= nt) {
            x = 0.0;
            y = 0.0;
            z = 1.0;
        }

        // ---- gather the task's input solids into LDS (pair p -> item p / sinp) ----
        {
            const int np = nt * sinp;
#pragma unroll 1
            for (int c0 = 0; c0 < np; c0 += 256 * CH) {
                R2 v[CH];
                int tt[CH], kk[CH];
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int p = c0 + tid + 256 * i;
                    const int pc = p < np ? p : np - 1;
                    const int t = fast_div(pc, sinp, inv_in);
                    tt[i] = t;
                    kk[i] = 2 * (pc - t * sinp);
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int64_t off = __shfl(my_in, tt[i]);
                    v[i] = *reinterpret_cast<const R2 *>(ain + off + kk[i]);
                }
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    if (c0 + tid + 256 * i < np)
                        *reinterpret_cast<P2 *>(&X[tt[i] * SP + kk[i]]) = P2{(Acc)v[i].x, (Acc)v[i].y};
            }
        }

        const Geometry g = shift_geometry(x, y, z);
        if (wave == 0) {
            bad[lane] = (g.valid == 1) ? 0 : (g.valid == 0 ? 1 : 2);
            const bool any = __any(g.valid != 1 && lane < nt);
            if (lane == 0) bad_flag = any ? 1 : 0;
        }
        Powers<Acc, PB, HOLD> pw;
        pw.init(g);
        const Acc s = (Acc)(g.valid == 1 ? g.s : 1.0);
        const Acc R = (Acc)(g.valid == 1 ? g.R : 1.0);
        Acc *Xt = X + lane * SP;
        lds_barrier();
        const bool bad_any = bad_flag != 0;

        // ---- forward rotation of the input rows n < p_in ----
        per_wave(wave, [&](auto wc) {
            static_for<0, PB>([&](auto nc) {
                constexpr int n = decltype(nc)::value;
                if constexpr (row_owner(PB, n) == decltype(wc)::value) {
                    if (n < p_in) {
                        Acc xr[n + 1], xi[n + 1], yr[n + 1], yi[n + 1];
#pragma unroll
                        for (int m = 0; m <= n; ++m) {
                            const P2 v = *reinterpret_cast<const P2 *>(&Xt[solid_pos(n, m)]);
                            xr[m] = v.x;
                            xi[m] = m ? v.y : (Acc)0;
                        }
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
                }
            });
        });
        lds_barrier();

        // ---- z-axis step, columns m < p_out (rows beyond the orders skipped) ----
        per_wave(wave, [&](auto wc) {
            static_for<0, PB>([&](auto mc) {
                constexpr int m = decltype(mc)::value;
                if constexpr (col_owner(PB, PB, m) == decltype(wc)::value) {
                    if (m < p_out) {
                        if (m >= p_in) {
#pragma unroll
                            for (int o = m; o < PB; ++o)
                                if (o < p_out) *reinterpret_cast<P2 *>(&Xt[solid_pos(o, m)]) = P2{(Acc)0, (Acc)0};
                        } else {
                            Acc ir[PB], ii[PB];
#pragma unroll
                            for (int k = m; k < PB; ++k) {
                                if (k < p_in) {
                                    const P2 v = *reinterpret_cast<const P2 *>(&Xt[solid_pos(k, m)]);
                                    ir[k] = v.x;
                                    ii[k] = v.y;
                                } else {
                                    ir[k] = 0;
                                    ii[k] = 0;
                                }
                            }
                            // coefficients of output o + 1 fetched while output o is summed
                            Acc cz[PB - m];
                            z_fetch<Real, Acc, OP, PB, m>(Z, m, cz);
#pragma unroll
                            for (int o = m; o < PB; ++o) {
                                Acc nz[PB - m];
                                if (o + 1 < PB) z_fetch<Real, Acc, OP, PB, m>(Z, o + 1, nz);
                                if (o < p_out) {
                                    // rows k >= p_in are zero in ir / ii, so their terms add
                                    // exact zeros: no per-term test (the compiler turned a test
                                    // on the task's p_in here into four selects per term)
                                    Acc orr = 0, oi = 0;
#pragma unroll
                                    for (int k = m; k < PB; ++k) {
                                        if (OP == OP_M2M && k > o) continue;
                                        if (OP == OP_L2L && k < o) continue;
                                        orr += cz[k - m] * ir[k];
                                        oi += cz[k - m] * ii[k];
                                    }
                                    *reinterpret_cast<P2 *>(&Xt[solid_pos(o, m)]) = P2{orr, oi};
                                }
                                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                                for (int k = 0; k < PB - m; ++k) cz[k] = nz[k];
                            }
                        }
                    }
                }
            });
        });
        lds_barrier();

        // ---- backward rotation of the output rows n < p_out ----
        per_wave(wave, [&](auto wc) {
            static_for<0, PB>([&](auto nc) {
                constexpr int n = decltype(nc)::value;
                if constexpr (row_owner(PB, n) == decltype(wc)::value) {
                    if (n < p_out) {
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
                        const Acc f = (OP == OP_M2M) ? ipow(R, n + 1) : ipow(s, n);
#pragma unroll
                        for (int m = 0; m <= n; ++m)
                            *reinterpret_cast<P2 *>(&Xt[solid_pos(n, m)]) = P2{xr[m] * f, m ? xi[m] * f : (Acc)0};
                    }
                }
            });
        });
        lds_barrier();

        // ---- scatter the outputs to the arena (pair p -> item p / soutp) ----
        {
            const int nq = nt * soutp;
#pragma unroll 1
            for (int c0 = 0; c0 < nq; c0 += 256 * CH) {
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int p = c0 + tid + 256 * i;
                    const int pc = p < nq ? p : nq - 1;
                    const int t = fast_div(pc, soutp, inv_out);
                    const int k = 2 * (pc - t * soutp);
                    const int64_t off = __shfl(my_out, t);
                    if (p < nq) {
                        const P2 v = *reinterpret_cast<const P2 *>(&X[t * SP + k]);
                        R2 w{(Real)v.x, (Real)v.y};
                        if (bad_any || acc) {
                            int n = (int)((sqrtf(4.0f * (float)k + 1.0f) - 1.0f) * 0.5f);
                            while ((n + 1) * (n + 2) <= k) ++n;
                            while (n * (n + 1) > k) --n;
                            const bool m0 = (k == n * (n + 1));
                            const int b = bad[t];
                            const bool ident = (b == 1 && OP != OP_M2L);
                            if (b != 0) {
                                if (ident) {
                                    // zero shift of M2M / L2L: identity, truncated / zero-padded
                                    const int64_t si = __shfl(my_in, t);
                                    const bool keep = n < p_in && n < p_out;
                                    w.x = keep ? ain[si + k] : (Real)0;
                                    w.y = (keep && !m0) ? ain[si + k + 1] : (Real)0;
                                } else {
                                    w.x = w.y = (Real)NAN;
                                    if (k == 0) raise_device_error(la.err, -3);
                                }
                            }
                            if (acc && (b == 0 || ident)) {
                                const R2 old = *reinterpret_cast<const R2 *>(aout + off + k);
                                w.x += old.x;
                                if (!m0) w.y += old.y;
                            }
                        }
                        *reinterpret_cast<R2 *>(aout + off + k) = w;
                    }
                }
            }
        }
        lds_barrier();
    }
}

template <typename Real, typename Acc, int OP, int PB>
hipError_t launch_list_one(const DevTables &tab, const ListArgs &la, hipStream_t s)
{
    const void *fn = reinterpret_cast<const void *>(&k_list_lpt<Real, Acc, OP, PB>);
    const int64_t res = resident_workgroups(fn);
    const dim3 grid((unsigned)(la.ntasks < res ? la.ntasks : res)), block(256);
    hipLaunchKernelGGL((k_list_lpt<Real, Acc, OP, PB>), grid, block, 0, s, tab, la);
    return hipGetLastError();
}

constexpr int kListBuckets[] = {4, 6, 8, 10, 12, 16};

// one (dtype, op) -> all buckets; instantiated in the k_list_<dtype>_<op>.hip units
template <typename Real, typename Acc, int OP>
hipError_t launch_list_fixed(int bucket, const DevTables &tab, const ListArgs &la, hipStream_t s)
{
    switch (bucket) {
    case 4: return launch_list_one<Real, Acc, OP, 4>(tab, la, s);
    case 6: return launch_list_one<Real, Acc, OP, 6>(tab, la, s);
    case 8: return launch_list_one<Real, Acc, OP, 8>(tab, la, s);
    case 10: return launch_list_one<Real, Acc, OP, 10>(tab, la, s);
    case 12: return launch_list_one<Real, Acc, OP, 12>(tab, la, s);
    case 16: return launch_list_one<Real, Acc, OP, 16>(tab, la, s);
    default: return hipErrorInvalidValue;
    }
}

extern template hipError_t launch_list_fixed<double, double, OP_M2M>(int, const DevTables &, const ListArgs &, hipStream_t);
extern template hipError_t launch_list_fixed<double, double, OP_M2L>(int, const DevTables &, const ListArgs &, hipStream_t);
extern template hipError_t launch_list_fixed<double, double, OP_L2L>(int, const DevTables &, const ListArgs &, hipStream_t);
extern template hipError_t launch_list_fixed<float, float, OP_M2M>(int, const DevTables &, const ListArgs &, hipStream_t);
extern template hipError_t launch_list_fixed<float, float, OP_M2L>(int, const DevTables &, const ListArgs &, hipStream_t);
extern template hipError_t launch_list_fixed<float, float, OP_L2L>(int, const DevTables &, const ListArgs &, hipStream_t);

}  // namespace lpt
}  // namespace shfmm
