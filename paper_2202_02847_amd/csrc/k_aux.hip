// Neighbouring kernels of the translation path:
//   * the direct O(P^4) double-height M2L (eq. m2lkernels, right), the baseline the paper
//     measures its scheme against (Section 4), with S by the Appendix recurrences;
//   * P2M (eq. MLexpansions: M_n^m = sum_j q_j R_n^m(y_j - x_A)), R by the Appendix
//     recurrences, used to build multipole inputs on the device;
//   * L2P: the potential of a local expansion (eq. MLexpansions) and its gradient at
//     target points;
//   * P2P: the direct near-field sum over neighbouring boxes (eq. nbody).
#include <type_traits>

#include "kernels.hpp"
#include "near_field.hpp"

namespace shfmm {

namespace {

// read-only device memory addressed wave-uniformly: loads through the scalar cache
using lpt_cptr = const __attribute__((address_space(4))) double *;

__device__ __forceinline__ int tri_row_aux(int c)
{
    int n = (int)((sqrtf(8.0f * (float)c + 1.0f) - 1.0f) * 0.5f);
    while ((n + 1) * (n + 2) / 2 <= c) ++n;
    while (n * (n + 1) / 2 > c) --n;
    return n;
}

// one wavefront per translation; S_j^i(r) for j < ps in LDS, M staged in LDS,
// lanes own outputs (n, m) and run the k, l double loop.
__global__ __launch_bounds__(64) void k_m2l_naive(TransArgs a)
{
    extern __shared__ double sm[];
    const int p_in = a.p_in, p_out = a.p_out;
    const int ps = p_in + p_out - 1;
    double *S = sm;                      // ps(ps+1)
    double *M = S + ps * (ps + 1);       // p_in(p_in+1)
    const int lane = threadIdx.x;
    const double *rr = reinterpret_cast<const double *>(a.r);
    const bool acc = (a.flags & 1u) != 0;
    for (int64_t t = blockIdx.x; t < a.count; t += gridDim.x) {
        const int64_t si = a.src ? a.src[t] : t;
        const int64_t di = a.dst ? a.dst[t] : t;
        const double *in = reinterpret_cast<const double *>(a.in) + si * a.ld_in;
        double *out = reinterpret_cast<double *>(a.out) + di * a.ld_out;
        const double x = rr[3 * t], y = rr[3 * t + 1], z = rr[3 * t + 2];
        const double r2 = x * x + y * y + z * z;
        if (!(r2 > 0.0) || !isfinite(r2)) {
            for (int i = lane; i < p_out * (p_out + 1); i += 64) out[i] = NAN;
            if (lane == 0) raise_device_error(a.err, -3);
            continue;
        }
        for (int i = lane; i < p_in * (p_in + 1); i += 64) M[i] = in[i];
        // diagonal S_n^n = (2n-1)(x+iy)/|r|^2 S_{n-1}^{n-1}
        if (lane == 0) {
            double pr = 1.0 / sqrt(r2), pi = 0.0;
            S[0] = pr;
            S[1] = 0.0;
            for (int n = 1; n < ps; ++n) {
                const double f = (2 * n - 1) / r2;
                const double nr = f * (x * pr - y * pi), ni = f * (x * pi + y * pr);
                pr = nr;
                pi = ni;
                S[solid_pos(n, n)] = pr;
                S[solid_pos(n, n) + 1] = pi;
            }
        }
        __syncthreads();
        // columns: |r|^2 S_n^m = (2n-1) z S_{n-1}^m - ((n-1)^2 - m^2) S_{n-2}^m
        for (int m = lane; m < ps; m += 64) {
            for (int n = m + 1; n < ps; ++n)
                for (int c = 0; c < 2; ++c) {
                    const double s1 = S[solid_pos(n - 1, m) + c];
                    const double s2 = (n - 2 >= m) ? S[solid_pos(n - 2, m) + c] : 0.0;
                    S[solid_pos(n, m) + c] = ((2 * n - 1) * z * s1 - ((double)(n - 1) * (n - 1) - (double)m * m) * s2) / r2;
                }
        }
        __syncthreads();
        const int tri = p_out * (p_out + 1) / 2;
        for (int c = lane; c < tri; c += 64) {
            const int n = tri_row_aux(c);
            const int m = c - n * (n + 1) / 2;
            double sr = 0.0, sI = 0.0;
            for (int k = 0; k < p_in; ++k)
                for (int l = -k; l <= k; ++l) {
                    const int al = l < 0 ? -l : l;
                    double mr = M[solid_pos(k, al)], mi = al ? M[solid_pos(k, al) + 1] : 0.0;
                    if (l < 0) {
                        const double sg = (al & 1) ? -1.0 : 1.0;
                        mr *= sg;
                        mi *= -sg;
                    }
                    const int j = n + k, i = m + l;
                    const int ai = i < 0 ? -i : i;
                    double tr = S[solid_pos(j, ai)], ti = S[solid_pos(j, ai) + 1];
                    if (i < 0) {
                        const double sg = (ai & 1) ? -1.0 : 1.0;
                        tr *= sg;
                        ti *= -sg;
                    }
                    sr += mr * tr + mi * ti;   // conj(M) * S
                    sI += mr * ti - mi * tr;
                }
            const double sg = (n & 1) ? -1.0 : 1.0;
            double vr = sg * sr, vi = m ? sg * sI : 0.0;
            if (acc) {
                vr += out[solid_pos(n, m)];
                if (m) vi += out[solid_pos(n, m) + 1];
            }
            out[solid_pos(n, m)] = vr;
            out[solid_pos(n, m) + 1] = vi;
        }
        __syncthreads();
    }
}

// One wavefront per cluster.  The 64 lanes form G = 64 / P groups of P lanes; lane (g, m)
// takes the points j = g, g + G, ... and accumulates column m of sum_j q_j R(y_j - c) into LDS
// copy g (the diagonal R_m^m takes m steps and the column P - 1 - m, so every lane does about
// P steps per point); the G copies are added at the end.
__global__ __launch_bounds__(64) void k_p2m(int P, int64_t count, const double *centres, int64_t npts,
                                            const double *pts, const double *q, double *Mout, int64_t ldM)
{
    extern __shared__ double accm[];  // G copies of P(P+1)
    const int lane = threadIdx.x;
    const int S = P * (P + 1);
    const int G = P <= 64 ? 64 / P : 1;
    const int g = lane / P, m0 = lane - g * P;
    const bool active = g < G;
    for (int64_t c = blockIdx.x; c < count; c += gridDim.x) {
        for (int i = lane; i < G * S; i += 64) accm[i] = 0.0;
        __syncthreads();
        const double cx = centres[3 * c], cy = centres[3 * c + 1], cz = centres[3 * c + 2];
        double *acc = accm + (active ? g : 0) * S;
        for (int64_t j = active ? g : npts; j < npts; j += G) {
            const double *pj = pts + 3 * (npts * c + j);
            const double x = pj[0] - cx, y = pj[1] - cy, z = pj[2] - cz;
            const double r2 = x * x + y * y + z * z;
            const double qj = q[npts * c + j];
            for (int m = m0; m < P; m += 64) {
                // R_m^m = prod_{i=1}^{m} (x+iy)/(2i)
                double dr = 1.0, di = 0.0;
                for (int i = 1; i <= m; ++i) {
                    const double nr = (x * dr - y * di) / (2 * i), ni = (x * di + y * dr) / (2 * i);
                    dr = nr;
                    di = ni;
                }
                // (n^2 - m^2) R_n^m = (2n-1) z R_{n-1}^m - |r|^2 R_{n-2}^m
                double ar = dr, ai = di, br = 0.0, bi = 0.0;  // R_{n-1}, R_{n-2}
                acc[solid_pos(m, m)] += qj * ar;
                acc[solid_pos(m, m) + 1] += qj * ai;
                for (int n = m + 1; n < P; ++n) {
                    const double d = (double)n * n - (double)m * m;
                    const double cr = ((2 * n - 1) * z * ar - r2 * br) / d;
                    const double ci = ((2 * n - 1) * z * ai - r2 * bi) / d;
                    br = ar;
                    bi = ai;
                    ar = cr;
                    ai = ci;
                    acc[solid_pos(n, m)] += qj * ar;
                    acc[solid_pos(n, m) + 1] += qj * ai;
                }
            }
        }
        __syncthreads();
        double *Mo = Mout + c * ldM;
        for (int i = lane; i < S; i += 64) {
            int n = (int)((sqrtf(4.0f * (float)i + 1.0f) - 1.0f) * 0.5f);
            while ((n + 1) * (n + 2) <= i) ++n;
            while (n * (n + 1) > i) --n;
            double v = 0.0;
            for (int k = 0; k < G; ++k) v += accm[k * S + i];
            Mo[i] = (i == n * (n + 1) + 1) ? 0.0 : v;
        }
        __syncthreads();
    }
}

// P2M for orders up to 16, with the order PO known at compile time: the same lane split as
// k_p2m, but each lane keeps the sums of its column m and the recurrence reciprocals
// 1/(n^2 - m^2) in registers, so the per-point work is a register FMA chain instead of
// dependent LDS read-modify-writes; the sums meet in LDS once per cluster.
template <int PO>
__global__ __launch_bounds__(64) void k_p2m_reg(int64_t count, const double *centres, int64_t npts,
                                                const double *pts, const double *q, double *Mout, int64_t ldM)
{
    extern __shared__ double accm[];  // G copies of PO(PO+1)
    constexpr int S = PO * (PO + 1);
    constexpr int G = 64 / PO;
    const int lane = threadIdx.x;
    const int g = lane / PO, m = lane - g * PO;
    const bool active = g < G;
    double inv[PO];
#pragma unroll
    for (int n = 0; n < PO; ++n) inv[n] = (n > m) ? 1.0 / ((double)n * n - (double)m * m) : 0.0;
    for (int64_t c = blockIdx.x; c < count; c += gridDim.x) {
        double sr[PO], si[PO];
#pragma unroll
        for (int n = 0; n < PO; ++n) {
            sr[n] = 0.0;
            si[n] = 0.0;
        }
        const double cx = centres[3 * c], cy = centres[3 * c + 1], cz = centres[3 * c + 2];
        for (int64_t j = active ? g : npts; j < npts; j += G) {
            const double *pj = pts + 3 * (npts * c + j);
            const double x = pj[0] - cx, y = pj[1] - cy, z = pj[2] - cz;
            const double r2 = x * x + y * y + z * z;
            const double qj = q[npts * c + j];
            // R_m^m = prod_{i=1}^{m} (x+iy)/(2i)
            double dr = 1.0, di = 0.0;
            for (int i = 1; i <= m; ++i) {
                const double f = 0.5 / (double)i;
                const double nr = (x * dr - y * di) * f, ni = (x * di + y * dr) * f;
                dr = nr;
                di = ni;
            }
            // (n^2 - m^2) R_n^m = (2n-1) z R_{n-1}^m - |r|^2 R_{n-2}^m, n > m
            double ar = dr, ai = di, br = 0.0, bi = 0.0;
#pragma unroll
            for (int n = 0; n < PO; ++n) {
                if (n > m) {
                    const double tz = (double)(2 * n - 1) * z;
                    const double cr = (tz * ar - r2 * br) * inv[n], ci = (tz * ai - r2 * bi) * inv[n];
                    br = ar;
                    bi = ai;
                    ar = cr;
                    ai = ci;
                }
                if (n >= m) {
                    sr[n] += qj * ar;
                    si[n] += qj * ai;
                }
            }
        }
        if (active) {
#pragma unroll
            for (int n = 0; n < PO; ++n)
                if (n >= m) {
                    accm[g * S + solid_pos(n, m)] = sr[n];
                    accm[g * S + solid_pos(n, m) + 1] = si[n];
                }
        }
        __syncthreads();
        double *Mo = Mout + c * ldM;
        for (int i = lane; i < S; i += 64) {
            int n = (int)((sqrtf(4.0f * (float)i + 1.0f) - 1.0f) * 0.5f);
            while ((n + 1) * (n + 2) <= i) ++n;
            while (n * (n + 1) > i) --n;
            double v = 0.0;
            for (int k = 0; k < G; ++k) v += accm[k * S + i];
            Mo[i] = (i == n * (n + 1) + 1) ? 0.0 : v;
        }
        __syncthreads();
    }
}

// L2P: one lane per target, the 64 lanes of a wavefront on targets of one box, so that the
// box's local expansion is read through the scalar cache.  R_k^j(x - c) is generated
// column by column (j) by the Appendix recurrences and used at once:
//   Phi    = Re sum_{k,j} conj(R_k^j) L_k^j,
//   grad   = Re sum_{k,j} conj(R_k^j) (X, Y, Z),  X = (L_{k+1}^{j+1} - L_{k+1}^{j-1}) / 2,
//            Y = -i (L_{k+1}^{j+1} + L_{k+1}^{j-1}) / 2,  Z = L_{k+1}^j,
// which is the derivative identities of the harmonics (d/dz R_n^m = R_{n-1}^m,
// d/dx R_n^m = (R_{n-1}^{m-1} - R_{n-1}^{m+1}) / 2, d/dy R_n^m = i (R_{n-1}^{m-1} + R_{n-1}^{m+1}) / 2)
// gathered per R_k^j instead of per L_n^m.  The term of -j equals the conjugate of that of
// j, so columns j > 0 count twice.  Im L_n^0 is ignored (read as 0).
// MB (boxes of at most 32 targets): a wavefront takes bpw = 64 / npts whole boxes, lane
// (kb, j) target j of box kb, and reads each lane's box data by vector loads (the lanes of one
// box share its cache lines); otherwise the wavefront covers 64 targets of one box.
template <bool MB>
__global__ __launch_bounds__(256) void k_l2p(int P, int64_t count, int64_t chunks, int64_t bpw, const double *centres,
                                             int64_t npts, const double *pts, const double *Lpool,
                                             int64_t ldL, double *out, unsigned flags)
{
    using RP = std::conditional_t<MB, const double *, lpt_cptr>;
    // recurrence constants, shared by the workgroup: rc[k P + j] = 1/(k^2 - j^2) (k > j),
    // rc[j P + j] = 1/(2j) (j > 0)
    extern __shared__ double rc[];
    for (int i = threadIdx.x; i < P * P; i += 256) {
        const int k = i / P, j = i - k * P;
        rc[i] = (k > j) ? 1.0 / ((double)k * k - (double)j * j) : ((k == j && j > 0) ? 0.5 / (double)j : 0.0);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t ntask = MB ? (count + bpw - 1) / bpw : count * chunks;
    const bool acc = (flags & 1u) != 0;
    for (int64_t task = (int64_t)blockIdx.x * 4 + wave; task < ntask; task += (int64_t)gridDim.x * 4) {
        int64_t c, j0;
        bool act;
        if constexpr (MB) {
            const int64_t kb = lane / npts;
            c = task * bpw + kb;
            j0 = lane - kb * npts;
            act = kb < bpw && c < count;
            if (!act) c = 0;  // idle lanes read box 0
        } else {
            c = task / chunks;
            j0 = (task - c * chunks) * 64 + lane;
            act = j0 < npts;
        }
        const int64_t t = c * npts + (act ? j0 : 0);
        const RP Lc = (RP)(Lpool + c * ldL);
        const RP cc = (RP)(centres + 3 * c);
        const double x = pts[3 * t] - cc[0], y = pts[3 * t + 1] - cc[1], z = pts[3 * t + 2] - cc[2];
        const double r2 = x * x + y * y + z * z;
        double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        double dr = 1.0, di = 0.0;  // R_j^j
        for (int j = 0; j < P; ++j) {
            if (j > 0) {
                const double f = rc[j * P + j];
                const double nr = (x * dr - y * di) * f, ni = (x * di + y * dr) * f;
                dr = nr;
                di = ni;
            }
            double ar = dr, ai = di, br = 0.0, bi = 0.0;  // R_k^j, R_{k-1}^j
            double cp = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
            for (int k = j; k < P; ++k) {
                if (k > j) {
                    const double inv = rc[k * P + j];
                    const double tz = (double)(2 * k - 1) * z;
                    const double nr = (tz * ar - r2 * br) * inv, ni = (tz * ai - r2 * bi) * inv;
                    br = ar;
                    bi = ai;
                    ar = nr;
                    ai = ni;
                }
                const int64_t pk = (int64_t)k * (k + 1) + 2 * j;
                cp += ar * Lc[pk] + (j ? ai * Lc[pk + 1] : 0.0);
                if (k + 1 < P) {
                    const int64_t pz = (int64_t)(k + 1) * (k + 2) + 2 * j;
                    const double zr = Lc[pz], zi = j ? Lc[pz + 1] : 0.0;
                    const double ur = Lc[pz + 2], ui = Lc[pz + 3];  // L_{k+1}^{j+1}
                    double vr, vi;                                   // L_{k+1}^{j-1}
                    if (j == 0) {
                        vr = -ur;
                        vi = ui;
                    } else {
                        vr = Lc[pz - 2];
                        vi = (j > 1) ? Lc[pz - 1] : 0.0;
                    }
                    cx += 0.5 * (ar * (ur - vr) + ai * (ui - vi));
                    cy += 0.5 * (ar * (ui + vi) - ai * (ur + vr));
                    cz += ar * zr + ai * zi;
                }
            }
            const double w = j ? 2.0 : 1.0;
            phi += w * cp;
            gx += w * cx;
            gy += w * cy;
            gz += w * cz;
        }
        if (act) {
            double *o = out + 4 * t;
            if (acc) {
                phi += o[0];
                gx += o[1];
                gy += o[2];
                gz += o[3];
            }
            *reinterpret_cast<double2 *>(o) = double2{phi, gx};
            *reinterpret_cast<double2 *>(o + 2) = double2{gy, gz};
        }
    }
}

// 1/sqrt(x) for x > 0: the hardware estimate (about 23 correct bits) refined by two
// Newton-Raphson steps for the reciprocal square root, y <- y (3 - x y^2) / 2, each of which
// roughly doubles the number of correct bits.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// P2P (the near field of eq. nbody with G = 1/|x - y|): one lane per target, the 64 lanes of a
// wavefront on targets of one box; the sources of each neighbour box (nbr[27c + k], -1 for
// none) are read by wave-uniform scalar loads.  Adds q_j / |x - y_j| and its gradient
// -q_j (x - y_j) / |x - y_j|^3 over sources at a distance > 0 (a target does not see itself).
// MB: several whole boxes per wavefront, as in k_l2p.
template <bool MB>
__global__ __launch_bounds__(256) void k_p2p(int64_t count, int64_t chunks, int64_t bpw, int64_t npts,
                                             const double *pts, const double *q, const int32_t *nbr, double *out,
                                             unsigned flags)
{
    using RP = std::conditional_t<MB, const double *, lpt_cptr>;
    using IP = std::conditional_t<MB, const int32_t *, const __attribute__((address_space(4))) int32_t *>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t ntask = MB ? (count + bpw - 1) / bpw : count * chunks;
    const bool acc = (flags & 1u) != 0;
    const RP P = (RP)pts;
    const RP Q = (RP)q;
    const IP NB = (IP)nbr;
    for (int64_t task = (int64_t)blockIdx.x * 4 + wave; task < ntask; task += (int64_t)gridDim.x * 4) {
        int64_t c, j0;
        bool act;
        if constexpr (MB) {
            const int64_t kb = lane / npts;
            c = task * bpw + kb;
            j0 = lane - kb * npts;
            act = kb < bpw && c < count;
            if (!act) c = 0;  // idle lanes read box 0
        } else {
            c = task / chunks;
            j0 = (task - c * chunks) * 64 + lane;
            act = j0 < npts;
        }
        const int64_t t = c * npts + (act ? j0 : 0);
        const double x = pts[3 * t], y = pts[3 * t + 1], z = pts[3 * t + 2];
        double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        for (int k = 0; k < 27; ++k) {
            const int32_t b = NB[27 * c + k];
            if (b < 0) continue;
            const int64_t s0 = (int64_t)b * npts;
            for (int64_t s = 0; s < npts; ++s) {
                const double dx = x - P[3 * (s0 + s)], dy = y - P[3 * (s0 + s) + 1], dz = z - P[3 * (s0 + s) + 2];
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double inv = (r2 > 0.0) ? rsqrt_nr(r2) : 0.0;
                const double qi = Q[s0 + s] * inv;
                const double qi3 = qi * inv * inv;
                phi += qi;
                gx -= qi3 * dx;
                gy -= qi3 * dy;
                gz -= qi3 * dz;
            }
        }
        if (act) {
            double *o = out + 4 * t;
            if (acc) {
                phi += o[0];
                gx += o[1];
                gy += o[2];
                gz += o[3];
            }
            *reinterpret_cast<double2 *>(o) = double2{phi, gx};
            *reinterpret_cast<double2 *>(o + 2) = double2{gy, gz};
        }
    }
}

// Segmented sum: L[b] = sum of the solids scratch[t - base] for t in [seg[b], seg[b + 1]),
// for targets b in [tb, te); one thread per (target, coefficient), coalesced over coefficients.
__global__ __launch_bounds__(256) void k_seg_sum(double *L, int64_t S, const int64_t *seg, int64_t tb, int64_t te,
                                                 int64_t base, const double *scratch)
{
    const int64_t n = (te - tb) * S;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * 256) {
        const int64_t b = tb + idx / S, i = idx - (idx / S) * S;
        double v = 0.0;
        for (int64_t t = seg[b] - base; t < seg[b + 1] - base; ++t) v += scratch[t * S + i];
        L[b * S + i] = v;
    }
}

}  // namespace

hipError_t launch_seg_sum(double *L, int64_t S, const int64_t *seg, int64_t tb, int64_t te, int64_t base,
                          const double *scratch, hipStream_t s)
{
    const int64_t n = (te - tb) * S;
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)(blocks < 16384 ? blocks : 16384)), dim3(256), 0, s, L, S, seg, tb, te,
                       base, scratch);
    return hipGetLastError();
}

hipError_t launch_m2l_naive(const TransArgs &a, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    const int ps = a.p_in + a.p_out - 1;
    const size_t smem = (size_t)(ps * (ps + 1) + a.p_in * (a.p_in + 1)) * sizeof(double);
    const int64_t grid64 = a.count < (1 << 20) ? a.count : (1 << 20);
    hipLaunchKernelGGL(k_m2l_naive, dim3((unsigned)grid64), dim3(64), smem, s, a);
    return hipGetLastError();
}

hipError_t launch_p2m(int P, int64_t count, const double *centres, int64_t npts, const double *pts,
                      const double *q, double *M, int64_t ldM, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const int G = P <= 64 ? 64 / P : 1;
    const size_t smem = (size_t)G * P * (P + 1) * sizeof(double);
    const int64_t grid64 = count < (1 << 20) ? count : (1 << 20);
    switch (P) {
#define SH_P2M_REG(PO)                                                                                              \
    case PO:                                                                                                        \
        hipLaunchKernelGGL(k_p2m_reg<PO>, dim3((unsigned)grid64), dim3(64), smem, s, count, centres, npts, pts, q, M, \
                           ldM);                                                                                    \
        return hipGetLastError();
        SH_P2M_REG(2)
        SH_P2M_REG(3)
        SH_P2M_REG(4)
        SH_P2M_REG(5)
        SH_P2M_REG(6)
        SH_P2M_REG(7)
        SH_P2M_REG(8)
        SH_P2M_REG(9)
        SH_P2M_REG(10)
        SH_P2M_REG(11)
        SH_P2M_REG(12)
        SH_P2M_REG(13)
        SH_P2M_REG(14)
        SH_P2M_REG(15)
        SH_P2M_REG(16)
#undef SH_P2M_REG
    default:
        break;
    }
    hipLaunchKernelGGL(k_p2m, dim3((unsigned)grid64), dim3(64), smem, s, P, count, centres, npts, pts, q, M, ldM);
    return hipGetLastError();
}

hipError_t launch_l2p(int P, int64_t count, const double *centres, int64_t npts, const double *pts,
                      const double *L, int64_t ldL, double *out, unsigned flags, hipStream_t s)
{
    if (count <= 0 || npts <= 0) return hipSuccess;
    const size_t smem = (size_t)P * P * sizeof(double);
    if (npts <= 32) {
        const int64_t bpw = 64 / npts;
        const int64_t blocks = ((count + bpw - 1) / bpw + 3) / 4;
        const int64_t grid64 = blocks < (1 << 16) ? blocks : (1 << 16);
        hipLaunchKernelGGL(k_l2p<true>, dim3((unsigned)grid64), dim3(256), smem, s, P, count, (int64_t)1, bpw, centres,
                           npts, pts, L, ldL, out, flags);
        return hipGetLastError();
    }
    const int64_t chunks = (npts + 63) / 64;
    const int64_t blocks = (count * chunks + 3) / 4;
    const int64_t grid64 = blocks < (1 << 16) ? blocks : (1 << 16);
    hipLaunchKernelGGL(k_l2p<false>, dim3((unsigned)grid64), dim3(256), smem, s, P, count, chunks, (int64_t)1, centres,
                       npts, pts, L, ldL, out, flags);
    return hipGetLastError();
}

hipError_t launch_p2p(int64_t count, int64_t npts, const double *pts, const double *q, const int32_t *nbr,
                      double *out, unsigned flags, hipStream_t s)
{
    if (count <= 0 || npts <= 0) return hipSuccess;
    if (npts <= 32) {
        const int64_t bpw = 64 / npts;
        const int64_t blocks = ((count + bpw - 1) / bpw + 3) / 4;
        const int64_t grid64 = blocks < (1 << 16) ? blocks : (1 << 16);
        hipLaunchKernelGGL(k_p2p<true>, dim3((unsigned)grid64), dim3(256), 0, s, count, (int64_t)1, bpw, npts, pts, q,
                           nbr, out, flags);
        return hipGetLastError();
    }
    const int64_t chunks = (npts + 63) / 64;
    const int64_t blocks = (count * chunks + 3) / 4;
    const int64_t grid64 = blocks < (1 << 16) ? blocks : (1 << 16);
    hipLaunchKernelGGL(k_p2p<false>, dim3((unsigned)grid64), dim3(256), 0, s, count, chunks, (int64_t)1, npts, pts, q,
                       nbr, out, flags);
    return hipGetLastError();
}

}  // namespace shfmm
