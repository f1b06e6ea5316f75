// Exact construction of the swap matrices and z-axis coefficients.  See tables.hpp.
#include "tables.hpp"
#include "layout.hpp"

#include <cmath>
#include <mutex>
#include <stdexcept>

namespace shfmm {

namespace {

using i128 = __int128;

// N_n^{m,l} = 2^n B_n^{m,l}, indices m,l in [-n, n] stored at [(m+n)*(2n+1) + (l+n)].
struct BInt {
    std::vector<std::vector<i128>> N;  // N[n]
    int built = -1;
    void build_to(int nmax)
    {
        if (built < 0) {
            N.push_back(std::vector<i128>{1});
            built = 0;
        }
        for (int n = built; n < nmax; ++n) {
            const int w = 2 * n + 1, w1 = 2 * n + 3;
            const std::vector<i128> &old = N[n];
            auto g = [&](int m, int l) -> i128 {
                if (m < -n || m > n || l < -n || l > n) return 0;
                return old[(size_t)(m + n) * w + (l + n)];
            };
            std::vector<i128> nw((size_t)w1 * w1, 0);
            auto at = [&](int m, int l) -> i128 & { return nw[(size_t)(m + n + 1) * w1 + (l + n + 1)]; };
            for (int m = -n; m <= n; ++m)
                for (int l = -(n + 1); l <= n + 1; ++l) at(m, l) = g(m, l - 1) - g(m, l + 1);
            for (int l = -(n + 1); l <= n + 1; ++l) {
                at(n + 1, l) = g(n, l - 1) + 2 * g(n, l) + g(n, l + 1);
                at(-(n + 1), l) = g(-n, l - 1) - 2 * g(-n, l) + g(-n, l + 1);
            }
            N.push_back(std::move(nw));
        }
        if (nmax > built) built = nmax;
    }
    i128 get(int n, int m, int l) const
    {
        if (m < -n || m > n || l < -n || l > n) return 0;
        return N[n][(size_t)(m + n) * (2 * n + 1) + (l + n)];
    }
};

BInt &bint()
{
    static BInt b;
    return b;
}

// the integer table is grown lazily; concurrent contexts / host calls serialise on it
std::mutex &bint_mutex()
{
    static std::mutex mu;
    return mu;
}

// exact folded integer (times 2^n) of the swap entry (m, l), m,l = 0..n
i128 folded(int n, SwapKind kind, int m, int l)
{
    const BInt &b = bint();
    const i128 sgn = (l % 2) ? -1 : 1;
    switch (kind) {
    case kF:
        return l == 0 ? b.get(n, 0, m) : b.get(n, l, m) + sgn * b.get(n, -l, m);
    case kG:
        return (l == 0 || m == 0) ? 0 : b.get(n, l, m) - sgn * b.get(n, -l, m);
    case kFL:
        return l == 0 ? b.get(n, m, 0) : b.get(n, m, l) + sgn * b.get(n, m, -l);
    case kGL:
        return (l == 0 || m == 0) ? 0 : b.get(n, m, l) - sgn * b.get(n, m, -l);
    }
    return 0;
}

// x! as long double (x <= 2 kMaxOrder), from a table filled once
long double fact_ld(int x)
{
    static const std::vector<long double> tab = [] {
        std::vector<long double> t(2 * kMaxOrder + 1);
        t[0] = 1;
        for (int j = 1; j <= 2 * kMaxOrder; ++j) t[j] = t[j - 1] * j;
        return t;
    }();
    if (x < 0 || x > 2 * kMaxOrder) throw std::out_of_range("factorial");
    return tab[x];
}

// w_n^m / w_n^l = sqrt((n+m)!(n-m)! / ((n+l)!(n-l)!)) in long double
long double wratio(int n, int m, int l)
{
    long double r = 1;
    if (m > l) {
        for (int j = n + l + 1; j <= n + m; ++j) r *= j;      // (n+m)!/(n+l)!
        for (int j = n - m + 1; j <= n - l; ++j) r /= j;      // (n-m)!/(n-l)!
    } else if (l > m) {
        for (int j = n + m + 1; j <= n + l; ++j) r /= j;
        for (int j = n - l + 1; j <= n - m; ++j) r *= j;
    }
    return sqrtl(r);
}

// w_n^m = sqrt((n+m)! (n-m)!) in long double
long double wabs(int n, int m) { return sqrtl(fact_ld(n + m) * fact_ld(n - m)); }

}  // namespace

double swap_entry_f64(int n, SwapKind kind, int m, int l)
{
    if (n < 0 || n >= kMaxOrder || m < 0 || m > n || l < 0 || l > n) throw std::out_of_range("entry");
    std::lock_guard<std::mutex> lk(bint_mutex());
    bint().build_to(n);
    // one rounding: exact integer -> nearest double, then an exact power-of-two scaling
    return ldexp((double)folded(n, kind, m, l), -n);
}

void swap_matrix_ld(int n, SwapKind kind, bool normalised, long double *out)
{
    if (n < 0 || n >= kMaxOrder) throw std::out_of_range("degree");
    std::lock_guard<std::mutex> lk(bint_mutex());
    bint().build_to(n);
    const long double scale = ldexpl(1.0L, -n);
    for (int m = 0; m <= n; ++m)
        for (int l = 0; l <= n; ++l) {
            long double v = (long double)folded(n, kind, m, l) * scale;
            if (normalised && v != 0) {
                // M side: C_hat = W C  =>  T_hat = W T W^{-1}:  (m,l) * w_m / w_l
                // L side: C_hat = W^{-1} C  =>  T_hat = W^{-1} T W:  (m,l) * w_l / w_m
                if (kind == kF || kind == kG)
                    v *= wratio(n, m, l);
                else
                    v *= wratio(n, l, m);
            }
            out[m * (n + 1) + l] = v;
        }
}

long double z_coefficient(ZKind kind, int m, int out, int in, bool normalised)
{
    // out, in are degrees >= m.
    switch (kind) {
    case kZM2L: {
        // L~_out^m = (-1)^{out+m} sum_in (out+in)! M~_in^m       (unit shift along +z)
        long double c = fact_ld(out + in);
        if ((out + m) % 2) c = -c;
        if (normalised) c /= wabs(out, m) * wabs(in, m);
        return c;
    }
    case kZM2M: {
        // M'_out^m = sum_{in <= out} R_{out-in}^0(0,0,-1) M_in^m = sum (-1)^{out-in}/(out-in)! M_in^m
        if (in > out) return 0;
        long double c = 1.0L / fact_ld(out - in);
        if ((out - in) % 2) c = -c;
        if (normalised) c *= wabs(out, m) / wabs(in, m);
        return c;
    }
    case kZL2L: {
        // L'_out^m = sum_{in >= out} L_in^m conj(R_{in-out}^0(0,0,1)) = sum L_in^m / (in-out)!
        if (in < out) return 0;
        long double c = 1.0L / fact_ld(in - out);
        if (normalised) c *= wabs(in, m) / wabs(out, m);
        return c;
    }
    }
    return 0;
}

void build_tables(int P, HostTables &t)
{
    if (P < 1 || P > kMaxOrder) throw std::out_of_range("order");
    t.P = P;
    std::vector<long double> tmp((size_t)P * P);
    for (int k = 0; k < 4; ++k) {
        t.swap64[k].assign(swap_table_size(P), 0.0);
        t.swap32[k].assign(swap_table_size(P), 0.0f);
        t.swap64n[k].assign(swap_table_size(P), 0.0);
        for (int n = 0; n < P; ++n) {
            const int64_t off = swap_offset(n);
            for (int m = 0; m <= n; ++m)
                for (int l = 0; l <= n; ++l)
                    t.swap64[k][off + m * (n + 1) + l] = swap_entry_f64(n, (SwapKind)k, m, l);
            swap_matrix_ld(n, (SwapKind)k, true, tmp.data());
            for (int i = 0; i < (n + 1) * (n + 1); ++i) {
                t.swap32[k][off + i] = (float)tmp[i];
                t.swap64n[k][off + i] = (double)tmp[i];
            }
        }
    }
    // packed non-zeros in the order the fixed-order kernels consume them
    auto pack = [&](const auto &re, const auto &im, auto &out) {
        out.assign(packed_off(P), 0);
        int64_t at = 0;
        for (int n = 0; n < P; ++n) {
            const int64_t off = swap_offset(n);
            for (int m = 0; m <= n; ++m) {
                for (int l = 0; l <= n; ++l)
                    if ((m + l + n) % 2 == 0) out[at++] = re[off + m * (n + 1) + l];
                if (m > 0)
                    for (int l = 1; l <= n; ++l)
                        if ((m + l + n) % 2 == 1) out[at++] = im[off + m * (n + 1) + l];
            }
        }
        if (at != packed_off(P)) throw std::logic_error("packed size");
    };
    for (int side = 0; side < 2; ++side) {
        pack(t.swap64[2 * side], t.swap64[2 * side + 1], t.pk64[side]);
        pack(t.swap32[2 * side], t.swap32[2 * side + 1], t.pk32[side]);
        pack(t.swap64n[2 * side], t.swap64n[2 * side + 1], t.pk64n[side]);
    }
    // MFMA fragments of the block kernel, from the dense tables rounded above
    for (int basis = 0; basis < 2; ++basis) {
        for (int side = 0; side < 2; ++side) {
            auto &out = t.bsw[basis][side];
            out.assign(big_swap_off(kBigOrder), 0.0);
            for (int n = 0; n < kBigOrder && n < P; ++n) {
                const int64_t off = swap_offset(n);
                for (int pm = 0; pm < 2; ++pm)
                    for (int q = 0; q < 2; ++q) {
                        const auto &dense = basis ? t.swap64n[2 * side + q] : t.swap64[2 * side + q];
                        const int pl = (n + pm + q) & 1;
                        for (int ks = 0; ks < 4; ++ks)
                            for (int l = 0; l < 64; ++l) {
                                const int m = 2 * (l % 16) + pm, lc = 2 * (4 * ks + l / 16) + pl;
                                double v = 0.0;
                                if (ks < big_ks(n) && m <= n && lc <= n && !(q == 1 && (m == 0 || lc == 0)))
                                    v = dense[off + m * (n + 1) + lc];
                                out[big_swap_off(n) + ((pm * 2 + q) * 4 + ks) * 64 + l] = v;
                            }
                    }
            }
        }
    }
    for (int k = 0; k < 3; ++k) {
        t.z64[k].assign(z_table_size(P), 0.0);
        t.z32[k].assign(z_table_size(P), 0.0f);
        t.z64n[k].assign(z_table_size(P), 0.0);
        for (int m = 0; m < P; ++m) {
            const int64_t off = z_offset(P, m);
            for (int o = m; o < P; ++o)
                for (int i = m; i < P; ++i) {
                    const int64_t at = off + (int64_t)(o - m) * (P - m) + (i - m);
                    t.z64[k][at] = (double)z_coefficient((ZKind)k, m, o, i, false);
                    long double cn = z_coefficient((ZKind)k, m, o, i, true);
                    t.z32[k][at] = (float)cn;
                    t.z64n[k][at] = (double)cn;
                }
        }
        for (int basis = 0; basis < 2; ++basis) {
            auto &out = t.bz[basis][k];
            out.assign(big_z_off(kBigOrder), 0.0);
            for (int m = 0; m < kBigOrder && m < P; ++m)
                for (int mt = 0; mt < 2; ++mt)
                    for (int ks = 0; ks < 8; ++ks)
                        for (int l = 0; l < 64; ++l) {
                            const int o = m + 16 * mt + l % 16, i = m + 4 * ks + l / 16;
                            double v = 0.0;
                            if (o < kBigOrder && i < kBigOrder && o < P && i < P)
                                v = (double)z_coefficient((ZKind)k, m, o, i, basis == 1);
                            out[big_z_off(m) + (mt * 8 + ks) * 64 + l] = v;
                        }
        }
    }
}

}  // namespace shfmm
