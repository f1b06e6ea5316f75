// Host-side checks of the table builder, built with AddressSanitizer and UndefinedBehavior-
// Sanitizer by tests/test_sanitizers.py (no GPU).  Exercises every table the library builds at
// context creation and checks properties fixed by the construction of the axis swap:
//   * F_n^2 = I and G_n^2 = I on orders m, l >= 1 (the swap x <-> z is an involution);
//   * the chequerboard: F^{m,l} = 0 unless m + l + n is even, G^{m,l} = 0 unless m + l + n is
//     odd and m, l >= 1 (Section 3.1, Fig. 2);
//   * F_L = D F^T D^{-1} with D = diag(2, 1, ..., 1) and G_L = G^T (the L-side swap);
//   * every built table has the size its layout promises and holds finite values.
// Exit status 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <vector>

#include "tables.hpp"

using namespace shfmm;

static int fails = 0;
static void expect(bool ok, const char *what, int n)
{
    if (!ok) {
        std::fprintf(stderr, "FAIL %s (n = %d)\n", what, n);
        ++fails;
    }
}

int main()
{
    HostTables t;
    build_tables(kMaxOrder, t);
    for (int k = 0; k < 4; ++k) {
        expect((int64_t)t.swap64[k].size() == swap_table_size(kMaxOrder), "swap64 size", k);
        expect(t.swap32[k].size() == t.swap64[k].size(), "swap32 size", k);
        for (double v : t.swap64n[k]) expect(std::isfinite(v), "swap64n finite", k);
    }
    for (int k = 0; k < 3; ++k) {
        expect(!t.z64[k].empty() && t.z32[k].size() == t.z64[k].size(), "z table sizes", k);
        for (float v : t.z32[k]) expect(std::isfinite(v), "z32 finite", k);
    }
    for (int n = 0; n < 26; ++n) {
        const int w = n + 1;
        std::vector<long double> F(w * w), G(w * w), FL(w * w), GL(w * w);
        swap_matrix_ld(n, kF, false, F.data());
        swap_matrix_ld(n, kG, false, G.data());
        swap_matrix_ld(n, kFL, false, FL.data());
        swap_matrix_ld(n, kGL, false, GL.data());
        long double worst_f = 0, worst_g = 0, scale = 1;
        for (long double v : F) scale = std::fmax(scale, std::fabs(v));
        for (int i = 0; i < w; ++i)
            for (int j = 0; j < w; ++j) {
                long double sf = 0, sg = 0;
                for (int q = 0; q < w; ++q) {
                    sf += F[i * w + q] * F[q * w + j];
                    sg += G[i * w + q] * G[q * w + j];
                }
                worst_f = std::fmax(worst_f, std::fabs(sf - (i == j ? 1.0L : 0.0L)));
                if (i >= 1 && j >= 1) worst_g = std::fmax(worst_g, std::fabs(sg - (i == j ? 1.0L : 0.0L)));
                const bool even = (i + j + n) % 2 == 0;
                expect(even || F[i * w + j] == 0, "F chequerboard", n);
                expect((!even && i >= 1 && j >= 1) || G[i * w + j] == 0, "G chequerboard", n);
                const long double d_i = i == 0 ? 2.0L : 1.0L, d_j = j == 0 ? 2.0L : 1.0L;
                expect(FL[i * w + j] == d_i * F[j * w + i] / d_j, "FL = D F^T D^-1", n);
                expect(GL[i * w + j] == G[j * w + i], "GL = G^T", n);
            }
        // entries are exact up to the rounding of long double; squares of the largest
        // entries bound the rounding of the products
        expect(worst_f <= 1e-17L * scale * scale * w, "F^2 = I", n);
        expect(worst_g <= 1e-17L * scale * scale * w, "G^2 = I", n);
    }
    for (int m = 0; m < 8; ++m)
        for (int o = m; o < 12; ++o)
            for (int i = m; i < 12; ++i)
                for (int k = 0; k < 3; ++k)
                    expect(std::isfinite((double)z_coefficient((ZKind)k, m, o, i, true)), "z coefficient", m);
    std::printf("tables_check: %d failures\n", fails);
    return fails ? 1 : 0;
}
