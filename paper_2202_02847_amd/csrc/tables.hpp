// Host-side generation of the constant tables of the rotation-based translations.
//
// All tables are produced in exact (integer / extended) arithmetic and rounded once
// to the storage type:
//  * axis-swap matrices: Dehnen's B_n (Appendix, "The Matrices B_n^{m,l}") is built
//    through the integer recurrence for N_n = 2^n B_n, which needs no division:
//      N_{n+1}^{m,l}        = N_n^{m,l-1} - N_n^{m,l+1}                 (|m| <= n)
//      N_{n+1}^{+-(n+1),l}  = N_n^{+-n,l-1} +- 2 N_n^{+-n,l} + N_n^{+-n,l+1}
//    (|N_n| <= 4^n, so __int128 holds every entry up to n = 63).
//  * from B_n, the real/imaginary swap matrices of Section 3.1 (eq. FGmappings):
//      M side:  F^{m,l} = B^{0,m}                 (l = 0),  B^{l,m} + (-1)^l B^{-l,m}  (l > 0)
//               G^{m,l} = B^{l,m} - (-1)^l B^{-l,m}  (m, l > 0), 0 otherwise
//      L side (from L -> B L of eq. swaptransform, folded the same way):
//               FL^{m,l} = B^{m,0}                (l = 0),  B^{m,l} + (-1)^l B^{m,-l}  (l > 0)
//               GL^{m,l} = B^{m,l} - (-1)^l B^{m,-l}  (m, l > 0), 0 otherwise
//    FL equals D F^T D^{-1} with D = diag(2,1,...,1), not F^T itself.
//  * z-axis coefficients (Section 2.3, eq. zm2l-matrix; M2M/L2L by the addition theorem
//    of the regular harmonics along the z axis, R_j^0(0,0,t) = t^j / j!), signs folded in.
//
// Two bases: "raw" (the paper's coefficients; FP64 path) and "normalised"
// (C_hat = C * w for M-type, C / w for L-type, w_n^m = sqrt((n+m)! (n-m)!); FP32 path,
// where raw coefficients and factorials leave the float range).
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

#include "layout.hpp"

namespace shfmm {

constexpr int kMaxOrder = 64;

enum SwapKind { kF = 0, kG = 1, kFL = 2, kGL = 3 };
enum ZKind { kZM2M = 0, kZM2L = 1, kZL2L = 2 };

// dense (n+1)x(n+1) row-major block of degree n starts at swap_offset(n)
inline int64_t swap_offset(int n) { return swap_off(n); }
inline int64_t swap_table_size(int P) { return swap_offset(P); }

// z-coefficient block of column m: (P-m) x (P-m), [out - m][in - m], starts at zoff(P, m)
inline int64_t z_offset(int P, int m)
{
    // sum_{j<m} (P-j)^2
    int64_t s = 0;
    for (int j = 0; j < m; ++j) s += (int64_t)(P - j) * (P - j);
    return s;
}
inline int64_t z_table_size(int P) { return z_offset(P, P); }

// Exact swap matrix entry values for degree n, rounded once to long double / double / float.
// out: (n+1)*(n+1) row-major.  normalised selects the normalised basis.
void swap_matrix_ld(int n, SwapKind kind, bool normalised, long double *out);
// Raw-basis entry (m, l) of degree n, correctly rounded to double from the exact value.
double swap_entry_f64(int n, SwapKind kind, int m, int l);

// Tables are always built for kMaxOrder: the layout (block offsets) then depends on
// compile-time constants only, and kernels can address entries with fixed offsets.
struct HostTables {
    int P = 0;                           // order the layout is built for (kMaxOrder)
    std::vector<double> swap64[4];       // raw basis, FP64
    std::vector<float> swap32[4];        // normalised basis, FP32
    std::vector<double> swap64n[4];      // normalised basis, FP64 (used by the MFMA forms)
    std::vector<double> z64[3];          // raw basis z coefficients, FP64
    std::vector<float> z32[3];           // normalised basis z coefficients, FP32
    std::vector<double> z64n[3];         // normalised basis z coefficients, FP64
    // packed non-zeros (layout.hpp): [0] M side from (F, G), [1] L side from (FL, GL)
    std::vector<double> pk64[2];
    std::vector<float> pk32[2];
    std::vector<double> pk64n[2];
    // MFMA fragments of the block kernel (layout.hpp): [basis: 0 paper, 1 normalised][side] and
    // [basis][op]
    std::vector<double> bsw[2][2];
    std::vector<double> bz[2][3];
};

// Builds every table for orders up to P (1 <= P <= kMaxOrder); sh_create uses kMaxOrder.
void build_tables(int P, HostTables &t);

// Single z coefficient (long double) -- used by build_tables and the host tests.
long double z_coefficient(ZKind kind, int m, int out, int in, bool normalised);

}  // namespace shfmm
