/*
 * Reference oracle for the solid-harmonic translations (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, slow, obviously-correct CPU implementation of what the translation
 * library computes, written from the definitions in Kirchhart, "solidfmm: A highly
 * optimised library of operations on the solid harmonics for use in fast multipole
 * methods" (arXiv 2202.02847).  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library; the GPU library
 * shares no code, headers, tables or helpers with it.
 *
 * Everything is computed from definitions, never by the rotation scheme:
 *   - regular / singular harmonics R_n^m, S_n^m: the recurrences of the Appendix
 *     ("Regular and Singular Harmonics"), negative m by the symmetry
 *     C_n^{-m} = (-1)^m conj(C_n^m) (Section 2.1);
 *   - P2M / P2L: M_n^m = sum_j q_j R_n^m(y_j - x_A), L_n^m = sum_j q_j S_n^m(y_j - x_B),
 *     the coefficients for which the expansions of eq. (MLexpansions) reproduce
 *     sum_j q_j / |x - y_j| (addition theorem of the harmonics);
 *   - M2L: the double-height kernel of eq. (m2lkernels), right-hand form, summed over
 *     every k < p_in and every l = -k..k; mixed orders keep k < p_in, n < p_out;
 *   - M2L, single-height kernel (eq. m2lkernels, left): the same sum truncated at
 *     n + k <= P - 1;
 *   - M2M / L2L (the paper omits them, Section 1.2): the addition theorem
 *     R_n^m(a + b) = sum_{k,l} R_k^l(a) R_{n-k}^{m-l}(b) applied to the definitions:
 *       M'_n^m = sum_{k<=n, k<p_in} sum_l R_{n-k}^{m-l}(-r) M_k^l,
 *       L'_k^l = sum_{n=k}^{p_in-1} sum_m L_n^m conj(R_{n-k}^{m-l}(r)),
 *     with r = (new centre) - (old centre), R_j^i = 0 for |i| > j;
 *   - evaluation of an M or L expansion (eq. MLexpansions) and the direct sum
 *     of eq. (nbody) with G = 1/|x - y|;
 *   - L2P: the L expansion's potential and its gradient, each R_n^m differentiated by
 *     the derivative identities of the harmonics (stated at or_l2p).
 *
 * Storage of a solid of order P (Section 2.1, Fig. 1): P(P+1) reals, row n (degree)
 * starting at n(n+1); Re C_n^m at n(n+1) + 2m, Im C_n^m at n(n+1) + 2m + 1,
 * m = 0..n.  Im C_n^0 is ignored on input and written as exactly 0 on output.
 *
 * The arithmetic type is REAL (double by default); building with
 * -DREAL="long double" gives the extended-precision self-check variant.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#define REAL double
#endif
typedef REAL real;

#if defined(ORACLE_LONG_DOUBLE)
#define SQRT sqrtl
#else
#define SQRT sqrt
#endif

/* position of Re C_n^m inside a solid */
static int64_t pos(int n, int m) { return (int64_t)n * (n + 1) + 2 * m; }

/* C_n^m for any |m| <= n, reading the stored m >= 0 half (Section 2.1 symmetry). */
static void get(const real *C, int n, int m, real *re, real *im)
{
    int am = m < 0 ? -m : m;
    real a = C[pos(n, am)];
    real b = (am == 0) ? 0 : C[pos(n, am) + 1];
    if (m < 0) {
        real sgn = (am % 2) ? -1 : 1;
        *re = sgn * a;
        *im = -sgn * b;
    } else {
        *re = a;
        *im = b;
    }
}

/* R_n^m(r), 0 <= m <= n < P, by the Appendix recurrences. */
void or_regular(const real *r, int P, real *R)
{
    real x = r[0], y = r[1], z = r[2];
    real r2 = x * x + y * y + z * z;
    if (P <= 0) return;
    memset(R, 0, sizeof(real) * (size_t)P * (P + 1));
    R[pos(0, 0)] = 1;
    /* diagonal: R_n^n = (x + iy)/(2n) R_{n-1}^{n-1} */
    for (int n = 1; n < P; ++n) {
        real pr = R[pos(n - 1, n - 1)], pi = R[pos(n - 1, n - 1) + 1];
        R[pos(n, n)]     = (x * pr - y * pi) / (2 * n);
        R[pos(n, n) + 1] = (x * pi + y * pr) / (2 * n);
    }
    /* columns: (n^2 - m^2) R_n^m = (2n-1) z R_{n-1}^m - |r|^2 R_{n-2}^m */
    for (int m = 0; m < P; ++m) {
        for (int n = m + 1; n < P; ++n) {
            for (int c = 0; c < 2; ++c) {
                real a = R[pos(n - 1, m) + c];
                real b = (n - 2 >= m) ? R[pos(n - 2, m) + c] : 0;
                R[pos(n, m) + c] = ((2 * n - 1) * z * a - r2 * b) / ((real)n * n - (real)m * m);
            }
        }
    }
}

/* S_n^m(r), 0 <= m <= n < P, by the Appendix recurrences (r != 0). */
void or_singular(const real *r, int P, real *S)
{
    real x = r[0], y = r[1], z = r[2];
    real r2 = x * x + y * y + z * z;
    if (P <= 0) return;
    memset(S, 0, sizeof(real) * (size_t)P * (P + 1));
    S[pos(0, 0)] = 1 / SQRT(r2);
    /* diagonal: S_n^n = (2n-1) (x + iy)/|r|^2 S_{n-1}^{n-1} */
    for (int n = 1; n < P; ++n) {
        real pr = S[pos(n - 1, n - 1)], pi = S[pos(n - 1, n - 1) + 1];
        S[pos(n, n)]     = (2 * n - 1) * (x * pr - y * pi) / r2;
        S[pos(n, n) + 1] = (2 * n - 1) * (x * pi + y * pr) / r2;
    }
    /* columns: |r|^2 S_n^m = (2n-1) z S_{n-1}^m - ((n-1)^2 - m^2) S_{n-2}^m */
    for (int m = 0; m < P; ++m) {
        for (int n = m + 1; n < P; ++n) {
            for (int c = 0; c < 2; ++c) {
                real a = S[pos(n - 1, m) + c];
                real b = (n - 2 >= m) ? S[pos(n - 2, m) + c] : 0;
                S[pos(n, m) + c] =
                    ((2 * n - 1) * z * a - ((real)(n - 1) * (n - 1) - (real)m * m) * b) / r2;
            }
        }
    }
}

/* M_n^m = sum_j q_j R_n^m(y_j - x_A) */
void or_p2m(int P, const real *centre, int64_t npts, const real *pts, const real *q, real *M)
{
    int64_t sz = (int64_t)P * (P + 1);
    real *R = (real *)malloc(sizeof(real) * (size_t)sz);
    memset(M, 0, sizeof(real) * (size_t)sz);
    for (int64_t j = 0; j < npts; ++j) {
        real d[3] = {pts[3 * j] - centre[0], pts[3 * j + 1] - centre[1], pts[3 * j + 2] - centre[2]};
        or_regular(d, P, R);
        for (int64_t i = 0; i < sz; ++i) M[i] += q[j] * R[i];
    }
    for (int n = 0; n < P; ++n) M[pos(n, 0) + 1] = 0;
    free(R);
}

/* L_n^m = sum_j q_j S_n^m(y_j - x_B) */
void or_p2l(int P, const real *centre, int64_t npts, const real *pts, const real *q, real *L)
{
    int64_t sz = (int64_t)P * (P + 1);
    real *S = (real *)malloc(sizeof(real) * (size_t)sz);
    memset(L, 0, sizeof(real) * (size_t)sz);
    for (int64_t j = 0; j < npts; ++j) {
        real d[3] = {pts[3 * j] - centre[0], pts[3 * j + 1] - centre[1], pts[3 * j + 2] - centre[2]};
        or_singular(d, P, S);
        for (int64_t i = 0; i < sz; ++i) L[i] += q[j] * S[i];
    }
    for (int n = 0; n < P; ++n) L[pos(n, 0) + 1] = 0;
    free(S);
}

/*
 * M2L, double-height kernel (eq. m2lkernels, right):
 *   L_n^m = (-1)^n sum_{k=0}^{p_in-1} sum_{l=-k}^{k} conj(M_k^l) S_{n+k}^{m+l}(r),
 * r = x_B - x_A, 0 <= m <= n < p_out.
 */
void or_m2l(int p_in, int p_out, const real *r, const real *M, real *L)
{
    int ps = p_in + p_out - 1;
    real *S = (real *)malloc(sizeof(real) * (size_t)ps * (ps + 1));
    or_singular(r, ps, S);
    for (int n = 0; n < p_out; ++n) {
        for (int m = 0; m <= n; ++m) {
            real sr = 0, si = 0;
            for (int k = 0; k < p_in; ++k) {
                for (int l = -k; l <= k; ++l) {
                    real mr, mi, tr, ti;
                    get(M, k, l, &mr, &mi);
                    get(S, n + k, m + l, &tr, &ti);
                    /* conj(M) * S */
                    sr += mr * tr + mi * ti;
                    si += mr * ti - mi * tr;
                }
            }
            real sgn = (n % 2) ? -1 : 1;
            L[pos(n, m)] = sgn * sr;
            L[pos(n, m) + 1] = (m == 0) ? 0 : sgn * si;
        }
    }
    free(S);
}

/*
 * M2L, single-height kernel (eq. m2lkernels, left), one order P for input and output:
 *   L_n^m = (-1)^n sum_{k=0}^{P-n-1} sum_{l=-k}^{k} conj(M_k^l) S_{n+k}^{m+l}(r),
 * so only S up to degree P-1 is needed.
 */
void or_m2l_single(int P, const real *r, const real *M, real *L)
{
    real *S = (real *)malloc(sizeof(real) * (size_t)P * (P + 1));
    or_singular(r, P, S);
    for (int n = 0; n < P; ++n) {
        for (int m = 0; m <= n; ++m) {
            real sr = 0, si = 0;
            for (int k = 0; k <= P - n - 1; ++k) {
                for (int l = -k; l <= k; ++l) {
                    real mr, mi, tr, ti;
                    get(M, k, l, &mr, &mi);
                    get(S, n + k, m + l, &tr, &ti);
                    sr += mr * tr + mi * ti;
                    si += mr * ti - mi * tr;
                }
            }
            real sgn = (n % 2) ? -1 : 1;
            L[pos(n, m)] = sgn * sr;
            L[pos(n, m) + 1] = (m == 0) ? 0 : sgn * si;
        }
    }
    free(S);
}

/* M2M: M'_n^m = sum_{k=0}^{min(n, p_in-1)} sum_{l} R_{n-k}^{m-l}(-r) M_k^l, r = x_new - x_old */
void or_m2m(int p_in, int p_out, const real *r, const real *M, real *Mout)
{
    real mr_[3] = {-r[0], -r[1], -r[2]};
    real *R = (real *)malloc(sizeof(real) * (size_t)p_out * (p_out + 1));
    or_regular(mr_, p_out, R);
    for (int n = 0; n < p_out; ++n) {
        for (int m = 0; m <= n; ++m) {
            real sr = 0, si = 0;
            for (int k = 0; k <= n && k < p_in; ++k) {
                for (int l = -k; l <= k; ++l) {
                    int j = n - k, i = m - l;
                    if (i > j || i < -j) continue;
                    real ar, ai, br, bi;
                    get(R, j, i, &ar, &ai);
                    get(M, k, l, &br, &bi);
                    sr += ar * br - ai * bi;
                    si += ar * bi + ai * br;
                }
            }
            Mout[pos(n, m)] = sr;
            Mout[pos(n, m) + 1] = (m == 0) ? 0 : si;
        }
    }
    free(R);
}

/* L2L: L'_k^l = sum_{n=k}^{p_in-1} sum_{m} L_n^m conj(R_{n-k}^{m-l}(r)), r = x_new - x_old */
void or_l2l(int p_in, int p_out, const real *r, const real *L, real *Lout)
{
    int pr_ = p_in > 0 ? p_in : 1;
    real *R = (real *)malloc(sizeof(real) * (size_t)pr_ * (pr_ + 1));
    or_regular(r, pr_, R);
    for (int k = 0; k < p_out; ++k) {
        for (int l = 0; l <= k; ++l) {
            real sr = 0, si = 0;
            for (int n = k; n < p_in; ++n) {
                for (int m = -n; m <= n; ++m) {
                    int j = n - k, i = m - l;
                    if (i > j || i < -j) continue;
                    real ar, ai, br, bi;
                    get(L, n, m, &ar, &ai);
                    get(R, j, i, &br, &bi);
                    /* L * conj(R) */
                    sr += ar * br + ai * bi;
                    si += ai * br - ar * bi;
                }
            }
            Lout[pos(k, l)] = sr;
            Lout[pos(k, l) + 1] = (l == 0) ? 0 : si;
        }
    }
    free(R);
}

/* Phi_M(x) = Re sum_{n<P} sum_{m=-n}^{n} M_n^m conj(S_n^m(x - x_A))  (eq. MLexpansions) */
real or_eval_m(int P, const real *centre, const real *M, const real *x)
{
    real d[3] = {x[0] - centre[0], x[1] - centre[1], x[2] - centre[2]};
    real *S = (real *)malloc(sizeof(real) * (size_t)P * (P + 1));
    or_singular(d, P, S);
    real acc = 0;
    for (int n = 0; n < P; ++n)
        for (int m = -n; m <= n; ++m) {
            real ar, ai, br, bi;
            get(M, n, m, &ar, &ai);
            get(S, n, m, &br, &bi);
            acc += ar * br + ai * bi; /* Re(a conj(b)) */
        }
    free(S);
    return acc;
}

/* Phi_L(x) = Re sum_{n<P} sum_{m=-n}^{n} L_n^m conj(R_n^m(x - x_B))  (eq. MLexpansions) */
real or_eval_l(int P, const real *centre, const real *L, const real *x)
{
    real d[3] = {x[0] - centre[0], x[1] - centre[1], x[2] - centre[2]};
    real *R = (real *)malloc(sizeof(real) * (size_t)P * (P + 1));
    or_regular(d, P, R);
    real acc = 0;
    for (int n = 0; n < P; ++n)
        for (int m = -n; m <= n; ++m) {
            real ar, ai, br, bi;
            get(L, n, m, &ar, &ai);
            get(R, n, m, &br, &bi);
            acc += ar * br + ai * bi;
        }
    free(R);
    return acc;
}

/* R_n^m(d) for any integer m (zero when |m| > n or n < 0), from a table of R_n^m, m >= 0. */
static void get_r(const real *R, int n, int m, real *re, real *im)
{
    if (n < 0 || m > n || -m > n) {
        *re = 0;
        *im = 0;
        return;
    }
    get(R, n, m, re, im);
}

/*
 * L2P: the potential Phi_L(x) = Re sum_{n<P} sum_{m=-n}^{n} L_n^m conj(R_n^m(x - x_B))
 * (eq. MLexpansions) and its gradient, out = {Phi, dPhi/dx, dPhi/dy, dPhi/dz}.
 * The gradient differentiates each R_n^m; for the harmonics defined by the Appendix
 * recurrences the derivatives are
 *   d/dz R_n^m = R_{n-1}^m,
 *   d/dx R_n^m = (R_{n-1}^{m-1} - R_{n-1}^{m+1}) / 2,
 *   d/dy R_n^m = i (R_{n-1}^{m-1} + R_{n-1}^{m+1}) / 2.
 */
void or_l2p(int P, const real *centre, const real *L, const real *x, real *out)
{
    real d[3] = {x[0] - centre[0], x[1] - centre[1], x[2] - centre[2]};
    real *R = (real *)malloc(sizeof(real) * (size_t)P * (P + 1));
    or_regular(d, P, R);
    real phi = 0, gx = 0, gy = 0, gz = 0;
    for (int n = 0; n < P; ++n)
        for (int m = -n; m <= n; ++m) {
            real lr, li, ar, ai, br, bi, cr, ci;
            get(L, n, m, &lr, &li);
            get(R, n, m, &ar, &ai);
            phi += lr * ar + li * ai; /* Re(L conj(R)) */
            get_r(R, n - 1, m - 1, &ar, &ai);
            get_r(R, n - 1, m + 1, &br, &bi);
            get_r(R, n - 1, m, &cr, &ci);
            /* dR/dx = (A - B)/2, dR/dy = i (A + B)/2 = (-(ai + bi) + i (ar + br))/2, dR/dz = C */
            real xr = (ar - br) / 2, xi = (ai - bi) / 2;
            real yr = -(ai + bi) / 2, yi = (ar + br) / 2;
            gx += lr * xr + li * xi;
            gy += lr * yr + li * yi;
            gz += lr * cr + li * ci;
        }
    free(R);
    out[0] = phi;
    out[1] = gx;
    out[2] = gy;
    out[3] = gz;
}

/* u(x) = sum_j q_j / |x - y_j|  (eq. nbody with G = 1/|x-y|) */
real or_direct(int64_t npts, const real *pts, const real *q, const real *x)
{
    real acc = 0;
    for (int64_t j = 0; j < npts; ++j) {
        real dx = x[0] - pts[3 * j], dy = x[1] - pts[3 * j + 1], dz = x[2] - pts[3 * j + 2];
        acc += q[j] / SQRT(dx * dx + dy * dy + dz * dz);
    }
    return acc;
}

/*
 * Batched forms: translation i reads its shift at r + 3i, its input solid at
 * in + i*ld_in and writes out + i*ld_out.  op: 0 = M2M, 1 = M2L, 2 = L2L.
 * Translations are independent; nthreads > 1 spreads them over OpenMP threads.
 */
void or_translate_batch(int op, int64_t count, int p_in, int p_out, const real *r,
                        const real *in, int64_t ld_in, real *out, int64_t ld_out, int nthreads)
{
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < count; ++i) {
        const real *ri = r + 3 * i;
        const real *src = in + i * ld_in;
        real *dst = out + i * ld_out;
        if (op == 0)
            or_m2m(p_in, p_out, ri, src, dst);
        else if (op == 1)
            or_m2l(p_in, p_out, ri, src, dst);
        else
            or_l2l(p_in, p_out, ri, src, dst);
    }
}

/* Single-height M2L over a batch (same layout as or_translate_batch, p_in = p_out = P). */
void or_m2l_single_batch(int64_t count, int P, const real *r, const real *in, int64_t ld_in, real *out,
                         int64_t ld_out, int nthreads)
{
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < count; ++i)
        or_m2l_single(P, r + 3 * i, in + i * ld_in, out + i * ld_out);
}

/* P2M of many clusters: cluster c has npts points at pts + 3*npts*c, charges q + npts*c. */
void or_p2m_batch(int64_t count, int P, const real *centres, int64_t npts, const real *pts,
                  const real *q, real *M, int64_t ldM, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t c = 0; c < count; ++c)
        or_p2m(P, centres + 3 * c, npts, pts + 3 * npts * c, q + npts * c, M + c * ldM);
}

/* P2L of many clusters (same layout as or_p2m_batch): local expansions about centres. */
void or_p2l_batch(int64_t count, int P, const real *centres, int64_t npts, const real *pts,
                  const real *q, real *L, int64_t ldL, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t c = 0; c < count; ++c)
        or_p2l(P, centres + 3 * c, npts, pts + 3 * npts * c, q + npts * c, L + c * ldL);
}

/* L2P of many boxes: box c has npts targets at pts + 3*npts*c and its local expansion at
 * L + c*ldL; target j of box c writes out[4*(npts*c + j) .. +3] = {Phi, grad Phi}. */
void or_l2p_batch(int64_t count, int P, const real *centres, int64_t npts, const real *pts,
                  const real *L, int64_t ldL, real *out, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t c = 0; c < count; ++c)
        for (int64_t j = 0; j < npts; ++j)
            or_l2p(P, centres + 3 * c, L + c * ldL, pts + 3 * (npts * c + j), out + 4 * (npts * c + j));
}

int or_real_size(void) { return (int)sizeof(real); }
