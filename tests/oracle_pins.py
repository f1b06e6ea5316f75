"""Pins that tie the CPU oracle to the paper and to mathematics, not to itself.

Each pin takes an oracle instance and returns ``(error, bound)``; the pin holds
when ``error <= bound``.  They are collected in ``PINS`` so that the planted-
mistake test can run the whole battery against deliberately broken copies of
the oracle and check that every planted mistake trips at least one pin.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np

from refmath import pos, size, regular_closed, singular_closed, max_degree_error

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _cluster(rng, n=20, half=0.5, centre=(0, 0, 0)):
    pts = rng.uniform(-half, half, (n, 3)) + np.asarray(centre, float)
    q = rng.uniform(-1, 1, n)
    return pts, q


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _random_solid(rng, P, decay=0.5):
    C = np.zeros(size(P))
    for n in range(P):
        for m in range(n + 1):
            s = decay ** n / math.factorial(n + m) ** 0.5
            C[pos(n, m)] = rng.normal() * s
            C[pos(n, m) + 1] = rng.normal() * s if m else 0.0
    return C


# ---------------------------------------------------------------- harmonics
def pin_regular_closed_form(o):
    """R by the Appendix recurrence == spherical closed form (Legendre, no CS phase)."""
    rng = _rng(11)
    err = 0.0
    for _ in range(4):
        r = rng.normal(size=3) * 1.3
        err = max(err, max_degree_error(o.regular(r, 12), regular_closed(r, 12), 12, "M"))
    return err, 1e-13


def pin_singular_closed_form(o):
    """S by the Appendix recurrence == spherical closed form."""
    rng = _rng(12)
    err = 0.0
    for _ in range(4):
        r = rng.normal(size=3) * 1.3
        err = max(err, max_degree_error(o.singular(r, 12), singular_closed(r, 12), 12, "L"))
    return err, 1e-13


def pin_zaxis_singular_golden(o):
    """S_n^m(0,0,R) == n!/R^{n+1} delta_{m0} (Section 2.3), exact-rational fixture."""
    err = 0.0
    rows = {}
    for line in open(os.path.join(GOLDEN, "zaxis_singular.txt")):
        if line.startswith("#"):
            continue
        R, n, m, re, im = line.split()
        rows.setdefault(R, []).append((int(n), int(m), float(Fraction(re)), float(Fraction(im))))
    for R, entries in rows.items():
        P = 1 + max(e[0] for e in entries)
        S = o.singular([0.0, 0.0, float(Fraction(R))], P)
        for n, m, re, im in entries:
            scale = max(abs(re), 1e-300) if m == 0 else float(Fraction(math.factorial(n))) / float(Fraction(R)) ** (n + 1)
            err = max(err, abs(S[pos(n, m)] - re) / scale, abs(S[pos(n, m) + 1] - im) / scale)
    return err, 4e-16


def pin_regular_diagonal_and_axis(o):
    """R_n^n = (x+iy)^n / (2^n n!) and R_n^0(0,0,z) = z^n / n! (consequences of the Appendix)."""
    rng = _rng(13)
    r = rng.normal(size=3)
    P = 14
    R = o.regular(r, P)
    err = 0.0
    w = complex(r[0], r[1])
    for n in range(P):
        ref = w ** n / (2 ** n * math.factorial(n))
        got = complex(R[pos(n, n)], R[pos(n, n) + 1] if n else 0.0)
        err = max(err, abs(got - ref) / abs(ref))
    z = 1.7
    Rz = o.regular([0.0, 0.0, z], P)
    for n in range(P):
        ref = z ** n / math.factorial(n)
        err = max(err, abs(Rz[pos(n, 0)] - ref) / ref)
        for m in range(1, n + 1):
            err = max(err, abs(Rz[pos(n, m)]) + abs(Rz[pos(n, m) + 1]))
    return err, 1e-14


def pin_addition_theorem(o):
    """1/|x-y| = sum_n sum_m R_n^m(y) conj(S_n^m(x)) for |y| < |x|, error ~ (|y|/|x|)^P."""
    rng = _rng(14)
    worst = 0.0
    for _ in range(3):
        x = _unit(rng) * 2.0
        y = _unit(rng) * 0.5
        exact = 1.0 / np.linalg.norm(x - y)
        for P in (8, 16, 24):
            R = o.regular(y, P)
            S = o.singular(x, P)
            acc = 0.0
            for n in range(P):
                acc += R[pos(n, 0)] * S[pos(n, 0)]
                for m in range(1, n + 1):
                    # m and -m together: 2 Re(R conj(S))
                    acc += 2 * (R[pos(n, m)] * S[pos(n, m)] + R[pos(n, m) + 1] * S[pos(n, m) + 1])
            bound = 2.0 * 0.25 ** P / (1 - 0.25) + 1e-15
            worst = max(worst, abs(acc - exact) / exact / bound)
    return worst, 1.0


# ---------------------------------------------------------------- M2L
def pin_m2l_charge_at_centre(o):
    """A unit charge at x_A: M = (q, 0, ...) and L_n^m = q S_n^m(x_A - x_B) exactly, every degree."""
    rng = _rng(21)
    err = 0.0
    for _ in range(3):
        r = _unit(rng) * rng.uniform(2, 4)
        P = 10
        M = o.p2m(P, [0, 0, 0], [[0.0, 0.0, 0.0]], [0.7])
        L = o.m2l(P, P, r, M)
        ref = 0.7 * singular_closed(-r, P)
        err = max(err, max_degree_error(L, ref, P, "L"))
    return err, 1e-13


def _golden_zaxis_m2l():
    M, L = {}, {}
    for line in open(os.path.join(GOLDEN, "zaxis_m2l.txt")):
        if line.startswith("#"):
            continue
        t, a, b, re, im = line.split()
        (M if t == "M" else L)[(int(a), int(b))] = (float(Fraction(re)), float(Fraction(im)))
    P = 1 + max(k for k, _ in M)
    Mv = np.zeros(size(P))
    for (k, m), (re, im) in M.items():
        Mv[pos(k, m)] = re
        Mv[pos(k, m) + 1] = im
    Lv = np.zeros(size(P))
    for (n, m), (re, im) in L.items():
        Lv[pos(n, m)] = re
        Lv[pos(n, m) + 1] = im
    return P, Mv, Lv


def pin_m2l_zaxis_golden(o):
    """Shift (0,0,1): L_n^m = (-1)^{n+m} sum_{k>=m} M_k^m (n+k)!  (eq. zm2lkernels), exact fixture."""
    P, M, Lref = _golden_zaxis_m2l()
    L = o.m2l(P, P, [0.0, 0.0, 1.0], M)
    return _rel(L, Lref), 1e-15


def pin_m2l_zaxis_scaled(o):
    """Shift (0,0,R): S_{n+k}^{m+l}(0,0,R) = delta (n+k)!/R^{n+k+1}, random M, mixed orders."""
    rng = _rng(22)
    err = 0.0
    for (p_in, p_out, R) in ((6, 6, 2.5), (7, 4, 3.0), (3, 8, 2.2)):
        M = _random_solid(rng, p_in)
        for sgn in (1.0, -1.0):
            L = o.m2l(p_in, p_out, [0.0, 0.0, sgn * R], M)
            ref = np.zeros(size(p_out))
            for n in range(p_out):
                for m in range(n + 1):
                    for c in (0, 1):
                        if c == 1 and m == 0:
                            continue
                        acc = 0.0
                        for k in range(m, p_in):
                            # S at (0,0,-R) picks up (-1)^{n+k}; the (-1)^m of conj(M^{-m}) and
                            # the (-1)^n prefactor combine to (-1)^{n+m}
                            s = 1.0 if sgn > 0 else (-1.0) ** (n + k)
                            acc += s * M[pos(k, m) + c] * math.factorial(n + k) / R ** (n + k + 1)
                        ref[pos(n, m) + c] = (-1) ** (n + m) * acc
            err = max(err, max_degree_error(L, ref, p_out, "L"))
    return err, 1e-14


def pin_m2l_vs_direct(o):
    """P2M -> M2L -> evaluate L == direct sum, error decaying with P (eq. nbody)."""
    rng = _rng(23)
    pts, q = _cluster(rng, 20)
    r = np.array([2.1, -1.3, 1.7])  # |r| ~ 3
    targets = r + rng.uniform(-0.5, 0.5, (6, 3))
    exact = np.array([o.direct(pts, q, t) for t in targets])
    errs = []
    for P in (4, 8, 12, 16):
        M = o.p2m(P, [0, 0, 0], pts, q)
        L = o.m2l(P, P, r, M)
        got = np.array([o.eval_l(P, r, L, t) for t in targets])
        errs.append(np.max(np.abs(got - exact)) / np.max(np.abs(exact)))
    decaying = all(errs[i + 1] < errs[i] * 0.2 for i in range(3))
    # geometric bound with rho = |y|max + |x-xB|max = 0.87 + 0.87 against |r| ~ 3
    ok_abs = errs[-1] < 1e-7
    return (0.0 if (decaying and ok_abs) else 1.0), 0.5


def pin_m2l_single_zaxis(o):
    """Single-height M2L (eq. m2lkernels, left) on the z axis: with S_j^i(0,0,R) =
    delta_{i0} j!/R^{j+1}, L_n^m = (-1)^{n+m} sum_{k=m}^{P-1-n} (n+k)! M_k^m / R^{n+k+1}
    (the z-axis form of eq. zm2lkernels with the single-height range of k)."""
    rng = _rng(25)
    err = 0.0
    for (P, R) in ((1, 2.0), (2, 2.5), (6, 2.5), (9, 3.0)):
        M = _random_solid(rng, P)
        for sgn in (1.0, -1.0):
            L = o.m2l_single(P, [0.0, 0.0, sgn * R], M)
            ref = np.zeros(size(P))
            for n in range(P):
                for m in range(n + 1):
                    for c in (0, 1):
                        if c == 1 and m == 0:
                            continue
                        acc = 0.0
                        for k in range(m, P - n):
                            s = 1.0 if sgn > 0 else (-1.0) ** (n + k)
                            acc += s * M[pos(k, m) + c] * math.factorial(n + k) / R ** (n + k + 1)
                        ref[pos(n, m) + c] = (-1) ** (n + m) * acc
            err = max(err, max_degree_error(L, ref, P, "L"))
    return err, 1e-14


def pin_m2l_single_vs_double_and_direct(o):
    """Single height keeps the terms n + k <= P-1 of the double-height sum: row 0 equals the
    double-height row 0, and a multipole with rows k < K only gives the double-height rows
    n <= P-K.  Its expansion reproduces the direct potential with an error that decays in P
    (eq. nbody), and a charge at the centre gives L_n^m = (-1)^n q S_n^m(r) (closed form);
    the batch form equals the single calls."""
    rng = _rng(26)
    err = 0.0
    pts, q = _cluster(rng, 20)
    r = np.array([2.1, -1.3, 1.7])
    for P in (5, 10):
        M = o.p2m(P, [0, 0, 0], pts, q)
        Ls, Ld = o.m2l_single(P, r, M), o.m2l(P, P, r, M)
        err = max(err, _rel(Ls[: size(1)], Ld[: size(1)]))
        K = 3
        Mk = M.copy()
        Mk[size(K):] = 0.0
        Ls, Ld = o.m2l_single(P, r, Mk), o.m2l(P, P, r, Mk)
        err = max(err, _rel(Ls[: size(P - K + 1)], Ld[: size(P - K + 1)]))
    targets = r + rng.uniform(-0.5, 0.5, (6, 3))
    exact = np.array([o.direct(pts, q, t) for t in targets])
    errs = []
    for P in (4, 8, 12, 16):
        M = o.p2m(P, [0, 0, 0], pts, q)
        L = o.m2l_single(P, r, M)
        got = np.array([o.eval_l(P, r, L, t) for t in targets])
        errs.append(np.max(np.abs(got - exact)) / np.max(np.abs(exact)))
    if not (all(errs[i + 1] < errs[i] * 0.5 for i in range(3)) and errs[-1] < 1e-5):
        err = max(err, 1.0)
    P = 8
    L = o.m2l_single(P, r, o.p2m(P, [0, 0, 0], [[0.0, 0.0, 0.0]], [0.7]))
    ref = np.zeros(size(P))
    Sc = singular_closed(r, P)
    for n in range(P):
        for m in range(n + 1):
            ref[pos(n, m)] = (-1) ** n * 0.7 * Sc[pos(n, m)]
            ref[pos(n, m) + 1] = (-1) ** n * 0.7 * Sc[pos(n, m) + 1] if m else 0.0
    err = max(err, max_degree_error(L, ref, P, "L"))
    rs = rng.normal(size=(3, 3)) * 2 + 3
    Ms = np.stack([_random_solid(rng, 7) for _ in range(3)])
    Lb = o.m2l_single_batch(7, rs, Ms, nthreads=2)
    for i in range(3):
        err = max(err, _rel(Lb[i], o.m2l_single(7, rs[i], Ms[i])))
    return err, 1e-13


def pin_m2l_mixed_orders(o):
    """The rows of a small p_out are the leading rows of a larger p_out (same p_in)."""
    rng = _rng(24)
    pts, q = _cluster(rng, 10)
    M = o.p2m(9, [0, 0, 0], pts, q)
    r = _unit(rng) * 3.0
    big = o.m2l(9, 12, r, M)
    small = o.m2l(9, 5, r, M)
    return _rel(small, big[: size(5)]), 0.0


# ---------------------------------------------------------------- M2M
def pin_m2m_exact(o):
    """M2M of P2M at x_A equals P2M at x_A + r (exact for truncated M2M)."""
    rng = _rng(31)
    err = 0.0
    for P in (6, 12):
        pts, q = _cluster(rng, 15)
        M = o.p2m(P, [0, 0, 0], pts, q)
        r = _unit(rng) * rng.uniform(0.25, 0.5)
        ref = o.p2m(P, r, pts, q)
        err = max(err, max_degree_error(o.m2m(P, P, r, M), ref, P, "M"))
    return err, 1e-13


def pin_m2m_composition(o):
    """M2M(a) then M2M(b) == M2M(a+b), and M2M(0) is the identity."""
    rng = _rng(32)
    P = 10
    pts, q = _cluster(rng, 15)
    M = o.p2m(P, [0, 0, 0], pts, q)
    a = _unit(rng) * 0.3
    b = _unit(rng) * 0.4
    two = o.m2m(P, P, b, o.m2m(P, P, a, M))
    one = o.m2m(P, P, a + b, M)
    e1 = max_degree_error(two, one, P, "M")
    e0 = _rel(o.m2m(P, P, [0.0, 0.0, 0.0], M), M)
    return max(e1, e0), 1e-13


def pin_m2m_mixed_orders(o):
    """p_in < p_out: rows n < p_in are exact; rows n >= p_in equal P2M of the truncated input."""
    rng = _rng(33)
    pts, q = _cluster(rng, 12)
    p_in, p_out = 5, 9
    Mbig = o.p2m(p_out, [0, 0, 0], pts, q)
    Min = Mbig[: size(p_in)]
    r = _unit(rng) * 0.4
    out = o.m2m(p_in, p_out, r, Min)
    padded = np.zeros(size(p_out))
    padded[: size(p_in)] = Min
    ref = o.m2m(p_out, p_out, r, padded)
    ref_exact = o.p2m(p_out, r, pts, q)
    e1 = _rel(out, ref)
    e2 = max_degree_error(out[: size(p_in)], ref_exact[: size(p_in)], p_in, "M")
    return max(e1, e2), 1e-13


# ---------------------------------------------------------------- L2L
def pin_l2l_polynomial(o):
    """An L expansion is a polynomial: re-centring preserves its values everywhere."""
    rng = _rng(41)
    err = 0.0
    for P in (5, 10):
        L = _random_solid(rng, P, decay=0.8)
        r = _unit(rng) * rng.uniform(0.25, 0.5)
        L2 = o.l2l(P, P, r, L)
        for _ in range(4):
            x = rng.uniform(-0.6, 0.6, 3)
            a = o.eval_l(P, [0, 0, 0], L, x)
            b = o.eval_l(P, r, L2, x)
            err = max(err, abs(a - b) / max(1e-3, abs(a)))
    return err, 1e-12


def pin_l2l_composition(o):
    """L2L(a) then L2L(b) == L2L(a+b), and L2L(0) is the identity."""
    rng = _rng(42)
    P = 9
    L = _random_solid(rng, P, decay=0.8)
    a = _unit(rng) * 0.3
    b = _unit(rng) * 0.45
    two = o.l2l(P, P, b, o.l2l(P, P, a, L))
    one = o.l2l(P, P, a + b, L)
    e1 = _rel(two, one)
    e0 = _rel(o.l2l(P, P, [0.0, 0.0, 0.0], L), L)
    return max(e1, e0), 1e-13


def pin_l2l_mixed_orders(o):
    """p_out < p_in keeps the leading rows; p_out > p_in gives zero rows k >= p_in."""
    rng = _rng(43)
    L = _random_solid(rng, 8, decay=0.8)
    r = _unit(rng) * 0.4
    full = o.l2l(8, 8, r, L)
    small = o.l2l(8, 5, r, L)
    big = o.l2l(8, 11, r, L)
    e = max(_rel(small, full[: size(5)]), _rel(big[: size(8)], full))
    e = max(e, float(np.max(np.abs(big[size(8):]))))
    return e, 0.0


def pin_l2l_after_m2l_vs_direct(o):
    """P2M -> M2L -> L2L -> evaluate == direct, to the truncation accuracy of the M2L."""
    rng = _rng(44)
    pts, q = _cluster(rng, 20)
    r = np.array([0.0, 3.2, 0.4])
    P = 14
    M = o.p2m(P, [0, 0, 0], pts, q)
    L = o.m2l(P, P, r, M)
    s = np.array([0.2, -0.15, 0.25])
    L2 = o.l2l(P, P, s, L)
    worst = 0.0
    for _ in range(4):
        t = r + s + rng.uniform(-0.2, 0.2, 3)
        worst = max(worst, abs(o.eval_l(P, r + s, L2, t) - o.direct(pts, q, t)) / abs(o.direct(pts, q, t)))
    return worst, 1e-8


def pin_p2l_closed_form_and_near_field(o):
    """P2L (eq. MLexpansions, local side): one charge q at y gives L_n^m = q S_n^m(y - x_B)
    (closed form, Legendre); a cluster about 3.5 away, evaluated within 0.3 of x_B,
    reproduces the direct potential (convergence ratio below 0.12 at P = 20); the batch
    form equals the single calls."""
    rng = _rng(47)
    err = 0.0
    P = 12
    for _ in range(3):
        y = _unit(rng) * rng.uniform(1.5, 3.0)
        xb = rng.uniform(-0.3, 0.3, 3)
        L = o.p2l(P, xb, [y], [0.45])
        err = max(err, max_degree_error(L, 0.45 * singular_closed(y - xb, P), P, "L"))
    P = 20
    pts, q = _cluster(rng, 20, centre=_unit(rng) * 3.5)
    L = o.p2l(P, [0, 0, 0], pts, q)
    for _ in range(4):
        t = _unit(rng) * 0.3
        err = max(err, abs(o.eval_l(P, [0, 0, 0], L, t) - o.direct(pts, q, t)) / abs(o.direct(pts, q, t)))
    centres = rng.uniform(-0.2, 0.2, (3, 3))
    cl = [_cluster(rng, 7, centre=c + [2.5, 0, 1]) for c in centres]
    Lb = o.p2l_batch(9, centres, np.stack([c[0] for c in cl]), np.stack([c[1] for c in cl]), nthreads=2)
    for i, c in enumerate(centres):
        err = max(err, _rel(Lb[i], o.p2l(9, c, cl[i][0], cl[i][1])))
    return err, 1e-12


# ---------------------------------------------------------------- evaluation
def pin_eval_m_far_field(o):
    """The M expansion reproduces the direct potential outside the cluster, error ~ (a/|x|)^P."""
    rng = _rng(51)
    pts, q = _cluster(rng, 20)
    P = 16
    M = o.p2m(P, [0, 0, 0], pts, q)
    worst = 0.0
    for _ in range(4):
        x = _unit(rng) * 4.0
        worst = max(worst, abs(o.eval_m(P, [0, 0, 0], M, x) - o.direct(pts, q, x)) / abs(o.direct(pts, q, x)))
    return worst, 1e-9


def pin_l2p_gradient_finite_difference(o):
    """L2P returns the potential of eq. MLexpansions (the pinned eval_l) and its gradient:
    a fourth-order central difference of eval_l (error O(h^4), the expansion is a
    polynomial) agrees with the returned gradient; the batch form equals the single calls."""
    rng = _rng(52)
    err = 0.0
    h = 1e-3
    for P in (1, 2, 6, 13):
        L = _random_solid(rng, P, decay=0.9)
        c = rng.uniform(-0.2, 0.2, 3)
        for _ in range(3):
            x = c + rng.uniform(-0.5, 0.5, 3)
            out = o.l2p(P, c, L, x)
            phi = o.eval_l(P, c, L, x)
            fd = np.zeros(3)
            for a in range(3):
                e = np.zeros(3)
                e[a] = h
                f = [o.eval_l(P, c, L, x + k * e) for k in (-2, -1, 1, 2)]
                fd[a] = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
            scale = max(1e-3, float(np.max(np.abs(fd))), abs(phi))
            err = max(err, abs(float(out[0]) - phi) / scale, float(np.max(np.abs(out[1:] - fd))) / scale)
    centres = rng.uniform(-0.2, 0.2, (3, 3))
    pts = centres[:, None, :] + rng.uniform(-0.4, 0.4, (3, 5, 3))
    Ls = np.stack([_random_solid(rng, 7) for _ in range(3)])
    ob = o.l2p_batch(7, centres, pts, Ls, nthreads=2)
    for i in range(3):
        for j in range(5):
            err = max(err, _rel(ob[i, j], o.l2p(7, centres[i], Ls[i], pts[i, j])))
    return err, 1e-8


def pin_l2p_vs_direct_field(o):
    """P2L of a far cluster, then L2P, reproduces the direct potential sum q_j/|x - y_j| and
    its gradient -sum q_j (x - y_j)/|x - y_j|^3 (eq. nbody), to the truncation accuracy."""
    rng = _rng(53)
    P = 20
    pts, q = _cluster(rng, 20, centre=_unit(rng) * 3.5)
    L = o.p2l(P, [0, 0, 0], pts, q)
    worst = 0.0
    for _ in range(4):
        t = _unit(rng) * 0.3
        d = t[None, :] - pts
        r = np.linalg.norm(d, axis=1)
        phi = float(np.sum(q / r))
        grad = -np.sum((q / r ** 3)[:, None] * d, axis=0)
        out = o.l2p(P, [0, 0, 0], L, t)
        scale = float(np.max(np.abs(grad)))
        worst = max(worst, abs(float(out[0]) - phi) / abs(phi), float(np.max(np.abs(out[1:] - grad))) / scale)
    return worst, 1e-8


# ---------------------------------------------------------------- batched entry points
def _strided(o, rows, ld, fill):
    a = np.full((rows, ld), fill, dtype=o.dtype)
    return a, a.ctypes.data_as(o._P)


def pin_batch_entry_points(o):
    """The batched forms (every op, mixed orders, padded strides, several threads) equal the
    single calls item by item, bit for bit, and write nothing past each output row.

    The single calls are pinned above against closed forms and the direct sum; this pin
    ties the batched dispatch, the op codes and the ld_in / ld_out strides to them.
    Input padding holds NaN, so a read through the wrong stride shows in the result."""
    rng = _rng(77)
    worst = 0.0
    single = {"m2m": o.m2m, "m2l": o.m2l, "l2l": o.l2l}
    count, sentinel = 23, 7.25
    for op, code in (("m2m", 0), ("m2l", 1), ("l2l", 2)):
        for p_in, p_out in ((7, 7), (5, 9), (9, 4)):
            ld_in, ld_out = size(p_in) + 5, size(p_out) + 3
            C, Cp = _strided(o, count, ld_in, np.nan)
            for i in range(count):
                C[i, : size(p_in)] = _random_solid(rng, p_in)
            lo, hi = (2.0, 4.0) if op == "m2l" else (0.25, 0.6)
            r = np.array([_unit(rng) * rng.uniform(lo, hi) for _ in range(count)], dtype=o.dtype)
            out, outp = _strided(o, count, ld_out, sentinel)
            o._lib.or_translate_batch(code, count, p_in, p_out, r.ctypes.data_as(o._P), Cp, ld_in, outp, ld_out, 3)
            for i in range(count):
                want = single[op](p_in, p_out, r[i], C[i, : size(p_in)])
                got = out[i, : size(p_out)]
                if not np.array_equal(got, want) or not np.all(out[i, size(p_out):] == sentinel):
                    worst = max(worst, _rel(got, want) if np.all(np.isfinite(got)) else np.inf, 1.0)
    # P2M / P2L: cluster c reads its points at pts + 3*npts*c and writes row c of stride ldM
    P, npts = 6, 5
    centres = rng.uniform(-1, 1, (count, 3)).astype(o.dtype)
    pts = (centres[:, None, :] + rng.uniform(-0.5, 0.5, (count, npts, 3))).astype(o.dtype)
    q = rng.uniform(-1, 1, (count, npts)).astype(o.dtype)
    for fn, one in ((o._lib.or_p2m_batch, o.p2m), (o._lib.or_p2l_batch, None)):
        out, outp = _strided(o, count, size(P) + 4, sentinel)
        far = centres if one is not None else centres + 3.0
        fn(count, P, np.ascontiguousarray(far).ctypes.data_as(o._P), npts, pts.ctypes.data_as(o._P),
           q.ctypes.data_as(o._P), outp, size(P) + 4, 2)
        for c in range(count):
            want = (one or o.p2l)(P, far[c], pts[c], q[c])
            if not np.array_equal(out[c, : size(P)], want) or not np.all(out[c, size(P):] == sentinel):
                worst = max(worst, 1.0)
    # single-height M2L batch and L2P batch
    Ms, Msp = _strided(o, count, size(P) + 2, np.nan)
    for i in range(count):
        Ms[i, : size(P)] = _random_solid(rng, P)
    r = np.array([_unit(rng) * rng.uniform(2, 4) for _ in range(count)], dtype=o.dtype)
    out, outp = _strided(o, count, size(P) + 1, sentinel)
    o._lib.or_m2l_single_batch(count, P, r.ctypes.data_as(o._P), Msp, size(P) + 2, outp, size(P) + 1, 2)
    for i in range(count):
        want = o.m2l_single(P, r[i], Ms[i, : size(P)])
        if not np.array_equal(out[i, : size(P)], want) or out[i, size(P)] != sentinel:
            worst = max(worst, 1.0)
    got = o.l2p_batch(P, centres, pts, Ms[:, : size(P)], nthreads=2)
    for c in range(count):
        for j in range(npts):
            if not np.array_equal(got[c, j], o.l2p(P, centres[c], Ms[c, : size(P)], pts[c, j])):
                worst = max(worst, 1.0)
    return worst, 0.0


PINS = [
    pin_regular_closed_form,
    pin_singular_closed_form,
    pin_zaxis_singular_golden,
    pin_regular_diagonal_and_axis,
    pin_addition_theorem,
    pin_m2l_charge_at_centre,
    pin_m2l_zaxis_golden,
    pin_m2l_zaxis_scaled,
    pin_m2l_vs_direct,
    pin_m2l_mixed_orders,
    pin_m2l_single_zaxis,
    pin_m2l_single_vs_double_and_direct,
    pin_m2m_exact,
    pin_m2m_composition,
    pin_m2m_mixed_orders,
    pin_l2l_polynomial,
    pin_l2l_composition,
    pin_l2l_mixed_orders,
    pin_l2l_after_m2l_vs_direct,
    pin_p2l_closed_form_and_near_field,
    pin_eval_m_far_field,
    pin_l2p_gradient_finite_difference,
    pin_l2p_vs_direct_field,
    pin_batch_entry_points,
]
