"""The library's exact swap tables against the paper and against the oracle (no GPU).

* The M-side matrices F, G must map the regular harmonics of a point to those of the
  point with x and z swapped (R' = B^T R, eq. swaptransform for M); the L-side FL, GL
  must do the same for the singular harmonics (S' = B S, the L rule).  The harmonics
  come from the oracle, so this pins the tables to the definitions.
* B_1 and B_2 from the exact-rational fixture (Appendix recurrence).
* One rounding: entries equal the correctly rounded exact rationals (C14 reading).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import paper_2202_02847_amd as sh
from refmath import pos

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _split(C, n):
    re = np.array([C[pos(n, m)] for m in range(n + 1)])
    im = np.array([C[pos(n, m) + 1] if m else 0.0 for m in range(n + 1)])
    return re, im


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 8, 11])
def test_M_side_swaps_regular_harmonics(n):
    o = oracle.get()
    F = sh.sh_swap_matrix_f64(n, 0)
    G = sh.sh_swap_matrix_f64(n, 1)
    rng = np.random.default_rng(n)
    for _ in range(3):
        y = rng.normal(size=3)
        a = o.regular(y, n + 1)
        b = o.regular(y[[2, 1, 0]], n + 1)
        are, aim = _split(a, n)
        bre, bim = _split(b, n)
        scale = max(np.max(np.abs(bre)), np.max(np.abs(bim)), 1e-300)
        assert np.max(np.abs(F @ are - bre)) / scale < 1e-13
        assert np.max(np.abs(G @ aim - bim)) / scale < 1e-13


@pytest.mark.parametrize("n", [0, 1, 2, 4, 7, 10])
def test_L_side_swaps_singular_harmonics(n):
    o = oracle.get()
    FL = sh.sh_swap_matrix_f64(n, 2)
    GL = sh.sh_swap_matrix_f64(n, 3)
    rng = np.random.default_rng(100 + n)
    for _ in range(3):
        y = rng.normal(size=3)
        a = o.singular(y, n + 1)
        b = o.singular(y[[2, 1, 0]], n + 1)
        are, aim = _split(a, n)
        bre, bim = _split(b, n)
        scale = max(np.max(np.abs(bre)), np.max(np.abs(bim)), 1e-300)
        assert np.max(np.abs(FL @ are - bre)) / scale < 1e-12
        assert np.max(np.abs(GL @ aim - bim)) / scale < 1e-12


def test_printed_L_side_transpose_differs_from_FL():
    """FL = D F^T D^-1 with D = diag(2,1,..,1): F^T itself is off by 2 in row/column 0."""
    for n in (2, 5, 9):
        F = sh.sh_swap_matrix_f64(n, 0)
        FL = sh.sh_swap_matrix_f64(n, 2)
        G = sh.sh_swap_matrix_f64(n, 1)
        GL = sh.sh_swap_matrix_f64(n, 3)
        D = np.diag([2.0] + [1.0] * n)
        assert np.allclose(FL, D @ F.T @ np.linalg.inv(D), rtol=1e-14, atol=1e-14)
        assert not np.allclose(FL, F.T)
        assert np.allclose(GL, G.T, rtol=1e-14, atol=1e-14)


def _golden_B():
    B = {}
    for line in open(os.path.join(GOLDEN, "swap_b.txt")):
        if line.startswith("#"):
            continue
        n, m, l, v = line.split()
        B[(int(n), int(m), int(l))] = Fraction(v)
    return B


def test_golden_B1_B2():
    B = _golden_B()
    for n in (1, 2):
        b = lambda m, l: B.get((n, m, l), Fraction(0))  # noqa: E731
        F = np.zeros((n + 1, n + 1)); G = np.zeros_like(F); FL = np.zeros_like(F); GL = np.zeros_like(F)
        for m in range(n + 1):
            for l in range(n + 1):
                s = (-1) ** l
                F[m, l] = b(0, m) if l == 0 else b(l, m) + s * b(-l, m)
                FL[m, l] = b(m, 0) if l == 0 else b(m, l) + s * b(m, -l)
                if l and m:
                    G[m, l] = b(l, m) - s * b(-l, m)
                    GL[m, l] = b(m, l) - s * b(m, -l)
        for k, ref in enumerate((F, G, FL, GL)):
            assert np.array_equal(sh.sh_swap_matrix_f64(n, k), ref), (n, k)


def test_involutions_and_chequerboard():
    for n in range(0, 12):
        F, G, FL, GL = (sh.sh_swap_matrix_f64(n, k) for k in range(4))
        I = np.eye(n + 1)
        Ip = I.copy(); Ip[0, 0] = 0.0
        tol = 1e-12 * max(1.0, np.max(np.abs(F)) ** 2)
        assert np.max(np.abs(F @ F - I)) < tol
        assert np.max(np.abs(FL @ FL - I)) < tol
        assert np.max(np.abs(G @ G - Ip)) < tol
        assert np.max(np.abs(GL @ GL - Ip)) < tol
        for m in range(n + 1):
            for l in range(n + 1):
                if (m + l + n) % 2:
                    assert F[m, l] == 0 and FL[m, l] == 0
                else:
                    assert G[m, l] == 0 and GL[m, l] == 0
                if m == 0 or l == 0:
                    assert G[m, l] == 0 and GL[m, l] == 0


def _exact_N(nmax):
    """N_n = 2^n B_n by the Appendix recurrence, in Python integers."""
    N = {0: {(0, 0): 1}}
    for n in range(nmax):
        g = N[n].get
        new = {}
        for m in range(-n, n + 1):
            for l in range(-(n + 1), n + 2):
                new[(m, l)] = g((m, l - 1), 0) - g((m, l + 1), 0)
        for l in range(-(n + 1), n + 2):
            new[(n + 1, l)] = g((n, l - 1), 0) + 2 * g((n, l), 0) + g((n, l + 1), 0)
            new[(-(n + 1), l)] = g((-n, l - 1), 0) - 2 * g((-n, l), 0) + g((-n, l + 1), 0)
        N[n + 1] = new
    return N


@pytest.mark.parametrize("n", [20, 29, 40])
def test_tables_rounded_once_from_exact(n):
    N = _exact_N(n)[n]
    F = sh.sh_swap_matrix_f64(n, 0)
    G = sh.sh_swap_matrix_f64(n, 1)
    for m in range(n + 1):
        for l in range(n + 1):
            s = (-1) ** l
            fex = N.get((0, m), 0) if l == 0 else N.get((l, m), 0) + s * N.get((-l, m), 0)
            gex = 0 if (l == 0 or m == 0) else N.get((l, m), 0) - s * N.get((-l, m), 0)
            assert F[m, l] == float(Fraction(fex, 2 ** n)), (m, l)
            assert G[m, l] == float(Fraction(gex, 2 ** n)), (m, l)


def test_normalised_tables_are_similarity_transforms():
    import math
    for n in (3, 9, 16):
        w = np.array([math.sqrt(math.factorial(n + m) * math.factorial(n - m)) for m in range(n + 1)])
        W = np.diag(w)
        Wi = np.diag(1 / w)
        for k, (left, right) in enumerate(((W, Wi), (W, Wi), (Wi, W), (Wi, W))):
            raw = sh.sh_swap_matrix_f64(n, k)
            nrm = sh.sh_swap_matrix_f64(n, k, normalised=True)
            ref = left @ raw @ right
            assert np.max(np.abs(nrm - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))
            # bounded in the normalised basis (the raw F_n grow like 2^n)
            assert np.max(np.abs(nrm)) <= 2.0
