"""The CPU oracle against what the paper and mathematics fix (no GPU)."""
import math

import mpmath
import numpy as np
import pytest

import oracle
from oracle_pins import PINS
from refmath import pos, singular_closed_mp, size


@pytest.fixture(scope="module")
def o64():
    return oracle.get("double")


@pytest.fixture(scope="module")
def old():
    return oracle.get("longdouble")


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin_double(o64, pin):
    err, bound = pin(o64)
    assert err <= bound, f"{pin.__name__}: {err:.3e} > {bound:.1e}"


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin_long_double(old, pin):
    err, bound = pin(old)
    assert err <= bound, f"{pin.__name__}: {err:.3e} > {bound:.1e}"


def _m2l_mp(p_in, p_out, r, M, dps=40):
    """Double-height M2L summed in mpmath with S from its closed form (independent of the recurrence)."""
    with mpmath.workdps(dps):
        S = singular_closed_mp(r, p_in + p_out - 1, dps)

        def sget(n, m):
            if m >= 0:
                return S[(n, m)]
            return (-1) ** (-m) * mpmath.conj(S[(n, -m)])

        def mget(k, l):
            a = complex(M[pos(k, abs(l))], M[pos(k, abs(l)) + 1] if l else 0.0)
            v = mpmath.mpc(a.real, a.imag)
            return v if l >= 0 else (-1) ** (-l) * mpmath.conj(v)

        out = {}
        for n in range(p_out):
            for m in range(n + 1):
                acc = mpmath.mpc(0)
                for k in range(p_in):
                    for l in range(-k, k + 1):
                        acc += mpmath.conj(mget(k, l)) * sget(n + k, m + l)
                out[(n, m)] = (-1) ** n * acc
        return out


def _exact(v):
    a, b = v.as_integer_ratio()
    return mpmath.mpf(a) / b


@pytest.mark.parametrize("P", [6, 10])
def test_oracle_rounding_certified(o64, old, P):
    """FP64 and long-double oracles against a 40-digit evaluation of the same definition.

    Certifies the rounding of the oracle itself: the per-coefficient error is measured
    against the degree's largest coefficient (normalised basis, weights sqrt((n+m)!(n-m)!))."""
    rng = np.random.default_rng(100 + P)
    pts = rng.uniform(-0.5, 0.5, (12, 3))
    q = rng.uniform(-1, 1, 12)
    M = o64.p2m(P, [0, 0, 0], pts, q)
    r = np.array([1.9, -2.2, 0.7])
    ref = _m2l_mp(P, P, r, M)
    for orc, tol in ((o64, 5e-15), (old, 5e-16)):
        L = orc.m2l(P, P, r, np.asarray(M, orc.dtype))
        for n in range(P):
            w = [math.sqrt(math.factorial(n + m) * math.factorial(n - m)) for m in range(n + 1)]
            scale = max(abs(complex(ref[(n, m)])) / w[m] for m in range(n + 1))
            for m in range(n + 1):
                got = mpmath.mpc(_exact(L[pos(n, m)]), _exact(L[pos(n, m) + 1]))
                err = abs(got - ref[(n, m)]) / w[m] / scale
                assert err < tol, (orc.kind, n, m, float(err))
