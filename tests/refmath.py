"""Independent closed forms and error metrics used by the tests.

Nothing here is shared with the oracle or the GPU library: the harmonics are
evaluated from their spherical closed forms (associated Legendre functions from
scipy, or mpmath for the high-precision check) instead of the Cartesian
recurrences, so that a mistake in either recurrence shows up as a mismatch.

Closed forms (the normalisation fixed by the Appendix recurrences, Legendre
functions WITHOUT the Condon-Shortley phase):
    R_n^m(r) = |r|^n     P_n^m(cos t) e^{i m p} / (n+m)!
    S_n^m(r) = (n-m)!    P_n^m(cos t) e^{i m p} / |r|^{n+1}
"""
from __future__ import annotations

import cmath
import math

import mpmath
import numpy as np
from scipy.special import lpmv


def pos(n: int, m: int) -> int:
    return n * (n + 1) + 2 * m


def size(P: int) -> int:
    return P * (P + 1)


def _sph(r):
    x, y, z = (float(v) for v in r)
    rho = math.sqrt(x * x + y * y + z * z)
    ct = z / rho if rho != 0 else 1.0
    ph = math.atan2(y, x)
    return rho, ct, ph


def _legendre_no_cs(n, m, ct):
    # scipy's lpmv carries the Condon-Shortley phase (-1)^m; remove it.
    return (-1) ** m * float(lpmv(m, n, ct))


def regular_closed(r, P):
    rho, ct, ph = _sph(r)
    out = np.zeros(size(P))
    for n in range(P):
        for m in range(n + 1):
            v = rho ** n * _legendre_no_cs(n, m, ct) * cmath.exp(1j * m * ph) / math.factorial(n + m)
            out[pos(n, m)] = v.real
            out[pos(n, m) + 1] = v.imag if m else 0.0
    return out


def singular_closed(r, P):
    rho, ct, ph = _sph(r)
    out = np.zeros(size(P))
    for n in range(P):
        for m in range(n + 1):
            v = math.factorial(n - m) * _legendre_no_cs(n, m, ct) * cmath.exp(1j * m * ph) / rho ** (n + 1)
            out[pos(n, m)] = v.real
            out[pos(n, m) + 1] = v.imag if m else 0.0
    return out


def singular_closed_mp(r, P, dps=40):
    """Same closed form in mpmath at ``dps`` digits (complex matrix Z[n, m], m >= 0)."""
    with mpmath.workdps(dps):
        x, y, z = (mpmath.mpf(float(v)) for v in r)
        rho = mpmath.sqrt(x * x + y * y + z * z)
        ct = z / rho
        ph = mpmath.atan2(y, x)
        Z = {}
        for n in range(P):
            for m in range(n + 1):
                Z[(n, m)] = (mpmath.factorial(n - m) * (-1) ** m * mpmath.legenp(n, m, ct)
                             * mpmath.expj(m * ph) / rho ** (n + 1))
        return Z


def to_complex(C, P):
    """Solid -> dict-free complex matrix Z[n, m] (m >= 0), zeros above the diagonal."""
    C = np.asarray(C, dtype=np.float64)
    Z = np.zeros((P, P), complex)
    for n in range(P):
        for m in range(n + 1):
            Z[n, m] = complex(C[pos(n, m)], C[pos(n, m) + 1] if m else 0.0)
    return Z


def weights(P):
    """w_n^m = sqrt((n+m)! (n-m)!), the factor that makes R w and S / w unit-sphere bounded."""
    W = np.ones((P, P))
    for n in range(P):
        for m in range(n + 1):
            W[n, m] = math.sqrt(math.factorial(n + m) * math.factorial(n - m))
    return W


def degree_errors(C, Cref, P, kind):
    """Per-degree relative error in the normalised basis.

    kind 'M' (multipole-type coefficients): C_hat = C * w;  kind 'L': C_hat = C / w.
    Returns an array e[n] = max_m |C_hat - Cref_hat| / max_m |Cref_hat| (0 where the
    reference degree is identically zero and so is the result).
    """
    Z = to_complex(C, P)
    Zr = to_complex(Cref, P)
    W = weights(P)
    if kind == "M":
        Z, Zr = Z * W, Zr * W
    else:
        Z, Zr = Z / W, Zr / W
    e = np.zeros(P)
    for n in range(P):
        den = np.max(np.abs(Zr[n, : n + 1]))
        num = np.max(np.abs(Z[n, : n + 1] - Zr[n, : n + 1]))
        if den == 0:
            e[n] = 0.0 if num == 0 else np.inf
        else:
            e[n] = num / den
    return e


def max_degree_error(C, Cref, P, kind):
    return float(np.max(degree_errors(C, Cref, P, kind)))


def raw_rel_error(C, Cref):
    """Plain max-norm relative difference of two raw coefficient vectors."""
    C = np.asarray(C, np.float64)
    Cref = np.asarray(Cref, np.float64)
    den = np.max(np.abs(Cref))
    return float(np.max(np.abs(C - Cref)) / (den if den else 1.0))
