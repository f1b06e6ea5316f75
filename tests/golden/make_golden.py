"""Writes the exact-rational golden fixtures of this directory.

Every value is the paper's: it comes from a formula the paper prints, evaluated in
exact rational arithmetic (fractions.Fraction); nothing here calls the oracle or
the GPU library.

  zaxis_singular.txt  S_n^m(0,0,R): (n)!/R^{n+1} if m = 0, else 0
                      (Section 2.3, the z-axis special case of the singular harmonics).
  zaxis_m2l.txt       unit z-shift M2L, double-height form (eq. zm2lkernels, right):
                      L_n^m = (-1)^{n+m} sum_{k=m}^{P-1} M_k^m (n+k)!  for a fixed
                      rational M given in the same file.
  swap_b.txt          B_1 and B_2 from the Appendix recurrence
                      2 B_{n+1}^{m,l} = B_n^{m,l-1} - B_n^{m,l+1},
                      2 B_{n+1}^{m+-1,l} = B_n^{m,l-1} +- 2 B_n^{m,l} + B_n^{m,l+1}
                      (second form only for the two new rows m = +-(n+1)).

Run:  python tests/golden/make_golden.py
"""
from fractions import Fraction as Fr
from math import factorial
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def zaxis_singular():
    lines = ["# S_n^m(0,0,R) exact; columns: R n m Re Im   (Section 2.3, z-axis singular harmonics)"]
    for R in (Fr(2), Fr(3, 2)):
        for n in range(12):
            for m in range(n + 1):
                re = Fr(factorial(n)) / R ** (n + 1) if m == 0 else Fr(0)
                lines.append(f"{R} {n} {m} {re} 0")
    return lines


def fixed_M(P):
    # an arbitrary exact multipole: Re M_k^m = (k+1)/(m+2) - 1/3, Im M_k^m = (m - k)/(k+3) (m>0)
    M = {}
    for k in range(P):
        for m in range(k + 1):
            M[(k, m)] = (Fr(k + 1, m + 2) - Fr(1, 3), Fr(m - k, k + 3) if m else Fr(0))
    return M


def zaxis_m2l():
    P = 5
    M = fixed_M(P)
    lines = [f"# unit z-shift M2L (eq. zm2lkernels, right), P={P}",
             "# M lines: 'M k m Re Im'; L lines: 'L n m Re Im'"]
    for (k, m), (a, b) in sorted(M.items()):
        lines.append(f"M {k} {m} {a} {b}")
    for n in range(P):
        for m in range(n + 1):
            re = sum(M[(k, m)][0] * factorial(n + k) for k in range(m, P))
            im = sum(M[(k, m)][1] * factorial(n + k) for k in range(m, P))
            s = -1 if (n + m) % 2 else 1
            lines.append(f"L {n} {m} {s * re} {s * im}")
    return lines


def swap_b():
    B = {0: {(0, 0): Fr(1)}}
    for n in range(0, 2):
        old = B[n]
        g = lambda m, l: old.get((m, l), Fr(0))  # noqa: E731
        new = {}
        for m in range(-n, n + 1):
            for l in range(-(n + 1), n + 2):
                new[(m, l)] = (g(m, l - 1) - g(m, l + 1)) / 2
        for l in range(-(n + 1), n + 2):
            new[(n + 1, l)] = (g(n, l - 1) + 2 * g(n, l) + g(n, l + 1)) / 2
            new[(-(n + 1), l)] = (g(-n, l - 1) - 2 * g(-n, l) + g(-n, l + 1)) / 2
        B[n + 1] = new
    lines = ["# B_n^{m,l} from the Appendix recurrence; columns: n m l value"]
    for n in (1, 2):
        for m in range(-n, n + 1):
            for l in range(-n, n + 1):
                lines.append(f"{n} {m} {l} {B[n][(m, l)]}")
    return lines


def main():
    for name, fn in (("zaxis_singular.txt", zaxis_singular), ("zaxis_m2l.txt", zaxis_m2l),
                     ("swap_b.txt", swap_b)):
        with open(os.path.join(HERE, name), "w") as f:
            f.write("\n".join(fn()) + "\n")


if __name__ == "__main__":
    main()
