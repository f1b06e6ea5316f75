"""Plants mistakes in copies of the oracle and checks that the pins catch every one.

Each mutant is a textual edit of ``oracle/oracle.c`` (a dropped term, a wrong sign
or index, a transposed operand); the copy is compiled to a temporary library and the
whole pin battery is run on it.  A mutant that passes every pin would mean the
pins cannot tell that mistake from the correct oracle.
"""
import os
import tempfile

import pytest

import oracle
from oracle_pins import PINS

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")

# (name, original text, mutated text, which occurrence (None = all))
MUTANTS = [
    ("m2l_sign_dropped", "real sgn = (n % 2) ? -1 : 1;", "real sgn = 1;", None),
    ("m2l_no_conj", "sr += mr * tr + mi * ti;", "sr += mr * tr - mi * ti;", None),
    ("m2l_transposed_l", "get(S, n + k, m + l, &tr, &ti);", "get(S, n + k, m - l, &tr, &ti);", None),
    ("m2l_last_row_dropped", "for (int k = 0; k < p_in; ++k) {", "for (int k = 0; k < p_in - 1; ++k) {", None),
    ("sym_sign", "real sgn = (am % 2) ? -1 : 1;", "real sgn = 1;", None),
    ("R_diag_factor", "/ (2 * n);", "/ (2 * n - 1);", None),
    ("R_column_sign", "((2 * n - 1) * z * a - r2 * b)", "((2 * n - 1) * z * a + r2 * b)", None),
    ("S_diag_factor", "(2 * n - 1) * (x * pr - y * pi) / r2", "(2 * n + 1) * (x * pr - y * pi) / r2", None),
    ("S_column_index", "((real)(n - 1) * (n - 1) - (real)m * m)", "((real)n * n - (real)m * m)", None),
    ("m2m_plus_r", "real mr_[3] = {-r[0], -r[1], -r[2]};", "real mr_[3] = {r[0], r[1], r[2]};", None),
    ("m2m_index_swap", "get(R, j, i, &ar, &ai);", "get(R, j, -i, &ar, &ai);", None),
    ("l2l_no_conj", "sr += ar * br + ai * bi;\n                    si += ai * br - ar * bi;",
     "sr += ar * br - ai * bi;\n                    si += ai * br + ar * bi;", None),
    ("l2l_index", "int j = n - k, i = m - l;", "int j = n - k, i = l - m;", 1),
    ("eval_l_no_conj", "acc += ar * br + ai * bi;", "acc += ar * br - ai * bi;", 1),
    ("m2l_single_range", "for (int k = 0; k <= P - n - 1; ++k) {", "for (int k = 0; k <= P - n; ++k) {", None),
    ("m2l_single_low_order_S", "    real *S = (real *)malloc(sizeof(real) * (size_t)P * (P + 1));\n    or_singular(r, P, S);",
     "    real *S = (real *)malloc(sizeof(real) * (size_t)P * (P + 1));\n    or_singular(r, P - 1, S);", None),
    ("l2p_dx_sign", "real xr = (ar - br) / 2, xi = (ai - bi) / 2;", "real xr = (br - ar) / 2, xi = (bi - ai) / 2;", None),
    ("l2p_dy_conj", "real yr = -(ai + bi) / 2, yi = (ar + br) / 2;", "real yr = (ai + bi) / 2, yi = -(ar + br) / 2;", None),
    ("l2p_dz_index", "get_r(R, n - 1, m, &cr, &ci);", "get_r(R, n - 1, m + 1, &cr, &ci);", None),
    ("l2p_dx_neighbour", "get_r(R, n - 1, m + 1, &br, &bi);", "get_r(R, n - 1, m, &br, &bi);", None),
    ("l2l_first_term_dropped", "for (int n = k; n < p_in; ++n) {", "for (int n = k + 1; n < p_in; ++n) {", None),
    ("batch_op_codes_swapped", "if (op == 0)\n            or_m2m", "if (op == 2)\n            or_m2m", None),
    ("batch_input_stride_from_ld_out", "const real *src = in + i * ld_in;", "const real *src = in + i * ld_out;",
     None),
    ("p2m_batch_point_stride", "or_p2m(P, centres + 3 * c, npts, pts + 3 * npts * c,",
     "or_p2m(P, centres + 3 * c, npts, pts + npts * c,", None),
]


def _mutate(text, old, new, which):
    assert old in text, old
    if which is None:
        return text.replace(old, new)
    parts = text.split(old)
    assert len(parts) > which + 1, (old, which)
    return old.join(parts[: which + 1]) + new + old.join(parts[which + 1:])


@pytest.mark.parametrize("name,old,new,which", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, old, new, which):
    text = open(SRC).read()
    mutated = _mutate(text, old, new, which)
    assert mutated != text
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "oracle_mut.c")
        lib = os.path.join(d, "liboracle_mut.so")
        open(src, "w").write(mutated)
        oracle.compile_variant(src, lib)
        o = oracle.Oracle("double", path=lib)
        tripped = []
        for pin in PINS:
            try:
                err, bound = pin(o)
                ok = err <= bound
            except Exception:  # a crash / nan also counts as caught
                ok = False
            if not ok:
                tripped.append(pin.__name__)
        assert tripped, f"mutant {name} passed every pin"
