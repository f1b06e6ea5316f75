"""The C-ABI library loads and exports every symbol its header declares (no GPU needed)."""
import ctypes
import re

import numpy as np
import pytest

import paper_2202_02847_amd as sh


def test_library_built_and_loads():
    L = sh.lib()
    assert L is not None


def test_every_header_symbol_exported():
    names = sh.header_symbols()
    assert len(names) >= 25
    L = ctypes.CDLL(sh.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_mirrors_header_names():
    for n in sh.header_symbols():
        assert hasattr(sh, n), n


def test_binding_constants_match_header():
    """Every #define SH_* and enumerator value of the header equals the binding's constant."""
    text = open(sh.HEADER).read()
    found = {}
    for name, val in re.findall(r"^#define (SH_[A-Z0-9_]+) (\d+)u?\b", text, re.M):
        found[name] = int(val)
    for name, val in re.findall(r"\b(SH_[A-Z0-9_]+) = (-?\d+)", text):
        found[name] = int(val)
    assert len(found) >= 20
    missing = [n for n in found if not hasattr(sh, n)]
    assert not missing, missing
    wrong = {n: (v, getattr(sh, n)) for n, v in found.items() if getattr(sh, n) != v}
    assert not wrong, wrong


def test_strerror_texts():
    for code in (sh.SH_OK, sh.SH_EINVAL, sh.SH_EORDER, sh.SH_ESHIFT, sh.SH_ENOMEM, sh.SH_EDEVICE, sh.SH_EBUSY):
        assert sh.sh_strerror(code)
    assert sh.sh_strerror(12345) == "unknown status"


def test_null_context_rejected():
    L = sh.lib()
    st = L.sh_m2l_batch_f64(None, 8, 8, 10, None, None, 72, None, 72, 0, None)
    assert st == sh.SH_EINVAL
    st = L.sh_translate_batch(None, 1, 0, 8, 8, 0, None, None, 72, None, 72, 0, None)
    assert st == sh.SH_EINVAL
    assert L.sh_max_order(None) == -1


def test_create_argument_checks():
    L = sh.lib()
    h = ctypes.c_void_p()
    assert L.sh_create(None, 8, 0) == sh.SH_EINVAL
    assert L.sh_create(ctypes.byref(h), 0, 0) == sh.SH_EORDER
    assert L.sh_create(ctypes.byref(h), sh.SH_MAX_ORDER + 1, 0) == sh.SH_EORDER
    assert L.sh_create(ctypes.byref(h), 8, -1) == sh.SH_EDEVICE


def test_host_helpers_argument_checks():
    L = sh.lib()
    out = np.zeros(4)
    assert L.sh_swap_matrix_f64(1, 4, 0, out.ctypes.data) == sh.SH_EINVAL
    assert L.sh_swap_matrix_f64(-1, 0, 0, out.ctypes.data) == sh.SH_EORDER
    assert L.sh_swap_matrix_f64(sh.SH_MAX_ORDER, 0, 0, out.ctypes.data) == sh.SH_EORDER
    assert L.sh_normalise_f64(2, 4, 1, out.ctypes.data, 20) == sh.SH_EINVAL


def test_normalise_roundtrip():
    rng = np.random.default_rng(0)
    P = 12
    a = rng.normal(size=(3, P * (P + 1)))
    for kind in (0, 1):
        b = sh.sh_denormalise_f64(kind, P, sh.sh_normalise_f64(kind, P, a))
        assert np.allclose(a, b, rtol=1e-15, atol=0)
    # M-type multiplies by w_n^m = sqrt((n+m)!(n-m)!): degree 3, order 1 -> sqrt(4! 2!)
    one = np.zeros(P * (P + 1))
    one[3 * 4 + 2] = 1.0
    assert np.isclose(sh.sh_normalise_f64(0, P, one)[3 * 4 + 2], np.sqrt(24 * 2))


def test_fmm_orders_for_tolerance():
    """Host-only order selection: one order for every level, growing as the target shrinks,
    the smallest P with 0.15 * 0.444^P <= tol; targets needing an order above the rule's
    measured range (18) and trees outside 2..4 levels refused."""
    prev = 0
    for tol in (0.5, 1e-2, 1e-3, 1e-5, 1e-7):
        for levels in (2, 3, 4):
            orders = sh.sh_fmm_orders_for_tolerance(tol, levels)
            assert len(orders) == levels - 1 and len(set(orders)) == 1
        P = orders[0]
        assert P >= prev
        prev = P
        assert P == 1 or 0.15 * 0.444 ** P <= tol * (1 + 1e-12)
        assert P == 1 or 0.15 * 0.444 ** (P - 1) > tol
    for tol, levels, status in ((0.0, 3, sh.SH_EINVAL), (1.0, 3, sh.SH_EINVAL), (1e-3, 1, sh.SH_EINVAL),
                                (1e-3, 5, sh.SH_EINVAL), (1e-8, 3, sh.SH_EORDER), (1e-15, 3, sh.SH_EORDER)):
        with pytest.raises(sh.ShError) as e:
            sh.sh_fmm_orders_for_tolerance(tol, levels)
        assert e.value.status == status
