"""sh_translate_single_noalloc: the single host-pointer translation staged through the
library's fixed device array instead of a per-call allocation.  Its result must equal the
allocating single call's bit for bit (same kernel, same staging layout) and the oracle within
the dtype's tolerance, on consecutive calls whose staging shrinks (the array keeps the
previous call's contents)."""
import numpy as np
import pytest

import oracle
import paper_2202_02847_amd as sh
from paper_2202_02847_amd import workloads as wl
from gpu_util import IN_KIND, OUT_KIND, TOL, check, from_basis, ld_ref, plain32_for, to_basis, torch_dev

pytestmark = pytest.mark.gpu

SINGLE = {(op, dt): getattr(sh, f"sh_{op}_{'f64' if dt == sh.SH_F64 else 'f32'}")
          for op in ("m2l", "m2m", "l2l") for dt in (sh.SH_F64, sh.SH_F32)}
LENGTHS = {"m2l": (2.0, 4.0), "m2m": (0.25, 0.5), "l2l": (0.25, 0.5)}


@pytest.fixture(scope="module")
def ctx():
    torch_dev()
    c = sh.Context(max_order=64, device=0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def _case(orc, op, p_in, seed):
    rng = np.random.default_rng(seed)
    pts, q = wl.clusters(rng, 1, 16)
    r = wl.random_shifts(rng, 1, *LENGTHS[op])
    if op == "l2l":
        C = orc.p2l_batch(p_in, np.zeros((1, 3)), pts + np.array([2.5, -1.0, 1.5]), q)
    else:
        C = orc.p2m_batch(p_in, np.zeros((1, 3)), pts, q)
    return r, C


# (op, dtype, p_in, p_out) of two consecutive calls: the second stages fewer reals
SEQUENCES = [
    [("m2l", sh.SH_F64, 30, 30), ("m2l", sh.SH_F64, 6, 5)],
    [("m2m", sh.SH_F64, 12, 16), ("l2l", sh.SH_F64, 9, 4)],
    [("m2l", sh.SH_F32, 16, 16), ("l2l", sh.SH_F32, 7, 7)],
    [("l2l", sh.SH_F32, 24, 20), ("m2m", sh.SH_F64, 3, 3)],
]


@pytest.mark.parametrize("seq", SEQUENCES, ids=lambda s: "+".join(f"{o}{a}-{b}" for o, _, a, b in s))
def test_noalloc_matches_single_call_twice(ctx, orc, seq):
    for k, (op, dt, p_in, p_out) in enumerate(seq):
        print(f"[noalloc] call {k}: {op} dtype={dt} {p_in}->{p_out}", flush=True)
        r, C = _case(orc, op, p_in, 40 + 7 * k + p_in)
        npdt = np.float64 if dt == sh.SH_F64 else np.float32
        r_in = r[0].astype(npdt)
        c_in = to_basis(C[0], p_in, IN_KIND[op], dt).astype(npdt)
        got = sh.sh_translate_single_noalloc(ctx, op, dt, p_in, p_out, r_in, c_in)
        want = SINGLE[(op, dt)](ctx, p_in, p_out, r_in, c_in)
        assert got.dtype == want.dtype
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), "differs from the allocating call"
        Cin = from_basis(c_in, p_in, IN_KIND[op], dt)[None, :]
        ref = orc.translate_batch(op, p_in, p_out, r_in.astype(np.float64)[None, :], Cin)
        g = from_basis(got, p_out, OUT_KIND[op], dt)[None, :]
        if dt == sh.SH_F64:
            check(g, ref, p_out, OUT_KIND[op], TOL[dt], f"noalloc {op}", ld_ref(op, p_in, p_out, r_in[None, :], Cin))
        else:
            check(g, ref, p_out, OUT_KIND[op], TOL[dt], f"noalloc {op}",
                  plain32=plain32_for(orc, op, p_in, p_out, r_in[None, :], Cin))
    assert ctx.device_error() == 0


def test_noalloc_errors(ctx):
    x = np.zeros(3)
    c = np.zeros(12)
    with pytest.raises(sh.ShError) as e:
        sh.sh_translate_single_noalloc(ctx, "m2l", sh.SH_F64, 3, 3, x, c)  # M2L with r = 0
    assert e.value.status == sh.SH_ESHIFT
    with pytest.raises(sh.ShError) as e:
        sh.sh_translate_single_noalloc(ctx, "m2l", sh.SH_F64, 65, 3, np.ones(3), np.zeros(65 * 66))
    assert e.value.status == sh.SH_EORDER
    L = sh.lib()
    assert L.sh_translate_single_noalloc(sh._h(ctx), 7, sh.SH_F64, 3, 3, np.ones(3).ctypes.data, c.ctypes.data,
                                         c.ctypes.data) == sh.SH_EINVAL
    assert L.sh_translate_single_noalloc(None, 1, 0, 3, 3, None, None, None) == sh.SH_EINVAL
