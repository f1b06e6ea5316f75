"""GPU parity of the single-height M2L (eq. m2lkernels, left: the double-height sum truncated
at n + k <= P - 1) against the CPU oracle, through the C ABI.

Same metric and bounds as the double-height parity tests: per-degree relative error in the
normalised basis, 1e-12 FP64 (against the long-double oracle, conditioned as there) and
1e-5 FP32, or twice the error of a plain FP32 evaluation of the same translation where that
is larger (gpu_util.Plain32).
"""
import numpy as np
import pytest

import oracle
import paper_2202_02847_amd as sh
from paper_2202_02847_amd import workloads as wl
from gpu_util import TOL, Plain32, check, run_batch, torch_dev
from refmath import size

pytestmark = pytest.mark.gpu

DTYPES = [sh.SH_F64, sh.SH_F32]
DT_ID = {sh.SH_F64: "f64", sh.SH_F32: "f32"}
# fixed-order kernel (2..16, 13..16 with one block per CU) and general kernel (1, 17..31)
ORDERS = [1, 2, 5, 10, 13, 16, 17, 24, 30]


@pytest.fixture(scope="module")
def ctx():
    c = sh.Context(max_order=32, device=0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def _inputs(orc, P, count, seed):
    """Multipoles of 12-point unit clusters (P2M), shifts of length 2..4 in random
    directions, a few on or near the z axis and along x and y."""
    rng = np.random.default_rng(seed)
    pts, q = wl.clusters(rng, count, 12)
    r = wl.random_shifts(rng, count, 2.0, 4.0)
    if count >= 8:
        r[0] = [0, 0, 2.1]
        r[1] = [0, 0, -2.2]
        r[2] = [1e-9, -1e-9, 3.9]
        r[3] = [2.05, 0, 0]
        r[4] = [0, -2.05, 0]
    M = orc.p2m_batch(P, np.zeros((count, 3)), pts, q)
    return r, M


def _refs(orc, dtype, P, r, M):
    ref = orc.m2l_single_batch(P, r, M)
    if dtype == sh.SH_F64:
        return ref, oracle.get("longdouble").m2l_single_batch(P, r, M, nthreads=8).astype(np.float64), None
    p32 = Plain32(lambda rr, CC: orc.m2l_single_batch(P, rr, CC, nthreads=8), P, P, "M", "L", r, M)
    return ref, None, p32


@pytest.mark.parametrize("dtype", DTYPES, ids=DT_ID.get)
@pytest.mark.parametrize("P", ORDERS)
def test_single_height_matches_oracle(ctx, orc, dtype, P):
    count = 67 if P <= 16 else 19  # ragged: not a multiple of the wavefront
    print(f"[single-height] dtype={DT_ID[dtype]} P={P} count={count}", flush=True)
    r, M = _inputs(orc, P, count, 3000 + P)
    ref, ref_ld, p32 = _refs(orc, dtype, P, r, M)
    got, _ = run_batch(ctx, "m2l", dtype, P, P, r, M, flags=sh.SH_SINGLE_HEIGHT)
    check(got, ref, P, "L", TOL[dtype], f"single-height {DT_ID[dtype]} P={P}", ref_ld, p32)
    assert ctx.device_error() == 0


def test_single_height_accumulate_and_indexed(ctx, orc):
    """SH_ACCUMULATE together with the flag, and the gather/scatter form over pools."""
    torch, dev = torch_dev()
    P, count = 10, 130
    S = size(P)
    r, M = _inputs(orc, P, count, 41)
    ref = orc.m2l_single_batch(P, r, M)
    rng = np.random.default_rng(42)
    init = rng.normal(size=(count, S)) * 1e-3
    init[:, [n * (n + 1) + 1 for n in range(P)]] = 0.0
    got, _ = run_batch(ctx, "m2l", sh.SH_F64, P, P, r, M, flags=sh.SH_SINGLE_HEIGHT | sh.SH_ACCUMULATE,
                       out_init=init)
    check(got - init, ref, P, "L", 1e-11, "single-height accumulate")
    src = rng.permutation(count).astype(np.int64)
    dst = rng.permutation(count + 20)[:count].astype(np.int64)
    d_in = torch.from_numpy(M[src.argsort()].copy()).to(dev)  # pool slot src[i] holds M[i]
    d_out = torch.zeros((count + 20, S), dtype=torch.float64, device=dev)
    sh.sh_translate_indexed(ctx, "m2l", sh.SH_F64, P, P, count, torch.from_numpy(r).to(dev),
                            torch.from_numpy(src).to(dev), d_in, S, torch.from_numpy(dst).to(dev), d_out, S,
                            sh.SH_SINGLE_HEIGHT)
    torch.cuda.synchronize()
    out = d_out.cpu().numpy()
    check(out[dst], ref, P, "L", TOL[sh.SH_F64], "single-height indexed")


def test_single_height_differs_from_double(ctx, orc):
    """The flag changes the result: row 0 equals the double-height row 0, the other rows
    differ by the dropped terms (far above the parity bound)."""
    P, count = 10, 64
    r, M = _inputs(orc, P, count, 43)
    s, _ = run_batch(ctx, "m2l", sh.SH_F64, P, P, r, M, flags=sh.SH_SINGLE_HEIGHT)
    d, _ = run_batch(ctx, "m2l", sh.SH_F64, P, P, r, M)
    assert np.allclose(s[:, :2], d[:, :2], rtol=1e-13, atol=0)
    rel = np.max(np.abs(s - d), axis=1) / np.max(np.abs(d), axis=1)
    assert float(np.min(rel)) > 1e-9


def test_single_height_rejected_where_undefined(ctx):
    torch, dev = torch_dev()
    x = torch.zeros((4, 110), dtype=torch.float64, device=dev)
    for op, p_in, p_out in (("m2l", 10, 8), ("m2m", 10, 10), ("l2l", 10, 10)):
        with pytest.raises(sh.ShError):
            sh.sh_translate_batch(ctx, op, sh.SH_F64, p_in, p_out, 1, x, x, 110, x, 110, sh.SH_SINGLE_HEIGHT)
    with pytest.raises(sh.ShError):
        sh.sh_m2l_naive_batch_f64(ctx, 10, 10, 1, x, x, 110, x, 110, sh.SH_SINGLE_HEIGHT)


def test_single_height_full_size_sampled(ctx, orc):
    """The uniform-octree M2L batch at P = 10 (2^20 translations) with the flag, checked on
    sampled translations."""
    torch, dev = torch_dev()
    P, n = 10, 1 << 20
    c = wl.config2(n_m2l=n, n_child=8, P=P)
    M = orc.p2m_batch(P, np.zeros((n, 3)), c["pts"], c["q"], nthreads=16)
    d_M = torch.from_numpy(M).to(dev)
    d_r = torch.from_numpy(c["r_m2l"]).to(dev)
    d_L = torch.empty((n, size(P)), dtype=torch.float64, device=dev)
    sh.sh_m2l_batch_f64(ctx, P, P, n, d_r, d_M, size(P), d_L, size(P), sh.SH_SINGLE_HEIGHT)
    torch.cuda.synchronize()
    rng = np.random.default_rng(P)
    idx = np.unique(np.concatenate([[0, 1, 63, 64, n - 1], rng.integers(0, n, 250)]))
    got = d_L[torch.from_numpy(idx).to(dev)].cpu().numpy()
    ref = orc.m2l_single_batch(P, c["r_m2l"][idx], M[idx])
    ref_ld = oracle.get("longdouble").m2l_single_batch(P, c["r_m2l"][idx], M[idx], nthreads=8).astype(np.float64)
    check(got, ref, P, "L", TOL[sh.SH_F64], "single-height octree P=10", ref_ld)
    assert ctx.device_error() == 0
