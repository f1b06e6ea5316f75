"""GPU parity: every translation kernel against the CPU oracle, through the C ABI.

Metric (per translation): the per-degree relative error in the normalised basis,
max_n ||C_hat_n - C_hat_n^ref||_inf / ||C_hat_n^ref||_inf; bound 1e-12 (FP64) and
1e-5 (FP32), written in gpu_util.TOL.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2202_02847_amd as sh
from paper_2202_02847_amd import workloads as wl
from gpu_util import TOL, IN_KIND, OUT_KIND, check as _check, from_basis, ld_ref as _ld_ref, plain32_for, run_batch, \
    to_basis, torch_dev
from refmath import max_degree_error, size

pytestmark = pytest.mark.gpu

DTYPES = [sh.SH_F64, sh.SH_F32]
DT_ID = {sh.SH_F64: "f64", sh.SH_F32: "f32"}


@pytest.fixture(scope="module")
def ctx():
    c = sh.Context(max_order=48, device=0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def _inputs(orc, op, p_in, count, seed, lengths):
    rng = np.random.default_rng(seed)
    pts, q = wl.clusters(rng, count, 12)
    lo, hi = lengths
    r = wl.random_shifts(rng, count, lo, hi)
    # a few axis-aligned shifts (x = y = 0, both signs) and shifts near the axis
    if count >= 8:
        r[0] = [0, 0, lo + 0.1]
        r[1] = [0, 0, -(lo + 0.2)]
        r[2] = [1e-9, -1e-9, hi - 0.1]
        r[3] = [lo + 0.05, 0, 0]
        r[4] = [0, -(lo + 0.05), 0]
    C = np.zeros((count, size(p_in)))
    for i in range(count):
        if op == "l2l":
            # a local expansion of a far cluster (P2L at a centre ~3 away)
            C[i] = orc.p2l(p_in, [0, 0, 0], pts[i] + np.array([2.5, -1.0, 1.5]), q[i])
        else:
            C[i] = orc.p2m(p_in, [0, 0, 0], pts[i], q[i])
    return r, C


LENGTHS = {"m2l": (2.0, 4.0), "m2m": (0.25, 0.5), "l2l": (0.25, 0.5)}

ORDER_CASES = [(1, 1), (2, 2), (3, 5), (5, 3), (8, 8), (10, 10), (11, 7), (16, 16), (12, 20), (24, 24),
               (30, 30), (40, 40)]


@pytest.mark.parametrize("dtype", DTYPES, ids=DT_ID.get)
@pytest.mark.parametrize("op", ["m2l", "m2m", "l2l"])
@pytest.mark.parametrize("p_in,p_out", ORDER_CASES, ids=[f"{a}-{b}" for a, b in ORDER_CASES])
def test_orders(ctx, orc, op, dtype, p_in, p_out):
    if dtype == sh.SH_F32 and max(p_in, p_out) > 30:
        pytest.skip("FP32 normalised basis is specified up to order 30")
    count = 67 if max(p_in, p_out) <= 16 else 19  # ragged: not a multiple of the wavefront
    print(f"[parity] op={op} dtype={DT_ID[dtype]} p_in={p_in} p_out={p_out} count={count}", flush=True)
    r, C = _inputs(orc, op, p_in, count, 1000 + 37 * p_in + p_out, LENGTHS[op])
    ref = orc.translate_batch(op, p_in, p_out, r, C)
    got, _ = run_batch(ctx, op, dtype, p_in, p_out, r, C)
    ref_ld = _ld_ref(op, p_in, p_out, r, C) if dtype == sh.SH_F64 else None
    p32 = plain32_for(orc, op, p_in, p_out, r, C) if dtype == sh.SH_F32 else None
    _check(got, ref, p_out, OUT_KIND[op], TOL[dtype], f"{op} {DT_ID[dtype]} {p_in}->{p_out}", ref_ld, p32)


@pytest.mark.parametrize("dtype", DTYPES, ids=DT_ID.get)
def test_config1_all_ops(ctx, orc, dtype):
    """The plain-method workload: 1000 each of M2L, M2M, L2L at P=8 (L2L inputs = M2L outputs)."""
    c = wl.config1()
    P = c["P"]
    print(f"[parity] config1 dtype={DT_ID[dtype]}", flush=True)
    M = orc.p2m_batch(P, np.zeros((1000, 3)), c["pts"], c["q"], nthreads=8)
    L = orc.translate_batch("m2l", P, P, c["r_m2l"], M, nthreads=8)
    M2 = orc.translate_batch("m2m", P, P, c["r_m2m"], M, nthreads=8)
    L2 = orc.translate_batch("l2l", P, P, c["r_l2l"], L, nthreads=8)
    for op, r, C, ref in (("m2l", c["r_m2l"], M, L), ("m2m", c["r_m2m"], M, M2), ("l2l", c["r_l2l"], L, L2)):
        got, _ = run_batch(ctx, op, dtype, P, P, r, C)
        p32 = plain32_for(orc, op, P, P, r, C) if dtype == sh.SH_F32 else None
        _check(got, ref, P, OUT_KIND[op], TOL[dtype], f"config1 {op}", plain32=p32)


@pytest.mark.parametrize("dtype", DTYPES, ids=DT_ID.get)
@pytest.mark.parametrize("P", [10, 16, 30])
def test_octree_full_size_sampled(ctx, orc, P, dtype):
    """Octree M2L at the full batch size the benchmark times (2^20 at P=10; P=16, 30 on the
    same generator), checked on sampled translations: FP64 in the paper's basis, FP32 in the
    normalised basis (2^12 samples, 2^10 at P=30)."""
    torch, dev = torch_dev()
    n = 1 << 20 if P <= 16 else 1 << 18
    f32 = dtype == sh.SH_F32
    print(f"[parity] octree full-size P={P} n={n} dtype={DT_ID[dtype]}", flush=True)
    c = wl.config2(n_m2l=n, n_child=8, P=P)
    M = orc.p2m_batch(P, np.zeros((n, 3)), c["pts"], c["q"], nthreads=16)
    S = P * (P + 1)
    rng = np.random.default_rng(P)
    extra = rng.choice(n, (1 << 10 if P > 16 else 1 << 12) if f32 else 250, replace=False)
    idx = np.unique(np.concatenate([[0, 1, 63, 64, n - 1], extra]))
    if f32:
        d_M = torch.from_numpy(to_basis(M, P, "M", dtype)).to(dev)
        d_r = torch.from_numpy(c["r_m2l"].astype(np.float32)).to(dev)
        d_L = torch.empty((n, S), dtype=torch.float32, device=dev)
        sh.sh_m2l_batch_f32(ctx, P, P, n, d_r, d_M, S, d_L, S)
    else:
        d_M = torch.from_numpy(M).to(dev)
        d_r = torch.from_numpy(c["r_m2l"]).to(dev)
        d_L = torch.empty((n, S), dtype=torch.float64, device=dev)
        sh.sh_m2l_batch_f64(ctx, P, P, n, d_r, d_M, S, d_L, S)
    torch.cuda.synchronize()
    got = from_basis(d_L[torch.from_numpy(idx).to(dev)].cpu().numpy(), P, "L", dtype)
    ref = orc.translate_batch("m2l", P, P, c["r_m2l"][idx], M[idx], nthreads=16)
    if f32:
        p32 = plain32_for(orc, "m2l", P, P, c["r_m2l"][idx], M[idx])
        worst = _check(got, ref, P, "L", TOL[dtype], f"octree P={P} f32", plain32=p32)
    else:
        ref_ld = _ld_ref("m2l", P, P, c["r_m2l"][idx], M[idx])
        worst = _check(got, ref, P, "L", TOL[dtype], f"octree P={P}", ref_ld)
    print(f"[parity] octree full-size P={P} {DT_ID[dtype]}: worst C15 error {worst:.2e} over {len(idx)}", flush=True)
    assert ctx.device_error() == 0


@pytest.mark.parametrize("P", [13, 14, 15, 16])
@pytest.mark.parametrize("op", ["m2l", "m2m", "l2l"])
def test_one_block_per_cu_orders(ctx, orc, op, P):
    """FP64 orders 13-16, where a block's 64 solids fill the CU's LDS and each lane reads its
    input rows straight into registers.  Three full blocks and a ragged one; one full block
    holds a zero shift (M2M/L2L identity, M2L error) among valid ones; then the same batch with
    valid shifts, accumulated into an existing output, and gathered/scattered through index
    arrays."""
    torch, dev = torch_dev()
    count = 3 * 64 + 9
    print(f"[parity] one-block-per-CU op={op} P={P} count={count}", flush=True)
    r, C = _inputs(orc, op, P, count, 700 + P, LENGTHS[op])
    r[64 + 17] = 0.0  # inside block 1
    live = np.ones(count, bool)
    live[64 + 17] = False
    ref = np.zeros((count, size(P)))
    ref[live] = orc.translate_batch(op, P, P, r[live], C[live])
    if op != "m2l":
        ref[64 + 17] = C[64 + 17]
        ref[64 + 17, [n * (n + 1) + 1 for n in range(P)]] = 0.0
    ctx.device_error()  # clear
    got, raw = run_batch(ctx, op, sh.SH_F64, P, P, r, C)
    if op == "m2l":
        assert np.isnan(raw[64 + 17]).all()
        assert ctx.device_error() == sh.SH_ESHIFT
    else:
        assert ctx.device_error() == 0
    ref_ld = np.zeros_like(ref)
    ref_ld[live] = _ld_ref(op, P, P, r[live], C[live])
    ref_ld[~live] = ref[~live]
    if op == "m2l":
        live_only = np.flatnonzero(live)
        _check(got[live_only], ref[live_only], P, OUT_KIND[op], TOL[sh.SH_F64], f"{op} P={P}",
               ref_ld[live_only])
    else:
        _check(got, ref, P, OUT_KIND[op], TOL[sh.SH_F64], f"{op} P={P}", ref_ld)

    # valid shifts only, against the oracle
    r2 = r.copy()
    r2[64 + 17] = r[64 + 18]
    plain, _ = run_batch(ctx, op, sh.SH_F64, P, P, r2, C)
    sel = np.arange(64, 128)
    _check(plain[sel], orc.translate_batch(op, P, P, r2[sel], C[sel]), P, OUT_KIND[op], TOL[sh.SH_F64],
           f"{op} P={P} block 1", _ld_ref(op, P, P, r2[sel], C[sel]))
    # accumulate: one FP64 addition per coefficient
    base = plain * np.random.default_rng(P).uniform(-2.0, 2.0, plain.shape)
    acc, _ = run_batch(ctx, op, sh.SH_F64, P, P, r2, C, flags=sh.SH_ACCUMULATE, out_init=base)
    assert np.array_equal(acc, base + plain)

    # indexed gather / scatter over pools: the same arithmetic as the batched call
    npool = count + 40
    rng = np.random.default_rng(P + 1)
    src = rng.integers(0, count, count)
    dst = rng.permutation(npool)[:count]
    pool = torch.from_numpy(np.ascontiguousarray(C)).to(dev)
    outp = torch.zeros((npool, size(P)), dtype=torch.float64, device=dev)
    d_src = torch.from_numpy(src.astype(np.int64)).to(dev)
    d_dst = torch.from_numpy(dst.astype(np.int64)).to(dev)
    d_r = torch.from_numpy(r2).to(dev)
    sh.sh_translate_indexed(ctx, op, sh.SH_F64, P, P, count, d_r, d_src, pool, size(P), d_dst, outp, size(P))
    goti = outp.cpu().numpy()
    gathered, _ = run_batch(ctx, op, sh.SH_F64, P, P, r2, C[src])
    assert np.array_equal(goti[dst], gathered)
    assert (goti[np.setdiff1d(np.arange(npool), dst)] == 0).all()
    assert ctx.device_error() == 0


@pytest.mark.parametrize("p_in,p_out", [(8, 8), (10, 10), (6, 9)])
def test_naive_kernel(ctx, orc, p_in, p_out):
    r, C = _inputs(orc, "m2l", p_in, 45, 7 + p_in, (2.0, 4.0))
    ref = orc.translate_batch("m2l", p_in, p_out, r, C)
    got, _ = run_batch(ctx, "m2l", sh.SH_F64, p_in, p_out, r, C, naive=True)
    _check(got, ref, p_out, "L", TOL[sh.SH_F64], "naive m2l")


def test_p2m_kernel(ctx, orc):
    torch, dev = torch_dev()
    rng = np.random.default_rng(5)
    count, npts, P = 70, 17, 12
    pts, q = wl.clusters(rng, count, npts)
    centres = rng.uniform(-0.1, 0.1, (count, 3))
    pts = pts + centres[:, None, :]
    ref = orc.p2m_batch(P, centres, pts, q)
    d = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in
         (("c", centres), ("p", pts), ("q", q))}
    d_M = torch.zeros((count, P * (P + 1)), dtype=torch.float64, device=dev)
    sh.sh_p2m_batch_f64(ctx, P, count, d["c"], npts, d["p"], d["q"], d_M, P * (P + 1))
    got = d_M.cpu().numpy()
    for i in range(count):
        assert max_degree_error(got[i], ref[i], P, "M") <= 1e-13


# ----------------------------------------------------------------------------- edge cases
@pytest.mark.parametrize("dtype", DTYPES, ids=DT_ID.get)
def test_count_zero_is_noop(ctx, dtype):
    torch, dev = torch_dev()
    out = torch.full((4, 110), 3.0, dtype=torch.float64 if dtype == sh.SH_F64 else torch.float32, device=dev)
    sh.sh_translate_batch(ctx, "m2l", dtype, 10, 10, 0, out, out, 110, out, 110)
    torch.cuda.synchronize()
    assert bool((out == 3.0).all())


@pytest.mark.parametrize("dtype", DTYPES, ids=DT_ID.get)
@pytest.mark.parametrize("op", ["m2m", "l2l"])
@pytest.mark.parametrize("p_in,p_out", [(6, 6), (6, 9), (9, 5)])
def test_zero_shift_is_identity(ctx, orc, op, dtype, p_in, p_out):
    r, C = _inputs(orc, op, p_in, 9, 3, (0.25, 0.5))
    r[:] = 0.0
    got, _ = run_batch(ctx, op, dtype, p_in, p_out, r, C)
    k = min(p_in, p_out)
    for i in range(9):
        ref = np.zeros(size(p_out))
        ref[: size(k)] = C[i, : size(k)]
        ref[[n * (n + 1) + 1 for n in range(p_out)]] = 0.0
        assert np.allclose(got[i], ref, rtol=TOL[dtype] * 10, atol=0), (op, i)
    assert ctx.device_error() == 0


def test_m2l_zero_or_nonfinite_shift_raises_flag(ctx, orc):
    r, C = _inputs(orc, "m2l", 8, 5, 4, (2.0, 4.0))
    r[2] = 0.0
    r[4] = [np.inf, 0.0, 1.0]
    ctx.device_error()  # clear
    got, raw = run_batch(ctx, "m2l", sh.SH_F64, 8, 8, r, C)
    assert np.isnan(raw[2]).all() and np.isnan(raw[4]).all()
    assert np.isfinite(raw[[0, 1, 3]]).all()
    assert ctx.device_error() == sh.SH_ESHIFT
    assert ctx.device_error() == 0


@pytest.mark.parametrize("dtype", DTYPES, ids=DT_ID.get)
def test_accumulate_and_strides(ctx, orc, dtype):
    p_in, p_out = 9, 7
    r, C = _inputs(orc, "m2l", p_in, 70, 11, (2.0, 4.0))
    ref = orc.translate_batch("m2l", p_in, p_out, r, C)
    # an existing output of the same per-degree size as the result
    base = ref * np.random.default_rng(2).uniform(-2.0, 2.0, ref.shape)
    ld_in, ld_out = size(p_in) + 5, size(p_out) + 3
    got, raw = run_batch(ctx, "m2l", dtype, p_in, p_out, r, C, ld_in=ld_in, ld_out=ld_out,
                         flags=sh.SH_ACCUMULATE, out_init=base)
    for i in range(70):
        e = max_degree_error(got[i] - base[i], ref[i], p_out, "L")
        # the sum carries the rounding of the base (|base| <= 2|ref| per coefficient)
        assert e <= 4 * TOL[dtype], (i, e)
    # the padding between solids is untouched (initialised to zero by run_batch)
    assert (raw[:, size(p_out):] == 0.0).all()


@pytest.mark.parametrize("dtype", DTYPES, ids=DT_ID.get)
def test_input_im0_ignored_output_im0_zero(ctx, orc, dtype):
    p = 8
    r, C = _inputs(orc, "m2l", p, 20, 12, (2.0, 4.0))
    C2 = C.copy()
    C2[:, [n * (n + 1) + 1 for n in range(p)]] = 123.0
    a, rawa = run_batch(ctx, "m2l", dtype, p, p, r, C)
    b, rawb = run_batch(ctx, "m2l", dtype, p, p, r, C2)
    assert np.array_equal(rawa, rawb)
    im0 = rawa[:, [n * (n + 1) + 1 for n in range(p)]]
    assert (im0 == 0.0).all() and not np.signbit(im0).any()


@pytest.mark.parametrize("dtype", DTYPES, ids=DT_ID.get)
def test_indexed_gather_scatter(ctx, orc, dtype):
    torch, dev = torch_dev()
    P = 10
    npool = 50
    r, C = _inputs(orc, "m2l", P, npool, 21, (2.0, 4.0))
    rng = np.random.default_rng(3)
    count = 40
    src = rng.integers(0, npool, count)
    dst = rng.permutation(npool)[:count]
    rr = wl.random_shifts(rng, count, 2.0, 4.0)
    ref = orc.translate_batch("m2l", P, P, rr, C[src])
    npdt = np.float64 if dtype == sh.SH_F64 else np.float32
    pool = torch.from_numpy(to_basis(C, P, "M", dtype).astype(npdt)).to(dev)
    outp = torch.zeros((npool, size(P)), dtype=pool.dtype, device=dev)
    d_src = torch.from_numpy(src.astype(np.int64)).to(dev)
    d_dst = torch.from_numpy(dst.astype(np.int64)).to(dev)
    d_r = torch.from_numpy(rr.astype(npdt)).to(dev)
    sh.sh_translate_indexed(ctx, "m2l", dtype, P, P, count, d_r, d_src, pool, size(P), d_dst, outp, size(P))
    got = from_basis(outp.cpu().numpy(), P, "L", dtype)
    for i in range(count):
        assert max_degree_error(got[dst[i]], ref[i], P, "L") <= TOL[dtype]
    untouched = np.setdiff1d(np.arange(npool), dst)
    assert (got[untouched] == 0).all()


def test_indexed_needs_both_index_arrays(ctx):
    """The indexed kernels read both index arrays: a call with only one of them is rejected
    with SH_EINVAL before anything is launched (a gather array with a null scatter array once
    reached the kernel and faulted)."""
    torch, dev = torch_dev()
    P, count = 10, 4
    idx = torch.zeros(count, dtype=torch.int64, device=dev)
    pool = torch.zeros((count, size(P)), dtype=torch.float64, device=dev)
    r = torch.full((count, 3), 2.0, dtype=torch.float64, device=dev)
    for src, dst in ((idx, None), (None, idx)):
        with pytest.raises(sh.ShError) as e:
            sh.sh_translate_indexed(ctx, "m2l", sh.SH_F64, P, P, count, r, src, pool, size(P), dst, pool, size(P))
        assert e.value.status == sh.SH_EINVAL
    torch.cuda.synchronize()
    assert ctx.device_error() == 0


@pytest.mark.parametrize("op", ["m2l", "m2m", "l2l"])
def test_single_host_calls(ctx, orc, op):
    p_in, p_out = 9, 11
    r, C = _inputs(orc, op, p_in, 3, 31, LENGTHS[op])
    for i in range(3):
        ref = orc.translate_batch(op, p_in, p_out, r[i:i + 1], C[i:i + 1])[0]
        got = getattr(sh, f"sh_{op}_f64")(ctx, p_in, p_out, r[i], C[i])
        assert max_degree_error(got, ref, p_out, OUT_KIND[op]) <= TOL[sh.SH_F64]
        w_in = np.asarray(C[i], np.float64)
        g32 = getattr(sh, f"sh_{op}_f32")(ctx, p_in, p_out, r[i].astype(np.float32),
                                           to_basis(w_in, p_in, IN_KIND[op], sh.SH_F32))
        assert max_degree_error(from_basis(g32, p_out, OUT_KIND[op], sh.SH_F32), ref, p_out,
                                OUT_KIND[op]) <= TOL[sh.SH_F32]
    with pytest.raises(sh.ShError) as ei:
        sh.sh_m2l_f64(ctx, 4, 4, [0.0, 0.0, 0.0], np.zeros(20))
    assert ei.value.status == sh.SH_ESHIFT


def test_order_validation(ctx):
    torch, dev = torch_dev()
    x = torch.zeros(16, dtype=torch.float64, device=dev)
    with pytest.raises(sh.ShError) as ei:
        sh.sh_m2l_batch_f64(ctx, 0, 4, 1, x, x, 20, x, 20)
    assert ei.value.status == sh.SH_EORDER
    with pytest.raises(sh.ShError) as ei:
        sh.sh_m2l_batch_f64(ctx, 49, 4, 1, x, x, 49 * 50, x, 20)
    assert ei.value.status == sh.SH_EORDER
    with pytest.raises(sh.ShError) as ei:
        sh.sh_m2l_batch_f64(ctx, 4, 4, 1, x, x, 19, x, 20)
    assert ei.value.status == sh.SH_EINVAL


def test_concurrent_host_threads(ctx, orc):
    """The context is immutable: calls from several host threads on their own streams agree
    with the serial results bit for bit."""
    import threading
    torch, dev = torch_dev()
    P = 10
    r, C = _inputs(orc, "m2l", P, 300, 41, (2.0, 4.0))
    d_r = torch.from_numpy(r).to(dev)
    d_C = torch.from_numpy(C).to(dev)
    serial = torch.empty((300, size(P)), dtype=torch.float64, device=dev)
    sh.sh_m2l_batch_f64(ctx, P, P, 300, d_r, d_C, size(P), serial, size(P))
    torch.cuda.synchronize()
    outs = [torch.empty_like(serial) for _ in range(4)]
    errs = []

    def work(k):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(5):
                    sh.sh_m2l_batch_f64(ctx, P, P, 300, d_r, d_C, size(P), outs[k], size(P), 0, s)
            s.synchronize()
        except Exception as e:  # pragma: no cover
            errs.append(e)

    th = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs
    for o in outs:
        assert torch.equal(o, serial)


def test_indexed_call_needs_both_index_arrays(ctx):
    """An indexed call with only one of its index arrays is rejected before any launch (the
    indexed kernels read both): SH_EINVAL, nothing written."""
    torch, dev = torch_dev()
    S = size(10)
    x = torch.full((4, S), 3.0, dtype=torch.float64, device=dev)
    y = torch.full((4, S), 5.0, dtype=torch.float64, device=dev)
    r = torch.ones((4, 3), dtype=torch.float64, device=dev)
    idx = torch.arange(4, dtype=torch.int64, device=dev)
    L = sh.lib()
    for src, dst in ((idx.data_ptr(), None), (None, idx.data_ptr())):
        st = L.sh_translate_indexed(ctx.handle, sh.SH_M2L, sh.SH_F64, 10, 10, 4, r.data_ptr(), src, x.data_ptr(), S,
                                    dst, y.data_ptr(), S, 0, None)
        assert st == sh.SH_EINVAL
    torch.cuda.synchronize()
    assert bool((y == 5.0).all())


def test_indexed_checked_rejects_bad_indices_and_matches_unchecked(ctx):
    """The checked indexed call refuses, before any launch, an index outside its pool, a
    repeated destination under SH_ACCUMULATE and (one pool for input and output) a destination
    that is also a source; a valid call gives the unchecked call's result bit for bit."""
    torch, dev = torch_dev()
    P, n_in, n_out, count = 8, 50, 40, 30
    S = size(P)
    rng = np.random.default_rng(12)
    M = torch.from_numpy(rng.normal(size=(n_in, S)) * 1e-2).to(dev)
    r = torch.from_numpy(wl.random_shifts(rng, count, 2.0, 6.0)).to(dev)
    src = rng.integers(0, n_in, count)
    dst = rng.permutation(n_out)[:count]
    d_src = torch.from_numpy(src.astype(np.int64)).to(dev)
    d_dst = torch.from_numpy(dst.astype(np.int64)).to(dev)

    def run(s, d, n_o=n_out, flags=0, out=None, n_i=n_in, inp=M):
        out = torch.full((n_o, S), 7.0, dtype=torch.float64, device=dev) if out is None else out
        sh.sh_translate_indexed_checked(ctx, "m2l", sh.SH_F64, P, P, count, r, s, inp, S, n_i, d, out, S, n_o, flags)
        torch.cuda.synchronize()
        return out

    got = run(d_src, d_dst)
    ref = torch.full((n_out, S), 7.0, dtype=torch.float64, device=dev)
    sh.sh_translate_indexed(ctx, "m2l", sh.SH_F64, P, P, count, r, d_src, M, S, d_dst, ref, S)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    bad = [(np.where(np.arange(count) == 3, n_in, src), dst, 0),       # source past the pool
           (src, np.where(np.arange(count) == 5, -1, dst), 0),         # negative destination
           (src, np.where(np.arange(count) == 7, n_out, dst), 0),      # destination past the pool
           (src, np.where(np.arange(count) == 9, dst[0], dst), sh.SH_ACCUMULATE)]  # repeated, accumulating
    for s_, d_, fl in bad:
        out = torch.full((n_out, S), 7.0, dtype=torch.float64, device=dev)
        with pytest.raises(sh.ShError) as e:
            run(torch.from_numpy(s_.astype(np.int64)).to(dev), torch.from_numpy(d_.astype(np.int64)).to(dev),
                flags=fl, out=out)
        assert e.value.status == sh.SH_EINVAL
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())
    # one pool for input and output: a destination that is also a source is refused
    pool = torch.from_numpy(rng.normal(size=(n_in, S)) * 1e-2).to(dev)
    keep = pool.clone()
    s_al = np.arange(count, dtype=np.int64)
    d_al = np.arange(count, dtype=np.int64) + 10  # overlaps sources 10..29
    with pytest.raises(sh.ShError) as e:
        sh.sh_translate_indexed_checked(ctx, "m2m", sh.SH_F64, P, P, count, r,
                                        torch.from_numpy(s_al).to(dev), pool, S, n_in,
                                        torch.from_numpy(d_al).to(dev), pool, S, n_in)
    assert e.value.status == sh.SH_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(pool, keep)
    # one pool read and written with two strides: the slot indices name different solids,
    # so the call is refused even with disjoint indices
    with pytest.raises(sh.ShError) as e:
        sh.sh_translate_indexed_checked(ctx, "m2m", sh.SH_F64, P, P, 5, r,
                                        torch.from_numpy(s_al[:5]).to(dev), pool, S, n_in // 2,
                                        torch.from_numpy(s_al[5:10]).to(dev), pool, 2 * S, n_in // 2)
    assert e.value.status == sh.SH_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(pool, keep)
