"""GPU parity of the shared-shift operators (BF16-split MFMA, FP32 accumulation).

Metric: per translation, the C15 error max_n max_m |L_hat - L_hat_ref| / max_m |L_hat_ref| in
the normalised basis, against the oracle.  Bound per translation: max(tol, 2 x the largest
error of a plain evaluation of the same translation in the form's own arithmetic over several
summation orders) (gpu_util.Plain32, which shows what that arithmetic itself costs where a
degree's coefficients cancel):
  * FP32 MFMA: FP32 products and sums of the operator rounded to FP32, tol = 1e-5;
  * BF16x6 / BF16x3: operator and input split into three BF16 pieces, the six / three piece
    products the kernel forms, summed in FP32; tol = 1e-5 for BF16x6 (about 24 bits of each
    product) and 2e-4 for BF16x3 (about 16 bits of each product).
"""
import numpy as np
import pytest

import oracle
import paper_2202_02847_amd as sh
from paper_2202_02847_amd import workloads as wl
from gpu_util import IN_KIND, OUT_KIND, PLAIN32_FACTOR, Plain32, check, from_basis, to_basis, torch_dev

pytestmark = pytest.mark.gpu

TOL_PREC = {sh.SH_SHARED_BF16X6: 1e-5, sh.SH_SHARED_BF16X3: 2e-4, sh.SH_SHARED_FP32: 1e-5}
BF16 = {sh.SH_SHARED_BF16X6: 6, sh.SH_SHARED_BF16X3: 3, sh.SH_SHARED_FP32: 0}
PREC_ID = {sh.SH_SHARED_BF16X6: "bf16x6", sh.SH_SHARED_BF16X3: "bf16x3", sh.SH_SHARED_FP32: "fp32"}


@pytest.fixture(scope="module")
def ctx():
    c = sh.Context(max_order=32, device=0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def class_inputs(orc, op, p_in, counts, seed):
    rng = np.random.default_rng(seed)
    n = int(sum(counts))
    pts, q = wl.clusters(rng, n, 12)
    C = np.zeros((n, p_in * (p_in + 1)))
    for i in range(n):
        if op == "l2l":
            C[i] = orc.p2l(p_in, [0, 0, 0], pts[i] + np.array([2.5, -1.0, 1.5]), q[i])
        else:
            C[i] = orc.p2m(p_in, [0, 0, 0], pts[i], q[i])
    return C


def run_shared(ctx, op, p_in, p_out, shifts, counts, C, prec, flags=0, out_init=None, ld_pad=0):
    torch, dev = torch_dev()
    n = int(sum(counts))
    K, N = p_in * (p_in + 1), p_out * (p_out + 1)
    ld_in, ld_out = K + ld_pad, N + ld_pad
    A = np.zeros((n, ld_in), np.float32)
    A[:, :K] = to_basis(C, p_in, IN_KIND[op], sh.SH_F32)
    cs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    d_in = torch.from_numpy(A).to(dev)
    if out_init is None:
        d_out = torch.full((n, ld_out), 5.0, dtype=torch.float32, device=dev)
    else:
        o = np.full((n, ld_out), 5.0, np.float32)
        o[:, :N] = out_init
        d_out = torch.from_numpy(o).to(dev)
    d_cs = torch.from_numpy(cs).to(dev)
    S = sh.Shared(ctx, op, p_in, p_out, shifts, prec)
    S.execute(n, d_cs, d_in, ld_in, d_out, ld_out, flags)
    torch.cuda.synchronize()
    out = d_out.cpu().numpy()
    S.close()
    return from_basis(out[:, :N], p_out, OUT_KIND[op], sh.SH_F32), out


def reference(orc, op, p_in, p_out, shifts, counts, C, prec, base=None):
    """The oracle's results and the plain evaluation in the form's arithmetic (Plain32) of the
    same translations."""
    r = np.repeat(np.reshape(shifts, (-1, 3)), counts, axis=0)
    ref = orc.translate_batch(op, p_in, p_out, r, C, nthreads=8)
    p32 = Plain32(lambda rr, CC: orc.translate_batch(op, p_in, p_out, rr, CC, nthreads=8), p_in, p_out,
                  IN_KIND[op], OUT_KIND[op], r, C, base, bf16=BF16[prec])
    return ref, p32


def check_shared(got, ref, p32, p_out, op, prec, what):
    return check(got, ref, p_out, OUT_KIND[op], TOL_PREC[prec], what, plain32=p32, factor32=PLAIN32_FACTOR)


# orders 5..20: 4-real and 2-real input rows, one and several K chunks, and (order 20) output
# rows that take two chunks of output tiles
CASES = [("m2l", 8, 8), ("m2l", 10, 10), ("m2l", 7, 12), ("m2l", 16, 16), ("m2m", 10, 10), ("l2l", 10, 10),
         ("m2m", 6, 9), ("l2l", 12, 5), ("m2l", 18, 20)]


@pytest.mark.parametrize("prec", [sh.SH_SHARED_BF16X6, sh.SH_SHARED_BF16X3, sh.SH_SHARED_FP32], ids=PREC_ID.get)
@pytest.mark.parametrize("op,p_in,p_out", CASES, ids=[f"{o}-{a}-{b}" for o, a, b in CASES])
def test_shared_vs_oracle(ctx, orc, op, p_in, p_out, prec):
    if op == "m2l":
        offs = wl.octree_offsets()[[0, 5, 57, 158, 200, 315]]
    else:
        offs = wl.child_offsets()[[0, 3, 6, 7]]
    counts = np.array([70, 1, 0, 130, 17, 64][:len(offs)])  # ragged, a single, an empty class
    print(f"[shared] {op} {p_in}->{p_out} {PREC_ID[prec]}", flush=True)
    C = class_inputs(orc, op, p_in, counts, 3 + p_in)
    got, raw = run_shared(ctx, op, p_in, p_out, offs, counts, C, prec)
    ref, p32 = reference(orc, op, p_in, p_out, offs, counts, C, prec)
    e = check_shared(got, ref, p32, p_out, op, prec, f"shared {op} {PREC_ID[prec]}")
    print(f"[shared] worst per-degree error {e:.2e}", flush=True)
    # Im C_n^0 written +0
    for nn in range(p_out):
        assert np.all(raw[:, nn * (nn + 1) + 1] == 0.0)


def test_shared_accumulate_ignored_im0_and_stride(ctx, orc):
    op, P = "m2l", 9
    offs = wl.octree_offsets()[[10, 20]]
    counts = np.array([40, 33])
    C = class_inputs(orc, op, P, counts, 77)
    ref = orc.translate_batch(op, P, P, np.repeat(offs, counts, axis=0), C)
    rng = np.random.default_rng(4)
    base = (rng.uniform(-2, 2, (len(C), 1)) * to_basis(ref, P, "L", sh.SH_F32)).astype(np.float32)
    for nn in range(P):
        base[:, nn * (nn + 1) + 1] = 0.0
    Cn = C.copy()
    for nn in range(P):
        Cn[:, nn * (nn + 1) + 1] = np.nan  # Im C_n^0 of the input is ignored
    got, raw = run_shared(ctx, op, P, P, offs, counts, Cn, sh.SH_SHARED_BF16X6, flags=sh.SH_ACCUMULATE,
                          out_init=base, ld_pad=6)
    b = from_basis(base, P, "L", sh.SH_F32)
    ref, p32 = reference(orc, op, P, P, offs, counts, C, sh.SH_SHARED_BF16X6, base=b)
    check_shared(got, ref, p32, P, op, sh.SH_SHARED_BF16X6, "shared accumulate")
    assert np.all(raw[:, P * (P + 1):] == 5.0)  # padding beyond the solid untouched


def test_shared_count_zero_and_validation(ctx):
    torch, dev = torch_dev()
    S = sh.Shared(ctx, "m2l", 6, 6, wl.octree_offsets()[:3], sh.SH_SHARED_BF16X3)
    assert S.nbytes() > 0
    cs = torch.zeros(4, dtype=torch.int64, device=dev)
    x = torch.zeros((4, 42), dtype=torch.float32, device=dev)
    S.execute(0, cs, x, 42, x, 42)
    for args in ((4, cs, x, 41, x, 42), (4, cs, x, 42, x, 41), (4, None, x, 42, x, 42), (-1, cs, x, 42, x, 42)):
        with pytest.raises(sh.ShError):
            S.execute(*args)
    with pytest.raises(sh.ShError) as e:
        S.execute(4, cs, x, 42, x, 42, flags=8)
    assert e.value.status == sh.SH_EINVAL
    S.close()
    for bad, status in (((0, 0, 0), sh.SH_ESHIFT), ((np.inf, 0, 1), sh.SH_ESHIFT)):
        with pytest.raises(sh.ShError) as e:
            sh.Shared(ctx, "m2l", 6, 6, [bad], sh.SH_SHARED_BF16X6)
        assert e.value.status == status
    with pytest.raises(sh.ShError) as e:
        sh.Shared(ctx, "m2l", 6, 33, [(3, 0, 0)], sh.SH_SHARED_BF16X6)
    assert e.value.status == sh.SH_EORDER
    with pytest.raises(sh.ShError) as e:
        sh.Shared(ctx, "m2l", 6, 6, [(3, 0, 0)], 5)
    assert e.value.status == sh.SH_EINVAL
    # M2M / L2L accept a zero shift (identity)
    sh.Shared(ctx, "m2m", 6, 6, [(0, 0, 0)], sh.SH_SHARED_BF16X6).close()


def test_shared_class_start_clamped(ctx, orc):
    """class_start entries outside [0, count] are clamped: nothing is read or written
    outside the count solids."""
    torch, dev = torch_dev()
    P = 6
    offs = wl.octree_offsets()[[1, 2, 3]]
    n = 20
    C = class_inputs(orc, "m2l", P, [n], 5)
    K = P * (P + 1)
    A = torch.from_numpy(to_basis(C, P, "M", sh.SH_F32)).to(dev)
    out = torch.full((n + 4, K), 5.0, dtype=torch.float32, device=dev)
    cs = torch.tensor([-5, 8, 8, 1000], dtype=torch.int64, device=dev)  # -> [0, 8, 8, 20]
    S = sh.Shared(ctx, "m2l", P, P, offs, sh.SH_SHARED_BF16X6)
    S.execute(n, cs, A, K, out, K)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.all(o[n:] == 5.0)
    got = from_basis(o[:n], P, "L", sh.SH_F32)
    ref, p32 = reference(orc, "m2l", P, P, offs[[0, 2]], [8, 12], C, sh.SH_SHARED_BF16X6)
    check_shared(got, ref, p32, P, "m2l", sh.SH_SHARED_BF16X6, "clamped")
    S.close()


ROT32 = 0  # the FP32 rotation path (sh_m2l_batch_f32) on the same batch


@pytest.mark.parametrize("prec", [sh.SH_SHARED_BF16X6, sh.SH_SHARED_FP32, ROT32],
                         ids=lambda p: PREC_ID.get(p, "rot32"))
def test_config3_full_size_sampled(ctx, orc, prec):
    """The precision workload: 2^20 M2L at P=16 grouped by the 316 octree offsets, FP32
    normalised solids, on MFMA (BF16x6, FP32) or through the FP32 rotation path; 2^14 sampled
    translations against the oracle, with the per-translation errors reported (median, p99,
    max)."""
    torch, dev = torch_dev()
    P, n = 16, 1 << 20
    K = P * (P + 1)
    c = wl.config2(n_m2l=n, n_child=8, P=P, seed_config=3)
    idx_sorted = np.argsort(c["dir_idx"], kind="stable")
    offs = wl.octree_offsets()
    counts = np.bincount(c["dir_idx"], minlength=len(offs))
    name = PREC_ID.get(prec, "rot32")
    print(f"[shared] config3 full size n={n} {name}", flush=True)
    M = orc.p2m_batch(P, np.zeros((n, 3)), c["pts"][idx_sorted], c["q"][idx_sorted], nthreads=16)
    A = torch.from_numpy(to_basis(M, P, "M", sh.SH_F32)).to(dev)
    out = torch.empty((n, K), dtype=torch.float32, device=dev)
    if prec == ROT32:
        d_r = torch.from_numpy(c["r_m2l"][idx_sorted].astype(np.float32)).to(dev)
        sh.sh_m2l_batch_f32(ctx, P, P, n, d_r, A, K, out, K)
        S = None
    else:
        cs = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)).to(dev)
        S = sh.Shared(ctx, "m2l", P, P, offs, prec)
        S.execute(n, cs, A, K, out, K)
    torch.cuda.synchronize()
    rng = np.random.default_rng(33)
    pick = np.sort(rng.choice(n, 1 << 14, replace=False))
    got = from_basis(out[torch.from_numpy(pick).to(dev)].cpu().numpy(), P, "L", sh.SH_F32)
    r = c["r_m2l"][idx_sorted][pick]
    ref = orc.translate_batch("m2l", P, P, r, M[pick], nthreads=16)
    p32 = Plain32(lambda rr, CC: orc.translate_batch("m2l", P, P, rr, CC, nthreads=16), P, P, "M", "L", r,
                  M[pick], bf16=0 if prec == ROT32 else BF16[prec])
    check_shared(got, ref, p32, P, "m2l", sh.SH_SHARED_FP32 if prec == ROT32 else prec, f"config3 {name}")
    from refmath import max_degree_error
    errs = np.array([max_degree_error(got[i], ref[i], P, "L") for i in range(len(pick))])
    print(f"[shared] config3 {name} per-translation C15 error over {len(pick)}: median "
          f"{np.median(errs):.2e} p99 {np.quantile(errs, 0.99):.2e} max {errs.max():.2e}", flush=True)
    if S is not None:
        S.close()
