"""GPU parity of the shared-shift operators (BF16-split MFMA, FP32 accumulation).

Metric: per translation and degree n, max_m |L_hat - L_hat_ref| / max_m |L_hat_ref| in the
normalised basis, against the oracle.  Each output coefficient is a dot product
sum_k T_hat[i, k] a_k of the class operator with the FP32 input, so any FP32 evaluation of it
errs by a few units of rounding of sum_k |T_hat[i, k]| |a_k|, not of the result: where the
degree's coefficients cancel (a small monopole, say) the relative error grows by the
cancellation factor kappa_n = max_m sum_k |T_hat| |a| / max_m |L_hat_ref|.  The bound per
degree is max(tol, 4 u kappa_n), with
  * BF16x6: u = 2^-24 (the dropped products a_mid b_lo, a_lo b_mid, a_lo b_lo and the split
    residuals are below 3 * 2^-24 of each product; accumulation in FP32), tol = 1e-5;
  * BF16x3: u = 2^-16 (the dropped a_mid b_mid and the two-piece residuals), tol = 2e-4;
  * FP32 MFMA: u = 2^-24 (the operator rounded once to FP32, FP32 products and sums), tol = 1e-5.
The worst error and the worst kappa are printed for each case.
"""
import numpy as np
import pytest

import oracle
import paper_2202_02847_amd as sh
from paper_2202_02847_amd import workloads as wl
from gpu_util import IN_KIND, OUT_KIND, from_basis, in32_ref, to_basis, torch_dev

pytestmark = pytest.mark.gpu

TOL_PREC = {sh.SH_SHARED_BF16X6: 1e-5, sh.SH_SHARED_BF16X3: 2e-4, sh.SH_SHARED_FP32: 1e-5}
UNIT = {sh.SH_SHARED_BF16X6: 2.0 ** -24, sh.SH_SHARED_BF16X3: 2.0 ** -16, sh.SH_SHARED_FP32: 2.0 ** -24}
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


def reference(orc, op, p_in, p_out, shifts, counts, C):
    r = np.repeat(np.reshape(shifts, (-1, 3)), counts, axis=0)
    ref = orc.translate_batch(op, p_in, p_out, r, C)
    r32 = in32_ref(orc, op, p_in, p_out, r, C)
    return ref, r32


def class_operator(orc, op, p_in, p_out, shift):
    """The oracle's translation as a dense matrix in the normalised basis (outputs x inputs):
    column j is the image of unit solid j."""
    from gpu_util import weights_flat
    K = p_in * (p_in + 1)
    T = orc.translate_batch(op, p_in, p_out, np.repeat(np.reshape(shift, (1, 3)), K, axis=0), np.eye(K),
                            nthreads=8).T
    s_in = weights_flat(p_in) if IN_KIND[op] == "M" else 1.0 / weights_flat(p_in)
    s_out = weights_flat(p_out) if OUT_KIND[op] == "M" else 1.0 / weights_flat(p_out)
    return T * s_out[:, None] / s_in[None, :]


def check_conditioned(got, ref, C, ops_per_row, p_in, p_out, op, prec, what):
    """Per-degree bound max(tol, 4 u kappa_n) (module docstring); returns (worst error,
    worst kappa)."""
    from gpu_util import weights_flat
    tol, u = TOL_PREC[prec], UNIT[prec]
    w_in, w_out = weights_flat(p_in), weights_flat(p_out)
    a = np.abs(C * (w_in if IN_KIND[op] == "M" else 1.0 / w_in))  # normalised basis, FP64
    for nn in range(p_in):
        a[:, nn * (nn + 1) + 1] = 0.0
    s_out = w_out if OUT_KIND[op] == "M" else 1.0 / w_out
    gn, rn = got * s_out, ref * s_out
    worst_e = worst_k = 0.0
    for i in range(len(got)):
        mag = np.abs(ops_per_row[i]) @ a[i]
        for nn in range(p_out):
            sl = slice(nn * (nn + 1), (nn + 1) * (nn + 2))
            den = max(np.abs(rn[i, sl]).max(), 1e-300)
            e = np.abs(gn[i, sl] - rn[i, sl]).max() / den
            kappa = mag[sl].max() / den
            bound = max(tol, 4.0 * u * kappa)
            assert e <= bound, f"{what} translation {i} degree {nn}: {e:.3e} > {bound:.2e} (kappa {kappa:.1e})"
            worst_e, worst_k = max(worst_e, e), max(worst_k, kappa)
    return worst_e, worst_k


CASES = [("m2l", 8, 8), ("m2l", 10, 10), ("m2l", 7, 12), ("m2l", 16, 16), ("m2m", 10, 10), ("l2l", 10, 10),
         ("m2m", 6, 9), ("l2l", 12, 5)]


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
    ref, _ = reference(orc, op, p_in, p_out, offs, counts, C)
    Ts = [class_operator(orc, op, p_in, p_out, o) for o in offs]
    rows = [Ts[c] for c in np.repeat(np.arange(len(offs)), counts)]
    e, k = check_conditioned(got, ref, C, rows, p_in, p_out, op, prec, f"shared {op} {PREC_ID[prec]}")
    print(f"[shared] worst per-degree error {e:.2e} (worst kappa {k:.1e})", flush=True)
    # Im C_n^0 written +0
    for nn in range(p_out):
        assert np.all(raw[:, nn * (nn + 1) + 1] == 0.0)


def test_shared_accumulate_ignored_im0_and_stride(ctx, orc):
    op, P = "m2l", 9
    offs = wl.octree_offsets()[[10, 20]]
    counts = np.array([40, 33])
    C = class_inputs(orc, op, P, counts, 77)
    ref, r32 = reference(orc, op, P, P, offs, counts, C)
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
    rows = [class_operator(orc, op, P, P, offs[c]) for c in np.repeat([0, 1], counts)]
    # the accumulated part alone, after removing the base (its rounding is below 2u of it)
    check_conditioned(got - b, ref, C, rows, P, P, op, sh.SH_SHARED_BF16X6, "shared accumulate")
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
    ref, _ = reference(orc, "m2l", P, P, offs[[0, 2]], [8, 12], C)
    rows = [class_operator(orc, "m2l", P, P, offs[c]) for c in [0] * 8 + [2] * 12]
    check_conditioned(got, ref, C, rows, P, P, "m2l", sh.SH_SHARED_BF16X6, "clamped")
    S.close()


@pytest.mark.parametrize("prec", [sh.SH_SHARED_BF16X6, sh.SH_SHARED_FP32], ids=PREC_ID.get)
def test_config3_full_size_sampled(ctx, orc, prec):
    """The precision workload: 2^20 M2L at P=16 grouped by the 316 octree offsets, FP32
    normalised solids, on MFMA; 2^14 sampled translations against the oracle, with the
    per-degree errors reported (median, p99, max)."""
    torch, dev = torch_dev()
    P, n = 16, 1 << 20
    K = P * (P + 1)
    c = wl.config2(n_m2l=n, n_child=8, P=P, seed_config=3)
    idx_sorted = np.argsort(c["dir_idx"], kind="stable")
    offs = wl.octree_offsets()
    counts = np.bincount(c["dir_idx"], minlength=len(offs))
    print(f"[shared] config3 full size n={n} {PREC_ID[prec]}", flush=True)
    M = orc.p2m_batch(P, np.zeros((n, 3)), c["pts"][idx_sorted], c["q"][idx_sorted], nthreads=16)
    A = torch.from_numpy(to_basis(M, P, "M", sh.SH_F32)).to(dev)
    out = torch.empty((n, K), dtype=torch.float32, device=dev)
    cs = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)).to(dev)
    S = sh.Shared(ctx, "m2l", P, P, offs, prec)
    S.execute(n, cs, A, K, out, K)
    torch.cuda.synchronize()
    rng = np.random.default_rng(33)
    pick = np.sort(rng.choice(n, 1 << 14, replace=False))
    got = from_basis(out[torch.from_numpy(pick).to(dev)].cpu().numpy(), P, "L", sh.SH_F32)
    r = c["r_m2l"][idx_sorted][pick]
    ref = orc.translate_batch("m2l", P, P, r, M[pick], nthreads=16)
    cls = np.repeat(np.arange(len(offs)), counts)[pick]
    Ts = {k: class_operator(orc, "m2l", P, P, offs[k]) for k in np.unique(cls)}
    e, k = check_conditioned(got, ref, M[pick], [Ts[k] for k in cls], P, P, "m2l", prec, "config3")
    from refmath import max_degree_error
    errs = np.array([max_degree_error(got[i], ref[i], P, "L") for i in range(len(pick))])
    print(f"[shared] config3 {PREC_ID[prec]} per-translation C15 error over {len(pick)}: median "
          f"{np.median(errs):.2e} p99 {np.quantile(errs, 0.99):.2e} max {errs.max():.2e} (worst kappa {k:.1e})",
          flush=True)
    S.close()
