"""GPU parity of mixed work lists (sh_plan_* and sh_translate_list) against the oracle.

Every item is held to the per-translation bound of the batched parity tests
(gpu_util.check): 1e-12 in FP64 (against the long-double oracle, condition-aware) and 1e-5
in FP32 (normalised basis, above the error the FP32 rounding of the input already causes).
"""
import numpy as np
import pytest

import oracle
import paper_2202_02847_amd as sh
from paper_2202_02847_amd import arena
from paper_2202_02847_amd import workloads as wl
from gpu_util import TOL, IN_KIND, OUT_KIND, check, from_basis, ld_ref, plain32_for, to_basis, torch_dev

pytestmark = pytest.mark.gpu

OPN = {sh.SH_M2M: "m2m", sh.SH_M2L: "m2l", sh.SH_L2L: "l2l"}
DT_ID = {sh.SH_F64: "f64", sh.SH_F32: "f32"}


@pytest.fixture(scope="module")
def ctx():
    c = sh.Context(max_order=48, device=0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def source_solid(orc, opc, p_in, pts, q):
    """Input of one item: the multipole of the cluster (M2M, M2L) or the local expansion,
    about the origin, of the cluster moved to a centre about 3 away (L2L)."""
    if opc == sh.SH_L2L:
        return orc.p2l(int(p_in), [0.0, 0.0, 0.0], pts + np.array([2.5, -1.0, 1.5]), q)
    return orc.p2m(int(p_in), [0.0, 0.0, 0.0], pts, q)


def make_list(orc, n, seed, pmax=30, lo=1):
    rng = np.random.default_rng(seed)
    op = rng.integers(0, 3, n).astype(np.int32)
    p_in = wl.mixed_orders(rng, n, lo, pmax).astype(np.int32)
    p_out = wl.mixed_orders(rng, n, lo, pmax).astype(np.int32)
    r = wl.random_shifts(rng, n, 2.0, 6.0)
    pts, q = wl.clusters(rng, n, 12)
    C = [source_solid(orc, op[i], p_in[i], pts[i], q[i]) for i in range(n)]
    return op, p_in, p_out, r, C


def pack_inputs(dtype, op, p_in, C):
    in_off, in_total = arena.packed_offsets(p_in)
    A = np.zeros(max(in_total, 2), np.float64 if dtype == sh.SH_F64 else np.float32)
    for i in range(len(op)):
        s = int(p_in[i]) * (int(p_in[i]) + 1)
        A[in_off[i]:in_off[i] + s] = to_basis(C[i], int(p_in[i]), IN_KIND[OPN[int(op[i])]], dtype)
    return A, in_off, in_total


def unpack(dtype, op, p_out, out, out_off):
    res = []
    for i in range(len(op)):
        s = int(p_out[i]) * (int(p_out[i]) + 1)
        res.append(from_basis(out[out_off[i]:out_off[i] + s], int(p_out[i]), OUT_KIND[OPN[int(op[i])]], dtype))
    return res


def run_list(ctx, dtype, op, p_in, p_out, r, C, plan_flags=0, out_init=None, one_shot=False):
    torch, dev = torch_dev()
    A, in_off, in_total = pack_inputs(dtype, op, p_in, C)
    out_off, out_total = arena.packed_offsets(p_out)
    tdt = torch.float64 if dtype == sh.SH_F64 else torch.float32
    items = sh.make_items(op, p_in, p_out, in_off, out_off, r)
    d_in = torch.from_numpy(A).to(dev)
    if out_init is None:
        d_out = torch.full((max(out_total, 2),), 7.0, dtype=tdt, device=dev)
    else:
        d_out = torch.from_numpy(np.ascontiguousarray(out_init)).to(dev)
    if one_shot:
        sh.sh_translate_list(ctx, dtype, items, d_in, in_total, d_out, out_total, plan_flags & sh.SH_ACCUMULATE)
        desc = None
    else:
        plan = sh.Plan(ctx, dtype, items, plan_flags)
        plan.execute(d_in, in_total, d_out, out_total)
        desc = plan.describe()
        torch.cuda.synchronize()
        plan.close()
    torch.cuda.synchronize()
    out = d_out.cpu().numpy()
    return unpack(dtype, op, p_out, out, out_off), out, desc


def check_items(orc, dtype, op, p_in, p_out, r, C, got, what, base=None):
    """Groups the items by (op, p_in, p_out) and checks each group against the oracle.
    base: per-item values already in the output before an accumulating call."""
    keys = {}
    for i in range(len(op)):
        keys.setdefault((int(op[i]), int(p_in[i]), int(p_out[i])), []).append(i)
    worst = 0.0
    for (o, pi, po), idx in keys.items():
        name = OPN[o]
        Cg = np.stack([C[i] for i in idx])
        rg = r[idx]
        ref = orc.translate_batch(name, pi, po, rg, Cg)
        g = np.stack([got[i] for i in idx])
        rl = ld_ref(name, pi, po, rg, Cg) if dtype == sh.SH_F64 else None
        b = np.stack([base[i] for i in idx]) if base is not None else None
        if b is not None:
            ref = ref + b
            rl = rl + b if rl is not None else None
        p32 = plain32_for(orc, name, pi, po, rg, Cg, b) if dtype == sh.SH_F32 else None
        worst = max(worst, check(g, ref, po, OUT_KIND[name], TOL[dtype], f"{what} {name} {pi}->{po}", rl, p32))
    return worst


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
@pytest.mark.parametrize("dtype", [sh.SH_F64, sh.SH_F32], ids=DT_ID.get)
def test_list_mixed_orders(ctx, orc, dtype, graph):
    pmax = 36 if dtype == sh.SH_F64 else 30
    print(f"[list] mixed dtype={DT_ID[dtype]} graph={graph}", flush=True)
    op, p_in, p_out, r, C = make_list(orc, 400, 11 + dtype, pmax=pmax)
    got, _, desc = run_list(ctx, dtype, op, p_in, p_out, r, C, 0 if graph else sh.SH_PLAN_NO_GRAPH)
    kinds = {b["mapping"] for b in desc["bins"]}
    assert "block" in kinds and "lpt64" in kinds
    if pmax > 31:
        assert "wave" in kinds
    assert sum(b["items"] for b in desc["bins"]) == 400
    check_items(orc, dtype, op, p_in, p_out, r, C, got, f"list {DT_ID[dtype]}")
    assert ctx.device_error() == 0


@pytest.mark.parametrize("dtype", [sh.SH_F64, sh.SH_F32], ids=DT_ID.get)
def test_list_tasks_ragged(ctx, orc, dtype):
    """One (op, p_in, p_out) over several full tasks and a ragged one, next to a single item
    of another order in the same bucket."""
    n = 64 * 3 + 17
    rng = np.random.default_rng(5)
    op = np.full(n + 1, sh.SH_M2L, np.int32)
    p_in = np.full(n + 1, 9, np.int32)
    p_out = np.full(n + 1, 7, np.int32)
    p_in[-1], p_out[-1] = 10, 4
    r = wl.random_shifts(rng, n + 1, 2.0, 6.0)
    pts, q = wl.clusters(rng, n + 1, 12)
    C = [source_solid(orc, op[i], p_in[i], pts[i], q[i]) for i in range(n + 1)]
    got, _, desc = run_list(ctx, dtype, op, p_in, p_out, r, C)
    (b,) = desc["bins"]
    assert b["mapping"] == "lpt64" and b["bucket"] == 10 and b["tasks"] == 4 + 1
    check_items(orc, dtype, op, p_in, p_out, r, C, got, "ragged")


def test_list_graph_replays(ctx, orc):
    """A captured plan replayed several times, with other device work and host
    synchronisation between the replays: every replay equals the eager result bit for bit
    and passes the oracle; new arenas recapture."""
    torch, dev = torch_dev()
    dtype = sh.SH_F64
    op, p_in, p_out, r, C = make_list(orc, 150, 23, pmax=24)
    A, in_off, in_total = pack_inputs(dtype, op, p_in, C)
    out_off, out_total = arena.packed_offsets(p_out)
    items = sh.make_items(op, p_in, p_out, in_off, out_off, r)
    d_in = torch.from_numpy(A).to(dev)
    eager = torch.zeros(out_total, dtype=torch.float64, device=dev)
    pe = sh.Plan(ctx, dtype, items, sh.SH_PLAN_NO_GRAPH)
    pe.execute(d_in, in_total, eager, out_total)
    torch.cuda.synchronize()
    ref = eager.cpu().numpy()
    check_items(orc, dtype, op, p_in, p_out, r, C, unpack(dtype, op, p_out, ref, out_off), "eager")
    pg = sh.Plan(ctx, dtype, items)
    d_out = torch.empty(out_total, dtype=torch.float64, device=dev)
    scratch = torch.ones(1 << 20, dtype=torch.float64, device=dev)
    for rep in range(4):
        d_out.fill_(float(rep) - 3.5)
        scratch.mul_(1.5).add_(rep)  # unrelated eager work between replays
        pg.execute(d_in, in_total, d_out, out_total)
        if rep % 2:
            torch.cuda.synchronize()
        got = d_out.cpu().numpy()
        assert np.array_equal(got, ref), f"replay {rep} differs from the eager run"
    d_out2 = torch.full((out_total + 64,), 9.0, dtype=torch.float64, device=dev)[64:]
    pg.execute(d_in, in_total, d_out2, out_total)
    torch.cuda.synchronize()
    assert np.array_equal(d_out2.cpu().numpy(), ref)
    pg.close()
    pe.close()


@pytest.mark.parametrize("pmax,lo", [(16, 3), (30, 17)], ids=["lpt-orders", "block-orders"])
def test_list_autotune(ctx, orc, pmax, lo):
    """Tuned plans choose a mapping per bin (task size or wavefront kernel up to order 16;
    block-kernel workgroup shape or wavefront kernel for orders 17..30) and stay within the
    bound."""
    dtype = sh.SH_F64
    op, p_in, p_out, r, C = make_list(orc, 300, 31 + pmax, pmax=pmax, lo=lo)
    got, _, desc = run_list(ctx, dtype, op, p_in, p_out, r, C, sh.SH_PLAN_AUTOTUNE)
    print("[list] tuned bins", [(b["mapping"], b["op"], b["items"]) for b in desc["bins"]], flush=True)
    assert desc["bins"] and all(b["tuned"] for b in desc["bins"] if b["op"] != "mixed")
    big = [b for b in desc["bins"] if b["pmax"] > 16]
    assert all(b["mapping"] in ("block", "block8", "wave") for b in big)
    if lo > 16:
        assert big
    check_items(orc, dtype, op, p_in, p_out, r, C, got, "tuned")


@pytest.mark.parametrize("dtype", [sh.SH_F64, sh.SH_F32], ids=DT_ID.get)
def test_list_accumulate(ctx, orc, dtype):
    op, p_in, p_out, r, C = make_list(orc, 120, 41 + dtype, pmax=20)
    rng = np.random.default_rng(3)
    base = []
    out_off, out_total = arena.packed_offsets(p_out)
    init = np.zeros(out_total, np.float64 if dtype == sh.SH_F64 else np.float32)
    plain, _, _ = run_list(ctx, dtype, op, p_in, p_out, r, C)
    for i in range(len(op)):
        s = int(p_out[i]) * (int(p_out[i]) + 1)
        b = plain[i] * rng.uniform(-2, 2)
        for n in range(int(p_out[i])):
            b[n * (n + 1) + 1] = 0.0  # Im of order 0 stays +0
        base.append(b)
        init[out_off[i]:out_off[i] + s] = to_basis(b, int(p_out[i]), OUT_KIND[OPN[int(op[i])]], dtype)
    base = [from_basis(init[out_off[i]:out_off[i] + int(p_out[i]) * (int(p_out[i]) + 1)], int(p_out[i]),
                       OUT_KIND[OPN[int(op[i])]], dtype) for i in range(len(op))]
    got, _, _ = run_list(ctx, dtype, op, p_in, p_out, r, C, sh.SH_ACCUMULATE, out_init=init)
    # the sum of two results of size ~x is checked at 4x the bound, as for the batched calls
    keys = {}
    for i in range(len(op)):
        keys.setdefault((int(op[i]), int(p_in[i]), int(p_out[i])), []).append(i)
    for (o, pi, po), idx in keys.items():
        name = OPN[o]
        Cg = np.stack([C[i] for i in idx])
        ref = orc.translate_batch(name, pi, po, r[idx], Cg) + np.stack([base[i] for i in idx])
        g = np.stack([got[i] for i in idx])
        tol = 4 * TOL[dtype]
        if dtype == sh.SH_F32:
            p32 = plain32_for(orc, name, pi, po, r[idx], Cg, np.stack([base[i] for i in idx]))
            check(g, ref, po, OUT_KIND[name], tol, f"acc {name}", plain32=p32)
        else:
            rl = ld_ref(name, pi, po, r[idx], Cg) + np.stack([base[i] for i in idx])
            check(g, ref, po, OUT_KIND[name], tol, f"acc {name}", ref_ld=rl)


def test_list_one_shot_matches_plan(ctx, orc):
    op, p_in, p_out, r, C = make_list(orc, 90, 51, pmax=28)
    a, _, _ = run_list(ctx, sh.SH_F64, op, p_in, p_out, r, C)
    b, _, _ = run_list(ctx, sh.SH_F64, op, p_in, p_out, r, C, one_shot=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("dtype", [sh.SH_F64, sh.SH_F32], ids=DT_ID.get)
def test_list_matches_batched_call(ctx, orc, dtype):
    """A homogeneous list gives the batched call's result (alone == in a list)."""
    torch, dev = torch_dev()
    from gpu_util import run_batch
    n, P = 130, 10
    rng = np.random.default_rng(77)
    r = wl.random_shifts(rng, n, 2.0, 6.0)
    pts, q = wl.clusters(rng, n, 12)
    C = [orc.p2m(P, [0, 0, 0], pts[i], q[i]) for i in range(n)]
    op = np.full(n, sh.SH_M2L, np.int32)
    pp = np.full(n, P, np.int32)
    got, _, _ = run_list(ctx, dtype, op, pp, pp, r, C)
    ref, _ = run_batch(ctx, "m2l", dtype, P, P, r, np.stack(C))
    worst = max(float(np.max(np.abs(g - b) / np.maximum(np.abs(b).max(), 1e-300))) for g, b in zip(got, ref))
    assert worst <= TOL[dtype]


@pytest.mark.parametrize("dtype", [sh.SH_F64, sh.SH_F32], ids=DT_ID.get)
def test_list_zero_shift_identity(ctx, orc, dtype):
    op = np.array([sh.SH_M2M, sh.SH_L2L, sh.SH_M2M, sh.SH_L2L, sh.SH_M2M, sh.SH_L2L, sh.SH_M2L], np.int32)
    p_in = np.array([6, 6, 6, 9, 20, 22, 6], np.int32)
    p_out = np.array([9, 9, 4, 5, 24, 18, 6], np.int32)
    rng = np.random.default_rng(9)
    pts, q = wl.clusters(rng, len(op), 12)
    C = [source_solid(orc, op[i], p_in[i], pts[i], q[i]) for i in range(len(op))]
    r = np.zeros((len(op), 3))
    r[-1] = [2.0, 1.0, -2.5]
    got, _, _ = run_list(ctx, dtype, op, p_in, p_out, r, C)
    check_items(orc, dtype, op, p_in, p_out, r, C, got, "zero shift")
    assert ctx.device_error() == 0


def test_list_shared_arena(ctx, orc):
    """Inputs and outputs in one buffer: allowed when no output meets an input."""
    torch, dev = torch_dev()
    op, p_in, p_out, r, C = make_list(orc, 40, 61, pmax=14)
    A, in_off, in_total = pack_inputs(sh.SH_F64, op, p_in, C)
    out_off, out_total = arena.packed_offsets(p_out)
    buf = torch.zeros(in_total + out_total, dtype=torch.float64, device=dev)
    buf[:in_total] = torch.from_numpy(A).to(dev)
    items = sh.make_items(op, p_in, p_out, in_off, out_off + in_total, r)
    plan = sh.Plan(ctx, sh.SH_F64, items)
    plan.execute(buf, in_total + out_total, buf, in_total + out_total)
    torch.cuda.synchronize()
    got = unpack(sh.SH_F64, op, p_out, buf.cpu().numpy()[in_total:], out_off)
    check_items(orc, sh.SH_F64, op, p_in, p_out, r, C, got, "shared arena")
    # outputs placed over the inputs of the same buffer are refused; in separate buffers
    # the same plan runs
    over = sh.Plan(ctx, sh.SH_F64, sh.make_items(op, p_in, p_out, in_off, out_off, r))
    with pytest.raises(sh.ShError) as e:
        over.execute(buf, in_total + out_total, buf, in_total + out_total)
    assert e.value.status == sh.SH_EINVAL
    sep = torch.zeros(out_total, dtype=torch.float64, device=dev)
    over.execute(buf, in_total, sep, out_total)
    torch.cuda.synchronize()
    assert np.array_equal(sep.cpu().numpy(), buf.cpu().numpy()[in_total:])
    over.close()
    plan.close()


def test_list_validation(ctx):
    torch, dev = torch_dev()
    base = sh.make_items([sh.SH_M2L, sh.SH_M2M], [4, 4], [4, 4], [0, 20], [0, 20], [[3, 0, 0], [0, 0, 1]])

    def status(items, flags=0):
        try:
            sh.Plan(ctx, sh.SH_F64, items, flags).close()
            return sh.SH_OK
        except sh.ShError as e:
            return e.status

    assert status(base) == sh.SH_OK
    bad = base.copy(); bad["in_off"][1] = 21
    assert status(bad) == sh.SH_EINVAL            # odd offset
    bad = base.copy(); bad["out_off"][1] = 10
    assert status(bad) == sh.SH_EINVAL            # overlapping outputs
    bad = base.copy(); bad["reserved"][0] = 1
    assert status(bad) == sh.SH_EINVAL
    bad = base.copy(); bad["op"][0] = 7
    assert status(bad) == sh.SH_EINVAL
    bad = base.copy(); bad["p_out"][0] = 49
    assert status(bad) == sh.SH_EORDER
    bad = base.copy(); bad["p_in"][1] = 0
    assert status(bad) == sh.SH_EORDER
    bad = base.copy(); bad["r"][0] = [0, 0, 0]
    assert status(bad) == sh.SH_ESHIFT            # M2L zero shift
    bad = base.copy(); bad["r"][1] = [np.nan, 0, 0]
    assert status(bad) == sh.SH_ESHIFT
    assert status(base, 1 << 7) == sh.SH_EINVAL   # unknown flag
    plan = sh.Plan(ctx, sh.SH_F64, base)
    d_in = torch.zeros(40, dtype=torch.float64, device=dev)
    d_out = torch.zeros(40, dtype=torch.float64, device=dev)
    for args in ((d_in, 39, d_out, 40), (d_in, 40, d_out, 39), (None, 40, d_out, 40),
                 (d_in.data_ptr() + 8, 40, d_out, 40)):
        with pytest.raises(sh.ShError) as e:
            plan.execute(*args)
        assert e.value.status == sh.SH_EINVAL
    plan.execute(d_in, 40, d_out, 40)
    torch.cuda.synchronize()
    plan.close()


def test_list_empty(ctx):
    torch, dev = torch_dev()
    plan = sh.Plan(ctx, sh.SH_F32, np.zeros(0, sh.SH_ITEM))
    plan.execute(None, 0, None, 0)
    assert plan.describe()["bins"] == []
    plan.close()
    sh.sh_translate_list(ctx, sh.SH_F64, np.zeros(0, sh.SH_ITEM), None, 0, None, 0)


@pytest.mark.parametrize("dtype", [sh.SH_F64, sh.SH_F32], ids=DT_ID.get)
def test_config4_full_size_sampled(ctx, orc, dtype):
    """The mixed work list at the size the benchmark times (500,000 items, orders 3..30),
    through one captured plan, checked on sampled items."""
    torch, dev = torch_dev()
    n = 500_000
    c = wl.config4(n)
    print(f"[list] config4 full size dtype={DT_ID[dtype]}", flush=True)
    op, p_in, p_out, r = c["op"], c["p_in"], c["p_out"], c["r"]
    in_off, in_total = arena.packed_offsets(p_in, group_by_order=True)
    out_off, out_total = arena.packed_offsets(p_out)
    npdt = np.float64 if dtype == sh.SH_F64 else np.float32
    A = np.zeros(in_total, npdt)
    for P, first, idx in arena.order_blocks(p_in, in_off):
        # blocks of equal order, items in list order: multipoles, or for L2L the local
        # expansion of the cluster moved about 3 away (as source_solid)
        is_l = op[idx] == sh.SH_L2L
        C = np.zeros((len(idx), P * (P + 1)))
        zero = np.zeros((len(idx), 3))
        if (~is_l).any():
            C[~is_l] = orc.p2m_batch(P, zero[~is_l], c["pts"][idx[~is_l]], c["q"][idx[~is_l]], nthreads=16)
        if is_l.any():
            far = c["pts"][idx[is_l]] + np.array([2.5, -1.0, 1.5])
            C[is_l] = orc.p2l_batch(P, zero[is_l], far, c["q"][idx[is_l]], nthreads=16)
        if dtype == sh.SH_F32:
            C[~is_l] = to_basis(C[~is_l], P, "M", dtype)
            C[is_l] = to_basis(C[is_l], P, "L", dtype)
        A[first:first + C.size] = C.reshape(-1)
    items = sh.make_items(op, p_in, p_out, in_off, out_off, r)
    d_in = torch.from_numpy(A).to(dev)
    d_out = torch.empty(out_total, dtype=torch.float64 if dtype == sh.SH_F64 else torch.float32, device=dev)
    plan = sh.Plan(ctx, dtype, items)
    plan.execute(d_in, in_total, d_out, out_total)
    torch.cuda.synchronize()
    rng = np.random.default_rng(100 + dtype)
    big = np.nonzero(np.maximum(p_in, p_out) >= 25)[0]
    idx = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 160), rng.choice(big, 40)]))
    out = d_out.cpu().numpy()
    got, Cs = [], []
    for i in idx:
        s_in = int(p_in[i]) * (int(p_in[i]) + 1)
        kind_in = IN_KIND[OPN[int(op[i])]]
        Cs.append(from_basis(A[in_off[i]:in_off[i] + s_in], int(p_in[i]), kind_in, dtype))
    got = unpack(dtype, op[idx], p_out[idx], out, out_off[idx])
    check_items(orc, dtype, op[idx], p_in[idx], p_out[idx], r[idx], Cs, got, "config4")
    plan.close()
    assert ctx.device_error() == 0
