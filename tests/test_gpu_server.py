"""GPU tests of the serving runtime (sh_server_*): results against the oracle, the same result
alone and in a mix of concurrent jobs (bit for bit: a translation's kernel follows from its
own operation and orders), admission by staging footprint, validation, statistics."""
import threading

import numpy as np
import pytest

import oracle
import paper_2202_02847_amd as sh
from paper_2202_02847_amd import workloads as wl
from gpu_util import TOL, check, from_basis, ld_ref, plain32_for, to_basis, torch_dev

pytestmark = pytest.mark.gpu

DT_ID = {sh.SH_F64: "f64", sh.SH_F32: "f32"}


@pytest.fixture(scope="module")
def ctx():
    torch_dev()
    c = sh.Context(max_order=32, device=0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def multipoles(orc, P, n, seed):
    rng = np.random.default_rng(seed)
    pts, q = wl.clusters(rng, n, 12)
    return orc.p2m_batch(P, np.zeros((n, 3)), pts, q, nthreads=8)


def locals_(orc, P, n, seed):
    rng = np.random.default_rng(seed)
    pts, q = wl.clusters(rng, n, 12)
    return orc.p2l_batch(P, np.zeros((n, 3)), pts + np.array([2.5, -1.0, 1.5]), q, nthreads=8)


def make_tree(srv, orc, dtype, P, n, seed):
    t = srv.tree_create(dtype, P, n, P, n)
    M = multipoles(orc, P, n, seed)
    L = locals_(orc, P, n, seed + 1)
    npdt = np.float64 if dtype == sh.SH_F64 else np.float32
    srv.tree_write(t, 0, 0, to_basis(M, P, "M", dtype).astype(npdt))
    srv.tree_write(t, 1, 0, to_basis(L, P, "L", dtype).astype(npdt))
    return t, M, L


def job_arrays(op, n_slots, count, seed):
    rng = np.random.default_rng(seed)
    r = wl.random_shifts(rng, count, 2.0, 6.0)
    if op == "m2l":
        src = rng.integers(0, n_slots, count)
        dst = rng.permutation(n_slots)[:count]
    else:  # sources in the first half, destinations in the second
        src = rng.integers(0, n_slots // 2, count)
        dst = n_slots // 2 + rng.permutation(n_slots - n_slots // 2)[:count]
    return r, src, dst


def read_pool(srv, t, pool, P, n, dtype):
    npdt = np.float64 if dtype == sh.SH_F64 else np.float32
    raw = srv.tree_read(t, pool, 0, n, P, npdt)
    return from_basis(raw, P, "M" if pool == 0 else "L", dtype), raw


def check_job(orc, dtype, op, P, r, C_in, got, what):
    ref = orc.translate_batch(op, P, P, r, C_in)
    rl = ld_ref(op, P, P, r, C_in) if dtype == sh.SH_F64 else None
    p32 = plain32_for(orc, op, P, P, r, C_in) if dtype == sh.SH_F32 else None
    return check(got, ref, P, "M" if op == "m2m" else "L", TOL[dtype], what, rl, p32)


@pytest.mark.parametrize("dtype", [sh.SH_F64, sh.SH_F32], ids=DT_ID.get)
@pytest.mark.parametrize("op", ["m2l", "m2m", "l2l"])
def test_server_job_vs_oracle(ctx, orc, dtype, op):
    P, n = 9, 300
    count = 211 if op == "m2l" else 140  # M2M / L2L write the second half of one pool
    print(f"[server] {op} {DT_ID[dtype]}", flush=True)
    srv = sh.Server(ctx, pool_bytes=64 << 20, staging_bytes=8 << 20)
    t, M, L = make_tree(srv, orc, dtype, P, n, 5)
    r, src, dst = job_arrays(op, n, count, 17)
    jid = srv.submit(t, op, r, src, dst)
    lat = srv.wait(jid)
    assert lat > 0
    pool_out = 0 if op == "m2m" else 1
    out, _ = read_pool(srv, t, pool_out, P, n, dtype)
    C = M if op != "l2l" else L
    # inputs as the device holds them (FP32: rounded through the normalised basis)
    Cin = from_basis(to_basis(C, P, "M" if op != "l2l" else "L", dtype), P, "M" if op != "l2l" else "L", dtype)
    check_job(orc, dtype, op, P, r, Cin[src] if dtype == sh.SH_F64 else C[src], out[dst], f"server {op}")
    untouched = np.setdiff1d(np.arange(n), dst)
    before = M if op == "m2m" else L
    before = from_basis(to_basis(before, P, "M" if op == "m2m" else "L", dtype), P, "M" if op == "m2m" else "L", dtype)
    assert np.array_equal(out[untouched], before[untouched])
    srv.close()


def test_server_alone_equals_mix(ctx, orc):
    """One job's result alone and among many concurrent jobs of other trees, orders and dtypes,
    submitted from several host threads."""
    P, n, count = 16, 4000, 3000
    print("[server] alone vs mix", flush=True)
    r, src, dst = job_arrays("m2l", n, count, 99)
    srv = sh.Server(ctx, pool_bytes=1 << 30, staging_bytes=16 << 20)
    t, M, L = make_tree(srv, orc, sh.SH_F64, P, n, 7)
    srv.wait(srv.submit(t, "m2l", r, src, dst))
    alone, _ = read_pool(srv, t, 1, P, n, sh.SH_F64)
    srv.close()

    srv = sh.Server(ctx, pool_bytes=2 << 30, staging_bytes=16 << 20, streams=3, max_batch_jobs=16)
    t, _, _ = make_tree(srv, orc, sh.SH_F64, P, n, 7)
    others = []
    for k, (dt, PP) in enumerate([(sh.SH_F64, 4), (sh.SH_F32, 8), (sh.SH_F64, 24), (sh.SH_F32, 30),
                                  (sh.SH_F64, 10), (sh.SH_F32, 16), (sh.SH_F64, 30)]):
        tt = srv.tree_create(dt, PP, 2000, PP, 2000)
        others.append((tt, dt, PP))
    ids, errors, lock = [], [], threading.Lock()

    def worker(w):
        try:
            rng = np.random.default_rng(1000 + w)
            for j in range(6):
                tt, dt, PP = others[(w * 6 + j) % len(others)]
                op = ["m2l", "m2m", "l2l"][j % 3]
                cnt = int(rng.integers(100, 1500 if op == "m2l" else 1000))
                rr, ss, dd = job_arrays(op, 2000, cnt, 31 * w + j)
                jid = srv.submit(tt, op, rr, ss, dd)
                with lock:
                    ids.append(jid)
        except Exception as exc:  # surfaced below
            with lock:
                errors.append(exc)

    ths = [threading.Thread(target=worker, args=(w,)) for w in range(3)]
    for th in ths:
        th.start()
    jid = srv.submit(t, "m2l", r, src, dst)
    for th in ths:
        th.join()
    assert not errors, errors
    assert len(ids) == 18
    srv.drain()
    for i in ids:
        srv.wait(i)
    srv.wait(jid)
    mixed, _ = read_pool(srv, t, 1, P, n, sh.SH_F64)
    st = srv.stats()
    print(f"[server] batches {st['batches']} mean jobs/batch {st['mean_batch_jobs']:.2f}", flush=True)
    assert np.array_equal(mixed, alone), "a job's result changed when it ran among other jobs"
    check_job(orc, sh.SH_F64, "m2l", P, r[:300], M[src[:300]], mixed[dst[:300]], "mix")
    assert st["jobs_done"] == len(ids) + 1 and st["jobs_failed"] == 0
    srv.close()


def test_server_admission_by_footprint(ctx, orc):
    """A staging arena that holds only a few jobs at a time: every job completes, the peak
    staging in use stays within the arena and jobs queue."""
    srv = sh.Server(ctx, pool_bytes=256 << 20, staging_bytes=256 << 10, streams=2, max_batch_jobs=8)
    trees = [srv.tree_create(sh.SH_F64, 8, 3000, 8, 3000) for _ in range(6)]
    jobs = [job_arrays("m2l", 3000, 2500, k) for k in range(30)]  # 202 KB of footprint each
    ids = [srv.submit(trees[k % 6], "m2l", *jobs[k]) for k in range(30)]
    for i in ids:
        srv.wait(i)
    st = srv.stats()
    print(f"[server] admission: queue peak {st['queue_peak']}, staging peak {st['staging_peak_bytes']}", flush=True)
    assert st["jobs_done"] == 30 and st["jobs_failed"] == 0
    assert 0 < st["staging_peak_bytes"] <= 256 << 10
    # two such jobs never fit together: every batch held exactly one job
    assert st["batches"] == 30
    assert 0 < st["p50_s"] <= st["p99_s"] <= st["max_s"]
    # a job whose footprint exceeds the whole arena can never be admitted
    big = srv.tree_create(sh.SH_F64, 8, 4000, 8, 4000)
    r, s, d = job_arrays("m2l", 4000, 3300, 77)  # 266 KB of footprint
    with pytest.raises(sh.ShError) as e:
        srv.submit(big, "m2l", r, s, d)
    assert e.value.status == sh.SH_EBUSY
    srv.close()


def test_server_validation(ctx):
    srv = sh.Server(ctx, pool_bytes=8 << 20, staging_bytes=1 << 20)
    t = srv.tree_create(sh.SH_F64, 6, 100, 6, 100)
    r = np.tile([[3.0, 0.0, 0.0]], (4, 1))

    def status(**kw):
        a = dict(tree=t, op="m2l", r=r, src=[0, 1, 2, 3], dst=[4, 5, 6, 7])
        a.update(kw)
        try:
            srv.wait(srv.submit(a["tree"], a["op"], a["r"], a["src"], a["dst"]))
            return sh.SH_OK
        except sh.ShError as e:
            return e.status

    assert status() == sh.SH_OK
    # pools whose byte size would overflow have no room (checked before any arithmetic wraps)
    with pytest.raises(sh.ShError) as e:
        srv.tree_create(sh.SH_F64, 30, 1 << 62, 30, 10)
    assert e.value.status == sh.SH_EBUSY
    assert status(dst=[4, 5, 5, 7]) == sh.SH_EINVAL          # repeated destination
    assert status(op="m2m", dst=[1, 5, 6, 7]) == sh.SH_EINVAL  # destination is a source
    assert status(dst=[4, 5, 6, 100]) == sh.SH_EINVAL        # slot out of range
    assert status(src=[-1, 1, 2, 3]) == sh.SH_EINVAL
    assert status(tree=12345) == sh.SH_EINVAL
    assert status(r=np.zeros((4, 3))) == sh.SH_ESHIFT        # M2L zero shift
    assert status(op="l2l", r=np.zeros((4, 3))) == sh.SH_OK  # L2L zero shift: identity
    assert status(src=[], dst=[], r=np.zeros((0, 3))) == sh.SH_OK
    with pytest.raises(sh.ShError) as e:
        srv.tree_create(sh.SH_F64, 30, 10 ** 6, 30, 10)
    assert e.value.status == sh.SH_EBUSY
    with pytest.raises(sh.ShError) as e:
        srv.tree_create(sh.SH_F64, 33, 10, 6, 10)
    assert e.value.status == sh.SH_EORDER
    srv.tree_destroy(t)
    assert srv.stats()["pool_used_bytes"] == 0
    srv.close()


def test_server_accumulate(ctx, orc):
    P, n = 7, 200
    srv = sh.Server(ctx, pool_bytes=32 << 20, staging_bytes=4 << 20)
    t, M, L = make_tree(srv, orc, sh.SH_F64, P, n, 3)
    r1, s1, d1 = job_arrays("m2l", n, 150, 1)
    r2 = wl.random_shifts(np.random.default_rng(2), 150, 2.0, 6.0)
    s2 = np.random.default_rng(3).integers(0, n, 150)
    a = srv.submit(t, "m2l", r1, s1, d1)                              # overwrite
    b = srv.submit(t, "m2l", r2, s2, d1, flags=sh.SH_ACCUMULATE)      # then add into the same slots
    srv.wait(a)
    srv.wait(b)
    out, _ = read_pool(srv, t, 1, P, n, sh.SH_F64)
    ref = orc.translate_batch("m2l", P, P, r1, M[s1]) + orc.translate_batch("m2l", P, P, r2, M[s2])
    ld = ld_ref("m2l", P, P, r1, M[s1]) + ld_ref("m2l", P, P, r2, M[s2])
    check(out[d1], ref, P, "L", 4 * TOL[sh.SH_F64], "server accumulate", ld)
    srv.close()


def test_server_shared_tree_order_and_alone_equals_mix(ctx, orc):
    """Overwriting M2L jobs with disjoint destinations share one tree; a later M2L job that
    overwrites some of the same slots, and an L2L job that reads what it wrote, still see the
    submission order.  The final pools are the same (bit for bit) whether every job ran alone
    (each waited for before the next is submitted) or all were queued at once."""
    P, n = 8, 4000
    rng = np.random.default_rng(404)
    jobs = []
    for k in range(6):  # disjoint destinations
        dst = np.arange(500 * k, 500 * (k + 1))
        jobs.append(("m2l", wl.random_shifts(rng, 500, 2.0, 6.0), rng.integers(0, n, 500), dst))
    dst7 = np.concatenate([np.arange(0, 250), np.arange(3000, 3250)])  # overlaps the first job
    jobs.append(("m2l", wl.random_shifts(rng, 500, 2.0, 6.0), rng.integers(0, n, 500), dst7))
    jobs.append(("l2l", wl.random_shifts(rng, 250, 0.25, 0.5), np.arange(3000, 3250), np.arange(3500, 3750)))

    def run(queued):
        srv = sh.Server(ctx, pool_bytes=64 << 20, staging_bytes=8 << 20, streams=3, max_batch_jobs=16)
        t, M, L = make_tree(srv, orc, sh.SH_F64, P, n, 21)
        ids = []
        for op, r, s, d in jobs:
            ids.append(srv.submit(t, op, r, s, d))
            if not queued:
                srv.wait(ids.pop())
        for i in ids:
            srv.wait(i)
        out, _ = read_pool(srv, t, 1, P, n, sh.SH_F64)
        st = srv.stats()
        srv.close()
        return out, M, L, st

    alone, M, L, _ = run(False)
    mixed, _, _, st = run(True)
    print(f"[server] one tree: {st['batches']} batches, mean jobs/batch {st['mean_batch_jobs']:.2f}", flush=True)
    assert np.array_equal(alone, mixed)
    exp = L.copy()
    for op, r, s, d in jobs[:7]:
        exp[d] = orc.translate_batch("m2l", P, P, r, M[s])
    op, r, s, d = jobs[7]
    exp[d] = orc.translate_batch("l2l", P, P, r, exp[s])
    check(mixed, exp, P, "L", 4 * TOL[sh.SH_F64], "shared tree")


@pytest.mark.parametrize("dtype", [sh.SH_F64, sh.SH_F32], ids=DT_ID.get)
def test_server_trees_of_one_order_share_a_call(ctx, orc, dtype):
    """Jobs on several trees of the same dtype and orders are fused into one indexed call per
    operation (slots addressed from the start of the pool arena): each job's result equals the
    oracle's and, bit for bit, the same job run alone on its own server."""
    P, n = 7, 400
    ops = ["m2l", "m2m", "m2l", "l2l", "m2l"]
    print(f"[server] shared call {DT_ID[dtype]}", flush=True)

    def run(which):
        srv = sh.Server(ctx, pool_bytes=64 << 20, staging_bytes=8 << 20, streams=1, max_batch_jobs=16)
        # a tree of another order first, so the pools of interest do not start at offset 0
        srv.tree_create(dtype, 5, 37, 9, 11)
        trees = [make_tree(srv, orc, dtype, P, n, 40 + k) for k in range(len(ops))]
        ids = [srv.submit(trees[k][0], ops[k], *job_arrays(ops[k], n, 150 + 7 * k, 60 + k)) for k in which]
        for i in ids:
            srv.wait(i)
        st = srv.stats()
        outs = {k: read_pool(srv, trees[k][0], 0 if ops[k] == "m2m" else 1, P, n, dtype)[1] for k in which}
        srv.close()
        return outs, trees, st

    together, trees, st = run(range(len(ops)))
    print(f"[server] shared call: {st['batches']} batches for {len(ops)} jobs", flush=True)
    for k, op in enumerate(ops):
        alone, _, _ = run([k])
        assert np.array_equal(alone[k], together[k]), f"job {k} ({op}) differs alone and fused"
        t, M, L = trees[k]
        r, src, dst = job_arrays(op, n, 150 + 7 * k, 60 + k)
        C = M if op != "l2l" else L
        kind_in = "M" if op != "l2l" else "L"
        Cin = from_basis(to_basis(C, P, kind_in, dtype), P, kind_in, dtype)
        out = from_basis(together[k], P, "M" if op == "m2m" else "L", dtype)
        check_job(orc, dtype, op, P, r, Cin[src] if dtype == sh.SH_F64 else C[src], out[dst], f"shared call {op}")


def test_server_pack_buffers_reused_and_stats_window(ctx, orc):
    """Jobs submitted one after another pack into buffers that completed jobs returned (a
    larger job takes a new buffer, a smaller one a free larger buffer), and jobs whose records
    are copied to the staging in pieces by several threads (over 1 MiB): every result equals
    the oracle, and a repeated job equals its first run bit for bit.  stats_reset starts a
    new statistics window."""
    P, n = 6, 60000
    dtype = sh.SH_F64
    print("[server] pack buffers and stats window", flush=True)
    srv = sh.Server(ctx, pool_bytes=256 << 20, staging_bytes=16 << 20, streams=2)
    t, M, L = make_tree(srv, orc, dtype, P, n, 7)
    Cin = from_basis(to_basis(M, P, "M", dtype), P, "M", dtype)
    first = {}
    for k, count in enumerate([5000, 5000, 50000, 3000, 50000, 5000]):
        r, src, dst = job_arrays("m2l", n, count, 900 + count)
        srv.wait(srv.submit(t, "m2l", r, src, dst))
        out, _ = read_pool(srv, t, 1, P, n, dtype)
        if count in first:
            assert np.array_equal(out[dst], first[count]), f"job {k} ({count}) differs from its first run"
        else:
            check_job(orc, dtype, "m2l", P, r, Cin[src], out[dst], f"pack buffers {count}")
            first[count] = out[dst].copy()
    assert srv.stats()["jobs_done"] == 6
    srv.stats_reset()
    st = srv.stats()
    assert st["jobs_done"] == 0 and st["batches"] == 0 and st["translations_done"] == 0
    assert st["elapsed_s"] == 0.0 and st["p99_s"] == 0.0
    r, src, dst = job_arrays("m2l", n, 4000, 77)
    srv.wait(srv.submit(t, "m2l", r, src, dst))
    st = srv.stats()
    assert st["jobs_done"] == 1 and st["translations_done"] == 4000 and st["elapsed_s"] > 0
    srv.close()
