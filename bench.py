"""Benchmark of the batched translations on one MI355X.

A step is one pass of the whole path over the uniform-octree batch: 2^20 M2L at P=10
(shifts from the 316 well-separated offsets, multipoles of 32 points per unit box),
plus 2^17 parent/child M2M and 2^17 L2L (offsets (+-1/4)^3; the L2L inputs are M2L
outputs), all FP64 in the paper's basis.  Inputs are generated and resident in HBM
before the timed region.  ``value`` is M2L translations per second of whole steps
(the M2M and L2L time counts against it).

Also reported (outside the timed steps): M2L at P=16 and P=30 on the same generator,
the FP32 normalised-basis path, the direct O(P^4) kernel, per-kernel HIP-event times,
the roofline of the dominant kernel and the CPU oracle timed on this host.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "M2L translations/s at P=10/16/30 vs plain FP64 path; p50/p99 job latency"
HBM_PEAK_GBS = 8000.0


def solid(P):
    return P * (P + 1)


def bytes_per_translation(p_in, p_out, elem):
    """Algorithmic HBM bytes of one translation: input solid + output solid + shift."""
    return (solid(p_in) + solid(p_out) + 3) * elem


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_octree_inputs(sh, ctx, torch, dev, P, n, npts=32, seed_config=2, n_child=0):
    from paper_2202_02847_amd import workloads as wl

    c = wl.config2(n_m2l=n, n_child=max(n_child, 1), npts=npts, P=P, seed_config=seed_config)
    d_pts = torch.from_numpy(c["pts"]).to(dev)
    d_q = torch.from_numpy(c["q"]).to(dev)
    d_c = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    d_M = torch.empty((n, solid(P)), dtype=torch.float64, device=dev)
    sh.sh_p2m_batch_f64(ctx, P, n, d_c, npts, d_pts, d_q, d_M, solid(P))
    d_r = torch.from_numpy(c["r_m2l"]).to(dev)
    out = {"M": d_M, "r": d_r, "r_m2m": torch.from_numpy(c["r_m2m"]).to(dev),
           "r_l2l": torch.from_numpy(c["r_l2l"]).to(dev)}
    del d_pts, d_q, d_c
    torch.cuda.synchronize()
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "m2l_p10_f64_octree_traffic.json")


def measured_traffic():
    """HBM bytes per launch of the M2L P=10 FP64 kernel from the committed FETCH_SIZE /
    WRITE_SIZE counter runs, if they were taken on the current kernel sources (else None)."""
    from paper_2202_02847_amd import profiling

    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != profiling.kernel_source_hash():
        return None
    return round(rec["traffic_bytes"])


def norm_weights(sh, torch, dev, P, kind):
    """Normalisation factors of a solid of order P (kind 0: multipole, 1: local), taken from
    the library's host helper applied to a solid of ones."""
    w = sh.sh_normalise_f64(kind, P, np.ones((1, solid(P))))[0]
    return torch.from_numpy(w).to(dev)


def run_mixed(sh, ctx, torch, dev, dtype, n=500_000, reps=5):
    """The mixed-order work list: n items (M2M/M2L/L2L, orders 3..30 skewed toward 6..12,
    |r| in [2, 6]) through one autotuned plan, executed as one graph launch per pass.
    Inputs are device P2M multipoles of 20-point clusters (used as the input of every
    item, L2L included: the values do not change the work), normalised for FP32."""
    from paper_2202_02847_amd import arena
    from paper_2202_02847_amd import workloads as wl

    c = wl.config4(n)
    op, p_in, p_out = c["op"], c["p_in"], c["p_out"]
    in_off, in_total = arena.packed_offsets(p_in, group_by_order=True)
    out_off, out_total = arena.packed_offsets(p_out)
    f32 = dtype == sh.SH_F32
    tdt = torch.float32 if f32 else torch.float64
    d_in = torch.empty(in_total, dtype=tdt, device=dev)
    npts = c["pts"].shape[1]
    for P, first, idx in arena.order_blocks(p_in, in_off):
        k = len(idx)
        d_pts = torch.from_numpy(np.ascontiguousarray(c["pts"][idx])).to(dev)
        d_q = torch.from_numpy(np.ascontiguousarray(c["q"][idx])).to(dev)
        d_c = torch.zeros((k, 3), dtype=torch.float64, device=dev)
        M = torch.empty((k, solid(P)), dtype=torch.float64, device=dev)
        sh.sh_p2m_batch_f64(ctx, P, k, d_c, npts, d_pts, d_q, M, solid(P))
        if f32:
            M = M * norm_weights(sh, torch, dev, P, 0)
        d_in[first:first + M.numel()] = M.reshape(-1).to(tdt)
    del c["pts"], c["q"]
    items = sh.make_items(op, p_in, p_out, in_off, out_off, c["r"])
    t0 = time.perf_counter()
    plan = sh.Plan(ctx, dtype, items, sh.SH_PLAN_AUTOTUNE)
    t_plan = time.perf_counter() - t0
    d_out = torch.empty(out_total, dtype=tdt, device=dev)
    t = time_launch(torch, lambda: plan.execute(d_in, in_total, d_out, out_total), reps)
    assert bool(torch.isfinite(d_out).all()), "non-finite output in the mixed list"
    elem = 4 if f32 else 8
    nbytes = float(np.sum(p_in.astype(np.int64) * (p_in + 1) + p_out.astype(np.int64) * (p_out + 1))) * elem \
        + 56.0 * n
    desc = plan.describe()
    plan.close()
    return {"items": n, "per_s": n / t, "ms": round(t * 1e3, 4), "frac_hbm": nbytes / t / 1e9 / HBM_PEAK_GBS,
            "plan_create_s": round(t_plan, 3),
            "bins": [f"{b['mapping']}:{b['op']}:{b['bucket']}:{b['items']}" for b in desc["bins"]]}


def degree_error(got, ref, P):
    """Per-translation max over degrees n of max_m |got - ref| / max_m |ref| (normalised basis)."""
    worst = np.zeros(got.shape[0])
    for n in range(P):
        a, b = n * (n + 1), (n + 1) * (n + 2)
        den = np.maximum(np.abs(ref[:, a:b]).max(axis=1), 1e-300)
        worst = np.maximum(worst, np.abs(got[:, a:b] - ref[:, a:b]).max(axis=1) / den)
    return worst


def run_precision(sh, ctx, torch, dev, P=16, n=1 << 20, reps=5, sample=4096):
    """Shared-direction M2L at order P: 2^20 translations grouped by the 316 octree offsets,
    FP32 normalised solids.  Times the BF16x6 and BF16x3 matrix-core paths, the FP32 and
    FP64 rotation paths on the same multipoles, and states each FP32 path's per-degree error
    against the FP64 GPU path (itself held to 1e-12 of the oracle by the tests): *_err against
    the FP64 result of the FP64 input, *_arith_err against the FP64 result of the FP32-rounded
    input (the form's own arithmetic), and input_rounding_err between those two references."""
    from paper_2202_02847_amd import workloads as wl

    c = wl.config2(n_m2l=n, n_child=8, npts=32, P=P, seed_config=3)
    order = np.argsort(c["dir_idx"], kind="stable")
    offs = wl.octree_offsets()
    counts = np.bincount(c["dir_idx"], minlength=len(offs))
    S = solid(P)
    d_pts = torch.from_numpy(np.ascontiguousarray(c["pts"][order])).to(dev)
    d_q = torch.from_numpy(np.ascontiguousarray(c["q"][order])).to(dev)
    d_r64 = torch.from_numpy(np.ascontiguousarray(c["r_m2l"][order])).to(dev)
    del c
    d_M = torch.empty((n, S), dtype=torch.float64, device=dev)
    sh.sh_p2m_batch_f64(ctx, P, n, torch.zeros((n, 3), dtype=torch.float64, device=dev), d_pts.shape[1], d_pts,
                        d_q, d_M, S)
    del d_pts, d_q
    wM, wL = norm_weights(sh, torch, dev, P, 0), norm_weights(sh, torch, dev, P, 1)
    d_M32 = (d_M * wM).float()
    d_cs = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)).to(dev)
    d_L64 = torch.empty((n, S), dtype=torch.float64, device=dev)
    d_L32 = torch.empty((n, S), dtype=torch.float32, device=dev)
    res = {"P": P, "translations": n, "classes": len(offs)}
    t = time_launch(torch, lambda: sh.sh_m2l_batch_f64(ctx, P, P, n, d_r64, d_M, S, d_L64, S), reps)
    res["rot_f64_per_s"] = n / t
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    pick = torch.from_numpy(np.sort(rng.choice(n, sample, replace=False))).to(dev)
    ref = (d_L64[pick] * wL).cpu().numpy()  # FP64 result in the normalised basis
    # the FP64 path on the FP32-rounded input (and shift): the exact result an FP32 entry point
    # can reach; its distance from ref is what rounding the input alone costs
    d_Mr = d_M32.double() / wM
    d_r32 = d_r64.float()
    d_Lr = torch.empty_like(d_L64)
    sh.sh_m2l_batch_f64(ctx, P, P, n, d_r32.double(), d_Mr, S, d_Lr, S)
    ref_r = (d_Lr[pick] * wL).cpu().numpy()
    del d_Mr, d_Lr
    e = degree_error(ref_r, ref, P)
    res["input_rounding_err_max"], res["input_rounding_err_p99"] = float(e.max()), float(np.quantile(e, 0.99))
    t = time_launch(torch, lambda: sh.sh_m2l_batch_f32(ctx, P, P, n, d_r32, d_M32, S, d_L32, S), reps)
    res["rot_f32_per_s"] = n / t
    got = d_L32[pick].double().cpu().numpy()
    e, ea = degree_error(got, ref, P), degree_error(got, ref_r, P)
    res["rot_f32_err_max"], res["rot_f32_err_p99"] = float(e.max()), float(np.quantile(e, 0.99))
    res["rot_f32_arith_err_max"], res["rot_f32_arith_err_p99"] = float(ea.max()), float(np.quantile(ea, 0.99))
    bpt = bytes_per_translation(P, P, 4) - 12  # FP32 solids in and out, no shift array
    for prec, name in ((sh.SH_SHARED_BF16X6, "bf16x6"), (sh.SH_SHARED_BF16X3, "bf16x3"), (sh.SH_SHARED_FP32, "fp32mfma")):
        t0 = time.perf_counter()
        op = sh.Shared(ctx, "m2l", P, P, offs, prec)
        res[f"{name}_build_s"] = round(time.perf_counter() - t0, 3)
        res[f"{name}_operator_bytes"] = op.nbytes()
        d_L32.zero_()
        t = time_launch(torch, lambda: op.execute(n, d_cs, d_M32, S, d_L32, S), reps)
        res[f"{name}_per_s"] = n / t
        res[f"{name}_ms"] = round(t * 1e3, 4)
        if prec == sh.SH_SHARED_FP32:
            res[f"{name}_frac_mfma_fp32"] = 2.0 * S * S * n / t / 157.3e12
        else:
            products = 6 if prec == sh.SH_SHARED_BF16X6 else 3
            res[f"{name}_frac_mfma_bf16"] = 2.0 * S * S * products * n / t / 2.5e15
        res[f"{name}_frac_hbm"] = bpt * n / t / 1e9 / HBM_PEAK_GBS
        got = d_L32[pick].double().cpu().numpy()
        e, ea = degree_error(got, ref, P), degree_error(got, ref_r, P)
        res[f"{name}_err_max"], res[f"{name}_err_p99"] = float(e.max()), float(np.quantile(e, 0.99))
        res[f"{name}_arith_err_max"], res[f"{name}_arith_err_p99"] = float(ea.max()), float(np.quantile(ea, 0.99))
        op.close()
    del d_M, d_M32, d_L64, d_L32
    torch.cuda.empty_cache()
    return res


SERVE_ORDERS = [4, 8, 16, 24, 30]


def _serving_trees(sh, srv, n_slots):
    """One resident tree per (order, dtype) of the serving workload, pools filled with a tiled
    random block (the values do not change the work)."""
    trees = {}
    for P in SERVE_ORDERS:
        for dt in (sh.SH_F64, sh.SH_F32):
            t = srv.tree_create(dt, P, n_slots, P, n_slots)
            npdt = np.float64 if dt == sh.SH_F64 else np.float32
            block = np.random.default_rng(P).normal(size=(1024, P * (P + 1))).astype(npdt) * 1e-2
            for pool_id in (0, 1):
                for first in range(0, n_slots, 1024):
                    srv.tree_write(t, pool_id, first, block[: min(1024, n_slots - first)])
            trees[(P, dt)] = t
    return trees


def _serving_job(sh, rng, n_slots):
    """One job of the serving workload: order, dtype, operation, shifts, source and destination
    slots.  M2L reads random multipole slots and writes a run of distinct local slots; M2M and
    L2L read the first half of a pool and write the second."""
    from paper_2202_02847_amd import workloads as wl

    P = SERVE_ORDERS[rng.integers(len(SERVE_ORDERS))]
    dt = (sh.SH_F64, sh.SH_F32)[rng.integers(2)]
    op = ("m2m", "m2l", "l2l")[rng.choice(3, p=[0.2, 0.6, 0.2])]
    count = int(10 ** rng.uniform(3, 5))
    r = wl.random_shifts(rng, count, 2.0, 6.0)
    if op == "m2l":
        src = rng.integers(0, n_slots, count)
        dst = (rng.integers(n_slots) + np.arange(count)) % n_slots
    else:
        half = n_slots // 2
        src = rng.integers(0, half, count)
        dst = half + (rng.integers(half) + np.arange(count)) % half
    return P, dt, op, r, src, dst


def _serving_stats(st, rate, staging):
    return {"jobs": st["jobs_done"], "failed": st["jobs_failed"], "offered_jobs_per_s": rate,
            "duration_s": round(st["elapsed_s"], 3),
            "translations_per_s": st["translations_done"] / max(st["elapsed_s"], 1e-9),
            "p50_ms": round(st["p50_s"] * 1e3, 3), "p99_ms": round(st["p99_s"] * 1e3, 3),
            "max_ms": round(st["max_s"] * 1e3, 3), "mean_batch_jobs": round(st["mean_batch_jobs"], 2),
            "batches": st["batches"], "queue_peak": st["queue_peak"], "jobs_deferred": st["jobs_deferred"],
            "staging_budget_mb": round(staging / 2 ** 20, 1),
            "staging_peak_mb": round(st["staging_peak_bytes"] / 2 ** 20, 1)}


def run_serving(sh, ctx, torch, dev, seconds=50.0, rate=200.0, n_slots=1 << 18, staging=10 << 20,
                sat_jobs=600, sat_threads=4):
    """The serving workload: a Poisson stream (mean `rate` jobs/s, for `seconds`) of jobs of
    10^3..10^5 translations (log-uniform), one order P in {4, 8, 16, 24, 30} and one dtype
    (FP32 or FP64) per job, on resident trees (one per order and dtype, n_slots multipoles and
    locals each).  Operations M2M / M2L / L2L with probabilities 0.2 / 0.6 / 0.2.  The staging
    budget (admission by footprint, 80 B per translation) holds one of the largest jobs (8 MB),
    so admission defers jobs under bursts.  Latency: submission to completion.

    Then a saturation leg: `sat_jobs` jobs of the same distribution queued at once (closed
    loop) by `sat_threads` client threads, through a new server with a staging budget 8x
    larger (one untimed pass, then the statistics window is reset and a second pass timed;
    each plain leg below is likewise run once untimed first), against the same job stream
    issued as plain calls: per job, its shift and slot arrays copied from the same host arrays
    to the device and one indexed batched call, on one stream.  Both legs are timed from the
    first submission (call) to the last completion; submit_s is the served leg's submission
    loop (validation and packing on the submitting thread).  plain_device_resident_s times the
    same calls with the job arrays already on the device (their transfer not timed): the plain
    path's device-side lower bound."""
    pool = sum(2 * n_slots * P * (P + 1) * (8 if dt == sh.SH_F64 else 4) for P in SERVE_ORDERS
               for dt in (sh.SH_F64, sh.SH_F32))
    srv = sh.Server(ctx, pool_bytes=pool + (64 << 20), staging_bytes=staging, streams=4, max_batch_jobs=64)
    trees = _serving_trees(sh, srv, n_slots)
    from paper_2202_02847_amd import workloads as wl

    rng = wl.rng_for(5, 0)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, int(rate * seconds * 1.5)))
    arrivals = arrivals[arrivals < seconds]
    ids = []
    log(f"[bench] serving {len(arrivals)} jobs over {seconds:.0f} s")
    t0 = time.perf_counter()
    for k, a in enumerate(arrivals):
        if k and k % 2000 == 0:
            log(f"[bench] serving: {k} jobs submitted")
        P, dt, op, r, src, dst = _serving_job(sh, rng, n_slots)
        delay = t0 + a - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(trees[(P, dt)], op, r, src, dst))
    srv.drain()
    for i in ids:
        srv.wait(i)
    res = _serving_stats(srv.stats(), rate, staging)
    srv.close()

    # ---- saturation: every job queued at once, served vs plain calls ----
    log(f"[bench] serving saturation: {sat_jobs} jobs")
    rng = wl.rng_for(5, 1)
    jobs = [_serving_job(sh, rng, n_slots) for _ in range(sat_jobs)]
    sat_staging = 8 * staging
    srv = sh.Server(ctx, pool_bytes=pool + (64 << 20), staging_bytes=sat_staging, streams=4, max_batch_jobs=64)
    trees = _serving_trees(sh, srv, n_slots)
    # clients: sat_threads host threads submit the jobs round robin (each call checks and packs
    # its job on the calling thread, outside the server lock)
    import threading

    def served_pass():
        ids_by = [[] for _ in range(sat_threads)]

        def client(k):
            for i in range(k, len(jobs), sat_threads):
                P, dt, op, r, src, dst = jobs[i]
                ids_by[k].append(srv.submit(trees[(P, dt)], op, r, src, dst))

        t0 = time.perf_counter()
        ths = [threading.Thread(target=client, args=(k,)) for k in range(sat_threads)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        t_submit = time.perf_counter() - t0
        srv.drain()
        for b in ids_by:
            for i in b:
                srv.wait(i)
        return t_submit

    # one untimed pass first, as the plain legs below run on warm allocators: the server's
    # pack buffers and staging are then in use, as in a server under steady load
    served_pass()
    srv.stats_reset()
    t_submit = served_pass()
    sat = _serving_stats(srv.stats(), None, sat_staging)
    srv.close()
    torch.cuda.empty_cache()
    # the plain path: resident pools as torch tensors, one indexed call per job on one stream
    pools = {}
    for P in SERVE_ORDERS:
        for dt in (sh.SH_F64, sh.SH_F32):
            tdt = torch.float64 if dt == sh.SH_F64 else torch.float32
            pools[(P, dt)] = [torch.full((n_slots, P * (P + 1)), 1e-2, dtype=tdt, device=dev) for _ in range(2)]

    def plain_pass():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for P, dt, op, r, src, dst in jobs:
            # the job as the server receives it: host arrays, shifts converted to the pool's dtype
            npdt = np.float64 if dt == sh.SH_F64 else np.float32
            d_r = torch.from_numpy(np.ascontiguousarray(r, npdt)).to(dev, non_blocking=True)
            d_s = torch.from_numpy(np.ascontiguousarray(src, np.int64)).to(dev, non_blocking=True)
            d_d = torch.from_numpy(np.ascontiguousarray(dst, np.int64)).to(dev, non_blocking=True)
            Mp, Lp = pools[(P, dt)]
            S = P * (P + 1)
            inp, out = (Mp, Lp) if op == "m2l" else ((Mp, Mp) if op == "m2m" else (Lp, Lp))
            sh.sh_translate_indexed(ctx, op, dt, P, P, len(src), d_r, d_s, inp, S, d_d, out, S)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    plain_pass()  # warm: torch's caching allocator holds the job arrays' sizes
    t_plain = plain_pass()
    # the same calls with every job's arrays already on the device (their transfer not timed):
    # the device-side lower bound of the plain path
    dev_jobs = []
    for P, dt, op, r, src, dst in jobs:
        npdt = np.float64 if dt == sh.SH_F64 else np.float32
        dev_jobs.append((P, dt, op, len(src), torch.from_numpy(np.ascontiguousarray(r, npdt)).to(dev),
                         torch.from_numpy(np.ascontiguousarray(src, np.int64)).to(dev),
                         torch.from_numpy(np.ascontiguousarray(dst, np.int64)).to(dev)))

    def resident_pass():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for P, dt, op, count, d_r, d_s, d_d in dev_jobs:
            Mp, Lp = pools[(P, dt)]
            S = P * (P + 1)
            inp, out = (Mp, Lp) if op == "m2l" else ((Mp, Mp) if op == "m2m" else (Lp, Lp))
            sh.sh_translate_indexed(ctx, op, dt, P, P, count, d_r, d_s, inp, S, d_d, out, S)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    resident_pass()
    t_resident = resident_pass()
    del dev_jobs
    ntr = sum(len(j[4]) for j in jobs)
    sat["plain_device_resident_s"] = round(t_resident, 4)
    sat["served_over_plain_device_resident"] = round(t_resident / max(sat["duration_s"], 1e-9), 3)
    sat["submit_s"] = round(t_submit, 4)
    sat["submit_threads"] = sat_threads
    sat["plain_translations_per_s"] = ntr / t_plain
    sat["plain_s"] = round(t_plain, 4)
    sat["served_over_plain"] = round(sat["translations_per_s"] / sat["plain_translations_per_s"], 3)
    res["saturation"] = sat
    del pools
    torch.cuda.empty_cache()
    return res


def l2p_flops_per_target(P):
    """Flops of the column-streamed L2P per target: for each of the P(P+1)/2 harmonics
    R_k^j, 6 for its recurrence, 4 for the potential term and 12 for the three gradient
    terms (reciprocals of the recurrence constants not counted)."""
    return 22 * P * (P + 1) // 2


def run_l2p(sh, ctx, torch, dev, P=10, boxes=1 << 14, npts=64, reps=10):
    """L2P (potential and gradient) of 2^14 boxes x 64 targets at P = 10: leaves of a
    uniform octree with 64 particles each, targets uniform in the box, local expansions
    of decaying random coefficients."""
    g = torch.Generator(device=dev)
    g.manual_seed(10)
    S = solid(P)
    c = torch.rand((boxes, 3), generator=g, device=dev, dtype=torch.float64)
    t = c[:, None, :] + torch.rand((boxes, npts, 3), generator=g, device=dev, dtype=torch.float64) - 0.5
    L = torch.randn((boxes, S), generator=g, device=dev, dtype=torch.float64) * 1e-2
    out = torch.empty((boxes, npts, 4), device=dev, dtype=torch.float64)
    s = time_launch(torch, lambda: sh.sh_l2p_batch_f64(ctx, P, boxes, c, npts, t, L, S, out), reps)
    n = boxes * npts
    flops = l2p_flops_per_target(P) * n / s
    return {"targets_per_s": n / s, "ms": round(s * 1e3, 4), "boxes": boxes, "targets_per_box": npts,
            "flops_per_target": l2p_flops_per_target(P), "frac_fp64_vector": round(flops / 78.6e12, 4),
            "bytes_per_target": 56}


def run_fmm(sh, ctx, torch, dev, P=10, levels=4, npts=64, reps=3):
    """One evaluation of the uniform-octree FMM (P2M, M2M, M2L, L2L, L2P, P2P) over 8^4 leaves
    of 64 uniform particles each (262,144 particles, charges uniform in [-1, 1])."""
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    n = 2 ** levels
    ijk = torch.stack(torch.meshgrid(*[torch.arange(n, device=dev, dtype=torch.float64)] * 3, indexing="ij"),
                      -1).reshape(-1, 3)
    pts = ((ijk[:, None, :] + torch.rand((n ** 3, npts, 3), generator=g, device=dev, dtype=torch.float64)) / n)
    pts = pts.reshape(-1, 3).contiguous()
    q = torch.rand((pts.shape[0],), generator=g, device=dev, dtype=torch.float64) * 2 - 1
    out = torch.empty((pts.shape[0], 4), device=dev, dtype=torch.float64)
    f = sh.Fmm(ctx, P, levels, (0.0, 0.0, 0.0), 1.0, npts)
    s = time_launch(torch, lambda: f.evaluate(pts, q, out), reps)
    d = f.describe()
    f.close()
    return {"particles": int(pts.shape[0]), "P": P, "levels": levels, "ms": round(s * 1e3, 3),
            "particles_per_s": pts.shape[0] / s, "m2l_per_eval": d["m2l"], "m2m_per_eval": d["m2m"],
            "l2l_per_eval": d["l2l"], "translation_calls": d["calls"]}


def time_launch(torch, fn, reps, warm_ms=30.0):
    """Average duration of fn() over reps launches, HIP events on torch's current stream
    (the stream the library launches on by default).  Untimed launches of fn run first until
    the device has been busy warm_ms (after the host-side setup between measurements the device
    runs the first 10-30 ms of work at a lower clock), and the start event is queued behind the
    last of them, so the device is still busy while the host issues the timed launches."""
    torch.cuda.synchronize()
    t_w = time.perf_counter()
    while True:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()
        if time.perf_counter() - t_w >= warm_ms / 1e3:
            break
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def cpu_baseline(seconds_target=10.0):
    import oracle
    from paper_2202_02847_amd import workloads as wl

    o = oracle.get()
    threads = len(os.sched_getaffinity(0))
    P = 10
    # calibrate on a small sample, then time a sample sized to ~seconds_target
    c = wl.config2(n_m2l=1 << 12, n_child=8, P=P)
    M = o.p2m_batch(P, np.zeros((1 << 12, 3)), c["pts"], c["q"], nthreads=threads)
    r = c["r_m2l"]
    t0 = time.perf_counter()
    o.translate_batch("m2l", P, P, r[:512], M[:512], nthreads=threads)
    dt = time.perf_counter() - t0
    # one pass over a 2^16-translation sample takes ~dt * 128; repeat it to ~seconds_target
    reps = (1 << 16) // len(M)
    Mr = np.tile(M, (reps, 1))
    rr = np.tile(r, (reps, 1))
    passes = int(max(1, min(64, seconds_target / max(dt * 128, 1e-6))))
    t0 = time.perf_counter()
    for _ in range(passes):
        o.translate_batch("m2l", P, P, rr, Mr, nthreads=threads)
    dt = time.perf_counter() - t0
    n = passes * len(Mr)
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    by_order = {}
    for PP, nn in ((16, 1 << 14), (30, 1 << 12)):
        cc = wl.config2(n_m2l=nn, n_child=8, P=PP)
        MM = o.p2m_batch(PP, np.zeros((nn, 3)), cc["pts"], cc["q"], nthreads=threads)
        t0 = time.perf_counter()
        o.translate_batch("m2l", PP, PP, cc["r_m2l"], MM, nthreads=threads)
        tt = time.perf_counter() - t0
        by_order[f"P{PP}"] = {"translations": nn, "seconds": round(tt, 3), "per_s": nn / tt,
                              "per_s_per_core": nn / tt / threads}
    return {"value": n / dt, "unit": "translations/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} M2L at P=10 FP64 (octree shifts, 32-point multipoles), "
                      f"double-height O(P^4) sum, OpenMP over {threads} threads, {dt:.1f} s; {cpu}",
            "per_core": n / dt / threads, "by_order": by_order}


def run_counters(sh, ctx, torch, dev, what, steps):
    """A short program for hardware-counter and kernel-trace runs: a plain copy of 2^27
    doubles (1 GiB read, 1 GiB written; the reference for FETCH_SIZE/WRITE_SIZE scaling),
    then `steps` launches of one workload and nothing else.

    what: "P" or "m2l:P"  octree M2L at order P, FP64 (2^20 translations, 2^18 above P=16)
          "m2l32:P"       the same in the FP32 normalised basis
          "shared6:P" / "shared3:P" / "sharedf32:P"
                          the shared-direction operator (BF16x6 / BF16x3 / FP32 MFMA) over
                          2^20 translations in the 316 octree classes
          "mixed64" / "mixed32"
                          the 500,000-item mixed-order list through one tuned plan
          "fmm"           the uniform-octree FMM, 262,144 particles at P=10"""
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()
    kind, _, arg = what.partition(":")
    if kind.isdigit():
        kind, arg = "m2l", kind
    steps = max(1, steps)
    if kind in ("m2l", "m2l32"):
        P = int(arg)
        n = 1 << 20 if P <= 16 else 1 << 18
        I = make_octree_inputs(sh, ctx, torch, dev, P, n)
        if kind == "m2l":
            d_in, d_r = I["M"], I["r"]
            d_out = torch.empty((n, solid(P)), dtype=torch.float64, device=dev)
            fn = sh.sh_m2l_batch_f64
        else:
            d_in = (I["M"] * norm_weights(sh, torch, dev, P, 0)).float()
            d_r = I["r"].float()
            d_out = torch.empty((n, solid(P)), dtype=torch.float32, device=dev)
            fn = sh.sh_m2l_batch_f32
        for _ in range(steps):
            fn(ctx, P, P, n, d_r, d_in, solid(P), d_out, solid(P))
    elif kind.startswith("shared"):
        from paper_2202_02847_amd import workloads as wl

        P = int(arg or 16)
        prec = {"shared6": sh.SH_SHARED_BF16X6, "shared3": sh.SH_SHARED_BF16X3,
                "sharedf32": sh.SH_SHARED_FP32}[kind]
        n = 1 << 20
        S = solid(P)
        c = wl.config2(n_m2l=n, n_child=8, npts=32, P=P, seed_config=3)
        order = np.argsort(c["dir_idx"], kind="stable")
        counts = np.bincount(c["dir_idx"], minlength=len(wl.octree_offsets()))
        d_pts = torch.from_numpy(np.ascontiguousarray(c["pts"][order])).to(dev)
        d_q = torch.from_numpy(np.ascontiguousarray(c["q"][order])).to(dev)
        del c
        d_M = torch.empty((n, S), dtype=torch.float64, device=dev)
        sh.sh_p2m_batch_f64(ctx, P, n, torch.zeros((n, 3), dtype=torch.float64, device=dev), d_pts.shape[1],
                            d_pts, d_q, d_M, S)
        d_M32 = (d_M * norm_weights(sh, torch, dev, P, 0)).float()
        del d_M, d_pts, d_q
        d_cs = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)).to(dev)
        d_L32 = torch.empty((n, S), dtype=torch.float32, device=dev)
        op = sh.Shared(ctx, "m2l", P, P, wl.octree_offsets(), prec)
        for _ in range(steps):
            op.execute(n, d_cs, d_M32, S, d_L32, S)
        torch.cuda.synchronize()
        op.close()
    elif kind in ("mixed64", "mixed32"):
        run_mixed(sh, ctx, torch, dev, sh.SH_F64 if kind == "mixed64" else sh.SH_F32, reps=steps)
    elif kind == "fmm":
        run_fmm(sh, ctx, torch, dev, reps=steps)
    else:
        raise SystemExit(f"unknown counter workload {what!r}")
    torch.cuda.synchronize()
    log(f"[counters] done: copy 1 GiB + {steps} x {what}")


def run_section(sh, ctx, torch, dev, name, args):
    """One extra section of the bench (returns its entries of the `extra` object)."""
    out = {}
    if name == "serving":
        log("[bench] serving")
        out["serving"] = run_serving(sh, ctx, torch, dev, seconds=args.serve_seconds)
    elif name == "precision":
        log("[bench] shared-direction precision forms P=16")
        out["precision_p16"] = run_precision(sh, ctx, torch, dev)
    elif name == "mixed":
        for dt, dname in ((sh.SH_F64, "f64"), (sh.SH_F32, "f32")):
            log(f"[bench] mixed-order list {dname}")
            out[f"mixed_list_{dname}"] = run_mixed(sh, ctx, torch, dev, dt)
            torch.cuda.empty_cache()
    elif name == "fmm":
        log("[bench] FMM P=10 262144 particles")
        out["fmm_p10_uniform_262k"] = run_fmm(sh, ctx, torch, dev)
    elif name == "l2p":
        log("[bench] L2P P=10")
        out["l2p_p10_f64"] = run_l2p(sh, ctx, torch, dev)
    elif name == "orders":
        for PP, nn_ in ((16, 1 << 20), (20, 1 << 18), (24, 1 << 18), (30, 1 << 18)):
            log(f"[bench] extra P={PP} n={nn_}")
            J = make_octree_inputs(sh, ctx, torch, dev, PP, nn_)
            SS = solid(PP)
            d_out = torch.empty((nn_, SS), dtype=torch.float64, device=dev)
            t = time_launch(torch, lambda: sh.sh_m2l_batch_f64(ctx, PP, PP, nn_, J["r"], J["M"], SS, d_out, SS), 3)
            out[f"m2l_p{PP}_f64_per_s"] = nn_ / t
            out[f"m2l_p{PP}_f64_frac_hbm"] = bytes_per_translation(PP, PP, 8) * nn_ / t / 1e9 / HBM_PEAK_GBS
            del J, d_out
            torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip P=16/30, FP32 and naive extras")
    ap.add_argument("--prewarm-ms", type=float, default=60.0,
                    help="untimed: run the step until the device has been busy this long before the "
                         "warm-up steps (after idle, MI355X runs the first 10-30 ms of work at a lower "
                         "clock)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--serve-seconds", type=float, default=50.0,
                    help="length of the serving workload's Poisson stream (200 jobs/s)")
    ap.add_argument("--counters", default="", metavar="WHAT",
                    help="counter/trace mode: one 1 GiB copy (the reference kernel for "
                         "FETCH_SIZE/WRITE_SIZE scaling), then --steps launches of one workload "
                         "(P or m2l:P, m2l32:P, shared6:P, shared3:P, sharedf32:P, mixed64, mixed32, "
                         "fmm), nothing else; prints no JSON line")
    ap.add_argument("--only", default="", choices=["", "serving", "precision", "mixed", "fmm", "l2p", "orders"],
                    help="run one extra section alone and print its JSON (no headline line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2202_02847_amd as sh

    dev = torch.device("cuda:0")
    ctx = sh.Context(max_order=32, device=0)
    if args.counters:
        run_counters(sh, ctx, torch, dev, args.counters, args.steps)
        return
    if args.only:
        print(json.dumps({"only": args.only, "extra": run_section(sh, ctx, torch, dev, args.only, args)}), flush=True)
        return
    P, n, nc = 10, 1 << 20, 1 << 17
    log(f"[bench] generating octree inputs P={P} n={n}")
    I = make_octree_inputs(sh, ctx, torch, dev, P, n, n_child=nc)
    S = solid(P)
    d_M, d_r = I["M"], I["r"]
    d_L = torch.empty((n, S), dtype=torch.float64, device=dev)
    d_M2 = torch.empty((nc, S), dtype=torch.float64, device=dev)
    d_L2 = torch.empty((nc, S), dtype=torch.float64, device=dev)
    r_m2m, r_l2l = I["r_m2m"][:nc].contiguous(), I["r_l2l"][:nc].contiguous()

    ev = []

    def m2l():
        sh.sh_m2l_batch_f64(ctx, P, P, n, d_r, d_M, S, d_L, S)

    def step(record=False):
        if record:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
        m2l()
        if record:
            e1.record()
            ev.append((e0, e1))
        sh.sh_m2m_batch_f64(ctx, P, P, nc, r_m2m, d_M, S, d_M2, S)
        sh.sh_l2l_batch_f64(ctx, P, P, nc, r_l2l, d_L, S, d_L2, S)

    # untimed: bring the device to its steady clock and power state (after idle, the M2L
    # launches of the first 10-30 ms ran up to 30% slower on one MI355X), ten steps at a time
    t_w, prewarm_steps = time.perf_counter(), 0
    while prewarm_steps == 0 or time.perf_counter() - t_w < args.prewarm_ms / 1e3:
        for _ in range(10):
            step()
        prewarm_steps += 10
        torch.cuda.synchronize()
    prewarm_ms = (time.perf_counter() - t_w) * 1e3
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps (after {prewarm_steps} untimed steps, {prewarm_ms:.0f} ms)")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(record=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert ctx.device_error() == 0
    ms_step = (t1 - t0) * 1e3 / args.steps
    m2l_s = float(np.mean([a.elapsed_time(b) for a, b in ev])) / 1e3
    value = n / (ms_step / 1e3)
    bpt = bytes_per_translation(P, P, 8)
    achieved = bpt * n / m2l_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                "kernel": "M2L P=10 FP64", "bytes_per_translation": bpt, "launch_ms": round(m2l_s * 1e3, 4)}
    extra = {"prewarm_steps": prewarm_steps, "prewarm_ms": round(prewarm_ms, 1),
             "m2l_p10_f64_per_s": n / m2l_s,
             "m2m_l2l_per_step_ms": round(ms_step - m2l_s * 1e3, 4),
             "all_translations_per_s": (n + 2 * nc) / (ms_step / 1e3)}

    if not args.no_extra:
        # device copy bandwidth (read + write) of a 2 GiB buffer, as measured context for the peak
        src = torch.ones(1 << 28, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        t = time_launch(torch, lambda: dst.copy_(src), 5)
        extra["copy_gbs"] = round(2 * src.numel() * 8 / t / 1e9, 1)
        del src, dst
        torch.cuda.empty_cache()
        # FP32 (normalised basis) at P=10 on the same multipoles
        w = norm_weights(sh, torch, dev, P, 0)
        d_M32 = (d_M * w).float()
        d_r32 = d_r.float()
        d_L32 = torch.empty((n, S), dtype=torch.float32, device=dev)
        t = time_launch(torch, lambda: sh.sh_m2l_batch_f32(ctx, P, P, n, d_r32, d_M32, S, d_L32, S), 20)
        extra["m2l_p10_f32_per_s"] = n / t
        extra["m2l_p10_f32_frac_hbm"] = bytes_per_translation(P, P, 4) * n / t / 1e9 / HBM_PEAK_GBS
        del d_M32, d_L32
        # single-height M2L (eq. m2lkernels, left) on the same batch
        t = time_launch(torch, lambda: sh.sh_m2l_batch_f64(ctx, P, P, n, d_r, d_M, S, d_L, S, sh.SH_SINGLE_HEIGHT), 20)
        extra["m2l_p10_single_height_f64_per_s"] = n / t
        extra["m2l_p10_single_height_f64_frac_hbm"] = bytes_per_translation(P, P, 8) * n / t / 1e9 / HBM_PEAK_GBS
        nv = 1 << 16
        t = time_launch(torch, lambda: sh.sh_m2l_naive_batch_f64(ctx, P, P, nv, d_r, d_M, S, d_L, S), 3)
        extra["m2l_p10_naive_f64_per_s"] = nv / t
        del d_M, d_L, d_M2, d_L2, I
        torch.cuda.empty_cache()
        for name in ("serving", "precision", "mixed", "fmm", "l2p", "orders"):
            extra.update(run_section(sh, ctx, torch, dev, name, args))
            torch.cuda.empty_cache()

    line = {"metric": METRIC, "value": value, "unit": "translations/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "uniform-octree batch: 2^20 M2L at P=10 (316 well-separated offsets, "
                                   "32-point multipoles) + 2^17 M2M + 2^17 L2L (offsets (+-1/4)^3), FP64",
                       "P": P, "m2l_per_step": n, "m2m_per_step": nc, "l2l_per_step": nc},
            "roofline": roofline}
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    line["extra"] = extra
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
