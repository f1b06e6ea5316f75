"""The uniform-octree FMM driver (sh_fmm_*) against the same FMM composed from oracle
primitives on the CPU, and against the direct sum (eq. nbody).

The CPU composition below builds its own box numbering, interaction lists and neighbour
lists with numpy (it shares nothing with the library's driver) and runs the oracle's P2M,
M2M, double-height M2L, L2L and L2P with the direct near field; the GPU result must match it
to 1e-11 of the largest value (the two differ only by rounding).  Against the direct sum the
error is the method's truncation error, which must fall with the order.
"""
import itertools

import numpy as np
import pytest

import oracle
import paper_2202_02847_amd as sh
from gpu_util import torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = sh.Context(max_order=32, device=0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def _grid(level):
    n = 2 ** level
    ijk = np.array(list(itertools.product(range(n), repeat=3)), dtype=np.int64)  # index (i n + j) n + k
    return n, ijk


def _centres(level, origin, width):
    n, ijk = _grid(level)
    return np.asarray(origin, float) + (ijk + 0.5) * (width / n)


def _particles(levels, npts, origin, width, seed):
    """npts uniform particles in every leaf, stored leaf by leaf; charges uniform in [-1, 1]."""
    rng = np.random.default_rng(seed)
    n, ijk = _grid(levels)
    w = width / n
    lo = np.asarray(origin, float) + ijk * w
    pts = lo[:, None, :] + rng.uniform(0.0, w, (len(ijk), npts, 3))
    q = rng.uniform(-1.0, 1.0, (len(ijk), npts))
    return pts, q


def _direct(pts, q, targets=None):
    """u(x_i) = sum_{j != i} q_j / |x_i - x_j| and its gradient (eq. nbody)."""
    x = pts.reshape(-1, 3)
    qq = q.reshape(-1)
    idx = np.arange(len(x)) if targets is None else targets
    out = np.zeros((len(idx), 4))
    step = max(1, min(256, (1 << 23) // len(x)))  # targets per pass: about 200 MB of differences
    for a in range(0, len(idx), step):
        ii = idx[a: a + step]
        d = x[ii][:, None, :] - x[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        r[np.arange(len(ii)), ii] = np.inf
        inv = 1.0 / r
        out[a: a + step, 0] = inv @ qq
        out[a: a + step, 1:] = -np.einsum("ij,ijk->ik", (inv ** 3) * qq[None, :], d)
    return out


def _oracle_fmm(orc, P, levels, origin, width, pts, q, orders=None):
    """The FMM from oracle primitives: P2M, M2M up, M2L over interaction lists, L2L down, L2P,
    plus the direct near field over the 27 neighbouring leaves.  orders[l - 2] is the order of
    level l (default P everywhere); M2M and L2L translate between the two levels' orders."""
    nleaf, npts = q.shape
    th = 16
    Pl = {lev: (orders[lev - 2] if orders else P) for lev in range(2, levels + 1)}
    M = {levels: orc.p2m_batch(Pl[levels], _centres(levels, origin, width), pts, q, nthreads=th)}
    for lev in range(levels, 2, -1):
        n, ijk = _grid(lev)
        parent = ((ijk[:, 0] // 2) * (n // 2) + ijk[:, 1] // 2) * (n // 2) + ijk[:, 2] // 2
        r = _centres(lev - 1, origin, width)[parent] - _centres(lev, origin, width)
        moved = orc.translate_batch("m2m", Pl[lev], Pl[lev - 1], r, M[lev], nthreads=th)
        M[lev - 1] = np.zeros((8 ** (lev - 1), moved.shape[1]))
        np.add.at(M[lev - 1], parent, moved)
    Lx = {}
    for lev in range(2, levels + 1):
        n, ijk = _grid(lev)
        c = _centres(lev, origin, width)
        src, dst = [], []
        for b, (i, j, k) in enumerate(ijk):
            for s, (a, bb, cc) in enumerate(ijk):
                if max(abs(a - i), abs(bb - j), abs(cc - k)) < 2:
                    continue  # neighbours (near field or parent level)
                if max(abs(a // 2 - i // 2), abs(bb // 2 - j // 2), abs(cc // 2 - k // 2)) > 1:
                    continue  # handled at the parent level
                src.append(s)
                dst.append(b)
        src, dst = np.array(src), np.array(dst)
        out = orc.translate_batch("m2l", Pl[lev], Pl[lev], c[dst] - c[src], M[lev][src], nthreads=th)
        Lx[lev] = np.zeros((8 ** lev, out.shape[1]))
        np.add.at(Lx[lev], dst, out)
    for lev in range(2, levels):
        n, ijk = _grid(lev + 1)
        parent = ((ijk[:, 0] // 2) * (n // 2) + ijk[:, 1] // 2) * (n // 2) + ijk[:, 2] // 2
        r = _centres(lev + 1, origin, width) - _centres(lev, origin, width)[parent]
        Lx[lev + 1] += orc.translate_batch("l2l", Pl[lev], Pl[lev + 1], r, Lx[lev][parent], nthreads=th)
    far = orc.l2p_batch(Pl[levels], _centres(levels, origin, width), pts, Lx[levels], nthreads=th)
    n, ijk = _grid(levels)
    near = np.zeros_like(far)
    for b, (i, j, k) in enumerate(ijk):
        nb = [s for s, (a, bb, cc) in enumerate(ijk) if max(abs(a - i), abs(bb - j), abs(cc - k)) <= 1]
        ys = pts[nb].reshape(-1, 3)
        qs = q[nb].reshape(-1)
        d = pts[b][:, None, :] - ys[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        inv = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 0.0)
        near[b, :, 0] = inv @ qs
        near[b, :, 1:] = -np.einsum("ij,ijk->ik", (inv ** 3) * qs[None, :], d)
    return (far + near).reshape(-1, 4)


def _gpu_fmm(ctx, P, levels, origin, width, pts, q, flags=0, orders=None):
    torch, dev = torch_dev()
    f = sh.Fmm(ctx, P, levels, origin, width, q.shape[1], orders=orders)
    d_p = torch.from_numpy(np.ascontiguousarray(pts.reshape(-1, 3))).to(dev)
    d_q = torch.from_numpy(np.ascontiguousarray(q.reshape(-1))).to(dev)
    d_o = torch.full((q.size, 4), np.nan, dtype=torch.float64, device=dev)
    f.evaluate(d_p, d_q, d_o, flags)
    torch.cuda.synchronize()
    desc = f.describe()
    f.close()
    return d_o.cpu().numpy(), desc


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# Leaves of at most 32 particles share a wavefront in L2P and the near field; larger leaves
# take one wavefront per 64 targets (40: one partial chunk, 70 and 130: several chunks).
@pytest.mark.parametrize("flags", [0, sh.SH_FMM_NO_GRAPH], ids=["graph", "eager"])
@pytest.mark.parametrize("P,levels,npts", [(6, 2, 5), (10, 3, 9), (17, 3, 3), (8, 2, 40), (7, 2, 70), (5, 2, 130)])
def test_fmm_matches_oracle_composition(ctx, orc, P, levels, npts, flags):
    origin, width = (-0.3, 0.1, 0.25), 2.0
    print(f"[fmm] P={P} levels={levels} npts={npts} flags={flags}", flush=True)
    pts, q = _particles(levels, npts, origin, width, seed=P * 10 + levels)
    got, desc = _gpu_fmm(ctx, P, levels, origin, width, pts, q, flags)
    assert np.isfinite(got).all()
    ref = _oracle_fmm(orc, P, levels, origin, width, pts, q)
    assert _rel(got[:, 0], ref[:, 0]) <= 1e-11
    assert _rel(got[:, 1:], ref[:, 1:]) <= 1e-11
    assert desc["leaves"] == 8 ** levels


@pytest.mark.parametrize("orders", [(12, 8), (7, 10), (16, 5)], ids=["12-8", "7-10", "16-5"])
def test_fmm_per_level_orders_match_oracle_composition(ctx, orc, orders):
    """Per-level orders (levels 2..L): M2M and L2L between different orders, M2L within a
    level, against the oracle composition with the same orders."""
    levels = len(orders) + 1
    npts = 4 if levels == 3 else 1
    origin, width = (0.2, -0.4, 0.0), 1.5
    print(f"[fmm] orders={orders}", flush=True)
    pts, q = _particles(levels, npts, origin, width, seed=sum(orders))
    got, desc = _gpu_fmm(ctx, 0, levels, origin, width, pts, q, orders=list(orders))
    ref = _oracle_fmm(orc, 0, levels, origin, width, pts, q, orders=list(orders))
    assert _rel(got[:, 0], ref[:, 0]) <= 1e-11
    assert _rel(got[:, 1:], ref[:, 1:]) <= 1e-11


def test_fmm_uniform_orders_equal_single_order(ctx):
    """sh_fmm_create(P) and sh_fmm_create_orders with P at every level run the same FMM."""
    levels, npts, P = 3, 5, 9
    origin, width = (0.0, 0.0, 0.0), 1.0
    pts, q = _particles(levels, npts, origin, width, seed=3)
    a, _ = _gpu_fmm(ctx, P, levels, origin, width, pts, q)
    b, _ = _gpu_fmm(ctx, 0, levels, origin, width, pts, q, orders=[P] * (levels - 1))
    assert np.array_equal(a, b)


def test_fmm_truncation_error_falls_with_order(ctx):
    """Against the direct sum: the error of the potential and gradient falls with P."""
    levels, npts = 3, 16
    origin, width = (0.0, 0.0, 0.0), 1.0
    pts, q = _particles(levels, npts, origin, width, seed=5)
    exact = _direct(pts, q)
    errs = []
    for P in (4, 8, 12, 16):
        got, _ = _gpu_fmm(ctx, P, levels, origin, width, pts, q)
        errs.append((_rel(got[:, 0], exact[:, 0]), _rel(got[:, 1:], exact[:, 1:])))
    print("[fmm] errors vs direct", errs, flush=True)
    for a, b in zip(errs, errs[1:]):
        assert b[0] < a[0] and b[1] < a[1]
    # the CPU composition of the same method gives 2.5e-7 and 8.4e-8 at P = 16
    assert errs[-1][0] < 1e-5 and errs[-1][1] < 1e-5


def test_fmm_graph_replays_match_eager(ctx):
    """The captured graph, replayed several times with eager evaluations of other inputs on
    the same handle in between, gives the eager result bit for bit every time."""
    torch, dev = torch_dev()
    P, levels, npts = 10, 3, 9
    origin, width = (0.0, 0.0, 0.0), 1.0
    pts, q = _particles(levels, npts, origin, width, seed=77)
    _, q2 = _particles(levels, npts, origin, width, seed=78)
    f = sh.Fmm(ctx, P, levels, origin, width, npts)
    d_p = torch.from_numpy(np.ascontiguousarray(pts.reshape(-1, 3))).to(dev)
    d_q = torch.from_numpy(np.ascontiguousarray(q.reshape(-1))).to(dev)
    d_q2 = torch.from_numpy(np.ascontiguousarray(q2.reshape(-1))).to(dev)
    d_o = torch.empty((q.size, 4), dtype=torch.float64, device=dev)
    d_o2 = torch.empty_like(d_o)
    f.evaluate(d_p, d_q, d_o, sh.SH_FMM_NO_GRAPH)
    torch.cuda.synchronize()
    eager = d_o.cpu().numpy().copy()
    for rep in range(4):
        d_o.fill_(np.nan)
        f.evaluate(d_p, d_q, d_o)  # captured on the first pass, replayed after
        torch.cuda.synchronize()
        assert np.array_equal(d_o.cpu().numpy(), eager), rep
        f.evaluate(d_p, d_q2, d_o2, sh.SH_FMM_NO_GRAPH)  # other work on the same pools
        torch.cuda.synchronize()
    f.close()


def test_fmm_error_is_set_by_the_lowest_level_order(ctx):
    """The premise of one order for every level: on a uniform 4-level tree the leaf level
    alone, and the two coarser levels alone, each leave about the error of the uniform choice.
    Raising the other levels' orders by 2-5 (each order is a factor of about 0.44 in the error)
    lowers the error by less than 1.7x, so a cheaper leaf order cannot be bought with dearer
    coarse ones."""
    levels, npts = 4, 4
    origin, width = (0.0, 0.0, 0.0), 1.0
    pts, q = _particles(levels, npts, origin, width, seed=101)
    exact = _direct(pts, q)[:, 0]
    err = {}
    for orders in ((10, 10, 10), (15, 13, 10), (10, 10, 12), (12, 12, 12)):
        got, _ = _gpu_fmm(ctx, 0, levels, origin, width, pts, q, orders=list(orders))
        err[orders] = _rel(got[:, 0], exact)
    print("[fmm] per-level orders", {k: f"{v:.2e}" for k, v in err.items()}, flush=True)
    uniform = err[(10, 10, 10)]
    assert err[(15, 13, 10)] > uniform / 1.7   # leaf at 10, coarse levels raised
    assert err[(10, 10, 12)] > uniform / 1.7   # coarse levels at 10, leaf raised
    assert err[(12, 12, 12)] < uniform / 2.5   # raising every level does lower it


@pytest.mark.parametrize("levels,npts", [(3, 10), (2, 30), (4, 4)], ids=["3x10", "2x30", "4x4"])
@pytest.mark.parametrize("tol", [1e-3, 1e-5])
def test_fmm_orders_for_tolerance_meet_target(ctx, tol, levels, npts):
    """Orders chosen for a target meet it against the direct sum on trees outside the
    measurements the rule was fitted to (3 levels with 10 particles per leaf, and the 2- and
    4-level ends of its range, seeds not used there)."""
    origin, width = (0.0, 0.0, 0.0), 1.0
    pts, q = _particles(levels, npts, origin, width, seed=29)
    orders = sh.sh_fmm_orders_for_tolerance(tol, levels)
    got, _ = _gpu_fmm(ctx, 0, levels, origin, width, pts, q, orders=orders)
    err = _rel(got[:, 0], _direct(pts, q)[:, 0])
    print(f"[fmm] levels={levels} npts={npts} tol={tol} orders={orders} err={err:.2e}", flush=True)
    assert err <= tol


def test_fmm_rejects_bad_arguments(ctx):
    with pytest.raises(sh.ShError):
        sh.Fmm(ctx, 10, 1, (0, 0, 0), 1.0, 8)  # fewer than two levels: no interaction list
    with pytest.raises(sh.ShError):
        sh.Fmm(ctx, 10, 7, (0, 0, 0), 1.0, 8)  # above SH_FMM_MAX_LEVELS
    with pytest.raises(sh.ShError):
        sh.Fmm(ctx, 10, 3, (0, 0, 0), 0.0, 8)  # empty cube
    with pytest.raises(sh.ShError):
        sh.Fmm(ctx, 33, 3, (0, 0, 0), 1.0, 8)  # order above the context's
    with pytest.raises(sh.ShError):
        sh.Fmm(ctx, 0, 3, (0, 0, 0), 1.0, 8, orders=[10, 0])  # an order below 1
    with pytest.raises(sh.ShError):
        sh.Fmm(ctx, 10, 3, (0, 0, 0), 1.0, 1 << 62)  # more than 2^31 particles (no overflow)


def test_fmm_bench_size_sampled_vs_direct(ctx):
    """The benchmark's FMM (4 levels x 64 uniform particles = 262,144, P = 10): 512 sampled
    particles against the direct sum.  The error is the method's truncation error at P = 10
    (about 2e-5 in the potential for these trees; 1e-4 is the bound)."""
    levels, npts, P = 4, 64, 10
    origin, width = (0.0, 0.0, 0.0), 1.0
    pts, q = _particles(levels, npts, origin, width, seed=11)
    got, desc = _gpu_fmm(ctx, P, levels, origin, width, pts, q)
    assert desc["leaves"] == 4096 and np.isfinite(got).all()
    pick = np.sort(np.random.default_rng(1).choice(q.size, 512, replace=False))
    exact = _direct(pts, q, pick)
    e_u, e_g = _rel(got[pick, 0], exact[:, 0]), _rel(got[pick, 1:], exact[:, 1:])
    print(f"[fmm] 262144 particles P=10: sampled error potential {e_u:.2e} gradient {e_g:.2e}", flush=True)
    assert e_u <= 1e-4 and e_g <= 1e-3
