"""Seeded synthetic inputs for the translation workloads.

This module holds random-number recipes only -- no harmonic or translation arithmetic --
so that the CPU oracle (tests) and the HIP path (tests, benchmark) can draw identical
inputs from it.  Multipole coefficients are produced from these point clouds by the
caller (the oracle's P2M in the tests, the library's device P2M in the benchmark).

Recipes (all coordinates relative to the expansion centre):
  * cluster: ``npts`` points uniform in the cube [-1/2, 1/2]^3 (a unit box), charges
    uniform in [-1, 1];
  * random shift: a direction uniform on the sphere (normalised Gaussian) times a length
    uniform in [lo, hi];
  * octree M2L shift: one of the 316 integer offsets in [-3, 3]^3 with max-norm > 1 (the
    well-separated boxes of a uniform-octree level of unit box width);
  * octree parent/child shift: one of the 8 offsets (+-1/4, +-1/4, +-1/4);
  * mixed work list: operation M2M / M2L / L2L with probabilities 0.2 / 0.6 / 0.2, input
    and output orders drawn independently, 70% from U{6..12} and 30% from U{3..30}, a
    random shift of length in [2, 6] for every operation.
"""
from __future__ import annotations

import itertools

import numpy as np

SEED_BASE = 2202


def rng_for(config: int, stream: int = 0) -> np.random.Generator:
    """Independent PCG64 stream per (config, purpose)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE + config, stream])))


def clusters(rng, count: int, npts: int, half: float = 0.5):
    pts = rng.uniform(-half, half, (count, npts, 3))
    q = rng.uniform(-1.0, 1.0, (count, npts))
    return pts, q


def directions(rng, count: int):
    v = rng.normal(size=(count, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def random_shifts(rng, count: int, lo: float, hi: float):
    return directions(rng, count) * rng.uniform(lo, hi, (count, 1))


def octree_offsets() -> np.ndarray:
    """The 316 well-separated integer offsets of a uniform octree level (343 - 27)."""
    offs = [o for o in itertools.product(range(-3, 4), repeat=3) if max(abs(c) for c in o) > 1]
    return np.array(offs, dtype=np.float64)


def child_offsets() -> np.ndarray:
    return np.array(list(itertools.product((-0.25, 0.25), repeat=3)), dtype=np.float64)


def octree_shifts(rng, count: int, grouped: bool = False):
    """M2L shifts drawn from the 316 offsets; grouped=True sorts them by direction index."""
    offs = octree_offsets()
    idx = rng.integers(0, len(offs), count)
    if grouped:
        idx = np.sort(idx)
    return offs[idx], idx


def child_shifts(rng, count: int):
    offs = child_offsets()
    idx = rng.integers(0, len(offs), count)
    return offs[idx], idx


def mixed_orders(rng, count: int, lo: int = 3, hi: int = 30, core=(6, 12), core_frac: float = 0.7):
    """Orders skewed toward the common range: core_frac from U{core}, the rest from U{lo..hi}."""
    core_draw = rng.integers(core[0], core[1] + 1, count)
    wide_draw = rng.integers(lo, hi + 1, count)
    pick = rng.uniform(size=count) < core_frac
    return np.where(pick, core_draw, wide_draw)


def config1(n: int = 1000, P: int = 8):
    """Plain method, FP64, P=8: M2L with |r| in [2,4]; M2M and L2L with |r| in [0.25,0.5]."""
    pts, q = clusters(rng_for(1, 0), n, 20)
    return {
        "P": P, "pts": pts, "q": q,
        "r_m2l": random_shifts(rng_for(1, 1), n, 2.0, 4.0),
        "r_m2m": random_shifts(rng_for(1, 2), n, 0.25, 0.5),
        "r_l2l": random_shifts(rng_for(1, 3), n, 0.25, 0.5),
    }


def config2(n_m2l: int = 1 << 20, n_child: int = 1 << 17, npts: int = 32, P: int = 10, seed_config: int = 2):
    """Uniform-octree batch: M2L over the 316 offsets and parent/child M2M, L2L."""
    pts, q = clusters(rng_for(seed_config, 0), n_m2l, npts)
    r, idx = octree_shifts(rng_for(seed_config, 1), n_m2l)
    rc, _ = child_shifts(rng_for(seed_config, 2), n_child)
    rl, _ = child_shifts(rng_for(seed_config, 3), n_child)
    return {"P": P, "pts": pts, "q": q, "r_m2l": r, "dir_idx": idx, "r_m2m": rc, "r_l2l": rl}


def config4(n: int = 500_000, npts: int = 20, lo: int = 3, hi: int = 30, seed_config: int = 4,
            op_prob=(0.2, 0.6, 0.2)):
    """Mixed-order work list: op codes (0 M2M, 1 M2L, 2 L2L), orders, shifts, and one
    cluster per item (its source points)."""
    op = rng_for(seed_config, 0).choice(3, size=n, p=list(op_prob)).astype(np.int32)
    p_in = mixed_orders(rng_for(seed_config, 1), n, lo, hi).astype(np.int32)
    p_out = mixed_orders(rng_for(seed_config, 2), n, lo, hi).astype(np.int32)
    r = random_shifts(rng_for(seed_config, 3), n, 2.0, 6.0)
    pts, q = clusters(rng_for(seed_config, 4), n, npts)
    return {"op": op, "p_in": p_in, "p_out": p_out, "r": r, "pts": pts, "q": q}
