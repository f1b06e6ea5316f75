"""Helpers for the GPU parity tests: move numpy inputs through the C ABI and back."""
from __future__ import annotations

import math

import numpy as np

import oracle
import paper_2202_02847_amd as sh
from refmath import max_degree_error

TOL = {sh.SH_F64: 1e-12, sh.SH_F32: 1e-5}


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def weights_flat(P):
    """w_n^m = sqrt((n+m)!(n-m)!) laid out like a solid (same weight for Re and Im)."""
    w = np.ones(P * (P + 1))
    for n in range(P):
        for m in range(n + 1):
            v = math.sqrt(math.factorial(n + m) * math.factorial(n - m))
            w[n * (n + 1) + 2 * m] = v
            w[n * (n + 1) + 2 * m + 1] = v
    return w


IN_KIND = {"m2l": "M", "m2m": "M", "l2l": "L"}
OUT_KIND = {"m2l": "L", "m2m": "M", "l2l": "L"}


def to_basis(C, P, kind, dtype):
    """Paper basis -> the basis the dtype's entry points use (normalised for FP32)."""
    if dtype == sh.SH_F64:
        return np.asarray(C, np.float64)
    w = weights_flat(P)
    return (np.asarray(C, np.float64) * (w if kind == "M" else 1.0 / w)).astype(np.float32)


def from_basis(C, P, kind, dtype):
    if dtype == sh.SH_F64:
        return np.asarray(C, np.float64)
    w = weights_flat(P)
    return np.asarray(C, np.float64) * (1.0 / w if kind == "M" else w)


def run_batch(ctx, op, dtype, p_in, p_out, r, C, ld_in=None, ld_out=None, flags=0, out_init=None,
              naive=False):
    """Runs one batched call on numpy inputs (paper basis) and returns the outputs (paper basis)."""
    torch, dev = torch_dev()
    count = r.shape[0]
    s_in, s_out = p_in * (p_in + 1), p_out * (p_out + 1)
    ld_in = ld_in or s_in
    ld_out = ld_out or s_out
    tdt = torch.float64 if dtype == sh.SH_F64 else torch.float32
    npdt = np.float64 if dtype == sh.SH_F64 else np.float32
    Cb = to_basis(C.reshape(count, -1)[:, :s_in], p_in, IN_KIND[op], dtype)
    inp = np.zeros((count, ld_in), npdt)
    inp[:, :s_in] = Cb
    d_in = torch.from_numpy(inp).to(dev)
    d_r = torch.from_numpy(np.ascontiguousarray(r, npdt)).to(dev)
    if out_init is None:
        d_out = torch.full((count, ld_out), 7.0, dtype=tdt, device=dev)
    else:
        oi = np.zeros((count, ld_out), npdt)
        oi[:, :s_out] = to_basis(out_init, p_out, OUT_KIND[op], dtype)
        d_out = torch.from_numpy(oi).to(dev)
    if naive:
        sh.sh_m2l_naive_batch_f64(ctx, p_in, p_out, count, d_r, d_in, ld_in, d_out, ld_out, flags)
    else:
        sh.sh_translate_batch(ctx, op, dtype, p_in, p_out, count, d_r, d_in, ld_in, d_out, ld_out, flags)
    torch.cuda.synchronize()
    out = d_out.cpu().numpy()
    return from_basis(out[:, :s_out], p_out, OUT_KIND[op], dtype), out


# Conditioning: for some inputs (high order, shift shorter than the cluster radius) the
# plain FP64 sums themselves lose digits -- the FP64 oracle then differs from the exact
# value by more than 1e-12.  FP64 results are therefore compared with the long-double
# oracle, against max(1e-12, COND_FACTOR x the FP64 oracle's own error): 1e-12 wherever
# the definition is that well conditioned in FP64, otherwise no worse than a small
# multiple of the plain FP64 definition.
COND_FACTOR = 16.0


def dense_operator(orc, op, p_in, p_out, r):
    """The oracle's translation by shift r as a dense real matrix in the normalised basis
    (outputs x inputs): column j is the image of unit solid j."""
    K = p_in * (p_in + 1)
    T = orc.translate_batch(op, p_in, p_out, np.repeat(np.reshape(r, (1, 3)), K, axis=0), np.eye(K)).T
    w_in, w_out = weights_flat(p_in), weights_flat(p_out)
    s_in = w_in if IN_KIND[op] == "M" else 1.0 / w_in
    s_out = w_out if OUT_KIND[op] == "M" else 1.0 / w_out
    return T * s_out[:, None] / s_in[None, :]


def _bf16(x):
    """Round float32 values to bfloat16 (round to nearest even), returned as float32."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def _split_bf16(x, pieces):
    """x (float64 or float32) as a sum of `pieces` bfloat16 values, each rounded from the
    remainder of the previous ones (the split of the matrix-core forms)."""
    rest = np.asarray(x, np.float64)
    out = []
    for _ in range(pieces):
        p = _bf16(rest.astype(np.float32))
        out.append(p)
        rest = rest - p.astype(np.float64)
    return out


# Products of the BF16 split forms: (operator piece, input piece) index pairs.
BF16_PRODUCTS = {3: [(0, 0), (0, 1), (1, 0)], 6: [(0, 0), (0, 1), (1, 0), (0, 2), (1, 1), (2, 0)]}


class Plain32:
    """A plain FP32 evaluation of the same translations, as the reference for FP32 bounds.

    Each output of a translation is a dot product sum_k T_hat[i, k] a_k of the translation's
    dense operator (normalised basis) with its input.  Here the operator is built exactly
    (the FP64 oracle applied to unit solids, for the shift rounded to FP32, as the FP32 entry
    points receive it) and rounded once to FP32, the input is the FP32 normalised solid the GPU
    receives, and the products and sums are formed one by one in FP32 (each rounded, no
    fused multiply-add), starting from the FP32 initial output for an accumulating call.

    A plain dot product has no preferred summation order, and where a degree's coefficients
    cancel the error of one order is a draw from a wide distribution: on one octree M2L at
    P = 16 (shift (1, 2, 2)) eight orders gave 1.5e-6 .. 1.5e-5, and on one L2L at P = 9 with
    |r| = 5.1, 5.5e-7 .. 9.4e-5.  error() is therefore the largest error over ORDERS summation
    orders (the natural one, the reversed one and seeded permutations): the error FP32
    arithmetic can make on that input, not one lucky draw.

    bf16 = 3 or 6 evaluates the BF16 split forms instead: operator and input split into BF16
    pieces (_split_bf16) and the listed piece products (exact in FP32) summed in FP32.

    apply(r_rows, C_rows) -> output rows is the oracle's operation (paper basis)."""

    ORDERS = 8

    def __init__(self, apply, p_in, p_out, in_kind, out_kind, r, C, base=None, bf16=0):
        self.apply, self.p_in, self.p_out = apply, p_in, p_out
        self.in_kind, self.out_kind = in_kind, out_kind
        self.r = np.asarray(r, np.float32).astype(np.float64).reshape(-1, 3)
        self.C = np.asarray(C, np.float64).reshape(self.r.shape[0], -1)
        self.base = None if base is None else np.asarray(base, np.float64)
        self.bf16 = bf16
        self._ops = {}

    def operator(self, r):
        """The translation's dense operator in the normalised basis: FP32, or for the BF16
        forms the list of its BF16 pieces."""
        key = tuple(r)
        if key not in self._ops:
            K = self.p_in * (self.p_in + 1)
            T = self.apply(np.repeat(np.reshape(r, (1, 3)), K, axis=0), np.eye(K)).T
            w_in, w_out = weights_flat(self.p_in), weights_flat(self.p_out)
            s_in = w_in if self.in_kind == "M" else 1.0 / w_in
            s_out = w_out if self.out_kind == "M" else 1.0 / w_out
            T = T * s_out[:, None] / s_in[None, :]
            self._ops[key] = _split_bf16(T, 3) if self.bf16 else T.astype(np.float32)
        return self._ops[key]

    def _terms(self, i):
        """Per input k, the FP32 contribution column (outputs x K) of translation i."""
        T = self.operator(self.r[i])
        a = to_basis(self.C[i, : self.p_in * (self.p_in + 1)], self.p_in, self.in_kind, sh.SH_F32)
        if not self.bf16:
            return T * a[None, :]
        ap = _split_bf16(a, 3)
        terms = np.zeros(T[0].shape, np.float32)
        for ti, ai in BF16_PRODUCTS[self.bf16]:
            terms = terms + T[ti] * ap[ai][None, :]  # each product exact, the sum rounded
        return terms

    def results(self, i):
        """The evaluations of translation i in ORDERS summation orders (paper basis)."""
        terms = self._terms(i)
        K = terms.shape[1]
        if self.base is None:
            y0 = np.zeros(terms.shape[0], np.float32)
        else:
            y0 = to_basis(self.base[i], self.p_out, self.out_kind, sh.SH_F32)
        rng = np.random.default_rng(1234 + i)
        orders = [np.arange(K), np.arange(K)[::-1]] + [rng.permutation(K) for _ in range(self.ORDERS - 2)]
        out = []
        for perm in orders:
            y = y0.copy()
            for k in perm:
                y = y + terms[:, k]
            out.append(from_basis(y, self.p_out, self.out_kind, sh.SH_F32))
        return out

    def error(self, i, ref_i):
        """Largest per-degree error of the plain evaluations of translation i against ref_i."""
        return max(max_degree_error(y, ref_i, self.p_out, self.out_kind) for y in self.results(i))


def plain32_for(orc, op, p_in, p_out, r, C, base=None):
    """Plain32 for a batched M2M / M2L / L2L."""
    return Plain32(lambda rr, CC: orc.translate_batch(op, p_in, p_out, rr, CC, nthreads=8), p_in, p_out,
                   IN_KIND[op], OUT_KIND[op], r, C, base)


# FP32 bound per translation: max(tol, PLAIN32_FACTOR x the error of plain FP32 evaluations of
# the same translation, Plain32).  FP32 results of the rotation path, of the FP64-arithmetic
# path at high orders and of the matrix-core forms all round at different places than the plain
# dot products; a factor 2 allows for that and nothing more.
PLAIN32_FACTOR = 2.0


class BoundStats:
    """Per check: how many translations needed more than the flat tolerance, and the worst."""

    def __init__(self):
        self.over = 0
        self.worst_over = 0.0

    def note(self, e, tol):
        if e > tol:
            self.over += 1
            self.worst_over = max(self.worst_over, e)


def check(got, ref, p_out, kind, tol, what, ref_ld=None, plain32=None, factor32=PLAIN32_FACTOR):
    """Per-translation C15 error of got against the oracle.

    FP64 (ref_ld = long-double oracle): error against ref_ld, bound max(tol, COND_FACTOR x the
    FP64 oracle's own error against ref_ld).  FP32 (plain32 = Plain32 of the same inputs): error
    against ref, bound max(tol, factor32 x the plain FP32 evaluation's error), computed only for
    translations above tol.  Otherwise: error against ref, bound tol.  Prints how many
    translations needed more than tol and the worst of them.  Returns the worst error."""
    worst = 0.0
    st = BoundStats()
    for i in range(ref.shape[0]):
        if ref_ld is not None:
            own = max_degree_error(ref[i], ref_ld[i], p_out, kind)
            bound = max(tol, COND_FACTOR * own)
            e = max_degree_error(got[i], ref_ld[i], p_out, kind)
        else:
            e = max_degree_error(got[i], ref[i], p_out, kind)
            bound = tol
            if e > tol and plain32 is not None:
                pe = plain32.error(i, ref[i])
                bound = max(tol, factor32 * pe)
                assert e <= bound, f"{what} translation {i}: {e:.3e} > {bound:.2e} (plain FP32 {pe:.2e})"
        st.note(e, tol)
        worst = max(worst, e)
        assert e <= bound, f"{what} translation {i}: {e:.3e} > {bound:.1e}"
    if st.over:
        print(f"[bound] {what}: {st.over} of {ref.shape[0]} above {tol:.0e}, worst {st.worst_over:.2e}", flush=True)
    return worst


def ld_ref(op, p_in, p_out, r, C):
    return oracle.get("longdouble").translate_batch(op, p_in, p_out, r, C, nthreads=8).astype(np.float64)
