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


class Plain32:
    """A plain FP32 evaluation of the same translations, as the reference for FP32 bounds.

    Each output of a translation is a dot product sum_k T_hat[i, k] a_k of the translation's
    dense operator (normalised basis) with its input.  Here the operator is built exactly
    (the FP64 oracle applied to unit solids, for the shift rounded to FP32, as the FP32 entry
    points receive it) and rounded once to FP32, the input is the FP32 normalised solid the GPU
    receives, and the products and sums are formed one by one in FP32 (each rounded, no
    fused multiply-add), starting from the FP32 initial output for an accumulating call.  Its
    per-degree error against the exact result measures what FP32 arithmetic costs on that
    input: where a degree's coefficients cancel, every FP32 evaluation errs by a few rounding
    units of sum_k |T_hat| |a_k| rather than of the result.

    apply(r_rows, C_rows) -> output rows is the oracle's operation (paper basis)."""

    def __init__(self, apply, p_in, p_out, in_kind, out_kind, r, C, base=None):
        self.apply, self.p_in, self.p_out = apply, p_in, p_out
        self.in_kind, self.out_kind = in_kind, out_kind
        self.r = np.asarray(r, np.float32).astype(np.float64).reshape(-1, 3)
        self.C = np.asarray(C, np.float64).reshape(self.r.shape[0], -1)
        self.base = None if base is None else np.asarray(base, np.float64)
        self._ops = {}

    def operator(self, r):
        key = tuple(r)
        if key not in self._ops:
            K = self.p_in * (self.p_in + 1)
            T = self.apply(np.repeat(np.reshape(r, (1, 3)), K, axis=0), np.eye(K)).T
            w_in, w_out = weights_flat(self.p_in), weights_flat(self.p_out)
            s_in = w_in if self.in_kind == "M" else 1.0 / w_in
            s_out = w_out if self.out_kind == "M" else 1.0 / w_out
            self._ops[key] = (T * s_out[:, None] / s_in[None, :]).astype(np.float32)
        return self._ops[key]

    def result(self, i):
        """The plain FP32 evaluation of translation i (paper basis, FP64 array)."""
        T = self.operator(self.r[i])
        a = to_basis(self.C[i, : self.p_in * (self.p_in + 1)], self.p_in, self.in_kind, sh.SH_F32)
        if self.base is None:
            y = np.zeros(T.shape[0], np.float32)
        else:
            y = to_basis(self.base[i], self.p_out, self.out_kind, sh.SH_F32)
        for k in range(T.shape[1]):
            y = y + T[:, k] * a[k]
        return from_basis(y, self.p_out, self.out_kind, sh.SH_F32)

    def error(self, i, ref_i):
        return max_degree_error(self.result(i), ref_i, self.p_out, self.out_kind)


def plain32_for(orc, op, p_in, p_out, r, C, base=None):
    """Plain32 for a batched M2M / M2L / L2L."""
    return Plain32(lambda rr, CC: orc.translate_batch(op, p_in, p_out, rr, CC, nthreads=8), p_in, p_out,
                   IN_KIND[op], OUT_KIND[op], r, C, base)


# FP32 bound per translation: max(tol, PLAIN32_FACTOR x the error of the plain FP32 evaluation
# of the same translation, Plain32).  FP32 results of the rotation path, of the FP64-arithmetic
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
