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


def check(got, ref, p_out, kind, tol, what, ref_ld=None, ref_in32=None):
    """ref_ld: long-double reference (FP64 path).  ref_in32: the FP64 oracle applied to the
    input rounded through the FP32 normalised basis -- its distance from ref is the error
    any FP32-input computation inherits; the FP32 bound is max(tol, COND_FACTOR x that)."""
    worst = 0.0
    for i in range(ref.shape[0]):
        if ref_in32 is not None:
            floor = max_degree_error(ref_in32[i], ref[i], p_out, kind)
            bound = max(tol, COND_FACTOR * floor)
            e = max_degree_error(got[i], ref[i], p_out, kind)
        elif ref_ld is not None:
            own = max_degree_error(ref[i], ref_ld[i], p_out, kind)
            bound = max(tol, COND_FACTOR * own)
            e = max_degree_error(got[i], ref_ld[i], p_out, kind)
        else:
            bound = tol
            e = max_degree_error(got[i], ref[i], p_out, kind)
        worst = max(worst, e)
        assert e <= bound, f"{what} translation {i}: {e:.3e} > {bound:.1e}"
    return worst


def in32_ref(orc, op, p_in, p_out, r, C):
    C32 = from_basis(to_basis(C, p_in, IN_KIND[op], sh.SH_F32), p_in, IN_KIND[op], sh.SH_F32)
    r32 = np.asarray(r, np.float32).astype(np.float64)
    return orc.translate_batch(op, p_in, p_out, r32, C32)


def ld_ref(op, p_in, p_out, r, C):
    return oracle.get("longdouble").translate_batch(op, p_in, p_out, r, C, nthreads=8).astype(np.float64)
