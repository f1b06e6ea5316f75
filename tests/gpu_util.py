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


def degree_kappa(orc, op, p_in, p_out, r, C):
    """Cancellation factor per output degree n of one translation: max_m sum_k |T_hat||a_hat| over
    max_m |L_hat_ref| in the normalised basis.  An FP32 evaluation errs by a few rounding units
    of the terms it sums, so its relative error in a degree grows by this factor."""
    T = dense_operator(orc, op, p_in, p_out, r)
    w_in, w_out = weights_flat(p_in), weights_flat(p_out)
    a = np.abs(C * (w_in if IN_KIND[op] == "M" else 1.0 / w_in))
    for nn in range(p_in):
        a[nn * (nn + 1) + 1] = 0.0
    s_out = w_out if OUT_KIND[op] == "M" else 1.0 / w_out
    ref = orc.translate_batch(op, p_in, p_out, np.reshape(r, (1, 3)), C[None, :])[0] * s_out
    mag = np.abs(T) @ a
    kap = np.zeros(p_out)
    for nn in range(p_out):
        sl = slice(nn * (nn + 1), (nn + 1) * (nn + 2))
        kap[nn] = mag[sl].max() / max(np.abs(ref[sl]).max(), 1e-300)
    return kap


def check(got, ref, p_out, kind, tol, what, ref_ld=None, ref_in32=None, cond=None):
    """ref_ld: long-double reference (FP64 path).  ref_in32: the FP64 oracle applied to the
    input rounded through the FP32 normalised basis -- its distance from ref is the error
    any FP32-input computation inherits; the FP32 bound is max(tol, COND_FACTOR x that).
    cond = (orc, op, p_in, r, C): for a translation above that bound, the per-degree FP32
    bound becomes max(bound, 4 u kappa_n) with u = 2^-24 and kappa_n from degree_kappa."""
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
        if e > bound and cond is not None:
            orc, op, p_in, r, C = cond
            kap = degree_kappa(orc, op, p_in, p_out, r[i], C[i])
            base = ref_ld[i] if ref_ld is not None else ref[i]
            for nn in range(p_out):
                sl = slice(nn * (nn + 1), (nn + 1) * (nn + 2))
                w = weights_flat(p_out)[sl]
                s = w if kind == "M" else 1.0 / w
                den = max(np.abs(base[sl] * s).max(), 1e-300)
                en = np.abs((got[i][sl] - base[sl]) * s).max() / den
                bn = max(bound, 4.0 * 2.0 ** -24 * kap[nn])
                assert en <= bn, f"{what} translation {i} degree {nn}: {en:.3e} > {bn:.1e} (kappa {kap[nn]:.1e})"
            worst = max(worst, e)
            continue
        worst = max(worst, e)
        assert e <= bound, f"{what} translation {i}: {e:.3e} > {bound:.1e}"
    return worst


def in32_ref(orc, op, p_in, p_out, r, C):
    C32 = from_basis(to_basis(C, p_in, IN_KIND[op], sh.SH_F32), p_in, IN_KIND[op], sh.SH_F32)
    r32 = np.asarray(r, np.float32).astype(np.float64)
    return orc.translate_batch(op, p_in, p_out, r32, C32)


def ld_ref(op, p_in, p_out, r, C):
    return oracle.get("longdouble").translate_batch(op, p_in, p_out, r, C, nthreads=8).astype(np.float64)
