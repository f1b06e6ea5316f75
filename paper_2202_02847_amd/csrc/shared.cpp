// Shared-shift operators: per shift class, the whole translation as one dense real matrix in
// the normalised basis, generated on the device in FP64 and applied on the matrix cores
// (k_shared.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "context.hpp"
#include "kernels.hpp"

using shfmm::DeviceGuard;

struct sh_shared {
    sh_ctx *ctx = nullptr;
    int op = 0, p_in = 0, p_out = 0, nclass = 0, prec = 0;
    int K = 0, Kp = 0, N = 0, NT = 0, KS = 0;
    void *mem = nullptr;
    void *frag = nullptr;  // BF16 pieces (x3, x6) or FP32 values
    unsigned char *live_in = nullptr, *live_out = nullptr;
    int64_t frag_class_stride = 0;
    ~sh_shared()
    {
        if (mem) {
            DeviceGuard g(ctx->device);
            (void)hipFree(mem);
        }
    }
};

namespace {

bool is_im0(int64_t idx)
{
    if (!(idx & 1)) return false;
    int64_t n = (int64_t)std::floor((std::sqrt(4.0 * (double)idx + 1.0) - 1.0) * 0.5);
    while ((n + 1) * (n + 2) <= idx) ++n;
    while (n * (n + 1) > idx) --n;
    return idx == n * (n + 1) + 1;
}

// normalisation factors of a solid of order P: w (multipole kind) or 1/w (local kind)
std::vector<double> basis_scale(int P, bool local)
{
    std::vector<double> s((size_t)P * (P + 1));
    for (int n = 0; n < P; ++n)
        for (int m = 0; m <= n; ++m) {
            const long double w = shfmm::norm_weight(n, m);
            const double v = (double)(local ? 1.0L / w : w);
            s[(size_t)n * (n + 1) + 2 * m] = v;
            s[(size_t)n * (n + 1) + 2 * m + 1] = v;
        }
    return s;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    hipError_t alloc(size_t b) { return hipMalloc(&p, b ? b : 1); }
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

sh_status build(sh_shared *o, const double *shifts)
{
    const int K = o->K, N = o->N;
    const int np = o->prec == 6 ? 3 : o->prec == 3 ? 2 : 1;
    hipError_t e;
    // unit input solids (the K x K identity; the Im C_n^0 columns are ignored by the kernels)
    std::vector<double> eye((size_t)K * K, 0.0);
    for (int j = 0; j < K; ++j) eye[(size_t)j * K + j] = 1.0;
    const bool in_local = o->op == SH_L2L, out_local = o->op != SH_M2M;
    const std::vector<double> s_in = basis_scale(o->p_in, in_local), s_out = basis_scale(o->p_out, out_local);
    // classes per pass, so that the FP64 images stay below 256 MB
    const int64_t per_class = (int64_t)K * N * 8;
    const int cc = (int)std::max<int64_t>(1, std::min<int64_t>(o->nclass, ((int64_t)256 << 20) / per_class));
    DevBuf d_eye, d_sin, d_sout, d_r, d_src, d_dst, d_raw;
    if ((e = d_eye.alloc(eye.size() * 8)) != hipSuccess || (e = d_sin.alloc(s_in.size() * 8)) != hipSuccess ||
        (e = d_sout.alloc(s_out.size() * 8)) != hipSuccess || (e = d_r.alloc((size_t)cc * K * 24)) != hipSuccess ||
        (e = d_src.alloc((size_t)cc * K * 8)) != hipSuccess || (e = d_dst.alloc((size_t)cc * K * 8)) != hipSuccess ||
        (e = d_raw.alloc((size_t)cc * per_class)) != hipSuccess)
        return e == hipErrorOutOfMemory ? SH_ENOMEM : SH_EDEVICE;
    if (hipMemcpy(d_eye.p, eye.data(), eye.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_sin.p, s_in.data(), s_in.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_sout.p, s_out.data(), s_out.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return SH_EDEVICE;
    std::vector<double> r((size_t)cc * K * 3);
    std::vector<int64_t> src((size_t)cc * K), dst_rows((size_t)cc * K);
    for (size_t i = 0; i < dst_rows.size(); ++i) dst_rows[i] = (int64_t)i;
    if (hipMemcpy(d_dst.p, dst_rows.data(), dst_rows.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return SH_EDEVICE;
    for (int c0 = 0; c0 < o->nclass; c0 += cc) {
        const int nc = std::min(cc, o->nclass - c0);
        for (int c = 0; c < nc; ++c)
            for (int j = 0; j < K; ++j) {
                const size_t i = (size_t)c * K + j;
                for (int d = 0; d < 3; ++d) r[3 * i + d] = shifts[3 * (c0 + c) + d];
                src[i] = j;
            }
        if (hipMemcpy(d_r.p, r.data(), (size_t)nc * K * 24, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_src.p, src.data(), (size_t)nc * K * 8, hipMemcpyHostToDevice) != hipSuccess)
            return SH_EDEVICE;
        // images of the unit solids: row (c, j) = T_c e_j (paper basis, FP64); the gather
        // reads unit solid j, the scatter writes row c K + j
        sh_status st = shfmm::translate_device(o->ctx, o->op, SH_F64, o->p_in, o->p_out, (int64_t)nc * K, d_r.p,
                                               d_src.as<int64_t>(), d_eye.p, K, d_dst.as<int64_t>(), d_raw.p, N, 0,
                                               nullptr);
        if (st != SH_OK) return st;
        hipError_t pe;
        if (o->prec == SH_SHARED_FP32) {
            float *dst = static_cast<float *>(o->frag) + (int64_t)c0 * o->frag_class_stride;
            pe = shfmm::launch_shared_prep_f32(d_raw.as<double>(), nc, K, N, o->KS, o->NT, d_sin.as<double>(),
                                               d_sout.as<double>(), dst, nullptr);
        } else {
            unsigned short *dst = static_cast<unsigned short *>(o->frag) + (int64_t)c0 * np * o->frag_class_stride;
            pe = shfmm::launch_shared_prep(d_raw.as<double>(), nc, K, N, o->KS, o->NT, np, d_sin.as<double>(),
                                           d_sout.as<double>(), dst, nullptr);
        }
        if (pe != hipSuccess || hipDeviceSynchronize() != hipSuccess) return SH_EDEVICE;
    }
    return SH_OK;
}

}  // namespace

extern "C" {

sh_status sh_shared_create(sh_ctx *ctx, int op, int p_in, int p_out, int nclass, const double *shifts, int precision,
                           sh_shared **out)
{
    if (!out) return SH_EINVAL;
    *out = nullptr;
    if (!ctx || !shifts || (op != SH_M2M && op != SH_M2L && op != SH_L2L) ||
        (precision != SH_SHARED_BF16X3 && precision != SH_SHARED_BF16X6 && precision != SH_SHARED_FP32) ||
        nclass < 1 ||
        nclass > shfmm::shared_max_classes())
        return SH_EINVAL;
    if (p_in < 1 || p_out < 1 || p_in > ctx->max_order || p_out > ctx->max_order) return SH_EORDER;
    for (int c = 0; c < nclass; ++c) {
        const double *s = shifts + 3 * c;
        if (!std::isfinite(s[0]) || !std::isfinite(s[1]) || !std::isfinite(s[2])) return SH_ESHIFT;
        if (op == SH_M2L && s[0] == 0 && s[1] == 0 && s[2] == 0) return SH_ESHIFT;
    }
    try {
        DeviceGuard g(ctx->device);
        if (!g.ok) return SH_EDEVICE;
        sh_shared *o = new sh_shared;
        o->ctx = ctx;
        o->op = op;
        o->p_in = p_in;
        o->p_out = p_out;
        o->nclass = nclass;
        o->prec = precision;
        o->K = p_in * (p_in + 1);
        o->Kp = (o->K + 31) / 32 * 32;
        o->N = p_out * (p_out + 1);
        o->NT = (o->N + 15) / 16;
        o->KS = o->Kp / 32;
        o->frag_class_stride = (int64_t)o->NT * o->KS * 512;
        // BF16 pieces (2 bytes, 3 or 2 per entry) or one FP32 value
        const size_t fb = precision == SH_SHARED_FP32 ? (size_t)nclass * o->frag_class_stride * 4
                                                      : (size_t)nclass * (precision == SH_SHARED_BF16X6 ? 3 : 2) *
                                                            o->frag_class_stride * 2;
        const size_t fa = (fb + 255) & ~size_t(255);
        if (hipMalloc(&o->mem, fa + (size_t)o->Kp + (size_t)o->N) != hipSuccess) {
            o->mem = nullptr;
            delete o;
            return SH_ENOMEM;
        }
        o->frag = o->mem;
        o->live_in = reinterpret_cast<unsigned char *>(o->mem) + fa;
        o->live_out = o->live_in + o->Kp;
        std::vector<unsigned char> li((size_t)o->Kp), lo((size_t)o->N);
        for (int k = 0; k < o->Kp; ++k) li[k] = (k < o->K && !is_im0(k)) ? 1 : 0;
        for (int n = 0; n < o->N; ++n) lo[n] = is_im0(n) ? 0 : 1;
        sh_status st = SH_OK;
        if (hipMemcpy(o->live_in, li.data(), li.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(o->live_out, lo.data(), lo.size(), hipMemcpyHostToDevice) != hipSuccess)
            st = SH_EDEVICE;
        if (st == SH_OK) st = build(o, shifts);
        if (st != SH_OK) {
            delete o;
            return st;
        }
        *out = o;
        return SH_OK;
    } catch (const std::bad_alloc &) {
        return SH_ENOMEM;
    } catch (...) {
        return SH_EDEVICE;
    }
}

sh_status sh_shared_execute(const sh_shared *o, int64_t count, const int64_t *class_start, const float *in,
                            int64_t ld_in, float *out, int64_t ld_out, unsigned flags, void *hip_stream)
{
    if (!o || count < 0 || (flags & ~SH_ACCUMULATE)) return SH_EINVAL;
    if (count == 0) return SH_OK;
    if (!class_start || !in || !out || ld_in < o->K || ld_out < o->N || (ld_in & 1) ||
        (reinterpret_cast<uintptr_t>(in) & 7))
        return SH_EINVAL;
    try {
        DeviceGuard g(o->ctx->device);
        if (!g.ok) return SH_EDEVICE;
        shfmm::SharedArgs a{};
        a.count = count;
        a.nclass = o->nclass;
        a.K = o->K;
        a.Kp = o->Kp;
        a.N = o->N;
        a.NT = o->NT;
        a.KS = o->KS;
        a.class_start = class_start;
        a.in = in;
        a.ld_in = ld_in;
        a.out = out;
        a.ld_out = ld_out;
        a.frag = o->frag;
        a.frag_class_stride = o->frag_class_stride;
        a.live_in = o->live_in;
        a.live_out = o->live_out;
        a.flags = flags;
        return shfmm::launch_shared_gemm(a, o->prec, reinterpret_cast<hipStream_t>(hip_stream)) == hipSuccess
                   ? SH_OK
                   : SH_EDEVICE;
    } catch (...) {
        return SH_EDEVICE;
    }
}

int64_t sh_shared_bytes(const sh_shared *o)
{
    if (!o) return -1;
    if (o->prec == SH_SHARED_FP32) return (int64_t)o->nclass * o->frag_class_stride * 4;
    const int np = o->prec == SH_SHARED_BF16X6 ? 3 : 2;
    return (int64_t)o->nclass * np * o->frag_class_stride * 2;
}

void sh_shared_destroy(sh_shared *o)
{
    try {
        delete o;
    } catch (...) {
    }
}

}  // extern "C"
