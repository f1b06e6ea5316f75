// Uniform-octree FMM driver: the translation path used as the paper intends it, inside a
// fast multipole method (Sections 1 and 2): P2M at the leaves, upward M2M, M2L over the
// interaction lists, downward L2L, L2P at the leaves and the direct near field P2P.
//
// The tree is a full octree of `levels` levels below a root cube [origin, origin + width)^3.
// Level l has n = 2^l boxes per side, box (ix, iy, iz) at index (ix n + iy) n + iz, centre
// origin + (i + 1/2) width / n.  Every leaf holds the same number of particles, stored leaf
// by leaf.  All index and shift arrays are built once on the host at creation and kept on the
// device; an evaluation only launches kernels.
//
// Launch grouping (each translation call needs distinct output solids when it accumulates):
//   * M2M, level l -> l-1: one call per child octant (each parent has one child per octant);
//     the first overwrites the parents, the other seven accumulate.
//   * M2L at level l >= 2, target-major: the pairs (source b + d -> target b), d in
//     [-3, 3]^3 \ [-1, 1]^3 with the parents of b and b + d neighbours (or equal), are listed
//     target by target, so each target's pairs are contiguous.  One indexed launch per chunk
//     of targets writes every translation to its own scratch solid, and a segmented sum adds
//     each target's run into its local expansion: a few large launches per level instead of
//     one small launch per offset (whose targets overlap across offsets).
//   * L2L, level l -> l+1: one call per child octant, accumulating into the children.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/shfmm.h"
#include "context.hpp"
#include "kernels.hpp"
#include "near_field.hpp"

namespace {

struct FmmCall {
    int op;
    int level_in, level_out;
    int64_t count;
    int64_t off;  // first pair in the shared src / dst / r arrays
};

// M2L of the targets [tb, te) of one level: pairs [off, off + count) of the shared arrays.
struct M2lChunk {
    int level;
    int64_t off, count;
    int64_t tb, te;
};

constexpr int64_t kScratchBytes = (int64_t)1 << 30;  // M2L scratch solids per chunk

}  // namespace

struct sh_fmm {
    sh_ctx *ctx = nullptr;
    int P = 0, levels = 0;          // P: order of the leaves
    std::vector<int> Pl;            // order of level l (levels 2..L)
    std::vector<int64_t> roff;      // level l's solids start at roff[l] reals in the M / L pools
    int64_t npts = 0;
    double origin[3] = {0, 0, 0};
    double width = 1;
    std::vector<FmmCall> up, down;
    std::vector<M2lChunk> m2l;
    std::vector<int64_t> seg_off;  // level l's target offsets start at seg + seg_off[l]
    int64_t chunk_cap = 0;         // iota entries: pairs of the largest chunk
    int64_t scratch_reals = 0;
    // device memory: one allocation
    void *mem = nullptr;
    double *M = nullptr, *L = nullptr;  // pools: boxes of levels 2..L, P_l(P_l+1) reals each
    double *scratch = nullptr;          // scratch_reals: one M2L result per solid
    int64_t *iota = nullptr;            // 0 .. chunk_cap - 1 (scratch slots)
    int64_t *seg = nullptr;             // per level: first pair of every target, and the end
    int64_t *src = nullptr, *dst = nullptr;
    double *r = nullptr;
    double *leaf_centres = nullptr;
    int32_t *nbr = nullptr;  // leaves x 27
    int64_t npairs = 0;
    // graph replay: captured on `cap` with branches on `side`, for one (pts, q, out)
    std::mutex mu;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;
    hipGraphExec_t exec = nullptr;
    const double *g_pts = nullptr, *g_q = nullptr;
    double *g_out = nullptr;
};

namespace {

using shfmm::DeviceGuard;

inline int64_t boxes_at(int l) { return (int64_t)1 << (3 * l); }
inline int64_t box_index(int64_t n, int64_t ix, int64_t iy, int64_t iz) { return (ix * n + iy) * n + iz; }

struct HostPlan {
    std::vector<int64_t> src, dst;
    std::vector<double> r;
    void add(int64_t s, int64_t d, double rx, double ry, double rz)
    {
        src.push_back(s);
        dst.push_back(d);
        r.push_back(rx);
        r.push_back(ry);
        r.push_back(rz);
    }
};

inline int64_t fdiv2(int64_t a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

void build(sh_fmm *f, HostPlan &hp, std::vector<int64_t> &seg, std::vector<double> &centres,
           std::vector<int32_t> &nbr)
{
    const int Lv = f->levels;
    // upward: children at level l (octant o) -> parents at level l - 1 >= 2 (the multipoles
    // of levels 0 and 1 have no interaction list to feed)
    for (int l = Lv; l >= 3; --l) {
        const int64_t n = (int64_t)1 << l, np = n / 2;
        const double w = f->width / (double)n;
        for (int o = 0; o < 8; ++o) {
            const int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
            FmmCall c{SH_M2M, l, l - 1, 0, (int64_t)hp.src.size()};
            for (int64_t px = 0; px < np; ++px)
                for (int64_t py = 0; py < np; ++py)
                    for (int64_t pz = 0; pz < np; ++pz)
                        hp.add(box_index(n, 2 * px + ox, 2 * py + oy, 2 * pz + oz), box_index(np, px, py, pz),
                               (0.5 - ox) * w, (0.5 - oy) * w, (0.5 - oz) * w);
            c.count = (int64_t)hp.src.size() - c.off;
            f->up.push_back(c);
        }
    }
    // M2L at levels 2..L, target by target: offsets d with max |d_i| >= 2, parents neighbours
    f->seg_off.assign(Lv + 1, 0);
    for (int l = 2; l <= Lv; ++l) {
        const int64_t S = (int64_t)f->Pl[l] * (f->Pl[l] + 1);
        const int64_t cap = std::max<int64_t>(189, kScratchBytes / (S * (int64_t)sizeof(double)));
        const int64_t n = (int64_t)1 << l;
        const double w = f->width / (double)n;
        f->seg_off[l] = (int64_t)seg.size();
        M2lChunk ck{l, (int64_t)hp.src.size(), 0, 0, 0};
        for (int64_t ix = 0; ix < n; ++ix)
            for (int64_t iy = 0; iy < n; ++iy)
                for (int64_t iz = 0; iz < n; ++iz) {
                    const int64_t b = box_index(n, ix, iy, iz);
                    const int64_t first = (int64_t)hp.src.size();
                    seg.push_back(first);
                    for (int dx = -3; dx <= 3; ++dx)
                        for (int dy = -3; dy <= 3; ++dy)
                            for (int dz = -3; dz <= 3; ++dz) {
                                if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) continue;
                                const int64_t sx = ix + dx, sy = iy + dy, sz = iz + dz;
                                if (sx < 0 || sy < 0 || sz < 0 || sx >= n || sy >= n || sz >= n) continue;
                                if (std::abs(fdiv2(sx) - fdiv2(ix)) > 1 || std::abs(fdiv2(sy) - fdiv2(iy)) > 1 ||
                                    std::abs(fdiv2(sz) - fdiv2(iz)) > 1)
                                    continue;
                                // r = x_B - x_A = centre(target) - centre(source) = -d w
                                hp.add(box_index(n, sx, sy, sz), b, -dx * w, -dy * w, -dz * w);
                            }
                    // close the chunk before this target if its pairs would not fit
                    if ((int64_t)hp.src.size() - ck.off > cap) {
                        ck.count = first - ck.off;
                        ck.te = b;
                        f->m2l.push_back(ck);
                        ck = M2lChunk{l, first, 0, b, 0};
                    }
                }
        seg.push_back((int64_t)hp.src.size());
        ck.count = (int64_t)hp.src.size() - ck.off;
        ck.te = boxes_at(l);
        f->m2l.push_back(ck);
    }
    // downward: parents at level l -> children at level l + 1 (octant o), from level 2
    for (int l = 2; l < Lv; ++l) {
        const int64_t np = (int64_t)1 << l, n = 2 * np;
        const double w = f->width / (double)n;
        for (int o = 0; o < 8; ++o) {
            const int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
            FmmCall c{SH_L2L, l, l + 1, 0, (int64_t)hp.src.size()};
            for (int64_t px = 0; px < np; ++px)
                for (int64_t py = 0; py < np; ++py)
                    for (int64_t pz = 0; pz < np; ++pz)
                        hp.add(box_index(np, px, py, pz), box_index(n, 2 * px + ox, 2 * py + oy, 2 * pz + oz),
                               (ox - 0.5) * w, (oy - 0.5) * w, (oz - 0.5) * w);
            c.count = (int64_t)hp.src.size() - c.off;
            f->down.push_back(c);
        }
    }
    // leaves: centres and the 27 neighbours (itself included), -1 outside the cube
    const int64_t n = (int64_t)1 << Lv;
    const double w = f->width / (double)n;
    centres.resize((size_t)(3 * boxes_at(Lv)));
    nbr.assign((size_t)(27 * boxes_at(Lv)), -1);
    for (int64_t ix = 0; ix < n; ++ix)
        for (int64_t iy = 0; iy < n; ++iy)
            for (int64_t iz = 0; iz < n; ++iz) {
                const int64_t b = box_index(n, ix, iy, iz);
                centres[3 * b] = f->origin[0] + (ix + 0.5) * w;
                centres[3 * b + 1] = f->origin[1] + (iy + 0.5) * w;
                centres[3 * b + 2] = f->origin[2] + (iz + 0.5) * w;
                int k = 0;
                for (int dx = -1; dx <= 1; ++dx)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dz = -1; dz <= 1; ++dz, ++k) {
                            const int64_t sx = ix + dx, sy = iy + dy, sz = iz + dz;
                            if (sx < 0 || sy < 0 || sz < 0 || sx >= n || sy >= n || sz >= n) continue;
                            nbr[27 * b + k] = (int32_t)box_index(n, sx, sy, sz);
                        }
            }
}

}  // namespace

extern "C" {

sh_status sh_fmm_create_orders(sh_ctx *ctx, int levels, const int *orders, const double origin[3], double width,
                               int64_t npts, sh_fmm **out)
{
    if (!out) return SH_EINVAL;
    *out = nullptr;
    if (!ctx || !orders || !origin || !(width > 0.0) || npts < 1 || levels < 2 || levels > SH_FMM_MAX_LEVELS)
        return SH_EINVAL;
    for (int l = 2; l <= levels; ++l)
        if (orders[l - 2] < 1 || orders[l - 2] > ctx->max_order) return SH_EORDER;
    if (boxes_at(levels) * npts > ((int64_t)1 << 31)) return SH_EINVAL;
    sh_fmm *f = new (std::nothrow) sh_fmm;
    if (!f) return SH_ENOMEM;
    f->ctx = ctx;
    f->levels = levels;
    f->Pl.assign(levels + 1, 0);
    for (int l = 2; l <= levels; ++l) f->Pl[l] = orders[l - 2];
    f->P = f->Pl[levels];
    f->npts = npts;
    std::memcpy(f->origin, origin, sizeof f->origin);
    f->width = width;
    f->roff.assign(levels + 2, 0);
    for (int l = 2; l <= levels; ++l) f->roff[l + 1] = f->roff[l] + boxes_at(l) * f->Pl[l] * (f->Pl[l] + 1);
    HostPlan hp;
    std::vector<int64_t> seg;
    std::vector<double> centres;
    std::vector<int32_t> nbr;
    try {
        build(f, hp, seg, centres, nbr);
    } catch (...) {
        delete f;
        return SH_ENOMEM;
    }
    f->npairs = (int64_t)hp.src.size();
    // scratch for the largest chunk built (chunks were cut at kScratchBytes)
    f->chunk_cap = 1;
    f->scratch_reals = 1;
    for (const M2lChunk &c : f->m2l) {
        f->chunk_cap = std::max(f->chunk_cap, c.count);
        f->scratch_reals = std::max(f->scratch_reals, c.count * f->Pl[c.level] * (f->Pl[c.level] + 1));
    }
    auto up256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bM = up256(sizeof(double) * (size_t)f->roff[levels + 1]);
    const size_t bI = up256(sizeof(int64_t) * (size_t)f->npairs);
    const size_t bR = up256(sizeof(double) * (size_t)(3 * f->npairs));
    const size_t bC = up256(sizeof(double) * centres.size());
    const size_t bN = up256(sizeof(int32_t) * nbr.size());
    DeviceGuard g(ctx->device);
    if (!g.ok) {
        delete f;
        return SH_EDEVICE;
    }
    const size_t bX = up256(sizeof(double) * (size_t)f->scratch_reals);
    const size_t bT = up256(sizeof(int64_t) * (size_t)f->chunk_cap);
    const size_t bG = up256(sizeof(int64_t) * seg.size());
    if (hipMalloc(&f->mem, 2 * bM + 2 * bI + bR + bC + bN + bX + bT + bG) != hipSuccess) {
        (void)hipGetLastError();
        delete f;
        return SH_ENOMEM;
    }
    char *p = static_cast<char *>(f->mem);
    f->M = reinterpret_cast<double *>(p);
    f->L = reinterpret_cast<double *>(p + bM);
    f->src = reinterpret_cast<int64_t *>(p + 2 * bM);
    f->dst = reinterpret_cast<int64_t *>(p + 2 * bM + bI);
    f->r = reinterpret_cast<double *>(p + 2 * bM + 2 * bI);
    f->leaf_centres = reinterpret_cast<double *>(p + 2 * bM + 2 * bI + bR);
    f->nbr = reinterpret_cast<int32_t *>(p + 2 * bM + 2 * bI + bR + bC);
    f->scratch = reinterpret_cast<double *>(p + 2 * bM + 2 * bI + bR + bC + bN);
    f->iota = reinterpret_cast<int64_t *>(p + 2 * bM + 2 * bI + bR + bC + bN + bX);
    f->seg = reinterpret_cast<int64_t *>(p + 2 * bM + 2 * bI + bR + bC + bN + bX + bT);
    std::vector<int64_t> iota((size_t)f->chunk_cap);
    for (int64_t i = 0; i < f->chunk_cap; ++i) iota[(size_t)i] = i;
    bool ok = hipMemcpy(f->src, hp.src.data(), sizeof(int64_t) * hp.src.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(f->dst, hp.dst.data(), sizeof(int64_t) * hp.dst.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(f->r, hp.r.data(), sizeof(double) * hp.r.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(f->leaf_centres, centres.data(), sizeof(double) * centres.size(), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(f->nbr, nbr.data(), sizeof(int32_t) * nbr.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(f->iota, iota.data(), sizeof(int64_t) * iota.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(f->seg, seg.data(), sizeof(int64_t) * seg.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        (void)hipFree(f->mem);
        delete f;
        return SH_EDEVICE;
    }
    *out = f;
    return SH_OK;
}

sh_status sh_fmm_create(sh_ctx *ctx, int P, int levels, const double origin[3], double width, int64_t npts,
                        sh_fmm **out)
{
    if (levels < 2 || levels > SH_FMM_MAX_LEVELS) {
        if (out) *out = nullptr;
        return SH_EINVAL;
    }
    int orders[SH_FMM_MAX_LEVELS];
    for (int l = 2; l <= levels; ++l) orders[l - 2] = P;
    return sh_fmm_create_orders(ctx, levels, orders, origin, width, npts, out);
}

void sh_fmm_destroy(sh_fmm *f)
{
    if (!f) return;
    {
        DeviceGuard g(f->ctx->device);
        if (f->exec) (void)hipGraphExecDestroy(f->exec);
        for (hipEvent_t e : f->ev) (void)hipEventDestroy(e);
        for (hipStream_t st : f->side) (void)hipStreamDestroy(st);
        if (f->cap) (void)hipStreamDestroy(f->cap);
        if (f->mem) (void)hipFree(f->mem);
    }
    delete f;
}

}  // extern "C"

namespace {

hipError_t status_to_hip(sh_status st) { return st == SH_OK ? hipSuccess : hipErrorUnknown; }

// Enqueues one evaluation on stream s.  With fork (graph capture), the near field runs on
// side[0] from the start: it writes the output first (overwrite) while the far field is
// computed, and L2P adds the far field last.
hipError_t enqueue(sh_fmm *f, const double *pts, const double *q, double *out, hipStream_t s, bool fork)
{
    const int Lv = f->levels, P = f->Pl[Lv];
    const int64_t S = (int64_t)P * (P + 1);  // leaves
    const int64_t nleaf = boxes_at(Lv);
    double *Mleaf = f->M + f->roff[Lv];
    double *Lleaf = f->L + f->roff[Lv];
    auto sz = [&](int l) { return (int64_t)f->Pl[l] * (f->Pl[l] + 1); };
    hipError_t e;
    hipStream_t near = s;
    if (fork) {
        if ((e = hipEventRecord(f->ev[0], s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(f->side[0], f->ev[0], 0)) != hipSuccess) return e;
        near = f->side[0];
    }
    if ((e = shfmm::launch_p2p(nleaf, f->npts, pts, q, f->nbr, out, 0u, near)) != hipSuccess) return e;
    if ((e = shfmm::launch_p2m(P, nleaf, f->leaf_centres, f->npts, pts, q, Mleaf, S, s)) != hipSuccess) return e;
    auto run = [&](const FmmCall &c, unsigned flags, double *pool) {
        const int li = c.level_in, lo = c.level_out;
        return status_to_hip(shfmm::translate_device(f->ctx, c.op, SH_F64, f->Pl[li], f->Pl[lo], c.count,
                                                     f->r + 3 * c.off, f->src + c.off, pool + f->roff[li], sz(li),
                                                     f->dst + c.off, pool + f->roff[lo], sz(lo), flags, s));
    };
    // upward pass: the first octant of a level overwrites its parents
    for (size_t i = 0; i < f->up.size(); ++i)
        if ((e = run(f->up[i], (i % 8 == 0) ? 0u : SH_ACCUMULATE, f->M)) != hipSuccess) return e;
    // M2L: every translation of a chunk into its scratch solid, then each target's run summed
    // into its local expansion (overwriting: every target of levels 2..L is in one chunk)
    for (const M2lChunk &c : f->m2l) {
        const int l = c.level;
        if ((e = status_to_hip(shfmm::translate_device(f->ctx, SH_M2L, SH_F64, f->Pl[l], f->Pl[l], c.count,
                                                       f->r + 3 * c.off, f->src + c.off, f->M + f->roff[l], sz(l),
                                                       f->iota, f->scratch, sz(l), 0u, s))) != hipSuccess)
            return e;
        if ((e = shfmm::launch_seg_sum(f->L + f->roff[l], sz(l), f->seg + f->seg_off[l], c.tb, c.te, c.off,
                                       f->scratch, s)) != hipSuccess)
            return e;
    }
    for (const FmmCall &c : f->down)
        if ((e = run(c, SH_ACCUMULATE, f->L)) != hipSuccess) return e;
    if (fork) {
        if ((e = hipEventRecord(f->ev[1], f->side[0])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, f->ev[1], 0)) != hipSuccess) return e;
    }
    return shfmm::launch_l2p(P, nleaf, f->leaf_centres, f->npts, pts, Lleaf, S, out, 1u, s);
}

hipError_t capture(sh_fmm *f, const double *pts, const double *q, double *out)
{
    hipError_t e;
    if (f->exec) {
        (void)hipGraphExecDestroy(f->exec);
        f->exec = nullptr;
    }
    if (!f->cap) {
        if ((e = hipStreamCreateWithFlags(&f->cap, hipStreamNonBlocking)) != hipSuccess) return e;
        {
            hipStream_t st;
            if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return e;
            f->side.push_back(st);
        }
        for (int i = 0; i < 2; ++i) {
            hipEvent_t ev;
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
            f->ev.push_back(ev);
        }
    }
    if ((e = hipStreamBeginCapture(f->cap, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
    const hipError_t le = enqueue(f, pts, q, out, f->cap, true);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(f->cap, &graph);
    if (le == hipSuccess && e == hipSuccess) e = hipGraphInstantiate(&f->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    f->g_pts = pts;
    f->g_q = q;
    f->g_out = out;
    return hipSuccess;
}

}  // namespace

extern "C" {

sh_status sh_fmm_evaluate(sh_fmm *f, const double *pts, const double *q, double *out, unsigned flags,
                          void *hip_stream)
{
    if (!f || !pts || !q || !out || (flags & ~SH_FMM_NO_GRAPH)) return SH_EINVAL;
    std::lock_guard<std::mutex> lk(f->mu);
    DeviceGuard g(f->ctx->device);
    if (!g.ok) return SH_EDEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    if (flags & SH_FMM_NO_GRAPH) return enqueue(f, pts, q, out, s, false) == hipSuccess ? SH_OK : SH_EDEVICE;
    if (!f->exec || f->g_pts != pts || f->g_q != q || f->g_out != out) {
        if (capture(f, pts, q, out) != hipSuccess) {
            (void)hipGetLastError();
            return SH_EDEVICE;
        }
    }
    return hipGraphLaunch(f->exec, s) == hipSuccess ? SH_OK : SH_EDEVICE;
}

sh_status sh_fmm_describe(const sh_fmm *f, int64_t *counts)
{
    if (!f || !counts) return SH_EINVAL;
    int64_t t[3] = {0, 0, 0};
    for (const FmmCall &c : f->up) t[0] += c.count;
    for (const M2lChunk &c : f->m2l) t[1] += c.count;
    for (const FmmCall &c : f->down) t[2] += c.count;
    counts[0] = t[0];
    counts[1] = t[1];
    counts[2] = t[2];
    counts[3] = (int64_t)(f->up.size() + f->m2l.size() + f->down.size());
    counts[4] = boxes_at(f->levels);
    return SH_OK;
}

}  // extern "C"
