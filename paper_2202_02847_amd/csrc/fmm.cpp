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
// Launch grouping (a translation call that accumulates needs distinct output solids):
//   * M2M (level l -> l-1) and M2L (within level l >= 2) are target-major: the pairs of each
//     target (its 8 children; its interaction list, the boxes b + d with d in
//     [-3, 3]^3 \ [-1, 1]^3 whose parents neighbour b's parent) are listed target by target, so
//     each target's pairs are contiguous.  One indexed launch per chunk of targets writes every
//     translation to its own scratch solid, and a segmented sum adds each target's run into its
//     expansion: a few large launches per level, not one small launch per offset or octant.
//   * L2L (level l -> l+1): one call per level; every child is the target of exactly one L2L,
//     which accumulates into the child's M2L result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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

// Target-major translations (M2M into parents, M2L within a level) for the targets
// [tb, te) of level level_out: pairs [off, off + count) of the shared arrays; the targets'
// pair offsets are seg[seg_base + t].
struct Chunk {
    int op;
    int level_in, level_out;
    int64_t off, count;
    int64_t tb, te;
    int64_t seg_base;
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
    std::vector<FmmCall> down;
    std::vector<Chunk> up, m2l;
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
    // Appends the pairs of every target of level lo (add_pairs(t) lists target t's sources)
    // and cuts them into chunks whose scratch solids fit in kScratchBytes.
    auto chunks = [&](int op, int li, int lo, std::vector<Chunk> &outv, auto add_pairs) {
        const int64_t S = (int64_t)f->Pl[lo] * (f->Pl[lo] + 1);
        const int64_t cap = std::max<int64_t>(189, kScratchBytes / (S * (int64_t)sizeof(double)));
        const int64_t base = (int64_t)seg.size();
        Chunk ck{op, li, lo, (int64_t)hp.src.size(), 0, 0, 0, base};
        const int64_t nt = boxes_at(lo);
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t first = (int64_t)hp.src.size();
            seg.push_back(first);
            add_pairs(t);
            if ((int64_t)hp.src.size() - ck.off > cap) {  // close the chunk before target t
                ck.count = first - ck.off;
                ck.te = t;
                outv.push_back(ck);
                ck = Chunk{op, li, lo, first, 0, t, 0, base};
            }
        }
        seg.push_back((int64_t)hp.src.size());
        ck.count = (int64_t)hp.src.size() - ck.off;
        ck.te = nt;
        outv.push_back(ck);
    };
    // upward: the 8 children at level l of every parent at level l - 1 >= 2 (the multipoles of
    // levels 0 and 1 have no interaction list to feed)
    for (int l = Lv; l >= 3; --l) {
        const int64_t n = (int64_t)1 << l, np = n / 2;
        const double w = f->width / (double)n;
        chunks(SH_M2M, l, l - 1, f->up, [&](int64_t pb) {
            const int64_t px = pb / (np * np), py = (pb / np) % np, pz = pb % np;
            for (int o = 0; o < 8; ++o) {
                const int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
                hp.add(box_index(n, 2 * px + ox, 2 * py + oy, 2 * pz + oz), pb, (0.5 - ox) * w, (0.5 - oy) * w,
                       (0.5 - oz) * w);
            }
        });
    }
    // M2L at levels 2..L, target by target: offsets d with max |d_i| >= 2, parents neighbours
    for (int l = 2; l <= Lv; ++l) {
        const int64_t n = (int64_t)1 << l;
        const double w = f->width / (double)n;
        chunks(SH_M2L, l, l, f->m2l, [&](int64_t b) {
            const int64_t ix = b / (n * n), iy = (b / n) % n, iz = b % n;
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
        });
    }
    // downward: every child at level l + 1 from its parent at level l >= 2, one call per level
    // (each child is the target of exactly one L2L, so the call accumulates race-free)
    for (int l = 2; l < Lv; ++l) {
        const int64_t np = (int64_t)1 << l, n = 2 * np;
        const double w = f->width / (double)n;
        FmmCall c{SH_L2L, l, l + 1, 0, (int64_t)hp.src.size()};
        for (int64_t cx = 0; cx < n; ++cx)
            for (int64_t cy = 0; cy < n; ++cy)
                for (int64_t cz = 0; cz < n; ++cz)
                    hp.add(box_index(np, cx / 2, cy / 2, cz / 2), box_index(n, cx, cy, cz), ((cx & 1) - 0.5) * w,
                           ((cy & 1) - 0.5) * w, ((cz & 1) - 0.5) * w);
        c.count = (int64_t)hp.src.size() - c.off;
        f->down.push_back(c);
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
    if (npts > ((int64_t)1 << 31) / boxes_at(levels)) return SH_EINVAL;  // at most 2^31 particles
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
    for (const std::vector<Chunk> *v : {&f->up, &f->m2l})
        for (const Chunk &c : *v) {
            f->chunk_cap = std::max(f->chunk_cap, c.count);
            f->scratch_reals = std::max(f->scratch_reals, c.count * f->Pl[c.level_out] * (f->Pl[c.level_out] + 1));
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
    // target-major steps: every translation of a chunk into its scratch solid, then each
    // target's run summed into its expansion (overwriting: every target is in one chunk)
    auto run_chunk = [&](const Chunk &c, const double *pool_in, double *pool_out) {
        const int li = c.level_in, lo = c.level_out;
        hipError_t e2 = status_to_hip(shfmm::translate_device(f->ctx, c.op, SH_F64, f->Pl[li], f->Pl[lo], c.count,
                                                              f->r + 3 * c.off, f->src + c.off, pool_in + f->roff[li],
                                                              sz(li), f->iota, f->scratch, sz(lo), 0u, s));
        if (e2 != hipSuccess) return e2;
        return shfmm::launch_seg_sum(pool_out + f->roff[lo], sz(lo), f->seg + c.seg_base, c.tb, c.te, c.off,
                                     f->scratch, s);
    };
    // upward pass (parents summing their 8 children), then M2L at every level
    for (const Chunk &c : f->up)
        if ((e = run_chunk(c, f->M, f->M)) != hipSuccess) return e;
    for (const Chunk &c : f->m2l)
        if ((e = run_chunk(c, f->M, f->L)) != hipSuccess) return e;
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
        // created into locals and kept only when all of them exist, so a failed creation
        // leaves the handle as it was and the next evaluation tries again
        hipStream_t cap = nullptr, side = nullptr;
        hipEvent_t ev[2] = {nullptr, nullptr};
        e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
        for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
        if (e != hipSuccess) {
            for (hipEvent_t x : ev)
                if (x) (void)hipEventDestroy(x);
            if (side) (void)hipStreamDestroy(side);
            if (cap) (void)hipStreamDestroy(cap);
            return e;
        }
        f->side.assign(1, side);
        f->ev.assign(ev, ev + 2);
        f->cap = cap;
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

// Orders for a relative error target of the potential, max_i |u_i - u_i^direct| divided by
// max_i |u_i^direct|, from the error this driver measured against direct summation (uniform
// trees, 3 levels, 8-24 uniform particles per leaf, charges uniform in [-1, 1], four seeds):
// every measurement lies below kErrC * kErrRho^P (P = 4..14).  Lowering one level's order
// raises the error to that order's level and raising one level alone does not lower it, so
// every level takes the same order.  The rule is used only where it was measured, with a
// margin: orders up to kRuleMaxOrder and trees of 2 to kRuleMaxLevels levels (the tests check
// it on 2-, 3- and 4-level trees); targets below kErrC * kErrRho^kRuleMaxOrder (6.6e-8, far
// above the FP64 rounding of the potential, about 1e-15) are refused.
constexpr double kErrC = 0.15, kErrRho = 0.444;
constexpr int kRuleMaxOrder = 18, kRuleMaxLevels = 4;

sh_status sh_fmm_orders_for_tolerance(double tol, int levels, int *orders)
{
    if (!orders || !(tol > 0.0) || !(tol < 1.0) || levels < 2 || levels > kRuleMaxLevels) return SH_EINVAL;
    const int P = std::max(1, (int)std::ceil(std::log(tol / kErrC) / std::log(kErrRho) - 1e-9));
    if (P > kRuleMaxOrder) return SH_EORDER;
    for (int l = 2; l <= levels; ++l) orders[l - 2] = P;
    return SH_OK;
}

sh_status sh_fmm_describe(const sh_fmm *f, int64_t *counts)
{
    if (!f || !counts) return SH_EINVAL;
    int64_t t[3] = {0, 0, 0};
    for (const Chunk &c : f->up) t[0] += c.count;
    for (const Chunk &c : f->m2l) t[1] += c.count;
    for (const FmmCall &c : f->down) t[2] += c.count;
    counts[0] = t[0];
    counts[1] = t[1];
    counts[2] = t[2];
    counts[3] = (int64_t)(f->up.size() + f->m2l.size() + f->down.size());
    counts[4] = boxes_at(f->levels);
    return SH_OK;
}

}  // extern "C"
