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
//   * M2L at level l >= 2: one call per offset d in [-3, 3]^3 \ [-1, 1]^3 (316 offsets); the
//     pairs (b + d -> b) of an offset have distinct targets b.  The pair is in the interaction
//     list of b when the parents of b and b + d are neighbours (or equal).
//   * L2L, level l -> l+1: one call per child octant, accumulating into the children.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
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

}  // namespace

struct sh_fmm {
    sh_ctx *ctx = nullptr;
    int P = 0, levels = 0;
    int64_t npts = 0;
    double origin[3] = {0, 0, 0};
    double width = 1;
    std::vector<int64_t> lvl_off;  // first box of level l in the M / L pools
    int64_t nbox = 0;
    std::vector<FmmCall> up, m2l, down;
    // device memory: one allocation
    void *mem = nullptr;
    double *M = nullptr, *L = nullptr;  // pools: nbox solids of P(P+1) reals
    int64_t *src = nullptr, *dst = nullptr;
    double *r = nullptr;
    double *leaf_centres = nullptr;
    int32_t *nbr = nullptr;  // leaves x 27
    int64_t npairs = 0;
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

void build(sh_fmm *f, HostPlan &hp, std::vector<double> &centres, std::vector<int32_t> &nbr)
{
    const int Lv = f->levels;
    // upward: children at level l (octant o) -> parents at level l - 1
    for (int l = Lv; l >= 1; --l) {
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
    // M2L at levels 2..L: offsets d with max |d_i| >= 2, parents neighbours
    for (int l = 2; l <= Lv; ++l) {
        const int64_t n = (int64_t)1 << l;
        const double w = f->width / (double)n;
        for (int dx = -3; dx <= 3; ++dx)
            for (int dy = -3; dy <= 3; ++dy)
                for (int dz = -3; dz <= 3; ++dz) {
                    if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) continue;
                    FmmCall c{SH_M2L, l, l, 0, (int64_t)hp.src.size()};
                    for (int64_t ix = 0; ix < n; ++ix) {
                        const int64_t sx = ix + dx;
                        if (sx < 0 || sx >= n) continue;
                        const int64_t ax = fdiv2(sx) - fdiv2(ix);
                        if (ax < -1 || ax > 1) continue;
                        for (int64_t iy = 0; iy < n; ++iy) {
                            const int64_t sy = iy + dy;
                            if (sy < 0 || sy >= n) continue;
                            const int64_t ay = fdiv2(sy) - fdiv2(iy);
                            if (ay < -1 || ay > 1) continue;
                            for (int64_t iz = 0; iz < n; ++iz) {
                                const int64_t sz = iz + dz;
                                if (sz < 0 || sz >= n) continue;
                                const int64_t az = fdiv2(sz) - fdiv2(iz);
                                if (az < -1 || az > 1) continue;
                                // r = x_B - x_A = centre(target) - centre(source) = -d w
                                hp.add(box_index(n, sx, sy, sz), box_index(n, ix, iy, iz), -dx * w, -dy * w, -dz * w);
                            }
                        }
                    }
                    c.count = (int64_t)hp.src.size() - c.off;
                    if (c.count > 0) f->m2l.push_back(c);
                }
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

sh_status sh_fmm_create(sh_ctx *ctx, int P, int levels, const double origin[3], double width, int64_t npts,
                        sh_fmm **out)
{
    if (!out) return SH_EINVAL;
    *out = nullptr;
    if (!ctx || !origin || !(width > 0.0) || npts < 1 || levels < 2 || levels > SH_FMM_MAX_LEVELS)
        return SH_EINVAL;
    if (P < 1 || P > ctx->max_order) return SH_EORDER;
    if (boxes_at(levels) * npts > ((int64_t)1 << 31)) return SH_EINVAL;
    sh_fmm *f = new (std::nothrow) sh_fmm;
    if (!f) return SH_ENOMEM;
    f->ctx = ctx;
    f->P = P;
    f->levels = levels;
    f->npts = npts;
    std::memcpy(f->origin, origin, sizeof f->origin);
    f->width = width;
    f->lvl_off.resize(levels + 2);
    f->lvl_off[0] = 0;
    for (int l = 0; l <= levels; ++l) f->lvl_off[l + 1] = f->lvl_off[l] + boxes_at(l);
    f->nbox = f->lvl_off[levels + 1];
    HostPlan hp;
    std::vector<double> centres;
    std::vector<int32_t> nbr;
    try {
        build(f, hp, centres, nbr);
    } catch (...) {
        delete f;
        return SH_ENOMEM;
    }
    f->npairs = (int64_t)hp.src.size();
    const int64_t S = (int64_t)P * (P + 1);
    auto up256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bM = up256(sizeof(double) * (size_t)(f->nbox * S));
    const size_t bI = up256(sizeof(int64_t) * (size_t)f->npairs);
    const size_t bR = up256(sizeof(double) * (size_t)(3 * f->npairs));
    const size_t bC = up256(sizeof(double) * centres.size());
    const size_t bN = up256(sizeof(int32_t) * nbr.size());
    DeviceGuard g(ctx->device);
    if (!g.ok) {
        delete f;
        return SH_EDEVICE;
    }
    if (hipMalloc(&f->mem, 2 * bM + 2 * bI + bR + bC + bN) != hipSuccess) {
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
    bool ok = hipMemcpy(f->src, hp.src.data(), sizeof(int64_t) * hp.src.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(f->dst, hp.dst.data(), sizeof(int64_t) * hp.dst.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(f->r, hp.r.data(), sizeof(double) * hp.r.size(), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(f->leaf_centres, centres.data(), sizeof(double) * centres.size(), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMemcpy(f->nbr, nbr.data(), sizeof(int32_t) * nbr.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        (void)hipFree(f->mem);
        delete f;
        return SH_EDEVICE;
    }
    *out = f;
    return SH_OK;
}

void sh_fmm_destroy(sh_fmm *f)
{
    if (!f) return;
    {
        DeviceGuard g(f->ctx->device);
        if (f->mem) (void)hipFree(f->mem);
    }
    delete f;
}

sh_status sh_fmm_evaluate(sh_fmm *f, const double *pts, const double *q, double *out, void *hip_stream)
{
    if (!f || !pts || !q || !out) return SH_EINVAL;
    DeviceGuard g(f->ctx->device);
    if (!g.ok) return SH_EDEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int P = f->P, Lv = f->levels;
    const int64_t S = (int64_t)P * (P + 1);
    const int64_t nleaf = boxes_at(Lv);
    double *Mleaf = f->M + f->lvl_off[Lv] * S;
    double *Lleaf = f->L + f->lvl_off[Lv] * S;
    if (shfmm::launch_p2m(P, nleaf, f->leaf_centres, f->npts, pts, q, Mleaf, S, s) != hipSuccess) return SH_EDEVICE;
    auto run = [&](const FmmCall &c, double *pool_in, double *pool_out, unsigned flags) {
        return shfmm::translate_device(f->ctx, c.op, SH_F64, P, P, c.count, f->r + 3 * c.off, f->src + c.off,
                                       pool_in + f->lvl_off[c.level_in] * S, S, f->dst + c.off,
                                       pool_out + f->lvl_off[c.level_out] * S, S, flags, hip_stream);
    };
    // upward pass: the first octant of a level overwrites its parents
    for (size_t i = 0; i < f->up.size(); ++i) {
        const sh_status st = run(f->up[i], f->M, f->M, (i % 8 == 0) ? 0u : SH_ACCUMULATE);
        if (st != SH_OK) return st;
    }
    // local expansions start at zero at levels 2..L (levels 0 and 1 have no interaction list)
    if (hipMemsetAsync(f->L + f->lvl_off[2] * S, 0, sizeof(double) * (size_t)((f->nbox - f->lvl_off[2]) * S), s) !=
        hipSuccess)
        return SH_EDEVICE;
    for (const FmmCall &c : f->m2l) {
        const sh_status st = run(c, f->M, f->L, SH_ACCUMULATE);
        if (st != SH_OK) return st;
    }
    for (const FmmCall &c : f->down) {
        const sh_status st = run(c, f->L, f->L, SH_ACCUMULATE);
        if (st != SH_OK) return st;
    }
    if (shfmm::launch_l2p(P, nleaf, f->leaf_centres, f->npts, pts, Lleaf, S, out, 0u, s) != hipSuccess)
        return SH_EDEVICE;
    if (shfmm::launch_p2p(nleaf, f->npts, pts, q, f->nbr, out, 1u, s) != hipSuccess) return SH_EDEVICE;
    return SH_OK;
}

sh_status sh_fmm_describe(const sh_fmm *f, int64_t *counts)
{
    if (!f || !counts) return SH_EINVAL;
    int64_t t[3] = {0, 0, 0};
    for (const FmmCall &c : f->up) t[0] += c.count;
    for (const FmmCall &c : f->m2l) t[1] += c.count;
    for (const FmmCall &c : f->down) t[2] += c.count;
    counts[0] = t[0];
    counts[1] = t[1];
    counts[2] = t[2];
    counts[3] = (int64_t)(f->up.size() + f->m2l.size() + f->down.size());
    counts[4] = boxes_at(f->levels);
    return SH_OK;
}

}  // extern "C"
