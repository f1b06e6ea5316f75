// Work-list planner: mixed M2M / M2L / L2L translations of any orders in one execution.
//
// A plan bins the items by kernel mapping:
//   * orders <= 16: the lane-per-translation list kernel, one bin per (operation, order
//     bucket); the bin's items are sorted by cost (largest orders first) and cut into
//     tasks of up to 64 (or 32) items sharing (p_in, p_out), one task per workgroup pass;
//   * larger orders, or bins the tuner assigns to it: the one-wavefront-per-translation
//     list kernel, one bin per (order class, arithmetic width), operations mixed.
// Each bin is one persistent launch.  Executions replay a HIP graph that holds every
// bin's launch on parallel branches, so one execution is one graph launch.  The tuner
// times the candidate mappings of each lane-per-translation bin on scratch arenas.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "context.hpp"
#include "kernels.hpp"
#include "list_plan.hpp"

using shfmm::DeviceGuard;
using shfmm::ListArgs;
using shfmm::ListItem;
using shfmm::ListTask;
using shfmm::ListBin;
using shfmm::MAP_BLOCK;
using shfmm::MAP_BLOCK8;
using shfmm::MAP_GENERAL;
using shfmm::MAP_LPT32;
using shfmm::MAP_LPT64;

static_assert(sizeof(sh_item) == sizeof(ListItem), "sh_item and ListItem must agree");
static_assert(offsetof(sh_item, in_off) == offsetof(ListItem, in_off), "sh_item layout");
static_assert(offsetof(sh_item, out_off) == offsetof(ListItem, out_off), "sh_item layout");
static_assert(offsetof(sh_item, r) == offsetof(ListItem, r), "sh_item layout");

namespace {

const char *mapping_name(int m)
{
    return m == MAP_LPT64   ? "lpt64"
           : m == MAP_LPT32 ? "lpt32"
           : m == MAP_BLOCK ? "block"
           : m == MAP_BLOCK8 ? "block8"
                             : "wave";
}

int64_t solid_reals(int p) { return (int64_t)p * (p + 1); }
int64_t cost(const ListItem &it) { return (int64_t)it.p_in * it.p_in * it.p_in + (int64_t)it.p_out * it.p_out * it.p_out; }

int general_class(int pm)
{
    return pm <= 16 ? 16 : pm <= 24 ? 24 : pm <= 32 ? 32 : pm <= 48 ? 48 : 64;
}

int lpt_bucket(int pm)
{
    int n = 0;
    const int *b = shfmm::list_buckets(&n);
    for (int i = 0; i < n; ++i)
        if (pm <= b[i]) return b[i];
    return 0;
}

// ---------------- tuning cache (per process, optionally mirrored in a file) ----------------

using TuneKey = std::tuple<int, int, int, int>;  // dtype, op, bucket, log2 count class
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
bool g_tune_loaded = false;

const char *tune_file() { return std::getenv("SHFMM_TUNE_FILE"); }

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *f = tune_file();
    if (!f || !*f) return;
    FILE *fp = std::fopen(f, "r");
    if (!fp) return;
    int d, o, b, c, m;
    char line[256];
    while (std::fgets(line, sizeof line, fp))
        if (std::sscanf(line, "%d %d %d %d %d", &d, &o, &b, &c, &m) == 5 && m >= 0 && m <= MAP_BLOCK8)
            g_tune[TuneKey{d, o, b, c}] = m;
    std::fclose(fp);
}

int count_class(int64_t n)
{
    int c = 0;
    while (((int64_t)1 << c) < n && c < 62) ++c;
    return c;
}

bool tune_lookup(const TuneKey &k, int *m)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(k);
    if (it == g_tune.end()) return false;
    *m = it->second;
    return true;
}

void tune_store(const TuneKey &k, int m)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tune[k] = m;
    const char *f = tune_file();
    if (!f || !*f) return;
    if (FILE *fp = std::fopen(f, "a")) {
        std::fprintf(fp, "%d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), m);
        std::fclose(fp);
    }
}

// ---------------- layout of a set of bins on the device ----------------

// Orders the items of one bin and, for lane-per-translation bins, cuts them into tasks.
void lay_out_bin(ListBin &b, std::vector<ListItem> &items, std::vector<ListTask> &tasks, int task_size)
{
    auto first = items.begin() + b.item_first, last = first + b.item_count;
    std::stable_sort(first, last, [](const ListItem &a, const ListItem &c) {
        const int64_t ca = cost(a), cc = cost(c);
        if (ca != cc) return ca > cc;
        if (a.p_in != c.p_in) return a.p_in > c.p_in;
        return a.p_out > c.p_out;
    });
    b.task_first = (int64_t)tasks.size();
    b.task_count = 0;
    if (b.mapping == MAP_GENERAL) return;
    for (int64_t i = 0; i < b.item_count;) {
        const ListItem &h = items[b.item_first + i];
        int64_t j = i + 1;
        while (j < b.item_count && j - i < task_size && items[b.item_first + j].p_in == h.p_in &&
               items[b.item_first + j].p_out == h.p_out)
            ++j;
        ListTask t{};
        t.p_in = h.p_in;
        t.p_out = h.p_out;
        t.count = (int32_t)(j - i);
        t.first = i;  // relative to the bin's first item
        tasks.push_back(t);
        i = j;
    }
    b.task_count = (int64_t)tasks.size() - b.task_first;
}

}  // namespace

hipError_t shfmm::launch_list_bin(const sh_ctx *ctx, bool f32, const ListBin &b, const ListItem *d_items,
                                  const ListTask *d_tasks, const void *in, void *out, unsigned flags, hipStream_t s)
{
    ListArgs la{};
    la.items = d_items + b.item_first;
    la.count = b.item_count;
    la.tasks = d_tasks + b.task_first;
    la.ntasks = b.task_count;
    la.arena_in = in;
    la.arena_out = out;
    la.flags = flags & SH_ACCUMULATE;
    la.err = ctx->err_flag;
    if (b.mapping == MAP_GENERAL) return shfmm::launch_list_general(ctx->tabs, la, f32, b.wide, b.pmax, s);
    if (shfmm::is_block(b.mapping))
        return shfmm::launch_list_big(ctx->tabs, la, b.op, f32, b.pmax, b.mapping == MAP_BLOCK ? 4 : 8, s);
    return shfmm::launch_list_lpt(ctx->tabs, la, b.op, f32, b.bucket, s);
}

namespace {

// Device copy of a laid-out item / task set: one allocation, items first.
struct DeviceLists {
    void *mem = nullptr;
    ListItem *items = nullptr;
    ListTask *tasks = nullptr;
    ~DeviceLists() { if (mem) (void)hipFree(mem); }
    hipError_t upload(const std::vector<ListItem> &it, const std::vector<ListTask> &tk)
    {
        const size_t ib = (it.size() * sizeof(ListItem) + 255) & ~size_t(255);
        const size_t tb = tk.size() * sizeof(ListTask);
        if (ib + tb == 0) return hipSuccess;
        hipError_t e = hipMalloc(&mem, ib + tb);
        if (e != hipSuccess) { mem = nullptr; return e; }
        items = reinterpret_cast<ListItem *>(mem);
        tasks = reinterpret_cast<ListTask *>(reinterpret_cast<char *>(mem) + ib);
        if (!it.empty() && (e = hipMemcpy(items, it.data(), it.size() * sizeof(ListItem), hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        if (!tk.empty() && (e = hipMemcpy(tasks, tk.data(), tb, hipMemcpyHostToDevice)) != hipSuccess) return e;
        return hipSuccess;
    }
};

// Times one mapping of a lane-per-translation bin on a sample of its items (offsets
// remapped densely into zero-filled scratch arenas).  Returns milliseconds, or < 0 on error.
float time_mapping(const sh_ctx *ctx, bool f32, const ListBin &proto, const std::vector<ListItem> &sample, int mapping,
                   unsigned flags, hipStream_t s)
{
    std::vector<ListItem> it(sample);
    int64_t in_total = 0, out_total = 0;
    for (auto &x : it) {
        x.in_off = in_total;
        x.out_off = out_total;
        in_total += solid_reals(x.p_in);
        out_total += solid_reals(x.p_out);
    }
    ListBin b = proto;
    b.mapping = mapping;
    b.item_first = 0;
    b.item_count = (int64_t)it.size();
    std::vector<ListTask> tk;
    lay_out_bin(b, it, tk, shfmm::task_size(mapping));
    DeviceLists dl;
    if (dl.upload(it, tk) != hipSuccess) return -1;
    const size_t elem = f32 ? sizeof(float) : sizeof(double);
    void *arena = nullptr;
    const size_t ab = (size_t)(in_total + out_total) * elem;
    if (hipMalloc(&arena, ab) != hipSuccess) return -1;
    float best = -1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMemsetAsync(arena, 0, ab, s) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess) {
        void *ain = arena, *aout = reinterpret_cast<char *>(arena) + (size_t)in_total * elem;
        bool ok = shfmm::launch_list_bin(ctx, f32, b, dl.items, dl.tasks, ain, aout, flags, s) == hipSuccess;
        for (int rep = 0; ok && rep < 3; ++rep) {
            ok = hipEventRecord(e0, s) == hipSuccess &&
                 shfmm::launch_list_bin(ctx, f32, b, dl.items, dl.tasks, ain, aout, flags, s) == hipSuccess &&
                 hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0;
            if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && (best < 0 || ms < best)) best = ms;
        }
        if (!ok) best = -1;
    }
    (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(arena);
    return best;
}

// Disjointness of half-open intervals [first, second).
bool disjoint_sorted(const std::vector<std::pair<int64_t, int64_t>> &v)
{
    for (size_t i = 1; i < v.size(); ++i)
        if (v[i].first < v[i - 1].second) return false;
    return true;
}

std::vector<std::pair<int64_t, int64_t>> merged(std::vector<std::pair<int64_t, int64_t>> v)
{
    std::sort(v.begin(), v.end());
    std::vector<std::pair<int64_t, int64_t>> out;
    for (auto &x : v) {
        if (!out.empty() && x.first <= out.back().second)
            out.back().second = std::max(out.back().second, x.second);
        else
            out.push_back(x);
    }
    return out;
}

// Whether any interval of `outs` (shifted by delta) meets the merged set `ins`.
bool meets(const std::vector<std::pair<int64_t, int64_t>> &outs, int64_t delta,
           const std::vector<std::pair<int64_t, int64_t>> &ins)
{
    for (auto &o : outs) {
        const int64_t a = o.first + delta, b = o.second + delta;
        auto it = std::upper_bound(ins.begin(), ins.end(), std::make_pair(a, INT64_MAX));
        if (it != ins.begin() && std::prev(it)->second > a) return true;
        if (it != ins.end() && it->first < b) return true;
    }
    return false;
}

}  // namespace

struct sh_plan {
    sh_ctx *ctx = nullptr;
    int dtype = SH_F64;
    unsigned flags = 0;
    int64_t count = 0;
    int64_t in_extent = 0, out_extent = 0;  // reals the arenas must hold
    std::vector<ListBin> bins;
    DeviceLists dev;
    std::vector<std::pair<int64_t, int64_t>> outs;  // output intervals, sorted
    std::vector<std::pair<int64_t, int64_t>> ins;   // merged input intervals
    std::mutex mu;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr, done = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *g_in = nullptr;
    void *g_out = nullptr;
    bool alias_checked = false;
    int64_t alias_delta = 0;

    ~sh_plan()
    {
        DeviceGuard g(ctx ? ctx->device : 0);
        if (done) (void)hipEventSynchronize(done);
        if (exec) (void)hipGraphExecDestroy(exec);
        for (auto s : side) (void)hipStreamDestroy(s);
        for (auto e : join) (void)hipEventDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
        if (fork) (void)hipEventDestroy(fork);
        if (done) (void)hipEventDestroy(done);
    }
};

namespace {

sh_status plan_build(sh_ctx *ctx, int dtype, const sh_item *items, int64_t count, unsigned flags, sh_plan *p)
{
    const bool f32 = dtype == SH_F32;
    std::vector<ListItem> list((size_t)count);
    if (count) std::memcpy(list.data(), items, (size_t)count * sizeof(ListItem));
    // validation
    p->outs.reserve((size_t)count);
    std::vector<std::pair<int64_t, int64_t>> ins;
    ins.reserve((size_t)count);
    for (const ListItem &it : list) {
        if (it.op != SH_M2M && it.op != SH_M2L && it.op != SH_L2L) return SH_EINVAL;
        if (it.reserved != 0) return SH_EINVAL;
        if (it.p_in < 1 || it.p_out < 1 || it.p_in > ctx->max_order || it.p_out > ctx->max_order) return SH_EORDER;
        const int64_t lim = (int64_t)1 << 60;
        if (it.in_off < 0 || it.out_off < 0 || it.in_off >= lim || it.out_off >= lim || (it.in_off & 1) ||
            (it.out_off & 1))
            return SH_EINVAL;
        if (!std::isfinite(it.r[0]) || !std::isfinite(it.r[1]) || !std::isfinite(it.r[2])) return SH_ESHIFT;
        if (it.op == SH_M2L && it.r[0] == 0 && it.r[1] == 0 && it.r[2] == 0) return SH_ESHIFT;
        p->outs.emplace_back(it.out_off, it.out_off + solid_reals(it.p_out));
        ins.emplace_back(it.in_off, it.in_off + solid_reals(it.p_in));
        p->in_extent = std::max(p->in_extent, ins.back().second);
        p->out_extent = std::max(p->out_extent, p->outs.back().second);
    }
    std::sort(p->outs.begin(), p->outs.end());
    if (!disjoint_sorted(p->outs)) return SH_EINVAL;
    p->ins = merged(std::move(ins));

    hipStream_t ts = nullptr;
    if ((flags & SH_PLAN_AUTOTUNE) && hipStreamCreateWithFlags(&ts, hipStreamNonBlocking) != hipSuccess)
        return SH_EDEVICE;
    auto choose = [&](ListBin &b, const std::vector<ListItem> &v) -> int {
        bool tuned = false;
        const bool block = shfmm::is_block(b.mapping);
        int m = shfmm::cached_mapping(dtype, b.op, b.bucket, (int64_t)v.size(), &tuned, b.mapping);
        if (tuned && block && m == MAP_BLOCK && !shfmm::big_list_two_per_cu(b.pmax)) m = MAP_BLOCK8;
        if (tuned || !(flags & SH_PLAN_AUTOTUNE)) {
            b.tuned = tuned;
            return m;
        }
        // candidates: the lane-per-translation task sizes and the wavefront kernel for orders
        // up to 16; the block kernel in both workgroup shapes (where two blocks' LDS fit) and
        // the wavefront kernel above
        std::vector<int> cands;
        if (!block)
            cands = {MAP_LPT64, MAP_LPT32, MAP_GENERAL};
        else if (shfmm::big_list_two_per_cu(b.pmax))
            cands = {MAP_BLOCK, MAP_BLOCK8, MAP_GENERAL};
        else
            cands = {MAP_BLOCK8, MAP_GENERAL};
        // a strided sample keeps the mix of orders of the bin
        const size_t kSample = 1 << 15;
        std::vector<ListItem> sample;
        const size_t stride = v.size() > kSample ? (v.size() + kSample - 1) / kSample : 1;
        for (size_t i = 0; i < v.size(); i += stride) sample.push_back(v[i]);
        float best = -1;
        for (int cand : cands) {
            const float ms = time_mapping(ctx, f32, b, sample, cand, flags, ts);
            if (ms < 0) return -1;
            if (best < 0 || ms < best) {
                best = ms;
                m = cand;
            }
        }
        tune_store(TuneKey{dtype, b.op, b.bucket, count_class((int64_t)v.size())}, m);
        b.tuned = true;
        return m;
    };
    std::vector<ListTask> tasks;
    const sh_status st = shfmm::bin_items(dtype, list, tasks, p->bins, choose);
    if (ts) (void)hipStreamDestroy(ts);
    if (st != SH_OK) return st;
    const hipError_t e = p->dev.upload(list, tasks);
    if (e == hipErrorOutOfMemory) return SH_ENOMEM;
    return e == hipSuccess ? SH_OK : SH_EDEVICE;
}

hipError_t capture(sh_plan *p, const void *in, void *out)
{
    hipError_t e;
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    const bool f32 = p->dtype == SH_F32;
    const size_t nside = std::min<size_t>(p->bins.size(), 4);
    if (!p->cap) {
        if ((e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming)) != hipSuccess) return e;
        for (size_t i = 0; i < nside; ++i) {
            hipStream_t s;
            hipEvent_t ev;
            if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return e;
            p->side.push_back(s);
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
            p->join.push_back(ev);
        }
    }
    if ((e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
    hipError_t le = hipEventRecord(p->fork, p->cap);
    for (size_t i = 0; le == hipSuccess && i < nside; ++i) le = hipStreamWaitEvent(p->side[i], p->fork, 0);
    for (size_t i = 0; le == hipSuccess && i < p->bins.size(); ++i)
        le = shfmm::launch_list_bin(p->ctx, f32, p->bins[i], p->dev.items, p->dev.tasks, in, out, p->flags, p->side[i % nside]);
    for (size_t i = 0; le == hipSuccess && i < nside; ++i) {
        le = hipEventRecord(p->join[i], p->side[i]);
        if (le == hipSuccess) le = hipStreamWaitEvent(p->cap, p->join[i], 0);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(p->cap, &graph);
    if (le == hipSuccess && e == hipSuccess) e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    p->g_in = in;
    p->g_out = out;
    return hipSuccess;
}

sh_status plan_execute(sh_plan *p, const void *in, int64_t in_reals, void *out, int64_t out_reals, void *stream)
{
    if (!p) return SH_EINVAL;
    if (p->count == 0) return SH_OK;
    if (!in || !out || in_reals < p->in_extent || out_reals < p->out_extent) return SH_EINVAL;
    const size_t elem = p->dtype == SH_F32 ? sizeof(float) : sizeof(double);
    if (reinterpret_cast<uintptr_t>(in) % (2 * elem) || reinterpret_cast<uintptr_t>(out) % (2 * elem))
        return SH_EINVAL;
    std::lock_guard<std::mutex> lk(p->mu);
    // arenas that share memory: no output may meet an input at the actual displacement
    const uintptr_t ib = reinterpret_cast<uintptr_t>(in), ob = reinterpret_cast<uintptr_t>(out);
    const uintptr_t ie = ib + (uintptr_t)in_reals * elem, oe = ob + (uintptr_t)out_reals * elem;
    if (ib < oe && ob < ie) {
        const intptr_t db = (intptr_t)(ob - ib);
        if (db % (intptr_t)elem) return SH_EINVAL;
        const int64_t delta = (int64_t)(db / (intptr_t)elem);
        if (!(p->alias_checked && p->alias_delta == delta)) {
            if (meets(p->outs, delta, p->ins)) return SH_EINVAL;
            p->alias_checked = true;
            p->alias_delta = delta;
        }
    }
    DeviceGuard g(p->ctx->device);
    if (!g.ok) return SH_EDEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool f32 = p->dtype == SH_F32;
    if (!p->done && hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) return SH_EDEVICE;
    if (p->flags & SH_PLAN_NO_GRAPH) {
        for (const ListBin &b : p->bins)
            if (shfmm::launch_list_bin(p->ctx, f32, b, p->dev.items, p->dev.tasks, in, out, p->flags, s) != hipSuccess)
                return SH_EDEVICE;
    } else {
        if (!p->exec || p->g_in != in || p->g_out != out) {
            if (capture(p, in, out) != hipSuccess) return SH_EDEVICE;
        }
        if (hipGraphLaunch(p->exec, s) != hipSuccess) return SH_EDEVICE;
    }
    return hipEventRecord(p->done, s) == hipSuccess ? SH_OK : SH_EDEVICE;
}

std::string describe(const sh_plan *p)
{
    std::string s = "{\"dtype\": \"";
    s += p->dtype == SH_F32 ? "f32" : "f64";
    s += "\", \"count\": " + std::to_string(p->count);
    s += ", \"graph\": ";
    s += (p->flags & SH_PLAN_NO_GRAPH) ? "false" : "true";
    s += ", \"in_extent\": " + std::to_string(p->in_extent) + ", \"out_extent\": " + std::to_string(p->out_extent);
    s += ", \"bins\": [";
    static const char *ops[] = {"m2m", "m2l", "l2l"};
    for (size_t i = 0; i < p->bins.size(); ++i) {
        const ListBin &b = p->bins[i];
        if (i) s += ", ";
        s += "{\"mapping\": \"";
        s += mapping_name(b.mapping);
        s += "\", \"op\": \"";
        s += b.op >= 0 ? ops[b.op] : "mixed";
        s += "\", \"bucket\": " + std::to_string(b.bucket) + ", \"pmax\": " + std::to_string(b.pmax);
        s += ", \"wide\": ";
        s += b.wide ? "true" : "false";
        s += ", \"items\": " + std::to_string(b.item_count) + ", \"tasks\": " + std::to_string(b.task_count);
        s += ", \"tuned\": ";
        s += b.tuned ? "true" : "false";
        s += "}";
    }
    s += "]}";
    return s;
}

}  // namespace

sh_status shfmm::bin_items(int dtype, std::vector<ListItem> &list, std::vector<ListTask> &tasks,
                           std::vector<ListBin> &bins, const MappingChoice &choose)
{
    const bool f32 = dtype == SH_F32;
    // group: lane-per-translation candidates by (op, bucket); the rest by (class, width)
    std::map<std::tuple<int, int, int, int>, std::vector<ListItem>> groups;  // (kind, op, bucket, wide)
    for (const ListItem &it : list) {
        const int pm = std::max(it.p_in, it.p_out);
        const int bk = lpt_bucket(pm);
        if (bk > 0)
            groups[std::make_tuple(0, it.op, bk, 0)].push_back(it);
        else if (shfmm::big_available(it.p_in, it.p_out))
            groups[std::make_tuple(2, it.op, pm <= 20 ? 20 : pm <= 24 ? 24 : shfmm::kBigOrder - 1, 0)].push_back(it);
        else {
            const bool wide = f32 && pm >= shfmm::kF32WideOrder;
            groups[std::make_tuple(1, -1, general_class(pm), wide ? 1 : 0)].push_back(it);
        }
    }
    list.clear();
    std::vector<ListBin> made;
    for (auto &g : groups) {
        auto &v = g.second;
        ListBin b;
        b.op = std::get<1>(g.first);
        b.bucket = std::get<2>(g.first);
        b.wide = std::get<3>(g.first) != 0;
        for (auto &x : v) b.pmax = std::max(b.pmax, std::max(x.p_in, x.p_out));
        if (std::get<0>(g.first) == 1) {
            b.mapping = MAP_GENERAL;
        } else if (std::get<0>(g.first) == 2) {
            b.mapping = shfmm::big_list_two_per_cu(b.pmax) ? MAP_BLOCK : MAP_BLOCK8;  // default
            b.wide = f32 && b.pmax >= shfmm::kF32WideOrder;  // should the wavefront kernel take it
            const int m = choose(b, v);
            if (m < 0) return SH_EDEVICE;
            b.mapping = m;
        } else {
            const int m = choose(b, v);
            if (m < 0) return SH_EDEVICE;
            b.mapping = m;
        }
        b.item_first = (int64_t)list.size();
        b.item_count = (int64_t)v.size();
        list.insert(list.end(), v.begin(), v.end());
        std::vector<ListItem>().swap(v);
        lay_out_bin(b, list, tasks, shfmm::task_size(b.mapping));
        made.push_back(b);
    }
    // largest bins first, so that their persistent grids start first on the device
    std::stable_sort(made.begin(), made.end(), [](const ListBin &a, const ListBin &b) {
        return a.item_count * a.pmax > b.item_count * b.pmax;
    });
    bins.insert(bins.end(), made.begin(), made.end());
    return SH_OK;
}

int shfmm::cached_mapping(int dtype, int op, int bucket, int64_t count, bool *tuned, int dflt)
{
    int m = dflt;
    const bool hit = tune_lookup(TuneKey{dtype, op, bucket, count_class(count)}, &m);
    if (tuned) *tuned = hit;
    return hit ? m : dflt;
}

extern "C" {

sh_status sh_plan_create(sh_ctx *ctx, int dtype, const sh_item *items, int64_t count, unsigned flags, sh_plan **out)
{
    if (!out) return SH_EINVAL;
    *out = nullptr;
    if (!ctx || (dtype != SH_F64 && dtype != SH_F32) || count < 0 || (count > 0 && !items) ||
        (flags & ~(SH_ACCUMULATE | SH_PLAN_AUTOTUNE | SH_PLAN_NO_GRAPH)))
        return SH_EINVAL;
    try {
        DeviceGuard g(ctx->device);
        if (!g.ok) return SH_EDEVICE;
        sh_plan *p = new sh_plan;
        p->ctx = ctx;
        p->dtype = dtype;
        p->flags = flags;
        p->count = count;
        const sh_status st = plan_build(ctx, dtype, items, count, flags, p);
        if (st != SH_OK) {
            delete p;
            return st;
        }
        *out = p;
        return SH_OK;
    } catch (const std::bad_alloc &) {
        return SH_ENOMEM;
    } catch (...) {
        return SH_EDEVICE;
    }
}

sh_status sh_plan_execute(sh_plan *plan, const void *arena_in, int64_t in_reals, void *arena_out, int64_t out_reals,
                          void *hip_stream)
{
    try {
        return plan_execute(plan, arena_in, in_reals, arena_out, out_reals, hip_stream);
    } catch (...) {
        return SH_EDEVICE;
    }
}

sh_status sh_plan_describe(const sh_plan *plan, char *buf, int64_t len, int64_t *needed)
{
    if (!plan || len < 0 || (len > 0 && !buf)) return SH_EINVAL;
    try {
        const std::string s = describe(plan);
        if (needed) *needed = (int64_t)s.size() + 1;
        if (len > 0) {
            const size_t n = std::min<size_t>(s.size(), (size_t)len - 1);
            std::memcpy(buf, s.data(), n);
            buf[n] = '\0';
        }
        return SH_OK;
    } catch (...) {
        return SH_EINVAL;
    }
}

void sh_plan_destroy(sh_plan *plan)
{
    try {
        delete plan;
    } catch (...) {
    }
}

sh_status sh_translate_list(sh_ctx *ctx, int dtype, const sh_item *items, int64_t count, const void *arena_in,
                            int64_t in_reals, void *arena_out, int64_t out_reals, unsigned flags, void *hip_stream)
{
    if (flags & ~SH_ACCUMULATE) return SH_EINVAL;
    sh_plan *p = nullptr;
    sh_status st = sh_plan_create(ctx, dtype, items, count, flags | SH_PLAN_NO_GRAPH, &p);
    if (st != SH_OK) return st;
    st = sh_plan_execute(p, arena_in, in_reals, arena_out, out_reals, hip_stream);
    if (st == SH_OK) {
        DeviceGuard g(ctx->device);
        if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess) st = SH_EDEVICE;
    }
    sh_plan_destroy(p);
    return st;
}

}  // extern "C"
