// Serving runtime: a request loop for translation jobs with continuous batching.
//
// * Resident pools.  A "tree" owns a multipole pool and a local pool (solids of one order
//   each) carved out of one device arena, and keeps them between jobs.
// * Admission by HBM footprint.  A job's footprint is the device staging its work records
//   take while it is in flight (an upper bound of 80 bytes per translation plus 2 KiB);
//   jobs are admitted, first come first served with backfill, while the staging arena has
//   room and nothing in flight on their tree conflicts with them: M2L jobs that overwrite
//   (no SH_ACCUMULATE) only read the multipole pool, so several of them run together on one
//   tree while their destination slots are disjoint; M2M, L2L and accumulating jobs run alone
//   on their tree.  A job passed over keeps every later job of its tree waiting, so jobs that
//   touch the same slots complete in submission order.
// * Continuous batching.  The scheduler thread fuses every admissible job into one batch:
//   one indexed translation call per (dtype, operation, orders, accumulate) group, on the
//   least loaded of a few streams, so batches overlap on the device and jobs arriving
//   meanwhile join the next batch as soon as staging frees up.
// * Latency.  One completion thread per stream waits for its batches in order and stamps
//   every job of a finished batch; p50 / p99 are taken over all completed jobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "context.hpp"
#include "kernels.hpp"

using shfmm::DeviceGuard;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int64_t kAlign = 256;
int64_t round_up(int64_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// First-fit range allocator over [0, size) with coalescing, 256-byte granules.
struct RangeAlloc {
    std::map<int64_t, int64_t> free_;  // offset -> length
    int64_t size = 0, used = 0, peak = 0;
    void init(int64_t s)
    {
        size = s;
        free_.clear();
        if (s > 0) free_[0] = s;
    }
    int64_t alloc(int64_t n)
    {
        n = round_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const int64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            used += n;
            peak = std::max(peak, used);
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t n)
    {
        n = round_up(n);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Tree {
    int dtype = SH_F64;
    int p_m = 0, p_l = 0;
    int64_t n_m = 0, n_l = 0;
    int64_t off_m = 0, off_l = 0;  // byte offsets of the pools in the arena (multiples of a solid)
    int64_t raw_m = 0, raw_l = 0;  // the allocated ranges (offset, length) they sit in
    int64_t bytes_m = 0, bytes_l = 0;
    int running = 0;               // jobs of this tree reserved for a batch or in flight
    bool exclusive = false;        // one of them needs the tree alone
    std::vector<unsigned char> claim;  // local slots written by running shared M2L jobs
    int pending = 0;               // jobs queued or in flight
};

// An overwriting M2L reads only multipoles and writes only its destination locals, so jobs of
// this kind share a tree while their destinations are disjoint.
bool shares_tree(int op, unsigned flags) { return op == SH_M2L && !(flags & SH_ACCUMULATE); }

// A host buffer for a job's packed records, taken from the server's free list and returned
// to it when the job completes, so that submissions write memory that is already mapped
// (packing into freshly allocated pages costs several times the packing itself).
struct Buf {
    std::unique_ptr<char[]> p;
    size_t cap = 0;
};

struct Job {
    int32_t tree = 0, op = 0;
    unsigned flags = 0;
    int64_t count = 0;
    // packed at submission: the source and the destination slots as solid indices counted
    // from the start of the pool arena (count each, so both stay 8-byte aligned), then the
    // shifts in the tree's dtype (count x 3)
    Buf packed;
    int64_t dst_base = 0;       // arena index of the destination pool's slot 0
    int64_t footprint = 0;
    double t_submit = 0, t_done = 0;
    bool done = false;
    bool deferred = false;  // passed over at least once for lack of staging
    int status = SH_OK;
};

struct Batch {
    int stream = 0;
    hipEvent_t ev = nullptr;
    std::vector<int64_t> jobs;
    std::vector<Job *> jp;          // the jobs (stable: owned by unique_ptr)
    std::vector<const Tree *> tp;   // their trees (stable: map nodes, kept while jobs pend)
    int64_t st_off = -1, st_bytes = 0;
    int64_t translations = 0;
    bool launched = true;
};

int64_t job_footprint(int64_t count) { return 80 * count + 2048; }

// Copies into the pinned staging, split over a few threads: one thread's memcpy moves a few
// GB/s, which at saturation falls behind the device.  Pieces of at most kCopyPiece bytes are
// taken in turn by the caller and kCopyThreads workers; run() returns when all are copied.
// Only the scheduler thread calls run().
struct CopySeg {
    char *dst;
    const char *src;
    size_t n;
};
constexpr size_t kCopyPiece = 1 << 20;
constexpr int kCopyThreads = 3;

void add_copy(std::vector<CopySeg> &v, char *dst, const char *src, size_t n)
{
    for (size_t o = 0; o < n; o += kCopyPiece) v.push_back(CopySeg{dst + o, src + o, std::min(kCopyPiece, n - o)});
}

struct CopyPool {
    std::vector<std::thread> th;
    std::mutex mu;
    std::condition_variable cv_go, cv_done;
    const std::vector<CopySeg> *segs = nullptr;
    size_t next = 0, left = 0;
    bool stop = false;

    void worker()
    {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_go.wait(lk, [&] { return stop || (segs && next < segs->size()); });
            if (!segs || next >= segs->size()) return;  // stopping, nothing left to copy
            const CopySeg sg = (*segs)[next++];
            lk.unlock();
            std::memcpy(sg.dst, sg.src, sg.n);
            lk.lock();
            if (--left == 0) cv_done.notify_all();
        }
    }
    void start()
    {
        for (int i = 0; i < kCopyThreads; ++i) th.emplace_back(&CopyPool::worker, this);
    }
    void finish()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_go.notify_all();
        for (auto &t : th)
            if (t.joinable()) t.join();
        th.clear();
    }
    void run(const std::vector<CopySeg> &v)
    {
        if (v.size() <= 1 || th.empty()) {
            for (const CopySeg &sg : v) std::memcpy(sg.dst, sg.src, sg.n);
            return;
        }
        std::unique_lock<std::mutex> lk(mu);
        segs = &v;
        next = 0;
        left = v.size();
        cv_go.notify_all();
        while (next < v.size()) {
            const CopySeg sg = v[next++];
            lk.unlock();
            std::memcpy(sg.dst, sg.src, sg.n);
            lk.lock();
            --left;
        }
        cv_done.wait(lk, [&] { return left == 0; });
        segs = nullptr;
    }
};

// destination slots of a job (relative to its pool), read back from its packed records
const int64_t *job_dst_abs(const Job &j)
{
    return reinterpret_cast<const int64_t *>(j.packed.p.get()) + j.count;
}

}  // namespace

struct sh_server {
    sh_ctx *ctx = nullptr;
    sh_server_config cfg{};
    void *pool = nullptr;        // device arena of resident pools
    void *dstage = nullptr;      // device staging (work records)
    void *hstage = nullptr;      // pinned host staging, same offsets
    RangeAlloc pool_alloc, stage_alloc;
    CopyPool copier;
    // free pack buffers (returned by completed jobs), at most kKeepBufBytes in all
    std::mutex buf_mu;
    std::vector<Buf> bufs;
    size_t bufs_bytes = 0;
    std::vector<hipStream_t> streams;
    std::vector<std::deque<Batch>> inflight;
    std::vector<std::thread> completers;
    std::thread scheduler;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_complete;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, std::unique_ptr<Job>> jobs;
    std::map<int32_t, Tree> trees;
    int32_t next_tree = 1;
    int64_t next_job = 1;
    bool stop = false;
    bool sched_done = false;
    // statistics
    std::vector<double> latencies;
    int64_t jobs_done = 0, translations_done = 0, batches = 0, batch_jobs = 0, queue_peak = 0, failed = 0;
    int64_t jobs_deferred = 0;
    double t_first_submit = -1, t_last_done = -1;

    int inflight_total() const
    {
        int n = 0;
        for (auto &d : inflight) n += (int)d.size();
        return n;
    }
};

namespace {

// Free pack buffers kept for reuse: up to 8x the staging budget (at least 64 MiB) in all.
size_t keep_buf_bytes(const sh_server *S) { return std::max<size_t>(size_t(64) << 20, 8 * (size_t)S->cfg.staging_bytes); }

// A pack buffer of at least n bytes: the smallest free one that fits, else a new one.
Buf take_buf(sh_server *S, size_t n)
{
    {
        std::lock_guard<std::mutex> lk(S->buf_mu);
        size_t best = SIZE_MAX;
        for (size_t i = 0; i < S->bufs.size(); ++i)
            if (S->bufs[i].cap >= n && (best == SIZE_MAX || S->bufs[i].cap < S->bufs[best].cap)) best = i;
        if (best != SIZE_MAX) {
            Buf b = std::move(S->bufs[best]);
            if (best + 1 != S->bufs.size()) S->bufs[best] = std::move(S->bufs.back());
            S->bufs.pop_back();
            S->bufs_bytes -= b.cap;
            return b;
        }
    }
    Buf b;
    b.p.reset(new char[n]);
    b.cap = n;
    return b;
}

// Returns a buffer to the free list (or frees it when the list is full).
void give_buf(sh_server *S, Buf &&b)
{
    if (!b.p) return;
    Buf drop;
    std::lock_guard<std::mutex> lk(S->buf_mu);
    if (S->bufs_bytes + b.cap > keep_buf_bytes(S)) {
        drop = std::move(b);
        return;
    }
    S->bufs_bytes += b.cap;
    S->bufs.push_back(std::move(b));
}

// Reserves (on) or releases (off) a job's claim on its tree: the running count, the tree
// alone for a job that does not share it, the destination slots for one that does.  Called
// with the server lock held.
void reserve_job(Tree &t, const Job &j, bool on)
{
    t.running += on ? 1 : -1;
    if (shares_tree(j.op, j.flags)) {
        const int64_t *d = job_dst_abs(j);
        for (int64_t i = 0; i < j.count; ++i) t.claim[(size_t)(d[i] - j.dst_base)] = on ? 1 : 0;
    } else {
        t.exclusive = on;
    }
}

// Builds and launches one batch (called by the scheduler without the lock; the batch's jobs
// and trees are reserved, so nothing it reads changes meanwhile).  The batch's jobs are grouped
// by (dtype, operation, orders, accumulate); each group runs as one indexed translation call
// whose slot indices count solids from the start of the pool arena (every pool sits at a
// multiple of its solid size), so jobs of different trees share the call.  Staging per group:
// the shifts (in the group's dtype), then the source and the destination indices, each run
// 256-byte aligned.  The kernel a translation runs on follows from its own operation and
// orders, never from its batch mates.
hipError_t launch_batch(sh_server *S, Batch &b)
{
    struct Group {
        int dtype, op, p_in, p_out;
        unsigned flags;
        std::vector<size_t> jobs;  // indices into b.jp
        int64_t count = 0, r_off = 0, s_off = 0, d_off = 0;
    };
    std::vector<Group> groups;
    for (size_t k = 0; k < b.jp.size(); ++k) {
        const Job &j = *b.jp[k];
        const Tree &t = *b.tp[k];
        const int p_in = j.op == SH_L2L ? t.p_l : t.p_m, p_out = j.op == SH_M2M ? t.p_m : t.p_l;
        const unsigned fl = j.flags & SH_ACCUMULATE;
        Group *g = nullptr;
        for (auto &x : groups)
            if (x.dtype == t.dtype && x.op == j.op && x.p_in == p_in && x.p_out == p_out && x.flags == fl) g = &x;
        if (!g) {
            groups.push_back(Group{t.dtype, j.op, p_in, p_out, fl, {}});
            g = &groups.back();
        }
        g->jobs.push_back(k);
        g->count += j.count;
    }
    int64_t bytes = 0;
    for (auto &g : groups) {
        const int64_t elem = g.dtype == SH_F32 ? 4 : 8;
        g.r_off = bytes;
        bytes = round_up(bytes + 3 * elem * g.count);
        g.s_off = bytes;
        bytes = round_up(bytes + 8 * g.count);
        g.d_off = bytes;
        bytes = round_up(bytes + 8 * g.count);
    }
    if (bytes > b.st_bytes) return hipErrorInvalidValue;  // footprint bound violated (cannot happen)
    char *h = static_cast<char *>(S->hstage) + b.st_off;
    char *d = static_cast<char *>(S->dstage) + b.st_off;
    std::vector<CopySeg> segs;
    for (auto &g : groups) {
        const int64_t elem = g.dtype == SH_F32 ? 4 : 8;
        int64_t at = 0;
        for (size_t k : g.jobs) {
            const Job &j = *b.jp[k];
            const size_t rb = (size_t)(3 * elem * j.count), ib = (size_t)(8 * j.count);
            const char *src = j.packed.p.get();
            add_copy(segs, h + g.s_off + 8 * at, src, ib);
            add_copy(segs, h + g.d_off + 8 * at, src + ib, ib);
            add_copy(segs, h + g.r_off + 3 * elem * at, src + 2 * ib, rb);
            at += j.count;
        }
    }
    S->copier.run(segs);
    hipStream_t s = S->streams[b.stream];
    hipError_t e = hipMemcpyAsync(d, h, (size_t)bytes, hipMemcpyHostToDevice, s);
    for (auto &g : groups) {
        if (e != hipSuccess) break;
        const int64_t ld_in = (int64_t)g.p_in * (g.p_in + 1), ld_out = (int64_t)g.p_out * (g.p_out + 1);
        const sh_status st = shfmm::translate_device(
            S->ctx, g.op, g.dtype, g.p_in, g.p_out, g.count, d + g.r_off, reinterpret_cast<const int64_t *>(d + g.s_off),
            S->pool, ld_in, reinterpret_cast<const int64_t *>(d + g.d_off), S->pool, ld_out, g.flags, s);
        if (st != SH_OK) e = hipErrorUnknown;
    }
    if (e == hipSuccess) e = hipEventRecord(b.ev, s);
    return e;
}

void scheduler_main(sh_server *S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // gather a batch: every queued job (first come first served, later ones backfill)
        // whose tree is idle and whose footprint fits the staging left
        Batch b;
        int stream = -1;
        size_t best = SIZE_MAX;
        for (size_t i = 0; i < S->inflight.size(); ++i)
            if (S->inflight[i].size() < 2 && S->inflight[i].size() < best) {
                best = S->inflight[i].size();
                stream = (int)i;
            }
        if (stream >= 0 && !S->queue.empty()) {
            int64_t need = 0;
            std::vector<size_t> take;
            std::vector<int32_t> blocked;  // trees with a job passed over in this scan
            const int64_t free_total = S->stage_alloc.size - S->stage_alloc.used;
            for (size_t qi = 0; qi < S->queue.size() && (int)take.size() < S->cfg.max_batch_jobs; ++qi) {
                Job &j = *S->jobs.at(S->queue[qi]);
                Tree &t = S->trees.at(j.tree);
                if (std::find(blocked.begin(), blocked.end(), j.tree) != blocked.end()) continue;
                const bool shared = shares_tree(j.op, j.flags);
                bool fits = shared ? !t.exclusive : t.running == 0;
                if (fits && shared) {
                    if (t.claim.size() != (size_t)t.n_l) t.claim.assign((size_t)t.n_l, 0);
                    const int64_t *d = job_dst_abs(j);
                    for (int64_t i = 0; i < j.count; ++i)
                        if (t.claim[(size_t)(d[i] - j.dst_base)]) {
                            fits = false;
                            break;
                        }
                }
                if (fits && need + j.footprint > free_total) {
                    fits = false;
                    if (!j.deferred) {
                        j.deferred = true;
                        ++S->jobs_deferred;
                    }
                }
                if (!fits) {
                    blocked.push_back(j.tree);
                    continue;
                }
                reserve_job(t, j, true);
                need += j.footprint;
                take.push_back(qi);
            }
            if (!take.empty()) {
                int64_t off = S->stage_alloc.alloc(need);
                while (off < 0 && !take.empty()) {  // fragmentation: shrink the batch
                    Job &j = *S->jobs.at(S->queue[take.back()]);
                    reserve_job(S->trees.at(j.tree), j, false);
                    need -= j.footprint;
                    take.pop_back();
                    off = take.empty() ? -1 : S->stage_alloc.alloc(need);
                }
                if (off >= 0) {
                    b.stream = stream;
                    b.st_off = off;
                    b.st_bytes = round_up(need);
                    for (size_t k = take.size(); k-- > 0;) {
                        const int64_t id = S->queue[take[k]];
                        b.jobs.push_back(id);
                        S->queue.erase(S->queue.begin() + (std::ptrdiff_t)take[k]);
                    }
                    std::reverse(b.jobs.begin(), b.jobs.end());
                    for (int64_t id : b.jobs) {
                        Job *j = S->jobs.at(id).get();
                        Tree &t = S->trees.at(j->tree);
                        b.jp.push_back(j);
                        b.tp.push_back(&t);
                        b.translations += j->count;
                    }
                }
            }
        }
        if (b.jobs.empty()) {
            if (S->stop && S->queue.empty()) break;
            S->cv_sched.wait(lk);
            continue;
        }
        // jobs, trees and staging of the batch are reserved: nothing launch_batch reads is
        // changed by other threads until the batch completes
        // launch outside the lock
        lk.unlock();
        hipError_t e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = launch_batch(S, b);
        lk.lock();
        b.launched = e == hipSuccess;
        if (!b.launched)
            for (Job *j : b.jp) j->status = SH_EDEVICE;
        ++S->batches;
        S->batch_jobs += (int64_t)b.jobs.size();
        S->inflight[b.stream].push_back(std::move(b));
        S->cv_complete.notify_all();
    }
    S->sched_done = true;
    S->cv_complete.notify_all();
}

void completer_main(sh_server *S, int stream)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_complete.wait(lk, [&] { return !S->inflight[stream].empty() || S->sched_done; });
        if (S->inflight[stream].empty()) break;  // the scheduler has finished and nothing is left
        Batch &b = S->inflight[stream].front();
        const hipEvent_t ev = b.ev;
        const bool launched = b.launched;
        lk.unlock();
        hipError_t e = hipSuccess;
        if (launched) e = hipEventSynchronize(ev);
        const double t = now_s();
        lk.lock();
        Batch done = std::move(S->inflight[stream].front());
        S->inflight[stream].pop_front();
        for (Job *jp : done.jp) {
            Job &j = *jp;
            j.done = true;
            j.t_done = t;
            if (e != hipSuccess) j.status = SH_EDEVICE;
            Tree &tr = S->trees.at(j.tree);
            reserve_job(tr, j, false);
            give_buf(S, std::move(j.packed));
            --tr.pending;
            if (j.status == SH_OK) {
                S->latencies.push_back(t - j.t_submit);
                ++S->jobs_done;
                S->translations_done += j.count;
            } else {
                ++S->failed;
            }
        }
        S->t_last_done = t;
        S->stage_alloc.release(done.st_off, done.st_bytes);
        if (done.ev) (void)hipEventDestroy(done.ev);
        S->cv_sched.notify_all();
        S->cv_done.notify_all();
        S->cv_complete.notify_all();
    }
}

// waits (with the lock held) until a tree has no queued or in-flight job
void wait_tree_idle(sh_server *S, std::unique_lock<std::mutex> &lk, int32_t tree)
{
    S->cv_done.wait(lk, [&] {
        auto it = S->trees.find(tree);
        return it == S->trees.end() || it->second.pending == 0;
    });
}

}  // namespace

extern "C" {

sh_status sh_server_create(sh_ctx *ctx, const sh_server_config *cfg, sh_server **out)
{
    if (!out) return SH_EINVAL;
    *out = nullptr;
    if (!ctx || !cfg || cfg->pool_bytes < 0 || cfg->staging_bytes < (1 << 16) || cfg->streams < 1 ||
        cfg->streams > 8 || cfg->max_batch_jobs < 1)
        return SH_EINVAL;
    try {
        DeviceGuard g(ctx->device);
        if (!g.ok) return SH_EDEVICE;
        sh_server *S = new sh_server;
        S->ctx = ctx;
        S->cfg = *cfg;
        S->cfg.pool_bytes = round_up(cfg->pool_bytes);
        S->cfg.staging_bytes = round_up(cfg->staging_bytes);
        bool ok = true;
        if (S->cfg.pool_bytes > 0 && hipMalloc(&S->pool, (size_t)S->cfg.pool_bytes) != hipSuccess) {
            S->pool = nullptr;
            ok = false;
        }
        if (ok && hipMalloc(&S->dstage, (size_t)S->cfg.staging_bytes) != hipSuccess) {
            S->dstage = nullptr;
            ok = false;
        }
        if (ok && hipHostMalloc(&S->hstage, (size_t)S->cfg.staging_bytes, hipHostMallocDefault) != hipSuccess) {
            S->hstage = nullptr;
            ok = false;
        }
        for (int i = 0; ok && i < cfg->streams; ++i) {
            hipStream_t s;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
                ok = false;
            else
                S->streams.push_back(s);
        }
        if (!ok) {
            for (auto s : S->streams) (void)hipStreamDestroy(s);
            if (S->hstage) (void)hipHostFree(S->hstage);
            if (S->dstage) (void)hipFree(S->dstage);
            if (S->pool) (void)hipFree(S->pool);
            delete S;
            return SH_ENOMEM;
        }
        S->pool_alloc.init(S->cfg.pool_bytes);
        S->stage_alloc.init(S->cfg.staging_bytes);
        S->inflight.resize(S->streams.size());
        S->copier.start();
        S->scheduler = std::thread(scheduler_main, S);
        for (size_t i = 0; i < S->streams.size(); ++i) S->completers.emplace_back(completer_main, S, (int)i);
        *out = S;
        return SH_OK;
    } catch (const std::bad_alloc &) {
        return SH_ENOMEM;
    } catch (...) {
        return SH_EDEVICE;
    }
}

void sh_server_destroy(sh_server *S)
{
    if (!S) return;
    try {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_sched.notify_all();
        S->cv_complete.notify_all();
        if (S->scheduler.joinable()) S->scheduler.join();
        S->cv_complete.notify_all();
        for (auto &t : S->completers)
            if (t.joinable()) t.join();
        S->copier.finish();
        DeviceGuard g(S->ctx->device);
        for (auto s : S->streams) (void)hipStreamDestroy(s);
        if (S->hstage) (void)hipHostFree(S->hstage);
        if (S->dstage) (void)hipFree(S->dstage);
        if (S->pool) (void)hipFree(S->pool);
        delete S;
    } catch (...) {
    }
}

sh_status sh_server_tree_create(sh_server *S, int dtype, int p_m, int64_t n_m, int p_l, int64_t n_l, int32_t *tree)
{
    if (!S || !tree || (dtype != SH_F64 && dtype != SH_F32) || n_m < 0 || n_l < 0) return SH_EINVAL;
    if (p_m < 1 || p_l < 1 || p_m > S->ctx->max_order || p_l > S->ctx->max_order) return SH_EORDER;
    try {
        const int64_t elem = dtype == SH_F32 ? 4 : 8;
        Tree t;
        t.dtype = dtype;
        t.p_m = p_m;
        t.p_l = p_l;
        t.n_m = n_m;
        t.n_l = n_l;
        // each pool starts at a multiple of its solid size in the arena, so that batches can
        // address every tree's slots by solid index from the arena's start; the allocation
        // holds one solid of slack for that
        const int64_t sz_m = (int64_t)p_m * (p_m + 1) * elem, sz_l = (int64_t)p_l * (p_l + 1) * elem;
        // the pools' byte sizes must not overflow (checked by division)
        if (n_m > INT64_MAX / sz_m - 2 || n_l > INT64_MAX / sz_l - 2) return SH_EBUSY;
        t.bytes_m = std::max<int64_t>(kAlign, (n_m + 1) * sz_m);
        t.bytes_l = std::max<int64_t>(kAlign, (n_l + 1) * sz_l);
        std::lock_guard<std::mutex> lk(S->mu);
        t.raw_m = S->pool_alloc.alloc(t.bytes_m);
        if (t.raw_m < 0) return SH_EBUSY;
        t.raw_l = S->pool_alloc.alloc(t.bytes_l);
        if (t.raw_l < 0) {
            S->pool_alloc.release(t.raw_m, t.bytes_m);
            return SH_EBUSY;
        }
        t.off_m = (t.raw_m + sz_m - 1) / sz_m * sz_m;
        t.off_l = (t.raw_l + sz_l - 1) / sz_l * sz_l;
        const int32_t id = S->next_tree++;
        S->trees[id] = t;
        *tree = id;
        return SH_OK;
    } catch (...) {
        return SH_ENOMEM;
    }
}

static sh_status tree_copy(sh_server *S, int32_t tree, int pool, int64_t first, int64_t n, void *host, bool write)
{
    if (!S || (pool != 0 && pool != 1) || first < 0 || n < 0 || (n > 0 && !host)) return SH_EINVAL;
    try {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->trees.find(tree);
        if (it == S->trees.end()) return SH_EINVAL;
        wait_tree_idle(S, lk, tree);
        it = S->trees.find(tree);
        if (it == S->trees.end()) return SH_EINVAL;
        const Tree t = it->second;
        const int p = pool == 0 ? t.p_m : t.p_l;
        const int64_t cnt = pool == 0 ? t.n_m : t.n_l;
        if (first + n > cnt) return SH_EINVAL;
        if (n == 0) return SH_OK;
        const int64_t elem = t.dtype == SH_F32 ? 4 : 8;
        const int64_t sz = (int64_t)p * (p + 1) * elem;
        char *dev = static_cast<char *>(S->pool) + (pool == 0 ? t.off_m : t.off_l) + first * sz;
        lk.unlock();
        DeviceGuard g(S->ctx->device);
        const hipError_t e = write ? hipMemcpy(dev, host, (size_t)(n * sz), hipMemcpyHostToDevice)
                                   : hipMemcpy(host, dev, (size_t)(n * sz), hipMemcpyDeviceToHost);
        return e == hipSuccess ? SH_OK : SH_EDEVICE;
    } catch (...) {
        return SH_EDEVICE;
    }
}

sh_status sh_server_tree_write(sh_server *S, int32_t tree, int pool, int64_t first, int64_t n, const void *host)
{
    return tree_copy(S, tree, pool, first, n, const_cast<void *>(host), true);
}

sh_status sh_server_tree_read(sh_server *S, int32_t tree, int pool, int64_t first, int64_t n, void *host)
{
    return tree_copy(S, tree, pool, first, n, host, false);
}

sh_status sh_server_tree_destroy(sh_server *S, int32_t tree)
{
    if (!S) return SH_EINVAL;
    try {
        std::unique_lock<std::mutex> lk(S->mu);
        if (S->trees.find(tree) == S->trees.end()) return SH_EINVAL;
        wait_tree_idle(S, lk, tree);
        auto it = S->trees.find(tree);
        if (it == S->trees.end()) return SH_EINVAL;
        S->pool_alloc.release(it->second.raw_m, it->second.bytes_m);
        S->pool_alloc.release(it->second.raw_l, it->second.bytes_l);
        S->trees.erase(it);
        return SH_OK;
    } catch (...) {
        return SH_EDEVICE;
    }
}

sh_status sh_server_submit(sh_server *S, const sh_job *job, int64_t *job_id)
{
    if (!S || !job || !job_id || job->count < 0 || (job->flags & ~SH_ACCUMULATE) ||
        (job->op != SH_M2M && job->op != SH_M2L && job->op != SH_L2L))
        return SH_EINVAL;
    if (job->count > 0 && (!job->r || !job->src || !job->dst)) return SH_EINVAL;
    try {
        Job j;
        j.tree = job->tree;
        j.op = job->op;
        j.flags = job->flags;
        j.count = job->count;
        const size_t n = (size_t)job->count;
        j.footprint = job_footprint(job->count);
        struct {
            int dtype, p_m, p_l;
            int64_t n_m, n_l, off_m, off_l;
        } t;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            auto it = S->trees.find(j.tree);
            if (it == S->trees.end()) return SH_EINVAL;
            const Tree &tr = it->second;
            t = {tr.dtype, tr.p_m, tr.p_l, tr.n_m, tr.n_l, tr.off_m, tr.off_l};
        }
        const int64_t n_in = j.op == SH_L2L ? t.n_l : t.n_m;
        const int64_t n_out = j.op == SH_M2M ? t.n_m : t.n_l;
        const bool f32 = t.dtype == SH_F32;
        const int64_t elem = f32 ? 4 : 8;
        const int64_t sz_m = (int64_t)t.p_m * (t.p_m + 1) * elem, sz_l = (int64_t)t.p_l * (t.p_l + 1) * elem;
        const int64_t base_in = j.op == SH_L2L ? t.off_l / sz_l : t.off_m / sz_m;
        const int64_t base_out = j.op == SH_M2M ? t.off_m / sz_m : t.off_l / sz_l;
        // one pass: check and pack every translation; destinations unique within the job
        // (a bit per slot of the destination pool)
        j.dst_base = base_out;
        if (n > 0) j.packed = take_buf(S, n * (size_t)(3 * elem + 16));
        int64_t *ps = reinterpret_cast<int64_t *>(j.packed.p.get()), *pd = ps + n;
        char *pr = reinterpret_cast<char *>(pd + n);
        // the bitset is kept per submitting thread and left all zero: on every exit the words
        // this job marked are cleared again (a fresh zeroed bitset per job costs more than
        // the check at large pools)
        thread_local std::vector<uint64_t> mark;
        if (mark.size() < (size_t)(n_out + 63) / 64) mark.resize((size_t)(n_out + 63) / 64, 0);
        struct Unmark {
            std::vector<uint64_t> &m;
            const int64_t *dst;
            size_t marked = 0;
            ~Unmark()
            {
                for (size_t i = 0; i < marked; ++i) m[(size_t)dst[i] >> 6] = 0;
            }
        } unmark{mark, job->dst};
        for (size_t i = 0; i < n; ++i) {
            const double x = job->r[3 * i], y = job->r[3 * i + 1], z = job->r[3 * i + 2];
            if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z)) return SH_ESHIFT;
            if (j.op == SH_M2L && x == 0 && y == 0 && z == 0) return SH_ESHIFT;
            const int64_t sv = job->src[i], dv = job->dst[i];
            if (sv < 0 || sv >= n_in || dv < 0 || dv >= n_out) return SH_EINVAL;
            uint64_t &w = mark[(size_t)dv >> 6];
            const uint64_t bit = uint64_t(1) << (dv & 63);
            if (w & bit) return SH_EINVAL;
            w |= bit;
            unmark.marked = i + 1;
            if (f32) {
                float *r = reinterpret_cast<float *>(pr) + 3 * i;
                r[0] = (float)x;
                r[1] = (float)y;
                r[2] = (float)z;
            } else {
                double *r = reinterpret_cast<double *>(pr) + 3 * i;
                r[0] = x;
                r[1] = y;
                r[2] = z;
            }
            ps[i] = base_in + sv;
            pd[i] = base_out + dv;
        }
        // for M2M / L2L (one pool) no destination is also a source
        if (j.op != SH_M2L)
            for (size_t i = 0; i < n; ++i) {
                const int64_t sv = job->src[i];
                if (mark[(size_t)sv >> 6] & (uint64_t(1) << (sv & 63))) return SH_EINVAL;
            }
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->trees.find(j.tree);
        // the tree must be the one checked above (destroyed and recreated meanwhile: refuse)
        if (it == S->trees.end() || it->second.off_m != t.off_m || it->second.off_l != t.off_l ||
            it->second.dtype != t.dtype || it->second.p_m != t.p_m || it->second.p_l != t.p_l)
            return SH_EINVAL;
        if (j.footprint > S->cfg.staging_bytes) return SH_EBUSY;  // can never be admitted
        const int64_t id = S->next_job++;
        j.t_submit = now_s();
        if (S->t_first_submit < 0) S->t_first_submit = j.t_submit;
        it->second.pending++;
        if (n == 0) {  // nothing to run: complete at once
            j.done = true;
            j.t_done = j.t_submit;
            it->second.pending--;
            S->latencies.push_back(0.0);
            ++S->jobs_done;
        } else {
            S->queue.push_back(id);
            S->queue_peak = std::max<int64_t>(S->queue_peak, (int64_t)S->queue.size());
        }
        S->jobs.emplace(id, std::unique_ptr<Job>(new Job(std::move(j))));
        *job_id = id;
        S->cv_sched.notify_all();
        return SH_OK;
    } catch (const std::bad_alloc &) {
        return SH_ENOMEM;
    } catch (...) {
        return SH_EDEVICE;
    }
}

sh_status sh_server_wait(sh_server *S, int64_t job_id, double *latency_s)
{
    if (!S) return SH_EINVAL;
    try {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->jobs.find(job_id);
        if (it == S->jobs.end()) return SH_EINVAL;
        S->cv_done.wait(lk, [&] { return S->jobs.at(job_id)->done; });
        const Job &j = *S->jobs.at(job_id);
        if (latency_s) *latency_s = j.t_done - j.t_submit;
        const int st = j.status;
        S->jobs.erase(job_id);
        return (sh_status)st;
    } catch (...) {
        return SH_EDEVICE;
    }
}

sh_status sh_server_drain(sh_server *S)
{
    if (!S) return SH_EINVAL;
    try {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_done.wait(lk, [&] { return S->queue.empty() && S->inflight_total() == 0; });
        return S->failed ? SH_EDEVICE : SH_OK;
    } catch (...) {
        return SH_EDEVICE;
    }
}

sh_status sh_server_stats_get(sh_server *S, sh_server_stats *st)
{
    if (!S || !st) return SH_EINVAL;
    try {
        std::lock_guard<std::mutex> lk(S->mu);
        std::memset(st, 0, sizeof(*st));
        st->jobs_done = S->jobs_done;
        st->jobs_failed = S->failed;
        st->translations_done = S->translations_done;
        st->batches = S->batches;
        st->mean_batch_jobs = S->batches ? (double)S->batch_jobs / (double)S->batches : 0.0;
        st->queue_peak = S->queue_peak;
        st->jobs_deferred = S->jobs_deferred;
        st->staging_peak_bytes = S->stage_alloc.peak;
        st->pool_used_bytes = S->pool_alloc.used;
        st->elapsed_s = (S->t_first_submit >= 0 && S->t_last_done >= 0) ? S->t_last_done - S->t_first_submit : 0.0;
        if (!S->latencies.empty()) {
            std::vector<double> v(S->latencies);
            std::sort(v.begin(), v.end());
            auto q = [&](double f) {
                const size_t k = (size_t)std::min<double>((double)v.size() - 1, std::ceil(f * (double)v.size()) - 1);
                return v[k];
            };
            st->p50_s = q(0.50);
            st->p99_s = q(0.99);
            st->max_s = v.back();
            double sum = 0;
            for (double x : v) sum += x;
            st->mean_s = sum / (double)v.size();
        }
        return SH_OK;
    } catch (...) {
        return SH_EDEVICE;
    }
}

sh_status sh_server_stats_reset(sh_server *S)
{
    if (!S) return SH_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    S->latencies.clear();
    S->jobs_done = S->translations_done = S->batches = S->batch_jobs = S->failed = S->jobs_deferred = 0;
    S->queue_peak = (int64_t)S->queue.size();
    S->stage_alloc.peak = S->stage_alloc.used;
    S->t_first_submit = S->t_last_done = -1;
    return SH_OK;
}

}  // extern "C"
