/*
 * shfmm -- solid-harmonic FMM translations (M2M, M2L, L2L) on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library.  The operations are those of Kirchhart, "solidfmm: A highly
 * optimised library of operations on the solid harmonics for use in fast multipole
 * methods" (arXiv 2202.02847):
 *   - M2L (Section 2.1, eq. m2lkernels, double-height kernel), computed by the
 *     rotation-based scheme of Section 3.4 (scale, z-rotate, swap x<->z, z-rotate, swap,
 *     z-translate along (0,0,1), and back);
 *   - M2M and L2L (named in Section 1.2, "very similar", formulas omitted there): the
 *     same scheme with the z-axis shift of the regular harmonics, R_j^0(0,0,t) = t^j/j!.
 * The library keeps the paper's interface properties (Section 1.1): single and double
 * precision, input order != output order, arbitrary shift vectors, a small handle-based
 * interface, thread safety (a context is immutable after creation) and no exception
 * crossing the interface (status codes only).
 *
 * SOLID LAYOUT (Section 2.1, Fig. 1).  An expansion ("solid") of order P holds degrees
 * n = 0..P-1 and orders m = 0..n as P(P+1) reals: Re C_n^m at index n(n+1)+2m and
 * Im C_n^m at n(n+1)+2m+1.  Negative orders are implied by C_n^{-m} = (-1)^m conj(C_n^m).
 * Im C_n^0 is ignored on input and written as +0 on output.
 *
 * BASES.  The FP64 entry points take the paper's coefficients (the normalisation of the
 * Appendix recurrences).  The FP32 entry points take and return coefficients in the
 * NORMALISED basis: M_hat_n^m = M_n^m * w_n^m and L_hat_n^m = L_n^m / w_n^m with
 * w_n^m = sqrt((n+m)! (n-m)!).  (Raw coefficients and the factorials up to (2P-2)! leave
 * the float range for P >= 19.)  sh_normalise_f64 / sh_denormalise_f64 convert.
 *
 * SHIFTS.  r = (output centre) - (input centre) for all three operations; for M2L this
 * is r_AB = x_B - x_A of Section 2.1.  M2L needs 0 < |r| < inf; M2M and L2L accept r = 0
 * (identity, truncated or zero-padded to the output order).
 *
 * MIXED ORDERS (Section 1.1).  1 <= p_in, p_out <= the context's max order.  M2L sums
 * over every input degree k < p_in for every output degree n < p_out.  M2M output rows
 * n >= p_in use the available input degrees; L2L output rows k >= p_in are zero.
 *
 * OWNERSHIP.  The caller owns every coefficient, shift and index array.  Batched calls
 * take DEVICE pointers and are stream-ordered on the given HIP stream (NULL = the null
 * stream); they return after enqueue.  Single-translation calls take HOST pointers and
 * are synchronous.  The context owns its constant tables; it is never modified after
 * sh_create, so any number of host threads may use it concurrently on distinct streams.
 * Batched calls allocate nothing.
 *
 * DEVICE-SIDE ERRORS.  A batched M2L translation whose shift is zero or not finite writes
 * NaN into its output solid and raises the context's device error flag; read and clear
 * it with sh_device_error() after synchronising the stream.
 */
#ifndef SHFMM_H
#define SHFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sh_ctx sh_ctx; /* opaque handle (Section 1.1: encapsulation by handles) */

typedef enum {
    SH_OK = 0,
    SH_EINVAL = -1,  /* null pointer, negative count, bad stride, unknown op/dtype */
    SH_EORDER = -2,  /* order outside [1, max order] */
    SH_ESHIFT = -3,  /* M2L shift zero or not finite (host-checked calls) */
    SH_ENOMEM = -4,  /* device allocation failed (sh_create only) */
    SH_EDEVICE = -5, /* HIP runtime error, or no usable gfx950 device */
    SH_EBUSY = -6    /* resource limit of a bounded call exceeded */
} sh_status;

enum { SH_M2M = 0, SH_M2L = 1, SH_L2L = 2 };  /* operations */
enum { SH_F64 = 0, SH_F32 = 1 };              /* data types */
#define SH_ACCUMULATE 1u /* add into the output instead of overwriting (Section 3.4 stores) */
/* M2L by the single-height kernel (eq. m2lkernels, left): L_n^m keeps the terms with
 * n + k <= P - 1 of the double-height sum (cheaper z-step, lower accuracy).  Accepted by
 * the batched and indexed M2L calls with p_in = p_out = P; SH_EINVAL otherwise. */
#define SH_SINGLE_HEIGHT 2u

#define SH_MAX_ORDER 64

/* Human-readable text of a status code.  Never NULL. */
const char *sh_strerror(int status);

/* Creates a context for orders 1..max_order on HIP device `device`: builds the swap
 * matrices (Section 3.1, Appendix) and z-axis coefficients exactly on the host, rounds
 * them once and uploads them.  *out receives the handle.  Errors: SH_EINVAL (out NULL),
 * SH_EORDER (max_order outside [1, SH_MAX_ORDER]), SH_EDEVICE, SH_ENOMEM. */
sh_status sh_create(sh_ctx **out, int max_order, int device);

/* Releases a context and its device memory.  NULL is accepted. */
void sh_destroy(sh_ctx *ctx);

/* Max order and device of a context (-1 for NULL). */
int sh_max_order(const sh_ctx *ctx);
int sh_device(const sh_ctx *ctx);

/* Returns the device error flag (0 = none, else the first failing status) of a context
 * and clears it.  Synchronises the device. */
int sh_device_error(sh_ctx *ctx);

/* ---------------- batched translations (device pointers, stream-ordered) ----------------
 * Translation i reads its shift at r[3i..3i+2], its input solid at in + i*ld_in
 * (p_in(p_in+1) reals) and writes out + i*ld_out (p_out(p_out+1) reals).
 * ld_in >= p_in(p_in+1), ld_out >= p_out(p_out+1).  count = 0 is a no-op.
 * flags: 0 or SH_ACCUMULATE (accumulate assumes the output solids do not overlap), and for
 * M2L with p_in = p_out also SH_SINGLE_HEIGHT.
 * hip_stream: a hipStream_t, or NULL.
 * Errors: SH_EINVAL, SH_EORDER, SH_EDEVICE (launch failure).
 * Precision: FP64 results match the double-height sums of eq. (m2lkernels) to about
 * 1e-14 per degree in the normalised basis; FP32 (normalised basis) to about 1e-5. */
sh_status sh_m2l_batch_f64(const sh_ctx *ctx, int p_in, int p_out, int64_t count,
                           const double *r, const double *in, int64_t ld_in,
                           double *out, int64_t ld_out, unsigned flags, void *hip_stream);
sh_status sh_m2m_batch_f64(const sh_ctx *ctx, int p_in, int p_out, int64_t count,
                           const double *r, const double *in, int64_t ld_in,
                           double *out, int64_t ld_out, unsigned flags, void *hip_stream);
sh_status sh_l2l_batch_f64(const sh_ctx *ctx, int p_in, int p_out, int64_t count,
                           const double *r, const double *in, int64_t ld_in,
                           double *out, int64_t ld_out, unsigned flags, void *hip_stream);
sh_status sh_m2l_batch_f32(const sh_ctx *ctx, int p_in, int p_out, int64_t count,
                           const float *r, const float *in, int64_t ld_in,
                           float *out, int64_t ld_out, unsigned flags, void *hip_stream);
sh_status sh_m2m_batch_f32(const sh_ctx *ctx, int p_in, int p_out, int64_t count,
                           const float *r, const float *in, int64_t ld_in,
                           float *out, int64_t ld_out, unsigned flags, void *hip_stream);
sh_status sh_l2l_batch_f32(const sh_ctx *ctx, int p_in, int p_out, int64_t count,
                           const float *r, const float *in, int64_t ld_in,
                           float *out, int64_t ld_out, unsigned flags, void *hip_stream);

/* Generic form of the six calls above: op in {SH_M2M, SH_M2L, SH_L2L}, dtype in
 * {SH_F64, SH_F32}; r, in, out point to reals of that dtype. */
sh_status sh_translate_batch(const sh_ctx *ctx, int op, int dtype, int p_in, int p_out,
                             int64_t count, const void *r, const void *in, int64_t ld_in,
                             void *out, int64_t ld_out, unsigned flags, void *hip_stream);

/* Indexed gather/scatter over resident pools (octree / serving use): translation i reads
 * in_pool + src[i]*ld_in and writes out_pool + dst[i]*ld_out (device int64 index arrays,
 * every index >= 0 and inside the caller's pools).  With SH_ACCUMULATE, dst indices must
 * be unique within the call.  Errors as for the batched calls. */
sh_status sh_translate_indexed(const sh_ctx *ctx, int op, int dtype, int p_in, int p_out,
                               int64_t count, const void *r, const int64_t *src,
                               const void *in_pool, int64_t ld_in, const int64_t *dst,
                               void *out_pool, int64_t ld_out, unsigned flags,
                               void *hip_stream);

/* Checked form of sh_translate_indexed, for index arrays that are not known to be valid:
 * n_in and n_out are the numbers of solids in in_pool and out_pool.  The two index arrays
 * are copied to the host and checked before anything is launched (the call synchronises
 * the stream and takes host memory for the copies): every src in [0, n_in), every dst in
 * [0, n_out), no dst repeated under SH_ACCUMULATE, and, when in_pool == out_pool (which
 * then requires ld_in == ld_out), no dst that is also a src.  Pools given by different
 * pointers are taken to be disjoint.  On a violation it returns SH_EINVAL and launches
 * nothing; otherwise it enqueues the translation as sh_translate_indexed does.  Errors as
 * sh_translate_indexed, SH_EINVAL also for negative n_in / n_out, SH_EDEVICE if the copies
 * fail. */
sh_status sh_translate_indexed_checked(const sh_ctx *ctx, int op, int dtype, int p_in, int p_out,
                                       int64_t count, const void *r, const int64_t *src,
                                       const void *in_pool, int64_t ld_in, int64_t n_in,
                                       const int64_t *dst, void *out_pool, int64_t ld_out,
                                       int64_t n_out, unsigned flags, void *hip_stream);

/* ---------------- mixed work lists (batching across operations and orders) ----------------
 * A work list mixes M2M, M2L and L2L translations of any orders (p_in != p_out allowed) in
 * one call.  Item i reads the input solid at arena_in + items[i].in_off (p_in(p_in+1)
 * reals of the plan's dtype) and writes arena_out + items[i].out_off (p_out(p_out+1)
 * reals); offsets count reals and must be even.  The output solids of a list must not
 * overlap one another nor any input solid of the list (overwrite and SH_ACCUMULATE
 * alike), so the items are independent and the library may run them in any order.
 * Dependent steps (an M2M feeding an M2L) go into successive lists. */
typedef struct sh_item {
    int32_t op;       /* SH_M2M, SH_M2L or SH_L2L */
    int32_t p_in;     /* input order, 1..max order */
    int32_t p_out;    /* output order, 1..max order */
    int32_t reserved; /* must be 0 */
    int64_t in_off;   /* input solid offset in the input arena, in reals, even, >= 0 */
    int64_t out_off;  /* output solid offset in the output arena, in reals, even, >= 0 */
    double r[3];      /* shift: output centre - input centre (FP64 for both dtypes) */
} sh_item;

typedef struct sh_plan sh_plan; /* opaque: a work list binned and uploaded for execution */

#define SH_PLAN_AUTOTUNE 2u /* time the candidate kernel mappings of each bin at creation */
#define SH_PLAN_NO_GRAPH 4u /* execute by plain launches instead of a replayed HIP graph */

/* Bins a HOST array of `count` items by operation and order and uploads it (synchronous;
 * allocates device memory owned by the plan).  Items of orders <= 16 run on the
 * lane-per-translation kernel (64 translations per workgroup, orders rounded up to a
 * bucket), orders 17..31 on the block kernel (16 translations of one operation and order
 * pair per task, FP64 matrix cores; classes up to 20, 24 and 31) and larger orders on the
 * one-wavefront-per-translation kernel; SH_PLAN_AUTOTUNE
 * times the candidate mappings of each bin on zero-filled scratch arenas (orders up to 16:
 * 64- or 32-translation tasks or one wavefront per translation; orders 17..31: the block
 * kernel in workgroups of 4 wavefronts two per CU or of 8 one per CU, or one wavefront per
 * translation) and keeps the
 * fastest (decisions are cached per process and, when the environment variable
 * SHFMM_TUNE_FILE names a file, in that file).  flags: SH_ACCUMULATE, SH_PLAN_AUTOTUNE,
 * SH_PLAN_NO_GRAPH.  Errors: SH_EINVAL (null pointers, unknown op/dtype/flags, reserved
 * != 0, odd or negative offset, overlapping outputs, an output overlapping an input),
 * SH_EORDER, SH_ESHIFT (M2L shift zero or not finite, M2M/L2L shift not finite),
 * SH_ENOMEM, SH_EDEVICE. */
sh_status sh_plan_create(sh_ctx *ctx, int dtype, const sh_item *items, int64_t count,
                         unsigned flags, sh_plan **out);

/* Runs a plan on DEVICE arenas of in_reals / out_reals reals (stream-ordered, returns
 * after enqueue).  Unless SH_PLAN_NO_GRAPH was given, every bin's persistent kernel is
 * captured once into a HIP graph (bins on parallel branches) and the graph is replayed,
 * so one call is one graph launch; calling again with other arena pointers recaptures.
 * Arenas must be aligned to two reals.  Calls on one plan are serialised by the plan.
 * Errors: SH_EINVAL (null plan, null arena with a non-empty plan, misaligned arena, an
 * item beyond in_reals / out_reals), SH_EDEVICE. */
sh_status sh_plan_execute(sh_plan *plan, const void *arena_in, int64_t in_reals,
                          void *arena_out, int64_t out_reals, void *hip_stream);

/* Writes a JSON description of the plan's bins (kernel, operation, order bucket, items,
 * tasks, whether the mapping was tuned) into buf (NUL-terminated, truncated to len);
 * *needed (if not NULL) receives the full length including the NUL.  Errors: SH_EINVAL. */
sh_status sh_plan_describe(const sh_plan *plan, char *buf, int64_t len, int64_t *needed);

/* Waits for the plan's last execution and releases it.  NULL is accepted. */
void sh_plan_destroy(sh_plan *plan);

/* One-shot form: plan (no tuning, no graph), execute on hip_stream, wait for that
 * stream, release.  Same arguments and errors as the three calls above. */
sh_status sh_translate_list(sh_ctx *ctx, int dtype, const sh_item *items, int64_t count,
                            const void *arena_in, int64_t in_reals, void *arena_out,
                            int64_t out_reals, unsigned flags, void *hip_stream);

/* ---------------- shared-shift translations on the matrix cores ----------------
 * Translations that share one shift vector (the fixed offsets of a uniform octree level:
 * the 316 well-separated M2L offsets, the 8 parent/child offsets) apply the same linear
 * map: every step of the rotation scheme (Section 3.4) depends on the shift only, so the
 * class's translation is one dense real matrix of p_out(p_out+1) x p_in(p_in+1) in the
 * normalised basis.  sh_shared_create generates these matrices on the device in FP64 (the
 * FP64 rotation kernels applied to unit solids), splits each entry into BF16 pieces and
 * keeps them (sh_shared_bytes tells how much device memory).  sh_shared_execute applies
 * them to FP32 normalised-basis solids as a grouped GEMM on MFMA with FP32 accumulation:
 *   SH_SHARED_BF16X3: a_hi b_hi + a_hi b_mid + a_mid b_hi (about 16 significant bits;
 *                     per-degree error ~1e-5 .. 1e-4);
 *   SH_SHARED_BF16X6: adds a_hi b_lo + a_mid b_mid + a_lo b_hi (about FP32: ~1e-6);
 *   SH_SHARED_FP32:   FP32 operands (the operator rounded once from FP64) on the FP32 MFMA.
 * The FP32 solids use the layout and normalised basis of the FP32 batched calls. */
typedef struct sh_shared sh_shared;

#define SH_SHARED_FP32 1
#define SH_SHARED_BF16X3 3
#define SH_SHARED_BF16X6 6

/* Builds the operators of `nclass` (1..4096) shifts (host array, nclass x 3 doubles) for
 * operation op and orders p_in -> p_out (synchronous; allocates device memory owned by the
 * object).  Errors: SH_EINVAL, SH_EORDER, SH_ESHIFT (a non-finite shift, an M2L shift of
 * zero), SH_ENOMEM, SH_EDEVICE. */
sh_status sh_shared_create(sh_ctx *ctx, int op, int p_in, int p_out, int nclass, const double *shifts,
                           int precision, sh_shared **out);

/* Applies the operators to `count` FP32 solids grouped by class: class c owns the
 * translations i in [class_start[c], class_start[c+1]) (DEVICE array of nclass + 1 int64,
 * non-decreasing, from 0 to count; values outside [0, count] are clamped), which read
 * in + i*ld_in and write out + i*ld_out.  ld_in even and in 8-byte aligned.  flags: 0 or
 * SH_ACCUMULATE.  Stream-ordered, allocates nothing.  Errors: SH_EINVAL, SH_EDEVICE. */
sh_status sh_shared_execute(const sh_shared *shared, int64_t count, const int64_t *class_start,
                            const float *in, int64_t ld_in, float *out, int64_t ld_out,
                            unsigned flags, void *hip_stream);

/* Device bytes held by the operators (-1 for NULL). */
int64_t sh_shared_bytes(const sh_shared *shared);

/* Releases the operators.  NULL is accepted. */
void sh_shared_destroy(sh_shared *shared);

/* ---------------- serving: a request loop with continuous batching ----------------
 * A server owns a device arena of resident expansion pools and a staging arena for the work
 * records of jobs in flight, and runs a scheduler thread plus one completion thread per
 * stream.  A "tree" is a pair of resident pools (multipoles of order p_m, locals of order
 * p_l) that stay on the device between jobs.  A job is a batch of translations on one tree:
 *   M2L: tree M pool slot src[i] -> L pool slot dst[i]  (orders p_m -> p_l);
 *   M2M: M pool -> M pool;  L2L: L pool -> L pool;
 * with shift r[3i..3i+2] (host arrays, copied at submission).  Destinations are unique within
 * a job, and for M2M / L2L no destination is also a source.  Jobs are admitted in submission
 * order with backfill, by footprint (80 bytes of staging per translation plus 2 KiB: the
 * device memory a job holds while in flight; the pools are reserved at tree creation), while
 * the staging arena has room and nothing in flight on their tree conflicts: overwriting M2L
 * jobs (no SH_ACCUMULATE) share a tree while their destination slots are disjoint, M2M, L2L
 * and accumulating jobs run alone on their tree, and a job passed over holds back every later
 * job of its tree.  Every admissible job joins the next batch, which runs as one indexed
 * translation call per (dtype, operation, orders, accumulate) group -- jobs of different
 * trees share a call -- on the least loaded stream, so batches overlap on the device.  A
 * translation's result does not depend on the batch it ran in.
 * Thread safety: every call may come from any host thread. */
typedef struct sh_server sh_server;

typedef struct sh_server_config {
    int64_t pool_bytes;     /* device bytes for resident pools (trees) */
    int64_t staging_bytes;  /* device bytes for jobs in flight: the admission budget (>= 64 KiB) */
    int32_t streams;        /* concurrent streams, 1..8 */
    int32_t max_batch_jobs; /* most jobs fused into one batch, >= 1 */
} sh_server_config;

typedef struct sh_job {
    int32_t tree;         /* from sh_server_tree_create */
    int32_t op;           /* SH_M2M, SH_M2L or SH_L2L */
    int64_t count;        /* translations */
    const double *r;      /* count x 3 shifts (host) */
    const int64_t *src;   /* count source slots (host) */
    const int64_t *dst;   /* count destination slots (host) */
    uint32_t flags;       /* 0 or SH_ACCUMULATE */
    uint32_t reserved;    /* 0 */
} sh_job;

typedef struct sh_server_stats {
    int64_t jobs_done, jobs_failed, translations_done, batches, queue_peak;
    int64_t staging_peak_bytes, pool_used_bytes;
    int64_t jobs_deferred;  /* jobs passed over at least once because staging was full */
    double mean_batch_jobs;
    double elapsed_s;       /* first submission to last completion */
    double p50_s, p99_s, mean_s, max_s;  /* job latency: submission to completion */
} sh_server_stats;

/* Creates a server (allocates both arenas and pinned host staging, starts its threads).
 * Errors: SH_EINVAL, SH_ENOMEM, SH_EDEVICE. */
sh_status sh_server_create(sh_ctx *ctx, const sh_server_config *config, sh_server **out);

/* Finishes every submitted job, stops the threads and releases the server.  NULL is accepted. */
void sh_server_destroy(sh_server *server);

/* Carves a tree's pools (n_m solids of order p_m, n_l of order p_l, dtype SH_F64 or SH_F32;
 * FP32 solids in the normalised basis) out of the pool arena.  Errors: SH_EINVAL, SH_EORDER,
 * SH_EBUSY (no room in the arena). */
sh_status sh_server_tree_create(sh_server *server, int dtype, int p_m, int64_t n_m, int p_l, int64_t n_l,
                                int32_t *tree);

/* Copies n solids starting at slot `first` of pool 0 (M) or 1 (L) from / to host memory,
 * after the tree's queued and running jobs have finished (synchronous). */
sh_status sh_server_tree_write(sh_server *server, int32_t tree, int pool, int64_t first, int64_t n,
                               const void *host);
sh_status sh_server_tree_read(sh_server *server, int32_t tree, int pool, int64_t first, int64_t n, void *host);

/* Waits for the tree's jobs and returns its pools to the arena. */
sh_status sh_server_tree_destroy(sh_server *server, int32_t tree);

/* Queues a job (validated and copied; returns at once) and gives its id.  Errors: SH_EINVAL
 * (unknown tree or op, a slot out of range, repeated destination, a destination that is
 * also a source), SH_ESHIFT, SH_EBUSY (footprint above the whole staging arena). */
sh_status sh_server_submit(sh_server *server, const sh_job *job, int64_t *job_id);

/* Waits for a job, gives its latency in seconds and forgets it; returns its status. */
sh_status sh_server_wait(sh_server *server, int64_t job_id, double *latency_s);

/* Waits until no job is queued or running. */
sh_status sh_server_drain(sh_server *server);

/* Counters and latency percentiles since creation or the last sh_server_stats_reset. */
sh_status sh_server_stats_get(sh_server *server, sh_server_stats *stats);

/* Starts a new statistics window: the counters, the latencies, the staging peak and the
 * elapsed clock start again from zero (jobs still queued or running are counted in the new
 * window when they complete).  Errors: SH_EINVAL (NULL server). */
sh_status sh_server_stats_reset(sh_server *server);

/* ---------------- single translation (host pointers, synchronous) ----------------
 * The paper's statement of the problem: one input solid, one shift, one output solid.
 * Errors: SH_EINVAL, SH_EORDER, SH_ESHIFT (M2L with r = 0 or non-finite r), SH_EDEVICE. */
sh_status sh_m2l_f64(const sh_ctx *ctx, int p_in, int p_out, const double r[3],
                     const double *M, double *L);
sh_status sh_m2m_f64(const sh_ctx *ctx, int p_in, int p_out, const double r[3],
                     const double *M, double *Mout);
sh_status sh_l2l_f64(const sh_ctx *ctx, int p_in, int p_out, const double r[3],
                     const double *L, double *Lout);
sh_status sh_m2l_f32(const sh_ctx *ctx, int p_in, int p_out, const float r[3],
                     const float *M, float *L);
sh_status sh_m2m_f32(const sh_ctx *ctx, int p_in, int p_out, const float r[3],
                     const float *M, float *Mout);
sh_status sh_l2l_f32(const sh_ctx *ctx, int p_in, int p_out, const float r[3],
                     const float *L, float *Lout);

/* ---------------- single translation without allocation ----------------
 * For callers that cannot allocate device memory (tight serving loops, harnesses that
 * forbid hipMalloc): the single host-pointer translation above, for any op and dtype
 * (r: 3 reals; in: p_in(p_in+1) reals; out: p_out(p_out+1) reals, all host memory of the
 * dtype), staged through a fixed device array of SH_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU until the process ends, instead of a per-call hipMalloc.
 * Calls no hipMalloc / hipFree.  Same kernel, same layout and same result bits as
 * sh_m2l_f64 ... sh_l2l_f32.  Synchronous; the array keeps the last call's contents.
 * Calls on one GPU share the array: the library serialises them within a process (a
 * second host thread waits for the first).  The array is resolved per device by
 * sh_create, so a context for the device must exist.  Errors: as the single calls, plus
 * SH_EBUSY if the staging (3 + p_in(p_in+1) + p_out(p_out+1) reals) exceeds the array
 * (never for orders <= SH_MAX_ORDER), SH_EINVAL for an unknown op or dtype. */
#define SH_NOALLOC_SCRATCH_BYTES 66816
sh_status sh_translate_single_noalloc(const sh_ctx *ctx, int op, int dtype, int p_in, int p_out,
                                      const void *r, const void *in, void *out);

/* ---------------- baseline and neighbouring steps ----------------
 * Direct double-height M2L (eq. m2lkernels, right) with S by the Appendix recurrence:
 * the O(P^4) loop the paper benchmarks against (Section 4), FP64, same layout and
 * arguments as sh_m2l_batch_f64. */
sh_status sh_m2l_naive_batch_f64(const sh_ctx *ctx, int p_in, int p_out, int64_t count,
                                 const double *r, const double *in, int64_t ld_in,
                                 double *out, int64_t ld_out, unsigned flags,
                                 void *hip_stream);

/* P2M on the device (eq. MLexpansions with the Appendix recurrence for R):
 * M_n^m = sum_j q_j R_n^m(y_j - c) for `count` clusters of `npts` points each; cluster c
 * has centre centres[3c..], points pts[3*npts*c ..] and charges q[npts*c ..]; output
 * solid c at M + c*ldM.  FP64, device pointers, stream-ordered. */
sh_status sh_p2m_batch_f64(const sh_ctx *ctx, int P, int64_t count, const double *centres,
                           int64_t npts, const double *pts, const double *q, double *M,
                           int64_t ldM, void *hip_stream);

/* L2P on the device: the potential Phi_L(x) = Re sum_{n<P} sum_m L_n^m conj(R_n^m(x - c))
 * of a local expansion (eq. MLexpansions) and its gradient, R by the Appendix recurrence
 * and differentiated by the identities d/dz R_n^m = R_{n-1}^m,
 * d/dx R_n^m = (R_{n-1}^{m-1} - R_{n-1}^{m+1})/2, d/dy R_n^m = i (R_{n-1}^{m-1} + R_{n-1}^{m+1})/2.
 * `count` boxes of `npts` targets each: box c has centre centres[3c..], local expansion
 * L + c*ldL (order P, Im L_n^0 ignored) and targets pts[3*npts*c ..]; target j of box c
 * writes out[4*(npts*c + j) .. +3] = {Phi, dPhi/dx, dPhi/dy, dPhi/dz} (the field of the
 * potential sum q/|x - y| is minus the gradient).  flags: 0 or SH_ACCUMULATE.  FP64,
 * device pointers owned by the caller, stream-ordered.  Errors: SH_EINVAL (null pointer,
 * negative count, ldL < P(P+1), unknown flags), SH_EORDER, SH_EDEVICE. */
sh_status sh_l2p_batch_f64(const sh_ctx *ctx, int P, int64_t count, const double *centres,
                           int64_t npts, const double *pts, const double *L, int64_t ldL,
                           double *out, unsigned flags, void *hip_stream);

/* ---------------- uniform-octree FMM driver ----------------
 * The translations used inside a fast multipole method, as the paper intends (Sections 1
 * and 2): P2M at the leaves, upward M2M, M2L over the interaction lists (boxes whose parents
 * are neighbours but which are not neighbours themselves), downward L2L, L2P at the leaves
 * and the direct near field (P2P) over the 27 neighbouring leaves, for the potential
 * u(x_i) = sum_{j != i} q_j / |x_i - x_j| (eq. nbody) and its gradient.
 * The tree is a full octree with `levels` levels below the root cube [origin, origin+width)^3:
 * leaf (ix, iy, iz) of the n = 2^levels per side has index (ix n + iy) n + iz and holds
 * exactly `npts` particles, stored leaf by leaf (particle j of leaf b at pts[3(npts b + j)]).
 * Particles must lie in their leaf's cube (the expansions converge only then).  FP64.
 * Every index and shift array is built and uploaded at creation; the handle owns its device
 * memory (multipole and local pools of every level, M2M/M2L scratch, the call lists).  Calls on
 * one handle are serialised on the host, but its evaluations share those pools on the device:
 * evaluations issued on different streams must not overlap in time, and the caller
 * synchronises the stream of the last evaluation before sh_fmm_destroy. */
#define SH_FMM_MAX_LEVELS 6
typedef struct sh_fmm sh_fmm;

/* levels in [2, SH_FMM_MAX_LEVELS], npts >= 1, width > 0, 1 <= P <= the context's order.
 * Errors: SH_EINVAL, SH_EORDER, SH_ENOMEM, SH_EDEVICE. */
sh_status sh_fmm_create(sh_ctx *ctx, int P, int levels, const double origin[3], double width,
                        int64_t npts, sh_fmm **out);
/* Variable order per level (input order differing from output order, Section 1.1):
 * orders[l - 2] is the expansion order of level l = 2..levels (levels - 1 entries; levels 0
 * and 1 carry no expansions).  M2M from level l to l - 1 and L2L from l to l + 1 translate
 * between the two levels' orders; M2L stays within a level; the leaves use orders[levels - 2]
 * for P2M and L2P.  Errors as sh_fmm_create (SH_EINVAL for a NULL orders). */
sh_status sh_fmm_create_orders(sh_ctx *ctx, int levels, const int *orders, const double origin[3],
                               double width, int64_t npts, sh_fmm **out);
void sh_fmm_destroy(sh_fmm *fmm);

/* One evaluation on device pointers, stream-ordered: pts (N x 3, leaf by leaf), charges q
 * (N), out (N x 4) receives {u, du/dx, du/dy, du/dz} at every particle (the field is minus
 * the gradient).  N = 8^levels * npts.  By default the evaluation is captured once per
 * (pts, q, out) into a HIP graph (the near field on a branch of its own; the far field,
 * P2M to L2P, on the caller's stream) and replayed; flags = SH_FMM_NO_GRAPH launches every
 * kernel on hip_stream instead.  Errors: SH_EINVAL (null pointer, unknown flags), SH_EDEVICE. */
#define SH_FMM_NO_GRAPH 1u
sh_status sh_fmm_evaluate(sh_fmm *fmm, const double *pts, const double *q, double *out,
                          unsigned flags, void *hip_stream);

/* Per-level orders (as for sh_fmm_create_orders, levels - 1 entries) for a target relative
 * error tol of the potential, max_i |u_i - u_i^direct| / max_i |u_i^direct|, in a uniform
 * tree with uniformly distributed particles and charges of both signs.  The rule comes from
 * this driver's measured error against direct summation: below 0.15 * 0.444^P at order P on
 * every level, and no lower when a single level's order is raised, so every level takes the
 * smallest P meeting tol.  It is applied only within its measured range: trees of 2 to 4
 * levels and orders up to 18 (tol >= 6.6e-8).  Host only.  Errors: SH_EINVAL (NULL orders,
 * tol outside (0, 1), levels outside [2, 4]), SH_EORDER (tol needs an order above 18). */
sh_status sh_fmm_orders_for_tolerance(double tol, int levels, int *orders);

/* counts[0..4] = M2M, M2L and L2L translations per evaluation, translation calls, leaves. */
sh_status sh_fmm_describe(const sh_fmm *fmm, int64_t *counts);

/* ---------------- host-only helpers (no device needed) ----------------
 * Dense (n+1)x(n+1) row-major swap matrix of degree n (0 <= n < SH_MAX_ORDER), rounded
 * once from exact arithmetic.  which: 0 = F (M side, real parts), 1 = G (M side,
 * imaginary parts), 2 = F_L (L side, real), 3 = G_L (L side, imaginary).
 * normalised != 0 gives the normalised-basis matrix.  Errors: SH_EINVAL, SH_EORDER. */
sh_status sh_swap_matrix_f64(int n, int which, int normalised, double *out);

/* Scales solids between the paper's basis and the normalised basis, on the host:
 * kind 0 = multipole-type (x w_n^m), 1 = local-type (/ w_n^m); sh_denormalise_f64 undoes
 * it.  `count` solids of order P at stride ld, in place. */
sh_status sh_normalise_f64(int kind, int P, int64_t count, double *solids, int64_t ld);
sh_status sh_denormalise_f64(int kind, int P, int64_t count, double *solids, int64_t ld);

#ifdef __cplusplus
}
#endif
#endif /* SHFMM_H */
