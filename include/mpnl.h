/*
 * mpnl.h -- C ABI of the MI355X (gfx950) library for massively parallelisable
 * non-linear (MPNL) uplink MIMO detection, arXiv 2409.14355 Sec. II
 * ("Background", the MPNL paragraph).
 *
 * The paper states the method only in prose: before transmission, the
 * channel alone decides which N_p rank patterns (per-depth choices of the
 * k-th closest point) are worth searching; during transmission one candidate
 * is built from each pattern, all in parallel, and the one with the smallest
 * metric is the detection result.  This library reads
 * that as (readings listed in the design notes):
 *   a1  sorted QR of every subcarrier's channel, H[:, perm] = Q R
 *       (smallest residual column first, equal norms -> lower column index,
 *       real positive diagonal of R);
 *   a2  the N_p position vectors with the smallest channel-only score
 *       sum_d R_{l,l}^2 (p_d - 1), depth d detecting row l = N-1-d, equal
 *       scores in lexicographic order of p;
 *   a3  rotation yt = Q^H y of every received vector;
 *   a4  one successive-interference-cancellation descent per position
 *       vector: at depth d the p_d-th closest constellation point to
 *       b = yt_l - sum_{j>l} R_{l,j} s_j (distance |b - R_{l,l} c|^2, equal
 *       distances -> lower constellation index), accumulating the distances;
 *   a5  the smallest accumulated metric wins (equal metrics -> earliest
 *       position vector) and its symbols are written in original user order.
 * The model is y = H s + n; no noise variance is needed by a1-a5.
 *
 * Data conventions (all arrays row-major, complex = interleaved float32
 * (re, im), i.e. the memory layout of torch.complex64):
 *   H    (S, M, N) complex   channel of each subcarrier, rx antenna major
 *   y    (T, S, M) complex   received vector per OFDM symbol and subcarrier
 *   out  (T, S, N) int32     detected constellation index per user
 *   llr  (T, S, N, b) float  max-log LLR per bit (b = bits per symbol)
 * Constellation index i (b bits): the high b/2 bits are the binary-reflected
 * Gray label of the in-phase PAM level, the low b/2 bits that of the
 * quadrature level; levels are (2m - L + 1) * Delta, m = 0..L-1, L = 2^(b/2),
 * scaled to unit average energy (Delta = 1/sqrt(2), 1/sqrt(10), 1/sqrt(42)).
 *
 * Every pointer passed to a detection call is a DEVICE pointer on the
 * context's device; the caller owns it and must keep it alive until the work
 * enqueued on `stream` has completed.  Calls only enqueue work on `stream`
 * (a hipStream_t, NULL = the legacy default stream) and return; nothing is
 * copied back to the host.  A context is not internally locked: use one
 * context per host thread.  No exception crosses this interface.
 *
 * Inputs are not scanned for NaN/Inf: such inputs give unspecified indices
 * (always within 0..|Q|-1) and never an out-of-bounds access.
 */
#ifndef MPNL_H
#define MPNL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define MPNL_OK 0
#define MPNL_E_INVAL (-1)       /* null pointer, a size <= 0, n_paths < 1    */
#define MPNL_E_UNSUPPORTED (-2) /* N > M, N or M above the limits, bad mod    */
#define MPNL_E_NOMEM (-3)       /* the context's HBM budget would be exceeded */
#define MPNL_E_HIP (-4)         /* a HIP runtime call failed, see
                                   mpnl_last_hip_error()                     */

/* ---- limits ------------------------------------------------------------ */
#define MPNL_MAX_USERS 32       /* N (streams / single-antenna users)        */
#define MPNL_MAX_ANTENNAS 32    /* M (receive antennas)                      */
#define MPNL_MAX_PATHS 4096     /* N_p after clamping to |Q|^N               */

/* modulation = bits per symbol */
#define MPNL_QPSK 2
#define MPNL_QAM16 4
#define MPNL_QAM64 6

/* arithmetic of the path search (a4/a5); a1-a3 always run in float32 */
#define MPNL_PREC_FP32 0        /* float32 residuals and metric              */
#define MPNL_PREC_FP16 1        /* float16 R / residual operands, float32
                                   accumulation of products and the metric  */
#define MPNL_PREC_BF16 2        /* as FP16 with bfloat16 operands            */

typedef struct mpnl_ctx mpnl_ctx;
typedef struct mpnl_slot mpnl_slot;

/* ---- lifecycle ---------------------------------------------------------- */

/* flags of mpnl_create */
#define MPNL_CREATE_NO_PRUNE 1u  /* run every path to the last depth.  By
   default a path-search wavefront stops once all its paths have a partial
   metric above the metric of path 0 (computed first), since the metric only
   grows along a path; the detected symbols are the same either way. */

/* A context is one device's share of the pooled detection resources that
   Sec. II-A describes (a distributed unit serving several radio units): it
   owns the device memory of the slots and workspace it runs, under a budget.
   Create a context on HIP device `device`.  `hbm_budget_bytes` caps the
   device memory the context may hold for slot state and workspace (0 = no
   cap).  `flags`: 0 or MPNL_CREATE_NO_PRUNE.  On success *ctx receives the
   context.  Errors: MPNL_E_INVAL (ctx NULL, unknown flags), MPNL_E_HIP (bad
   device). */
int mpnl_create(mpnl_ctx **ctx, int device, size_t hbm_budget_bytes,
                unsigned flags);

/* Free a context and every slot it still owns.  Synchronises the device.
   NULL is accepted. */
int mpnl_destroy(mpnl_ctx *ctx);

/* Static English text for a return code. */
const char *mpnl_strerror(int code);

/* hipError_t value of the last failed HIP call in this context (0 if none). */
int mpnl_last_hip_error(const mpnl_ctx *ctx);

/* Select the path-search arithmetic (MPNL_PREC_*) for later detect calls.
   Errors: MPNL_E_INVAL (ctx NULL or unknown precision). */
int mpnl_set_precision(mpnl_ctx *ctx, int precision);

/* Bytes of device memory the context currently holds (slots, workspace and
   cached blocks); `in_use` receives the part not free for reuse. */
int mpnl_memory_usage(const mpnl_ctx *ctx, size_t *held, size_t *in_use);

/* ---- measurement ------------------------------------------------------------ */

/* Diagnostics for the roofline (not a detection call): time `waves`
   one-wavefront workgroups that each run `iters` rounds of eight
   independent VALU chains of one kind on `device` (0: v_fma_f32; 1: the
   point-choice mix of the path search, round / clamp / subtract / square /
   compare / select; 2: DPP row shifts), the second of two launches.
   *ms_out receives the launch time.  Together with the counters of the same
   launch (VALU wave-instructions) it gives the issue rate the compute units
   reach for that mix.  Allocates and frees a small output buffer.  Errors:
   MPNL_E_INVAL (kind outside 0..2, waves or iters < 1, null ms_out),
   MPNL_E_HIP. */
int mpnl_diag_valu_rate(int device, int kind, int waves, int iters, double *ms_out);

/* Stages reported by the kernel timers. */
#define MPNL_STAGE_SQRD 0        /* a1 sorted QR                               */
#define MPNL_STAGE_POSVEC 1      /* a2 position-vector set                     */
#define MPNL_STAGE_ROTATE 2      /* a3 yt = Q^H y                              */
#define MPNL_STAGE_PATHS 3       /* a4 + a5 path search and minimum            */
#define MPNL_STAGE_BOUND 4       /* path 0's metric per vector (pruning bound) */
#define MPNL_STAGE_PATH_WINDOW 5 /* planned batch only: from its first bound or
                                    path launch to the end of its last one, on
                                    the batch's stream; the launches may run
                                    side by side on graph branches, so this
                                    wall time can be below the PATHS + BOUND
                                    sums, which count each launch in full     */
#define MPNL_NUM_STAGES 6

/* Enable (1) or disable (0) kernel timers: while enabled every kernel launch
   of the context is bracketed by two HIP events recorded on its stream.
   Errors: MPNL_E_INVAL. */
int mpnl_profile_enable(mpnl_ctx *ctx, int enable);

/* Wait for every timed launch, then return per stage (index MPNL_STAGE_*)
   the summed kernel time in milliseconds and the number of launches, and
   forget them.  Either array may be NULL.
   Errors: MPNL_E_INVAL, MPNL_E_HIP. */
int mpnl_profile_collect(mpnl_ctx *ctx, double *total_ms, int *launches);

/* ---- one-shot detection (a1 .. a5) --------------------------------------- */

/* MPNL detection, Sec. II (the MPNL paragraph): the channel-only steps a1
   and a2 followed by the per-vector steps a3 .. a5 (readings at the top of
   this file).  Detect T*S received vectors that share one channel per
   subcarrier (a slot; Sec. III-B: 14 OFDM symbols share a slot).  n_paths
   (N_p) is clamped to min(n_paths, |Q|^N); with the clamp reached the
   result is exact maximum-likelihood detection.
   Errors: MPNL_E_INVAL, MPNL_E_UNSUPPORTED (N > M, N > 32, M > 32,
   unknown mod, clamped N_p > MPNL_MAX_PATHS), MPNL_E_NOMEM, MPNL_E_HIP. */
int mpnl_detect(mpnl_ctx *ctx, const void *H, const void *y, int S, int T,
                int M, int N, int mod, int n_paths, int32_t *out,
                void *stream);

/* ---- allocation-free one-shot detection ------------------------------------ */

/* Size of the device scratch area behind mpnl_detect_static(). */
#define MPNL_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory: code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation.  The same
   a1 .. a5 as mpnl_detect() on the same arguments, with the same result,
   but every intermediate buffer (slot state, rotated vectors, pruning
   record, path-group partials) lives in one fixed area of
   MPNL_STATIC_SCRATCH_BYTES in device memory that the library holds on each
   device it runs on until the process ends (located when the first context
   on that device is created).  The stages run one after another on
   `stream` (no second stream, no events), and the call neither allocates
   nor frees device or host memory; the context's budget does not count the
   area.  Every call on a device shares that device's area and leaves its
   contents behind: calls that may overlap on one device (other streams,
   other contexts or threads) race and give undefined results, so order them
   on one stream.  About 100 MB covers a 24-user, 3276-subcarrier slot of 14
   symbols with 256 paths; the need grows with S (M N + N N + K N) and
   with T S N.  Errors: as mpnl_detect(); MPNL_E_NOMEM when the call's
   buffers do not fit the area (nothing is enqueued); MPNL_E_HIP when the
   area could not be located on the device (see mpnl_last_hip_error()). */
int mpnl_detect_static(mpnl_ctx *ctx, const void *H, const void *y, int S,
                       int T, int M, int N, int mod, int n_paths,
                       int32_t *out, void *stream);

/* ---- slot-resident state (serving) ---------------------------------------- */

/* The part of MPNL that needs only the channel (Sec. II: the rank patterns
   to search depend on the channel alone, so they are settled before any
   data arrives): a1 (sorted QR) and a2 (position-vector set) for one slot's
   channel; Q, R, perm and the position vectors stay on the device until
   mpnl_slot_release().  The channel is only read by the enqueued work.
   On success *slot receives a handle owned by the context.
   Errors as mpnl_detect(). */
int mpnl_slot_prepare(mpnl_ctx *ctx, const void *H, int S, int M, int N,
                      int mod, int n_paths, void *stream, mpnl_slot **slot);

/* The per-transmission part of MPNL (Sec. II: the candidates are formed and
   evaluated in parallel, the best is the result): a3 .. a5 for T symbols of
   a prepared slot, y (T, S, M) -> out (T, S, N).
   May be called any number of times on any stream; work on a stream other
   than the prepare stream must be ordered after it by the caller.
   Errors: MPNL_E_INVAL (null, T <= 0), MPNL_E_NOMEM, MPNL_E_HIP. */
int mpnl_slot_detect(mpnl_ctx *ctx, mpnl_slot *slot, const void *y, int T,
                     int32_t *out, void *stream);

/* Soft input for the channel decoder behind detection (Sec. III-B decodes
   with LDPC before measuring PER).  As mpnl_slot_detect(), plus max-log
   soft output from the path list: for
   bit k of user u, llr = (min metric over paths whose symbol has bit k = 1
   minus min metric over paths with bit k = 0) / sigma2, positive favouring
   0, clipped to [-clip, clip] and set to +-clip when one hypothesis has no
   path.  Bits count from the most significant bit of the index.
   llr is (T, S, N, bits) float32.  `out` may be NULL.
   Errors: as mpnl_slot_detect(), MPNL_E_INVAL for sigma2 <= 0 or clip <= 0. */
int mpnl_slot_detect_soft(mpnl_ctx *ctx, mpnl_slot *slot, const void *y,
                          int T, float sigma2, float clip, float *llr,
                          int32_t *out, void *stream);

/* Release a slot; its memory returns to the context once the work already
   enqueued on the slot's streams has finished.  NULL is accepted. */
int mpnl_slot_release(mpnl_ctx *ctx, mpnl_slot *slot);

/* Copy a prepared slot's a1/a2 results into caller device buffers, in the
   depth order the path search uses (depth d detects row l = N-1-d):
     perm (S, N) int32      original user index detected at depth d
     w (S, N) double        R_{l,l}^2, the float64 pivot norm the position
                            set is built from (R_{l,l} = sqrt(w))
     roff (S, N, N) complex R_{l',l} at [d][d'] for d' > d (l' = N-1-d'),
                            other entries unspecified
     P (S, K, N) uint8      position vectors, K = clamped N_p
   Any pointer may be NULL to skip it.  Errors: MPNL_E_INVAL, MPNL_E_HIP. */
int mpnl_slot_export(mpnl_ctx *ctx, const mpnl_slot *slot, int32_t *perm,
                     double *w, void *roff, uint8_t *P, void *stream);

/* Shape of a prepared slot: S, M, N, mod and the clamped path count K. */
int mpnl_slot_info(const mpnl_slot *slot, int *S, int *M, int *N, int *mod,
                   int *K);

/* ---- uneven multi-cell batch ---------------------------------------------- */

typedef struct mpnl_job {
    const void *H;   /* (S, M, N) complex, device                          */
    const void *y;   /* (T, S, M) complex, device                          */
    int32_t *out;    /* (T, S, N) int32, device                             */
    int S, T, M, N;
    int mod;         /* MPNL_QPSK / MPNL_QAM16 / MPNL_QAM64                 */
    int n_paths;
} mpnl_job;

/* Pooled processing of several cells on one device (Sec. II-A: one
   distributed unit serves the traffic of many radio units, and processing
   goes where the traffic is).  Detect several independent jobs (cells) of
   different shapes with the steps of mpnl_detect(): the sorted
   QR, position sets and rotation run per job, then the path searches of all
   jobs with the same user count, modulation and paths rounded up to a
   wavefront run in one launch, each received vector's paths split into
   one-wavefront path groups whose best a second kernel reduces; a job with
   more than 256 paths runs its own path search.  Each job's result is identical
   to mpnl_detect() on it alone, in the context's precision.  Errors: as
   mpnl_detect() for any job (shape errors are found before anything is
   enqueued); MPNL_E_NOMEM / MPNL_E_HIP may leave earlier jobs done. */
int mpnl_detect_batch(mpnl_ctx *ctx, const mpnl_job *jobs, int n_jobs,
                      void *stream);

/* ---- regularised MPNL: overloaded systems (N > M) ---------------------------- */

/* MPNL on the MMSE-extended system H_x = [H; sqrt(sigma2) I_N],
   y_x = [y; 0]: the same five steps with the metric
   ||y - H s||^2 + sigma2 ||s||^2 and the MMSE detection order, which also
   works with more users than antennas (the paper's overloaded regime,
   Secs. III-IV; the paper gives no method for it, this is one reading).
   Layouts as mpnl_detect(); needs M + N <= 32 (the extended column height).
   sigma2 = 0 with N <= M is plain MPNL.  Errors: MPNL_E_INVAL (null, sizes,
   sigma2 < 0 or not finite, sigma2 = 0 with N > M), MPNL_E_UNSUPPORTED
   (M + N > 32, bad mod, paths), MPNL_E_NOMEM, MPNL_E_HIP. */
int mpnl_detect_regularized(mpnl_ctx *ctx, const void *H, const void *y, int S,
                            int T, int M, int N, int mod, int n_paths,
                            float sigma2, int32_t *out, void *stream);

/* ---- linear MMSE, the paper's comparison detector ---------------------------- */

/* Linear MMSE detection (the comparison detector of Sec. I and the baseline
   of Sec. III-B): per subcarrier x = (H^H H + sigma2 I)^-1 H^H y, each x_k
   divided by (W H)_kk (unbiased), then the closest constellation point.
   Same layouts as mpnl_detect(); no permutation (out is in user order).
   Works for N > M (overloaded) when sigma2 > 0; sigma2 = 0 is zero-forcing.
   FP32 throughout.  Errors: MPNL_E_INVAL (null, sizes <= 0, sigma2 < 0 or
   not finite, sigma2 = 0 with N > M), MPNL_E_UNSUPPORTED (N above 32, M
   above 64, bad mod), MPNL_E_HIP. */
int mpnl_mmse_detect(mpnl_ctx *ctx, const void *H, const void *y, int S, int T,
                     int M, int N, int mod, float sigma2, int32_t *out,
                     void *stream);

/* ---- planned batch: fixed shapes, one graph replay per run ------------------- */

typedef struct mpnl_batch mpnl_batch;

/* flags of mpnl_batch_create */
#define MPNL_BATCH_AUTOTUNE 1u  /* on the first run, time the candidate
                                   shapes of every path-search launch (path
                                   groups of one wavefront or of the whole
                                   vector, group- or vector-major order,
                                   times 1, 2 or 4 work items per workgroup)
                                   and keep the fastest before capturing;
                                   without it every launch runs
                                   one-wavefront groups, group major, four
                                   per workgroup                            */
#define MPNL_BATCH_SERIAL 2u    /* one pipeline phase: every path search
                                   after every channel step (a1 .. a3);
                                   without it the jobs split into two
                                   phases by path-search work and the
                                   channel steps of the second run beside
                                   the path searches of the first          */

/* Pooled processing as mpnl_detect_batch() (Sec. II-A) for a set of cells
   whose shapes repeat from slot to slot.  Plan an uneven multi-cell batch
   whose job shapes (S, T, M, N, mod, n_paths;
   the pointers are ignored) stay fixed across runs.  Allocates every job's
   slot state and workspace once from the context budget and groups the jobs
   into batched launches: sorted QR per antenna-count bucket, position sets
   per path-count bucket, one rotation launch, and one path-search launch per
   (user count, modulation, workgroup size), all of these per pipeline phase
   (MPNL_BATCH_SERIAL); the path searches run on three graph branches,
   balanced by their work.  The first
   mpnl_batch_run() captures the sequence (job-table upload + launches) into
   HIP graphs that later runs replay.  Every job needs n_paths clamped to
   <= 256.  Errors: as mpnl_detect() for any job, MPNL_E_UNSUPPORTED for more
   than 256 paths, MPNL_E_NOMEM.  The path metrics use the precision the
   context has when the batch is created; mpnl_destroy() frees batches
   still open. */
int mpnl_batch_create(mpnl_ctx *ctx, const mpnl_job *shapes, int n_jobs,
                      unsigned flags, mpnl_batch **batch);

/* Detect a planned batch on new buffers: `jobs` must have the planned shapes
   in the planned order; only H, y and out are read from it.  Enqueues one
   graph launch on `stream`.  Runs of one batch share its workspace: order
   them on one stream.  Errors: MPNL_E_INVAL (null, shape mismatch),
   MPNL_E_HIP. */
int mpnl_batch_run(mpnl_ctx *ctx, mpnl_batch *batch, const mpnl_job *jobs,
                   void *stream);

/* Launch shapes of the batch's path-search launches: n_launches receives
   their number; shapes (room for max launches, 7 ints each) receives per
   launch {N, mod, lanes per received vector (paths rounded up to 64), lanes
   per path group (64: one wavefront per group, whose best paths a second
   kernel reduces; else the whole vector), work items (vector, path group)
   per workgroup, 1 if the items are numbered path group major (all
   vectors' first group, then the second, ...) else 0, workgroups}.  Errors: MPNL_E_INVAL for a null batch or a
   negative max. */
int mpnl_batch_info(const mpnl_batch *batch, int *n_launches, int *shapes,
                    int max);

/* Free a batch (waits for its runs).  NULL is accepted. */
int mpnl_batch_destroy(mpnl_ctx *ctx, mpnl_batch *batch);

/* ---- serving: continuous batching of arriving slot jobs -------------------- */
/* The detector run as a service for the pooled processing of Sec. II-A (a
   distributed unit serving the slots of many radio units as their traffic
   arrives): slot-detection jobs arrive over time, wait for admission, are
   merged into launches and complete asynchronously.  A job larger than
   split_vectors runs as pieces of whole subcarriers (subcarriers are
   independent, so its result does not change), which lets smaller jobs run
   between the pieces of a large one.  The scheduler is host code behind an
   executor interface; the device executor runs each launch as one
   mpnl_detect_batch() on its own stream, so launches overlap on the GPU,
   and times completion with events. */

typedef struct mpnl_server mpnl_server;

typedef struct {
    size_t hbm_budget;   /* device bytes that admitted jobs may hold together,
                            counted with mpnl_job_bytes() (0: no limit)      */
    int max_batch_jobs;  /* most jobs merged into one launch (>= 1)         */
    int max_inflight;    /* most launches on the device at once (1..8)      */
    int max_queue;       /* most jobs waiting for admission; an arrival past
                            it is rejected (0: no limit)                    */
    double deadline_us;  /* latency target (arrival to completion)          */
    int drop_late;       /* 1: a job that has already waited past the
                            deadline when it would be admitted (and none of
                            whose pieces has started) is dropped             */
    int policy;          /* admission order: MPNL_SCHED_FIFO or
                            MPNL_SCHED_SLACK                                */
    int64_t split_vectors; /* a job with more received vectors (S * T) runs
                            as pieces of whole subcarriers, each of at most
                            max(T, split_vectors) vectors (0: never split)  */
    double est_fixed_us; /* service-time model of the slack policy: a piece */
    double est_us_per_gflop; /* takes est_fixed_us + est_us_per_gflop * its
                            path-search GFLOP (4 N (N - 1) + 11 N flops per
                            path and received vector)                       */
} mpnl_server_config;

/* admission orders */
#define MPNL_SCHED_FIFO 0   /* arrival order; the head of the queue blocks   */
#define MPNL_SCHED_SLACK 1  /* least slack first among the jobs that can
   still meet the deadline, slack = arrival + deadline - now - estimated time
   of the job's pieces not yet admitted; jobs that can no longer meet it
   follow in arrival order.  The first piece in this order that does not fit
   the budget waits for memory and blocks the rest.                        */

/* job outcomes */
#define MPNL_JOB_DONE 0
#define MPNL_JOB_REJECTED 1  /* queue full, or larger than the budget      */
#define MPNL_JOB_DROPPED 2   /* past the deadline before admission         */
#define MPNL_JOB_FAILED 3    /* its launch returned an error (see error)   */

typedef struct {
    int64_t id;
    int status;          /* MPNL_JOB_*                                      */
    int error;           /* MPNL_* code when FAILED, else MPNL_OK           */
    double arrival_us;   /* server clock                                    */
    double start_us;     /* launch enqueued (admission)                     */
    double done_us;      /* device completion (or decision time)            */
} mpnl_completion;

/* Device bytes a job holds while it runs (slot state, rotated vectors,
   partial results); the unit of the server's budget.  0 for an invalid
   shape. */
size_t mpnl_job_bytes(int S, int T, int M, int N, int mod, int n_paths);

/* Errors: MPNL_E_INVAL (null, max_batch_jobs < 1, max_inflight outside
   1..8, negative limits), MPNL_E_HIP, MPNL_E_NOMEM. */
int mpnl_server_create(mpnl_ctx *ctx, const mpnl_server_config *cfg,
                       mpnl_server **srv);
/* Server clock in microseconds (steady host clock, 0 at creation). */
double mpnl_server_now_us(const mpnl_server *srv);
/* Queue a job that arrived at arrival_us (server clock).  The job's
   buffers must stay valid until its completion is polled.  Shape errors are
   returned at once (nothing queued); a rejection is reported through
   mpnl_server_poll(). */
int mpnl_server_submit(mpnl_server *srv, const mpnl_job *job, int64_t id,
                       double arrival_us);
/* Advance the scheduler: retire finished launches, admit waiting jobs into
   new launches while launch slots and budget allow, and return up to max
   completions (n_done receives their number).  Never blocks. */
int mpnl_server_poll(mpnl_server *srv, mpnl_completion *done, int max,
                     int *n_done);
/* Jobs not yet completed (waiting + running). */
int mpnl_server_pending(const mpnl_server *srv);
/* Drive n_jobs Poisson arrivals (rate_hz, exponential gaps from a seeded
   64-bit generator), each a uniformly drawn entry of pool, through the
   server, polling until every job has completed; out[i] receives job i's
   completion and entry[i] (entry may be NULL) its pool index.  Several jobs
   may use one pool entry (and its output buffer).  The server must be idle
   (MPNL_E_INVAL otherwise). */
int mpnl_server_run_poisson(mpnl_server *srv, const mpnl_job *pool, int pool_n,
                            int n_jobs, double rate_hz, uint64_t seed,
                            mpnl_completion *out, int32_t *entry);
/* Waits for running launches, then frees the server.  NULL is accepted. */
int mpnl_server_destroy(mpnl_server *srv);

/* The same scheduler on a virtual clock with a modelled device, for tests of
   the serving logic without a GPU.  A launch takes launch_us +
   per_vector_us * (its S * T sum) (+ slow_extra_us if it holds job
   slow_job) and launches run one after another.  A job split by
   split_vectors becomes ceil(vectors / split_vectors) pieces of near-equal
   vectors, with bytes and gflop shared in proportion; launch number fail_launch
   (0-based, -1 for none) fails with MPNL_E_HIP.  jobs must be sorted by
   arrival; out[i] receives job i's completion; n_launches (may be NULL)
   receives the number of launches. */
typedef struct {
    int64_t id;
    double arrival_us;
    size_t bytes;
    int64_t vectors;
    double gflop;        /* path-search work (slack policy's estimate)     */
} mpnl_sim_job;

typedef struct {
    double launch_us;
    double per_vector_us;
    int fail_launch;
    int64_t slow_job;
    double slow_extra_us;
} mpnl_sim_device;

int mpnl_sched_simulate(const mpnl_server_config *cfg, const mpnl_sim_device *dev,
                        const mpnl_sim_job *jobs, int n_jobs,
                        mpnl_completion *out, int *n_launches);

#ifdef __cplusplus
}
#endif

#endif /* MPNL_H */
