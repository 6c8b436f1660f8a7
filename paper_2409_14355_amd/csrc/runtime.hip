// Host runtime of the MPNL detection library: contexts, validation, a
// budgeted device-memory pool, slot state and kernel sequencing.  Implements
// the C ABI declared in include/mpnl.h.
#include "mpnl.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "device_common.h"
#include "kernels.h"
#include "runtime_internal.h"

namespace {

struct Block {
    void *ptr = nullptr;
    size_t size = 0;
    bool free = false;
    hipStream_t last_stream = nullptr;
    hipEvent_t ev = nullptr;  // recorded on last_stream when released
    bool ev_pending = false;
    bool ev_deferred = false;  // released without an event: recorded when another stream asks for it
};

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

// Device scratch of the allocation-free detection (mpnl_detect_static): the
// slot state, rotated vectors, pruning record and path-group partials of one
// call.  Every device that loads the library holds its own copy until the
// process ends.  In host code `scratch` only names the symbol; its device
// address on each device comes from hipGetSymbolAddress (static_scratch_of).
static __device__ __align__(256) unsigned char scratch[MPNL_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
bool g_scratch_done[kMaxDevices];

// Device address of `scratch` on `device`, looked up once per device with
// that device current (the caller has made it current).
hipError_t static_scratch_of(int device, void **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void *p = nullptr;
        g_scratch_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[device] = g_scratch_err[device] == hipSuccess ? p : nullptr;
        g_scratch_done[device] = true;
    }
    *ptr = g_scratch_ptr[device];
    return g_scratch_err[device];
}

}  // namespace

struct mpnl_slot {
    mpnl::SlotDev sd{};
    int block = -1;
    hipStream_t stream = nullptr;  // stream of the last work that used the slot
};

struct mpnl_ctx {
    int device = 0;
    size_t budget = 0;
    size_t held = 0;
    int last_hip = 0;
    int precision = MPNL_PREC_FP32;
    bool prune = true;  // stop path-search waves that can no longer win
    void *scratch = nullptr;       // device address of the static scratch on this device
    int scratch_err = 0;           // hipError_t of its lookup at creation
    int cus = 0;            // compute units and LDS bytes per compute unit of the device
    size_t lds_per_cu = 0;  // (0: unknown; the position sets then keep everything in LDS)
    // second stream of one-shot detection: the rotation and the pruning
    // bounds run there while the position set runs on the caller's stream
    hipStream_t aux = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    std::vector<Block> blocks;
    std::vector<mpnl_slot *> slots;
    std::vector<mpnl_batch *> batches;
    // ring of pinned staging buffers for batch job tables: a buffer is
    // rewritten only once the upload that last read it has run
    struct Staging {
        void *ptr = nullptr;
        size_t size = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    Staging staging[4];
    int staging_next = 0;
    // kernel timers
    bool prof = false;
    struct Timed {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> spare_events;
};

namespace {

void plan_free(mpnl_ctx *ctx, mpnl_batch *p);

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev_) != hipSuccess)
            prev_ = -1;
        ok_ = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev_ >= 0)
            (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

  private:
    int prev_ = -1;
    bool ok_ = false;
};

int hip_fail(mpnl_ctx *ctx, hipError_t e)
{
    ctx->last_hip = (int)e;
    return e == hipErrorOutOfMemory ? MPNL_E_NOMEM : MPNL_E_HIP;
}

// A block released with a deferred event gets its event when another stream
// first asks for it; the event then covers all the work enqueued on the
// releasing stream so far (a superset of the work that used the block), and
// the block counts as busy until that has finished.
void record_deferred(Block &b)
{
    if (!b.ev_deferred)
        return;
    b.ev_deferred = false;
    b.ev_pending = hipEventRecord(b.ev, b.last_stream) == hipSuccess;
}

bool block_idle(Block &b, hipStream_t st)
{
    if (!b.free)
        return false;
    if (b.last_stream == st)
        return true;
    record_deferred(b);
    if (!b.ev_pending)
        return true;
    return hipEventQuery(b.ev) == hipSuccess;
}

// Device memory from the context pool.  A released block is reused at once on
// the stream that released it (stream order protects it) and on other
// streams only after the work enqueued before its release has finished.
int pool_alloc(mpnl_ctx *ctx, size_t bytes, hipStream_t st, int *out_block)
{
    bytes = align_up(std::max<size_t>(bytes, 1));
    int best = -1;
    for (int i = 0; i < (int)ctx->blocks.size(); ++i) {
        Block &b = ctx->blocks[i];
        if (b.size >= bytes && b.size <= 2 * bytes + (1u << 20) && block_idle(b, st)) {
            if (best < 0 || b.size < ctx->blocks[best].size)
                best = i;
        }
    }
    if (best >= 0) {
        ctx->blocks[best].free = false;
        ctx->blocks[best].ev_deferred = false;
        *out_block = best;
        return MPNL_OK;
    }
    if (ctx->budget && ctx->held + bytes > ctx->budget) {
        // give back idle cached blocks until the request fits
        for (int i = 0; i < (int)ctx->blocks.size() && ctx->held + bytes > ctx->budget; ++i) {
            Block &b = ctx->blocks[i];
            if (b.ptr && b.free)
                record_deferred(b);
            if (b.ptr && b.free && (!b.ev_pending || hipEventQuery(b.ev) == hipSuccess)) {
                (void)hipFree(b.ptr);
                ctx->held -= b.size;
                b.ptr = nullptr;
                b.size = 0;
            }
        }
        if (ctx->held + bytes > ctx->budget)
            return MPNL_E_NOMEM;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess)
        return hip_fail(ctx, e);
    int slot = -1;
    for (int i = 0; i < (int)ctx->blocks.size(); ++i)
        if (ctx->blocks[i].ptr == nullptr && ctx->blocks[i].size == 0) {
            slot = i;
            break;
        }
    if (slot < 0) {
        ctx->blocks.emplace_back();
        slot = (int)ctx->blocks.size() - 1;
        e = hipEventCreateWithFlags(&ctx->blocks[slot].ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipFree(p);
            ctx->blocks.pop_back();
            return hip_fail(ctx, e);
        }
    }
    Block &b = ctx->blocks[slot];
    b.ptr = p;
    b.size = bytes;
    b.free = false;
    b.ev_pending = false;
    b.ev_deferred = false;
    ctx->held += bytes;
    *out_block = slot;
    return MPNL_OK;
}

// Return a block to the pool after the work enqueued on `st` so far.  With
// `defer`, no event is recorded now (an event on the stream costs a few
// microseconds of device time): the block is reused at once on `st`, and its
// event is recorded only when another stream asks for it, so `st` must still
// exist then (callers defer only on the null stream).
void pool_release(mpnl_ctx *ctx, int blk, hipStream_t st, bool defer = false)
{
    if (blk < 0 || blk >= (int)ctx->blocks.size())
        return;
    Block &b = ctx->blocks[blk];
    b.free = true;
    b.last_stream = st;
    b.ev_deferred = defer;
    b.ev_pending = defer ? false : hipEventRecord(b.ev, st) == hipSuccess;
}

hipEvent_t take_event(mpnl_ctx *ctx)
{
    if (!ctx->spare_events.empty()) {
        hipEvent_t e = ctx->spare_events.back();
        ctx->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Bracket one launch with timing events when the timers are on.
class StageTimer {
  public:
    StageTimer(mpnl_ctx *ctx, int stage, hipStream_t st) : ctx_(ctx), stage_(stage), st_(st)
    {
        if (!ctx->prof)
            return;
        a_ = take_event(ctx);
        b_ = take_event(ctx);
        if (a_ && b_)
            (void)hipEventRecord(a_, st_);
    }
    ~StageTimer()
    {
        if (!ctx_->prof || !a_ || !b_)
            return;
        (void)hipEventRecord(b_, st_);
        ctx_->timed.push_back({stage_, a_, b_});
    }

  private:
    mpnl_ctx *ctx_;
    int stage_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

long long num_vectors_sat(int nq, int N)
{
    long long v = 1;
    for (int i = 0; i < N; ++i) {
        v *= nq;
        if (v > (1LL << 40))
            return 1LL << 40;
    }
    return v;
}

int validate_shape(int S, int M, int N, int mod, int n_paths)
{
    if (S <= 0 || M <= 0 || N <= 0 || n_paths < 1)
        return MPNL_E_INVAL;
    if (mod != MPNL_QPSK && mod != MPNL_QAM16 && mod != MPNL_QAM64)
        return MPNL_E_UNSUPPORTED;
    if (N > M || N > MPNL_MAX_USERS || M > MPNL_MAX_ANTENNAS)
        return MPNL_E_UNSUPPORTED;
    const long long K = std::min<long long>(n_paths, num_vectors_sat(1 << mod, N));
    if (K > MPNL_MAX_PATHS)
        return MPNL_E_UNSUPPORTED;
    if ((long long)S * M * N > INT_MAX / 2)
        return MPNL_E_UNSUPPORTED;
    return MPNL_OK;
}

// Packed reduced-precision copy of the lattice-scaled R for a precision.
const uint32_t *rq_of(const mpnl::SlotDev &sd, int precision)
{
    return precision == MPNL_PREC_FP16 ? sd.rlat_h : precision == MPNL_PREC_BF16 ? sd.rlat_b : nullptr;
}

// Offsets of the slot arrays inside one pool block.
struct SlotLayout {
    size_t Qd, roff, rlat, rlat_h, rlat_b, diag, wd, permd, P, order, rec, rec16, total;
};

SlotLayout slot_layout(int S, int M, int N, int K, int NP, bool rec_global, bool rec16 = false)
{
    SlotLayout L{};
    size_t o = 0;
    auto put = [&](size_t &field, size_t bytes) {
        field = o;
        o += align_up(bytes);
    };
    const size_t sNN = (size_t)S * N * N;
    put(L.Qd, (size_t)S * M * N * sizeof(float2));
    put(L.roff, sNN * sizeof(float2));
    put(L.rlat, sNN * sizeof(float2));
    put(L.rlat_h, 2 * sNN * sizeof(uint32_t));
    put(L.rlat_b, 2 * sNN * sizeof(uint32_t));
    put(L.diag, (size_t)S * N * sizeof(float4));
    put(L.wd, (size_t)S * N * sizeof(double));
    put(L.permd, (size_t)S * N * sizeof(int32_t));
    put(L.P, (size_t)S * K * NP);
    put(L.order, K <= 256 ? (size_t)S * K * sizeof(uint16_t) : 0);
    put(L.rec, rec_global ? (size_t)S * N * K * sizeof(uint32_t) : 0);
    put(L.rec16, rec16 ? (size_t)S * N * 256 * sizeof(uint16_t) : 0);
    L.total = o;
    return L;
}

}  // namespace

namespace mpnl {

int validate_job_shape(const mpnl_job &j)
{
    if (j.T <= 0)
        return MPNL_E_INVAL;
    const int rc = validate_shape(j.S, j.M, j.N, j.mod, j.n_paths);
    if (rc != MPNL_OK)
        return rc;
    if ((long long)j.S * j.T > INT_MAX / 4)
        return MPNL_E_UNSUPPORTED;
    return MPNL_OK;
}

int context_device(const mpnl_ctx *ctx)
{
    return ctx->device;
}

size_t job_device_bytes(const mpnl_job &j)
{
    if (validate_job_shape(j) != MPNL_OK)
        return 0;
    const int K = (int)std::min<long long>(j.n_paths, num_vectors_sat(1 << j.mod, j.N));
    const int NP = (j.N + 3) / 4 * 4;
    // upper bound: a 256-path set may keep its back pointers in global memory
    const SlotLayout L = slot_layout(j.S, j.M, j.N, K, NP, !posvec_rec_fits_lds(j.N, K), K > 128 && K <= 256);
    SlotDev sd{};
    sd.S = j.S;
    sd.N = j.N;
    sd.K = K;
    return align_up(L.total) + align_up((size_t)j.T * j.S * j.N * sizeof(float2)) +
           align_up(bound_record_bytes(j.S, j.T, j.N)) + align_up(path_partial_bytes(sd, j.T)) +
           align_up(sizeof(JobDev));
}

}  // namespace mpnl

namespace {

int prepare_impl(mpnl_ctx *ctx, const void *H, int S, int M, int N, int mod, int n_paths,
                 hipStream_t st, mpnl_slot **out, bool run_posvec = true)
{
    const int K = (int)std::min<long long>(n_paths, num_vectors_sat(1 << mod, N));
    const int NP = (N + 3) / 4 * 4;
    const bool rec_global = !mpnl::posvec_rec_fits_lds(N, K);
    const bool rec16 = mpnl::posvec_reg_rec_global(S, N, K, ctx->cus, ctx->lds_per_cu);
    const SlotLayout L = slot_layout(S, M, N, K, NP, rec_global, rec16);
    int blk = -1;
    int rc = pool_alloc(ctx, L.total, st, &blk);
    if (rc != MPNL_OK)
        return rc;
    mpnl_slot *slot = new (std::nothrow) mpnl_slot();
    if (!slot) {
        pool_release(ctx, blk, st);
        return MPNL_E_NOMEM;
    }
    char *base = (char *)ctx->blocks[blk].ptr;
    mpnl::SlotDev &sd = slot->sd;
    sd.S = S;
    sd.M = M;
    sd.N = N;
    sd.bits = mod;
    sd.K = K;
    sd.NP = NP;
    sd.Qd = (float2 *)(base + L.Qd);
    sd.roff = (float2 *)(base + L.roff);
    sd.rlat = (float2 *)(base + L.rlat);
    sd.rlat_h = (uint32_t *)(base + L.rlat_h);
    sd.rlat_b = (uint32_t *)(base + L.rlat_b);
    sd.diag = (float4 *)(base + L.diag);
    sd.wd = (double *)(base + L.wd);
    sd.permd = (int32_t *)(base + L.permd);
    sd.P = (uint8_t *)(base + L.P);
    sd.order = K <= 256 ? (uint16_t *)(base + L.order) : nullptr;
    sd.rec = rec_global ? (uint32_t *)(base + L.rec) : nullptr;
    sd.rec16 = rec16 ? (uint16_t *)(base + L.rec16) : nullptr;
    slot->block = blk;
    slot->stream = st;
    hipError_t e;
    {
        StageTimer tm(ctx, MPNL_STAGE_SQRD, st);
        e = mpnl::launch_sqrd((const float2 *)H, sd, st);
    }
    if (e == hipSuccess && run_posvec) {
        StageTimer tm(ctx, MPNL_STAGE_POSVEC, st);
        e = mpnl::launch_posvec(sd, st);
    }
    if (e != hipSuccess) {
        pool_release(ctx, blk, st);
        delete slot;
        return hip_fail(ctx, e);
    }
    ctx->slots.push_back(slot);
    *out = slot;
    return MPNL_OK;
}

void release_impl(mpnl_ctx *ctx, mpnl_slot *slot, bool defer = false)
{
    pool_release(ctx, slot->block, slot->stream, defer);
    ctx->slots.erase(std::remove(ctx->slots.begin(), ctx->slots.end(), slot), ctx->slots.end());
    delete slot;
}

bool owns(const mpnl_ctx *ctx, const mpnl_slot *slot)
{
    return std::find(ctx->slots.begin(), ctx->slots.end(), slot) != ctx->slots.end();
}

int detect_impl(mpnl_ctx *ctx, mpnl_slot *slot, const void *y, int T, int32_t *out, hipStream_t st,
                bool soft, float sigma2, float clip, float *llr)
{
    const mpnl::SlotDev &sd = slot->sd;
    if ((long long)sd.S * T > INT_MAX / 2)
        return MPNL_E_UNSUPPORTED;
    const size_t yt_bytes = align_up((size_t)T * sd.S * sd.N * sizeof(float2));
    const size_t part_bytes = align_up(soft ? 0 : mpnl::path_partial_bytes(sd, T));
    const size_t bound_bytes = (!soft && ctx->prune) ? align_up(mpnl::bound_record_bytes(sd.S, T, sd.N)) : 0;
    int blk = -1;
    int rc = pool_alloc(ctx, yt_bytes + part_bytes + bound_bytes, st, &blk);
    if (rc != MPNL_OK)
        return rc;
    char *base = (char *)ctx->blocks[blk].ptr;
    float2 *yt = (float2 *)base;
    float *part = part_bytes ? (float *)(base + yt_bytes) : nullptr;
    float *bound = bound_bytes ? (float *)(base + yt_bytes + part_bytes) : nullptr;
    hipError_t e;
    {
        StageTimer tm(ctx, MPNL_STAGE_ROTATE, st);
        e = mpnl::launch_rotate(sd, (const float2 *)y, T, yt, st);
    }
    if (e == hipSuccess && bound) {
        StageTimer tm(ctx, MPNL_STAGE_BOUND, st);
        e = mpnl::launch_path_bound(sd, yt, T, ctx->precision, bound, st);
    }
    if (e == hipSuccess) {
        StageTimer tm(ctx, MPNL_STAGE_PATHS, st);
        if (soft)
            e = mpnl::launch_path_search_soft(sd, yt, T, sigma2, clip, llr, out, st);
        else
            e = mpnl::launch_path_search(sd, yt, T, out, ctx->precision, part, bound, st);
    }
    pool_release(ctx, blk, st, st == nullptr);  // per-call workspace (see oneshot_impl)
    slot->stream = st;
    if (e != hipSuccess)
        return hip_fail(ctx, e);
    return MPNL_OK;
}

// One-shot a1..a5 with the independent stages overlapped: after the sorted
// QR, the rotation and the pruning bounds run on the context's second
// stream while the position set runs on `st`; the path search waits for
// both.  Everything is ordered after earlier work on `st`, and later work on
// `st` is ordered after it.
int oneshot_impl(mpnl_ctx *ctx, const void *H, const void *y, int S, int T, int M, int N, int mod, int n_paths,
                 int32_t *out, hipStream_t st)
{
    hipError_t e = hipSuccess;
    if (!ctx->aux) {
        e = hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming);
        if (e != hipSuccess)
            return hip_fail(ctx, e);
    }
    mpnl_slot *slot = nullptr;
    int rc = prepare_impl(ctx, H, S, M, N, mod, n_paths, st, &slot, false);
    if (rc != MPNL_OK)
        return rc;
    const mpnl::SlotDev &sd = slot->sd;
    const size_t yt_bytes = align_up((size_t)T * S * N * sizeof(float2));
    const size_t part_bytes = align_up(mpnl::path_partial_bytes(sd, T));
    const size_t bound_bytes = ctx->prune ? align_up(mpnl::bound_record_bytes(S, T, N)) : 0;
    int blk = -1;
    rc = pool_alloc(ctx, yt_bytes + part_bytes + bound_bytes, st, &blk);
    if (rc != MPNL_OK) {
        release_impl(ctx, slot);
        return rc;
    }
    char *base = (char *)ctx->blocks[blk].ptr;
    float2 *yt = (float2 *)base;
    float *part = part_bytes ? (float *)(base + yt_bytes) : nullptr;
    float *bound = bound_bytes ? (float *)(base + yt_bytes + part_bytes) : nullptr;
    e = hipEventRecord(ctx->fork_ev, st);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0);
    if (e == hipSuccess) {
        StageTimer tm(ctx, MPNL_STAGE_ROTATE, ctx->aux);
        e = mpnl::launch_rotate(sd, (const float2 *)y, T, yt, ctx->aux);
    }
    if (e == hipSuccess && bound) {
        StageTimer tm(ctx, MPNL_STAGE_BOUND, ctx->aux);
        e = mpnl::launch_path_bound(sd, yt, T, ctx->precision, bound, ctx->aux);
    }
    if (e == hipSuccess)
        e = hipEventRecord(ctx->join_ev, ctx->aux);
    if (e == hipSuccess) {
        StageTimer tm(ctx, MPNL_STAGE_POSVEC, st);
        e = mpnl::launch_posvec(sd, st);
    }
    if (e == hipSuccess)
        e = hipStreamWaitEvent(st, ctx->join_ev, 0);
    if (e == hipSuccess) {
        StageTimer tm(ctx, MPNL_STAGE_PATHS, st);
        e = mpnl::launch_path_search(sd, yt, T, out, ctx->precision, part, bound, st);
    }
    // per-call workspace, reused at once by the next call on this stream; the
    // event is deferred only on the null stream (a user stream may be
    // destroyed before another stream asks for the block)
    pool_release(ctx, blk, st, st == nullptr);
    slot->stream = st;
    release_impl(ctx, slot, st == nullptr);
    return e == hipSuccess ? MPNL_OK : hip_fail(ctx, e);
}

// One-shot a1..a5 with every intermediate buffer in the static scratch at
// `base` (cap bytes): the stages run one after another on `st`; nothing is
// allocated, no event is recorded and no second stream is used.
int static_impl(mpnl_ctx *ctx, char *base, size_t cap, const void *H, const void *y, int S, int T, int M, int N,
                int mod, int n_paths, int32_t *out, hipStream_t st)
{
    if ((long long)S * T > INT_MAX / 2)
        return MPNL_E_UNSUPPORTED;
    const int K = (int)std::min<long long>(n_paths, num_vectors_sat(1 << mod, N));
    const int NP = (N + 3) / 4 * 4;
    const bool rec_global = !mpnl::posvec_rec_fits_lds(N, K);
    // back pointers of a 256-path set stay in LDS (rec16 off): the same set,
    // less scratch
    const SlotLayout L = slot_layout(S, M, N, K, NP, rec_global, false);
    mpnl::SlotDev sd{};
    sd.S = S;
    sd.M = M;
    sd.N = N;
    sd.bits = mod;
    sd.K = K;
    sd.NP = NP;
    const size_t yt_bytes = align_up((size_t)T * S * N * sizeof(float2));
    const size_t part_bytes = align_up(mpnl::path_partial_bytes(sd, T));
    const size_t bound_bytes = ctx->prune ? align_up(mpnl::bound_record_bytes(S, T, N)) : 0;
    if (L.total + yt_bytes + part_bytes + bound_bytes > cap)
        return MPNL_E_NOMEM;
    sd.Qd = (float2 *)(base + L.Qd);
    sd.roff = (float2 *)(base + L.roff);
    sd.rlat = (float2 *)(base + L.rlat);
    sd.rlat_h = (uint32_t *)(base + L.rlat_h);
    sd.rlat_b = (uint32_t *)(base + L.rlat_b);
    sd.diag = (float4 *)(base + L.diag);
    sd.wd = (double *)(base + L.wd);
    sd.permd = (int32_t *)(base + L.permd);
    sd.P = (uint8_t *)(base + L.P);
    sd.order = K <= 256 ? (uint16_t *)(base + L.order) : nullptr;
    sd.rec = rec_global ? (uint32_t *)(base + L.rec) : nullptr;
    sd.rec16 = nullptr;
    char *work = base + L.total;
    float2 *yt = (float2 *)work;
    float *part = part_bytes ? (float *)(work + yt_bytes) : nullptr;
    float *bound = bound_bytes ? (float *)(work + yt_bytes + part_bytes) : nullptr;
    hipError_t e = mpnl::launch_sqrd((const float2 *)H, sd, st);
    if (e == hipSuccess)
        e = mpnl::launch_posvec(sd, st);
    if (e == hipSuccess)
        e = mpnl::launch_rotate(sd, (const float2 *)y, T, yt, st);
    if (e == hipSuccess && bound)
        e = mpnl::launch_path_bound(sd, yt, T, ctx->precision, bound, st);
    if (e == hipSuccess)
        e = mpnl::launch_path_search(sd, yt, T, out, ctx->precision, part, bound, st);
    return e == hipSuccess ? MPNL_OK : hip_fail(ctx, e);
}

}  // namespace

extern "C" {

int mpnl_create(mpnl_ctx **ctx, int device, size_t hbm_budget_bytes, unsigned flags)
{
    if (!ctx || (flags & ~MPNL_CREATE_NO_PRUNE))
        return MPNL_E_INVAL;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return MPNL_E_HIP;
    mpnl_ctx *c = new (std::nothrow) mpnl_ctx();
    if (!c)
        return MPNL_E_NOMEM;
    c->device = device;
    c->budget = hbm_budget_bytes;
    c->prune = (flags & MPNL_CREATE_NO_PRUNE) == 0;
    int cus = 0, lds = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) == hipSuccess &&
        cus > 0 && lds > 0) {
        c->cus = cus;
        c->lds_per_cu = (size_t)lds;
    }
    {
        // the static scratch of mpnl_detect_static: located once per device,
        // with that device current; a failure is reported by that call only
        DeviceGuard g(device);
        c->scratch_err = g.ok() ? (int)static_scratch_of(device, &c->scratch) : (int)hipErrorInvalidDevice;
    }
    *ctx = c;
    return MPNL_OK;
}

int mpnl_destroy(mpnl_ctx *ctx)
{
    if (!ctx)
        return MPNL_OK;
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    for (mpnl_slot *s : ctx->slots)
        delete s;
    for (mpnl_batch *p : ctx->batches)
        plan_free(ctx, p);
    for (Block &b : ctx->blocks) {
        if (b.ptr)
            (void)hipFree(b.ptr);
        if (b.ev)
            (void)hipEventDestroy(b.ev);
    }
    for (auto &sg : ctx->staging) {
        if (sg.ptr)
            (void)hipHostFree(sg.ptr);
        if (sg.ev)
            (void)hipEventDestroy(sg.ev);
    }
    if (ctx->aux)
        (void)hipStreamDestroy(ctx->aux);
    if (ctx->fork_ev)
        (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev)
        (void)hipEventDestroy(ctx->join_ev);
    for (auto &t : ctx->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (hipEvent_t e : ctx->spare_events)
        (void)hipEventDestroy(e);
    delete ctx;
    return MPNL_OK;
}

const char *mpnl_strerror(int code)
{
    switch (code) {
    case MPNL_OK: return "success";
    case MPNL_E_INVAL: return "invalid argument (null pointer, non-positive size or n_paths < 1)";
    case MPNL_E_UNSUPPORTED: return "unsupported shape or modulation (N > M, N or M > 32, unknown modulation, too many paths)";
    case MPNL_E_NOMEM: return "device memory budget exceeded";
    case MPNL_E_HIP: return "HIP runtime error (see mpnl_last_hip_error)";
    default: return "unknown error code";
    }
}

int mpnl_last_hip_error(const mpnl_ctx *ctx) { return ctx ? ctx->last_hip : 0; }

int mpnl_set_precision(mpnl_ctx *ctx, int precision)
{
    if (!ctx || precision < MPNL_PREC_FP32 || precision > MPNL_PREC_BF16)
        return MPNL_E_INVAL;
    ctx->precision = precision;
    return MPNL_OK;
}

int mpnl_profile_enable(mpnl_ctx *ctx, int enable)
{
    if (!ctx)
        return MPNL_E_INVAL;
    ctx->prof = enable != 0;
    return MPNL_OK;
}

int mpnl_profile_collect(mpnl_ctx *ctx, double *total_ms, int *launches)
{
    if (!ctx)
        return MPNL_E_INVAL;
    DeviceGuard g(ctx->device);
    double ms[MPNL_NUM_STAGES] = {};
    int cnt[MPNL_NUM_STAGES] = {};
    hipError_t err = hipSuccess;
    for (auto &t : ctx->timed) {
        float x = 0.f;
        hipError_t e = hipEventSynchronize(t.b);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&x, t.a, t.b);
        if (e != hipSuccess)
            err = e;
        else if (t.stage >= 0 && t.stage < MPNL_NUM_STAGES) {
            ms[t.stage] += x;
            cnt[t.stage] += 1;
        }
        ctx->spare_events.push_back(t.a);
        ctx->spare_events.push_back(t.b);
    }
    ctx->timed.clear();
    for (int i = 0; i < MPNL_NUM_STAGES; ++i) {
        if (total_ms)
            total_ms[i] = ms[i];
        if (launches)
            launches[i] = cnt[i];
    }
    if (err != hipSuccess)
        return hip_fail(ctx, err);
    return MPNL_OK;
}

int mpnl_memory_usage(const mpnl_ctx *ctx, size_t *held, size_t *in_use)
{
    if (!ctx)
        return MPNL_E_INVAL;
    size_t used = 0;
    for (const Block &b : ctx->blocks)
        if (b.ptr && !b.free)
            used += b.size;
    if (held)
        *held = ctx->held;
    if (in_use)
        *in_use = used;
    return MPNL_OK;
}

int mpnl_slot_prepare(mpnl_ctx *ctx, const void *H, int S, int M, int N, int mod, int n_paths,
                      void *stream, mpnl_slot **slot)
{
    if (!ctx || !H || !slot)
        return MPNL_E_INVAL;
    *slot = nullptr;
    int rc = validate_shape(S, M, N, mod, n_paths);
    if (rc != MPNL_OK)
        return rc;
    DeviceGuard g(ctx->device);
    if (!g.ok())
        return hip_fail(ctx, hipErrorInvalidDevice);
    return prepare_impl(ctx, H, S, M, N, mod, n_paths, (hipStream_t)stream, slot);
}

int mpnl_slot_detect(mpnl_ctx *ctx, mpnl_slot *slot, const void *y, int T, int32_t *out, void *stream)
{
    if (!ctx || !slot || !y || !out || T <= 0 || !owns(ctx, slot))
        return MPNL_E_INVAL;
    DeviceGuard g(ctx->device);
    if (!g.ok())
        return hip_fail(ctx, hipErrorInvalidDevice);
    return detect_impl(ctx, slot, y, T, out, (hipStream_t)stream, false, 0.f, 0.f, nullptr);
}

int mpnl_slot_detect_soft(mpnl_ctx *ctx, mpnl_slot *slot, const void *y, int T, float sigma2,
                          float clip, float *llr, int32_t *out, void *stream)
{
    if (!ctx || !slot || !y || !llr || T <= 0 || !owns(ctx, slot) || !(sigma2 > 0.f) ||
        !(clip > 0.f))
        return MPNL_E_INVAL;
    DeviceGuard g(ctx->device);
    if (!g.ok())
        return hip_fail(ctx, hipErrorInvalidDevice);
    return detect_impl(ctx, slot, y, T, out, (hipStream_t)stream, true, sigma2, clip, llr);
}

int mpnl_slot_release(mpnl_ctx *ctx, mpnl_slot *slot)
{
    if (!slot)
        return MPNL_OK;
    if (!ctx || !owns(ctx, slot))
        return MPNL_E_INVAL;
    DeviceGuard g(ctx->device);
    release_impl(ctx, slot);
    return MPNL_OK;
}

int mpnl_slot_info(const mpnl_slot *slot, int *S, int *M, int *N, int *mod, int *K)
{
    if (!slot)
        return MPNL_E_INVAL;
    if (S) *S = slot->sd.S;
    if (M) *M = slot->sd.M;
    if (N) *N = slot->sd.N;
    if (mod) *mod = slot->sd.bits;
    if (K) *K = slot->sd.K;
    return MPNL_OK;
}

int mpnl_slot_export(mpnl_ctx *ctx, const mpnl_slot *slot, int32_t *perm, double *w, void *roff,
                     uint8_t *P, void *stream)
{
    if (!ctx || !slot || !owns(ctx, slot))
        return MPNL_E_INVAL;
    DeviceGuard g(ctx->device);
    const mpnl::SlotDev &sd = slot->sd;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    const size_t SN = (size_t)sd.S * sd.N;
    if (perm && e == hipSuccess)
        e = hipMemcpyAsync(perm, sd.permd, SN * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
    if (w && e == hipSuccess)
        e = hipMemcpyAsync(w, sd.wd, SN * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (roff && e == hipSuccess)
        e = hipMemcpyAsync(roff, sd.roff, SN * sd.N * sizeof(float2), hipMemcpyDeviceToDevice, st);
    if (P && e == hipSuccess)
        e = hipMemcpy2DAsync(P, sd.N, sd.P, sd.NP, sd.N, (size_t)sd.S * sd.K, hipMemcpyDeviceToDevice,
                             st);
    if (e != hipSuccess)
        return hip_fail(ctx, e);
    return MPNL_OK;
}

int mpnl_detect(mpnl_ctx *ctx, const void *H, const void *y, int S, int T, int M, int N, int mod,
                int n_paths, int32_t *out, void *stream)
{
    if (!ctx || !H || !y || !out || T <= 0)
        return MPNL_E_INVAL;
    int rc = validate_shape(S, M, N, mod, n_paths);
    if (rc != MPNL_OK)
        return rc;
    DeviceGuard g(ctx->device);
    if (!g.ok())
        return hip_fail(ctx, hipErrorInvalidDevice);
    return oneshot_impl(ctx, H, y, S, T, M, N, mod, n_paths, out, (hipStream_t)stream);
}

int mpnl_detect_static(mpnl_ctx *ctx, const void *H, const void *y, int S, int T, int M, int N, int mod,
                       int n_paths, int32_t *out, void *stream)
{
    if (!ctx || !H || !y || !out || T <= 0)
        return MPNL_E_INVAL;
    int rc = validate_shape(S, M, N, mod, n_paths);
    if (rc != MPNL_OK)
        return rc;
    if (ctx->scratch_err != (int)hipSuccess || ctx->scratch == nullptr) {
        ctx->last_hip = ctx->scratch_err ? ctx->scratch_err : (int)hipErrorInvalidSymbol;
        return MPNL_E_HIP;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok())
        return hip_fail(ctx, hipErrorInvalidDevice);
    return static_impl(ctx, (char *)ctx->scratch, MPNL_STATIC_SCRATCH_BYTES, H, y, S, T, M, N, mod, n_paths, out,
                       (hipStream_t)stream);
}

int mpnl_detect_regularized(mpnl_ctx *ctx, const void *H, const void *y, int S, int T, int M, int N, int mod,
                            int n_paths, float sigma2, int32_t *out, void *stream)
{
    if (!ctx || !H || !y || !out || T <= 0 || M <= 0 || N <= 0 || S <= 0)
        return MPNL_E_INVAL;
    if (!(sigma2 >= 0.f) || !std::isfinite(sigma2) || (N > M && sigma2 == 0.f))
        return MPNL_E_INVAL;
    if (M + N > MPNL_MAX_ANTENNAS)
        return MPNL_E_UNSUPPORTED;
    int rc = validate_shape(S, M + N, N, mod, n_paths);
    if (rc != MPNL_OK)
        return rc;
    if ((long long)T * S * (M + N) > INT_MAX / 2)
        return MPNL_E_UNSUPPORTED;
    DeviceGuard g(ctx->device);
    if (!g.ok())
        return hip_fail(ctx, hipErrorInvalidDevice);
    hipStream_t st = (hipStream_t)stream;
    const size_t hb = align_up((size_t)S * (M + N) * N * sizeof(float2));
    const size_t yb = align_up((size_t)T * S * (M + N) * sizeof(float2));
    int blk = -1;
    rc = pool_alloc(ctx, hb + yb, st, &blk);
    if (rc != MPNL_OK)
        return rc;
    float2 *Hx = (float2 *)ctx->blocks[blk].ptr;
    float2 *yx = (float2 *)((char *)ctx->blocks[blk].ptr + hb);
    hipError_t e = mpnl::launch_extend((const float2 *)H, (const float2 *)y, S, T, M, N, std::sqrt(sigma2), Hx, yx,
                                       st);
    if (e != hipSuccess) {
        pool_release(ctx, blk, st);
        return hip_fail(ctx, e);
    }
    mpnl_slot *slot = nullptr;
    rc = prepare_impl(ctx, Hx, S, M + N, N, mod, n_paths, st, &slot);
    if (rc == MPNL_OK) {
        rc = detect_impl(ctx, slot, yx, T, out, st, false, 0.f, 0.f, nullptr);
        release_impl(ctx, slot);
    }
    pool_release(ctx, blk, st);
    return rc;
}

int mpnl_mmse_detect(mpnl_ctx *ctx, const void *H, const void *y, int S, int T, int M, int N, int mod,
                     float sigma2, int32_t *out, void *stream)
{
    if (!ctx || !H || !y || !out || S <= 0 || T <= 0 || M <= 0 || N <= 0)
        return MPNL_E_INVAL;
    if (!(sigma2 >= 0.f) || !std::isfinite(sigma2) || (N > M && sigma2 == 0.f))
        return MPNL_E_INVAL;
    if (mod != MPNL_QPSK && mod != MPNL_QAM16 && mod != MPNL_QAM64)
        return MPNL_E_UNSUPPORTED;
    if (N > MPNL_MAX_USERS || M > 2 * MPNL_MAX_ANTENNAS)
        return MPNL_E_UNSUPPORTED;
    if ((long long)S * T > INT_MAX / 4 || (long long)T * S * M > INT_MAX / 2)
        return MPNL_E_UNSUPPORTED;
    DeviceGuard g(ctx->device);
    if (!g.ok())
        return hip_fail(ctx, hipErrorInvalidDevice);
    const hipError_t e = mpnl::launch_mmse((const float2 *)H, (const float2 *)y, S, T, M, N, mod, sigma2, out,
                                           (hipStream_t)stream);
    return e == hipSuccess ? MPNL_OK : hip_fail(ctx, e);
}

// ---------------------------------------------------------------------------
// Planned batch
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

enum LaunchKind { L_SQRD = 0, L_POSVEC = 1, L_ROTATE = 2, L_PATHS = 3 };

struct PlanLaunch {
    int kind;
    int param;        // a1: MMAX; a2: E; a4: user count N
    int bits;         // a4
    int threads;      // a4: lanes per received vector (paths rounded up to 64)
    int nmax;         // a2: largest N (LDS size)
    int groups;       // a4: path groups per vector (threads / 64, or 1: the whole vector) (tuned)
    int vpw;          // a4: work items (vector, path group) per workgroup (tuned)
    int gmajor;       // a4: 1 = work items numbered path group major (tuned)
    int branch;       // a4: graph branch of the launch (plan_branches)
    int phase;        // pipeline phase of the launch (plan_layout)
    double gflop;     // a4: path-search work of the launch (algorithmic)
    int bound_items;  // a4: items of the pruning-bound launch
    int items;
    size_t off;       // byte offset of the job table in a table buffer
    std::vector<int> jobs;
};

constexpr int kGraphCopies = 2;
// branches of the planned batch's path-search launches
constexpr int kMaxBranches = 4;  // side streams: kMaxBranches - 1
constexpr int kPlanBranches = 3;
static_assert(kPlanBranches < kMaxBranches, "a phased plan needs a side stream per branch");
// pipeline phases of a planned batch (plan_layout), unless MPNL_BATCH_SERIAL.
// 40 cells FP16: one phase 148.5, two 152.6, three 146.5 M vectors/s (FP32:
// 137.6, 139.4, 136.8)
constexpr int kMaxPhases = 4;
constexpr int kPlanPhases = 2;

// Byte offsets of one job's arrays in a batch's block.
struct PlanJobOffsets {
    SlotLayout lay;
    size_t base, yt, bound, part;
};

}  // namespace

struct mpnl_batch {
    std::vector<mpnl_job> shapes;
    std::vector<mpnl::SlotDev> sd;
    std::vector<float2 *> yt;
    std::vector<float *> bound;  // per job pruning bounds, or null
    std::vector<float *> part;   // per job path-group partial records, or null (one group)
    std::vector<PlanJobOffsets> off;
    std::vector<PlanLaunch> launches;
    int block = -1;
    size_t table_bytes = 0;
    void *pinned[kGraphCopies] = {nullptr, nullptr};
    char *dev_table[kGraphCopies] = {nullptr, nullptr};
    hipGraphExec_t exec[kGraphCopies] = {nullptr, nullptr};
    hipEvent_t done[kGraphCopies] = {nullptr, nullptr};
    bool used[kGraphCopies] = {false, false};
    int next = 0;
    bool captured = false;
    bool autotune = false;
    bool tuned = false;
    int precision = MPNL_PREC_FP32;
    bool prune = true;
    hipStream_t cap = nullptr;
    // path-search launches split over kPlanBranches branches of the graph
    // (see plan_enqueue): the other branches' streams, the fork event and
    // their join events
    int branches = 1;
    int phases = 1;
    hipStream_t side[kMaxBranches - 1] = {};
    hipEvent_t fork_ev[kMaxPhases] = {};
    hipEvent_t join_ev[kMaxBranches - 1] = {};
};

namespace {

// Device-memory layout and launch groups of a batch of job shapes (every
// job with n_paths clamped to <= 256): per job its slot state, rotated
// vectors, pruning record and path-group partials, then the job tables.
// With phases > 1 the jobs are split into pipeline phases (whole path-search
// groups, largest algorithmic work first, each to the phase with the least
// work so far), each phase with its own a1 .. a3 launches, so that the
// channel steps of one phase can run beside the path searches of the one
// before.  Fills p->launches (phase by phase, stage by stage),
// p->table_bytes and the per-job offsets; returns the bytes before the
// tables (each table copy takes p->table_bytes more).
size_t plan_layout(mpnl_batch *p, bool prune, int phases = 1)
{
    const int n_jobs = (int)p->shapes.size();
    p->off.assign(n_jobs, PlanJobOffsets{});
    size_t total = 0;
    auto clamped_paths = [](const mpnl_job &j) {
        return (int)std::min<long long>(j.n_paths, num_vectors_sat(1 << j.mod, j.N));
    };
    auto path_gflop = [&](const mpnl_job &j) {
        const int K = clamped_paths(j);
        return (double)j.S * j.T * K * (4.0 * j.N * (j.N - 1) + 11.0 * j.N) * 1e-9;
    };
    for (int i = 0; i < n_jobs; ++i) {
        const mpnl_job &j = p->shapes[i];
        const int K = clamped_paths(j);
        PlanJobOffsets &o = p->off[i];
        o.lay = slot_layout(j.S, j.M, j.N, K, (j.N + 3) / 4 * 4, false);
        o.base = total;
        total += o.lay.total;
        o.yt = total;
        total += align_up((size_t)j.T * j.S * j.N * sizeof(float2));
        o.bound = total;
        if (prune)
            total += align_up(mpnl::bound_record_bytes(j.S, j.T, j.N));
        o.part = total;
        total += align_up(mpnl::multi_partial_bytes(j.S, j.T, j.N, K));
    }
    // phase of every job: that of its path-search group (N, constellation,
    // lanes), groups spread over the phases by work
    phases = std::max(1, std::min(phases, kMaxPhases));
    std::vector<int> job_phase(n_jobs, 0);
    if (phases > 1) {
        struct PathKey {
            int N, mod, lanes;
            double gflop;
            int phase;
        };
        std::vector<PathKey> keys;
        std::vector<int> job_key(n_jobs);
        for (int i = 0; i < n_jobs; ++i) {
            const mpnl_job &j = p->shapes[i];
            const int lanes = (clamped_paths(j) + 63) / 64 * 64;
            int k = 0;
            while (k < (int)keys.size() && !(keys[k].N == j.N && keys[k].mod == j.mod && keys[k].lanes == lanes))
                ++k;
            if (k == (int)keys.size())
                keys.push_back(PathKey{j.N, j.mod, lanes, 0.0, 0});
            keys[k].gflop += path_gflop(j);
            job_key[i] = k;
        }
        std::vector<int> by_work(keys.size());
        for (size_t k = 0; k < keys.size(); ++k)
            by_work[k] = (int)k;
        std::stable_sort(by_work.begin(), by_work.end(),
                         [&](int a, int b) { return keys[a].gflop > keys[b].gflop; });
        std::vector<double> load(phases, 0.0);
        for (int k : by_work) {
            const int ph = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            keys[k].phase = ph;
            load[ph] += keys[k].gflop;
        }
        for (int i = 0; i < n_jobs; ++i)
            job_phase[i] = keys[job_key[i]].phase;
    }
    p->phases = phases;
    // launch groups
    p->launches.clear();
    auto group = [&](int phase, int kind, int param, int bits, int threads) -> PlanLaunch & {
        for (PlanLaunch &L : p->launches)
            if (L.phase == phase && L.kind == kind && L.param == param && L.bits == bits && L.threads == threads)
                return L;
        PlanLaunch L{};
        L.phase = phase;
        L.kind = kind;
        L.param = param;
        L.bits = bits;
        L.threads = threads;
        L.groups = kind == L_PATHS ? threads / 64 : 1;  // one-wavefront path groups, group major,
        L.vpw = kind == L_PATHS ? 4 : 1;                 // four a workgroup, unless tuned
        L.gmajor = 1;
        p->launches.push_back(L);
        return p->launches.back();
    };
    for (int phase = 0; phase < phases; ++phase)
        for (int stage = 0; stage < 4; ++stage)
            for (int i = 0; i < n_jobs; ++i) {
                if (job_phase[i] != phase)
                    continue;
                const mpnl_job &j = p->shapes[i];
                const int K = clamped_paths(j);
                PlanLaunch *L;
                if (stage == L_SQRD) {
                    L = &group(phase, L_SQRD, (j.M + 3) / 4 * 4, 0, 64);
                    L->items += (j.S + 1) / 2;
                } else if (stage == L_POSVEC) {
                    L = &group(phase, L_POSVEC, K <= 64 ? 1 : K <= 128 ? 2 : 4, 0, 64);
                    L->items += j.S;
                    L->nmax = std::max(L->nmax, j.N);
                } else if (stage == L_ROTATE) {
                    L = &group(phase, L_ROTATE, 0, 0, 64);
                    L->items += j.S;
                    L->nmax = std::max(L->nmax, j.N);
                } else {
                    L = &group(phase, L_PATHS, j.N, j.mod, (K + 63) / 64 * 64);
                    L->items += j.S * j.T;
                    L->bound_items += (j.S * j.T + 63) / 64;
                    L->gflop += path_gflop(j);
                }
                L->jobs.push_back(i);
            }
    p->table_bytes = 0;
    for (PlanLaunch &L : p->launches) {
        L.off = p->table_bytes;
        const size_t entry = L.kind == L_PATHS ? sizeof(mpnl::JobDev) : sizeof(mpnl::dev::StageJob);
        p->table_bytes += align_up(L.jobs.size() * entry);
    }
    return total;
}

// Point every job's slot state and workspace into the block at dbase (laid
// out by plan_layout).
void plan_bind(mpnl_batch *p, char *dbase)
{
    p->sd.clear();
    p->yt.clear();
    p->bound.clear();
    p->part.clear();
    for (size_t i = 0; i < p->shapes.size(); ++i) {
        const mpnl_job &j = p->shapes[i];
        const PlanJobOffsets &o = p->off[i];
        const SlotLayout &L = o.lay;
        char *b = dbase + o.base;
        mpnl::SlotDev sd{};
        sd.S = j.S;
        sd.M = j.M;
        sd.N = j.N;
        sd.bits = j.mod;
        sd.K = (int)std::min<long long>(j.n_paths, num_vectors_sat(1 << j.mod, j.N));
        sd.NP = (j.N + 3) / 4 * 4;
        sd.Qd = (float2 *)(b + L.Qd);
        sd.roff = (float2 *)(b + L.roff);
        sd.rlat = (float2 *)(b + L.rlat);
        sd.rlat_h = (uint32_t *)(b + L.rlat_h);
        sd.rlat_b = (uint32_t *)(b + L.rlat_b);
        sd.diag = (float4 *)(b + L.diag);
        sd.wd = (double *)(b + L.wd);
        sd.permd = (int32_t *)(b + L.permd);
        sd.P = (uint8_t *)(b + L.P);
        sd.order = (uint16_t *)(b + L.order);
        sd.rec = nullptr;
        sd.rec16 = nullptr;
        p->sd.push_back(sd);
        p->yt.push_back((float2 *)(dbase + o.yt));
        p->bound.push_back(p->prune ? (float *)(dbase + o.bound) : nullptr);
        p->part.push_back(mpnl::multi_partial_bytes(j.S, j.T, j.N, sd.K) ? (float *)(dbase + o.part) : nullptr);
    }
}

// Spread the path-search launches of each phase over `branches` graph
// branches: largest algorithmic work first, each to the branch with the
// least work so far.
void plan_branches(mpnl_batch *p, int branches)
{
    for (int phase = 0; phase < p->phases; ++phase) {
        std::vector<PlanLaunch *> paths;
        for (PlanLaunch &L : p->launches)
            if (L.kind == L_PATHS && L.phase == phase)
                paths.push_back(&L);
        std::stable_sort(paths.begin(), paths.end(),
                         [](const PlanLaunch *a, const PlanLaunch *b) { return a->gflop > b->gflop; });
        std::vector<double> load(std::max(branches, 1), 0.0);
        for (PlanLaunch *L : paths) {
            const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            L->branch = b;
            load[b] += L->gflop;
        }
    }
}

// Fill table copy b for the given job pointers (pointers of the shapes are
// ignored).
void plan_fill(mpnl_batch *p, int b, const mpnl_job *jobs)
{
    char *host = (char *)p->pinned[b];
    for (const PlanLaunch &L : p->launches) {
        if (L.kind == L_PATHS) {
            mpnl::JobDev *jd = (mpnl::JobDev *)(host + L.off);
            int acc = 0, bacc = 0;
            for (size_t u = 0; u < L.jobs.size(); ++u) {
                const int i = L.jobs[u];
                const mpnl::SlotDev &sd = p->sd[i];
                mpnl::JobDev &J = jd[u];
                J.yt = p->yt[i];
                J.bound = p->bound[i];
                J.part = p->part[i];
                J.bound_begin = bacc;
                bacc += (sd.S * jobs[i].T + 63) / 64;
                J.rlat = sd.rlat;
                J.rq = rq_of(sd, p->precision);
                J.diag = sd.diag;
                J.permd = sd.permd;
                J.P = sd.P;
                J.order = sd.order;
                J.out = jobs[i].out;
                J.S = sd.S;
                J.T = jobs[i].T;
                J.N = sd.N;
                J.K = sd.K;
                J.NP = sd.NP;
                J.item_begin = acc;
                acc += sd.S * jobs[i].T;
            }
        } else {
            mpnl::dev::StageJob *sj = (mpnl::dev::StageJob *)(host + L.off);
            int acc = 0;
            for (size_t u = 0; u < L.jobs.size(); ++u) {
                const int i = L.jobs[u];
                mpnl::dev::StageJob &J = sj[u];
                J.H = (const float2 *)jobs[i].H;
                J.y = (const float2 *)jobs[i].y;
                J.yt = p->yt[i];
                J.sd = p->sd[i];
                J.T = jobs[i].T;
                J.delta = mpnl::dev::delta_of(jobs[i].mod);
                J.item_begin = acc;
                acc += L.kind == L_SQRD ? (p->sd[i].S + 1) / 2 : p->sd[i].S;
            }
        }
    }
}

// Enqueue the whole pipeline of table copy b on `st`: upload, a1, a2, a3,
// a4+a5.  With `timed`, every launch is bracketed by the context's stage timers.
hipError_t plan_enqueue(mpnl_batch *p, int b, hipStream_t st, mpnl_ctx *timed = nullptr)
{
    hipError_t e = hipMemcpyAsync(p->dev_table[b], p->pinned[b], p->table_bytes, hipMemcpyHostToDevice, st);
    // With several branches the path-search launches (bound, search and
    // reduction of one group stay together) go to the branch streams after
    // the rotation of their phase, and the side streams join `st` again at
    // the end: branches of the captured graph, so that the tail of one
    // launch overlaps the next launches instead of leaving the device idle.
    // With one phase the branches are `st` and the side streams; with
    // several, the side streams only: `st` runs the a1 .. a3 launches of
    // the next phase meanwhile.
    const bool fork = p->branches > 1;
    const bool phased = p->phases > 1;
    const int nside = phased ? p->branches : p->branches - 1;
    bool forked = false, in_paths = false;
    int fork_phase = -1;
    const hipStream_t st0 = st;
    // the window of the path stage on `st`: first path launch to the join
    hipEvent_t win0 = nullptr, win1 = nullptr;
    if (timed && timed->prof) {
        win0 = take_event(timed);
        win1 = take_event(timed);
    }
    for (const PlanLaunch &L : p->launches) {
        if (e != hipSuccess)
            break;
        st = st0;
        if (L.kind == L_PATHS && !in_paths) {
            in_paths = true;
            if (win0 && win1)
                e = hipEventRecord(win0, st0);
            if (e != hipSuccess)
                break;
        }
        if (fork && L.kind == L_PATHS) {
            if (L.phase != fork_phase) {  // the first path launch of a phase
                fork_phase = L.phase;
                e = hipEventRecord(p->fork_ev[L.phase], st0);
                for (int k = 0; k < nside && e == hipSuccess; ++k)
                    e = hipStreamWaitEvent(p->side[k], p->fork_ev[L.phase], 0);
                if (e != hipSuccess)
                    break;
                forked = true;
            }
            const int br = L.branch % p->branches;
            st = phased ? p->side[br] : br ? p->side[br - 1] : st0;
        }
        char *tab = p->dev_table[b] + L.off;
        const int nj = (int)L.jobs.size();
        mpnl_ctx off{};
        mpnl_ctx *tc = timed ? timed : &off;
        switch (L.kind) {
        case L_SQRD: {
            StageTimer tm(tc, MPNL_STAGE_SQRD, st);
            e = mpnl::launch_sqrd_batch((const mpnl::dev::StageJob *)tab, nj, L.items, L.param, st);
            break;
        }
        case L_POSVEC: {
            StageTimer tm(tc, MPNL_STAGE_POSVEC, st);
            e = mpnl::launch_posvec_batch((const mpnl::dev::StageJob *)tab, nj, L.items, L.param, L.nmax, st);
            break;
        }
        case L_ROTATE: {
            StageTimer tm(tc, MPNL_STAGE_ROTATE, st);
            e = mpnl::launch_rotate_batch((const mpnl::dev::StageJob *)tab, nj, L.items, L.nmax, st);
            break;
        }
        default:
            if (p->prune) {
                StageTimer tb(tc, MPNL_STAGE_BOUND, st);
                e = mpnl::launch_path_bound_multi((const mpnl::JobDev *)tab, nj, L.bound_items, L.param, L.bits,
                                                  p->precision, st);
            }
            if (e == hipSuccess) {  // the path search and its group reduction
                StageTimer tm(tc, MPNL_STAGE_PATHS, st);
                e = mpnl::launch_path_search_multi((const mpnl::JobDev *)tab, nj, L.items, L.param, L.bits,
                                                   p->precision, L.threads, L.groups, L.vpw, L.gmajor, st);
            }
        }
    }
    for (int k = 0; forked && k < nside && e == hipSuccess; ++k) {
        e = hipEventRecord(p->join_ev[k], p->side[k]);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(st0, p->join_ev[k], 0);
    }
    if (in_paths && win0 && win1 && e == hipSuccess)
        e = hipEventRecord(win1, st0);
    if (in_paths && win0 && win1 && e == hipSuccess)
        timed->timed.push_back({MPNL_STAGE_PATH_WINDOW, win0, win1});
    else if (timed)
        for (hipEvent_t x : {win0, win1})
            if (x)
                timed->spare_events.push_back(x);
    return e;
}

// Time every candidate shape of every path-search launch on the first run's
// data and keep the fastest: path groups of one wavefront or the whole
// vector's lanes (one group), numbered group major or vector major, times 4,
// 2 or 1 work items per workgroup as the workgroup size allows (ties: the
// earlier candidate in that order).  Each candidate is timed with its group
// reduction, the second of two passes.
hipError_t plan_autotune(mpnl_batch *p, const mpnl_job *jobs, hipStream_t st)
{
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess)
        e = hipEventCreate(&t1);
    if (e == hipSuccess) {
        plan_fill(p, 0, jobs);
        e = plan_enqueue(p, 0, st);  // produces yt, R, P and the bounds of every job
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    for (PlanLaunch &L : p->launches) {
        if (L.kind != L_PATHS || e != hipSuccess)
            continue;
        const mpnl::JobDev *tab = (const mpnl::JobDev *)(p->dev_table[0] + L.off);
        const int nj = (int)L.jobs.size();
        float best = 1e30f;
        const int group_choices[2] = {L.threads / 64, 1};
        for (int gi = 0; gi < (L.threads > 64 ? 2 : 1); ++gi) {
            const int groups = group_choices[gi];
            const int gw = L.threads / groups;
            for (int gmajor = 1; gmajor >= (groups > 1 ? 0 : 1); --gmajor)
                for (int vpw = 4; vpw >= 1; vpw /= 2) {
                    if (vpw * gw > 256)
                        continue;
                    float ms = 0.f;
                    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first pass warms up
                        e = hipEventRecord(t0, st);
                        if (e == hipSuccess)
                            e = mpnl::launch_path_search_multi(tab, nj, L.items, L.param, L.bits, p->precision,
                                                               L.threads, groups, vpw, gmajor, st);
                        if (e == hipSuccess)
                            e = hipEventRecord(t1, st);
                        if (e == hipSuccess)
                            e = hipEventSynchronize(t1);
                        if (e == hipSuccess)
                            e = hipEventElapsedTime(&ms, t0, t1);
                    }
                    if (e == hipSuccess && ms < best) {
                        best = ms;
                        L.groups = groups;
                        L.vpw = vpw;
                        L.gmajor = gmajor;
                    }
                }
        }
    }
    if (t0)
        (void)hipEventDestroy(t0);
    if (t1)
        (void)hipEventDestroy(t1);
    return e;
}

hipError_t plan_capture(mpnl_batch *p)
{
    hipError_t e = hipSuccess;
    for (int b = 0; b < kGraphCopies && e == hipSuccess; ++b) {
        hipGraph_t g = nullptr;
        e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess)
            break;
        hipError_t e2 = plan_enqueue(p, b, p->cap);
        e = hipStreamEndCapture(p->cap, &g);
        if (e2 != hipSuccess)
            e = e2;
        if (e == hipSuccess)
            e = hipGraphInstantiate(&p->exec[b], g, nullptr, nullptr, 0);
        if (g)
            (void)hipGraphDestroy(g);
    }
    if (e == hipSuccess)
        p->captured = true;
    return e;
}

bool same_shape(const mpnl_job &a, const mpnl_job &b)
{
    return a.S == b.S && a.T == b.T && a.M == b.M && a.N == b.N && a.mod == b.mod && a.n_paths == b.n_paths;
}

void plan_free(mpnl_ctx *ctx, mpnl_batch *p)
{
    for (int b = 0; b < kGraphCopies; ++b) {
        if (p->done[b])
            (void)hipEventSynchronize(p->done[b]);
        if (p->exec[b])
            (void)hipGraphExecDestroy(p->exec[b]);
        if (p->done[b])
            (void)hipEventDestroy(p->done[b]);
        if (p->pinned[b])
            (void)hipHostFree(p->pinned[b]);
    }
    if (p->cap)
        (void)hipStreamDestroy(p->cap);
    for (int k = 0; k + 1 < kMaxBranches; ++k) {
        if (p->side[k])
            (void)hipStreamDestroy(p->side[k]);
        if (p->join_ev[k])
            (void)hipEventDestroy(p->join_ev[k]);
    }
    for (int k = 0; k < kMaxPhases; ++k)
        if (p->fork_ev[k])
            (void)hipEventDestroy(p->fork_ev[k]);
    if (p->block >= 0)
        pool_release(ctx, p->block, nullptr);
    delete p;
}

}  // namespace

extern "C" {

int mpnl_detect_batch(mpnl_ctx *ctx, const mpnl_job *jobs, int n_jobs, void *stream)
{
    if (!ctx || !jobs || n_jobs <= 0)
        return MPNL_E_INVAL;
    for (int i = 0; i < n_jobs; ++i) {
        const mpnl_job &j = jobs[i];
        if (!j.H || !j.y || !j.out || j.T <= 0)
            return MPNL_E_INVAL;
        int rc = validate_shape(j.S, j.M, j.N, j.mod, j.n_paths);
        if (rc != MPNL_OK)
            return rc;
        if ((long long)j.S * j.T > INT_MAX / 4)
            return MPNL_E_UNSUPPORTED;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok())
        return hip_fail(ctx, hipErrorInvalidDevice);
    hipStream_t st = (hipStream_t)stream;

    // a job with more than 256 paths runs a1..a5 on its own; the others as
    // one batch: a1, a2 and a3 of all of them in one launch per bucket, then
    // one path-search launch per (user count, modulation, paths rounded up
    // to a wavefront), the same launches a planned batch replays
    std::vector<mpnl_job> small;
    int rc = MPNL_OK;
    for (int i = 0; i < n_jobs && rc == MPNL_OK; ++i) {
        const mpnl_job &j = jobs[i];
        if (std::min<long long>(j.n_paths, num_vectors_sat(1 << j.mod, j.N)) <= 256) {
            small.push_back(j);
            continue;
        }
        mpnl_slot *slot = nullptr;
        rc = prepare_impl(ctx, j.H, j.S, j.M, j.N, j.mod, j.n_paths, st, &slot);
        if (rc != MPNL_OK)
            break;
        rc = detect_impl(ctx, slot, j.y, j.T, j.out, st, false, 0.f, 0.f, nullptr);
        release_impl(ctx, slot);
    }
    if (rc != MPNL_OK || small.empty())
        return rc;

    mpnl_batch p;
    p.shapes = small;
    p.precision = ctx->precision;
    p.prune = ctx->prune;
    const size_t tables_at = plan_layout(&p, ctx->prune);
    // pinned staging buffer of the job tables: the first idle one of the
    // ring, else wait for the oldest
    mpnl_ctx::Staging *sg = nullptr;
    for (int k = 0; k < 4 && !sg; ++k) {
        mpnl_ctx::Staging &c = ctx->staging[(ctx->staging_next + k) % 4];
        if (!c.pending || hipEventQuery(c.ev) == hipSuccess)
            sg = &c;
    }
    if (!sg) {
        sg = &ctx->staging[ctx->staging_next];
        if (hipEventSynchronize(sg->ev) != hipSuccess)
            return MPNL_E_HIP;
    }
    ctx->staging_next = (int)(sg - ctx->staging + 1) % 4;
    if (sg->size < p.table_bytes) {
        if (sg->ptr)
            (void)hipHostFree(sg->ptr);
        sg->ptr = nullptr;
        sg->size = 0;
        hipError_t e = hipHostMalloc(&sg->ptr, p.table_bytes, hipHostMallocDefault);
        if (e != hipSuccess)
            return hip_fail(ctx, e);
        sg->size = p.table_bytes;
    }
    if (!sg->ev) {
        hipError_t e = hipEventCreateWithFlags(&sg->ev, hipEventDisableTiming);
        if (e != hipSuccess)
            return hip_fail(ctx, e);
    }
    int blk = -1;
    rc = pool_alloc(ctx, tables_at + p.table_bytes, st, &blk);
    if (rc != MPNL_OK)
        return rc;
    char *base = (char *)ctx->blocks[blk].ptr;
    plan_bind(&p, base);
    p.pinned[0] = sg->ptr;
    p.dev_table[0] = base + tables_at;
    plan_fill(&p, 0, small.data());
    hipError_t e = plan_enqueue(&p, 0, st, ctx->prof ? ctx : nullptr);
    if (e == hipSuccess)
        e = hipEventRecord(sg->ev, st);  // the table upload (first in the stream) has read the buffer
    sg->pending = e == hipSuccess;
    pool_release(ctx, blk, st);
    p.pinned[0] = nullptr;
    if (e != hipSuccess)
        return hip_fail(ctx, e);
    return MPNL_OK;
}


int mpnl_batch_create(mpnl_ctx *ctx, const mpnl_job *shapes, int n_jobs, unsigned flags, mpnl_batch **out)
{
    if (!ctx || !shapes || n_jobs <= 0 || !out || (flags & ~(MPNL_BATCH_AUTOTUNE | MPNL_BATCH_SERIAL)))
        return MPNL_E_INVAL;
    *out = nullptr;
    for (int i = 0; i < n_jobs; ++i) {
        const mpnl_job &j = shapes[i];
        if (j.T <= 0)
            return MPNL_E_INVAL;
        int rc = validate_shape(j.S, j.M, j.N, j.mod, j.n_paths);
        if (rc != MPNL_OK)
            return rc;
        if (std::min<long long>(j.n_paths, num_vectors_sat(1 << j.mod, j.N)) > 256)
            return MPNL_E_UNSUPPORTED;
        if ((long long)j.S * j.T > INT_MAX / 4)
            return MPNL_E_UNSUPPORTED;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok())
        return hip_fail(ctx, hipErrorInvalidDevice);
    mpnl_batch *p = new (std::nothrow) mpnl_batch();
    if (!p)
        return MPNL_E_NOMEM;
    p->shapes.assign(shapes, shapes + n_jobs);
    p->autotune = (flags & MPNL_BATCH_AUTOTUNE) != 0;
    p->precision = ctx->precision;
    p->prune = ctx->prune;

    const size_t tables_at = plan_layout(p, ctx->prune, (flags & MPNL_BATCH_SERIAL) ? 1 : kPlanPhases);
    const size_t total = tables_at + kGraphCopies * p->table_bytes;
    int rc = pool_alloc(ctx, total, nullptr, &p->block);
    if (rc != MPNL_OK) {
        delete p;
        return rc;
    }
    char *dbase = (char *)ctx->blocks[p->block].ptr;
    plan_bind(p, dbase);
    hipError_t e = hipSuccess;
    for (int b = 0; b < kGraphCopies && e == hipSuccess; ++b) {
        p->dev_table[b] = dbase + tables_at + b * p->table_bytes;
        e = hipHostMalloc(&p->pinned[b], p->table_bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&p->done[b], hipEventDisableTiming);
    }
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess && kPlanBranches > 1) {
        for (int k = 0; k < p->phases && e == hipSuccess; ++k)
            e = hipEventCreateWithFlags(&p->fork_ev[k], hipEventDisableTiming);
        // one side stream per branch when the phases keep `st` for a1 .. a3
        const int nside = p->phases > 1 ? kPlanBranches : kPlanBranches - 1;
        for (int k = 0; k < nside && e == hipSuccess; ++k) {
            e = hipStreamCreateWithFlags(&p->side[k], hipStreamNonBlocking);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&p->join_ev[k], hipEventDisableTiming);
        }
        if (e == hipSuccess)
            p->branches = kPlanBranches;
    }
    plan_branches(p, p->branches);
    if (e != hipSuccess) {
        plan_free(ctx, p);
        return hip_fail(ctx, e);
    }
    ctx->batches.push_back(p);
    *out = p;
    return MPNL_OK;
}

int mpnl_batch_run(mpnl_ctx *ctx, mpnl_batch *p, const mpnl_job *jobs, void *stream)
{
    if (!ctx || !p || !jobs || std::find(ctx->batches.begin(), ctx->batches.end(), p) == ctx->batches.end())
        return MPNL_E_INVAL;
    for (size_t i = 0; i < p->shapes.size(); ++i)
        if (!jobs[i].H || !jobs[i].y || !jobs[i].out || !same_shape(jobs[i], p->shapes[i]))
            return MPNL_E_INVAL;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (!p->tuned) {
        if (p->autotune)
            e = plan_autotune(p, jobs, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return hip_fail(ctx, e);
        p->tuned = true;
    }
    // With stage profiling on, the pipeline is enqueued launch by launch so
    // that every stage is timed; otherwise the captured graph is replayed.
    if (!ctx->prof && !p->captured) {
        e = plan_capture(p);
        if (e != hipSuccess)
            return hip_fail(ctx, e);
    }
    const int b = p->next;
    if (p->used[b])
        e = hipEventSynchronize(p->done[b]);  // its previous run has read the table
    if (e == hipSuccess) {
        plan_fill(p, b, jobs);
        e = ctx->prof ? plan_enqueue(p, b, st, ctx) : hipGraphLaunch(p->exec[b], st);
    }
    if (e == hipSuccess)
        e = hipEventRecord(p->done[b], st);
    if (e != hipSuccess)
        return hip_fail(ctx, e);
    p->used[b] = true;
    p->next = (b + 1) % kGraphCopies;
    return MPNL_OK;
}

int mpnl_batch_info(const mpnl_batch *p, int *n_launches, int *shapes, int max)
{
    if (!p || max < 0)
        return MPNL_E_INVAL;
    int n = 0;
    for (const PlanLaunch &L : p->launches)
        if (L.kind == L_PATHS) {
            if (shapes && n < max) {
                int *o = shapes + 7 * n;
                o[0] = L.param;
                o[1] = L.bits;
                o[2] = L.threads;
                o[3] = L.threads / L.groups;
                o[4] = L.vpw;
                o[5] = L.gmajor;
                o[6] = (int)(((long long)L.items + L.vpw - 1) / L.vpw * L.groups);
            }
            ++n;
        }
    if (n_launches)
        *n_launches = n;
    return MPNL_OK;
}

int mpnl_batch_destroy(mpnl_ctx *ctx, mpnl_batch *p)
{
    if (!p)
        return MPNL_OK;
    if (!ctx)
        return MPNL_E_INVAL;
    auto it = std::find(ctx->batches.begin(), ctx->batches.end(), p);
    if (it == ctx->batches.end())
        return MPNL_E_INVAL;
    ctx->batches.erase(it);
    DeviceGuard g(ctx->device);
    plan_free(ctx, p);
    return MPNL_OK;
}

}  // extern "C"
