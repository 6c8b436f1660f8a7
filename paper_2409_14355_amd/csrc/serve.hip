// Serving core: slot-detection jobs arrive over time, wait for admission
// (launch slots and the device-memory budget), are merged into launches
// (continuous batching: whatever waits when a launch slot frees up goes into
// the next launch) and complete asynchronously.  A large job may run as
// pieces of whole subcarriers; the job completes with its last piece.  The
// scheduler only talks to an Executor: the device executor runs a launch as
// one mpnl_detect_batch() on its own stream and times it with events; the
// modelled executor runs on a virtual clock for tests without a GPU.
#include "mpnl.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <new>
#include <vector>

#include "runtime_internal.h"

namespace mpnl {
namespace serve {

// A unit of admission: a whole job, or one piece (a range of whole
// subcarriers) of a split job.
struct Job {
    int64_t id;        // the submitted job's id
    double arrival;
    size_t bytes;      // device bytes while it runs
    int64_t vectors;
    double est_us;     // the slack policy's estimate of its service time
    mpnl_job job;      // the piece's shape; H / y / out of the whole job
    int s0 = 0;        // first subcarrier of the piece
    int s_full = 0;    // subcarriers of the whole job (0: not split)
    int parent = -1;   // scheduler's record of the submitted job
};

class Executor {
  public:
    virtual ~Executor() = default;
    virtual double now() = 0;
    // Start one launch of these jobs: a token >= 0, or an MPNL error code (< 0).
    virtual int launch(const std::vector<Job> &jobs) = 0;
    // 1 once launch `token` has finished (its completion time and error
    // code), 0 while it runs.
    virtual int finished(int token, double *done, int *error) = 0;
    // The launch slot of a retired token may be reused.
    virtual void release(int token) = 0;
};

mpnl_completion make_completion(int64_t id, double arrival, int status, int error, double start, double done)
{
    mpnl_completion c;
    c.id = id;
    c.status = status;
    c.error = error;
    c.arrival_us = arrival;
    c.start_us = start;
    c.done_us = done;
    return c;
}

// Path-search GFLOP of a job shape: 4 N (N - 1) + 11 N flops per path and
// received vector, paths clamped to |Q|^N.
double job_gflop(const mpnl_job &j)
{
    double K = (double)j.n_paths;
    const double q = (double)(1 << j.mod);
    if (j.N * std::log2(q) < 40.0)
        K = std::min(K, std::pow(q, (double)j.N));
    return (double)j.S * j.T * K * (4.0 * j.N * (j.N - 1) + 11.0 * j.N) * 1e-9;
}

class Scheduler {
  public:
    Scheduler(const mpnl_server_config &cfg, Executor &ex) : cfg_(cfg), ex_(ex) {}

    double estimate(double gflop) const { return cfg_.est_fixed_us + cfg_.est_us_per_gflop * gflop; }

    // Queue a submitted job as its pieces (one piece when it is not split).
    void submit(int64_t id, double arrival, std::vector<Job> pieces, std::vector<mpnl_completion> &out)
    {
        bool too_big = false;
        for (const Job &p : pieces)
            too_big |= cfg_.hbm_budget != 0 && p.bytes > cfg_.hbm_budget;
        const bool full = cfg_.max_queue > 0 && queued_jobs_ >= cfg_.max_queue;
        if (too_big || full || pieces.empty()) {
            const double t = ex_.now();
            out.push_back(make_completion(id, arrival, MPNL_JOB_REJECTED, MPNL_OK, t, t));
            return;
        }
        const int pi = new_parent();
        Parent &P = parents_[pi];
        P = Parent{};
        P.id = id;
        P.arrival = arrival;
        P.left = (int)pieces.size();
        P.waiting = (int)pieces.size();
        P.live = true;
        for (Job &p : pieces) {
            p.parent = pi;
            P.est_left += p.est_us;
            wait_.push_back(p);
        }
        ++queued_jobs_;
        ++open_jobs_;
    }

    // Retire finished launches, then admit waiting pieces into new launches
    // while launch slots and budget allow.
    void progress(std::vector<mpnl_completion> &out)
    {
        for (size_t i = 0; i < flights_.size();) {
            Flight &f = flights_[i];
            double done = 0.0;
            int err = MPNL_OK;
            if (!ex_.finished(f.token, &done, &err)) {
                ++i;
                continue;
            }
            for (const Job &j : f.jobs)
                piece_done(j.parent, err, done, out);
            held_ -= f.bytes;
            ex_.release(f.token);
            flights_.erase(flights_.begin() + (long)i);
        }
        while ((int)flights_.size() < cfg_.max_inflight && !wait_.empty()) {
            const double t = ex_.now();
            if (cfg_.drop_late)
                drop_late(t, out);
            if (wait_.empty())
                break;
            order(t);
            std::vector<Job> batch;
            size_t bytes = 0;
            size_t k = 0;
            while (k < wait_.size() && (int)batch.size() < cfg_.max_batch_jobs) {
                const Job &h = wait_[k];
                if (cfg_.hbm_budget != 0 && held_ + bytes + h.bytes > cfg_.hbm_budget)
                    break;  // waits for memory and blocks the pieces behind it
                bytes += h.bytes;
                batch.push_back(h);
                ++k;
            }
            if (batch.empty())
                break;
            wait_.erase(wait_.begin(), wait_.begin() + (long)k);
            for (const Job &j : batch) {
                Parent &P = parents_[j.parent];
                P.est_left -= j.est_us;
                --P.waiting;
                if (P.start < 0.0) {
                    P.start = t;
                    --queued_jobs_;
                }
            }
            const int tok = ex_.launch(batch);
            ++launches_;
            if (tok < 0) {
                const double te = ex_.now();
                for (const Job &j : batch)
                    piece_done(j.parent, tok, te, out);
                continue;
            }
            held_ += bytes;
            flights_.push_back(Flight{tok, std::move(batch), t, bytes});
        }
    }

    int pending() const { return open_jobs_; }
    int launches() const { return launches_; }
    bool idle() const { return flights_.empty() && wait_.empty(); }

  private:
    struct Parent {
        int64_t id = 0;
        double arrival = 0.0;
        int left = 0;         // pieces not yet finished
        int waiting = 0;      // pieces not yet admitted
        double est_left = 0;  // estimated time of the pieces not yet admitted
        double start = -1.0;  // first admission
        double done = 0.0;    // latest piece completion
        int error = MPNL_OK;
        bool live = false;
    };
    struct Flight {
        int token;
        std::vector<Job> jobs;
        double start;
        size_t bytes;
    };

    int new_parent()
    {
        if (!free_.empty()) {
            const int i = free_.back();
            free_.pop_back();
            return i;
        }
        parents_.emplace_back();
        return (int)parents_.size() - 1;
    }

    void finish_parent(int pi, int status, std::vector<mpnl_completion> &out)
    {
        Parent &P = parents_[pi];
        out.push_back(make_completion(P.id, P.arrival, status, P.error, P.start, P.done));
        P.live = false;
        free_.push_back(pi);
        --open_jobs_;
    }

    void piece_done(int pi, int err, double done, std::vector<mpnl_completion> &out)
    {
        Parent &P = parents_[pi];
        P.done = std::max(P.done, done);
        if (err != MPNL_OK && P.error == MPNL_OK)
            P.error = err;
        if (--P.left == 0)
            finish_parent(pi, P.error == MPNL_OK ? MPNL_JOB_DONE : MPNL_JOB_FAILED, out);
    }

    // A job that has waited past the deadline and has no piece running or
    // done yet is dropped with all its pieces.
    void drop_late(double t, std::vector<mpnl_completion> &out)
    {
        std::vector<int> gone;
        for (const Job &j : wait_) {
            const Parent &P = parents_[j.parent];
            if (P.start < 0.0 && t - P.arrival > cfg_.deadline_us &&
                std::find(gone.begin(), gone.end(), j.parent) == gone.end())
                gone.push_back(j.parent);
        }
        if (gone.empty())
            return;
        wait_.erase(std::remove_if(wait_.begin(), wait_.end(),
                                   [&](const Job &j) {
                                       return std::find(gone.begin(), gone.end(), j.parent) != gone.end();
                                   }),
                    wait_.end());
        for (int pi : gone) {
            Parent &P = parents_[pi];
            P.start = t;
            P.done = t;
            --queued_jobs_;
            finish_parent(pi, MPNL_JOB_DROPPED, out);
        }
    }

    // Admission order of the waiting pieces (stable: arrival order, then
    // piece order, breaks every tie).
    void order(double t)
    {
        if (cfg_.policy != MPNL_SCHED_SLACK)
            return;
        std::stable_sort(wait_.begin(), wait_.end(), [&](const Job &a, const Job &b) {
            const Parent &A = parents_[a.parent], &B = parents_[b.parent];
            const double sa = A.arrival + cfg_.deadline_us - t - A.est_left;
            const double sb = B.arrival + cfg_.deadline_us - t - B.est_left;
            const bool fa = sa >= 0.0, fb = sb >= 0.0;
            if (fa != fb)
                return fa;                        // jobs that can still make it first
            if (fa && sa != sb)
                return sa < sb;                   // least slack first
            if (a.arrival != b.arrival)
                return a.arrival < b.arrival;     // then arrival order
            return a.parent == b.parent && a.s0 < b.s0;
        });
    }

    mpnl_server_config cfg_;
    Executor &ex_;
    std::deque<Job> wait_;
    std::vector<Flight> flights_;
    std::vector<Parent> parents_;
    std::vector<int> free_;
    size_t held_ = 0;
    int queued_jobs_ = 0;  // submitted jobs none of whose pieces was admitted yet
    int open_jobs_ = 0;    // submitted jobs not yet completed
    int launches_ = 0;
};

// ---------------------------------------------------------------------------
// Device executor: launch slot k owns stream k and a timing event recorded
// after the launch; completion times come from the event, measured against a
// reference event taken when the executor started.
// ---------------------------------------------------------------------------
class GpuExecutor : public Executor {
  public:
    GpuExecutor(mpnl_ctx *ctx, int device, int slots) : ctx_(ctx), device_(device), n_(slots) {}

    int init()
    {
        t0_ = std::chrono::steady_clock::now();
        streams_.assign(n_, nullptr);
        done_.assign(n_, nullptr);
        busy_.assign(n_, false);
        tmp_.assign(n_, nullptr);
        cap_.assign(n_, 0);
        int prev = -1;
        (void)hipGetDevice(&prev);
        hipError_t e = hipSetDevice(device_);
        for (int k = 0; k < n_ && e == hipSuccess; ++k) {
            e = hipStreamCreateWithFlags(&streams_[k], hipStreamNonBlocking);
            if (e == hipSuccess)
                e = hipEventCreate(&done_[k]);
        }
        if (e == hipSuccess)
            e = hipEventCreate(&ref_);
        if (e == hipSuccess) {
            const double before = now();
            e = hipEventRecord(ref_, streams_[0]);
            if (e == hipSuccess)
                e = hipEventSynchronize(ref_);
            ref_us_ = 0.5 * (before + now());
        }
        if (prev >= 0)
            (void)hipSetDevice(prev);
        return e == hipSuccess ? MPNL_OK : MPNL_E_HIP;
    }

    ~GpuExecutor() override
    {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(device_);
        for (int k = 0; k < n_; ++k) {
            if (streams_.size() > (size_t)k && streams_[k]) {
                (void)hipStreamSynchronize(streams_[k]);
                (void)hipStreamDestroy(streams_[k]);
            }
            if (done_.size() > (size_t)k && done_[k])
                (void)hipEventDestroy(done_[k]);
        }
        if (ref_)
            (void)hipEventDestroy(ref_);
        for (void *b : tmp_)
            if (b)
                (void)hipFree(b);
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }

    double now() override
    {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0_).count();
    }

    // A piece of a split job reads its subcarriers of y and writes those of
    // out, which are strided in the job's (T, S, .) arrays: its y rows are
    // gathered into the launch slot's staging buffer before the launch and
    // its decisions scattered back after it (device-to-device copies on the
    // slot's stream).
    int launch(const std::vector<Job> &jobs) override
    {
        int k = 0;
        while (k < n_ && busy_[k])
            ++k;
        if (k == n_)
            return MPNL_E_INVAL;  // the scheduler keeps at most n_ launches
        hipStream_t st = streams_[k];
        size_t need = 0;
        for (const Job &j : jobs)
            if (j.s_full)
                need += staging_bytes(j.job);
        if (need > cap_[k]) {  // the slot is idle: nothing of it is in flight
            if (tmp_[k])
                (void)hipFree(tmp_[k]);
            tmp_[k] = nullptr;
            cap_[k] = 0;
            if (hipMalloc(&tmp_[k], need) != hipSuccess)
                return MPNL_E_NOMEM;
            cap_[k] = need;
        }
        std::vector<mpnl_job> js(jobs.size());
        char *at = (char *)tmp_[k];
        for (size_t i = 0; i < jobs.size(); ++i) {
            const Job &j = jobs[i];
            js[i] = j.job;
            if (!j.s_full)
                continue;
            const mpnl_job &w = j.job;  // H / y / out of the whole job, S = the piece's
            const size_t yrow = (size_t)w.S * w.M * sizeof(float2), orow = (size_t)w.S * w.N * sizeof(int32_t);
            js[i].H = (const float2 *)w.H + (size_t)j.s0 * w.M * w.N;
            js[i].y = at;
            js[i].out = (int32_t *)(at + align_up(w.T * yrow));
            if (hipMemcpy2DAsync(at, yrow, (const float2 *)w.y + (size_t)j.s0 * w.M,
                                 (size_t)j.s_full * w.M * sizeof(float2), yrow, w.T, hipMemcpyDeviceToDevice,
                                 st) != hipSuccess)
                return MPNL_E_HIP;
            at += staging_bytes(w);
        }
        const int rc = mpnl_detect_batch(ctx_, js.data(), (int)js.size(), st);
        if (rc != MPNL_OK)
            return rc;
        for (size_t i = 0; i < jobs.size(); ++i) {
            const Job &j = jobs[i];
            if (!j.s_full)
                continue;
            const mpnl_job &w = j.job;
            const size_t orow = (size_t)w.S * w.N * sizeof(int32_t);
            if (hipMemcpy2DAsync(w.out + (size_t)j.s0 * w.N, (size_t)j.s_full * w.N * sizeof(int32_t), js[i].out,
                                 orow, orow, w.T, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return MPNL_E_HIP;
        }
        if (hipEventRecord(done_[k], st) != hipSuccess)
            return MPNL_E_HIP;
        busy_[k] = true;
        return k;
    }

    static size_t align_up(size_t x) { return (x + 255) / 256 * 256; }
    // staging of one piece: its y rows, then its decisions
    static size_t staging_bytes(const mpnl_job &piece)
    {
        return align_up((size_t)piece.T * piece.S * piece.M * sizeof(float2)) +
               align_up((size_t)piece.T * piece.S * piece.N * sizeof(int32_t));
    }

    int finished(int token, double *done, int *error) override
    {
        const hipError_t q = hipEventQuery(done_[token]);
        if (q == hipErrorNotReady)
            return 0;
        *error = MPNL_OK;
        float ms = 0.f;
        if (q != hipSuccess || hipEventElapsedTime(&ms, ref_, done_[token]) != hipSuccess) {
            *error = MPNL_E_HIP;
            *done = now();
            return 1;
        }
        *done = ref_us_ + 1000.0 * (double)ms;
        return 1;
    }

    void release(int token) override { busy_[token] = false; }

  private:
    mpnl_ctx *ctx_;
    int device_;
    int n_;
    std::chrono::steady_clock::time_point t0_;
    std::vector<hipStream_t> streams_;
    std::vector<hipEvent_t> done_;
    std::vector<bool> busy_;
    std::vector<void *> tmp_;   // per launch slot: staging of split pieces
    std::vector<size_t> cap_;
    hipEvent_t ref_ = nullptr;
    double ref_us_ = 0.0;
};

// ---------------------------------------------------------------------------
// Modelled device on a virtual clock: launches run one after another, each
// taking launch_us + per_vector_us * vectors (+ slow_extra_us).
// ---------------------------------------------------------------------------
class SimExecutor : public Executor {
  public:
    explicit SimExecutor(const mpnl_sim_device &d) : d_(d) {}
    double now() override { return clock; }

    int launch(const std::vector<Job> &jobs) override
    {
        const int idx = count_++;
        if (idx == d_.fail_launch)
            return MPNL_E_HIP;
        double dur = d_.launch_us;
        for (const Job &j : jobs) {
            dur += d_.per_vector_us * (double)j.vectors;
            if (j.id == d_.slow_job)
                dur += d_.slow_extra_us;
        }
        const double start = std::max(clock, free_at_);
        free_at_ = start + dur;
        done_.push_back(free_at_);
        return (int)done_.size() - 1;
    }

    int finished(int token, double *done, int *error) override
    {
        if (clock < done_[token])
            return 0;
        *done = done_[token];
        *error = MPNL_OK;
        return 1;
    }

    void release(int token) override { retired_.push_back(token); }

    // Earliest completion among launches not yet retired (infinity if none).
    double next_done() const
    {
        double t = INFINITY;
        for (size_t k = 0; k < done_.size(); ++k)
            if (std::find(retired_.begin(), retired_.end(), (int)k) == retired_.end())
                t = std::min(t, done_[k]);
        return t;
    }

    double clock = 0.0;

  private:
    mpnl_sim_device d_;
    int count_ = 0;
    double free_at_ = 0.0;
    std::vector<double> done_;
    std::vector<int> retired_;
};

bool config_ok(const mpnl_server_config *c)
{
    return c && c->max_batch_jobs >= 1 && c->max_inflight >= 1 && c->max_inflight <= 8 && c->max_queue >= 0 &&
           c->deadline_us >= 0.0 && (c->policy == MPNL_SCHED_FIFO || c->policy == MPNL_SCHED_SLACK) &&
           c->split_vectors >= 0 && std::isfinite(c->est_fixed_us) && std::isfinite(c->est_us_per_gflop);
}

// A device job as its pieces: whole subcarrier ranges of at most
// max(T, split_vectors) vectors when it has more than split_vectors, else
// one piece.  A piece carries the whole job's H / y / out and its own S; its
// bytes add the staging of its y rows and decisions.
std::vector<Job> device_pieces(const Scheduler &sch, const mpnl_server_config &cfg, const mpnl_job &job, int64_t id,
                               double arrival)
{
    std::vector<Job> out;
    const int64_t vec = (int64_t)job.S * job.T;
    if (cfg.split_vectors <= 0 || vec <= cfg.split_vectors) {
        out.push_back(Job{id, arrival, job_device_bytes(job), vec, sch.estimate(job_gflop(job)), job});
        return out;
    }
    const int per = (int)std::max<int64_t>(1, cfg.split_vectors / job.T);  // subcarriers a piece
    const int n = (job.S + per - 1) / per;
    for (int i = 0; i < n; ++i) {
        const int s0 = (int)((int64_t)job.S * i / n), s1 = (int)((int64_t)job.S * (i + 1) / n);
        mpnl_job p = job;
        p.S = s1 - s0;
        Job j{id, arrival, job_device_bytes(p) + GpuExecutor::staging_bytes(p), (int64_t)p.S * p.T,
              sch.estimate(job_gflop(p)), p};
        j.s0 = s0;
        j.s_full = job.S;
        out.push_back(j);
    }
    return out;
}

// A modelled job as its pieces: near-equal vector counts, bytes and work
// shared in proportion.
std::vector<Job> sim_pieces(const Scheduler &sch, const mpnl_server_config &cfg, const mpnl_sim_job &sj)
{
    std::vector<Job> out;
    const int64_t n = (cfg.split_vectors > 0 && sj.vectors > cfg.split_vectors)
                          ? (sj.vectors + cfg.split_vectors - 1) / cfg.split_vectors
                          : 1;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t v0 = sj.vectors * i / n, v1 = sj.vectors * (i + 1) / n;
        const double f = sj.vectors > 0 ? (double)(v1 - v0) / (double)sj.vectors : 1.0 / (double)n;
        Job j{sj.id, sj.arrival_us, (size_t)std::ceil((double)sj.bytes * f), v1 - v0, sch.estimate(sj.gflop * f),
              mpnl_job{}};
        j.s0 = (int)i;
        j.s_full = n > 1 ? 1 : 0;
        out.push_back(j);
    }
    return out;
}

// splitmix64: seeded stream of uniform 64-bit words
uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// exponential gap with mean 1 / rate_hz, in microseconds
double exp_gap_us(uint64_t &s, double rate_hz)
{
    const double u = ((double)(splitmix64(s) >> 11) + 1.0) * (1.0 / 9007199254740992.0);  // (0, 1]
    return -std::log(u) / rate_hz * 1e6;
}

}  // namespace serve
}  // namespace mpnl

struct mpnl_server {
    mpnl_ctx *ctx = nullptr;
    mpnl_server_config cfg{};
    mpnl::serve::GpuExecutor *ex = nullptr;
    mpnl::serve::Scheduler *sched = nullptr;
    std::vector<mpnl_completion> ready;
};

extern "C" {

size_t mpnl_job_bytes(int S, int T, int M, int N, int mod, int n_paths)
{
    mpnl_job j{};
    j.S = S;
    j.T = T;
    j.M = M;
    j.N = N;
    j.mod = mod;
    j.n_paths = n_paths;
    return mpnl::job_device_bytes(j);
}

int mpnl_server_create(mpnl_ctx *ctx, const mpnl_server_config *cfg, mpnl_server **out)
{
    using namespace mpnl::serve;
    if (!ctx || !out || !config_ok(cfg))
        return MPNL_E_INVAL;
    *out = nullptr;
    const int device = mpnl::context_device(ctx);
    mpnl_server *s = new (std::nothrow) mpnl_server();
    if (!s)
        return MPNL_E_NOMEM;
    s->ctx = ctx;
    s->cfg = *cfg;
    s->ex = new (std::nothrow) GpuExecutor(ctx, device, cfg->max_inflight);
    int rc = s->ex ? s->ex->init() : MPNL_E_NOMEM;
    if (rc == MPNL_OK) {
        s->sched = new (std::nothrow) Scheduler(s->cfg, *s->ex);
        if (!s->sched)
            rc = MPNL_E_NOMEM;
    }
    if (rc != MPNL_OK) {
        delete s->ex;
        delete s;
        return rc;
    }
    *out = s;
    return MPNL_OK;
}

double mpnl_server_now_us(const mpnl_server *s)
{
    return s ? s->ex->now() : 0.0;
}

int mpnl_server_submit(mpnl_server *s, const mpnl_job *job, int64_t id, double arrival_us)
{
    if (!s || !job || !job->H || !job->y || !job->out)
        return MPNL_E_INVAL;
    const int rc = mpnl::validate_job_shape(*job);
    if (rc != MPNL_OK)
        return rc;
    s->sched->submit(id, arrival_us, mpnl::serve::device_pieces(*s->sched, s->cfg, *job, id, arrival_us), s->ready);
    return MPNL_OK;
}

int mpnl_server_poll(mpnl_server *s, mpnl_completion *done, int max, int *n_done)
{
    if (!s || max < 0 || (max > 0 && !done))
        return MPNL_E_INVAL;
    s->sched->progress(s->ready);
    const int n = std::min<int>(max, (int)s->ready.size());
    std::copy(s->ready.begin(), s->ready.begin() + n, done);
    s->ready.erase(s->ready.begin(), s->ready.begin() + n);
    if (n_done)
        *n_done = n;
    return MPNL_OK;
}

int mpnl_server_pending(const mpnl_server *s)
{
    return s ? s->sched->pending() + (int)s->ready.size() : 0;
}

int mpnl_server_run_poisson(mpnl_server *s, const mpnl_job *pool, int pool_n, int n_jobs, double rate_hz,
                            uint64_t seed, mpnl_completion *out, int32_t *entry)
{
    using namespace mpnl::serve;
    if (!s || !pool || pool_n <= 0 || n_jobs < 0 || !(rate_hz > 0.0) || (n_jobs > 0 && !out) ||
        !s->sched->idle() || !s->ready.empty())
        return MPNL_E_INVAL;
    for (int p = 0; p < pool_n; ++p) {
        if (!pool[p].H || !pool[p].y || !pool[p].out)
            return MPNL_E_INVAL;
        const int rc = mpnl::validate_job_shape(pool[p]);
        if (rc != MPNL_OK)
            return rc;
    }
    uint64_t rng = seed;
    std::vector<char> seen(n_jobs, 0);
    int submitted = 0, completed = 0;
    double t_next = s->ex->now() + exp_gap_us(rng, rate_hz);
    std::vector<mpnl_completion> got;
    while (completed < n_jobs) {
        const double t = s->ex->now();
        while (submitted < n_jobs && t_next <= t) {
            const int p = (int)(splitmix64(rng) % (uint64_t)pool_n);
            if (entry)
                entry[submitted] = p;
            s->sched->submit(submitted, t_next, device_pieces(*s->sched, s->cfg, pool[p], submitted, t_next), got);
            ++submitted;
            t_next += exp_gap_us(rng, rate_hz);
        }
        s->sched->progress(got);
        for (const mpnl_completion &c : got)
            if (c.id >= 0 && c.id < n_jobs && !seen[c.id]) {
                seen[c.id] = 1;
                out[c.id] = c;
                ++completed;
            }
        got.clear();
    }
    return MPNL_OK;
}

int mpnl_server_destroy(mpnl_server *s)
{
    if (!s)
        return MPNL_OK;
    delete s->sched;
    delete s->ex;  // waits for its streams
    delete s;
    return MPNL_OK;
}

int mpnl_sched_simulate(const mpnl_server_config *cfg, const mpnl_sim_device *dev, const mpnl_sim_job *jobs,
                        int n_jobs, mpnl_completion *out, int *n_launches)
{
    using namespace mpnl::serve;
    if (!config_ok(cfg) || !dev || n_jobs < 0 || (n_jobs > 0 && (!jobs || !out)))
        return MPNL_E_INVAL;
    for (int i = 0; i < n_jobs; ++i)
        if (jobs[i].id != i || (i > 0 && jobs[i].arrival_us < jobs[i - 1].arrival_us))
            return MPNL_E_INVAL;  // ids 0..n-1 in arrival order
    SimExecutor ex(*dev);
    Scheduler sched(*cfg, ex);
    std::vector<char> seen(n_jobs, 0);
    std::vector<mpnl_completion> got;
    int next = 0, completed = 0;
    while (completed < n_jobs) {
        while (next < n_jobs && jobs[next].arrival_us <= ex.clock) {
            const mpnl_sim_job &sj = jobs[next];
            sched.submit(sj.id, sj.arrival_us, sim_pieces(sched, *cfg, sj), got);
            ++next;
        }
        sched.progress(got);
        for (const mpnl_completion &c : got) {
            seen[c.id] = 1;
            out[c.id] = c;
            ++completed;
        }
        got.clear();
        if (completed == n_jobs)
            break;
        // next event: an arrival or a launch completion
        double t = ex.next_done();
        if (next < n_jobs)
            t = std::min(t, jobs[next].arrival_us);
        if (!(t < INFINITY))
            return MPNL_E_INVAL;  // nothing can happen any more (cannot occur)
        ex.clock = std::max(ex.clock, t);
    }
    if (n_launches)
        *n_launches = sched.launches();
    return MPNL_OK;
}

}  // extern "C"
