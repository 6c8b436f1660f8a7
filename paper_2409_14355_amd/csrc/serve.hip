// Serving core: slot-detection jobs arrive over time, wait in a FIFO for
// admission (launch slots and the device-memory budget), are merged into
// launches (continuous batching: whatever waits when a launch slot frees up
// goes into the next launch) and complete asynchronously.  The scheduler
// only talks to an Executor: the device executor runs a launch as one
// mpnl_detect_batch() on its own stream and times it with events; the
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

struct Job {
    int64_t id;
    double arrival;
    size_t bytes;
    int64_t vectors;
    mpnl_job job;
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

mpnl_completion make_completion(const Job &j, int status, int error, double start, double done)
{
    mpnl_completion c;
    c.id = j.id;
    c.status = status;
    c.error = error;
    c.arrival_us = j.arrival;
    c.start_us = start;
    c.done_us = done;
    return c;
}

class Scheduler {
  public:
    Scheduler(const mpnl_server_config &cfg, Executor &ex) : cfg_(cfg), ex_(ex) {}

    void submit(const Job &j, std::vector<mpnl_completion> &out)
    {
        const bool too_big = cfg_.hbm_budget != 0 && j.bytes > cfg_.hbm_budget;
        const bool full = cfg_.max_queue > 0 && (int)wait_.size() >= cfg_.max_queue;
        if (too_big || full) {
            const double t = ex_.now();
            out.push_back(make_completion(j, MPNL_JOB_REJECTED, MPNL_OK, t, t));
            return;
        }
        wait_.push_back(j);
    }

    // Retire finished launches, then admit waiting jobs into new launches
    // while launch slots and budget allow.  The queue is served in arrival
    // order: a head job that does not fit the budget waits for memory to be
    // freed and blocks the jobs behind it.
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
                out.push_back(make_completion(j, err == MPNL_OK ? MPNL_JOB_DONE : MPNL_JOB_FAILED, err, f.start, done));
            held_ -= f.bytes;
            running_ -= (int)f.jobs.size();
            ex_.release(f.token);
            flights_.erase(flights_.begin() + (long)i);
        }
        while ((int)flights_.size() < cfg_.max_inflight && !wait_.empty()) {
            const double t = ex_.now();
            std::vector<Job> batch;
            size_t bytes = 0;
            while (!wait_.empty() && (int)batch.size() < cfg_.max_batch_jobs) {
                const Job &h = wait_.front();
                if (cfg_.drop_late && t - h.arrival > cfg_.deadline_us) {
                    out.push_back(make_completion(h, MPNL_JOB_DROPPED, MPNL_OK, t, t));
                    wait_.pop_front();
                    continue;
                }
                if (cfg_.hbm_budget != 0 && held_ + bytes + h.bytes > cfg_.hbm_budget)
                    break;
                bytes += h.bytes;
                batch.push_back(h);
                wait_.pop_front();
            }
            if (batch.empty())
                break;
            const int tok = ex_.launch(batch);
            ++launches_;
            if (tok < 0) {
                const double te = ex_.now();
                for (const Job &j : batch)
                    out.push_back(make_completion(j, MPNL_JOB_FAILED, tok, t, te));
                continue;
            }
            held_ += bytes;
            running_ += (int)batch.size();
            flights_.push_back(Flight{tok, std::move(batch), t, bytes});
        }
    }

    int pending() const { return (int)wait_.size() + running_; }
    int launches() const { return launches_; }
    bool idle() const { return flights_.empty() && wait_.empty(); }

  private:
    struct Flight {
        int token;
        std::vector<Job> jobs;
        double start;
        size_t bytes;
    };
    mpnl_server_config cfg_;
    Executor &ex_;
    std::deque<Job> wait_;
    std::vector<Flight> flights_;
    size_t held_ = 0;
    int running_ = 0;
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
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }

    double now() override
    {
        return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0_).count();
    }

    int launch(const std::vector<Job> &jobs) override
    {
        int k = 0;
        while (k < n_ && busy_[k])
            ++k;
        if (k == n_)
            return MPNL_E_INVAL;  // the scheduler keeps at most n_ launches
        std::vector<mpnl_job> js(jobs.size());
        for (size_t i = 0; i < jobs.size(); ++i)
            js[i] = jobs[i].job;
        const int rc = mpnl_detect_batch(ctx_, js.data(), (int)js.size(), streams_[k]);
        if (rc != MPNL_OK)
            return rc;
        if (hipEventRecord(done_[k], streams_[k]) != hipSuccess)
            return MPNL_E_HIP;
        busy_[k] = true;
        return k;
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
           c->deadline_us >= 0.0;
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
    mpnl::serve::Job j{id, arrival_us, mpnl::job_device_bytes(*job), (int64_t)job->S * job->T, *job};
    s->sched->submit(j, s->ready);
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
    std::vector<size_t> bytes(pool_n);
    for (int p = 0; p < pool_n; ++p) {
        if (!pool[p].H || !pool[p].y || !pool[p].out)
            return MPNL_E_INVAL;
        const int rc = mpnl::validate_job_shape(pool[p]);
        if (rc != MPNL_OK)
            return rc;
        bytes[p] = mpnl::job_device_bytes(pool[p]);
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
            Job j{submitted, t_next, bytes[p], (int64_t)pool[p].S * pool[p].T, pool[p]};
            s->sched->submit(j, got);
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
            Job j{sj.id, sj.arrival_us, sj.bytes, sj.vectors, mpnl_job{}};
            sched.submit(j, got);
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
