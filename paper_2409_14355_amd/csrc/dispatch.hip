// Dispatch of the path-search launches to the user-count buckets.
#include "device_common.h"

namespace mpnl {

hipError_t path_launch_nmax8(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_nmax16(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_nmax24(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_nmax32(const dev::PathArgs &, int, int, hipStream_t);
hipError_t soft_launch_nmax8(const dev::PathArgs &, int, hipStream_t);
hipError_t soft_launch_nmax16(const dev::PathArgs &, int, hipStream_t);
hipError_t soft_launch_nmax24(const dev::PathArgs &, int, hipStream_t);
hipError_t soft_launch_nmax32(const dev::PathArgs &, int, hipStream_t);
hipError_t batch_launch_nmax8(const dev::BatchArgs &, int, int, int, hipStream_t);
hipError_t batch_launch_nmax16(const dev::BatchArgs &, int, int, int, hipStream_t);
hipError_t batch_launch_nmax24(const dev::BatchArgs &, int, int, int, hipStream_t);
hipError_t batch_launch_nmax32(const dev::BatchArgs &, int, int, int, hipStream_t);

namespace {
using namespace dev;
PathArgs path_args(const SlotDev &sd, const float2 *yt, int T, int32_t *out)
{
    PathArgs a;
    a.yt = yt;
    a.diag = sd.diag;
    a.roff = sd.roff;
    a.roffq = nullptr;
    a.permd = sd.permd;
    a.P = sd.P;
    a.out = out;
    a.llr = nullptr;
    a.S = sd.S;
    a.T = T;
    a.N = sd.N;
    a.K = sd.K;
    a.NP = sd.NP;
    a.delta = delta_of(sd.bits);
    a.sigma2 = 1.f;
    a.clip = 0.f;
    return a;
}

}  // namespace

hipError_t launch_path_search_q(const SlotDev &sd, const float2 *yt, int T, int32_t *out,
                                int precision, const uint32_t *roffq, hipStream_t st)
{
    PathArgs a = path_args(sd, yt, T, out);
    a.roffq = roffq;
    switch (nmax_bucket(sd.N)) {
    case 8: return path_launch_nmax8(a, sd.bits, precision, st);
    case 16: return path_launch_nmax16(a, sd.bits, precision, st);
    case 24: return path_launch_nmax24(a, sd.bits, precision, st);
    default: return path_launch_nmax32(a, sd.bits, precision, st);
    }
}

hipError_t launch_path_search_soft(const SlotDev &sd, const float2 *yt, int T, float sigma2,
                                   float clip, float *llr, int32_t *out, hipStream_t st)
{
    PathArgs a = path_args(sd, yt, T, out);
    a.llr = llr;
    a.sigma2 = sigma2;
    a.clip = clip;
    switch (nmax_bucket(sd.N)) {
    case 8: return soft_launch_nmax8(a, sd.bits, st);
    case 16: return soft_launch_nmax16(a, sd.bits, st);
    case 24: return soft_launch_nmax24(a, sd.bits, st);
    default: return soft_launch_nmax32(a, sd.bits, st);
    }
}

hipError_t launch_path_search_batch(const JobDev *jobs_dev, int n_jobs, int total_items,
                                    int nmax_bkt, int bits, int threads, unsigned *counter,
                                    int grid, hipStream_t st)
{
    BatchArgs a;
    a.jobs = jobs_dev;
    a.n_jobs = n_jobs;
    a.total_items = total_items;
    a.counter = counter;
    a.delta = delta_of(bits);
    switch (nmax_bkt) {
    case 8: return batch_launch_nmax8(a, bits, threads, grid, st);
    case 16: return batch_launch_nmax16(a, bits, threads, grid, st);
    case 24: return batch_launch_nmax24(a, bits, threads, grid, st);
    default: return batch_launch_nmax32(a, bits, threads, grid, st);
    }
}

}  // namespace mpnl
