// Dispatch of the path-search launches to the per-user-count kernels.
#include "device_common.h"

namespace mpnl {

// One launcher per user count 1..32 of each kind (defined in path_n<N>.hip and
// path_bucket<NMAX>.hip); the tables below are indexed by N - 1.
#define MPNL_FOR_N(X)                                                                                   \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) \
        X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

#define MPNL_DECLARE(n)                                                                 \
    hipError_t path_launch_n##n(const dev::PathArgs &, int, int, hipStream_t);          \
    hipError_t path_multi_launch_n##n(const dev::MultiArgs &, int, int, int, dim3, hipStream_t); \
    hipError_t path_bound_launch_n##n(const dev::PathArgs &, int, int, hipStream_t);    \
    hipError_t path_bound_multi_launch_n##n(const JobDev *, int, int, int, int, hipStream_t);
MPNL_FOR_N(MPNL_DECLARE)
#undef MPNL_DECLARE
hipError_t soft_launch_nmax8(const dev::PathArgs &, int, hipStream_t);
hipError_t soft_launch_nmax16(const dev::PathArgs &, int, hipStream_t);
hipError_t soft_launch_nmax24(const dev::PathArgs &, int, hipStream_t);
hipError_t soft_launch_nmax32(const dev::PathArgs &, int, hipStream_t);

namespace {

using namespace dev;

typedef hipError_t (*PathLaunch)(const PathArgs &, int, int, hipStream_t);
typedef hipError_t (*MultiLaunch)(const MultiArgs &, int, int, int, dim3, hipStream_t);
typedef hipError_t (*BoundLaunch)(const PathArgs &, int, int, hipStream_t);
typedef hipError_t (*BoundMultiLaunch)(const JobDev *, int, int, int, int, hipStream_t);

#define MPNL_ENTRY(n) path_launch_n##n,
const PathLaunch kPathLaunch[32] = {MPNL_FOR_N(MPNL_ENTRY)};
#undef MPNL_ENTRY
#define MPNL_ENTRY(n) path_multi_launch_n##n,
const MultiLaunch kMultiLaunch[32] = {MPNL_FOR_N(MPNL_ENTRY)};
#undef MPNL_ENTRY
#define MPNL_ENTRY(n) path_bound_launch_n##n,
const BoundLaunch kBoundLaunch[32] = {MPNL_FOR_N(MPNL_ENTRY)};
#undef MPNL_ENTRY
#define MPNL_ENTRY(n) path_bound_multi_launch_n##n,
const BoundMultiLaunch kBoundMultiLaunch[32] = {MPNL_FOR_N(MPNL_ENTRY)};
#undef MPNL_ENTRY
#undef MPNL_FOR_N

PathArgs path_args(const SlotDev &sd, const float2 *yt, int T, int32_t *out)
{
    PathArgs a;
    a.yt = yt;
    a.diag = sd.diag;
    a.rlat = sd.rlat;
    a.rq = nullptr;
    a.permd = sd.permd;
    a.P = sd.P;
    a.order = sd.order;
    a.out = out;
    a.llr = nullptr;
    a.part = nullptr;
    a.bound = nullptr;
    a.S = sd.S;
    a.T = T;
    a.N = sd.N;
    a.K = sd.K;
    a.NP = sd.NP;
    a.sigma2 = 1.f;
    a.clip = 0.f;
    return a;
}

}  // namespace

int nmax_bucket(int N)
{
    return N <= 8 ? 8 : N <= 16 ? 16 : N <= 24 ? 24 : 32;
}

size_t path_partial_bytes(const SlotDev &sd, int T)
{
    const int groups = (sd.K + 63) / 64;
    if (groups <= 1)
        return 0;
    return (size_t)sd.S * T * groups * (2 + (sd.N + 3) / 4) * sizeof(float);
}

hipError_t launch_path_search(const SlotDev &sd, const float2 *yt, int T, int32_t *out,
                              int precision, float *part, float *bound, hipStream_t st)
{
    if (sd.N < 1 || sd.N > 32)
        return hipErrorInvalidValue;
    PathArgs a = path_args(sd, yt, T, out);
    a.rq = precision == PREC_FP16 ? sd.rlat_h : precision == PREC_BF16 ? sd.rlat_b : nullptr;
    a.bound = bound;
    const int groups = (sd.K + 63) / 64;
    if (groups > 1) {
        if (part == nullptr)
            return hipErrorInvalidValue;
        a.part = part;
    }
    if ((long long)sd.S * T * groups > INT_MAX)
        return hipErrorInvalidValue;
    // one-wavefront path groups, one a workgroup, group major on a 2-D grid
    // (measured on MI355X, 16 users x 1200 x 14, 256 paths: 0.085 ms; the
    // same numbered vector major took 0.150 ms, and needed four items a
    // workgroup to reach 0.095 ms; 24 users x 3276 x 14: 0.243 ms)
    hipError_t e = kPathLaunch[sd.N - 1](a, sd.bits, precision, st);
    if (e != hipSuccess || groups <= 1)
        return e;
    const int vecs = sd.S * T;
    const dim3 grid((vecs + 63) / 64), block(64);  // one lane a vector; many small workgroups spread the loads
    if (sd.bits == 2)
        hipLaunchKernelGGL(path_group_reduce_kernel<2>, grid, block, 0, st, a, groups);
    else if (sd.bits == 4)
        hipLaunchKernelGGL(path_group_reduce_kernel<4>, grid, block, 0, st, a, groups);
    else
        hipLaunchKernelGGL(path_group_reduce_kernel<8>, grid, block, 0, st, a, groups);
    return hipGetLastError();
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

hipError_t launch_path_bound(const SlotDev &sd, const float2 *yt, int T, int precision, float *bound,
                             hipStream_t st)
{
    if (sd.N < 1 || sd.N > 32 || bound == nullptr)
        return hipErrorInvalidValue;
    PathArgs a = path_args(sd, yt, T, nullptr);
    a.rq = precision == PREC_FP16 ? sd.rlat_h : precision == PREC_BF16 ? sd.rlat_b : nullptr;
    a.bound = bound;
    return kBoundLaunch[sd.N - 1](a, sd.bits, precision, st);
}

hipError_t launch_path_bound_multi(const JobDev *jobs_dev, int n_jobs, int bound_items, int N, int bits,
                                   int precision, hipStream_t st)
{
    if (N < 1 || N > 32 || bound_items < 1)
        return hipErrorInvalidValue;
    return kBoundMultiLaunch[N - 1](jobs_dev, n_jobs, bound_items, bits, precision, st);
}

hipError_t launch_path_search_multi(const JobDev *jobs_dev, int n_jobs, int total_items, int N, int bits,
                                    int precision, int threads, int groups, int ipw, int gmajor, hipStream_t st)
{
    if (N < 1 || N > 32 || threads < 64 || threads > 256 || threads % 64 || groups < 1 || threads % groups ||
        (threads / groups) % 64 || (ipw != 1 && ipw != 2 && ipw != 4) || ipw * (threads / groups) > 256 ||
        total_items < 1)
        return hipErrorInvalidValue;
    MultiArgs a;
    a.jobs = jobs_dev;
    a.n_jobs = n_jobs;
    a.total_items = total_items;
    a.ipw = ipw;
    a.gw = threads / groups;
    a.groups = groups;
    a.gmajor = gmajor;
    const long long nvb = ((long long)total_items + ipw - 1) / ipw;  // workgroups per path group
    if (nvb * groups > INT_MAX)
        return hipErrorInvalidValue;
    // group major: grid (workgroups per group, groups); vector major: 1-D
    const dim3 grid = gmajor ? dim3((unsigned)nvb, (unsigned)groups) : dim3((unsigned)(nvb * groups));
    hipError_t e = kMultiLaunch[N - 1](a, bits, precision, ipw * a.gw, grid, st);
    if (e != hipSuccess || groups == 1)
        return e;
    const dim3 rgrid((total_items + 63) / 64), rblock(64);  // one lane a vector
    if (bits == 2)
        hipLaunchKernelGGL(path_group_reduce_multi_kernel<2>, rgrid, rblock, 0, st, a);
    else if (bits == 4)
        hipLaunchKernelGGL(path_group_reduce_multi_kernel<4>, rgrid, rblock, 0, st, a);
    else
        hipLaunchKernelGGL(path_group_reduce_multi_kernel<8>, rgrid, rblock, 0, st, a);
    return hipGetLastError();
}

}  // namespace mpnl
