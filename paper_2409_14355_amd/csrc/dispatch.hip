// Dispatch of the path-search launches to the per-user-count kernels.
#include "device_common.h"

namespace mpnl {

hipError_t path_launch_n1(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n2(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n3(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n4(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n5(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n6(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n7(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n8(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n9(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n10(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n11(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n12(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n13(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n14(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n15(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n16(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n17(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n18(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n19(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n20(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n21(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n22(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n23(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n24(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n25(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n26(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n27(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n28(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n29(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n30(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n31(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_launch_n32(const dev::PathArgs &, int, int, hipStream_t);
hipError_t soft_launch_nmax8(const dev::PathArgs &, int, hipStream_t);
hipError_t soft_launch_nmax16(const dev::PathArgs &, int, hipStream_t);
hipError_t soft_launch_nmax24(const dev::PathArgs &, int, hipStream_t);
hipError_t soft_launch_nmax32(const dev::PathArgs &, int, hipStream_t);

hipError_t path_multi_launch_n1(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n2(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n3(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n4(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n5(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n6(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n7(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n8(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n9(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n10(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n11(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n12(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n13(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n14(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n15(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n16(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n17(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n18(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n19(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n20(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n21(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n22(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n23(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n24(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n25(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n26(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n27(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n28(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n29(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n30(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n31(const dev::MultiArgs &, int, int, int, int, hipStream_t);
hipError_t path_multi_launch_n32(const dev::MultiArgs &, int, int, int, int, hipStream_t);

hipError_t path_bound_launch_n1(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n2(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n3(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n4(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n5(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n6(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n7(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n8(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n9(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n10(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n11(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n12(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n13(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n14(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n15(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n16(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n17(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n18(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n19(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n20(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n21(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n22(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n23(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n24(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n25(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n26(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n27(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n28(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n29(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n30(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n31(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_launch_n32(const dev::PathArgs &, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n1(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n2(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n3(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n4(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n5(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n6(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n7(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n8(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n9(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n10(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n11(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n12(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n13(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n14(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n15(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n16(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n17(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n18(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n19(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n20(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n21(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n22(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n23(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n24(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n25(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n26(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n27(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n28(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n29(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n30(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n31(const JobDev *, int, int, int, int, hipStream_t);
hipError_t path_bound_multi_launch_n32(const JobDev *, int, int, int, int, hipStream_t);

namespace {
using namespace dev;

typedef hipError_t (*PathLaunch)(const PathArgs &, int, int, hipStream_t);
const PathLaunch kPathLaunch[32] = {
    path_launch_n1,
    path_launch_n2,
    path_launch_n3,
    path_launch_n4,
    path_launch_n5,
    path_launch_n6,
    path_launch_n7,
    path_launch_n8,
    path_launch_n9,
    path_launch_n10,
    path_launch_n11,
    path_launch_n12,
    path_launch_n13,
    path_launch_n14,
    path_launch_n15,
    path_launch_n16,
    path_launch_n17,
    path_launch_n18,
    path_launch_n19,
    path_launch_n20,
    path_launch_n21,
    path_launch_n22,
    path_launch_n23,
    path_launch_n24,
    path_launch_n25,
    path_launch_n26,
    path_launch_n27,
    path_launch_n28,
    path_launch_n29,
    path_launch_n30,
    path_launch_n31,
    path_launch_n32};

typedef hipError_t (*MultiLaunch)(const MultiArgs &, int, int, int, int, hipStream_t);
const MultiLaunch kMultiLaunch[32] = {
    path_multi_launch_n1,
    path_multi_launch_n2,
    path_multi_launch_n3,
    path_multi_launch_n4,
    path_multi_launch_n5,
    path_multi_launch_n6,
    path_multi_launch_n7,
    path_multi_launch_n8,
    path_multi_launch_n9,
    path_multi_launch_n10,
    path_multi_launch_n11,
    path_multi_launch_n12,
    path_multi_launch_n13,
    path_multi_launch_n14,
    path_multi_launch_n15,
    path_multi_launch_n16,
    path_multi_launch_n17,
    path_multi_launch_n18,
    path_multi_launch_n19,
    path_multi_launch_n20,
    path_multi_launch_n21,
    path_multi_launch_n22,
    path_multi_launch_n23,
    path_multi_launch_n24,
    path_multi_launch_n25,
    path_multi_launch_n26,
    path_multi_launch_n27,
    path_multi_launch_n28,
    path_multi_launch_n29,
    path_multi_launch_n30,
    path_multi_launch_n31,
    path_multi_launch_n32,
};

typedef hipError_t (*BoundLaunch)(const PathArgs &, int, int, hipStream_t);
const BoundLaunch kBoundLaunch[32] = {
    path_bound_launch_n1,
    path_bound_launch_n2,
    path_bound_launch_n3,
    path_bound_launch_n4,
    path_bound_launch_n5,
    path_bound_launch_n6,
    path_bound_launch_n7,
    path_bound_launch_n8,
    path_bound_launch_n9,
    path_bound_launch_n10,
    path_bound_launch_n11,
    path_bound_launch_n12,
    path_bound_launch_n13,
    path_bound_launch_n14,
    path_bound_launch_n15,
    path_bound_launch_n16,
    path_bound_launch_n17,
    path_bound_launch_n18,
    path_bound_launch_n19,
    path_bound_launch_n20,
    path_bound_launch_n21,
    path_bound_launch_n22,
    path_bound_launch_n23,
    path_bound_launch_n24,
    path_bound_launch_n25,
    path_bound_launch_n26,
    path_bound_launch_n27,
    path_bound_launch_n28,
    path_bound_launch_n29,
    path_bound_launch_n30,
    path_bound_launch_n31,
    path_bound_launch_n32,
};

typedef hipError_t (*BoundMultiLaunch)(const JobDev *, int, int, int, int, hipStream_t);
const BoundMultiLaunch kBoundMultiLaunch[32] = {
    path_bound_multi_launch_n1,
    path_bound_multi_launch_n2,
    path_bound_multi_launch_n3,
    path_bound_multi_launch_n4,
    path_bound_multi_launch_n5,
    path_bound_multi_launch_n6,
    path_bound_multi_launch_n7,
    path_bound_multi_launch_n8,
    path_bound_multi_launch_n9,
    path_bound_multi_launch_n10,
    path_bound_multi_launch_n11,
    path_bound_multi_launch_n12,
    path_bound_multi_launch_n13,
    path_bound_multi_launch_n14,
    path_bound_multi_launch_n15,
    path_bound_multi_launch_n16,
    path_bound_multi_launch_n17,
    path_bound_multi_launch_n18,
    path_bound_multi_launch_n19,
    path_bound_multi_launch_n20,
    path_bound_multi_launch_n21,
    path_bound_multi_launch_n22,
    path_bound_multi_launch_n23,
    path_bound_multi_launch_n24,
    path_bound_multi_launch_n25,
    path_bound_multi_launch_n26,
    path_bound_multi_launch_n27,
    path_bound_multi_launch_n28,
    path_bound_multi_launch_n29,
    path_bound_multi_launch_n30,
    path_bound_multi_launch_n31,
    path_bound_multi_launch_n32,
};

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
                                    int precision, int threads, int vpw, hipStream_t st)
{
    if (N < 1 || N > 32 || threads < 64 || threads % 64 || (vpw != 1 && vpw != 2 && vpw != 4) ||
        threads * vpw > 256 || total_items < 1)
        return hipErrorInvalidValue;
    MultiArgs a;
    a.jobs = jobs_dev;
    a.n_jobs = n_jobs;
    a.total_items = total_items;
    a.vpw = vpw;
    const int grid = (total_items + vpw - 1) / vpw;
    return kMultiLaunch[N - 1](a, bits, precision, threads * vpw, grid, st);
}

}  // namespace mpnl
