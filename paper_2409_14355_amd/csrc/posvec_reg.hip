// a2 for up to 256 paths: the position-vector set kept in registers.
//
// Same definition as posvec_kernel (prep.hip): the K cheapest position
// vectors in (score, lexicographic) order, score = sum_d w_d (p_d - 1)
// accumulated in depth order in float64.  Depth by depth the list of the K
// cheapest prefixes A is extended by rank doubling:
//     U_0 = A (rank 0 at this depth),   U_{j+1} = topK(U_j  U  raise(U_j, 2^j)),
// where raise(., c) adds c to the last rank (score parent + w_d * k, always
// recomputed from the parent), so U_j holds the K cheapest extensions with
// rank below 2^j; log2 |Q| merges cover every rank.  The top K of a union is
// the top K of the unions of top Ks, which makes each step exact.
// Here every merge is a bitonic network over registers: lane l holds list
// entries g = j * 64 + l (j < E); one half-cleaner stage compares A with
// the reversed shifted list, log2(64 E) compare-exchange stages sort the K
// smallest, using register swaps for distances >= 64 and cross-lane shuffles
// below.  An entry is (score, packed) with packed = parent position (12 bits)
// | k (6 bits) << 12 | lexical rank of the parent (12 bits) << 18, so the key
// (score, parent rank, k) compares as (score, packed >> 12).
#include "device_common.h"

namespace mpnl {
namespace dev {
namespace {

constexpr uint32_t kSentinel = 0xffffffffu;

// (score, packed) entries are kept as two parallel register arrays: struct
// values would be spilled to scratch memory by the selects below.
__device__ __forceinline__ bool key_lt(double as, uint32_t ap, double bs, uint32_t bp)
{
    return as < bs || (as == bs && (ap >> 12) < (bp >> 12));
}

__device__ __forceinline__ double cand_score_r(double parent, double w, int k)
{
    return __dadd_rn(parent, __dmul_rn(w, (double)k));
}

// Sort a bitonic sequence of 64 E entries ascending.
template <int E>
__device__ __forceinline__ void bitonic_finish(double (&cs)[E], uint32_t (&cp)[E], int lane)
{
#pragma unroll
    for (int js = E / 2; js >= 1; js >>= 1) {
#pragma unroll
        for (int j = 0; j < E; ++j)
            if ((j & js) == 0) {
                const double ls = cs[j], hs = cs[j + js];
                const uint32_t lp = cp[j], hp = cp[j + js];
                const bool sw = key_lt(hs, hp, ls, lp);
                cs[j] = sw ? hs : ls;
                cp[j] = sw ? hp : lp;
                cs[j + js] = sw ? ls : hs;
                cp[j + js] = sw ? lp : hp;
            }
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        const bool lower = (lane & s) == 0;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const double os = __shfl_xor(cs[j], s);
            const uint32_t op = __shfl_xor(cp[j], s);
            const bool take = lower == key_lt(os, op, cs[j], cp[j]);
            cs[j] = take ? os : cs[j];
            cp[j] = take ? op : cp[j];
        }
    }
}

// Full ascending bitonic sort of 64 E entries (entry g = j * 64 + lane).
template <int E>
__device__ __forceinline__ void bitonic_sort_full(double (&cs)[E], uint32_t (&cp)[E], int lane)
{
    constexpr int KP = 64 * E;
#pragma unroll
    for (int size = 2; size <= KP; size <<= 1) {
#pragma unroll
        for (int stride = size / 2; stride >= 1; stride >>= 1) {
            if (stride >= 64) {
                const int js = stride / 64;
#pragma unroll
                for (int j = 0; j < E; ++j)
                    if ((j & js) == 0) {
                        const bool asc = ((j * 64) & size) == 0;
                        const double ls = cs[j], hs = cs[j + js];
                        const uint32_t lp = cp[j], hp = cp[j + js];
                        const bool sw = asc == key_lt(hs, hp, ls, lp);
                        cs[j] = sw ? hs : ls;
                        cp[j] = sw ? hp : lp;
                        cs[j + js] = sw ? ls : hs;
                        cp[j + js] = sw ? lp : hp;
                    }
            } else {
                const bool lower = (lane & stride) == 0;
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    const bool asc = ((j * 64 + lane) & size) == 0;
                    const double os = __shfl_xor(cs[j], stride);
                    const uint32_t op = __shfl_xor(cp[j], stride);
                    const bool take = (lower == asc) == key_lt(os, op, cs[j], cp[j]);
                    cs[j] = take ? os : cs[j];
                    cp[j] = take ? op : cp[j];
                }
            }
        }
    }
}

template <int E>
__device__ __forceinline__ void posvec_body(const PosArgs &a, int s, unsigned char *smem)
{
    constexpr int KP = 64 * E;
    constexpr double INF = (double)INFINITY;
    double *scA = (double *)smem;             // KP: scores of list A by position
    uint32_t *cnt = (uint32_t *)(scA + KP);  // KP: children per parent rank
    uint32_t *rec = cnt + KP;                 // N * KP: (parent, k) per depth
    const int lane = threadIdx.x;
    const int K = a.K, N = a.N, nq = a.nq;
    const int jK = (K - 1) >> 6, lK = (K - 1) & 63;  // slot of entry K-1

    double As[E];
    uint32_t Ap[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int g = j * 64 + lane;
        As[j] = g == 0 ? 0.0 : INF;
        Ap[j] = g == 0 ? 0u : kSentinel;
        scA[g] = As[j];
    }
    __syncthreads();

    for (int d = 0; d < N; ++d) {
        const double w = a.w[(size_t)s * N + d];
        double Zs[E];
        uint32_t Zp[E];
#pragma unroll
        for (int j = 0; j < E; ++j) {
            Zs[j] = As[j];
            Zp[j] = Ap[j];
        }
        const double a0s = __shfl(As[0], 0);
        const uint32_t a0p = __shfl(Ap[0], 0);
        // Z covers the ranks k < span of this depth; merging Z with its copy
        // raised by span covers k < 2 span (|Q| is a power of two, so the
        // raised ranks never pass |Q| - 1)
        for (int span = 1; span < nq; span <<= 1) {
            // stop when the cheapest entry with rank span can no longer
            // enter a full list
            double ls = Zs[0];
            uint32_t lp = Zp[0];
#pragma unroll
            for (int j = 1; j < E; ++j) {
                ls = (j == jK) ? Zs[j] : ls;
                lp = (j == jK) ? Zp[j] : lp;
            }
            ls = __shfl(ls, lK);
            lp = __shfl(lp, lK);
            if (ls < INF) {
                const double cs = cand_score_r(a0s, w, span);
                const uint32_t cpk = (a0p & 0xfffc0fffu) | ((uint32_t)span << 12);
                if (!key_lt(cs, cpk, ls, lp))
                    break;
            }
            double Bs[E];
            uint32_t Bp[E];
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const bool ok = Zs[j] < INF;
                const int par = Zp[j] & 0xfff;
                const int k1 = ((Zp[j] >> 12) & 63) + span;
                Bs[j] = ok ? cand_score_r(scA[ok ? par : 0], w, k1) : INF;
                Bp[j] = ok ? Zp[j] + ((uint32_t)span << 12) : kSentinel;
            }
            // half cleaner: entry g of Z against entry KP-1-g of B
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const double rs = __shfl_xor(Bs[E - 1 - j], 63);
                const uint32_t rp = __shfl_xor(Bp[E - 1 - j], 63);
                const bool tb = key_lt(rs, rp, Zs[j], Zp[j]);
                Zs[j] = tb ? rs : Zs[j];
                Zp[j] = tb ? rp : Zp[j];
            }
            bitonic_finish<E>(Zs, Zp, lane);
#pragma unroll
            for (int j = 0; j < E; ++j)
                if (j * 64 + lane >= K) {
                    Zs[j] = INF;
                    Zp[j] = kSentinel;
                }
        }
        // lexical ranks of the new prefixes: the children of a parent are
        // k = 0..c-1, consecutive in lexical order
#pragma unroll
        for (int j = 0; j < E; ++j)
            cnt[j * 64 + lane] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < E; ++j)
            if (Zs[j] < INF)
                atomicMax(&cnt[Zp[j] >> 18], ((Zp[j] >> 12) & 63) + 1);
        __syncthreads();
        {
            uint32_t v[E], local = 0;
#pragma unroll
            for (int j = 0; j < E; ++j) {
                v[j] = cnt[lane * E + j];
                local += v[j];
            }
            uint32_t incl = local;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t t = __shfl_up(incl, off);
                if (lane >= off)
                    incl += t;
            }
            uint32_t run = incl - local;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < E; ++j) {
                cnt[lane * E + j] = run;
                run += v[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int g = j * 64 + lane;
            if (Zs[j] < INF) {
                const uint32_t k = (Zp[j] >> 12) & 63;
                const uint32_t lx = cnt[Zp[j] >> 18] + k;
                rec[(size_t)d * KP + g] = (Zp[j] & 0xfff) | (k << 16);
                As[j] = Zs[j];
                Ap[j] = (uint32_t)g | (lx << 18);
            } else {
                As[j] = INF;
                Ap[j] = kSentinel;
            }
            scA[g] = As[j];
        }
        __syncthreads();
    }

    // rebuild the position vectors (ranks 1..|Q|), rows padded with 1, and
    // note for each which depths ask for a rank >= 3 and >= 2
    const int nw = a.NP >> 2;
    double ks[E];
    uint32_t kr[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int r = j * 64 + lane;
        ks[j] = INF;
        kr[j] = (uint32_t)r << 12;
        if (r >= K)
            continue;
        uint32_t wv[kMaxN / 4];
#pragma unroll
        for (int w = 0; w < kMaxN / 4; ++w)
            wv[w] = 0x01010101u;
        uint32_t m3 = 0, m2 = 0;
        int pidx = r;
        for (int d = N - 1; d >= 0; --d) {
            const uint32_t e = rec[(size_t)d * KP + pidx];
            const uint32_t pk = (e >> 16) + 1u;
            pidx = (int)(e & 0xffffu);
            m3 |= (pk >= 3u ? 1u : 0u) << d;
            m2 |= (pk >= 2u ? 1u : 0u) << d;
#pragma unroll
            for (int w = 0; w < kMaxN / 4; ++w)
                if (w == (d >> 2))
                    wv[w] = (wv[w] & ~(0xffu << ((d & 3) * 8))) | (pk << ((d & 3) * 8));
        }
        uint32_t *dst = (uint32_t *)(a.P + ((size_t)s * a.K + r) * a.NP);
#pragma unroll
        for (int w = 0; w < kMaxN / 4; ++w)
            if (w < nw)
                dst[w] = wv[w];
        // sort key: depths with rank >= 3 first, then depths with rank >= 2
        // (as a double the low bits of the second mask may round; the key
        // only groups paths, any order is correct)
        ks[j] = (double)m3 * 4294967296.0 + (double)m2;
    }
    // Lane order: paths sorted by that key, so that the lanes of one
    // wavefront need the costly point choices at the same depths.
    // order[i] = path run by lane i.
    if (a.order != nullptr) {
        bitonic_sort_full<E>(ks, kr, lane);
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int g = j * 64 + lane;
            if (g < K)
                a.order[(size_t)s * K + g] = (uint16_t)(kr[j] >> 12);
        }
    }
}

template <int E>
__global__ __launch_bounds__(64) void posvec_reg_kernel(PosArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    posvec_body<E>(a, blockIdx.x, smem);
}

// One launch for the position sets of many jobs (all with N_p <= 64 E):
// workgroup b runs subcarrier b - item_begin of the job that owns item b.
template <int E>
__global__ __launch_bounds__(64) void posvec_batch_kernel(const StageJob *jobs, int n_jobs)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const StageJob &j = jobs[find_job(jobs, n_jobs, blockIdx.x)];
    PosArgs a;
    a.w = j.sd.wd;
    a.S = j.sd.S;
    a.N = j.sd.N;
    a.nq = 1 << j.sd.bits;
    a.K = j.sd.K;
    a.NP = j.sd.NP;
    a.P = j.sd.P;
    a.rec_g = nullptr;
    a.order = j.sd.order;
    posvec_body<E>(a, blockIdx.x - j.item_begin, smem);
}

}  // namespace
}  // namespace dev

size_t posvec_reg_lds_bytes(int N, int K)
{
    const int KP = K <= 64 ? 64 : K <= 128 ? 128 : 256;
    return (size_t)KP * (sizeof(double) + sizeof(uint32_t)) + (size_t)N * KP * sizeof(uint32_t);
}

hipError_t launch_posvec_batch(const dev::StageJob *jobs, int n_jobs, int items, int E, int Nmax,
                               hipStream_t st)
{
    using namespace dev;
    const size_t lds = posvec_reg_lds_bytes(Nmax, 64 * E);
    if (E == 1)
        hipLaunchKernelGGL(posvec_batch_kernel<1>, dim3(items), dim3(64), lds, st, jobs, n_jobs);
    else if (E == 2)
        hipLaunchKernelGGL(posvec_batch_kernel<2>, dim3(items), dim3(64), lds, st, jobs, n_jobs);
    else if (E == 4)
        hipLaunchKernelGGL(posvec_batch_kernel<4>, dim3(items), dim3(64), lds, st, jobs, n_jobs);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_posvec_reg(const dev::PosArgs &a, hipStream_t st)
{
    using namespace dev;
    const size_t lds = posvec_reg_lds_bytes(a.N, a.K);
    if (a.K <= 64)
        hipLaunchKernelGGL(posvec_reg_kernel<1>, dim3(a.S), dim3(64), lds, st, a);
    else if (a.K <= 128)
        hipLaunchKernelGGL(posvec_reg_kernel<2>, dim3(a.S), dim3(64), lds, st, a);
    else if (a.K <= 256)
        hipLaunchKernelGGL(posvec_reg_kernel<4>, dim3(a.S), dim3(64), lds, st, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace mpnl
