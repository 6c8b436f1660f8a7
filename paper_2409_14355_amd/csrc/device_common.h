// Device code shared by the kernel translation units of the MPNL library
// (helpers, the a4 point choice and the path-search kernel templates).
#pragma once
#include "kernels.h"

#include <float.h>
#include <limits.h>
#include <math.h>

namespace mpnl {
namespace dev {

constexpr int kMaxN = 32;

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf162_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int gray_code(int m) { return m ^ (m >> 1); }
__device__ __forceinline__ int gray_decode(int g) { return g ^ (g >> 1) ^ (g >> 2); }

template <int L>
struct Axis {
    static constexpr int HB = (L == 2) ? 1 : (L == 4) ? 2 : 3;  // bits per axis
};

// Hardware dispatches consecutive workgroup ids round-robin over the 8 XCDs
// (each with its own L2).  Give every XCD a contiguous range of logical block
// ids so that the blocks of one subcarrier (its R, P and yt) share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks)
{
    constexpr int X = 8;
    const int xcd = bid % X, local = bid / X;
    const int q = nblocks / X, rem = nblocks % X;
    return xcd * q + min(xcd, rem) + local;
}

// ============================================================================
// a4: choice of the k-th closest constellation point at one depth.
// Distances are taken per axis, e(m) = (u - (2m - L + 1) a)^2 with
// a = R_ll * Delta, so |b - R_ll c|^2 = e_I(mI) + e_Q(mQ).  Order: distance,
// then constellation index (gray(mI) << HB | gray(mQ)).
// ============================================================================
template <int L>
__device__ __forceinline__ float axis_err(float u, float a, int m)
{
    const float dlt = fmaf(-(float)(2 * m - (L - 1)), a, u);
    return dlt * dlt;
}

template <int L>
__device__ __forceinline__ int axis_nearest(float u, float a, float inv2a, float &e)
{
    float pos = fmaf(u, inv2a, 0.5f * (float)(L - 1));
    pos = fminf(fmaxf(pos, 0.f), (float)(L - 1));
    const int m0 = (int)floorf(pos);
    const int m1 = min(m0 + 1, L - 1);
    const float e0 = axis_err<L>(u, a, m0), e1 = axis_err<L>(u, a, m1);
    const bool t1 = (e1 < e0) || (e1 == e0 && gray_code(m1) < gray_code(m0));
    e = t1 ? e1 : e0;
    return t1 ? m1 : m0;
}

// second closest level on one axis: the better neighbour of the closest
template <int L>
__device__ __forceinline__ int axis_second(float u, float a, int m0, float &e)
{
    const int lo = m0 - 1, hi = m0 + 1;
    const float elo = lo >= 0 ? axis_err<L>(u, a, lo) : INFINITY;
    const float ehi = hi < L ? axis_err<L>(u, a, hi) : INFINITY;
    bool take_hi;
    if (lo < 0)
        take_hi = true;
    else if (hi >= L)
        take_hi = false;
    else
        take_hi = (ehi < elo) || (ehi == elo && gray_code(hi) < gray_code(lo));
    e = take_hi ? ehi : elo;
    return take_hi ? hi : lo;
}

template <int L>
__device__ __noinline__ void kth_general(float2 b, float a, float inv2a, int k, int &mI, int &mQ,
                                         float &dist)
{
    constexpr int HB = Axis<L>::HB;
    // quadrature axis sorted by (distance, gray label): two-pointer zig-zag
    float eq0;
    const int mq0 = axis_nearest<L>(b.y, a, inv2a, eq0);
    int ordQ[L], gQ[L];
    float eQ[L];
    ordQ[0] = mq0;
    eQ[0] = eq0;
    int lo = mq0 - 1, hi = mq0 + 1;
#pragma unroll
    for (int t = 1; t < L; ++t) {
        const float elo = lo >= 0 ? axis_err<L>(b.y, a, lo) : INFINITY;
        const float ehi = hi < L ? axis_err<L>(b.y, a, hi) : INFINITY;
        bool take_hi;
        if (lo < 0)
            take_hi = true;
        else if (hi >= L)
            take_hi = false;
        else
            take_hi = (ehi < elo) || (ehi == elo && gray_code(hi) < gray_code(lo));
        ordQ[t] = take_hi ? hi : lo;
        eQ[t] = take_hi ? ehi : elo;
        hi += take_hi ? 1 : 0;
        lo -= take_hi ? 0 : 1;
    }
#pragma unroll
    for (int t = 0; t < L; ++t)
        gQ[t] = gray_code(ordQ[t]);
    // one sorted row per in-phase level; L-way merge of the rows
    float eI[L], cand[L];
    int gI[L], ptr[L], cidx[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        eI[i] = axis_err<L>(b.x, a, i);
        gI[i] = gray_code(i) << HB;
        ptr[i] = 0;
        cand[i] = eI[i] + eQ[0];
        cidx[i] = gI[i] | gQ[0];
    }
    int bi = 0;
    float bc = cand[0];
    for (int step = 0;; ++step) {
        bi = 0;
        bc = cand[0];
        int bx = cidx[0];
#pragma unroll
        for (int i = 1; i < L; ++i) {
            const bool lt = cand[i] < bc || (cand[i] == bc && cidx[i] < bx);
            bi = lt ? i : bi;
            bc = lt ? cand[i] : bc;
            bx = lt ? cidx[i] : bx;
        }
        if (step >= k - 1 || step >= L * L - 1)
            break;
        int p = 0, gi = 0;
        float ei = 0.f;
#pragma unroll
        for (int i = 0; i < L; ++i)
            if (i == bi) {
                p = ptr[i];
                ei = eI[i];
                gi = gI[i];
            }
        ++p;
        float eq = INFINITY;
        int gq = 0;
#pragma unroll
        for (int t = 0; t < L; ++t)
            if (t == p) {
                eq = eQ[t];
                gq = gQ[t];
            }
        const float nc = ei + eq;
#pragma unroll
        for (int i = 0; i < L; ++i)
            if (i == bi) {
                ptr[i] = p;
                cand[i] = nc;
                cidx[i] = gi | gq;
            }
    }
    int pp = 0;
#pragma unroll
    for (int i = 0; i < L; ++i)
        if (i == bi)
            pp = ptr[i];
    int mq = 0;
#pragma unroll
    for (int t = 0; t < L; ++t)
        if (t == pp)
            mq = ordQ[t];
    mI = bi;
    mQ = mq;
    dist = bc;
}

template <int L>
__device__ __forceinline__ void select_point(float2 b, float a, float inv2a, int k, int &mI, int &mQ,
                                             float &dist)
{
    constexpr int HB = Axis<L>::HB;
    if (a == 0.f) {  // R_ll = 0: every point is equally far; index order decides
        const int idx = min(max(k - 1, 0), L * L - 1);
        mI = gray_decode(idx >> HB);
        mQ = gray_decode(idx & (L - 1));
        dist = b.x * b.x + b.y * b.y;
        return;
    }
    float eI0, eQ0;
    const int mI0 = axis_nearest<L>(b.x, a, inv2a, eI0);
    const int mQ0 = axis_nearest<L>(b.y, a, inv2a, eQ0);
    if (k <= 1) {
        mI = mI0;
        mQ = mQ0;
        dist = eI0 + eQ0;
    } else if (k == 2) {
        float eI1, eQ1;
        const int mI1 = axis_second<L>(b.x, a, mI0, eI1);
        const int mQ1 = axis_second<L>(b.y, a, mQ0, eQ1);
        const float cA = eI0 + eQ1;  // (closest I, second Q)
        const float cB = eI1 + eQ0;  // (second I, closest Q)
        const int iA = (gray_code(mI0) << HB) | gray_code(mQ1);
        const int iB = (gray_code(mI1) << HB) | gray_code(mQ0);
        const bool tb = (cB < cA) || (cB == cA && iB < iA);
        mI = tb ? mI1 : mI0;
        mQ = tb ? mQ0 : mQ1;
        dist = tb ? cB : cA;
    } else {
        kth_general<L>(b, a, inv2a, k, mI, mQ, dist);
    }
}

// ============================================================================
// a4 + a5: path search.
// ============================================================================
struct PathArgs {
    const float2 *yt;       // (T, S, N)
    const float4 *diag;     // (S, N)
    const float2 *roff;     // (S, N, N)
    const uint32_t *roffq;  // (S, N, N) half2 / bf16x2 of R * Delta, or null
    const int32_t *permd;   // (S, N)
    const uint8_t *P;       // (S, K, NP)
    int32_t *out;           // (T, S, N)
    float *llr;             // (T, S, N, bits) or null
    int S, T, N, K, NP;
    float delta, sigma2, clip;
};

enum { PREC_FP32 = 0, PREC_FP16 = 1, PREC_BF16 = 2 };

// One SIC descent driven by the position vector in pw.  Residuals b[e] for
// the depths e not yet decided are updated right after each decision
// (b_e -= R_{l_e, l_d} s_d).  Returns the accumulated metric; the chosen
// constellation indices are packed four per word into dec.
template <int NMAX, int L, int PREC>
__device__ __forceinline__ float descend(const float2 *__restrict__ yv, const float4 *__restrict__ dg,
                                        const float2 *__restrict__ roff,
                                        const uint32_t *__restrict__ roffq, int N,
                                        const uint32_t *pw, uint32_t *dec, float delta)
{
    constexpr int HB = Axis<L>::HB;
    float2 b[NMAX];
#pragma unroll
    for (int d = 0; d < NMAX; ++d)
        if (d < N)
            b[d] = yv[d];
    float metric = 0.f;
#pragma unroll
    for (int d = 0; d < NMAX; ++d) {
        if (d < N) {
        const int k = (pw[d >> 2] >> ((d & 3) * 8)) & 0xff;
        const float4 g = dg[d];
        int mI, mQ;
        float dist;
        select_point<L>(b[d], g.y, g.z, k, mI, mQ, dist);
        metric += dist;
        const int idx = (gray_code(mI) << HB) | gray_code(mQ);
        dec[d >> 2] |= (uint32_t)idx << ((d & 3) * 8);
        const int lI = 2 * mI - (L - 1), lQ = 2 * mQ - (L - 1);
        if constexpr (PREC == PREC_FP32) {
            const float sI = (float)lI * delta, sQ = (float)lQ * delta;
#pragma unroll
            for (int e = d + 1; e < NMAX; ++e) {
                if (e < N) {
                    const float2 r = roff[d * N + e];
                    b[e].x = fmaf(-r.x, sI, b[e].x);
                    b[e].x = fmaf(r.y, sQ, b[e].x);
                    b[e].y = fmaf(-r.x, sQ, b[e].y);
                    b[e].y = fmaf(-r.y, sI, b[e].y);
                }
            }
        } else if constexpr (PREC == PREC_FP16) {
            half2_t sa, sb;  // (-sI, sQ) and (-sQ, -sI) as exact small integers
            sa.x = (_Float16)(float)(-lI);
            sa.y = (_Float16)(float)(lQ);
            sb.x = (_Float16)(float)(-lQ);
            sb.y = (_Float16)(float)(-lI);
#pragma unroll
            for (int e = d + 1; e < NMAX; ++e) {
                if (e < N) {
                    const half2_t r = __builtin_bit_cast(half2_t, roffq[d * N + e]);
                    b[e].x = __builtin_amdgcn_fdot2(r, sa, b[e].x, false);
                    b[e].y = __builtin_amdgcn_fdot2(r, sb, b[e].y, false);
                }
            }
        } else {
            bf162_t sa, sb;
            sa.x = (__bf16)(float)(-lI);
            sa.y = (__bf16)(float)(lQ);
            sb.x = (__bf16)(float)(-lQ);
            sb.y = (__bf16)(float)(-lI);
#pragma unroll
            for (int e = d + 1; e < NMAX; ++e) {
                if (e < N) {
                    const bf162_t r = __builtin_bit_cast(bf162_t, roffq[d * N + e]);
                    b[e].x = __builtin_amdgcn_fdot2_f32_bf16(r, sa, b[e].x, false);
                    b[e].y = __builtin_amdgcn_fdot2_f32_bf16(r, sb, b[e].y, false);
                }
            }
        }
        }
    }
    return (metric == metric) ? metric : INFINITY;
}

__device__ __forceinline__ bool better(float m, int r, float bm, int br)
{
    return m < bm || (m == bm && r < br);
}

template <int NMAX, int L, int PREC>
__global__ __launch_bounds__(256) void path_search_kernel(PathArgs a)
{
    constexpr int NW = NMAX / 4;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int s = lb / a.T, t = lb - s * a.T;
    const int N = a.N;
    const float2 *yv = a.yt + ((size_t)t * a.S + s) * N;
    const float4 *dg = a.diag + (size_t)s * N;
    const float2 *roff = a.roff + (size_t)s * N * N;
    const uint32_t *roffq = a.roffq ? a.roffq + (size_t)s * N * N : nullptr;
    const int nw = a.NP >> 2;
    const uint32_t *Pw = (const uint32_t *)(a.P + (size_t)s * a.K * a.NP);

    float bm = INFINITY;
    int br = INT_MAX;
    uint32_t bdec[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w)
        bdec[w] = 0;
    for (int r = threadIdx.x; r < a.K; r += blockDim.x) {
        uint32_t pw[NW], dec[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            pw[w] = (w < nw) ? Pw[(size_t)r * nw + w] : 0x01010101u;
            dec[w] = 0;
        }
        const float m = descend<NMAX, L, PREC>(yv, dg, roff, roffq, N, pw, dec, a.delta);
        if (better(m, r, bm, br)) {
            bm = m;
            br = r;
#pragma unroll
            for (int w = 0; w < NW; ++w)
                bdec[w] = dec[w];
        }
    }
    // a5: minimum metric over the workgroup (equal metrics: lowest path)
    float wm = bm;
    int wr = br;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float om = __shfl_xor(wm, off);
        const int orr = __shfl_xor(wr, off);
        if (better(om, orr, wm, wr)) {
            wm = om;
            wr = orr;
        }
    }
    __shared__ float sm[4];
    __shared__ int sr[4];
    const int wid = threadIdx.x >> 6;
    const int nwv = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) {
        sm[wid] = wm;
        sr[wid] = wr;
    }
    __syncthreads();
    float gm = sm[0];
    int gr = sr[0];
    for (int w = 1; w < nwv; ++w)
        if (better(sm[w], sr[w], gm, gr)) {
            gm = sm[w];
            gr = sr[w];
        }
    if (br == gr) {
        int32_t *o = a.out + ((size_t)t * a.S + s) * N;
        const int32_t *pm = a.permd + (size_t)s * N;
#pragma unroll
        for (int d = 0; d < NMAX; ++d) {
            if (d < N) {
                const int u = pm[d];
                if ((unsigned)u < (unsigned)N)  // permd is a permutation for finite inputs
                    o[u] = (int32_t)((bdec[d >> 2] >> ((d & 3) * 8)) & 0xffu);
            }
        }
    }
}

// ============================================================================
// a4 + a5 with max-log soft output: every path's metric and symbols go to
// LDS; for each (user, bit) the smallest metric with the bit at 0 and at 1
// is found by one lane scanning the K paths.
// ============================================================================
template <int NMAX, int L>
__global__ __launch_bounds__(256) void path_search_soft_kernel(PathArgs a)
{
    constexpr int NW = NMAX / 4;
    constexpr int HB = Axis<L>::HB;
    constexpr int BITS = 2 * HB;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int s = lb / a.T, t = lb - s * a.T;
    const int N = a.N, K = a.K;
    const float2 *yv = a.yt + ((size_t)t * a.S + s) * N;
    const float4 *dg = a.diag + (size_t)s * N;
    const float2 *roff = a.roff + (size_t)s * N * N;
    const int nw = a.NP >> 2;
    const uint32_t *Pw = (const uint32_t *)(a.P + (size_t)s * K * a.NP);
    float *mets = (float *)smem;                   // K
    uint32_t *decs = (uint32_t *)(mets + K);       // K * NW

    for (int r = threadIdx.x; r < K; r += blockDim.x) {
        uint32_t pw[NW], dec[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            pw[w] = (w < nw) ? Pw[(size_t)r * nw + w] : 0x01010101u;
            dec[w] = 0;
        }
        mets[r] = descend<NMAX, L, PREC_FP32>(yv, dg, roff, nullptr, N, pw, dec, a.delta);
#pragma unroll
        for (int w = 0; w < NW; ++w)
            decs[(size_t)r * NW + w] = dec[w];
    }
    __syncthreads();
    const int32_t *pm = a.permd + (size_t)s * N;
    const size_t vbase = ((size_t)t * a.S + s) * N;
    for (int q = threadIdx.x; q < N * BITS; q += blockDim.x) {
        const int d = q / BITS, bit = q - d * BITS;
        float m0 = INFINITY, m1 = INFINITY;
        for (int r = 0; r < K; ++r) {
            const int idx = (decs[(size_t)r * NW + (d >> 2)] >> ((d & 3) * 8)) & 0xff;
            const float m = mets[r];
            if ((idx >> (BITS - 1 - bit)) & 1)
                m1 = fminf(m1, m);
            else
                m0 = fminf(m0, m);
        }
        float v;
        if (m1 == INFINITY)
            v = a.clip;
        else if (m0 == INFINITY)
            v = -a.clip;
        else
            v = fminf(fmaxf((m1 - m0) / a.sigma2, -a.clip), a.clip);
        const int u = pm[d];
        if ((unsigned)u < (unsigned)N)
            a.llr[(vbase + u) * BITS + bit] = v;
    }
    if (a.out != nullptr && threadIdx.x == 0) {
        float bm = INFINITY;
        int br = 0;
        for (int r = 0; r < K; ++r)
            if (mets[r] < bm) {
                bm = mets[r];
                br = r;
            }
        for (int d = 0; d < N; ++d) {
            const int u = pm[d];
            if ((unsigned)u < (unsigned)N)
                a.out[vbase + u] = (int32_t)((decs[(size_t)br * NW + (d >> 2)] >> ((d & 3) * 8)) & 0xffu);
        }
    }
}

// ============================================================================
// Batched path search: one persistent launch for many jobs (cells) of one
// (NMAX bucket, modulation).  Workgroups take (job, subcarrier, symbol) items
// from a device counter until the queue is empty; every item is processed
// exactly as path_search_kernel would, so results equal the per-job launch.
// ============================================================================
struct BatchArgs {
    const JobDev *jobs;
    int n_jobs, total_items;
    unsigned *counter;
    float delta;
};

template <int NMAX, int L>
__global__ __launch_bounds__(256) void path_search_batch_kernel(BatchArgs a)
{
    constexpr int NW = NMAX / 4;
    __shared__ int item_s;
    __shared__ float sm[4];
    __shared__ int sr[4];
    for (;;) {
        if (threadIdx.x == 0)
            item_s = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= a.total_items)
            break;
        int jb = 0;  // job owning the item (jobs sorted by item_begin)
        {
            int lo = 0, hi = a.n_jobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.jobs[mid].item_begin <= item)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            jb = lo;
        }
        const JobDev j = a.jobs[jb];
        const int li = item - j.item_begin;
        const int s = li / j.T, t = li - s * j.T;
        const int N = j.N;
        const float2 *yv = j.yt + ((size_t)t * j.S + s) * N;
        const float4 *dg = j.diag + (size_t)s * N;
        const float2 *roff = j.roff + (size_t)s * N * N;
        const int nw = j.NP >> 2;
        const uint32_t *Pw = (const uint32_t *)(j.P + (size_t)s * j.K * j.NP);
        float bm = INFINITY;
        int br = INT_MAX;
        uint32_t bdec[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w)
            bdec[w] = 0;
        for (int r = threadIdx.x; r < j.K; r += blockDim.x) {
            uint32_t pw[NW], dec[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                pw[w] = (w < nw) ? Pw[(size_t)r * nw + w] : 0x01010101u;
                dec[w] = 0;
            }
            const float m = descend<NMAX, L, PREC_FP32>(yv, dg, roff, nullptr, N, pw, dec, a.delta);
            if (better(m, r, bm, br)) {
                bm = m;
                br = r;
#pragma unroll
                for (int w = 0; w < NW; ++w)
                    bdec[w] = dec[w];
            }
        }
        float wm = bm;
        int wr = br;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float om = __shfl_xor(wm, off);
            const int orr = __shfl_xor(wr, off);
            if (better(om, orr, wm, wr)) {
                wm = om;
                wr = orr;
            }
        }
        const int wid = threadIdx.x >> 6;
        const int nwv = (blockDim.x + 63) >> 6;
        if ((threadIdx.x & 63) == 0) {
            sm[wid] = wm;
            sr[wid] = wr;
        }
        __syncthreads();
        float gm = sm[0];
        int gr = sr[0];
        for (int w = 1; w < nwv; ++w)
            if (better(sm[w], sr[w], gm, gr)) {
                gm = sm[w];
                gr = sr[w];
            }
        if (br == gr) {
            int32_t *o = j.out + ((size_t)t * j.S + s) * N;
            const int32_t *pm = j.permd + (size_t)s * N;
#pragma unroll
            for (int d = 0; d < NMAX; ++d) {
                if (d < N) {
                    const int u = pm[d];
                    if ((unsigned)u < (unsigned)N)
                        o[u] = (int32_t)((bdec[d >> 2] >> ((d & 3) * 8)) & 0xffu);
                }
            }
        }
        __syncthreads();
    }
}


inline float delta_of(int bits)
{
    const int L = 1 << (bits / 2);
    return (float)sqrt(3.0 / (2.0 * (L * L - 1)));
}

inline int threads_for(int K)
{
    return K >= 256 ? 256 : ((K + 63) / 64) * 64;
}

}  // namespace dev
}  // namespace mpnl
