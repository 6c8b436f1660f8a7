// Device code shared by the kernel translation units of the MPNL library:
// helpers, the a4 point choice and the a4 + a5 path-search kernel templates.
//
// Lattice units.  On row l the residual b_l is kept divided by
// a_l = R_ll * Delta, so every constellation level of an axis sits on an odd
// integer -(L-1) .. L-1 and the distance of point c is
//     |b_l - R_ll c|^2 = a_l^2 ((z_I - c_I)^2 + (z_Q - c_Q)^2),   z = b_l / a_l.
// The sorted QR writes R already scaled this way (R'[d][e] = R_{l_e,l_d}
// Delta / a_{l_e}) and the rotation writes yt / a_l, so the descent needs
// no division: the nearest level is a round and a clamp.
// Rows with R_ll = 0 keep scale 1 and are handled by index order.
//
// Uniform data (R, yt, the per-depth diagonal) are read through the constant
// address space: the same address in every lane becomes a scalar load, and
// the values feed the VALU as SGPR operands.
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

template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

// Uniform arrays are read as plain floats (the HIP vector classes cannot be
// copied out of another address space).
__device__ __forceinline__ cptr<float> uniform_ptr(const float2 *p) { return (cptr<float>)p; }
__device__ __forceinline__ cptr<float> uniform_ptr(const float4 *p) { return (cptr<float>)p; }
__device__ __forceinline__ cptr<uint32_t> uniform_ptr(const uint32_t *p) { return (cptr<uint32_t>)p; }
__device__ __forceinline__ cptr<float> uniform_ptr(const float *p) { return (cptr<float>)p; }

__device__ __forceinline__ float2 ld2(cptr<float> p, int i) { return make_float2(p[2 * i], p[2 * i + 1]); }

// ---------------------------------------------------------------------------
// Lane exchanges inside a 64-lane wavefront done by the VALU (DPP row
// operations and gfx950's row swaps), with no trip through the LDS crossbar:
// lane_xor<S>(x) returns x of lane (lane ^ S).  The block size must be a
// multiple of 64 (the lane is the low six bits of threadIdx.x).
// ---------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ uint32_t lane_xor(uint32_t x)
{
    const int v = (int)x;
    if constexpr (S == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
    } else if constexpr (S == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
    } else if constexpr (S == 4) {
        // row_shl:4 for every lane, then row_shr:4 written into banks 1 and 3
        // only (the lanes with bit 2 set; the others keep the first move)
        const int up = __builtin_amdgcn_mov_dpp(v, 0x104, 0xF, 0xF, true);
        return (uint32_t)__builtin_amdgcn_update_dpp(up, v, 0x114, 0xF, 0xA, false);
    } else if constexpr (S == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true);  // row_ror:8
    } else if constexpr (S == 16) {
        const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return (threadIdx.x & 16u) ? p[0] : p[1];
    } else {
        static_assert(S == 32, "lane distance must be a power of two up to 32");
        const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return (threadIdx.x & 32u) ? p[0] : p[1];
    }
}

// Run-time distance (constant after unrolling at every call site).
__device__ __forceinline__ uint32_t lane_xor_n(uint32_t x, int s)
{
    switch (s) {
    case 1: return lane_xor<1>(x);
    case 2: return lane_xor<2>(x);
    case 4: return lane_xor<4>(x);
    case 8: return lane_xor<8>(x);
    case 16: return lane_xor<16>(x);
    default: return lane_xor<32>(x);
    }
}
__device__ __forceinline__ int lane_xor_n(int x, int s) { return (int)lane_xor_n((uint32_t)x, s); }
__device__ __forceinline__ float lane_xor_n(float x, int s)
{
    return __uint_as_float(lane_xor_n(__float_as_uint(x), s));
}
__device__ __forceinline__ double lane_xor_n(double x, int s)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t lo = lane_xor_n((uint32_t)u, s), hi = lane_xor_n((uint32_t)(u >> 32), s);
    return __longlong_as_double((long long)(lo | (hi << 32)));
}

// Both ends of the distance-S lane pair this lane belongs to, for S = 16 or
// 32: lo = x of lane (lane & ~S), hi = x of lane (lane | S).  One row or
// half-wave swap gives both (a compare-exchange then picks from lo and hi by
// the lane's side, with no select of the partner's value first).
template <int S>
__device__ __forceinline__ void lane_pair(uint32_t x, uint32_t &lo, uint32_t &hi)
{
    static_assert(S == 16 || S == 32, "lane pairs by swap need a distance of 16 or 32");
    if constexpr (S == 16) {
        const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        lo = p[0];
        hi = p[1];
    } else {
        const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        lo = p[0];
        hi = p[1];
    }
}
template <int S>
__device__ __forceinline__ void lane_pair(double x, double &lo, double &hi)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    uint32_t l0, h0, l1, h1;
    lane_pair<S>((uint32_t)u, l0, h0);
    lane_pair<S>((uint32_t)(u >> 32), l1, h1);
    lo = __longlong_as_double((long long)((uint64_t)l0 | ((uint64_t)l1 << 32)));
    hi = __longlong_as_double((long long)((uint64_t)h0 | ((uint64_t)h1 << 32)));
}

// Active lanes of the wave where c holds, as a lane mask.  A compare passed
// straight in becomes the mask itself (HIP's __ballot and __all take an
// int: a select and a compare more per vote).
__device__ __forceinline__ uint64_t lane_mask(bool c) { return __builtin_amdgcn_ballot_w64(c); }

// x of lane l (l uniform across the wave).
__device__ __forceinline__ uint32_t lane_read(uint32_t x, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
__device__ __forceinline__ double lane_read(double x, int l)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t lo = lane_read((uint32_t)u, l), hi = lane_read((uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(lo | (hi << 32)));
}

// 64-bit words through the 32-bit moves above, one half at a time.
__device__ __forceinline__ uint64_t lane_join(uint32_t lo, uint32_t hi) { return (uint64_t)lo | ((uint64_t)hi << 32); }
__device__ __forceinline__ uint64_t lane_xor_n(uint64_t x, int s)
{
    return lane_join(lane_xor_n((uint32_t)x, s), lane_xor_n((uint32_t)(x >> 32), s));
}
__device__ __forceinline__ uint64_t lane_read(uint64_t x, int l)
{
    return lane_join(lane_read((uint32_t)x, l), lane_read((uint32_t)(x >> 32), l));
}
template <int S>
__device__ __forceinline__ void lane_pair(uint64_t x, uint64_t &lo, uint64_t &hi)
{
    uint32_t l0, h0, l1, h1;
    lane_pair<S>((uint32_t)x, l0, h0);
    lane_pair<S>((uint32_t)(x >> 32), l1, h1);
    lo = lane_join(l0, l1);
    hi = lane_join(h0, h1);
}

// x of lane 63 - lane: mirror inside each row of 16, then swap the rows.
__device__ __forceinline__ uint32_t lane_mirror(uint32_t x)
{
    const uint32_t m = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, true);  // row_mirror
    return lane_xor<32>(lane_xor<16>(m));
}
__device__ __forceinline__ double lane_mirror(double x)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t lo = lane_mirror((uint32_t)u), hi = lane_mirror((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(lo | (hi << 32)));
}
__device__ __forceinline__ uint64_t lane_mirror(uint64_t x)
{
    return lane_join(lane_mirror((uint32_t)x), lane_mirror((uint32_t)(x >> 32)));
}

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

// a2 depth costs.  The cost of a position vector is sum_d c_d (p_d - 1) in
// integers, c_d = rint(w_d / max_e w_e * 2^kCostBits): the depth weights of
// the subcarrier scaled so that the largest becomes 2^kCostBits, rounded to
// the nearest integer (ties to even).  Sums stay below 2^31 for 32 depths and
// ranks up to 64, so costs and their comparisons are exact.  A weight that is
// not a number, or a subcarrier whose largest weight is not a positive finite
// number, gives cost 0.
constexpr int kCostBits = 20;
__device__ __forceinline__ uint32_t cost_unit(double w, double wmax)
{
    const double x = (w / wmax) * (double)(1 << kCostBits);
    return (wmax > 0.0 && wmax <= 1.7976931348623157e308 && x >= 0.0 && x <= (double)(1 << kCostBits))
               ? (uint32_t)rint(x)
               : 0u;
}

// a2 arguments (position-vector set kernels)
struct PosArgs {
    const double *w;  // (S, N)
    int S, N, nq, K, NP;
    uint8_t *P;       // (S, K, NP)
    uint16_t *order;  // (S, K) path run by each lane, or null (identity)
    uint32_t *rec_g;  // (S, N, K) when the back pointers do not fit in LDS
    uint16_t *rec16;  // (S, N, 256) back pointers of a 256-path set in global memory, or null (LDS)
};

// One job of a batched launch of a1 / a2 / a3 (slot state and workspace of
// the job, its input and the first work item of the job in the launch).
struct StageJob {
    const float2 *H;  // (S, M, N)
    const float2 *y;  // (T, S, M)
    float2 *yt;       // (T, S, N)
    SlotDev sd;
    int T;
    float delta;
    int item_begin;
};

// index of the job owning work item `item` (jobs sorted by item_begin)
template <typename J>
__device__ __forceinline__ int find_job(const J *jobs, int n_jobs, int item)
{
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].item_begin <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ============================================================================
// a4: choice of the k-th closest constellation point at one depth, in lattice
// units.  Level index m in 0..L-1 <-> level value 2m - (L-1).
// ============================================================================
// x * x rounded on its own: never fused into the sum that follows, so every
// distance of the descent (first choice or k-th) rounds alike in every kernel
// that runs it, whatever code surrounds it.  The path kernel repeats path 0
// of the pruning record, and the batched and one-shot kernels of the same
// job must reach the same bits.
__device__ __forceinline__ float square_rn(float x)
{
#pragma clang fp contract(off)
    return x * x;
}

template <int L>
__device__ __forceinline__ float level_of(float m)
{
    return fmaf(m, 2.f, -(float)(L - 1));
}

// closest level: round the level coordinate, clamp to the constellation
template <int L>
__device__ __forceinline__ float nearest_level(float z, float &m)
{
    m = __builtin_amdgcn_fmed3f(rintf(fmaf(z, 0.5f, 0.5f * (float)(L - 1))), 0.f, (float)(L - 1));
    return level_of<L>(m);
}

// second closest level of one axis: the neighbour of the closest level m0
// on the side of z (dz = z - level of m0), or at the edge of the constellation
// the other neighbour: m0 + s reflected back into 0 .. L-1 (exact small
// integers; no compare and select)
template <int L>
__device__ __forceinline__ void axis_second(float z, float dz, float m0, float &m1, float &e1)
{
    constexpr float top = (float)(L - 1);
    const float s = __builtin_copysignf(1.f, dz);  // dz = +0 when z is on the level: upward, as z >= level
    m1 = top - fabsf(top - fabsf(m0 + s));
    e1 = square_rn(z - level_of<L>(m1));
}

// Levels of rank 1..3 of one axis, rank 0 being the closest level m0: the
// zig-zag from m0 that starts on the side of z, levels beyond the
// constellation skipped.  With |z - lv0| <= 1 the zig-zag is sorted by
// distance; when z lies beyond the outermost level only one side exists and
// the order is monotone.  In mirrored coordinates (z at or above its closest
// level m') the level index of rank t depends on m' alone:
constexpr int zigzag_rank(int L, int mp, int t)
{
    const int up = L - 1 - mp, down = mp;  // levels above and below m'
    const int q = up < down ? up : down;
    if (t <= 2 * q)
        return (t & 1) ? mp + (t + 1) / 2 : mp - t / 2;
    return up > down ? mp + (t - q) : mp - (t - q);
}
// ... tabulated for L = 4 and 8 as the mirrored level value v = 2 r - (L - 1)
// of rank t, a signed field of 32 / L bits per m'
constexpr uint32_t zigzag_word(int L, int t)
{
    uint32_t w = 0;
    for (int mp = 0; mp < L; ++mp) {
        const int v = 2 * zigzag_rank(L, mp, t) - (L - 1);
        w |= ((uint32_t)v & ((1u << (32 / L)) - 1u)) << ((32 / L) * mp);
    }
    return w;
}

// Ranks 1..R (R <= 3) of one axis (L = 4 or 8): mirrored level values v[t]
// and squared distances e[t], with the mirror sign s (s = +1: z at or above
// the level of m0, the level of rank t is s v[t]).  The distance is taken in
// mirrored coordinates, (s z - v)^2: negation is exact and rounding
// symmetric, so it is the same bits as (z - s v)^2.
template <int L, int R>
__device__ __forceinline__ void axis_ranks(float z, float m0, float lv0, float (&v)[3], float (&e)[3], float &s)
{
    static_assert(L == 4 || L == 8, "tabulated zig-zag: 4 or 8 levels an axis");
    constexpr int FW = 32 / L;
    constexpr float H = 0.5f * (float)(FW * (L - 1));
    s = __builtin_copysignf(1.f, z - lv0);  // +0 on the level: upward, as z >= level
    const float zs = s * z;
    const uint32_t off = (uint32_t)fmaf(s, fmaf(m0, (float)FW, -H), H);  // FW m'
#pragma unroll
    for (int t = 0; t < R; ++t) {
        v[t] = (float)(int)__builtin_amdgcn_sbfe((int)zigzag_word(L, t + 1), off, FW);
        e[t] = square_rn(zs - v[t]);
    }
}

// Rank 3 or 4 (L = 4 or 8) from the frontier of the per-axis orders; FOUR =
// false: every lane asks for rank 3.
template <int L, bool FOUR>
__device__ __forceinline__ float kth_frontier(float zI, float zQ, int k, float &mI, float lI, float eI,
                                              float &mQ, float lQ, float eQ)
{
    constexpr int R = FOUR ? 3 : 2;
    float vi[3], ei[3], vq[3], eq[3], sI, sQ;
    axis_ranks<L, R>(zI, mI, lI, vi, ei, sI);
    axis_ranks<L, R>(zQ, mQ, lQ, vq, eq, sQ);
    const float A1 = ei[0] + eQ, A2 = ei[1] + eQ;  // (t, 0)
    const float B1 = eI + eq[0], B2 = eI + eq[1];  // (0, t)
    const bool firstI = A1 <= B1;                  // rank 2 = (1,0), else (0,1)
    const bool t20 = firstI & (A2 <= B1);          // ranks 2, 3 = (1,0), (2,0)
    const bool t02 = !firstI & (B2 < A1);          // ranks 2, 3 = (0,1), (0,2)
    bool i1 = !firstI & !t02, i2 = t20, i3 = false;
    bool q1 = firstI & !t20, q2 = t02, q3 = false, c11 = false;
    float A3 = 0.f, B3 = 0.f, C = 0.f;
    if constexpr (FOUR) {
        A3 = ei[2] + eQ;
        B3 = eI + eq[2];
        C = ei[0] + eq[0];  // (1, 1)
        // rank 4 after (1,0), (2,0): (3,0) or (0,1); after (0,1), (0,2):
        // (1,0) or (0,3); after (1,0), (0,1): (2,0), (1,1) or (0,2)
        const bool k3 = k == 3;
        const bool mid = !t20 & !t02;
        const bool x20 = (A2 <= C) & (A2 <= B2), x11 = !x20 & (C <= B2);
        i1 = k3 ? i1 : (t02 & (A1 <= B3));
        i2 = k3 ? i2 : (mid & x20);
        i3 = !k3 & t20 & (A3 <= B1);
        q1 = k3 ? q1 : (t20 & !(A3 <= B1));
        q2 = k3 ? q2 : (mid & !x20 & !x11);
        q3 = !k3 & t02 & !(A1 <= B3);
        c11 = !k3 & mid & x11;
    }
    // level index from the mirrored level value: m = (s v + L - 1) / 2
    const float vI = i3 ? vi[2] : i2 ? vi[1] : vi[0];
    const float vQ = q3 ? vq[2] : q2 ? vq[1] : vq[0];
    mI = (i1 | i2 | i3 | c11) ? fmaf(vI, 0.5f * sI, 0.5f * (float)(L - 1)) : mI;
    mQ = (q1 | q2 | q3 | c11) ? fmaf(vQ, 0.5f * sQ, 0.5f * (float)(L - 1)) : mQ;
    return i1 ? A1 : i2 ? A2 : i3 ? A3 : q1 ? B1 : q2 ? B2 : q3 ? B3 : C;
}

// Exact 3rd or 4th closest point from the per-axis orders: ranks 2..4 of
// the sum of two sorted lists come from the in-phase chain (t, 0), the
// quadrature chain (0, t) and the corner (1, 1), which can only follow both
// (1, 0) and (0, 1): the frontier {(1,0), (0,1)}, then {(2,0), (0,1)} or
// {(1,0), (0,2)}, then one of (3,0), (2,0), (1,1), (0,2), (0,3) depending on
// the earlier ranks.  Equal costs: the larger in-phase step first.  Every
// lane evaluates the same compares and the choice is a few selects (no
// divergent branches); returns the point's squared distance, the sum of the
// two axes' distances as for any other rank.
template <int L>
__device__ __forceinline__ float kth_small(float zI, float zQ, int k, float &mI, float lI, float eI,
                                           float &mQ, float lQ, float eQ)
{
    if constexpr (L == 2) {
        // two levels an axis: rank 3 is the single step rank 2 did not
        // take, rank 4 the corner
        const float m1I = 1.f - mI, m1Q = 1.f - mQ;
        const float e1I = square_rn(zI - level_of<L>(m1I)), e1Q = square_rn(zQ - level_of<L>(m1Q));
        const float A1 = e1I + eQ, B1 = eI + e1Q;
        const bool firstI = A1 <= B1;
        const bool inI = (k == 3) & !firstI, inQ = (k == 3) & firstI;
        mI = inQ ? mI : m1I;
        mQ = inI ? mQ : m1Q;
        return inI ? A1 : inQ ? B1 : e1I + e1Q;
    } else {
        // the third level of an axis and the compares of rank 4 only where
        // some lane of the wave asks for rank 4 (a wave-uniform branch)
        if (__builtin_amdgcn_ballot_w64(k == 4) != 0)
            return kth_frontier<L, true>(zI, zQ, k, mI, lI, eI, mQ, lQ, eQ);
        return kth_frontier<L, false>(zI, zQ, k, mI, lI, eI, mQ, lQ, eQ);
    }
}

// Lanes of a bitonic compare-exchange step (block size `size`, distance j,
// rows of npt lanes) that keep the smaller key when lower == up: a constant
// of the lane pattern, turned into a lane predicate by an inverse ballot (a
// scalar constant, not a mask computed and held per wave).
constexpr uint64_t bitonic_keep_low(int size, int j, int npt)
{
    uint64_t m = 0;
    for (int l = 0; l < 64; ++l) {
        const bool up = size == npt || (l & size) == 0;
        const bool lower = (l & j) == 0;
        if (lower == up)
            m |= 1ull << l;
    }
    return m;
}

// Exact k-th closest point for k > 4, computed by the whole wavefront.  The
// lanes that need it at this depth are served in rounds: a round takes the
// received value z of one of them, lane c evaluates constellation point
// c mod L^2 against z, the wave sorts the points by (cost, constellation
// index) with a bitonic network over L^2 lanes, and every needing lane whose
// value equals z reads entry k-1 of the sorted list.  Lanes that share a
// path prefix share z, so one round usually serves all of them.  Must be
// reached by every lane of the wave.
template <int L>
__device__ __forceinline__ void kth_wave(bool need, float zI, float zQ, int k, float &mI, float &mQ, float &e)
{
    constexpr int HB = Axis<L>::HB;
    constexpr int NPT = L * L;  // 16 or 64 points: sorted within rows of NPT lanes
    const int lane = (int)(threadIdx.x & 63u);
    const int c = lane & (NPT - 1);
    const int cI = c & (L - 1), cQ = c >> HB;
    const int cidx = (gray_code(cI) << HB) | gray_code(cQ);
    const float vI = level_of<L>((float)cI), vQ = level_of<L>((float)cQ);
    uint64_t pend = lane_mask(need);
    while (pend) {
        const int src = __builtin_ctzll(pend);
        const float zi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zI), src));
        const float zq = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(zQ), src));
        const float dI = zi - vI, dQ = zq - vQ;
        // (cost, index) as one 64-bit key: costs are sums of squares (+0
        // or more), whose bit patterns order as the values do
        uint64_t key = lane_join((uint32_t)cidx, __float_as_uint(square_rn(dI) + square_rn(dQ)));
#pragma unroll
        for (int size = 2; size <= NPT; size <<= 1) {
#pragma unroll
            for (int j = size >> 1; j > 0; j >>= 1) {
                const uint64_t ok = lane_xor_n(key, j);
                const bool keep_low = __builtin_amdgcn_inverse_ballot_w64(bitonic_keep_low(size, j, NPT));
                const bool take = keep_low == (ok < key);
                key = take ? ok : key;
            }
        }
        const bool mine = need && ((zI == zi && zQ == zq) || lane == src);
        const int from = (lane & ~(NPT - 1)) + min(max(k, 1), NPT) - 1;
        const int got = __shfl((int)(uint32_t)key, from);
        if (mine) {
            mI = (float)gray_decode(got >> HB);
            mQ = (float)gray_decode(got & (L - 1));
            e = square_rn(zI - level_of<L>(mI)) + square_rn(zQ - level_of<L>(mQ));
        }
        pend &= ~lane_mask(mine);
    }
}

// ============================================================================
// a4 + a5: path search.
// ============================================================================
struct PathArgs {
    const float2 *yt;      // (T, S, N) rotated received vectors, lattice units
    const float4 *diag;    // (S, N) (a^2 or 1, R_ll == 0, 1/a or 1, R_ll)
    const float2 *rlat;    // (S, N, N) R' transposed, lattice units: [d][e] = coefficient of s_e in row d
    const uint32_t *rq;    // (S, N, N, 2) packed FP16 / BF16 pairs of rlat (SlotDev::rlat_h), or null
    const int32_t *permd;  // (S, N)
    const uint8_t *P;      // (S, K, NP)
    const uint16_t *order; // (S, K) path run by each lane, or null (identity)
    int32_t *out;          // (T, S, N)
    float *llr;            // (T, S, N, bits) or null
    float *part;           // per path group best (metric, path, decisions) or null
    float *bound;          // (T, S) metric of path 0 per vector (pruning), or null
    int S, T, N, K, NP;
    float sigma2, clip;
};

enum { PREC_FP32 = 0, PREC_FP16 = 1, PREC_BF16 = 2 };

// Decisions are packed as level codes c = mI + L mQ (< 64), four per float:
// digit d & 3 of decf[d >> 2] in base 64, exact in a float mantissa.
__device__ __forceinline__ constexpr float code_weight(int d)
{
    return (d & 3) == 0 ? 1.f : (d & 3) == 1 ? 64.f : (d & 3) == 2 ? 4096.f : 262144.f;
}

// Pruning.  The accumulated metric never decreases along a path, so a path
// whose partial metric already exceeds the metric of some complete path can
// no longer be the minimum.  Path 0 (the first choice at every depth) is
// evaluated per received vector before the search (path_bound_kernel), which
// leaves a record per vector: the metric of path 0, then its packed decisions.
// In the search, a wavefront whose paths all exceed that bound (padded by
// kBoundPad) stops descending, and the lane of path 0 takes its metric and
// decisions from the record, so it holds no wavefront up.  Both evaluations
// of path 0 run the same arithmetic in the same order, so its metric is the
// same bits either way.  The winner and its tie rule are unchanged: every
// pruned path has a metric strictly above the minimum.
constexpr float kBoundPad = 1.0001f;

// FP32 descents above this many users keep their decided symbols as half2
// (descend).  Mixed FMAs issue slower than plain ones here: in the one-job
// search at 16 users the float2 form (no spills) is 6% faster, at 24 users 1%.
constexpr int kHalfStateN = 24;
// ... and in the multi-job search, which holds more state: 40 cells of
// 4..32 users in FP32, 121.6 M vectors/s with the float2 form, 127.3 M above
// 24 users, 129.3 M above 16 users
constexpr int kHalfStateNMulti = 16;

// Received values of one descent: yt of the vector in depth order, read
// where each depth needs it, from a wave-uniform pointer (scalar loads) ...
struct YUniform {
    cptr<float> p;
    __device__ __forceinline__ float2 operator()(int d) const { return ld2(p, d); }
};
// ... or from registers loaded up front (one received vector per lane).
template <int N>
struct YLanes {
    float2 v[N];
    __device__ __forceinline__ float2 operator()(int d) const { return v[d]; }
};

// The subcarrier's triangular factor as the descent reads it: the diagonal
// record (a^2, R_ll == 0 flag, ...) per depth and R' transposed (rl, FP32;
// rq, packed FP16 / BF16 pairs (x, y), (y, -x): with the decided symbol
// packed as (-s_I, s_Q), one dot2 with each gives the I and the Q term),
// through a wave-uniform pointer (scalar loads) ...
struct RUniform {
    cptr<float> dg, rl;
    cptr<uint32_t> rq;
    __device__ __forceinline__ float gw(int d) const { return dg[4 * d]; }
    // R_ll == 0 flag (0.f or 1.f) tested on its bits: a scalar compare
    __device__ __forceinline__ bool gzero(int d) const { return __float_as_uint(dg[4 * d + 1]) != 0u; }
    __device__ __forceinline__ float2 r(int i) const { return ld2(rl, i); }
    __device__ __forceinline__ uint2 q(int i) const { return make_uint2(rq[2 * i], rq[2 * i + 1]); }
};
// ... or through a pointer of each lane's own subcarrier (vector loads).
struct RLanes {
    const float *dg, *rl;
    const uint32_t *rq;
    __device__ __forceinline__ float gw(int d) const { return dg[4 * d]; }
    __device__ __forceinline__ bool gzero(int d) const { return dg[4 * d + 1] != 0.f; }
    __device__ __forceinline__ float2 r(int i) const { return ((const float2 *)rl)[i]; }
    __device__ __forceinline__ uint2 q(int i) const { return ((const uint2 *)rq)[i]; }
};

// One SIC descent driven by the position vector in pw, left-looking: the
// residual of depth d is formed when depth d is reached, y_d minus R'[e][d]
// s_e for the depths e above it, accumulated in depth order (the same
// operations in the same order as updating every lower row after each
// decision, so the same bits), and a wavefront that stops early never
// computes the rows below.  rl holds R' transposed: rl[d N + e] is the
// coefficient of s_e in row d (lattice units of row d).  `prune`: the wave
// stops once no lane with live = true has a metric at or below it (a NaN
// metric counts as above; all lanes must take part).  A lane with live =
// false returns +inf (a finite prune) or a metric of no use: its caller
// discards it.  FIRST: every rank is 1 (path 0), the choice code for higher
// ranks is left out.
template <int N, int L, int PREC, bool FIRST = false, int HSN = kHalfStateN, typename YF, typename RF>
__device__ __forceinline__ float descend(const YF &y, const RF &R, const uint32_t *pw, float *decf, float prune,
                                         bool live)
{
    // lanes that take no part in the stop (live = false) start above any
    // bound, so the ballot of the metric alone decides it
    float metric = live ? 0.f : INFINITY;
    // FP32: (s_I, s_Q) of the decided depths, as a float2, or above HSN
    // users as a half2 (small odd integers, exact) that mixed
    // FMAs widen exactly where they read it: the same products and sums in
    // half the registers, for user counts where the float2 form spills
    constexpr bool HS = PREC == PREC_FP32 && N > HSN;
    float2 sv[HS ? 1 : N];
    uint32_t sh[HS ? N : 1];
    uint32_t sa[N];                // FP16 / BF16: packed (-s_I, s_Q)
#pragma unroll
    for (int d = 0; d < N; ++d) {
        const int k = (pw[d >> 2] >> ((d & 3) * 8)) & 0xff;
        const float gw = R.gw(d);
        const bool gzero = R.gzero(d);
        const float2 yd = y(d);
        float zI = yd.x, zQ = yd.y;
        if constexpr (PREC == PREC_FP32) {
#pragma unroll
            for (int e = 0; e < d; ++e) {
                const float2 r = R.r(d * N + e);
                float sI, sQ;
                if constexpr (HS) {
                    uint32_t she = sh[e];
                    asm("" : "+v"(she));  // a fresh value per depth: widened where used, not kept widened
                    const half2_t se = __builtin_bit_cast(half2_t, she);
                    sI = (float)se.x;
                    sQ = (float)se.y;
                } else {
                    sI = sv[e].x;
                    sQ = sv[e].y;
                }
                zI = fmaf(-r.x, sI, zI);
                zI = fmaf(r.y, sQ, zI);
                zQ = fmaf(-r.x, sQ, zQ);
                zQ = fmaf(-r.y, sI, zQ);
            }
        } else if constexpr (PREC == PREC_FP16) {
#pragma unroll
            for (int e = 0; e < d; ++e) {
                const uint2 r = R.q(d * N + e);
                const half2_t se = __builtin_bit_cast(half2_t, sa[e]);
                zI = __builtin_amdgcn_fdot2(__builtin_bit_cast(half2_t, r.x), se, zI, false);
                zQ = __builtin_amdgcn_fdot2(__builtin_bit_cast(half2_t, r.y), se, zQ, false);
            }
        } else {
#pragma unroll
            for (int e = 0; e < d; ++e) {
                const uint2 r = R.q(d * N + e);
                const bf162_t se = __builtin_bit_cast(bf162_t, sa[e]);
                zI = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf162_t, r.x), se, zI, false);
                zQ = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf162_t, r.y), se, zQ, false);
            }
        }
        float mI, mQ, e;  // the chosen point and its squared distance
        if (gzero) {
            // R_ll = 0: every point is equally far; the k-th in index order
            const int idx = min(max(k - 1, 0), L * L - 1);
            mI = (float)gray_decode(idx >> Axis<L>::HB);
            mQ = (float)gray_decode(idx & (L - 1));
            e = square_rn(zI) + square_rn(zQ);
        } else {
            const float lI = nearest_level<L>(zI, mI), lQ = nearest_level<L>(zQ, mQ);
            const float dI = zI - lI, dQ = zQ - lQ;
            float eI = square_rn(dI), eQ = square_rn(dQ);
            e = eI + eQ;
            if (FIRST) {
            } else if (k == 2) {
                // rank 2 is (second I, closest Q) or (closest I, second Q):
                // every other point is farther than one of the two
                float mI1, eI1, mQ1, eQ1;
                axis_second<L>(zI, dI, mI, mI1, eI1);
                axis_second<L>(zQ, dQ, mQ, mQ1, eQ1);
                const float cI = eI1 + eQ, cQ = eI + eQ1;
                const bool inI = cI <= cQ;
                mI = inI ? mI1 : mI;
                mQ = inI ? mQ : mQ1;
                e = inI ? cI : cQ;
            } else if (k == 3 || k == 4) {
                e = kth_small<L>(zI, zQ, k, mI, lI, eI, mQ, lQ, eQ);
            }
            if constexpr (L > 2 && !FIRST)
                kth_wave<L>(k > 4, zI, zQ, k, mI, mQ, e);
        }
        metric = fmaf(gw, e, metric);
        decf[d >> 2] = fmaf(fmaf(mQ, (float)L, mI), code_weight(d), decf[d >> 2]);
        if (d + 1 < N && lane_mask(metric <= prune) == 0)
            break;
        const float sI = level_of<L>(mI), sQ = level_of<L>(mQ);
        if constexpr (HS) {
            half2_t hs;
            hs.x = (_Float16)sI;
            hs.y = (_Float16)sQ;
            sh[d] = __builtin_bit_cast(uint32_t, hs);
        } else if constexpr (PREC == PREC_FP32) {
            sv[d] = make_float2(sI, sQ);
        } else if constexpr (PREC == PREC_FP16) {
            half2_t ha;  // small odd integers, exact
            ha.x = (_Float16)(-sI);
            ha.y = (_Float16)sQ;
            sa[d] = __builtin_bit_cast(uint32_t, ha);
        } else {
            bf162_t ha;
            ha.x = (__bf16)(-sI);
            ha.y = (__bf16)sQ;
            sa[d] = __builtin_bit_cast(uint32_t, ha);
        }
    }
    return (metric == metric) ? metric : INFINITY;
}

// constellation index chosen at depth d of a packed decision record
template <int L>
__device__ __forceinline__ int32_t decision_index(const float *decf, int d)
{
    const uint32_t word = (uint32_t)decf[d >> 2];
    const int code = (int)((word >> (6 * (d & 3))) & 63u);
    const int mI = code & (L - 1), mQ = (code >> Axis<L>::HB) & (L - 1);
    return (gray_code(mI) << Axis<L>::HB) | gray_code(mQ);
}

__device__ __forceinline__ bool better(float m, int r, float bm, int br)
{
    return (m < bm) | ((m == bm) & (r < br));
}

// Minimum (metric, path) over the workgroup; returns the winning path index.
__device__ __forceinline__ int block_argmin(float bm, int br, int W, float *sm, int *sr)
{
    float wm = bm;
    int wr = br;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float om = lane_xor_n(wm, off);
        const int orr = lane_xor_n(wr, off);
        if (better(om, orr, wm, wr)) {
            wm = om;
            wr = orr;
        }
    }
    if (W == 64)  // one wave per vector: no exchange between waves
        return wr;
    const int wid = threadIdx.x >> 6;
    const int wpv = W >> 6;
    const int w0 = wid - wid % wpv;
    if ((threadIdx.x & 63) == 0) {
        sm[wid] = wm;
        sr[wid] = wr;
    }
    __syncthreads();
    float gm = sm[w0];
    int gr = sr[w0];
    for (int w = 1; w < wpv; ++w)
        if (better(sm[w0 + w], sr[w0 + w], gm, gr)) {
            gm = sm[w0 + w];
            gr = sr[w0 + w];
        }
    return gr;
}

// The W lanes (whole waves) tid = 0..W-1 given to one received vector run
// one path each: lane tid of path group g runs path g * W + tid.  With one
// group the winner writes its symbols in user order; with several, each group
// leaves its best (metric, path, decisions) for path_group_reduce_kernel.
// Every lane of the workgroup calls this (it may synchronise the workgroup);
// lanes of an inactive vector do no work.
// b0 / b0d: path 0's metric and packed decisions from the pruning record
// (b0d null: no record, path 0 is searched like the others).  HSN: descend's
// half2 threshold.
template <int N, int L, int PREC, int HSN = kHalfStateN>
__device__ __forceinline__ void search_vector(cptr<float> yv, cptr<float> dg, cptr<float> rl,
                                              cptr<uint32_t> rq, const uint8_t *Pbase,
                                              const uint16_t *order, int K, int NP, int group,
                                              const int32_t *pm, int32_t *o, float *part, float *sm,
                                              int *sr, int W, int tid, bool active, float b0,
                                              const float *b0d)
{
    const float prune = b0 * kBoundPad;
    constexpr int NW = (N + 3) / 4;
    const uint32_t *Pw = (const uint32_t *)Pbase;
    const int nw = NP >> 2;
    const int li = group * W + tid;
    float bm = INFINITY;
    int br = INT_MAX;
    float decf[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w)
        decf[w] = 0.f;
    // Whole waves descend (the k > 4 choice is wave-cooperative); lanes past
    // the last path follow the first choice everywhere and are discarded.
    if (active && li - (int)(threadIdx.x & 63u) < K) {
        const bool valid = li < K;
        const int r = valid ? (order ? (int)order[li] : li) : 0;
        uint32_t pw[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w)
            pw[w] = valid ? Pw[(size_t)r * nw + w] : 0x01010101u;
        const bool known = valid && r == 0 && b0d != nullptr;
        const float m = descend<N, L, PREC, false, HSN>(YUniform{yv}, RUniform{dg, rl, rq}, pw, decf, prune,
                                                         valid && !known);
        if (valid) {
            bm = known ? b0 : m;
            br = r;
        }
        if (known) {
#pragma unroll
            for (int w = 0; w < NW; ++w)
                decf[w] = b0d[w];
        }
    }
    const int gr = block_argmin(bm, br, W, sm, sr);
    if (!active || br != gr)
        return;
    if (part == nullptr) {
#pragma unroll
        for (int d = 0; d < N; ++d) {
            const int u = pm[d];
            if ((unsigned)u < (unsigned)N)  // permd is a permutation for finite inputs
                o[u] = decision_index<L>(decf, d);
        }
    } else {
        part[0] = bm;
        part[1] = __int_as_float(br);
#pragma unroll
        for (int w = 0; w < NW; ++w)
            part[2 + w] = decf[w];
    }
}

// Occupancy of the path searches: eight wavefronts per SIMD (64 VGPRs) in
// every precision.  The descent is bound by the latency of its per-depth
// scalar loads of R and y as much as by VALU issue, so more resident
// wavefronts pay even where the decided symbols of the deeper depths spill
// to scratch (FP32, 16 users: 0.128 -> 0.116 ms per 1200 x 14 launch; 24
// users: 0.477 -> 0.352 ms per 3276 x 14, before the one-wavefront path
// groups).  FP16 / BF16 keep one packed register per decided depth (the
// paired R copy); with two they ran six wavefronts, and with one, eight
// against six measured: 40 cells 3.71 against 3.83 ms of path stage, the
// 24-user slot 0.222 against 0.229 ms, 16 users equal.
template <int PREC>
struct PathOccupancy {
    static constexpr int waves = 8;
};

// Work item (vector, path group) of slot q of this workgroup, for `groups`
// path groups a vector and ipw items a workgroup.  Group-major (a 2-D grid:
// x = workgroups per group, y = the group): all vectors' group 0 first, then
// group 1, ... (a workgroup holds ipw vectors of one group), which is the
// order in which the groups' costs are most alike when a launch fills the
// device.  Vector-major (a 1-D grid): the groups of a vector are neighbours.
// Either way every XCD gets a contiguous range of vectors, so the workgroups
// of one subcarrier share an L2.  (The 2-D grid measured 4-6% faster than
// the same group-major order numbered on a 1-D grid: 16x16 slot 0.085 against
// 0.090 ms, 24x24 0.243 against 0.254 ms.)
__device__ __forceinline__ void work_item(int q, int groups, int ipw, bool gmajor, int &vi, int &g)
{
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    if (gmajor) {
        g = (int)blockIdx.y;
        vi = b * ipw + q;
    } else {
        const int w = b * ipw + q;
        vi = w / groups;
        g = w - vi * groups;
    }
}

// One work item (received vector, path group of one wavefront) a workgroup
// of 64 lanes; grid (S * T, path groups), vectors numbered subcarrier-major
// (s T + t).
// partials: (S * T, groups, 2 + (N + 3) / 4)
template <int N, int L, int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PathOccupancy<PREC>::waves))) void
path_search_kernel(PathArgs a)
{
    __shared__ float sm[4];
    __shared__ int sr[4];
    const int groups = (int)gridDim.y, g = (int)blockIdx.y;
    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int s = lb / a.T, t = lb - s * a.T;
    const size_t sN = (size_t)s * N;
    const size_t v = (size_t)t * a.S + s;
    cptr<uint32_t> rq = a.rq ? uniform_ptr(a.rq + 2 * sN * N) : nullptr;
    float *part = a.part ? a.part + (v * groups + g) * (2 + (N + 3) / 4) : nullptr;
    const float b0 = a.bound ? uniform_ptr(a.bound + v)[0] : INFINITY;
    const float *b0d = a.bound ? a.bound + (size_t)a.S * a.T + v * ((N + 3) / 4) : nullptr;
    search_vector<N, L, PREC>(uniform_ptr(a.yt + v * N), uniform_ptr(a.diag + sN), uniform_ptr(a.rlat + sN * N),
                              rq, a.P + (size_t)s * a.K * a.NP, a.order ? a.order + (size_t)s * a.K : nullptr,
                              a.K, a.NP, g, a.permd + sN, a.out + v * N, part, sm, sr, 64,
                              (int)(threadIdx.x & 63u), true, b0, b0d);
}

// Best of the path groups of one received vector (equal metrics: lowest
// path), written in user order.  p: the vector's `groups` partial records of
// 2 + (N + 3) / 4 floats (metric, path, packed decisions).
template <int L>
__device__ __forceinline__ void reduce_groups(const float *p, int groups, int N, const int32_t *pm, int32_t *o)
{
    const int stride = 2 + (N + 3) / 4;
    int best = 0;
    for (int g = 1; g < groups; ++g)
        if (better(p[g * stride], __float_as_int(p[g * stride + 1]), p[best * stride],
                   __float_as_int(p[best * stride + 1])))
            best = g;
    const float *dec = p + best * stride + 2;
    for (int d = 0; d < N; ++d) {
        const int u = pm[d];
        if ((unsigned)u < (unsigned)N)
            o[u] = decision_index<L>(dec, d);
    }
}

// One lane per received vector.
template <int L>
__global__ __launch_bounds__(256) void path_group_reduce_kernel(PathArgs a, int groups)
{
    const size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (size_t)a.S * a.T)
        return;
    const int N = a.N;
    const int s = (int)(v % a.S);
    reduce_groups<L>(a.part + v * groups * (2 + (N + 3) / 4), groups, N, a.permd + (size_t)s * N, a.out + v * N);
}

// ============================================================================
// a4 + a5 with max-log soft output: every path's metric and decisions go to
// LDS; for each (user, bit) one lane scans the K paths for the smallest
// metric with the bit at 0 and at 1.
// ============================================================================
template <int N, int L>
__device__ __forceinline__ void soft_vector(const PathArgs &a, int s, int t, unsigned char *smem)
{
    constexpr int NW = (N + 3) / 4;
    constexpr int HB = Axis<L>::HB;
    constexpr int BITS = 2 * HB;
    const int K = a.K;
    const size_t sN = (size_t)s * N;
    cptr<float> yv = uniform_ptr(a.yt + ((size_t)t * a.S + s) * N);
    cptr<float> dg = uniform_ptr(a.diag + sN);
    cptr<float> rl = uniform_ptr(a.rlat + sN * N);
    const int nw = a.NP >> 2;
    const uint32_t *Pw = (const uint32_t *)(a.P + (size_t)s * K * a.NP);
    float *mets = (float *)smem;          // K
    float *decs = mets + K;               // K * NW
    // whole waves descend (see search_vector)
    for (int r0 = 0; r0 < K; r0 += blockDim.x) {
        const int r = r0 + (int)threadIdx.x;
        if (r - (int)(threadIdx.x & 63u) >= K)
            continue;
        const bool valid = r < K;
        uint32_t pw[NW];
        float decf[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            pw[w] = valid ? Pw[(size_t)r * nw + w] : 0x01010101u;
            decf[w] = 0.f;
        }
        const float m = descend<N, L, PREC_FP32>(YUniform{yv}, RUniform{dg, rl, nullptr}, pw, decf, INFINITY, valid);
        if (valid) {
            mets[r] = m;
#pragma unroll
            for (int w = 0; w < NW; ++w)
                decs[(size_t)r * NW + w] = decf[w];
        }
    }
    __syncthreads();
    const int32_t *pm = a.permd + sN;
    const size_t vbase = ((size_t)t * a.S + s) * N;
    for (int q = threadIdx.x; q < N * BITS; q += blockDim.x) {
        const int d = q / BITS, bit = q - d * BITS;
        float m0 = INFINITY, m1 = INFINITY;
        for (int r = 0; r < K; ++r) {
            const int idx = decision_index<L>(decs + (size_t)r * NW, d);
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
                a.out[vbase + u] = decision_index<L>(decs + (size_t)br * NW, d);
        }
    }
    __syncthreads();
}

// Instantiate f<N> for the user counts of one bucket (NMAX-7 .. NMAX) and
// call the one matching the runtime N (uniform across the workgroup).
#define MPNL_BUCKET_SWITCH(NMAX, N, CALL)                                                          \
    switch ((NMAX) - (N)) {                                                                        \
    case 0: { constexpr int NN = (NMAX); CALL; } break;                                            \
    case 1: { constexpr int NN = (NMAX) - 1; CALL; } break;                                        \
    case 2: { constexpr int NN = (NMAX) - 2; CALL; } break;                                        \
    case 3: { constexpr int NN = (NMAX) - 3; CALL; } break;                                        \
    case 4: { constexpr int NN = (NMAX) - 4; CALL; } break;                                        \
    case 5: { constexpr int NN = (NMAX) - 5; CALL; } break;                                        \
    case 6: { constexpr int NN = (NMAX) - 6; CALL; } break;                                        \
    case 7: { constexpr int NN = (NMAX) - 7; CALL; } break;                                        \
    default: break;                                                                                \
    }

template <int NMAX, int L>
__global__ __launch_bounds__(256) void path_search_soft_kernel(PathArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int s = lb / a.T, t = lb - s * a.T;
    MPNL_BUCKET_SWITCH(NMAX, a.N, (soft_vector<NN, L>(a, s, t, smem)))
}

// ============================================================================
// Path search over many jobs (cells) that share the user count N, the
// modulation and the lanes per received vector (paths rounded up to a
// wavefront).  Received vectors are numbered job by job, (job, subcarrier,
// symbol), subcarrier-major.  Each vector's paths split into `groups` path
// groups of gw = lanes / groups lanes (whole wavefronts); a workgroup runs
// ipw work items (vector, group).
// Item (vector, g) (numbered as work_item says) runs paths g gw .. g gw +
// gw - 1 exactly as path_search_kernel runs them, so a job's result depends neither on the
// other jobs of the launch nor on the launch shape.  With one group the
// winner writes the vector's symbols; with several, each group leaves its
// best in the job's partial records (JobDev::part) for
// path_group_reduce_multi_kernel.  One-wavefront groups (gw = 64) share no
// barrier, so a wavefront that pruning stops early frees its slot at once.
// ============================================================================
struct MultiArgs {
    const JobDev *jobs;
    int n_jobs;
    int total_items;  // received vectors of all jobs
    int ipw;          // work items per workgroup
    int gw;           // lanes per path group (64 or the whole vector's lanes)
    int groups;       // path groups per vector
    int gmajor;       // 1: work items numbered path group major (work_item)
};

template <int N, int L, int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PathOccupancy<PREC>::waves))) void
path_search_multi_kernel(MultiArgs a)
{
    __shared__ float sm[4];
    __shared__ int sr[4];
    constexpr int NW = (N + 3) / 4;
    const int W = a.gw;
    const int q = __builtin_amdgcn_readfirstlane((int)threadIdx.x / W);  // whole waves per item
    int vitem, g;
    work_item(q, a.groups, a.ipw, a.gmajor != 0, vitem, g);
    const bool active = vitem < a.total_items && g < a.groups;
    const int item = active ? vitem : a.total_items - 1;
    const JobDev &j = a.jobs[find_job(a.jobs, a.n_jobs, item)];
    const int li = item - j.item_begin;
    const int s = li / j.T, t = li - s * j.T;
    const size_t sN = (size_t)s * N;
    const size_t v = (size_t)t * j.S + s;
    cptr<uint32_t> rq = j.rq ? uniform_ptr(j.rq + 2 * sN * N) : nullptr;
    const float b0 = j.bound ? uniform_ptr(j.bound + v)[0] : INFINITY;
    const float *b0d = j.bound ? j.bound + (size_t)j.S * j.T + v * NW : nullptr;
    float *part = a.groups > 1 ? j.part + (v * a.groups + g) * (2 + NW) : nullptr;
    search_vector<N, L, PREC, kHalfStateNMulti>(
        uniform_ptr(j.yt + v * N), uniform_ptr(j.diag + sN), uniform_ptr(j.rlat + sN * N), rq,
        j.P + (size_t)s * j.K * j.NP, j.order ? j.order + (size_t)s * j.K : nullptr, j.K, j.NP, g, j.permd + sN,
        j.out + v * N, part, sm, sr, W, (int)threadIdx.x - q * W, active, b0, b0d);
}

// Best of the path groups of every received vector of a multi-job launch.
// One lane per received vector (numbered as in path_search_multi_kernel).
template <int L>
__global__ __launch_bounds__(64) void path_group_reduce_multi_kernel(MultiArgs a)
{
    const int item = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (item >= a.total_items)
        return;
    const JobDev &j = a.jobs[find_job(a.jobs, a.n_jobs, item)];
    const int li = item - j.item_begin;
    const int s = li / j.T, t = li - s * j.T;
    const size_t v = (size_t)t * j.S + s;
    const int N = j.N;
    reduce_groups<L>(j.part + v * a.groups * (2 + (N + 3) / 4), a.groups, N, j.permd + (size_t)s * N,
                     j.out + v * N);
}

// ============================================================================
// Pruning record: path 0 (first choice at every depth) of every received
// vector, computed with the same descent as the path search; the metrics,
// (T, S) floats, then the packed decisions, (T, S, (N + 3) / 4) floats.
// One lane per received vector, vectors numbered subcarrier-major (index
// s T + t), so the lanes of a wavefront share few subcarriers and every lane
// does work; R is read through each lane's own subcarrier.
template <int N, int L, int PREC>
__device__ __forceinline__ void bound_body(const float2 *yt, const float4 *diag, const float2 *rlat,
                                           const uint32_t *rq, int S, int T, int i0, float *bound)
{
    constexpr int NW = (N + 3) / 4;
    const int i = i0 + (int)(threadIdx.x & 63u);
    const int ic = min(i, S * T - 1);
    const int s = ic / T, t = ic - s * T;
    const size_t sN = (size_t)s * N;
    YLanes<N> yl;
    const float2 *yv = yt + ((size_t)t * S + s) * N;
#pragma unroll
    for (int d = 0; d < N; ++d)
        yl.v[d] = yv[d];
    const RLanes R{(const float *)(diag + sN), (const float *)(rlat + sN * N), rq ? rq + 2 * sN * N : nullptr};
    uint32_t pw[NW];
    float decf[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        pw[w] = 0x01010101u;
        decf[w] = 0.f;
    }
    const float m = descend<N, L, PREC, true>(yl, R, pw, decf, INFINITY, true);
    if (i < S * T) {
        const size_t v = (size_t)t * S + s;
        bound[v] = m;
        float *dec = bound + (size_t)S * T + v * NW;
#pragma unroll
        for (int w = 0; w < NW; ++w)
            dec[w] = decf[w];
    }
}

// grid: ceil(S * T / 64) wavefronts
template <int N, int L, int PREC>
__global__ __launch_bounds__(64) void path_bound_kernel(PathArgs a)
{
    bound_body<N, L, PREC>(a.yt, a.diag, a.rlat, a.rq, a.S, a.T, (int)blockIdx.x * 64, a.bound);
}

// Many jobs of one (N, L): item = (job, 64 received vectors), numbered job by
// job from JobDev::bound_begin (ceil(S * T / 64) items a job).
__device__ __forceinline__ int find_bound_job(const JobDev *jobs, int n_jobs, int item)
{
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].bound_begin <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int N, int L, int PREC>
__global__ __launch_bounds__(64) void path_bound_multi_kernel(const JobDev *jobs, int n_jobs)
{
    const JobDev &j = jobs[find_bound_job(jobs, n_jobs, (int)blockIdx.x)];
    bound_body<N, L, PREC>(j.yt, j.diag, j.rlat, j.rq, j.S, j.T, ((int)blockIdx.x - j.bound_begin) * 64, j.bound);
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
