// a2 for up to 256 paths: the position-vector set held by one workgroup of
// E wavefronts, one list entry per lane.
//
// Same definition as posvec_kernel (prep.hip): the K cheapest position
// vectors, cost = sum_d c_d (p_d - 1) in exact integers (cost_unit), equal
// costs ordered by the cost of the longest prefix, then the next shorter,
// and equal prefix costs throughout lexicographically: the key
// (C_N, C_{N-1}, ..., C_1, p), which is exactly (cost, position of the
// parent prefix in its own sorted list, k) applied depth by depth.  Depth by
// depth the list of the K cheapest prefixes A is extended by rank doubling:
//     U_0 = A (rank 0 at this depth),   U_{j+1} = topK(U_j  U  raise(U_j, 2^j)),
// where raise(., c) adds c to the last rank (cost parent + c_d k), so U_j
// holds the K cheapest extensions with rank below 2^j; log2 |Q| merges cover
// every rank.  The top K of a union is the top K of the unions of top Ks,
// which makes each step exact, and raising adds the same c_d 2^j to every
// entry, so the raised list stays sorted.
// Every merge is a bitonic network: thread g holds entry g of the list
// (g = 64 w + lane for wavefront w).  One half-cleaner stage compares U_j
// with the reversed raised list, then log2(64 E) compare-exchange stages sort
// the K smallest.  The half cleaner and each stage across wavefronts go
// through LDS (alternating buffers, one barrier each), the stages inside a
// wavefront use DPP / row-swap lane exchanges.  An entry is one 64-bit key,
// cost << 32 | parent position << 6 | k, so that (cost, parent, k) compares
// as one unsigned integer; an entry of A is its own parent with k = 0 at the
// next depth, so no rank of the new list has to be computed.
#include "device_common.h"

#include <algorithm>

namespace mpnl {
namespace dev {
namespace {

constexpr uint64_t kNone = ~0ull;  // empty list entry: above every key

__device__ __forceinline__ uint64_t pkey(uint32_t cost, uint32_t packed)
{
    return ((uint64_t)cost << 32) | packed;
}
__device__ __forceinline__ uint32_t key_cost(uint64_t k) { return (uint32_t)(k >> 32); }
__device__ __forceinline__ uint32_t key_packed(uint64_t k) { return (uint32_t)k; }

// Compare-exchange of key c with the key of lane ^ S, keeping the smaller in
// the lower lane when `asc`, the larger otherwise.  At distance 16 or 32 one
// swap gives both keys of the pair and the lane's side picks; below, the
// partner's key comes from DPP.
template <int S>
__device__ __forceinline__ void lane_stage(uint64_t &c, bool asc)
{
    if constexpr (S >= 16) {
        uint64_t lo, hi;
        lane_pair<S>(c, lo, hi);
        const bool upper = (threadIdx.x & (unsigned)S) != 0;
        c = ((hi < lo) != upper) == asc ? hi : lo;
    } else {
        const uint64_t o = lane_xor_n(c, S);
        const bool lower = (threadIdx.x & (unsigned)S) == 0;
        c = ((lower == asc) == (o < c)) ? o : c;
    }
}

// The same at a run-time distance (constant after unrolling).
__device__ __forceinline__ void lane_stage_n(uint64_t &c, int s, bool asc)
{
    switch (s) {
    case 1: lane_stage<1>(c, asc); break;
    case 2: lane_stage<2>(c, asc); break;
    case 4: lane_stage<4>(c, asc); break;
    case 8: lane_stage<8>(c, asc); break;
    case 16: lane_stage<16>(c, asc); break;
    default: lane_stage<32>(c, asc); break;
    }
}

// Inclusive prefix sum over the 64 lanes: four row shifts inside each row of
// 16, then row 0's total into row 1 and row 2's into row 3 (row_bcast:15),
// then the total of rows 0-1 into rows 2-3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false); // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false); // row_bcast:31
    return v;
}

template <int E>
struct PosLds {
    static constexpr int KP = 64 * E;
    uint64_t xk[2][2][KP]; // exchange: [buffer][Z | B] keys
    uint64_t bck[2];       // broadcast of entry K-1 of Z
    uint64_t akK1[2];      // key of entry K - 1 of A (two buffers, as scA)
    uint32_t scA[2][KP];   // costs of list A by position: the current list and the next
};

// LDS of one workgroup: PosLds, then N * KP back pointers per depth, 16 bits
// each (parent position | k << 8).  For 256 paths and N = 16 that is 18 KB,
// so eight workgroups fit a compute unit and a 1200-subcarrier slot runs in a
// single round of workgroups.  REC_LDS = false: the back pointers live in
// global memory (PosArgs::rec16) and the LDS holds PosLds only (10 KB for 256
// paths), for slots where the larger count saves a round.
template <int E, bool REC_LDS = true>
constexpr size_t pos_lds_bytes(int N)
{
    return sizeof(PosLds<E>) + (REC_LDS ? (size_t)N * 64 * E * sizeof(uint16_t) : 0);
}

template <int E, bool REC_LDS = true>
__device__ __forceinline__ void posvec_body(const PosArgs &a, int s, unsigned char *smem)
{
    constexpr int KP = 64 * E;
    PosLds<E> &sh = *(PosLds<E> *)smem;
    uint16_t *rec = REC_LDS ? (uint16_t *)(smem + sizeof(PosLds<E>)) : a.rec16 + (size_t)s * a.N * KP;
    const int g = (int)threadIdx.x;  // list entry of this lane
    const int lane = g & 63, wv = g >> 6;
    const int K = a.K, N = a.N, nq = a.nq;

    uint64_t Ak = g == 0 ? 0ull : kNone;  // the root: cost 0, packed 0
    int cur = 0;                          // buffer of the current list A
    sh.scA[0][g] = key_cost(Ak);
    if (g == K - 1)
        sh.akK1[0] = Ak;
    // the depth costs, lane d holding c_d (N <= 32), read per depth from a
    // register instead of a dependent load
    const double wl = lane < N ? a.w[(size_t)s * N + lane] : 0.0;
    double wmax = wl;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1)
        wmax = fmax(wmax, lane_xor_n(wmax, o));  // every lane: the largest weight
    const uint32_t cl = cost_unit(wl, wmax);
    __syncthreads();

    int buf = 0;
    for (int d = 0; d < N; ++d) {
        const uint32_t c = lane_read(cl, d);
        uint64_t Z = Ak;  // every entry of A as parent with k = 0
        const uint32_t *scA = sh.scA[cur];
        const uint32_t a0s = scA[0];
        // A full list that not even the cheapest entry with rank 2 at this
        // depth (entry 0 raised by one) can enter: every prefix extends by
        // rank 1 only, so positions and costs stay as they are and only the
        // back pointers (parent = itself, k = 0) are written; no LDS state
        // changes, no barrier.  (The merge loop below would stop at its
        // first check.)  The decision reads LDS written before the last
        // barrier, so every lane takes it alike.
        if (d > 0) {
            const uint64_t last = sh.akK1[cur];
            if (last != kNone && !(pkey(a0s + c, 1u) < last)) {
                if (Ak != kNone)
                    rec[(size_t)d * KP + g] = (uint16_t)(g & 0xff);
                continue;
            }
        }
        // The first depth extends the root only: its children k = 0 .. |Q|-1
        // are already in key order (costs non-decreasing in k, equal costs
        // ordered by k), so entry g is child g and no merge is needed.
        if (d == 0)
            Z = g < min(nq, K) ? pkey(c * (uint32_t)g, (uint32_t)g) : kNone;
        // Z covers the ranks k < span of this depth; merging Z with its copy
        // raised by span covers k < 2 span (|Q| is a power of two, so the
        // raised ranks never pass |Q| - 1)
        for (int span = d == 0 ? nq : 1; span < nq; span <<= 1) {
            const bool ok = Z != kNone;
            const uint32_t zp = key_packed(Z);
            const uint32_t k1 = (zp & 63) + (uint32_t)span;
            const uint64_t B = ok ? pkey(scA[ok ? (zp >> 6) : 0] + c * k1, zp + (uint32_t)span) : kNone;
            uint64_t l, m;
            if constexpr (E == 1) {
                l = lane_read(Z, K - 1);
                const uint64_t r = lane_mirror(B);  // entry 63 - g of B
                m = r < Z ? r : Z;
            } else {
                buf ^= 1;
                sh.xk[buf][1][g] = B;
                if (g == K - 1)
                    sh.bck[buf] = Z;
                __syncthreads();
                l = sh.bck[buf];
            }
            // stop when the cheapest entry with rank span can no longer
            // enter a full list (the same decision in every lane)
            if (l != kNone && !(pkey(a0s + c * (uint32_t)span, (uint32_t)span) < l))
                break;
            if constexpr (E > 1) {
                // half cleaner (entry g against entry KP - 1 - g of B), then
                // the stages across wavefronts, one LDS exchange each
                // (alternating buffers: one barrier per exchange)
                {
                    const uint64_t r = sh.xk[buf][1][KP - 1 - g];
                    m = r < Z ? r : Z;
                }
#pragma unroll
                for (int js = E / 2; js >= 1; js >>= 1) {
                    buf ^= 1;
                    sh.xk[buf][0][g] = m;
                    __syncthreads();
                    const uint64_t o = sh.xk[buf][0][g ^ (64 * js)];
                    const bool lower = (g & (64 * js)) == 0;
                    m = (lower == (o < m)) ? o : m;
                }
            }
            Z = m;
            lane_stage<32>(Z, true);
            lane_stage<16>(Z, true);
            lane_stage<8>(Z, true);
            lane_stage<4>(Z, true);
            lane_stage<2>(Z, true);
            lane_stage<1>(Z, true);
            if (g >= K)
                Z = kNone;
        }
        // the new list: back pointers, and every entry the parent of rank 0
        // at the next depth
        if (Z != kNone) {
            const uint32_t zp = key_packed(Z);
            rec[(size_t)d * KP + g] = (uint16_t)(((zp >> 6) & 0xffu) | ((zp & 63u) << 8));  // parent < 256
            Ak = pkey(key_cost(Z), (uint32_t)g << 6);
        } else {
            Ak = kNone;
        }
        // into the other buffer (its last readers passed the barrier that
        // ended the previous depth), then one barrier
        sh.scA[cur ^ 1][g] = key_cost(Ak);
        if (g == K - 1)
            sh.akK1[cur ^ 1] = Ak;
        cur ^= 1;
        __syncthreads();
    }

    // rebuild the position vectors (ranks 1..|Q|), rows padded with 1, and
    // note for each which depths ask for a rank >= 3 and >= 2
    const int r = g;
    uint64_t ks = kNone;  // sort key of path r; paths past K sort last
    if (r < K) {
        // one word of four depths at a time, written when its lowest depth
        // is in (the top word keeps its padding bytes)
        uint32_t *dst = (uint32_t *)(a.P + ((size_t)s * a.K + r) * a.NP);
        uint32_t w = 0x01010101u;
        uint32_t m5 = 0, m3 = 0, m2 = 0;
        int pidx = r;
        for (int d = N - 1; d >= 0; --d) {
            const uint32_t e = rec[(size_t)d * KP + pidx];
            const uint32_t pk = (e >> 8) + 1u;
            pidx = (int)(e & 0xffu);
            m5 |= (pk >= 5u ? 1u : 0u) << d;
            m3 |= (pk >= 3u ? 1u : 0u) << d;
            m2 |= (pk >= 2u ? 1u : 0u) << d;
            const uint32_t sh8 = (uint32_t)(d & 3) * 8u;
            w = (w & ~(0xffu << sh8)) | (pk << sh8);
            if ((d & 3) == 0) {
                dst[d >> 2] = w;
                w = 0x01010101u;
            }
        }
        // sort key: the first depth with a rank >= 2 (paths that leave the
        // first-choice path early are pruned early, and the pruning stops
        // whole wavefronts), the first depths with a rank >= 3 and >= 5 (the
        // costly point choices start together), then folds of the depths
        // with rank >= 3 and >= 2 (the key only groups paths; any order is
        // correct), then the path itself.  Fields: 6 + 6 + 6 + 20 + 15 + 8
        // bits.
        const uint32_t fd = m2 ? (uint32_t)__builtin_ctz(m2) : (uint32_t)N;
        const uint32_t f3 = m3 ? (uint32_t)__builtin_ctz(m3) : (uint32_t)N;
        const uint32_t f5 = m5 ? (uint32_t)__builtin_ctz(m5) : (uint32_t)N;
        const uint32_t m3f = (m3 ^ (m3 >> 20)) & 0xfffffu;
        const uint32_t m2f = (m2 ^ (m2 >> 15) ^ (m2 >> 30)) & 0x7fffu;
        ks = ((uint64_t)fd << 55) | ((uint64_t)f3 << 49) | ((uint64_t)f5 << 43) | ((uint64_t)m3f << 23) |
             ((uint64_t)m2f << 8) | (uint64_t)r;
    }
    // Lane order: paths sorted by that key, so that the lanes of one
    // wavefront leave path 0 at about the same depth and need the costly
    // point choices at the same depths.
    // order[i] = path run by lane i.  Full bitonic sort of the KP entries;
    // distances of 64 and more go through LDS.
    if (a.order != nullptr) {
#pragma unroll
        for (int size = 2; size <= KP; size <<= 1) {
            const bool asc = (g & size) == 0;
#pragma unroll
            for (int stride = size / 2; stride >= 1; stride >>= 1) {
                if (stride >= 64) {
                    sh.xk[buf][0][g] = ks;
                    __syncthreads();
                    const uint64_t o = sh.xk[buf][0][g ^ stride];
                    buf ^= 1;
                    const bool lower = (g & stride) == 0;
                    ks = ((lower == asc) == (o < ks)) ? o : ks;
                } else {
                    lane_stage_n(ks, stride, asc);
                }
            }
        }
        if (g < K)
            a.order[(size_t)s * K + g] = (uint16_t)(ks & 0xffu);
    }
}

template <int E, bool REC_LDS>
__global__ __launch_bounds__(64 * E) void posvec_reg_kernel(PosArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    posvec_body<E, REC_LDS>(a, blockIdx.x, smem);
}

// One launch for the position sets of many jobs (all with N_p <= 64 E and
// N <= the launch's largest N, which sizes the LDS):
// workgroup b runs subcarrier b - item_begin of the job that owns item b.
template <int E>
__global__ __launch_bounds__(64 * E) void posvec_batch_kernel(const StageJob *jobs, int n_jobs)
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
    a.rec16 = nullptr;
    a.order = j.sd.order;
    posvec_body<E>(a, blockIdx.x - j.item_begin, smem);
}

}  // namespace
}  // namespace dev

size_t posvec_reg_lds_bytes(int N, int K)
{
    using namespace dev;
    return K <= 64 ? pos_lds_bytes<1>(N) : K <= 128 ? pos_lds_bytes<2>(N) : pos_lds_bytes<4>(N);
}

hipError_t launch_posvec_batch(const dev::StageJob *jobs, int n_jobs, int items, int E, int Nmax,
                               hipStream_t st)
{
    using namespace dev;
    if (E == 1)
        hipLaunchKernelGGL(posvec_batch_kernel<1>, dim3(items), dim3(64), pos_lds_bytes<1>(Nmax), st, jobs, n_jobs);
    else if (E == 2)
        hipLaunchKernelGGL(posvec_batch_kernel<2>, dim3(items), dim3(128), pos_lds_bytes<2>(Nmax), st, jobs,
                           n_jobs);
    else if (E == 4)
        hipLaunchKernelGGL(posvec_batch_kernel<4>, dim3(items), dim3(256), pos_lds_bytes<4>(Nmax), st, jobs,
                           n_jobs);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_posvec_reg(const dev::PosArgs &a, hipStream_t st)
{
    using namespace dev;
    if (a.K <= 64)
        hipLaunchKernelGGL((posvec_reg_kernel<1, true>), dim3(a.S), dim3(64), pos_lds_bytes<1>(a.N), st, a);
    else if (a.K <= 128)
        hipLaunchKernelGGL((posvec_reg_kernel<2, true>), dim3(a.S), dim3(128), pos_lds_bytes<2>(a.N), st, a);
    else if (a.K <= 256 && a.rec16 == nullptr)
        hipLaunchKernelGGL((posvec_reg_kernel<4, true>), dim3(a.S), dim3(256), pos_lds_bytes<4>(a.N), st, a);
    else if (a.K <= 256) {
        const size_t lds = pos_lds_bytes<4, false>(a.N);
        hipLaunchKernelGGL((posvec_reg_kernel<4, false>), dim3(a.S), dim3(256), lds, st, a);
    }
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

bool posvec_reg_rec_global(int S, int N, int K, int cus, size_t lds_per_cu)
{
    using namespace dev;
    if (K <= 128 || K > 256 || cus <= 0 || lds_per_cu == 0)
        return false;
    // workgroups of 4 wavefronts a compute unit: at most 8 (eight wavefronts
    // a SIMD), fewer when the LDS runs out
    const long with = std::min<long>(8, (long)(lds_per_cu / pos_lds_bytes<4>(N)));
    const long without = std::min<long>(8, (long)(lds_per_cu / pos_lds_bytes<4, false>(N)));
    if (with <= 0)
        return without > 0;
    const long rounds_with = (S + cus * with - 1) / (cus * with);
    const long rounds_without = (S + cus * without - 1) / (cus * without);
    return rounds_without < rounds_with;
}

}  // namespace mpnl
