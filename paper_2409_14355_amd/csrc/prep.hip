// a1 (sorted QR), a2 (position-vector set) and a3 (rotation on MFMA) kernels
// of the MPNL uplink detector (arXiv 2409.14355, Sec. II), gfx950.
#include "device_common.h"

namespace mpnl {
namespace dev {

// ============================================================================
// a1: sorted QR.
// Lane c of a half-wave holds column c of H (rows padded with zeros to MMAX).
// Step i: every column not yet placed computes its residual norm^2 over rows
// >= i (float32 FMAs; float64 took 8% more of the batched a1 and decided no
// tested pivot differently); the smallest (equal: lower column index) is placed at
// position i.  Its Householder reflector H_i = I - tau v v^H maps the
// residual onto e_i; it is broadcast through LDS and applied to every column
// not yet placed.  Row i of R is then rotated by conj(phi_i) so that R_ii is
// real and positive, and Q's column i by phi_i (Q R is unchanged).
// Q = H_0 H_1 ... H_{N-1} [I; 0] is accumulated per column at the end.
// ============================================================================
struct SqrdArgs {
    const float2 *H;
    int S, M, N;
    float delta;
    SlotDev sd;
};

__device__ __forceinline__ uint32_t pack_half2(float x, float y)
{
    half2_t h;
    h.x = (_Float16)x;
    h.y = (_Float16)y;
    return __builtin_bit_cast(uint32_t, h);
}

__device__ __forceinline__ uint32_t bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u)  // NaN: keep it a NaN
        return (u >> 16) | 0x40u;
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;  // round to nearest even
}

template <int MMAX>
__device__ __forceinline__ void sqrd_body(const SqrdArgs &a, int pair)
{
    __shared__ float2 V[2][kMaxN][MMAX];
    __shared__ float TAU[2][kMaxN];
    __shared__ float2 PHI[2][kMaxN];

    const int half = threadIdx.x >> 5;
    const int c = threadIdx.x & 31;
    const int s = pair * 2 + half;
    const int M = a.M, N = a.N;
    const bool active = (s < a.S) && (c < N);

    float2 col[MMAX];
#pragma unroll
    for (int m = 0; m < MMAX; ++m) {
        col[m] = make_float2(0.f, 0.f);
        if (active && m < M)
            col[m] = a.H[((size_t)s * M + m) * N + c];
    }

    bool placed = false;
    int pos = 0;
    double wnorm = 0.0;

#pragma unroll
    for (int i = 0; i < MMAX; ++i) {
        if (i < N) {
        float nu = 0.f;
#pragma unroll
        for (int m = i; m < MMAX; ++m)
            nu = fmaf(col[m].y, col[m].y, fmaf(col[m].x, col[m].x, nu));

        const bool cand = active && !placed;
        float key = cand ? nu : INFINITY;
        int id = cand ? c : (1 << 20);
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) {
            const float ok = lane_xor_n(key, off);  // stays inside the 32-lane half
            const int oid = lane_xor_n(id, off);
            if ((ok < key) | ((ok == key) & (oid < id))) {
                key = ok;
                id = oid;
            }
        }
        const bool me = cand && (c == id);
        if (me) {
            const float alpha = (float)sqrt(nu);
            const float2 x0 = col[i];
            const float ax0 = sqrtf(x0.x * x0.x + x0.y * x0.y);
            float2 e = make_float2(1.f, 0.f);
            if (ax0 > 0.f) {
                const float r = 1.f / ax0;  // one division for both components
                e = make_float2(x0.x * r, x0.y * r);
            }
#pragma unroll
            for (int m = 0; m < MMAX; ++m) {
                float2 v = (m < i) ? make_float2(0.f, 0.f) : col[m];
                if (m == i) {
                    v.x += e.x * alpha;
                    v.y += e.y * alpha;
                }
                V[half][i][m] = v;
            }
            TAU[half][i] = (alpha > 0.f) ? 1.f / (alpha * (alpha + ax0)) : 0.f;
            PHI[half][i] = make_float2(-e.x, -e.y);
            placed = true;
            pos = i;
            wnorm = nu;
        }
        __syncthreads();
        if (active && (!placed || me)) {
            const float tau = TAU[half][i];
            float gr = 0.f, gi = 0.f;  // v^H col
#pragma unroll
            for (int m = i; m < MMAX; ++m) {
                const float2 v = V[half][i][m];
                gr = fmaf(v.x, col[m].x, gr);
                gr = fmaf(v.y, col[m].y, gr);
                gi = fmaf(v.x, col[m].y, gi);
                gi = fmaf(-v.y, col[m].x, gi);
            }
            gr *= tau;
            gi *= tau;
#pragma unroll
            for (int m = i; m < MMAX; ++m) {
                const float2 v = V[half][i][m];
                // col -= g v as two FMAs a component (a product-then-
                // difference form took a multiply, an FMA and a subtraction;
                // a1 of 40 cells 0.96 -> 0.89 ms)
                col[m].x = fmaf(gi, v.y, fmaf(-gr, v.x, col[m].x));
                col[m].y = fmaf(-gi, v.x, fmaf(-gr, v.y, col[m].y));
            }
            const float2 ph = PHI[half][i];  // row i *= conj(phi_i)
            const float xr = col[i].x * ph.x + col[i].y * ph.y;
            const float xi = col[i].y * ph.x - col[i].x * ph.y;
            col[i] = make_float2(xr, xi);
            if (me) {
                col[i] = make_float2((float)sqrt(nu), 0.f);
#pragma unroll
                for (int m = i + 1; m < MMAX; ++m)
                    col[m] = make_float2(0.f, 0.f);
            }
        }
        }
    }

    // ---- outputs of R, in depth order ----
    // a = R_ll * Delta of every row, shared so that entries can be put in the
    // lattice units of the row they update
    __shared__ float INVA[2][kMaxN];
    const int d = N - 1 - pos;
    const float rll = (float)sqrt(wnorm);
    const float aa = rll * a.delta;
    const float inva = aa > 0.f ? 1.f / aa : 1.f;
    if (active)
        INVA[half][pos] = inva;
    __syncthreads();
    if (active) {
        const size_t sN = (size_t)s * N;
        a.sd.diag[sN + d] = make_float4(aa > 0.f ? aa * aa : 1.f, aa > 0.f ? 0.f : 1.f, inva, rll);
        a.sd.wd[sN + d] = wnorm;
        a.sd.permd[sN + d] = c;
#pragma unroll
        for (int m = 0; m < MMAX; ++m) {
            if (m < pos) {
                const int d2 = N - 1 - m;
                const size_t o = (sN + d) * N + d2;   // roff: [d][d2]
                const size_t ot = (sN + d2) * N + d;  // lattice copies transposed: row d2, term of depth d
                const float sc = a.delta * INVA[half][m];
                const float lx = col[m].x * sc, ly = col[m].y * sc;
                a.sd.roff[o] = col[m];
                a.sd.rlat[ot] = make_float2(lx, ly);
                a.sd.rlat_h[2 * ot] = pack_half2(lx, ly);
                a.sd.rlat_h[2 * ot + 1] = pack_half2(ly, -lx);
                a.sd.rlat_b[2 * ot] = bf16_bits(lx) | (bf16_bits(ly) << 16);
                a.sd.rlat_b[2 * ot + 1] = bf16_bits(ly) | (bf16_bits(-lx) << 16);
            }
        }
    }

    // ---- Q column = phi_pos * H_0 ... H_pos e_pos ----
    float2 q[MMAX];
#pragma unroll
    for (int m = 0; m < MMAX; ++m)
        q[m] = make_float2(m == pos ? 1.f : 0.f, 0.f);
#pragma unroll
    for (int j = MMAX - 1; j >= 0; --j) {
        if (j < N && active && j <= pos) {
            const float tau = TAU[half][j];
            float gr = 0.f, gi = 0.f;
#pragma unroll
            for (int m = j; m < MMAX; ++m) {
                const float2 v = V[half][j][m];
                gr = fmaf(v.x, q[m].x, gr);
                gr = fmaf(v.y, q[m].y, gr);
                gi = fmaf(v.x, q[m].y, gi);
                gi = fmaf(-v.y, q[m].x, gi);
            }
            gr *= tau;
            gi *= tau;
#pragma unroll
            for (int m = j; m < MMAX; ++m) {
                const float2 v = V[half][j][m];
                q[m].x = fmaf(gi, v.y, fmaf(-gr, v.x, q[m].x));
                q[m].y = fmaf(-gi, v.x, fmaf(-gr, v.y, q[m].y));
            }
        }
    }
    if (active) {
        const float2 ph = PHI[half][pos];
#pragma unroll
        for (int m = 0; m < MMAX; ++m) {
            if (m < M) {
                const float2 z = q[m];
                a.sd.Qd[((size_t)s * M + m) * N + d] =
                    make_float2(z.x * ph.x - z.y * ph.y, z.x * ph.y + z.y * ph.x);
            }
        }
    }
}

template <int MMAX>
__global__ __launch_bounds__(64) void sqrd_kernel(SqrdArgs a)
{
    sqrd_body<MMAX>(a, blockIdx.x);
}

// One launch for the sorted QRs of many jobs: workgroup b runs subcarrier
// pair b - item_begin of the job that owns item b.
template <int MMAX>
__global__ __launch_bounds__(64) void sqrd_batch_kernel(const StageJob *jobs, int n_jobs)
{
    const StageJob &j = jobs[find_job(jobs, n_jobs, blockIdx.x)];
    SqrdArgs a;
    a.H = j.H;
    a.S = j.sd.S;
    a.M = j.sd.M;
    a.N = j.sd.N;
    a.delta = j.delta;
    a.sd = j.sd;
    sqrd_body<MMAX>(a, blockIdx.x - j.item_begin);
}

// ============================================================================
// a2: position-vector set.
// The cost of a position vector is sum_d c_d (p_d - 1) in exact integers
// (cost_unit: the depth weights scaled to 2^kCostBits of the largest and
// rounded).  Depth by depth, the list of the K cheapest prefixes (in key
// order, below) is extended: candidates are (prefix i, k) with cost
// sc_i + c_d k, k = 0..|Q|-1.  Because every copy "list + k c_d" is a
// shifted copy of the sorted list, the top-K of their union is built as
//     Z_0 = list,  Z_m = topK(list  U  shift(Z_{m-1})),
// stopping when the cheapest entry with p_d = m+1 can no longer enter.
// Each merge is a merge-path over two sorted lists in LDS.  Ties in cost are
// ordered by the position of the parent prefix in its sorted list, then k:
// the key (C_N, C_{N-1}, ..., C_1, p) of the definition, C_j the cost of the
// first j depths.  Back pointers (parent, k) per depth rebuild the vectors
// at the end.
// ============================================================================

__device__ __forceinline__ bool key_less(uint32_t sa, int la, int ka, uint32_t sb, int lb, int kb)
{
    return sa < sb || (sa == sb && (la < lb || (la == lb && ka < kb)));
}

template <bool REC_LDS>
__global__ __launch_bounds__(64) void posvec_kernel(PosArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int K = a.K, N = a.N, nq = a.nq;
    const int lane = threadIdx.x;
    const int s = blockIdx.x;

    uint32_t *A_sc = (uint32_t *)smem;
    uint32_t *Zs[2] = {A_sc + K, A_sc + 2 * K};
    uint16_t *Zp[2] = {(uint16_t *)(A_sc + 3 * K), (uint16_t *)(A_sc + 3 * K) + K};
    uint16_t *Zk[2] = {Zp[1] + K, Zp[1] + 2 * K};
    uint32_t *rec = REC_LDS ? (uint32_t *)(Zp[0] + ((4 * K + 1) & ~1)) : (a.rec_g + (size_t)s * N * K);

    if (lane == 0)
        A_sc[0] = 0u;
    int n = 1;
    double wmax = 0.0;
    for (int d = 0; d < N; ++d)
        wmax = fmax(wmax, a.w[(size_t)s * N + d]);
    __syncthreads();

    for (int d = 0; d < N; ++d) {
        const uint32_t cd = cost_unit(a.w[(size_t)s * N + d], wmax);
        int cur = 0;
        for (int i = lane; i < n; i += 64) {
            Zs[0][i] = A_sc[i];
            Zp[0][i] = (uint16_t)i;
            Zk[0][i] = 0;
        }
        int zn = n;
        __syncthreads();
        for (int m = 1; m < nq; ++m) {
            if (zn == K) {
                const uint32_t nm = A_sc[0] + cd * (uint32_t)m;
                const int zp = Zp[cur][K - 1];
                if (!key_less(nm, 0, m, Zs[cur][K - 1], zp, Zk[cur][K - 1]))
                    break;
            }
            // merge list A (k = 0) with B = shift(Z_cur) into Z_nxt
            const int nxt = cur ^ 1;
            const int total = min(K, n + zn);
            const int chunk = (total + 63) / 64;
            const int p0 = min(total, lane * chunk);
            const int p1 = min(total, p0 + chunk);
            const uint16_t *zp = Zp[cur];
            const uint16_t *zk = Zk[cur];
            if (p0 < p1) {
                int lo = max(0, p0 - zn), hi = min(p0, n);
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const int j = p0 - mid - 1;
                    const int par = zp[j];
                    const int kb = zk[j] + 1;
                    const uint32_t sb = A_sc[par] + cd * (uint32_t)kb;
                    if (key_less(A_sc[mid], mid, 0, sb, par, kb))
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                int i = lo, j = p0 - lo;
                for (int p = p0; p < p1; ++p) {
                    bool takeA;
                    uint32_t sb = 0u;
                    int par = 0, kb = 0;
                    if (j < zn) {
                        par = zp[j];
                        kb = zk[j] + 1;
                        sb = A_sc[par] + cd * (uint32_t)kb;
                    }
                    if (i >= n)
                        takeA = false;
                    else if (j >= zn)
                        takeA = true;
                    else
                        takeA = key_less(A_sc[i], i, 0, sb, par, kb);
                    if (takeA) {
                        Zs[nxt][p] = A_sc[i];
                        Zp[nxt][p] = (uint16_t)i;
                        Zk[nxt][p] = 0;
                        ++i;
                    } else {
                        Zs[nxt][p] = sb;
                        Zp[nxt][p] = (uint16_t)par;
                        Zk[nxt][p] = (uint16_t)kb;
                        ++j;
                    }
                }
            }
            __syncthreads();
            cur = nxt;
            zn = total;
        }
        for (int j = lane; j < zn; j += 64) {
            A_sc[j] = Zs[cur][j];
            rec[(size_t)d * K + j] = (uint32_t)Zp[cur][j] | ((uint32_t)Zk[cur][j] << 16);
        }
        n = zn;
        __syncthreads();
    }

    // rebuild the position vectors (ranks 1..|Q|), rows padded with 1: one
    // word of four depths at a time, stored when its lowest depth is in
    for (int r = lane; r < n; r += 64) {
        uint32_t *dst = (uint32_t *)(a.P + ((size_t)s * a.K + r) * a.NP);
        uint32_t w = 0x01010101u;
        int pidx = r;
        for (int d = N - 1; d >= 0; --d) {
            const uint32_t e = rec[(size_t)d * K + pidx];
            const uint32_t pk = (e >> 16) + 1u;
            pidx = (int)(e & 0xffffu);
            const uint32_t sh8 = (uint32_t)(d & 3) * 8u;
            w = (w & ~(0xffu << sh8)) | (pk << sh8);
            if ((d & 3) == 0) {
                dst[d >> 2] = w;
                w = 0x01010101u;
            }
        }
    }
}

// ============================================================================
// a3: yt = Q^H y on MFMA, each row then put in lattice units (times 1/a_l).
// Real form of the complex product:
//   [Re yt_d]   sum_m [ qr  qi ] [yr_m]
//   [Im yt_d] =       [-qi  qr ] [yi_m]
// A (2N x 2M) times B (2M x T) with v_mfma_f32_16x16x4_f32: lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; it receives D[4(l/16)+v][l%16], v = 0..3.
// ============================================================================
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct RotArgs {
    const float4 *diag;  // (S, N) .z = 1/a of the row
    const float2 *Qd;  // (S, M, N)
    const float2 *y;   // (T, S, M)
    float2 *yt;        // (T, S, N)
    int S, M, N, T;
};

// One workgroup per subcarrier.  Two forms with the same products in the
// same order (the same bits):
// rotate_body_direct: the B operands straight from HBM (16 bytes per lane,
// lanes a row of S M complex apart) and yt written per entry; lowest latency
// per subcarrier, used by the one-slot launches (a few thousand subcarriers,
// hidden behind the position set on the second stream).
__device__ __forceinline__ void rotate_body_direct(const RotArgs &a, int s)
{
    const int lane = threadIdx.x;
    const int i16 = lane & 15, kq = lane >> 4;
    const int M = a.M, N = a.N, T = a.T, S = a.S;
    const float2 *Qs = a.Qd + (size_t)s * M * N;
    const int rtiles = (2 * N + 15) / 16;
    const int ksteps = (2 * M + 3) / 4;
    const int ctiles = (T + 15) / 16;
    float *yt = (float *)a.yt;
    for (int ct = 0; ct < ctiles; ++ct) {
        const int tt = ct * 16 + i16;
        for (int rt = 0; rt < rtiles; ++rt) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
            const int row = rt * 16 + i16;
            const int d = row >> 1, part = row & 1;
            for (int ks = 0; ks < ksteps; ++ks) {
                const int k = ks * 4 + kq;
                const int m = k >> 1, cp = k & 1;
                float av = 0.f, bv = 0.f;
                if (m < M && d < N) {
                    const float2 qv = Qs[(size_t)m * N + d];
                    av = part == 0 ? (cp == 0 ? qv.x : qv.y) : (cp == 0 ? -qv.y : qv.x);
                }
                if (m < M && tt < T) {
                    const float2 yv = a.y[((size_t)tt * S + s) * M + m];
                    bv = cp == 0 ? yv.x : yv.y;
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int orow = rt * 16 + 4 * kq + v;
                const int od = orow >> 1, opart = orow & 1;
                if (od < N && tt < T)
                    yt[(((size_t)tt * S + s) * N + od) * 2 + opart] = acc[v] * a.diag[(size_t)s * N + od].z;
            }
        }
    }
}

// rotate_body_staged: 16 symbols at a time, the block of y (16 rows
// of M complex, each row contiguous in HBM) is loaded into LDS with
// consecutive lanes on consecutive entries of a row, the products take their
// B operands from there, and the outputs go through LDS again so that every
// row of yt (N complex) is written contiguously.  Used by the batched launch
// (tens of thousands of subcarriers), where HBM efficiency decides: 0.554 ->
// 0.485 ms for the rotation of 40 uneven cells; a 1200-subcarrier slot alone
// takes 0.028 ms this way against 0.019 direct.  One wavefront per row tile of
// 16 (the workgroup sized for the launch's largest N, waves past a job's
// tiles idle): 0.495 -> 0.440 ms for the 40 cells against one wavefront doing
// every tile.
__device__ __forceinline__ void rotate_body_staged(const RotArgs &a, int s)
{
    __shared__ float2 ys[16 * kMaxN];      // y of the block: [t][m]
    __shared__ float os[16 * 2 * kMaxN];   // yt of the block: [t][2 d + part]
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6, nw = nthr >> 6;  // one row tile per wavefront
    const int i16 = lane & 15, kq = lane >> 4;
    const int M = a.M, N = a.N, T = a.T, S = a.S;
    const float2 *Qs = a.Qd + (size_t)s * M * N;
    const float4 *dg = a.diag + (size_t)s * N;
    const int rtiles = (2 * N + 15) / 16;
    const int ksteps = (2 * M + 3) / 4;
    const int ctiles = (T + 15) / 16;
    float *yt = (float *)a.yt;
    for (int ct = 0; ct < ctiles; ++ct) {
        const int t0 = ct * 16;
        const int nt = min(16, T - t0);
        for (int f = tid; f < nt * M; f += nthr) {
            const int tl = f / M, m = f - tl * M;
            ys[tl * M + m] = a.y[((size_t)(t0 + tl) * S + s) * M + m];
        }
        __syncthreads();
        for (int rt = wv; rt < rtiles; rt += nw) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
            const int row = rt * 16 + i16;
            const int d = row >> 1, part = row & 1;
            for (int ks = 0; ks < ksteps; ++ks) {
                const int k = ks * 4 + kq;
                const int m = k >> 1, cp = k & 1;
                float av = 0.f, bv = 0.f;
                if (m < M && d < N) {
                    const float2 qv = Qs[(size_t)m * N + d];
                    av = part == 0 ? (cp == 0 ? qv.x : qv.y) : (cp == 0 ? -qv.y : qv.x);
                }
                if (m < M && i16 < nt) {
                    const float2 yv = ys[i16 * M + m];
                    bv = cp == 0 ? yv.x : yv.y;
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int orow = rt * 16 + 4 * kq + v;
                const int od = orow >> 1;
                if (od < N && i16 < nt)
                    os[i16 * 2 * N + orow] = acc[v] * dg[od].z;
            }
        }
        __syncthreads();
        for (int f = tid; f < nt * 2 * N; f += nthr) {
            const int tl = f / (2 * N), j = f - tl * 2 * N;
            yt[((size_t)(t0 + tl) * S + s) * N * 2 + j] = os[f];
        }
        __syncthreads();  // the next block rewrites ys and os
    }
}


__global__ __launch_bounds__(64) void rotate_kernel(RotArgs a)
{
    rotate_body_direct(a, blockIdx.x);
}

// One launch for the rotations of many jobs: workgroup b runs subcarrier
// b - item_begin of the job that owns item b.
__global__ __launch_bounds__(256) void rotate_batch_kernel(const StageJob *jobs, int n_jobs)
{
    const StageJob &j = jobs[find_job(jobs, n_jobs, blockIdx.x)];
    RotArgs a;
    a.diag = j.sd.diag;
    a.Qd = j.sd.Qd;
    a.y = j.y;
    a.yt = j.yt;
    a.S = j.sd.S;
    a.M = j.sd.M;
    a.N = j.sd.N;
    a.T = j.T;
    rotate_body_staged(a, blockIdx.x - j.item_begin);
}

template <int MMAX>
hipError_t sqrd_launch_t(const float2 *H, const SlotDev &sd, hipStream_t st)
{
    SqrdArgs a;
    a.H = H;
    a.S = sd.S;
    a.M = sd.M;
    a.N = sd.N;
    a.delta = delta_of(sd.bits);
    a.sd = sd;
    const int grid = (sd.S + 1) / 2;
    hipLaunchKernelGGL(sqrd_kernel<MMAX>, dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace dev

using namespace dev;

hipError_t launch_sqrd_batch(const StageJob *jobs, int n_jobs, int items, int mmax, hipStream_t st)
{
    switch (mmax) {
    case 4: hipLaunchKernelGGL(sqrd_batch_kernel<4>, dim3(items), dim3(64), 0, st, jobs, n_jobs); break;
    case 8: hipLaunchKernelGGL(sqrd_batch_kernel<8>, dim3(items), dim3(64), 0, st, jobs, n_jobs); break;
    case 12: hipLaunchKernelGGL(sqrd_batch_kernel<12>, dim3(items), dim3(64), 0, st, jobs, n_jobs); break;
    case 16: hipLaunchKernelGGL(sqrd_batch_kernel<16>, dim3(items), dim3(64), 0, st, jobs, n_jobs); break;
    case 20: hipLaunchKernelGGL(sqrd_batch_kernel<20>, dim3(items), dim3(64), 0, st, jobs, n_jobs); break;
    case 24: hipLaunchKernelGGL(sqrd_batch_kernel<24>, dim3(items), dim3(64), 0, st, jobs, n_jobs); break;
    case 28: hipLaunchKernelGGL(sqrd_batch_kernel<28>, dim3(items), dim3(64), 0, st, jobs, n_jobs); break;
    case 32: hipLaunchKernelGGL(sqrd_batch_kernel<32>, dim3(items), dim3(64), 0, st, jobs, n_jobs); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rotate_batch(const StageJob *jobs, int n_jobs, int items, int nmax, hipStream_t st)
{
    if (nmax < 1 || nmax > kMaxN)
        return hipErrorInvalidValue;
    const int waves = (2 * nmax + 15) / 16;  // row tiles of the largest job
    hipLaunchKernelGGL(rotate_batch_kernel, dim3(items), dim3(64 * waves), 0, st, jobs, n_jobs);
    return hipGetLastError();
}



bool posvec_rec_fits_lds(int N, int K)
{
    return posvec_lds_bytes(N, K, true) <= 64 * 1024;
}

size_t posvec_lds_bytes(int N, int K, bool rec_in_lds)
{
    size_t b = (size_t)K * 3 * sizeof(uint32_t);         // A_sc, Zs[2]
    b += (size_t)((4 * K + 1) & ~1) * sizeof(uint16_t);  // Zp[2], Zk[2]
    if (rec_in_lds)
        b += (size_t)N * K * sizeof(uint32_t);
    return b;
}

hipError_t launch_sqrd(const float2 *H, const SlotDev &sd, hipStream_t st)
{
    const int mm = ((sd.M + 3) / 4) * 4;
    switch (mm) {
    case 4: return sqrd_launch_t<4>(H, sd, st);
    case 8: return sqrd_launch_t<8>(H, sd, st);
    case 12: return sqrd_launch_t<12>(H, sd, st);
    case 16: return sqrd_launch_t<16>(H, sd, st);
    case 20: return sqrd_launch_t<20>(H, sd, st);
    case 24: return sqrd_launch_t<24>(H, sd, st);
    case 28: return sqrd_launch_t<28>(H, sd, st);
    case 32: return sqrd_launch_t<32>(H, sd, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_posvec_reg(const dev::PosArgs &a, hipStream_t st);

hipError_t launch_posvec(const SlotDev &sd, hipStream_t st)
{
    PosArgs a;
    a.w = sd.wd;
    a.S = sd.S;
    a.N = sd.N;
    a.nq = 1 << sd.bits;
    a.K = sd.K;
    a.NP = sd.NP;
    a.P = sd.P;
    a.rec_g = sd.rec;
    a.rec16 = sd.K <= 256 ? sd.rec16 : nullptr;
    a.order = sd.order;
    if (sd.K <= 256)
        return launch_posvec_reg(a, st);
    const bool in_lds = posvec_rec_fits_lds(sd.N, sd.K);
    const size_t lds = posvec_lds_bytes(sd.N, sd.K, in_lds);
    if (in_lds) {
        hipLaunchKernelGGL(posvec_kernel<true>, dim3(sd.S), dim3(64), lds, st, a);
    } else {
        hipError_t e = hipFuncSetAttribute((const void *)posvec_kernel<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(posvec_kernel<false>, dim3(sd.S), dim3(64), lds, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_rotate(const SlotDev &sd, const float2 *y, int T, float2 *yt, hipStream_t st)
{
    RotArgs a;
    a.diag = sd.diag;
    a.Qd = sd.Qd;
    a.y = y;
    a.yt = yt;
    a.S = sd.S;
    a.M = sd.M;
    a.N = sd.N;
    a.T = T;
    hipLaunchKernelGGL(rotate_kernel, dim3(sd.S), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace mpnl

// ============================================================================
// Regularised (MMSE-extended) system for overloaded detection:
//     H_x = [H; sigma I_N]  ((M + N) x N per subcarrier),   y_x = [y; 0].
// ||y_x - H_x s||^2 = ||y - H s||^2 + sigma^2 ||s||^2, so the sorted QR and
// the path search of H_x give the MMSE-ordered, regularised form of the
// detector, which also exists when N > M.
// ============================================================================
namespace mpnl {
namespace dev {
namespace {

__global__ __launch_bounds__(256) void extend_kernel(const float2 *H, const float2 *y, int S, int T, int M, int N,
                                                     float sigma, float2 *Hx, float2 *yx)
{
    const int Mx = M + N;
    const size_t nH = (size_t)S * Mx * N, ny = (size_t)T * S * Mx;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nH + ny; i += (size_t)gridDim.x * blockDim.x) {
        if (i < nH) {
            const size_t s = i / ((size_t)Mx * N);
            const int r = (int)(i / N % Mx), c = (int)(i % N);
            Hx[i] = r < M ? H[(s * M + r) * N + c] : make_float2(r - M == c ? sigma : 0.f, 0.f);
        } else {
            const size_t j = i - nH;
            const size_t ts = j / Mx;  // t * S + s
            const int r = (int)(j % Mx);
            yx[j] = r < M ? y[ts * M + r] : make_float2(0.f, 0.f);
        }
    }
}

}  // namespace
}  // namespace dev

hipError_t launch_extend(const float2 *H, const float2 *y, int S, int T, int M, int N, float sigma, float2 *Hx,
                         float2 *yx, hipStream_t st)
{
    const size_t n = (size_t)S * (M + N) * N + (size_t)T * S * (M + N);
    const int grid = (int)std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(dev::extend_kernel, dim3(grid), dim3(256), 0, st, H, y, S, T, M, N, sigma, Hx, yx);
    return hipGetLastError();
}

}  // namespace mpnl
