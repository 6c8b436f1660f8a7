// Linear MMSE detection, the comparison detector of the paper (Sec. I and
// the baseline of Sec. III-B): per subcarrier
//     G = H^H H + s2 I,   x = G^-1 H^H y,   x_k <- x_k / (W H)_kk,
// with (W H)_kk = 1 - s2 (G^-1)_kk (W = G^-1 H^H), then the closest
// constellation point per user.  One wavefront per subcarrier: the Gram
// matrix and H^H y are MFMA products of the real 2x2-block forms, G is
// factored G = L L^H in LDS, L^-1 gives both the diagonal of G^-1 and the
// solve x = L^-H (L^-1 H^H y).
#include "device_common.h"

namespace mpnl {
namespace dev {
namespace {

typedef float floatx4_t __attribute__((ext_vector_type(4)));

struct MmseArgs {
    const float2 *H;  // (S, M, N)
    const float2 *y;  // (T, S, M)
    int32_t *out;     // (T, S, N)
    int S, T, M, N, bits;
    float sigma2;
    float inv_delta;  // 1 / Delta: constellation levels are odd multiples of Delta
};

constexpr int kTc = 64;  // received vectors per solve chunk (one per lane)

template <int L>
__device__ __forceinline__ int32_t slice_index(float xr, float xi, float inv_delta)
{
    // level m in 0..L-1 sits at (2m - (L-1)) Delta
    const float ui = fmaf(xr * inv_delta, 0.5f, 0.5f * (float)(L - 1));
    const float uq = fmaf(xi * inv_delta, 0.5f, 0.5f * (float)(L - 1));
    const float mi = __builtin_amdgcn_fmed3f(rintf(ui), 0.f, (float)(L - 1));
    const float mq = __builtin_amdgcn_fmed3f(rintf(uq), 0.f, (float)(L - 1));
    const int mI = mi == mi ? (int)mi : 0, mQ = mq == mq ? (int)mq : 0;  // NaN: level 0
    return (gray_code(mI) << Axis<L>::HB) | gray_code(mQ);
}

__global__ __launch_bounds__(64) void mmse_kernel(MmseArgs a)
{
    __shared__ float2 Lm[kMaxN][kMaxN + 1];   // G, then its factor L (lower)
    __shared__ float2 Vi[kMaxN][kMaxN + 1];   // L^-1 (lower)
    __shared__ float2 Z[kMaxN][kTc + 1];      // H^H y, then L^-1 H^H y
    __shared__ float gk[kMaxN];               // (W H)_kk
    const int s = blockIdx.x;
    const int lane = threadIdx.x;
    const int i16 = lane & 15, kq = lane >> 4;
    const int M = a.M, N = a.N, T = a.T, S = a.S;
    const float2 *Hs = a.H + (size_t)s * M * N;
    const int rtiles = (2 * N + 15) / 16;
    const int ksteps = (2 * M + 3) / 4;

    // Gram matrix: row 2i + part of the real form, column j
    // (part 0: Re G_ij = sum Re(h_i) Re(h_j) + Im(h_i) Im(h_j); part 1: Im G_ij)
    for (int ct = 0; ct < (N + 15) / 16; ++ct) {
        const int j = ct * 16 + i16;
        for (int rt = 0; rt < rtiles; ++rt) {
            floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
            const int row = rt * 16 + i16;
            const int d = row >> 1, part = row & 1;
            for (int ks = 0; ks < ksteps; ++ks) {
                const int k = ks * 4 + kq;
                const int m = k >> 1, cp = k & 1;
                float av = 0.f, bv = 0.f;
                if (m < M && d < N) {
                    const float2 q = Hs[(size_t)m * N + d];
                    av = part == 0 ? (cp == 0 ? q.x : q.y) : (cp == 0 ? -q.y : q.x);
                }
                if (m < M && j < N) {
                    const float2 h = Hs[(size_t)m * N + j];
                    bv = cp == 0 ? h.x : h.y;
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int orow = rt * 16 + 4 * kq + v;
                const int od = orow >> 1, op = orow & 1;
                if (od < N && j < N) {
                    if (op == 0)
                        Lm[od][j].x = acc[v];
                    else
                        Lm[od][j].y = acc[v];
                }
            }
        }
    }
    __syncthreads();
    if (lane < N)
        Lm[lane][lane] = make_float2(Lm[lane][lane].x + a.sigma2, 0.f);
    __syncthreads();

    // Cholesky G = L L^H, column by column; lane i owns row i
    for (int k = 0; k < N; ++k) {
        const float lkk = sqrtf(Lm[k][k].x);
        const float inv = 1.f / lkk;
        __syncthreads();
        if (lane > k && lane < N)
            Lm[lane][k] = make_float2(Lm[lane][k].x * inv, Lm[lane][k].y * inv);
        if (lane == k)
            Lm[k][k] = make_float2(lkk, 0.f);
        __syncthreads();
        if (lane > k && lane < N) {
            const float2 lik = Lm[lane][k];
            for (int j = k + 1; j <= lane; ++j) {
                const float2 ljk = Lm[j][k];  // G_ij -= L_ik conj(L_jk)
                float2 g = Lm[lane][j];
                g.x -= lik.x * ljk.x + lik.y * ljk.y;
                g.y -= lik.y * ljk.x - lik.x * ljk.y;
                Lm[lane][j] = g;
            }
        }
        __syncthreads();
    }

    // L^-1 by columns (lane c owns column c), then (W H)_cc
    if (lane < N) {
        const int c = lane;
        const float dcc = Lm[c][c].x;
        Vi[c][c] = make_float2(1.f / dcc, 0.f);
        float nrm = 1.f / (dcc * dcc);
        for (int i = c + 1; i < N; ++i) {
            float sr = 0.f, si = 0.f;  // sum_{j=c}^{i-1} L_ij v_j
            for (int j = c; j < i; ++j) {
                const float2 l = Lm[i][j], v = Vi[j][c];
                sr += l.x * v.x - l.y * v.y;
                si += l.x * v.y + l.y * v.x;
            }
            const float r = -1.f / Lm[i][i].x;
            const float2 vi = make_float2(sr * r, si * r);
            Vi[i][c] = vi;
            nrm += vi.x * vi.x + vi.y * vi.y;
        }
        gk[c] = 1.f - a.sigma2 * nrm;
    }
    __syncthreads();

    const int L = 1 << (a.bits / 2);
    for (int t0 = 0; t0 < T; t0 += kTc) {
        // Z = H^H y for symbols t0 .. t0 + 63 (same product as the rotation)
        for (int ct = 0; ct < kTc / 16; ++ct) {
            const int tt = t0 + ct * 16 + i16;
            for (int rt = 0; rt < rtiles; ++rt) {
                floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
                const int row = rt * 16 + i16;
                const int d = row >> 1, part = row & 1;
                for (int ks = 0; ks < ksteps; ++ks) {
                    const int k = ks * 4 + kq;
                    const int m = k >> 1, cp = k & 1;
                    float av = 0.f, bv = 0.f;
                    if (m < M && d < N) {
                        const float2 q = Hs[(size_t)m * N + d];
                        av = part == 0 ? (cp == 0 ? q.x : q.y) : (cp == 0 ? -q.y : q.x);
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
                    const int od = orow >> 1, op = orow & 1;
                    if (od < N) {
                        if (op == 0)
                            Z[od][ct * 16 + i16].x = acc[v];
                        else
                            Z[od][ct * 16 + i16].y = acc[v];
                    }
                }
            }
        }
        __syncthreads();
        // lane t: w = L^-1 z (in place, bottom row first), x = L^-H w, unbias, slice
        const int t = t0 + lane;
        if (t < T) {
            for (int i = N - 1; i >= 0; --i) {
                float sr = 0.f, si = 0.f;
                for (int j = 0; j <= i; ++j) {
                    const float2 v = Vi[i][j], z = Z[j][lane];
                    sr += v.x * z.x - v.y * z.y;
                    si += v.x * z.y + v.y * z.x;
                }
                Z[i][lane] = make_float2(sr, si);
            }
            int32_t *o = a.out + ((size_t)t * S + s) * N;
            for (int k = 0; k < N; ++k) {
                float sr = 0.f, si = 0.f;  // sum_{i >= k} conj(V_ik) w_i
                for (int i = k; i < N; ++i) {
                    const float2 v = Vi[i][k], w = Z[i][lane];
                    sr += v.x * w.x + v.y * w.y;
                    si += v.x * w.y - v.y * w.x;
                }
                const float g = 1.f / gk[k];
                const float xr = sr * g, xi = si * g;
                o[k] = L == 2 ? slice_index<2>(xr, xi, a.inv_delta)
                       : L == 4 ? slice_index<4>(xr, xi, a.inv_delta)
                                : slice_index<8>(xr, xi, a.inv_delta);
            }
        }
        __syncthreads();
    }
}

}  // namespace
}  // namespace dev

hipError_t launch_mmse(const float2 *H, const float2 *y, int S, int T, int M, int N, int bits, float sigma2,
                       int32_t *out, hipStream_t st)
{
    dev::MmseArgs a;
    a.H = H;
    a.y = y;
    a.out = out;
    a.S = S;
    a.T = T;
    a.M = M;
    a.N = N;
    a.bits = bits;
    a.sigma2 = sigma2;
    a.inv_delta = 1.f / dev::delta_of(bits);
    hipLaunchKernelGGL(dev::mmse_kernel, dim3(S), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace mpnl
