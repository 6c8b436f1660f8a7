/*
 * FP64 CPU oracle for massively parallelisable non-linear (MPNL) uplink MIMO
 * detection (arXiv 2409.14355, Sec. II "Background", the MPNL paragraph).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the HIP library.
 *
 * Model (the paper names the detection problem of jointly processing the
 * mutually interfering streams, Sec. II, but never writes it out):
 *     y = H s + n,  H in C^{M x N}, M >= N, s in Q^N, n ~ CN(0, sigma^2 I).
 *
 * Everything is plain, slow and in double precision: std C99 complex, no SIMD,
 * no blocking, no fusion.  Where the paper is silent the reading taken is
 * stated at the function.  Floating-point contraction is disabled at build
 * time (-ffp-contract=off) so every sum below is evaluated exactly as written.
 *
 * Array layouts (row-major, interleaved complex):
 *   H   : (S, M, N)   one channel matrix per subcarrier
 *   y   : (T, S, M)   one received vector per (symbol, subcarrier)
 *   out : (T, S, N)   int32 constellation index per user, original user order
 *   P   : (K, N)      uint8 position vectors, depth order, ranks 1..|Q|
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_MAXN 32
#define ORC_MAXQ 64

/* ------------------------------------------------------------------------ */
/* Constellation.  The paper only names QPSK and MCS groups (Sec. IV); the   */
/* mapping taken is square QAM with unit average energy and a per-axis       */
/* binary-reflected Gray label: index i = (gI << b/2) | gQ, where gI / gQ    */
/* are the Gray labels of the in-phase / quadrature PAM levels               */
/* (2m - L + 1) * Delta, m = 0..L-1, Delta^2 = 3 / (2 (L^2 - 1)).            */
/* ------------------------------------------------------------------------ */

/* Level m whose Gray code m ^ (m >> 1) equals g. */
static int gray_inverse(int g)
{
    int m = 0;
    for (; g; g >>= 1)
        m ^= g;
    return m;
}

int orc_constellation(int bits, cplx *pts)
{
    if (bits != 2 && bits != 4 && bits != 6)
        return -1;
    int half = bits / 2;
    int L = 1 << half;
    double delta = sqrt(3.0 / (2.0 * (double)(L * L - 1)));
    for (int i = 0; i < (1 << bits); i++) {
        int mI = gray_inverse(i >> half);
        int mQ = gray_inverse(i & (L - 1));
        double re = (double)(2 * mI - L + 1) * delta;
        double im = (double)(2 * mQ - L + 1) * delta;
        pts[i] = CMPLX(re, im);
    }
    return 1 << bits;
}

static double abs2(cplx z) { return creal(z) * creal(z) + cimag(z) * cimag(z); }

/* Nearest constellation point to x; equal distances go to the lower index. */
static int slice(const cplx *pts, int nq, cplx x)
{
    int best = 0;
    double bd = abs2(x - pts[0]);
    for (int c = 1; c < nq; c++) {
        double d = abs2(x - pts[c]);
        if (d < bd) {
            bd = d;
            best = c;
        }
    }
    return best;
}

static double rel_gap(double a, double b)
{
    double m = fmax(fabs(a), fabs(b));
    if (m == 0.0)
        return 0.0;
    return fabs(a - b) / m;
}

/* ||y - H s||^2 for the symbol vector with indices idx (original order). */
double orc_residual_norm2(const cplx *H, const cplx *y, int M, int N, int bits,
                          const int32_t *idx)
{
    cplx pts[ORC_MAXQ];
    orc_constellation(bits, pts);
    double acc = 0.0;
    for (int m = 0; m < M; m++) {
        cplx r = y[m];
        for (int n = 0; n < N; n++)
            r -= H[m * N + n] * pts[idx[n]];
        acc += abs2(r);
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* O1: exhaustive maximum-likelihood detection, the joint non-linear         */
/* detector of Sec. II: argmin over all s in Q^N of ||y - H s||^2.           */
/* Vectors are visited in lexicographic index order (user 0 most            */
/* significant) and only a strictly smaller metric replaces the incumbent,  */
/* so ties go to the lexicographically smallest index vector.                */
/* ------------------------------------------------------------------------ */
int orc_ml_vector(const cplx *H, const cplx *y, int M, int N, int bits,
                  int32_t *idx_out, double *metric_out)
{
    cplx pts[ORC_MAXQ];
    int nq = orc_constellation(bits, pts);
    if (nq < 0 || N < 1 || N > ORC_MAXN)
        return -1;
    int32_t cur[ORC_MAXN];
    memset(cur, 0, sizeof(cur));
    double best = INFINITY;
    for (;;) {
        double m2 = orc_residual_norm2(H, y, M, N, bits, cur);
        if (m2 < best) {
            best = m2;
            memcpy(idx_out, cur, sizeof(int32_t) * N);
        }
        int u = N - 1; /* odometer, last user least significant */
        while (u >= 0 && cur[u] == nq - 1) {
            cur[u] = 0;
            u--;
        }
        if (u < 0)
            break;
        cur[u]++;
    }
    if (metric_out)
        *metric_out = best;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dense complex linear solve A X = B (A n x n, B n x m, both overwritten),  */
/* Gaussian elimination with partial pivoting.  Used by ZF, MMSE and         */
/* ZF-SIC only.                                                              */
/* ------------------------------------------------------------------------ */
static int solve(cplx *A, cplx *B, int n, int m)
{
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (cabs(A[r * n + c]) > cabs(A[piv * n + c]))
                piv = r;
        if (cabs(A[piv * n + c]) == 0.0)
            return -1;
        if (piv != c) {
            for (int k = 0; k < n; k++) {
                cplx t = A[c * n + k];
                A[c * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            for (int k = 0; k < m; k++) {
                cplx t = B[c * m + k];
                B[c * m + k] = B[piv * m + k];
                B[piv * m + k] = t;
            }
        }
        for (int r = 0; r < n; r++) {
            if (r == c)
                continue;
            cplx f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; k++)
                A[r * n + k] -= f * A[c * n + k];
            for (int k = 0; k < m; k++)
                B[r * m + k] -= f * B[c * m + k];
        }
    }
    for (int r = 0; r < n; r++) {
        cplx d = A[r * n + r];
        for (int k = 0; k < m; k++)
            B[r * m + k] /= d;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O2 / O3: linear zero-forcing and MMSE, the linear detectors the paper     */
/* compares against (Sec. I; MMSE is the baseline of Sec. III-B).            */
/* ZF:   x = (H^H H)^{-1} H^H y, slice each stream.                          */
/* MMSE: W = (H^H H + sigma^2 I)^{-1} H^H, x = W y; the estimate is unbiased */
/*       before slicing by dividing x_k by (W H)_kk.                         */
/* ------------------------------------------------------------------------ */
static int linear_estimate(const cplx *H, const cplx *y, int M, int N, double sigma2,
                           int unbiased, cplx *x_out)
{
    cplx *G = malloc(sizeof(cplx) * N * N);
    cplx *B = malloc(sizeof(cplx) * N * (M + 1));
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            cplx a = 0;
            for (int m = 0; m < M; m++)
                a += conj(H[m * N + i]) * H[m * N + j];
            G[i * N + j] = a + ((i == j) ? sigma2 : 0.0);
        }
    /* right-hand sides: columns 0..M-1 = H^H (gives W), column M = H^H y */
    for (int i = 0; i < N; i++) {
        cplx hy = 0;
        for (int m = 0; m < M; m++) {
            B[i * (M + 1) + m] = conj(H[m * N + i]);
            hy += conj(H[m * N + i]) * y[m];
        }
        B[i * (M + 1) + M] = hy;
    }
    int rc = solve(G, B, N, M + 1);
    if (rc == 0) {
        for (int k = 0; k < N; k++) {
            cplx x = B[k * (M + 1) + M];
            if (unbiased) {
                cplx g = 0; /* (W H)_kk */
                for (int m = 0; m < M; m++)
                    g += B[k * (M + 1) + m] * H[m * N + k];
                x /= g;
            }
            x_out[k] = x;
        }
    }
    free(G);
    free(B);
    return rc;
}

static int linear_detect(const cplx *H, const cplx *y, int M, int N, int bits,
                         double sigma2, int unbiased, int32_t *idx_out)
{
    cplx pts[ORC_MAXQ];
    int nq = orc_constellation(bits, pts);
    if (nq < 0 || N < 1 || N > ORC_MAXN)
        return -1;
    cplx x[ORC_MAXN];
    int rc = linear_estimate(H, y, M, N, sigma2, unbiased, x);
    if (rc == 0)
        for (int k = 0; k < N; k++)
            idx_out[k] = slice(pts, nq, x[k]);
    return rc;
}

/* The unbiased MMSE estimate itself (before slicing), for decision margins. */
int orc_mmse_estimate(const cplx *H, const cplx *y, int M, int N, double sigma2,
                      cplx *x_out)
{
    if (N < 1 || N > ORC_MAXN)
        return -1;
    return linear_estimate(H, y, M, N, sigma2, 1, x_out);
}

int orc_zf_vector(const cplx *H, const cplx *y, int M, int N, int bits,
                  int32_t *idx_out)
{
    return linear_detect(H, y, M, N, bits, 0.0, 0, idx_out);
}

int orc_mmse_vector(const cplx *H, const cplx *y, int M, int N, int bits,
                    double sigma2, int32_t *idx_out)
{
    return linear_detect(H, y, M, N, bits, sigma2, 1, idx_out);
}

/* ------------------------------------------------------------------------ */
/* O4: sorted QR decomposition.  The paper's pre-processing looks at the    */
/* channel alone, ahead of any data (Sec. II); the reading                  */
/* taken is the sorted QR of Wuebben et al. (2001): modified Gram-Schmidt   */
/* where step i takes, among the columns not yet placed, the one with the   */
/* smallest residual norm (equal norms: smaller original column index).     */
/* The chosen column is re-orthogonalised once against q_0..q_{i-1} before  */
/* normalising, which keeps Q orthonormal to working precision.             */
/* Outputs: perm (H[:, perm] = Q R), Q (M x N), R (N x N, upper, real       */
/* non-negative diagonal).  pivot_margin = smallest relative gap between    */
/* the chosen residual norm^2 and the next smallest one, over all steps.    */
/* ------------------------------------------------------------------------ */
int orc_sqrd(const cplx *H, int M, int N, cplx *Q, cplx *R, int32_t *perm,
             double *pivot_margin)
{
    if (N < 1 || N > ORC_MAXN || M < N)
        return -1;
    memcpy(Q, H, sizeof(cplx) * M * N);
    memset(R, 0, sizeof(cplx) * N * N);
    for (int i = 0; i < N; i++)
        perm[i] = i;
    double margin = INFINITY;

    for (int i = 0; i < N; i++) {
        double nrm[ORC_MAXN];
        for (int k = i; k < N; k++) {
            double a = 0.0;
            for (int m = 0; m < M; m++)
                a += abs2(Q[m * N + k]);
            nrm[k] = a;
        }
        int kmin = i;
        for (int k = i + 1; k < N; k++)
            if (nrm[k] < nrm[kmin] || (nrm[k] == nrm[kmin] && perm[k] < perm[kmin]))
                kmin = k;
        for (int k = i; k < N; k++)
            if (k != kmin) {
                double g = rel_gap(nrm[kmin], nrm[k]);
                if (g < margin)
                    margin = g;
            }
        if (kmin != i) {
            for (int m = 0; m < M; m++) {
                cplx t = Q[m * N + i];
                Q[m * N + i] = Q[m * N + kmin];
                Q[m * N + kmin] = t;
            }
            for (int r = 0; r < i; r++) {
                cplx t = R[r * N + i];
                R[r * N + i] = R[r * N + kmin];
                R[r * N + kmin] = t;
            }
            int t = perm[i];
            perm[i] = perm[kmin];
            perm[kmin] = t;
        }
        /* re-orthogonalisation pass of the chosen column */
        for (int j = 0; j < i; j++) {
            cplx c = 0;
            for (int m = 0; m < M; m++)
                c += conj(Q[m * N + j]) * Q[m * N + i];
            for (int m = 0; m < M; m++)
                Q[m * N + i] -= c * Q[m * N + j];
            R[j * N + i] += c;
        }
        double rii = 0.0;
        for (int m = 0; m < M; m++)
            rii += abs2(Q[m * N + i]);
        rii = sqrt(rii);
        R[i * N + i] = rii;
        if (rii > 0.0)
            for (int m = 0; m < M; m++)
                Q[m * N + i] /= rii;
        /* deflate the remaining columns */
        for (int k = i + 1; k < N; k++) {
            cplx c = 0;
            for (int m = 0; m < M; m++)
                c += conj(Q[m * N + i]) * Q[m * N + k];
            R[i * N + k] = c;
            for (int m = 0; m < M; m++)
                Q[m * N + k] -= c * Q[m * N + i];
        }
    }
    if (pivot_margin)
        *pivot_margin = margin;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O5: the set of position vectors.  The paper fixes where the best        */
/* candidate solutions lie relative to one another from the channel alone, */
/* before transmission (Sec. II).  Reading taken: depth d detects row       */
/* l = N-1-d of R; a position vector p (p_d in 1..|Q|) asks for the p_d-th  */
/* closest symbol at depth d; its cost is                                   */
/*      score(p) = sum_d c_d (p_d - 1),   c_d = rint(2^20 w_d / max_e w_e),  */
/*      w_d = R_{l,l}^2,                                                    */
/* integer depth costs: each weight relative to the largest, in units of   */
/* 2^-20, rounded to the nearest integer (ties to even); a weight that is  */
/* not a number, or a largest weight that is not positive and finite,      */
/* gives cost 0.  Sums of such integers are exact, so ties are exact ties. */
/* The set is the first K = min(N_p, |Q|^N) vectors in ascending order of  */
/* the key (C_N, C_{N-1}, ..., C_1, p_0, ..., p_{N-1}), C_j = the cost of  */
/* the prefix of the first j depths (C_N = score): equal scores go by the   */
/* cheaper longest prefix, then the next, and the same costs throughout by  */
/* p lexicographically.                                                     */
/*                                                                          */
/* Best-first search: pop the smallest vector, emit it, push its canonical  */
/* children p + e_j for every j >= last(p) with p_j < |Q|, where last(p) is */
/* the last depth with p_d > 1 (0 for the all-ones vector).  Every vector   */
/* has exactly one parent (undo the increment at its last depth > 1) and a  */
/* child never precedes its parent, so the pops come out in order.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    double score;
    uint8_t p[ORC_MAXN];
} pv_entry;

#define ORC_COST_BITS 20

/* c_d from w_d (integers held in doubles, exact). */
static void depth_costs(const double *w_depth, int N, double *c)
{
    double wmax = 0.0;
    for (int d = 0; d < N; d++)
        if (w_depth[d] > wmax)
            wmax = w_depth[d];
    const double one = (double)(1 << ORC_COST_BITS);
    for (int d = 0; d < N; d++) {
        const double x = (w_depth[d] / wmax) * one;
        c[d] = (wmax > 0.0 && wmax <= DBL_MAX && x >= 0.0 && x <= one) ? rint(x) : 0.0;
    }
}

static double pv_score(const double *c, const uint8_t *p, int N)
{
    double s = 0.0;
    for (int d = 0; d < N; d++)
        s += c[d] * (double)(p[d] - 1);
    return s;
}

static int pv_before(const pv_entry *a, const pv_entry *b, int N, const double *c)
{
    if (a->score != b->score)
        return a->score < b->score;
    /* equal scores: prefix costs C_{N-1} .. C_1 (exact integer arithmetic) */
    double pa = a->score, pb = b->score;
    for (int d = N - 1; d >= 1; d--) {
        pa -= c[d] * (double)(a->p[d] - 1);
        pb -= c[d] * (double)(b->p[d] - 1);
        if (pa != pb)
            return pa < pb;
    }
    return memcmp(a->p, b->p, (size_t)N) < 0;
}

static void heap_push(pv_entry *h, int *n, const pv_entry *e, int N, const double *c)
{
    int i = (*n)++;
    h[i] = *e;
    while (i > 0) {
        int parent = (i - 1) / 2;
        if (!pv_before(&h[i], &h[parent], N, c))
            break;
        pv_entry t = h[i];
        h[i] = h[parent];
        h[parent] = t;
        i = parent;
    }
}

static pv_entry heap_pop(pv_entry *h, int *n, int N, const double *c)
{
    pv_entry top = h[0];
    h[0] = h[--(*n)];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < *n && pv_before(&h[l], &h[m], N, c))
            m = l;
        if (r < *n && pv_before(&h[r], &h[m], N, c))
            m = r;
        if (m == i)
            break;
        pv_entry t = h[i];
        h[i] = h[m];
        h[m] = t;
        i = m;
    }
    return top;
}

/* |Q|^N, saturated at 2^30. */
long orc_num_vectors(int nq, int N)
{
    long v = 1;
    for (int i = 0; i < N; i++) {
        v *= nq;
        if (v > (1L << 30))
            return 1L << 30;
    }
    return v;
}

/* Returns K (number of vectors written); boundary_margin = relative gap   */
/* between the scores at ranks K and K+1 (infinite when K = |Q|^N).        */
int orc_position_set(const double *w_depth, int N, int nq, int n_paths,
                     uint8_t *P_out, double *score_out, double *boundary_margin)
{
    if (N < 1 || N > ORC_MAXN || n_paths < 1)
        return -1;
    long total = orc_num_vectors(nq, N);
    int K = (long)n_paths < total ? n_paths : (int)total;
    long cap = (long)(K + 1) * N + 1;
    pv_entry *h = malloc(sizeof(pv_entry) * cap);
    double c[ORC_MAXN];
    depth_costs(w_depth, N, c);
    int n = 0;
    pv_entry root;
    memset(&root, 0, sizeof(root));
    for (int d = 0; d < N; d++)
        root.p[d] = 1;
    root.score = pv_score(c, root.p, N);
    heap_push(h, &n, &root, N, c);
    double last_score = 0.0;
    for (int k = 0; k <= K && n > 0; k++) {
        pv_entry e = heap_pop(h, &n, N, c);
        if (k == K) {
            if (boundary_margin)
                *boundary_margin = rel_gap(last_score, e.score);
            break;
        }
        memcpy(P_out + (long)k * N, e.p, (size_t)N);
        if (score_out)
            score_out[k] = e.score;
        last_score = e.score;
        int last = 0;
        for (int d = 0; d < N; d++)
            if (e.p[d] > 1)
                last = d;
        for (int j = last; j < N; j++)
            if (e.p[j] < nq) {
                pv_entry ch = e;
                ch.p[j]++;
                ch.score = pv_score(c, ch.p, N);
                heap_push(h, &n, &ch, N, c);
            }
    }
    if (K == total && boundary_margin)
        *boundary_margin = INFINITY;
    free(h);
    return K;
}

/* Brute force over all |Q|^N vectors (tiny sizes only): score every one,  */
/* sort by the key above, keep the first K.                                 */
static int g_sort_n;
static const double *g_sort_c;
static int pv_cmp(const void *a, const void *b)
{
    const pv_entry *x = a, *y = b;
    if (pv_before(x, y, g_sort_n, g_sort_c))
        return -1;
    if (pv_before(y, x, g_sort_n, g_sort_c))
        return 1;
    return 0;
}

int orc_position_set_brute(const double *w_depth, int N, int nq, int n_paths,
                           uint8_t *P_out, double *score_out)
{
    long total = orc_num_vectors(nq, N);
    if (total > (1L << 22) || n_paths < 1)
        return -1;
    pv_entry *all = malloc(sizeof(pv_entry) * total);
    double c[ORC_MAXN];
    depth_costs(w_depth, N, c);
    uint8_t cur[ORC_MAXN];
    for (int d = 0; d < N; d++)
        cur[d] = 1;
    for (long v = 0; v < total; v++) {
        memset(&all[v], 0, sizeof(pv_entry));
        memcpy(all[v].p, cur, (size_t)N);
        all[v].score = pv_score(c, cur, N);
        int d = N - 1;
        while (d >= 0 && cur[d] == nq) {
            cur[d] = 1;
            d--;
        }
        if (d >= 0)
            cur[d]++;
    }
    g_sort_n = N;
    g_sort_c = c;
    qsort(all, (size_t)total, sizeof(pv_entry), pv_cmp);
    int K = (long)n_paths < total ? n_paths : (int)total;
    for (int k = 0; k < K; k++) {
        memcpy(P_out + (long)k * N, all[k].p, (size_t)N);
        if (score_out)
            score_out[k] = all[k].score;
    }
    free(all);
    return K;
}

/* ------------------------------------------------------------------------ */
/* O6: MPNL detection of one received vector (Sec. II: the N_p most         */
/* promising solutions are formed and processed in parallel, the best one  */
/* solves the detection problem).                                          */
/*   1. rotate:  yt = Q^H y.                                               */
/*   2. for every position vector r (in set order) run one successive-     */
/*      interference-cancellation descent: at depth d (row l = N-1-d)      */
/*        b = yt_l - sum_{j = l+1}^{N-1} R_{l,j} s_j                        */
/*      rank every constellation point c by |b - R_{l,l} c|^2 (equal       */
/*      distances: lower index), take the P[r][d]-th, and add its distance */
/*      to the path metric.                                                */
/*   3. keep the path with the smallest metric (equal: lowest r) and write */
/*      its symbols back in original user order, out[perm[l]] = idx_l.     */
/* diag (optional, 4 doubles): [0] unused here (pivot, filled by caller),  */
/* [1] unused here (set boundary), [2] k-th-best margin: the smallest      */
/* relative gap between the chosen rank's distance and its neighbouring    */
/* ranks, over the (path, depth) pairs where a different choice could      */
/* still change the result, [3] relative gap between the best and          */
/* second-best path metric, [4] (if diag is given) the k-th-best margin   */
/* over every (path, depth) pair, for outputs that use every path's metric */
/* (soft output).                                                           */
/* A k-th-best near-tie at depth d of path r can only matter when the      */
/* partial metric of r through d is not already above the final minimum:   */
/* the alternative path shares that partial metric (up to the tiny gap)   */
/* and metrics only grow, so otherwise it can never win (KTH_REACH pads    */
/* the comparison far beyond float32 rounding).  Depths with R_ll = 0 are */
/* left out as well: every point ties there exactly and both the oracle    */
/* and any implementation of the reading take them in index order.         */
/* metrics_out (optional, K doubles): every path's metric.                 */
/* ------------------------------------------------------------------------ */
#define KTH_REACH 1e-3
int orc_mpnl_vector(const cplx *Q, const cplx *R, const int32_t *perm,
                    const uint8_t *P, int K, const cplx *y, int M, int N,
                    int bits, int32_t *idx_out, double *best_metric,
                    double *diag, double *metrics_out, int32_t *paths_out)
{
    cplx pts[ORC_MAXQ];
    int nq = orc_constellation(bits, pts);
    if (nq < 0 || N < 1 || N > ORC_MAXN || K < 1)
        return -1;
    cplx yt[ORC_MAXN];
    for (int l = 0; l < N; l++) {
        cplx a = 0;
        for (int m = 0; m < M; m++)
            a += conj(Q[m * N + l]) * y[m];
        yt[l] = a;
    }
    double best = INFINITY, second = INFINITY, kth_margin = INFINITY;
    int32_t best_idx[ORC_MAXN];
    /* per (path, depth): the k-th-best gap and the partial metric through d */
    double *gap = malloc(sizeof(double) * (size_t)K * N);
    double *partial = malloc(sizeof(double) * (size_t)K * N);
    if (!gap || !partial) {
        free(gap);
        free(partial);
        return -1;
    }
    for (int r = 0; r < K; r++) {
        cplx s[ORC_MAXN];
        int32_t sidx[ORC_MAXN];
        double metric = 0.0;
        for (int d = 0; d < N; d++) {
            int l = N - 1 - d;
            cplx b = yt[l];
            for (int j = l + 1; j < N; j++)
                b -= R[l * N + j] * s[j];
            double dist[ORC_MAXQ];
            int order[ORC_MAXQ];
            for (int c = 0; c < nq; c++) {
                dist[c] = abs2(b - R[l * N + l] * pts[c]);
                order[c] = c;
            }
            /* insertion sort by (distance, index) */
            for (int a = 1; a < nq; a++) {
                int v = order[a], z = a;
                while (z > 0 && (dist[order[z - 1]] > dist[v] ||
                                 (dist[order[z - 1]] == dist[v] && order[z - 1] > v))) {
                    order[z] = order[z - 1];
                    z--;
                }
                order[z] = v;
            }
            int k = P[(long)r * N + d] - 1;
            int c = order[k];
            double gmin = INFINITY;
            if (R[l * N + l] != 0) {
                if (k > 0)
                    gmin = fmin(gmin, rel_gap(dist[order[k - 1]], dist[c]));
                if (k + 1 < nq)
                    gmin = fmin(gmin, rel_gap(dist[c], dist[order[k + 1]]));
            }
            s[l] = pts[c];
            sidx[l] = c;
            metric += dist[c];
            gap[(long)r * N + d] = gmin;
            partial[(long)r * N + d] = metric;
        }
        if (metrics_out)
            metrics_out[r] = metric;
        if (paths_out)
            for (int l = 0; l < N; l++)
                paths_out[(long)r * N + perm[l]] = sidx[l];
        if (metric < best) {
            second = best;
            best = metric;
            memcpy(best_idx, sidx, sizeof(int32_t) * N);
        } else if (metric < second) {
            second = metric;
        }
    }
    double kth_all = INFINITY;
    for (long i = 0; i < (long)K * N; i++) {
        if (partial[i] <= best * (1.0 + KTH_REACH) && gap[i] < kth_margin)
            kth_margin = gap[i];
        if (gap[i] < kth_all)
            kth_all = gap[i];
    }
    free(gap);
    free(partial);
    for (int l = 0; l < N; l++)
        idx_out[perm[l]] = best_idx[l];
    if (best_metric)
        *best_metric = best;
    if (diag) {
        diag[2] = kth_margin;
        diag[3] = (K > 1) ? rel_gap(best, second) : INFINITY;
        diag[4] = kth_all;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O7: ordered zero-forcing successive interference cancellation with the  */
/* detection order perm (last column first).  At step k the stream perm[k] */
/* is nulled by row k of the pseudo-inverse of H[:, perm[0..k]], solved    */
/* from the normal equations, applied to y minus the already-detected      */
/* streams; the estimate is sliced and cancelled.                          */
/* ------------------------------------------------------------------------ */
int orc_zfsic_vector(const cplx *H, const cplx *y, int M, int N, int bits,
                     const int32_t *perm, int32_t *idx_out)
{
    cplx pts[ORC_MAXQ];
    int nq = orc_constellation(bits, pts);
    if (nq < 0 || N < 1 || N > ORC_MAXN)
        return -1;
    cplx *r = malloc(sizeof(cplx) * M);
    memcpy(r, y, sizeof(cplx) * M);
    for (int k = N - 1; k >= 0; k--) {
        int n = k + 1;
        cplx *G = malloc(sizeof(cplx) * n * n);
        cplx *B = malloc(sizeof(cplx) * n);
        for (int i = 0; i < n; i++) {
            for (int j = 0; j < n; j++) {
                cplx a = 0;
                for (int m = 0; m < M; m++)
                    a += conj(H[m * N + perm[i]]) * H[m * N + perm[j]];
                G[i * n + j] = a;
            }
            cplx a = 0;
            for (int m = 0; m < M; m++)
                a += conj(H[m * N + perm[i]]) * r[m];
            B[i] = a;
        }
        int rc = solve(G, B, n, 1);
        cplx x = B[k];
        free(G);
        free(B);
        if (rc != 0) {
            free(r);
            return -1;
        }
        int c = slice(pts, nq, x);
        idx_out[perm[k]] = c;
        for (int m = 0; m < M; m++)
            r[m] -= H[m * N + perm[k]] * pts[c];
    }
    free(r);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O1b: exact maximum-likelihood detection by sphere decoding, the classic  */
/* non-linear detector the paper contrasts MPNL with (Sec. I): a depth-     */
/* first tree search with Schnorr-Euchner enumeration (C. P. Schnorr and   */
/* M. Euchner, Math. Programming 66, 1994; for MIMO detection see E. Agrell */
/* et al., IEEE Trans. IT 48(8), 2002).  It reaches the ML result where     */
/* enumerating Q^N is impossible (16 users, 16-QAM).                        */
/* On the QR form of the channel (Q, R, perm from O4),                      */
/*   ||y - H s||^2 = sum_l |yt_l - sum_{j>=l} R_{l,j} s'_j|^2 + const,      */
/* yt = Q^H y, s' = s in the column order perm, the search assigns levels   */
/* l = N-1 down to 0.  At a node the points of level l are taken in order  */
/* of increasing |b - R_{l,l} c|^2, b = yt_l - sum_{j>l} R_{l,j} s'_j      */
/* (equal distances: lower index), and a child is entered only while the   */
/* partial metric stays below the best complete metric found so far; that */
/* radius starts infinite, so the first leaf reached is the ordered        */
/* ZF-SIC decision.  Since partial metrics only grow along a branch and    */
/* the points of a node are visited in increasing distance, the first     */
/* point that fails the test ends the node.  Every vector with a metric    */
/* below the final radius is thus visited: the result minimises            */
/* ||y - H s||^2 (among equal metrics, which have probability zero with    */
/* continuous noise, the first leaf found is kept).  max_nodes bounds the  */
/* work (visited nodes); -2 when it is exceeded.  metric_out: the QR-form  */
/* metric sum_l |...|^2 of the result (||y - H s||^2 minus ||y||^2 -       */
/* ||yt||^2).                                                              */
/* ------------------------------------------------------------------------ */
int orc_sphere_vector(const cplx *Q, const cplx *R, const int32_t *perm,
                      const cplx *y, int M, int N, int bits, long max_nodes,
                      int32_t *idx_out, double *metric_out, long *nodes_out)
{
    cplx pts[ORC_MAXQ];
    int nq = orc_constellation(bits, pts);
    if (nq < 0 || N < 1 || N > ORC_MAXN)
        return -1;
    cplx yt[ORC_MAXN];
    for (int l = 0; l < N; l++) {
        cplx a = 0;
        for (int m = 0; m < M; m++)
            a += conj(Q[m * N + l]) * y[m];
        yt[l] = a;
    }
    int order[ORC_MAXN][ORC_MAXQ];
    double dist[ORC_MAXN][ORC_MAXQ];
    int next[ORC_MAXN];        /* next position in order[l] to try        */
    double above[ORC_MAXN + 1]; /* partial metric of the levels above l    */
    cplx s[ORC_MAXN];
    int32_t sidx[ORC_MAXN], best_idx[ORC_MAXN];
    double best = INFINITY;
    long nodes = 0;
    int l = N - 1;
    above[N] = 0.0;
    int enter = 1;
    for (;;) {
        if (enter) {
            /* distances of every point at level l given the levels above */
            cplx b = yt[l];
            for (int j = l + 1; j < N; j++)
                b -= R[l * N + j] * s[j];
            for (int c = 0; c < nq; c++) {
                dist[l][c] = abs2(b - R[l * N + l] * pts[c]);
                order[l][c] = c;
            }
            for (int a = 1; a < nq; a++) { /* insertion sort by (distance, index) */
                int v = order[l][a], z = a;
                while (z > 0 && (dist[l][order[l][z - 1]] > dist[l][v] ||
                                 (dist[l][order[l][z - 1]] == dist[l][v] && order[l][z - 1] > v))) {
                    order[l][z] = order[l][z - 1];
                    z--;
                }
                order[l][z] = v;
            }
            next[l] = 0;
            enter = 0;
        }
        int moved = 0;
        if (next[l] < nq) {
            int c = order[l][next[l]];
            double m = above[l + 1] + dist[l][c];
            if (m < best) {
                next[l]++;
                s[l] = pts[c];
                sidx[l] = c;
                if (++nodes > max_nodes)
                    return -2;
                if (l == 0) {
                    best = m;
                    memcpy(best_idx, sidx, sizeof(int32_t) * N);
                } else {
                    above[l] = m;
                    l--;
                    enter = 1;
                }
                moved = 1;
            }
        }
        if (!moved) { /* node exhausted or pruned: back to the level above */
            l++;
            if (l == N)
                break;
        }
    }
    for (int k = 0; k < N; k++)
        idx_out[perm[k]] = best_idx[k];
    if (metric_out)
        *metric_out = best;
    if (nodes_out)
        *nodes_out = nodes;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Max-log soft output from the MPNL path list (the paper measures packet  */
/* errors after LDPC decoding, Sec. III-B, which consumes per-bit soft     */
/* values).  For bit b of user u:                                          */
/*    LLR = ( min_{paths with bit = 1} metric - min_{paths with bit = 0}    */
/*            metric ) / sigma^2,                                           */
/* positive favouring bit 0; when one hypothesis has no path the value is  */
/* +clip or -clip.  Bit b counts from the most significant bit of the     */
/* constellation index.                                                    */
/* ------------------------------------------------------------------------ */
int orc_llr_from_paths(const double *metrics, const int32_t *paths, int K,
                       int N, int bits, double sigma2, double clip,
                       double *llr_out)
{
    for (int u = 0; u < N; u++)
        for (int b = 0; b < bits; b++) {
            double m0 = INFINITY, m1 = INFINITY;
            for (int r = 0; r < K; r++) {
                int bit = (paths[(long)r * N + u] >> (bits - 1 - b)) & 1;
                if (bit)
                    m1 = fmin(m1, metrics[r]);
                else
                    m0 = fmin(m0, metrics[r]);
            }
            double v;
            if (isinf(m1))
                v = clip;
            else if (isinf(m0))
                v = -clip;
            else {
                v = (m1 - m0) / sigma2;
                if (v > clip)
                    v = clip;
                if (v < -clip)
                    v = -clip;
            }
            llr_out[u * bits + b] = v;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Whole-slot drivers.  Subcarriers are independent; the loop over them is */
/* the only place OpenMP appears (it changes no arithmetic).               */
/* method: 0 = MPNL, 1 = ML, 2 = ZF, 3 = MMSE, 4 = ZF-SIC (SQRD order).     */
/* diag (optional): (T, S, 4) doubles [pivot, boundary, kth, metric].      */
/* ------------------------------------------------------------------------ */
/* work bound of one sphere-decoded vector in the slot driver */
#define ORC_SPHERE_MAX_NODES 200000000L

int orc_detect_slot(int method, const cplx *H, const cplx *y, int S, int T,
                    int M, int N, int bits, int n_paths, double sigma2,
                    int32_t *out, double *diag, int nthreads)
{
    if (S < 0 || T < 0 || M < 1 || N < 1 || N > ORC_MAXN || M < N)
        return -1;
    int nq = 1 << bits;
    int failed = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int s = 0; s < S; s++) {
        const cplx *Hs = H + (long)s * M * N;
        cplx *Q = malloc(sizeof(cplx) * M * N);
        cplx *R = malloc(sizeof(cplx) * N * N);
        int32_t perm[ORC_MAXN];
        double pivot_margin = INFINITY, boundary = INFINITY;
        uint8_t *P = NULL;
        int K = 0;
        if (method == 0 || method == 4 || method == 5) {
            orc_sqrd(Hs, M, N, Q, R, perm, &pivot_margin);
        }
        if (method == 0) {
            double w[ORC_MAXN];
            for (int d = 0; d < N; d++) {
                int l = N - 1 - d;
                w[d] = creal(R[l * N + l]) * creal(R[l * N + l]);
            }
            long total = orc_num_vectors(nq, N);
            int Kmax = (long)n_paths < total ? n_paths : (int)total;
            P = malloc((size_t)Kmax * N);
            K = orc_position_set(w, N, nq, n_paths, P, NULL, &boundary);
        }
        for (int t = 0; t < T; t++) {
            const cplx *yv = y + ((long)t * S + s) * M;
            int32_t *o = out + ((long)t * S + s) * N;
            double dv[5] = {pivot_margin, boundary, INFINITY, INFINITY, INFINITY};
            int rc = 0;
            switch (method) {
            case 0:
                rc = orc_mpnl_vector(Q, R, perm, P, K, yv, M, N, bits, o, NULL, dv, NULL, NULL);
                break;
            case 1:
                rc = orc_ml_vector(Hs, yv, M, N, bits, o, NULL);
                break;
            case 2:
                rc = orc_zf_vector(Hs, yv, M, N, bits, o);
                break;
            case 3:
                rc = orc_mmse_vector(Hs, yv, M, N, bits, sigma2, o);
                break;
            case 4:
                rc = orc_zfsic_vector(Hs, yv, M, N, bits, perm, o);
                break;
            case 5:
                rc = orc_sphere_vector(Q, R, perm, yv, M, N, bits, ORC_SPHERE_MAX_NODES, o, NULL, NULL);
                break;
            default:
                rc = -1;
            }
            if (rc != 0) {
#pragma omp atomic write
                failed = 1;
            }
            if (diag)
                memcpy(diag + ((long)t * S + s) * 4, dv, 4 * sizeof(double));
        }
        free(P);
        free(Q);
        free(R);
    }
    return failed ? -1 : 0;
}
