// Internal interface between the host runtime and the gfx950 kernels of the
// MPNL detection library.  Not part of the public ABI (see include/mpnl.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpnl {

// Per-slot device state written by the sorted-QR and position-set kernels.
// Everything is stored in *depth order*: depth d detects row l = N-1-d of R.
struct SlotDev {
    int S, M, N, bits, K;  // K = clamped number of paths
    int NP;                // position-vector row stride in bytes (N rounded up to 4)
    float2 *Qd;            // (S, M, N)  column d = Q[:, N-1-d]
    float2 *roff;          // (S, N, N)  [d][d'] = R[N-1-d'][N-1-d] for d' > d
    float2 *rlat;          // (S, N, N)  the same entries in lattice units, times Delta / a_{d'},
                           //            transposed: [d'][d] (row d', term of depth d < d')
    uint32_t *rlat_h;      // (S, N, N, 2)  rlat entry (x, y) as half2 pairs (x, y), (y, -x) (MPNL_PREC_FP16)
    uint32_t *rlat_b;      // (S, N, N, 2)  the same as bf16x2 pairs (MPNL_PREC_BF16)
    float4 *diag;          // (S, N)     (a^2 or 1, R_ll == 0, 1/a or 1, R_ll), a = R_ll Delta
    double *wd;            // (S, N)     R_ll^2 from the float64 pivot norm
    int32_t *permd;        // (S, N)     original user detected at depth d
    uint8_t *P;            // (S, K, NP) ranks 1..|Q| per depth, padded with 1
    uint16_t *order;       // (S, K)     path run by each lane (K <= 256), else null
    uint32_t *rec;         // (S, N, K)  position-set back pointers when they do not fit in LDS
    uint16_t *rec16;       // (S, N, 256) back pointers of a 256-path set in global memory when that
                           //            saves a round of workgroups (posvec_reg_rec_global), else null
};

// Work item of the batched path search: one job (cell) of an uneven batch.
struct JobDev {
    const float2 *yt;      // (T, S, N) rotated received vectors, depth order, lattice units
    const float2 *rlat;
    const uint32_t *rq;    // packed FP16 / BF16 pairs of rlat for reduced precision, else null
    const float4 *diag;
    const int32_t *permd;
    const uint8_t *P;
    const uint16_t *order;
    int32_t *out;          // (T, S, N)
    float *bound;          // pruning record (bound_record_bytes), or null
    float *part;           // per path group best of every vector (multi_partial_bytes), or null
    int S, T, N, K, NP;
    int item_begin;        // first global work item of this job
    int bound_begin;       // first item of this job in the bound launch (ceil(S T / 64) items a job)
};

// Pruning record of a (S, T) job with N users: path 0's metric per vector,
// (T, S) floats, then its packed decisions, (T, S, (N + 3) / 4) floats.
inline size_t bound_record_bytes(int S, int T, int N)
{
    return (size_t)S * T * (1 + (N + 3) / 4) * sizeof(float);
}

// Partial records of a multi-job launch that splits each vector's K paths
// into path groups of one wavefront: (T, S, groups) records of 2 + (N + 3) / 4
// floats (metric, path, packed decisions); 0 with a single group.
inline size_t multi_partial_bytes(int S, int T, int N, int K)
{
    const int groups = (K + 63) / 64;
    return groups > 1 ? (size_t)S * T * groups * (2 + (N + 3) / 4) * sizeof(float) : 0;
}

// Kernel launchers (enqueue only; return hipError_t of the launch).
// a1; writes R both as is (roff) and in lattice units (rlat, rlat_h, rlat_b).
hipError_t launch_sqrd(const float2 *H, const SlotDev &sd, hipStream_t st);
hipError_t launch_posvec(const SlotDev &sd, hipStream_t st);
hipError_t launch_rotate(const SlotDev &sd, const float2 *y, int T, float2 *yt, hipStream_t st);
// K > 64 paths run as ceil(K / 64) one-wavefront workgroups per vector whose
// best paths meet in `part` (path_partial_bytes(); null when K <= 64).
size_t path_partial_bytes(const SlotDev &sd, int T);
hipError_t launch_path_search(const SlotDev &sd, const float2 *yt, int T, int32_t *out,
                              int precision, float *part, float *bound, hipStream_t st);
// Pruning record (path 0's metric and decisions of every vector,
// bound_record_bytes) for launch_path_search; run before it on the same
// stream (or joined to it by an event).
hipError_t launch_path_bound(const SlotDev &sd, const float2 *yt, int T, int precision, float *bound,
                             hipStream_t st);
hipError_t launch_path_search_soft(const SlotDev &sd, const float2 *yt, int T, float sigma2,
                                   float clip, float *llr, int32_t *out, hipStream_t st);
// Regularised (MMSE-extended) system of the overloaded detection:
// H_x = [H; sigma I] ((S, M + N, N)) and y_x = [y; 0] ((T, S, M + N)).
hipError_t launch_extend(const float2 *H, const float2 *y, int S, int T, int M, int N, float sigma, float2 *Hx,
                         float2 *yx, hipStream_t st);

// Linear MMSE detection of a whole slot (one wavefront per subcarrier).
hipError_t launch_mmse(const float2 *H, const float2 *y, int S, int T, int M, int N, int bits, float sigma2,
                       int32_t *out, hipStream_t st);

// Path search of many jobs with the same N, modulation and lanes per
// received vector (`threads`: n_paths rounded up to a multiple of 64, at most
// 256).  Each vector's paths run as `groups` path groups of threads / groups
// lanes (groups = 1, or threads / 64 for one-wavefront groups), `ipw` work
// items (vector, group) per workgroup (ipw * threads / groups <= 256),
// numbered path group major (gmajor = 1) or vector major.  With several
// groups every job needs JobDev::part, and a second small kernel takes the
// best group of every vector.
hipError_t launch_path_search_multi(const JobDev *jobs_dev, int n_jobs, int total_items, int N, int bits,
                                    int precision, int threads, int groups, int ipw, int gmajor,
                                    hipStream_t st);
// Pruning records (path 0 of every vector) for the jobs of a multi-job
// launch whose JobDev::bound is set: ceil(S T / 64) items per job, numbered
// from JobDev::bound_begin.  Run before launch_path_search_multi.
hipError_t launch_path_bound_multi(const JobDev *jobs_dev, int n_jobs, int bound_items, int N, int bits,
                                   int precision, hipStream_t st);

namespace dev {
struct StageJob;
}
// Batched a1 / a2 / a3 over a device table of jobs sorted by item_begin
// (items: subcarrier pairs for a1, subcarriers for a2 and a3).
hipError_t launch_sqrd_batch(const dev::StageJob *jobs, int n_jobs, int items, int mmax, hipStream_t st);
hipError_t launch_posvec_batch(const dev::StageJob *jobs, int n_jobs, int items, int E, int Nmax,
                               hipStream_t st);
hipError_t launch_rotate_batch(const dev::StageJob *jobs, int n_jobs, int items, int nmax, hipStream_t st);
size_t posvec_reg_lds_bytes(int N, int K);
// Whether a slot's 256-path position set keeps its back pointers in global
// memory (SlotDev::rec16): when, with cus compute units of lds_per_cu bytes of
// LDS, that takes fewer rounds of workgroups than holding them in LDS.
bool posvec_reg_rec_global(int S, int N, int K, int cus, size_t lds_per_cu);

size_t posvec_lds_bytes(int N, int K, bool rec_in_lds);
bool posvec_rec_fits_lds(int N, int K);
int nmax_bucket(int N);

}  // namespace mpnl
