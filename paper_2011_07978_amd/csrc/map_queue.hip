// Reference mapping (paper Sec. 2.3), work-queue construction and the
// mapped-cell update.  These kernels stream the structure-of-arrays state once
// and are bound by HBM bandwidth; one thread per cell, consecutive threads on
// consecutive cells, so every species row of Y is read fully coalesced.
#include <hip/hip_runtime.h>
#include <math.h>
#include "mech_dev.hpp"
#include "wave.hpp"

namespace chem {

constexpr int MAP_BLOCK = 256;

// ---------------------------------------------------------------- mapping ---
__global__ void k_map_init(unsigned long long *ref_tmp, unsigned long long none) {
    *ref_tmp = none;
}

// Z_i = (beta_i - beta_ox)/(beta_f - beta_ox), beta_i = sum_k w_k Y_ik summed in
// ascending k with separately rounded products and sums (no contraction), so
// the candidate test Z_i < Z_tol is reproducible bit for bit.
__global__ __launch_bounds__(MAP_BLOCK) void k_map_candidates(
    int64_t ncells, int N, const double *__restrict__ Y, const double *__restrict__ w,
    double beta_f, double beta_ox, double Z_tol, uint8_t *__restrict__ flags,
    unsigned long long *ref_tmp) {
    __shared__ unsigned long long smin[MAP_BLOCK / 64];
    const int64_t i = (int64_t)blockIdx.x * MAP_BLOCK + threadIdx.x;
    unsigned long long cand_idx = ~0ull;
    if (i < ncells) {
        double beta = 0.0;
        for (int k = 0; k < N; ++k) beta = __dadd_rn(beta, __dmul_rn(w[k], Y[(int64_t)k * ncells + i]));
        const double Z = __ddiv_rn(__dsub_rn(beta, beta_ox), __dsub_rn(beta_f, beta_ox));
        const bool cand = Z < Z_tol;
        flags[i] = cand ? 1 : 0;
        if (cand) cand_idx = (unsigned long long)i;
    }
    // wave minimum, then block minimum, then one atomic per block
    unsigned long long v = cand_idx;
    for (int m = 1; m < 64; m <<= 1) {
        unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffu), m);
        unsigned hi = __shfl_xor((unsigned)(v >> 32), m);
        const unsigned long long o = ((unsigned long long)hi << 32) | lo;
        v = o < v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = smin[0];
        for (int q = 1; q < MAP_BLOCK / 64; ++q) b = smin[q] < b ? smin[q] : b;
        if (b != ~0ull) atomicMin(ref_tmp, b);
    }
}

__global__ __launch_bounds__(MAP_BLOCK) void k_map_flags(
    int64_t ncells, const double *__restrict__ T, double T_tol, int use_T,
    uint8_t *__restrict__ flags, const unsigned long long *ref_tmp, int64_t *ref_out) {
    const unsigned long long r = *ref_tmp;
    const int64_t ref = r == ~0ull ? -1 : (int64_t)r;
    const int64_t i = (int64_t)blockIdx.x * MAP_BLOCK + threadIdx.x;
    if (i == 0) *ref_out = ref;
    if (i >= ncells) return;
    if (ref < 0) { flags[i] = 0; return; }
    const bool cand = flags[i] != 0;
    uint8_t f = 0;
    if (i == ref) f = 1;
    else if (cand && i > ref && (!use_T || fabs(T[i] - T[ref]) < T_tol)) f = 2;
    flags[i] = f;
}

// ---------------------------------------------------- reference snapshot ---
// snap = (T, Y) of the reference cell before integration; delta after it.
__global__ void k_ref_snapshot(int64_t ncells, int N, const double *__restrict__ T,
                               const double *__restrict__ Y, const int64_t *ref, double *snap) {
    const int64_t r = *ref;
    if (r < 0) return;
    for (int k = threadIdx.x; k <= N; k += blockDim.x)
        snap[k] = k == 0 ? T[r] : Y[(int64_t)(k - 1) * ncells + r];
}

__global__ void k_ref_delta(int64_t ncells, int N, const double *__restrict__ Y,
                            const int64_t *ref, const double *snap, double *delta) {
    const int64_t r = *ref;
    if (r < 0) return;
    for (int k = threadIdx.x; k < N; k += blockDim.x)
        delta[k] = Y[(int64_t)k * ncells + r] - snap[1 + k];
}

// Mapped cells: Y' = Y + dY_ref and T' from h(T', Y') = h(T, Y).  The mixture
// enthalpy is a polynomial in T whose coefficients sum_k Y_k c_km / W_k are
// gathered in one pass over the species; Newton on it to |dT| < 1e-10 K.
// If the reference cell's own integration failed (ref_status != 0: step
// limit, step underflow, non-finite or bad input) its increment is not a
// solution, so mapped cells keep their state and take status 7 (counted as
// failed) instead of inheriting it.
__global__ __launch_bounds__(MAP_BLOCK) void k_map_scatter(
    int64_t ncells, int N, double *__restrict__ T, double *__restrict__ Y,
    const uint8_t *__restrict__ flags, const int64_t *ref, const double *__restrict__ delta,
    const double *__restrict__ nasa_t, const double *__restrict__ invW, uint8_t *status,
    uint32_t *cost, unsigned long long *stats, const int *ref_status) {
    const int64_t i = (int64_t)blockIdx.x * MAP_BLOCK + threadIdx.x;
    bool mapped = false, refused = false;
    const bool ref_ok = *ref_status == 0;
    if (i < ncells && *ref >= 0 && flags[i] == 2 && !ref_ok) {
        refused = true;
        if (status) status[i] = 7;
    } else if (i < ncells && *ref >= 0 && flags[i] == 2) {
        mapped = true;
        // h/R = sum_k Y_k/W_k (a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a5 T^5/5 + a6)
        double Bo[6] = {0, 0, 0, 0, 0, 0}, Bn[6] = {0, 0, 0, 0, 0, 0};
        for (int k = 0; k < N; ++k) {
            double *yp = Y + (int64_t)k * ncells + i;
            const double yo = *yp;
            const double yn = yo + delta[k];
            *yp = yn;
            const double iw = invW[k];
            const double c[6] = {nasa_t[k], nasa_t[7 * N + k], nasa_t[8 * N + k],
                                 nasa_t[9 * N + k], nasa_t[10 * N + k], nasa_t[5 * N + k]};
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                Bo[m] += yo * iw * c[m];
                Bn[m] += yn * iw * c[m];
            }
        }
        const double T0 = T[i];
        const double h0 = Bo[5] + T0 * (Bo[0] + T0 * (Bo[1] + T0 * (Bo[2] + T0 * (Bo[3] + T0 * Bo[4]))));
        double Tn = T0;
        for (int it = 0; it < 50; ++it) {
            const double F = Bn[5] + Tn * (Bn[0] + Tn * (Bn[1] + Tn * (Bn[2] + Tn * (Bn[3] + Tn * Bn[4])))) - h0;
            const double dF = Bn[0] + Tn * (2.0 * Bn[1] + Tn * (3.0 * Bn[2] + Tn * (4.0 * Bn[3] + Tn * 5.0 * Bn[4])));
            const double dT = F / dF;
            Tn -= dT;
            if (fabs(dT) < 1e-10) break;
        }
        T[i] = Tn;
        if (status) status[i] = 5;
    } else if (i < ncells && flags[i] == 3) {
        // advanced by the surrogate: its solver cost is unknown, so should the
        // gate send it back next time it is queued first (heavy-first order)
        if (status) status[i] = 6;
        if (cost) cost[i] = 0x7fffffffu;
    }
    const unsigned long long cnt = __ballot(mapped);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(&stats[5], (unsigned long long)__popcll(cnt));
    const unsigned long long nf = __ballot(refused);
    if ((threadIdx.x & 63) == 0 && nf) atomicAdd(&stats[3], (unsigned long long)__popcll(nf));
}

// ------------------------------------------------------------------ queue ---
// Heavy-first order: bucket = 31 - floor(log2(cost + 1)), so the most expensive
// cells of the previous call come first; cells flagged 2 (mapped) or 3 (surrogate) are skipped.
__device__ __forceinline__ int cost_bucket(const uint32_t *cost, int64_t i) {
    if (!cost) return NBUCKET - 1;
    uint32_t c = cost[i];
    c = c > 0x7fffffffu ? 0x7fffffffu : c;
    const int lg = 31 - __clz((int)(c + 1));
    return NBUCKET - 1 - lg;
}

__global__ void k_queue_reset(int *hist, int *cursor, int *seg_ctr, int *n_active,
                              unsigned long long *stats, int *ref_status) {
    const int t = threadIdx.x;
    if (t == 0) *ref_status = 0;
    if (t < NBUCKET) { hist[t] = 0; cursor[t] = 0; }
    if (t < NSEG) seg_ctr[t] = 0;
    if (t < 8) stats[t] = 0;
    if (t == 0) *n_active = 0;
}

__global__ __launch_bounds__(MAP_BLOCK) void k_queue_count(int64_t ncells, const uint8_t *flags,
                                                           const uint32_t *cost, int *hist) {
    __shared__ int sh[NBUCKET];
    if (threadIdx.x < NBUCKET) sh[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * MAP_BLOCK + threadIdx.x;
    if (i < ncells && !(flags && flags[i] >= 2)) atomicAdd(&sh[cost_bucket(cost, i)], 1);
    __syncthreads();
    if (threadIdx.x < NBUCKET && sh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], sh[threadIdx.x]);
}

__global__ void k_queue_scan(int *hist, int *n_active) {
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int b = 0; b < NBUCKET; ++b) {
            const int c = hist[b];
            hist[b] = acc;   // exclusive offsets
            acc += c;
        }
        *n_active = acc;
    }
}

// Each workgroup ranks its cells within their buckets in LDS, then reserves
// one contiguous range per non-empty bucket with a single global atomic, so
// the global counters see a few adds per workgroup instead of one per cell.
__global__ __launch_bounds__(MAP_BLOCK) void k_queue_scatter(int64_t ncells, const uint8_t *flags,
                                                             const uint32_t *cost,
                                                             const int *offsets, int *cursor,
                                                             int *queue) {
    __shared__ int cnt[NBUCKET], base[NBUCKET];
    if (threadIdx.x < NBUCKET) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * MAP_BLOCK + threadIdx.x;
    const bool act = i < ncells && !(flags && flags[i] >= 2);
    int b = 0, rank = 0;
    if (act) {
        b = cost_bucket(cost, i);
        rank = atomicAdd(&cnt[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < NBUCKET && cnt[threadIdx.x] > 0)
        base[threadIdx.x] = offsets[threadIdx.x] + atomicAdd(&cursor[threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (act) queue[base[b] + rank] = (int)i;
}

// --------------------------------------------------------------- launchers --
static unsigned nblk(int64_t n) { return (unsigned)((n + MAP_BLOCK - 1) / MAP_BLOCK); }

hipError_t launch_map(int64_t ncells, int N, const double *T, const double *Y, const double *w,
                      double beta_f, double beta_ox, double Z_tol, double T_tol, int use_T,
                      uint8_t *flags, unsigned long long *ref_tmp, int64_t *ref_out,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_map_init, dim3(1), dim3(1), 0, s, ref_tmp, ~0ull);
    if (ncells > 0)
        hipLaunchKernelGGL(k_map_candidates, dim3(nblk(ncells)), dim3(MAP_BLOCK), 0, s, ncells, N, Y,
                           w, beta_f, beta_ox, Z_tol, flags, ref_tmp);
    hipLaunchKernelGGL(k_map_flags, dim3(ncells > 0 ? nblk(ncells) : 1), dim3(MAP_BLOCK), 0, s,
                       ncells, T, T_tol, use_T, flags, ref_tmp, ref_out);
    return hipGetLastError();
}

hipError_t launch_queue_reset(int *hist, int *cursor, int *seg_ctr, int *n_active,
                              unsigned long long *stats, int *ref_status, hipStream_t s) {
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, hist, cursor, seg_ctr, n_active, stats,
                       ref_status);
    return hipGetLastError();
}

hipError_t launch_queue_build(int64_t ncells, const uint8_t *flags, const uint32_t *cost, int *hist,
                              int *cursor, int *n_active, int *queue, hipStream_t s) {
    if (ncells > 0)
        hipLaunchKernelGGL(k_queue_count, dim3(nblk(ncells)), dim3(MAP_BLOCK), 0, s, ncells, flags,
                           cost, hist);
    hipLaunchKernelGGL(k_queue_scan, dim3(1), dim3(64), 0, s, hist, n_active);
    if (ncells > 0)
        hipLaunchKernelGGL(k_queue_scatter, dim3(nblk(ncells)), dim3(MAP_BLOCK), 0, s, ncells, flags,
                           cost, hist, cursor, queue);
    return hipGetLastError();
}

hipError_t launch_ref_snapshot(int64_t ncells, int N, const double *T, const double *Y,
                               const int64_t *ref, double *snap, hipStream_t s) {
    hipLaunchKernelGGL(k_ref_snapshot, dim3(1), dim3(64), 0, s, ncells, N, T, Y, ref, snap);
    return hipGetLastError();
}

hipError_t launch_map_scatter(int64_t ncells, int N, double *T, double *Y, const uint8_t *flags,
                              const int64_t *ref, const double *snap, double *delta,
                              const double *nasa_t, const double *invW, uint8_t *status,
                              uint32_t *cost, unsigned long long *stats, const int *ref_status,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_ref_delta, dim3(1), dim3(64), 0, s, ncells, N, Y, ref, snap, delta);
    if (ncells > 0)
        hipLaunchKernelGGL(k_map_scatter, dim3(nblk(ncells)), dim3(MAP_BLOCK), 0, s, ncells, N, T, Y,
                           flags, ref, delta, nasa_t, invW, status, cost, stats, ref_status);
    return hipGetLastError();
}

}  // namespace chem
