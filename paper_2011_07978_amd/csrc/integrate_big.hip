// Per-cell stiff chemistry integration for large mechanisms (64 < n <= ~138
// unknowns), FP64, gfx950.
//
// A workgroup of four wavefronts owns one cell; thread i holds unknown i of
// y = (T, Y_1..Y_N).  The iteration matrix M = I/(gamma h) - J (n x n) lives
// in LDS (up to ~150 KB, so one cell per CU); the Jacobian is kept for reuse
// after a rejected step in a global workspace that exists only for the
// workgroups in flight (one slot per persistent workgroup), not per cell.
//   - right-hand side and analytic Jacobian: the formulas of the wavefront
//     kernel, reaction pass over 256 threads with LDS float atomics issued one
//     wavefront at a time, block reductions combined in a fixed order, so the
//     result does not depend on scheduling;
//   - LU with partial pivoting, right-looking and blocked by 16 columns: each
//     panel is factored column by column (rows swapped in place), the block
//     row of U by a forward substitution, and the trailing submatrix updated
//     on the FP64 matrix cores (v_mfma_f64_16x16x4f64);
//   - triangular solves blocked by 16 rows: one wavefront solves each
//     diagonal block, then every thread updates its row.
#include <hip/hip_runtime.h>
#include <math.h>
#include "mech_dev.hpp"
#include "wave.hpp"

namespace chem {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int BT = 256;   // threads per cell
constexpr int NB = 16;    // LU block
constexpr int SB = 16;    // triangular-solve block

__constant__ double kBigA[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.544, 0, 0, 0, 0, 0},
    {0.9466785280815826, 0.2557011698983284, 0, 0, 0, 0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0, 0}};
__constant__ double kBigC[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {-5.6688, 0, 0, 0, 0, 0},
    {-2.430093356833875, -0.2063599157091915, 0, 0, 0, 0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0, 0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0, 0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
     -6.058818238834054, 0}};
constexpr double kBigGamma = 0.25;

__device__ __forceinline__ void lds_add_b(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// LDS layout of one cell (in doubles); lda is odd so that thread-per-row
// accesses fall into distinct banks.
struct BigLds {
    int n, N, lda;
    double *A, *C, *g, *hh, *e, *cp, *tb, *w, *vec, *red;
    int *ipiv, *perm;
};

__host__ __device__ inline int big_lda(int n) { return n | 1; }
__host__ __device__ inline size_t big_lds_doubles(int n) {
    const int N = n - 1;
    return (size_t)n * big_lda(n) + 4 * (N + 1) + 2 * N + n + n + 16 + n;  // ipiv, perm share n doubles
}

__device__ __forceinline__ BigLds big_layout(int n, double *lds) {
    BigLds L;
    L.n = n;
    L.N = n - 1;
    L.lda = big_lda(n);
    double *q = lds;
    L.A = q; q += (size_t)n * L.lda;
    L.C = q; q += L.N + 1;
    L.g = q; q += L.N + 1;
    L.hh = q; q += L.N + 1;
    L.w = q; q += L.N + 1;
    L.e = q; q += L.N;
    L.cp = q; q += L.N;
    L.tb = q; q += n;
    L.vec = q; q += n;
    L.red = q; q += 16;
    L.ipiv = (int *)q;          // n ints
    L.perm = L.ipiv + n;        // n ints (2n ints fit in n doubles)
    return L;
}

// Sum / max over the 256 threads; every thread returns the same bits.
__device__ __forceinline__ double block_sum(double v, double *red) {
    const double s = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}
__device__ __forceinline__ double block_max(double v, double *red) {
    const double s = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[4 + (threadIdx.x >> 6)] = s;
    __syncthreads();
    return max2(max2(red[4], red[5]), max2(red[6], red[7]));
}
__device__ __forceinline__ bool block_any(bool p, double *red) {
    return block_max(p ? 1.0 : 0.0, red) > 0.0;
}
// value of thread `src` to every thread
__device__ __forceinline__ double block_bcast(double v, int src, double *red) {
    __syncthreads();
    if ((int)threadIdx.x == src) red[8] = v;
    __syncthreads();
    return red[8];
}

// -----------------------------------------------------------------------------
// f(y) and, with JAC, the analytic Jacobian into L.A (row-major, stride lda).
// Thread i returns f_i.  Same formulas as the wavefront kernel.
// -----------------------------------------------------------------------------
template <bool JAC>
__device__ double rhs_big(const MechDev *__restrict__ Mp, const double p, const double y,
                          const BigLds &L) {
    const MechDev &M = *Mp;
    const int tid = threadIdx.x;
    const int N = M.N, R = M.R, n = M.n, lda = L.lda;
    const double T = block_bcast(y, 0, L.red);
    const double lnT = log(T);
    const double invT = 1.0 / T;
    const bool sp = tid >= 1 && tid <= N;
    const int k = sp ? tid - 1 : 0;
    double cpR = 0.0, hRT = 0.0, gRT = 0.0, dcpR = 0.0, invWk = 0.0, Wk = 0.0;
    if (sp) {
        const auto *a = gbl(M.spc) + k * SPC_STRIDE;
        const double a1 = a[0], a2 = a[1], a3 = a[2], a4 = a[3], a5 = a[4], a6 = a[5], a7 = a[6];
        const double h2 = a[7], h3 = a[8], h4 = a[9], h5 = a[10];
        const double s3 = a[11], s4 = a[12], s5 = a[13];
        cpR = a1 + T * (a2 + T * (a3 + T * (a4 + T * a5)));
        hRT = a1 + T * (h2 + T * (h3 + T * (h4 + T * h5))) + a6 * invT;
        const double sR = a1 * lnT + T * (a2 + T * (s3 + T * (s4 + T * s5))) + a7;
        gRT = hRT - sR;
        if (JAC) dcpR = a2 + T * (2.0 * a3 + T * (3.0 * a4 + T * (4.0 * a5)));
        Wk = a[14];
        invWk = a[15];
    }
    const double yw = sp ? y * invWk : 0.0;
    const double sumYW = block_sum(yw, L.red);
    const double rho = p / (RU_ERG * T * sumYW);
    const double Ctot = rho * sumYW;
    if (sp) {
        L.C[k] = rho * yw;
        L.g[k] = gRT;
        if (JAC) {
            L.hh[k] = hRT;
            L.e[k] = hRT * invWk;
            L.cp[k] = cpR * invWk;
        }
    }
    if (tid <= N) L.w[tid] = 0.0;
    if (JAC) {
        for (int i = tid; i < n * lda; i += BT) L.A[i] = 0.0;
        if (tid < n) L.tb[tid] = 0.0;
    }
    __syncthreads();

    const double ln_patm_RT = log(P_ATM / (RU_ERG * T));
    const double lnp = log(p);
    const auto *rxn = gbl(M.rxn);
    double *Cl = L.C, *gl = L.g, *hl = L.hh, *wl = L.w, *Jl = L.A, *tbl = L.tb;
    // Reactions j0 + tid are evaluated by all four wavefronts at once; their
    // LDS float-atomic scatter is done one wavefront after the other, so the
    // order of every sum (and the result) does not depend on scheduling.
    const int wv = tid >> 6;
#pragma unroll 1
    for (int j0 = 0; j0 < R; j0 += BT) {
        const bool valid = j0 + tid < R;
        const auto &rec = rxn[valid ? j0 + tid : R - 1];
        const int ix0 = rec.idx[0], ix1 = rec.idx[1], ix2 = rec.idx[2], ix3 = rec.idx[3];
        const int r0 = ix0 & 0xffff, r1 = (int)((unsigned)ix0 >> 16);
        const int p0 = ix1 & 0xffff, p1 = (int)((unsigned)ix1 >> 16);
        const int p2 = ix2 & 0xffff, tbw = (int)((unsigned)ix2 >> 16);
        const int tb = tbw & TB_CODE;
        const double snu = (double)((ix3 & 0xff) - 8);
        const int es0 = (ix3 >> 8) & 0xff, es1 = (ix3 >> 16) & 0xff;
        const int es2 = (int)((unsigned)ix3 >> 24);
        const double Cr0 = Cl[r0], Cr1 = Cl[r1], Cp0 = Cl[p0], Cp1 = Cl[p1], Cp2 = Cl[p2];
        const double dG = -gl[r0] - gl[r1] + gl[p0] + gl[p1] + gl[p2];
        double lnAj = rec.lnA, bj = rec.b, EaRj = rec.EaR;
        if (tbw & TB_PLOG)
            plog_arrhenius(M.plog + (size_t)(valid ? j0 + tid : R - 1) * PLOG_STRIDE, lnp, lnAj, bj, EaRj);
        const double ln_kf = lnAj + bj * lnT - EaRj * invT;
        const double ln_Kc = -dG + snu * ln_patm_RT;
        const double kf = exp(ln_kf);
        const double kr = exp(ln_kf - ln_Kc);
        const double Pf = Cr0 * Cr1;
        const double Pr = Cp0 * Cp1 * Cp2;
        const double e0v = rec.eff[0], e1v = rec.eff[1], e2v = rec.eff[2];
        double m = tb == TB_NONE ? 1.0 : Ctot + e0v * Cl[es0] + e1v * Cl[es1] + e2v * Cl[es2];
        if (tb >= TB_LIST0) {
            const int e1 = M.tb_ptr[tb - TB_LIST0 + 1];
            for (int e = M.tb_ptr[tb - TB_LIST0]; e < e1; ++e) m += M.eff_am1[e] * Cl[M.eff_sp[e]];
        }
        // fall-off: the rate constant is k_inf G([M], T) in place of k [M]
        double dGdM = 1.0, dlnGdT = 0.0;
        if (tbw & TB_FALLOFF) {
            double G;
            falloff_eval(M.fo + (size_t)(valid ? j0 + tid : R - 1) * FO_STRIDE, T, invT, lnT, kf,
                         bj * invT + EaRj * invT * invT, m, G, dGdM, dlnGdT);
            m = G;
        }
        const double Delta = kf * Pf - kr * Pr;
        const double q = m * Delta;
        double dqdT = 0.0, ds[5] = {0, 0, 0, 0, 0};
        if (JAC) {
            const double dlnkf = bj * invT + EaRj * invT * invT + dlnGdT;
            const double dH = -hl[r0] - hl[r1] + hl[p0] + hl[p1] + hl[p2];
            const double dlnkr = dlnkf - (dH - snu) * invT;
            const double mkf = m * kf, mkr = m * kr;
            dqdT = mkf * dlnkf * Pf - mkr * dlnkr * Pr;
            ds[0] = mkf * Cr1;
            ds[1] = mkf * Cr0;
            ds[2] = -mkr * Cp1 * Cp2;
            ds[3] = -mkr * Cp0 * Cp2;
            ds[4] = -mkr * Cp0 * Cp1;
        }
        for (int turn = 0; turn < BT / 64; ++turn) {
            if (wv == turn && valid) {
                lds_add_b(wl + r0, -q);
                lds_add_b(wl + r1, -q);
                lds_add_b(wl + p0, q);
                lds_add_b(wl + p1, q);
                lds_add_b(wl + p2, q);
                if (JAC) {
                    const int sl[5] = {r0, r1, p0, p1, p2};
#pragma unroll
                    for (int a = 0; a < 5; ++a) {
                        const int sa = sl[a];
                        if (sa >= N) continue;
                        const double nu = a < 2 ? -1.0 : 1.0;
                        double *row = Jl + (size_t)(sa + 1) * lda;
                        lds_add_b(row, nu * dqdT);
#pragma unroll
                        for (int b = 0; b < 5; ++b)
                            if (sl[b] < N) lds_add_b(row + 1 + sl[b], nu * ds[b]);
                        if (tb != TB_NONE) {
                            const double nd = nu * Delta * dGdM;
                            lds_add_b(tbl + sa + 1, nd);
                            if (es0 < N) lds_add_b(row + 1 + es0, nd * e0v);
                            if (es1 < N) lds_add_b(row + 1 + es1, nd * e1v);
                            if (es2 < N) lds_add_b(row + 1 + es2, nd * e2v);
                            if (tb >= TB_LIST0) {
                                const int e1 = M.tb_ptr[tb - TB_LIST0 + 1];
                                for (int e = M.tb_ptr[tb - TB_LIST0]; e < e1; ++e)
                                    lds_add_b(row + 1 + M.eff_sp[e], nd * M.eff_am1[e]);
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
    }

    const double fk = sp ? Wk * wl[k] / rho : 0.0;
    const double hs = block_sum(sp ? hRT * invWk * fk : 0.0, L.red);
    const double cps = block_sum(sp ? y * cpR * invWk : 0.0, L.red);
    const double fT = -T * hs / cps;
    if (JAC) {
        const double cpf = block_sum(sp ? cpR * invWk * fk : 0.0, L.red);
        const double dcps = block_sum(sp ? y * dcpR * invWk : 0.0, L.red);
        const double Wbar = 1.0 / sumYW;
        if (sp) {
            double *row = Jl + (size_t)tid * lda;
            const double tbk = tbl[tid];
            double s0 = 0.0, s1 = 0.0;
            int l = 0;
            for (; l + 1 < N; l += 2) {
                s0 += (row[1 + l] + tbk) * Cl[l];
                s1 += (row[2 + l] + tbk) * Cl[l + 1];
            }
            if (l < N) s0 += (row[1 + l] + tbk) * Cl[l];
            const double s = s0 + s1;
            const double cst = fk * Wbar - Wk * Wbar * s / rho;
            const auto *iw = gbl(M.invW);
            for (int i = 0; i < N; ++i) row[1 + i] = iw[i] * (Wk * (row[1 + i] + tbk) + cst);
            row[0] = Wk / rho * (row[0] - s * invT) + fk * invT;
        }
        __syncthreads();
        if (tid < n) {
            double a0 = 0.0, a1 = 0.0;
            int kk = 0;
            for (; kk + 1 < N; kk += 2) {
                a0 += L.e[kk] * Jl[(size_t)(kk + 1) * lda + tid];
                a1 += L.e[kk + 1] * Jl[(size_t)(kk + 2) * lda + tid];
            }
            if (kk < N) a0 += L.e[kk] * Jl[(size_t)(kk + 1) * lda + tid];
            const double acc = (a0 + a1) * T;
            double v;
            if (tid == 0) v = -(cpf + acc) / cps - fT * dcps / cps;
            else v = -acc / cps - fT * L.cp[tid - 1] / cps;
            // row 0 is read by the loop above only through rows kk + 1 >= 1
            Jl[tid] = v;
        }
        __syncthreads();
    }
    return tid == 0 ? fT : fk;
}

// -----------------------------------------------------------------------------
// LU of L.A (n x n) with partial pivoting, thread i owning physical row i.
// Rows never move: step k's pivot is the free row with the largest |a_ik|
// (upper 48 bits of |a|, ties to the lowest row), found by an LDS 64-bit
// atomic maximum while the rows update the previous column, so each step
// costs one barrier.  On return L.perm[k] = the physical row of step k (its
// L part in columns before k, its U part from k on).  Returns false if a
// pivot is zero or not finite.
// -----------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long pivot_key(double v, int row) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(v));
    return ((b >> 16) << 16) | (unsigned long long)(0xffff - row);
}
__device__ __forceinline__ void key_max(unsigned long long *p, unsigned long long v) {
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ bool lu_big(const BigLds &L) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = L.n, lda = L.lda;
    double *A = L.A;
    int *prow = L.perm, *rem = L.ipiv;
    unsigned long long *slot = reinterpret_cast<unsigned long long *>(L.vec);   // one per column
    int *nrem = reinterpret_cast<int *>(L.red + 12);
    bool ok = true;
    bool free_row = tid < n;   // this thread's row has not been pivot yet
    for (int i = tid; i < n; i += BT) slot[i] = 0ull;
    __syncthreads();
    if (free_row) key_max(&slot[0], pivot_key(A[(size_t)tid * lda], tid));
    __syncthreads();
    for (int kb = 0; kb < n; kb += NB) {
        const int jb = min(NB, n - kb), ke = kb + jb;
        for (int k = kb; k < ke; ++k) {
            const int pr = 0xffff - (int)(slot[k] & 0xffffull);
            if (tid == 0) prow[k] = pr;
            const double *rp = A + (size_t)pr * lda;
            const double piv = rp[k];
            if (!(fabs(piv) > 0.0) || !(fabs(piv) < INFINITY)) ok = false;
            const double rinv = 1.0 / piv;
            if (tid == pr) free_row = false;
            if (free_row) {
                double *ri = A + (size_t)tid * lda;
                const double l = ri[k] * rinv;
                ri[k] = l;
                for (int j = k + 1; j < ke; ++j) ri[j] = fma(-l, rp[j], ri[j]);
                if (k + 1 < ke) key_max(&slot[k + 1], pivot_key(ri[k + 1], tid));
            }
            __syncthreads();
        }
        if (ke < n) {
            // block row of U: U12 = L11^-1 A12 on the block's pivot rows, one
            // thread per column; the remaining rows are listed for the update
            if (tid == 0) *nrem = 0;
            int pq[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) pq[q] = q < jb ? prow[kb + q] : 0;
            for (int j = ke + tid; j < n; j += BT) {
                double x[NB];
#pragma unroll
                for (int q = 0; q < NB; ++q) x[q] = q < jb ? A[(size_t)pq[q] * lda + j] : 0.0;
#pragma unroll
                for (int r = 1; r < NB; ++r) {
                    if (r < jb) {
                        double s = x[r];
#pragma unroll
                        for (int q = 0; q < r; ++q) s = fma(-A[(size_t)pq[r] * lda + kb + q], x[q], s);
                        x[r] = s;
                    }
                }
#pragma unroll
                for (int q = 1; q < NB; ++q)
                    if (q < jb) A[(size_t)pq[q] * lda + j] = x[q];
            }
            __syncthreads();
            if (free_row) rem[__hip_atomic_fetch_add(nrem, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)] = tid;
            __syncthreads();
            // trailing update A22 -= L21 U12 on the matrix cores, 16 x 16
            // tiles over the listed rows (each row's result does not depend
            // on its tile or position).  A wavefront takes whole rows of
            // tiles: their rows and L21 operands are loaded once, then it
            // walks the column tiles.
            const int m = n - ke, tiles = (m + 15) >> 4;
            const int lr = lane & 15, lk = lane >> 4;
            int brow[NB / 4];
#pragma unroll
            for (int ks = 0; ks < NB / 4; ++ks) {
                const int kk = kb + 4 * ks + lk;
                brow[ks] = kk < ke ? prow[kk] : -1;
            }
            for (int rt = wv; rt < tiles; rt += 4) {
                const int r0 = 16 * rt;
                int drow[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int rr = r0 + lk + 4 * i;
                    drow[i] = rr < m ? rem[rr] : -1;
                }
                const int ar = r0 + lr;
                const int arow = ar < m ? rem[ar] : -1;
                // v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16], B[l / 16][l % 16]
                // and D[l / 16 + 4 i][l % 16], i = 0..3 (checked on gfx950)
                double a[NB / 4];
#pragma unroll
                for (int ks = 0; ks < NB / 4; ++ks) {
                    const int kk = kb + 4 * ks + lk;
                    a[ks] = (arow >= 0 && kk < ke) ? -A[(size_t)arow * lda + kk] : 0.0;
                }
                for (int ct = 0; ct < tiles; ++ct) {
                    const int col = ke + 16 * ct + lr;
                    f64x4 acc;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[i] = (drow[i] >= 0 && col < n) ? A[(size_t)drow[i] * lda + col] : 0.0;
#pragma unroll
                    for (int ks = 0; ks < NB / 4; ++ks) {
                        const double b = (col < n && brow[ks] >= 0) ? A[(size_t)brow[ks] * lda + col] : 0.0;
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b, acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (drow[i] >= 0 && col < n) A[(size_t)drow[i] * lda + col] = acc[i];
                }
            }
            __syncthreads();
            // the next block's first pivot
            if (free_row) key_max(&slot[ke], pivot_key(A[(size_t)tid * lda + ke], tid));
            __syncthreads();
        }
    }
    return ok;
}

// Solve (L U) x = P b with the factors of lu_big (logical row k in physical
// row L.perm[k]); thread i passes b_i and receives x_i.
__device__ double solve_big(const BigLds &L, double b) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = L.n, lda = L.lda;
    const double *A = L.A;
    // b in row order in L.vec, the working vector in pivot order in L.w (the
    // production-rate array, free between RHS evaluations)
    double *v = L.w;
    if (tid < n) L.vec[tid] = b;
    __syncthreads();
    if (tid < n) v[tid] = L.vec[L.perm[tid]];
    __syncthreads();
    // forward, unit lower.  Wavefront 0 solves the diagonal block with the
    // block's entries loaded up front (lane r: row kb + r, zero where the
    // lane takes no update), so only readlane and FMA remain on the chain.
    for (int kb = 0; kb < n; kb += SB) {
        const int jb = min(SB, n - kb), ke = kb + jb;
        if (wv == 0) {
            const double *rl = A + (size_t)L.perm[kb + (lane < jb ? lane : 0)] * lda + kb;
            double a[SB];
#pragma unroll
            for (int q = 0; q < SB; ++q) a[q] = (lane > q && lane < jb) ? rl[q] : 0.0;
            double x = lane < jb ? v[kb + lane] : 0.0;
#pragma unroll
            for (int q = 0; q < SB; ++q)
                if (q < jb) x = fma(-a[q], readlane_d(x, q), x);
            if (lane < jb) v[kb + lane] = x;
        }
        __syncthreads();
        for (int i = ke + tid; i < n; i += BT) {
            const double *ri = A + (size_t)L.perm[i] * lda + kb;
            double r[SB], w[SB];
#pragma unroll
            for (int q = 0; q < SB; ++q) {
                r[q] = q < jb ? ri[q] : 0.0;
                w[q] = q < jb ? v[kb + q] : 0.0;
            }
            double s = v[i];
#pragma unroll
            for (int q = 0; q < SB; ++q)
                if (q < jb) s = fma(-r[q], w[q], s);
            v[i] = s;
        }
        __syncthreads();
    }
    // backward, upper
    const int last = ((n - 1) / SB) * SB;
    for (int kb = last; kb >= 0; kb -= SB) {
        const int jb = min(SB, n - kb);
        if (wv == 0) {
            // lane r: row kb + r of the diagonal block above the diagonal, and
            // the reciprocal of its diagonal entry
            const double *rl = A + (size_t)L.perm[kb + (lane < jb ? lane : 0)] * lda + kb;
            double a[SB];
#pragma unroll
            for (int q = 0; q < SB; ++q) a[q] = (lane < q && q < jb) ? rl[q] : 0.0;
            const double dinv = lane < jb ? 1.0 / rl[lane] : 0.0;
            double x = lane < jb ? v[kb + lane] : 0.0;
#pragma unroll
            for (int q = SB - 1; q >= 0; --q) {
                if (q < jb) {
                    const double xq = readlane_d(x * dinv, q);
                    x = lane == q ? xq : fma(-a[q], xq, x);
                }
            }
            if (lane < jb) v[kb + lane] = x;
        }
        __syncthreads();
        for (int i = tid; i < kb; i += BT) {
            const double *ri = A + (size_t)L.perm[i] * lda + kb;
            double r[SB], w[SB];
#pragma unroll
            for (int q = 0; q < SB; ++q) {
                r[q] = q < jb ? ri[q] : 0.0;
                w[q] = q < jb ? v[kb + q] : 0.0;
            }
            double s = v[i];
#pragma unroll
            for (int q = 0; q < SB; ++q)
                if (q < jb) s = fma(-r[q], w[q], s);
            v[i] = s;
        }
        __syncthreads();
    }
    const double x = tid < n ? v[tid] : 0.0;
    __syncthreads();
    return x;
}

// M = diag - J from the Jacobian slot into LDS
__device__ __forceinline__ void build_big(const BigLds &L, const double *__restrict__ Jg, double diag) {
    const int n = L.n, lda = L.lda;
    for (int i = threadIdx.x; i < n * n; i += BT) {
        const int r = i / n, c = i - r * n;
        L.A[(size_t)r * lda + c] = (r == c ? diag : 0.0) - Jg[i];
    }
    __syncthreads();
}

__device__ __forceinline__ void save_jac(const BigLds &L, double *__restrict__ Jg) {
    const int n = L.n, lda = L.lda;
    for (int i = threadIdx.x; i < n * n; i += BT) {
        const int r = i / n, c = i - r * n;
        Jg[i] = L.A[(size_t)r * lda + c];
    }
    __syncthreads();
}

__device__ bool rodas_attempt_big(const MechDev *__restrict__ M, const BigLds &L, const double *Jg,
                                  double p, double y, double f0, double h, double &ynew, double &err) {
    build_big(L, Jg, 1.0 / (kBigGamma * h));
    if (!lu_big(L)) return false;
    double u[6] = {0, 0, 0, 0, 0, 0};
    double ys = y;
    for (int s = 0; s < 6; ++s) {
        double rv = f0;
        if (s > 0) {
            ys = y;
            for (int j = 0; j < 5; ++j) ys += kBigA[s][j] * u[j];
            rv = rhs_big<false>(M, p, ys, L);
            for (int j = 0; j < 5; ++j) rv += (kBigC[s][j] / h) * u[j];
        }
        const double us = solve_big(L, rv);
#pragma unroll
        for (int j = 0; j < 6; ++j) u[j] = j == s ? us : u[j];
    }
    ynew = ys + u[5];
    err = u[5];
    return true;
}

__device__ __forceinline__ void init_big(const BigLds &L) {
    if (threadIdx.x == 0) {
        L.C[L.N] = 1.0;
        L.g[L.N] = 0.0;
        L.hh[L.N] = 0.0;
    }
    __syncthreads();
}

// Adaptive integration of one cell; control logic of the wavefront kernel.
__device__ void integrate_cell_big(const MechDev *__restrict__ M, const IntParams &P, int64_t cell,
                                   const BigLds &L, double *__restrict__ Jg) {
    const int tid = threadIdx.x;
    const int n = M->n, N = M->N;
    const double dt = P.dt;
    const double p = P.p[cell];
    double y = 0.0;
    if (tid == 0) y = P.T[cell];
    else if (tid <= N) y = P.Y[(int64_t)(tid - 1) * P.ncells + cell];
    const double T0 = block_bcast(y, 0, L.red);
    const bool bad_in = block_any(tid < n && !isfinite(y), L.red) || !(T0 > 0.0) || !(p > 0.0) ||
                        !isfinite(p);
    if (bad_in) {
        if (tid == 0) {
            if (P.status) P.status[cell] = 4;
            if (P.ref_status && P.flags && P.flags[cell] == 1) *P.ref_status = 4;
            if (P.steps) { P.steps[2 * cell] = 0; P.steps[2 * cell + 1] = 0; }
            if (P.cost) P.cost[cell] = 0;
            atomicAdd(&P.stats[0], 1ull);
            atomicAdd(&P.stats[3], 1ull);
        }
        __syncthreads();
        return;
    }
    double h = P.h ? P.h[cell] : 0.0;
    if (!(h > 0.0)) h = dt;
    double hnext = h, t = 0.0;
    int nacc = 0, nrej = 0, status = 0;
    bool rej_last = false;
    double f0 = rhs_big<true>(M, p, y, L);
    save_jac(L, Jg);
    while (t < dt) {
        if (nacc + nrej >= P.max_steps) { status = 1; break; }
        bool last = false;
        if (h >= dt - t) { h = dt - t; last = true; }
        if (h < P.hmin_frac * dt) { status = 2; break; }
        double ynew = 0.0, ev = 0.0;
        const bool ok = rodas_attempt_big(M, L, Jg, p, y, f0, h, ynew, ev);
        double e = 0.0;
        bool bad = !ok;
        if (ok) {
            const double sc = P.atol + P.rtol * fmax(fabs(y), fabs(ynew));
            const double r = tid < n ? fabs(ev) / sc : 0.0;
            bad = block_any(r != r, L.red);
            e = block_max(r, L.red);
        }
        if (!bad && e <= 1.0) {
            double fac = (e == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(e, -0.25)));
            if (rej_last) fac = fmin(fac, 1.0);
            y = ynew;
            t = last ? dt : t + h;
            ++nacc;
            hnext = h * fac;
            h = hnext;
            rej_last = false;
            if (t < dt) {
                f0 = rhs_big<true>(M, p, y, L);
                save_jac(L, Jg);
            }
        } else {
            const double fac = bad ? 0.2 : fmax(0.2, 0.9 * pow(e, -0.25));
            h = h * fac;
            ++nrej;
            rej_last = true;
        }
    }
    if (status == 0 && block_any(tid < n && !isfinite(y), L.red)) status = 3;
    if (tid == 0) P.T[cell] = y;
    else if (tid <= N) P.Y[(int64_t)(tid - 1) * P.ncells + cell] = y;
    if (tid == 0) {
        if (P.h) P.h[cell] = hnext;
        if (P.cost) P.cost[cell] = (uint32_t)(nacc + nrej);
        if (P.status) P.status[cell] = (uint8_t)status;
        if (P.ref_status && P.flags && P.flags[cell] == 1) *P.ref_status = status;
        if (P.steps) { P.steps[2 * cell] = nacc; P.steps[2 * cell + 1] = nrej; }
        atomicAdd(&P.stats[0], 1ull);
        atomicAdd(&P.stats[1], (unsigned long long)nacc);
        atomicAdd(&P.stats[2], (unsigned long long)nrej);
        if (status) atomicAdd(&P.stats[3], 1ull);
        atomicMax(&P.stats[4], (unsigned long long)(nacc + nrej));
    }
    __syncthreads();
}

// Static schedule: workgroup b takes cells b, b + grid, b + 2 grid, ...
__global__ __launch_bounds__(BT) void k_big_plain(const MechDev *__restrict__ M, IntParams P,
                                                  double *jws) {
    extern __shared__ double lds[];
    const BigLds L = big_layout(M->n, lds);
    init_big(L);
    double *Jg = jws + (size_t)blockIdx.x * M->n * M->n;
    // round robin over the slots, or (block_static) one contiguous block each
    const int64_t B = (P.ncells + gridDim.x - 1) / gridDim.x;
    const int64_t c0 = P.block_static ? blockIdx.x * B : blockIdx.x;
    const int64_t c1 = P.block_static ? (c0 + B < P.ncells ? c0 + B : P.ncells) : P.ncells;
    const int64_t stride = P.block_static ? 1 : gridDim.x;
    for (int64_t cell = c0; cell < c1; cell += stride) {
        if (P.flags && P.flags[cell] >= 2) continue;
        integrate_cell_big(M, P, cell, L, Jg);
    }
}

// Work queue with XCD segments and stealing, as in the wavefront kernel.
__global__ __launch_bounds__(BT) void k_big_queue(const MechDev *__restrict__ M, IntParams P,
                                                  double *jws) {
    extern __shared__ double lds[];
    const BigLds L = big_layout(M->n, lds);
    init_big(L);
    double *Jg = jws + (size_t)blockIdx.x * M->n * M->n;
    const int nact = *P.n_active;
    const int chunk = P.chunk;
    int seg = blockIdx.x % NSEG;
    int probes = 0;
    while (probes < NSEG) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const int c = atomicAdd(&P.seg_ctr[seg], chunk);
            L.red[9] = (double)c;
        }
        __syncthreads();
        const int c = (int)L.red[9];
        const int first = seg + NSEG * c;
        if (first >= nact) {
            seg = seg + 1 == NSEG ? 0 : seg + 1;
            ++probes;
            continue;
        }
        probes = 0;
        for (int q = 0; q < chunk; ++q) {
            const int pos = first + NSEG * q;
            if (pos >= nact) break;
            integrate_cell_big(M, P, P.queue[pos], L, Jg);
        }
    }
}

// Kernel-level checks: f and J per cell; one fixed Rodas4 step per cell.
__global__ __launch_bounds__(BT) void k_big_rhs_jac(const MechDev *__restrict__ M, IntParams P,
                                                    double *fout, double *Jout) {
    extern __shared__ double lds[];
    const BigLds L = big_layout(M->n, lds);
    init_big(L);
    const int64_t cell = blockIdx.x;
    const int tid = threadIdx.x, n = M->n, N = M->N;
    double y = 0.0;
    if (tid == 0) y = P.T[cell];
    else if (tid <= N) y = P.Y[(int64_t)(tid - 1) * P.ncells + cell];
    const double f = rhs_big<true>(M, P.p[cell], y, L);
    if (fout && tid < n) fout[cell * n + tid] = f;
    if (Jout)
        for (int i = tid; i < n * n; i += BT)
            Jout[cell * n * n + i] = L.A[(size_t)(i / n) * L.lda + (i % n)];
}

__global__ __launch_bounds__(BT) void k_big_rodas_step(const MechDev *__restrict__ M, IntParams P,
                                                       double h, double *ynew_out, double *err_out,
                                                       double *jws) {
    extern __shared__ double lds[];
    const BigLds L = big_layout(M->n, lds);
    init_big(L);
    const int64_t cell = blockIdx.x;
    const int tid = threadIdx.x, n = M->n, N = M->N;
    double *Jg = jws + (size_t)blockIdx.x * n * n;
    double y = 0.0;
    if (tid == 0) y = P.T[cell];
    else if (tid <= N) y = P.Y[(int64_t)(tid - 1) * P.ncells + cell];
    const double p = P.p[cell];
    const double f0 = rhs_big<true>(M, p, y, L);
    save_jac(L, Jg);
    double ynew = 0.0, err = 0.0;
    const bool ok = rodas_attempt_big(M, L, Jg, p, y, f0, h, ynew, err);
    if (!ok) { ynew = NAN; err = NAN; }
    if (tid < n) {
        ynew_out[cell * n + tid] = ynew;
        err_out[cell * n + tid] = err;
    }
}

// ---------------------------------------------------------------- host ------
size_t big_lds_bytes(int n) { return sizeof(double) * big_lds_doubles(n); }

static hipError_t set_lds(const void *k, size_t sh) {
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
}

hipError_t big_prepare(int n) {
    const size_t sh = big_lds_bytes(n);
    hipError_t e;
    if ((e = set_lds((const void *)k_big_plain, sh))) return e;
    if ((e = set_lds((const void *)k_big_queue, sh))) return e;
    if ((e = set_lds((const void *)k_big_rhs_jac, sh))) return e;
    return set_lds((const void *)k_big_rodas_step, sh);
}

hipError_t launch_integrate_big(const MechDev &M, const MechDev *Md, const IntParams &P,
                                int schedule, int grid, double *jws, hipStream_t s) {
    const size_t sh = big_lds_bytes(M.n);
    if (schedule != 1)   // plain round robin, or static blocks (P.block_static)
        hipLaunchKernelGGL(k_big_plain, dim3((unsigned)grid), dim3(BT), sh, s, Md, P, jws);
    else
        hipLaunchKernelGGL(k_big_queue, dim3((unsigned)grid), dim3(BT), sh, s, Md, P, jws);
    return hipGetLastError();
}

hipError_t launch_big_rhs_jac(const MechDev &M, const MechDev *Md, const IntParams &P, double *f,
                              double *J, hipStream_t s) {
    hipLaunchKernelGGL(k_big_rhs_jac, dim3((unsigned)P.ncells), dim3(BT), big_lds_bytes(M.n), s, Md,
                       P, f, J);
    return hipGetLastError();
}

hipError_t launch_big_rodas_step(const MechDev &M, const MechDev *Md, const IntParams &P, double h,
                                 double *ynew, double *err, double *jws, hipStream_t s) {
    hipLaunchKernelGGL(k_big_rodas_step, dim3((unsigned)P.ncells), dim3(BT), big_lds_bytes(M.n), s,
                       Md, P, h, ynew, err, jws);
    return hipGetLastError();
}

int big_occupancy(int n) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_big_queue, BT, big_lds_bytes(n)) !=
        hipSuccess)
        return 0;
    return blocks;
}

}  // namespace chem
