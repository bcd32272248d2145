// Per-cell stiff chemistry integration on CDNA4 (gfx950), FP64.
//
// One 64-lane wavefront owns one cell.  Lane r holds unknown r of the state
// y = (T, Y_1..Y_N), so species k lives on lane k + 1.  The right-hand side
// (mass-action kinetics with reverse rates from equilibrium constants of the
// NASA-7 thermo, third-body enhancement), the analytic Jacobian and the Rodas4
// stages are evaluated cooperatively:
//   - reaction pass, lane = reaction (stride 64): rate constants and rates of
//     progress, scattered to the production rates of their species with LDS
//     float atomics, and for the Jacobian the per-slot derivatives, scattered
//     into an LDS Jacobian the same way (one wavefront issues every atomic, so
//     the order of the sums is fixed);
//   - species pass, lane = species: dY/dt and dT/dt from the production rates,
//     and the chain rule from concentrations to (T, Y) on the Jacobian rows;
//   - LU with partial pivoting, row-per-lane in registers: lane r holds row r
//     of M = I/(gamma h) - J; the pivot row is broadcast with readlane and no
//     row moves while factorising (a lane remembers at which step it became
//     pivot); at the end the rows are put in pivot order;
//   - triangular solves follow the same layout.
// The cell's arithmetic does not depend on which workgroup runs it, so the
// static launch and the work-queue launch give bit-identical results.
//
// LDS of a work-queue workgroup: the shared species and reaction records,
// one small region per wavefront (concentrations, Gibbs energies, production
// rates, solve results), and a pool of Jacobian slots smaller than the number
// of wavefronts.  A wavefront holds a slot only from the Jacobian's assembly
// until the iteration matrix has been built in its registers; after a
// rejected step it assembles the (identical) Jacobian again.  This keeps
// eight wavefronts, two per SIMD, on a CU for the 53-species mechanism.
#include <hip/hip_runtime.h>
#include <math.h>
#include "mech_dev.hpp"
#include "wave.hpp"

namespace chem {

// Rodas4, Hairer & Wanner, Solving ODEs II, Sec. IV.7, transformed form:
// (I/(gamma h) - J) u_i = f(y + sum_j a_ij u_j) + sum_j (c_ij / h) u_j.
// Row 5 of A is the stage-6 input (a_5j, then 1 for u_5).
static __constant__ double kRodasA[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.544, 0, 0, 0, 0, 0},
    {0.9466785280815826, 0.2557011698983284, 0, 0, 0, 0},
    {3.314825187068521, 2.896124015972201, 0.9986419139977817, 0, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 0, 0},
    {1.221224509226641, 6.019134481288629, 12.53708332932087, -0.6878860361058950, 1.0, 0}};
static __constant__ double kRodasC[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {-5.6688, 0, 0, 0, 0, 0},
    {-2.430093356833875, -0.2063599157091915, 0, 0, 0, 0},
    {-0.1073529058151375, -9.594562251023355, -20.47028614809616, 0, 0, 0},
    {7.496443313967647, -10.24680431464352, -33.99990352819905, 11.70890893206160, 0, 0},
    {8.083246795921522, -7.981132988064893, -31.52159432874371, 16.31930543123136,
     -6.058818238834054, 0}};
constexpr double kGamma = 0.25;

__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A workgroup holds up to eight wavefronts, each integrating its own cells in
// its own LDS region; they share one LDS copy of the species and reaction
// records (placed first) and the pool of Jacobian slots.  Within a cell only
// the wavefront synchronises: LDS operations of one wavefront complete in
// order, so ordering them needs a compiler barrier and a wavefront-scope
// fence, not a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

extern __shared__ double lds_all[];

// The workgroup's LDS copy of the records is field-major: field f of species
// k at f N + k, field f of reaction j at N SPC_STRIDE + f R + j (a reaction
// record is 8 doubles, its four index words packed two per double), so the
// lanes of a wavefront, each on its own species or reaction, read
// consecutive doubles.
constexpr int RXN_FIELDS = (int)(sizeof(RxnRec) / sizeof(double));
static_assert(RXN_FIELDS == 8, "reaction record of 8 doubles");

__host__ __device__ inline int table_doubles(const MechDev &M) {
    return M.N * SPC_STRIDE + M.R * RXN_FIELDS;
}
constexpr int kLockDoubles = 8;   // slot locks (up to 16 ints) ahead of the slots

// The Jacobian slot of one wavefront.  With as many slots as wavefronts
// (nslots == 0 here: a private slot) nothing is shared and the Jacobian stays
// valid until the next assembly; otherwise a slot is taken from the pool with
// an LDS compare-and-swap before assembly and given back once the iteration
// matrix is in registers.  A holder never waits for anything, so every
// waiting wavefront eventually gets a slot.
struct JacSlot {
    double *J;        // the held (or private) slot, row-major with stride ldj
    double *pool;     // first slot of the pool
    int *locks;       // one int per pooled slot: 0 free, 1 held
    int nslots;       // pooled slots; 0: private slot
    int held;         // index of the held pooled slot, -1 none
    int jdoubles;

    __device__ __forceinline__ bool pooled() const { return nslots > 0; }
    __device__ __forceinline__ void acquire() {
        if (!pooled() || held >= 0) return;
        int s = -1;
        while (true) {
            if ((threadIdx.x & 63u) == 0) {
                for (int k = 0; k < nslots; ++k) {
                    int expect = 0;
                    if (__hip_atomic_compare_exchange_strong(&locks[k], &expect, 1, __ATOMIC_ACQUIRE,
                                                             __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_WORKGROUP)) {
                        s = k;
                        break;
                    }
                }
            }
            s = __builtin_amdgcn_readfirstlane(s);
            if (s >= 0) break;
            __builtin_amdgcn_s_sleep(2);
        }
        held = s;
        J = pool + (size_t)s * jdoubles;
        wave_sync();
    }
    __device__ __forceinline__ void release() {
        if (!pooled() || held < 0) return;
        wave_sync();
        if ((threadIdx.x & 63u) == 0)
            __hip_atomic_store(&locks[held], 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        held = -1;
    }
};

// -----------------------------------------------------------------------------
// f(y), and with JAC the analytic Jacobian into LDS (row-major, stride ldj).
// Returns f_r on lane r.  All lanes of the wave must call it.
// -----------------------------------------------------------------------------
// Species sums: with at most 16 unknowns every species sits in lanes 0..15.
template <int NP>
__device__ __forceinline__ double species_sum(double v) {
    if constexpr (NP <= 16) return wave_sum_row0(v);
    else return wave_sum(v);
}

template <int NP, bool JAC, bool LT, bool FO>
__device__ __forceinline__ double rhs_eval(const MechDev *__restrict__ Mp, const double p,
                                           const double y, double *__restrict__ lds,
                                           double *__restrict__ Jl) {
    // The memory clobber keeps the descriptor loads, and the opaque lane index
    // every per-lane address, local to this call instead of being hoisted out
    // of the step loop and held in registers across it.  The sizes are made
    // opaque too: the trip counts and strides derived from them are then
    // formed here rather than held (spilled) across the step loop.
    asm volatile("" ::: "memory");
    int lane = lane_id();
    asm volatile("" : "+v"(lane));
    const MechDev &M = *Mp;
    int N = M.N, R = M.R, n = M.n, ldj = M.ldj;
    asm volatile("" : "+s"(N), "+s"(R), "+s"(n), "+s"(ldj));
    double *__restrict__ wl = lds + M.off_q;    // production rates omega_k (+ sentinel)
    double *__restrict__ Cl = lds + M.off_C;
    double *__restrict__ gl = lds + M.off_g;
    double *__restrict__ gil = lds + M.off_gi;
    double *__restrict__ hl = lds + M.off_h;
    double *__restrict__ el = lds + M.off_e;
    double *__restrict__ cpl = lds + M.off_cp;
    double *__restrict__ tbl = lds + M.off_tb;

    const double T = readlane_d(y, 0);
    const double lnT = log(T);
    const double ln_patm_RT = kLnPatmRu - lnT;   // ln(p_atm / (R T))
    const double invT = 1.0 / T;
    const bool sp = lane >= 1 && lane <= N;
    const int k = sp ? lane - 1 : 0;

    // species thermo (NASA-7 single range), Horner form
    double cpR = 0.0, hRT = 0.0, gRT = 0.0, dcpR = 0.0, invWk = 0.0, Wk = 0.0;
    if (sp) {
        const double *a = LT ? lds_all + k : (const double *)(gbl(M.spc) + k * SPC_STRIDE);
        const int fs = LT ? N : 1;   // distance between fields
        const double a1 = a[0], a2 = a[fs], a3 = a[2 * fs], a4 = a[3 * fs], a5 = a[4 * fs];
        const double a6 = a[5 * fs], a7 = a[6 * fs];
        const double h2 = a[7 * fs], h3 = a[8 * fs], h4 = a[9 * fs], h5 = a[10 * fs];
        const double s3 = a[11 * fs], s4 = a[12 * fs], s5 = a[13 * fs];
        cpR = a1 + T * (a2 + T * (a3 + T * (a4 + T * a5)));
        hRT = a1 + T * (h2 + T * (h3 + T * (h4 + T * h5))) + a6 * invT;
        const double sR = a1 * lnT + T * (a2 + T * (s3 + T * (s4 + T * s5))) + a7;
        gRT = hRT - sR;
        if (JAC) dcpR = a2 + T * (2.0 * a3 + T * (3.0 * a4 + T * (4.0 * a5)));
        Wk = a[14 * fs];
        invWk = a[15 * fs];
    }
    const double yw = sp ? y * invWk : 0.0;
    const double sumYW = species_sum<NP>(yw);
    const double rho = p / (RU_ERG * T * sumYW);
    const double irho = (RU_ERG * T * sumYW) / p;
    const double Ctot = rho * sumYW;
    if (sp) {
        Cl[k] = rho * yw;
        // species factors of the equilibrium constant: a reaction's
        // 1 / K_c = prod_products E_k / prod_reactants E_k, E_k = exp(g_k) RT / p_atm
        const double gx = gRT - ln_patm_RT;
        gl[k] = exp(gx);
        gil[k] = exp(-gx);
        if (JAC) {
            hl[k] = hRT;
            el[k] = hRT * invWk;
            cpl[k] = cpR * invWk;
        }
    }
    if (lane <= N) wl[lane] = 0.0;
    if (JAC) {
        for (int i = lane; i < n * ldj; i += 64) Jl[i] = 0.0;
        if (lane < n) tbl[lane] = 0.0;
    }
    wave_sync();

    // reaction pass: rates of progress scattered to the production rates of
    // their reactant and product slots (LDS float atomics; missing slots hit
    // the sentinel entry N)
    const double lnp = FO ? log(p) : 0.0;
    const double *rtab = lds_all + N * SPC_STRIDE;
    const RxnRec *rxn = (const RxnRec *)gbl(M.rxn);
    auto reaction = [&](const int j, const bool valid) {
        RxnRec rec;
        if (LT) {
            const double *r = rtab + j;
            rec.lnA = r[0];
            rec.b = r[R];
            rec.EaR = r[2 * R];
            rec.eff[0] = r[3 * R];
            rec.eff[1] = r[4 * R];
            rec.eff[2] = r[5 * R];
            const double w01 = r[6 * R], w23 = r[7 * R];
            rec.idx[0] = __double2loint(w01);
            rec.idx[1] = __double2hiint(w01);
            rec.idx[2] = __double2loint(w23);
            rec.idx[3] = __double2hiint(w23);
        } else {
            rec = rxn[j];
        }
        const int ix0 = rec.idx[0], ix1 = rec.idx[1], ix2 = rec.idx[2], ix3 = rec.idx[3];
        const int r0 = ix0 & 0xffff, r1 = (int)((unsigned)ix0 >> 16);
        const int p0 = ix1 & 0xffff, p1 = (int)((unsigned)ix1 >> 16);
        const int p2 = ix2 & 0xffff, tbw = (int)((unsigned)ix2 >> 16);
        const int tb = tbw & TB_CODE;
        const double snu = (double)((ix3 & 0xff) - 8);
        const int es0 = (ix3 >> 8) & 0xff, es1 = (ix3 >> 16) & 0xff;
        const int es2 = (int)((unsigned)ix3 >> 24);
        const double Cr0 = Cl[r0], Cr1 = Cl[r1], Cp0 = Cl[p0], Cp1 = Cl[p1], Cp2 = Cl[p2];
        double lnAj = rec.lnA, bj = rec.b, EaRj = rec.EaR;
        if (FO && (tbw & TB_PLOG)) plog_arrhenius(M.plog + (size_t)j * PLOG_STRIDE, lnp, lnAj, bj, EaRj);
        const double ln_kf = lnAj + bj * lnT - EaRj * invT;
        const double kf = exp(ln_kf);
        const double kr = kf * ((gl[p0] * gil[r0]) * (gl[p1] * gil[r1]) * gl[p2]);
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
        if (FO && (tbw & TB_FALLOFF)) {
            double G;
            falloff_eval(M.fo + (size_t)j * FO_STRIDE, T, invT, lnT, kf,
                         bj * invT + EaRj * invT * invT, m, G, dGdM, dlnGdT);
            m = G;
        }
        const double Delta = valid ? kf * Pf - kr * Pr : 0.0;
        const double q = m * Delta;
        lds_add(wl + r0, -q);
        lds_add(wl + r1, -q);
        lds_add(wl + p0, q);
        lds_add(wl + p1, q);
        lds_add(wl + p2, q);
        if (JAC) {
            const double dlnkf = bj * invT + EaRj * invT * invT + dlnGdT;
            const double dH = -hl[r0] - hl[r1] + hl[p0] + hl[p1] + hl[p2];
            const double dlnkr = dlnkf - (dH - snu) * invT;
            const double mkf = valid ? m * kf : 0.0, mkr = valid ? m * kr : 0.0;
            const double dqdT = mkf * dlnkf * Pf - mkr * dlnkr * Pr;
            const int sl[5] = {r0, r1, p0, p1, p2};
            const double ds[5] = {mkf * Cr1, mkf * Cr0, -mkr * Cp1 * Cp2, -mkr * Cp0 * Cp2,
                                  -mkr * Cp0 * Cp1};
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                const int sa = sl[a];
                if (sa >= N) continue;
                const double nu = a < 2 ? -1.0 : 1.0;
                double *row = Jl + (sa + 1) * ldj;
                lds_add(row, nu * dqdT);
#pragma unroll
                for (int b = 0; b < 5; ++b)
                    if (sl[b] < N) lds_add(row + 1 + sl[b], nu * ds[b]);
                if (tb != TB_NONE) {
                    const double nd = nu * Delta * dGdM;
                    lds_add(tbl + sa + 1, nd);
                    if (es0 < N) lds_add(row + 1 + es0, nd * e0v);
                    if (es1 < N) lds_add(row + 1 + es1, nd * e1v);
                    if (es2 < N) lds_add(row + 1 + es2, nd * e2v);
                    if (tb >= TB_LIST0) {
                        const int e1 = M.tb_ptr[tb - TB_LIST0 + 1];
                        for (int e = M.tb_ptr[tb - TB_LIST0]; e < e1; ++e)
                            lds_add(row + 1 + M.eff_sp[e], nd * M.eff_am1[e]);
                    }
                }
            }
        }
    };
    // one reaction per lane and trip: with two wavefronts per SIMD the other
    // wavefront covers this one's load, exp and LDS latencies, and the
    // smaller loop body keeps registers free
#pragma unroll 1
    for (int j = lane; j < R; j += 64) reaction(j, true);
    wave_sync();

    // species: dY_k/dt = W_k omega_k / rho; dT/dt = -sum_k H_k omega_k / (rho cp)
    const double fk = sp ? Wk * wl[k] * irho : 0.0;
    const double hs = species_sum<NP>(sp ? hRT * invWk * fk : 0.0);
    const double cps = species_sum<NP>(sp ? y * cpR * invWk : 0.0);
    const double icps = 1.0 / cps;
    const double fT = -T * hs * icps;

    if (JAC) {
        const double cpf = species_sum<NP>(sp ? cpR * invWk * fk : 0.0);
        const double dcps = species_sum<NP>(sp ? y * dcpR * invWk : 0.0);
        const double Wbar = 1.0 / sumYW;
        // species rows: chain rule from concentrations to (T, Y)
        if (sp) {
            double *row = Jl + lane * ldj;
            const double tbk = tbl[lane];
            double s0 = 0.0, s1 = 0.0;
            int l = 0;
#pragma unroll 4
            for (; l + 1 < N; l += 2) {
                s0 += (row[1 + l] + tbk) * Cl[l];
                s1 += (row[2 + l] + tbk) * Cl[l + 1];
            }
            if (l < N) s0 += (row[1 + l] + tbk) * Cl[l];
            const double s = s0 + s1;
            const double cst = fk * Wbar - Wk * Wbar * s * irho;
            if (LT) {
                // 1/W_i from the species records in the shared table (broadcast reads)
#pragma unroll 8
                for (int i = 0; i < N; ++i)
                    row[1 + i] = lds_all[15 * N + i] * (Wk * (row[1 + i] + tbk) + cst);
            } else {
                const auto *iw = gbl(M.invW);
#pragma unroll 8
                for (int i = 0; i < N; ++i) row[1 + i] = iw[i] * (Wk * (row[1 + i] + tbk) + cst);
            }
            row[0] = Wk * irho * (row[0] - s * invT) + fk * invT;
        }
        wave_sync();
        // temperature row: J_T,c = -(sum_k e_k J_kc)/cp - f_T dcp/dy_c / cp
        if (lane < n) {
            double a0 = 0.0, a1 = 0.0;
            int kk = 0;
#pragma unroll 4
            for (; kk + 1 < N; kk += 2) {
                a0 += el[kk] * Jl[(kk + 1) * ldj + lane];
                a1 += el[kk + 1] * Jl[(kk + 2) * ldj + lane];
            }
            if (kk < N) a0 += el[kk] * Jl[(kk + 1) * ldj + lane];
            const double acc = (a0 + a1) * T;
            double v;
            if (lane == 0) v = -(cpf + acc) * icps - fT * dcps * icps;
            else v = -acc * icps - fT * cpl[lane - 1] * icps;
            Jl[lane] = v;
        }
        wave_sync();
    }
    return lane == 0 ? fT : fk;
}

// -----------------------------------------------------------------------------
// Dense linear algebra of the Rodas stages, one matrix row per lane.
// -----------------------------------------------------------------------------
// Pivot search for one column, cut into stages that the LU interleaves with
// the previous step's trailing update (lookahead), so that the search's
// dependent chain overlaps independent work.  The search compares the upper
// 32 bits of |a| (sign, exponent and 20 mantissa bits): the chosen row is
// within a factor 1 + 2^-20 of the largest candidate, ties going to the
// lowest lane.  A NaN entry sorts above every number and is caught by the
// reciprocal check after the factorisation.
template <int NP>
struct PivotSearch {
    unsigned key, v;
    int p;
    double piv, r, e;
    // cand: this lane's row may be pivot; candm: the same as a scalar lane mask
    __device__ __forceinline__ void stage(int s, double col, bool cand, unsigned long long candm) {
        switch (s) {
            case 0:
                key = cand ? ((unsigned)__double2hiint(col) & 0x7fffffffu) : 0u;
                v = max(key, (unsigned)__builtin_amdgcn_update_dpp(0, (int)key, 0xB1, 0xf, 0xf, false));
                break;
            case 1: v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false)); break;
            case 2: v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false)); break;
            case 3: v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false)); break;
            case 4: {
                if constexpr (NP <= 16) {   // candidates only in lanes 0..15
                    v = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
                } else {
                    // each 16-lane row holds its maximum; row broadcasts fold
                    // row 0 into row 1 and row 2 into row 3, then rows 0-1 into
                    // rows 2-3, so lane 63 holds the maximum of the wavefront
                    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
                    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
                    v = (unsigned)__builtin_amdgcn_readlane((int)v, 63);
                }
                break;
            }
            case 5: {
                const unsigned long long bal = ballot(key == v) & candm;
                p = bal ? (int)__builtin_ctzll(bal) : 0;
                break;
            }
            case 6: piv = readlane_d(col, p); break;
            case 7: r = __builtin_amdgcn_rcp(piv); e = fma(-piv, r, 1.0); break;
            case 8: r = fma(r, e, r); e = fma(-piv, r, 1.0); break;
            default: r = fma(r, e, r); break;   // 1/piv: estimate + two Newton-Raphson steps
        }
    }
};
constexpr int kSearchStages = 10;
constexpr int kColsPerStage = 4;

// LU with partial pivoting, row-per-lane.  No row moves while factorising:
// a lane remembers the step t at which its row became pivot.  At the end the
// rows are put in pivot order (one ds_bpermute per register), so on return
// lane k holds the row that was pivot at step k: L in columns before k, U from
// k on; dinv = 1/U_kk; pk = the lane that row came from (identity beyond the
// matrix).
template <int NP>
__device__ __forceinline__ bool lu_factor(double (&a)[NP], double &dinv, int &pk) {
    int lane = lane_id();
    asm volatile("" : "+v"(lane));
    const bool active = lane < NP;
    int t = -1;
    dinv = 0.0;
    // rows not yet pivot, as a scalar lane mask: the per-lane tests below
    // read it directly instead of comparing vector registers
    unsigned long long rem = NP >= 64 ? ~0ull : (1ull << NP) - 1ull;
    PivotSearch<NP> ps;
#pragma unroll
    for (int s = 0; s < kSearchStages; ++s) ps.stage(s, a[0], active, rem);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int p = ps.p;
        const double rinv = ps.r;
        const unsigned long long pm = 1ull << p;
        if (__builtin_amdgcn_inverse_ballot_w64(pm)) {
            t = k;
            dinv = rinv;
        }
        rem &= ~pm;
        const bool upd = __builtin_amdgcn_inverse_ballot_w64(rem);
        const double l = upd ? a[k] * rinv : 0.0;
        if (upd) a[k] = l;
        // column k + 1 first: the next pivot search starts from it and runs
        // in stages between groups of the remaining column updates
        int stage = 0;
#pragma unroll
        for (int j = k + 1; j < NP; ++j) {
            const double pj = readlane_d(a[j], p);
            a[j] = fma(-l, pj, a[j]);
            if (j == k + 1 || (j - k - 1) % kColsPerStage == 0) {
                if (stage < kSearchStages) ps.stage(stage, a[k + 1], upd, rem);
                ++stage;
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (k + 1 < NP) {
#pragma unroll
            for (int s = 0; s < kSearchStages; ++s)
                if (s >= stage) ps.stage(s, a[k + 1], upd, rem);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    // singular (zero pivot -> infinite reciprocal), NaN pivots, or an active
    // row that never became pivot
    const bool bad = active && (t < 0 || !(fabs(dinv) < INFINITY));
    const int dst = active && t >= 0 ? t : lane;
    pk = __builtin_amdgcn_ds_permute(dst << 2, lane);
#pragma unroll
    for (int j = 0; j < NP; ++j) a[j] = shfl_d(a[j], pk);
    dinv = shfl_d(dinv, pk);
    return !wave_any(bad);
}

// Solve with the factors of lu_factor (rows in pivot order).  b is first put
// in the same order; step k's value is read from lane k before that lane's
// own update at step k, so every lane updates unconditionally: lanes whose
// value was already taken only accumulate terms nobody reads.  The values
// taken (y_k forward, x_k backward) are kept in LDS (sv, 2 x 64 doubles of
// this wavefront), written by lane 0 eight at a time; lane k returns x_k.
template <int NP>
__device__ __forceinline__ double lu_solve(const double (&a)[NP], const double dinv, int pk,
                                           double b, double *sv) {
    asm volatile("" : "+v"(pk));
    const int lane = lane_id();
    b = shfl_d(b, pk);
#pragma unroll
    for (int k0 = 0; k0 < NP; k0 += 8) {
        double yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u;
            if (k < NP) {
                yv[u] = readlane_d(b, k);
                b = fma(-a[k], yv[u], b);
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < NP) sv[k0 + u] = yv[u];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    wave_sync();
    b = sv[lane < NP ? lane : 0];
#pragma unroll
    for (int k0 = NP - 1; k0 >= 0; k0 -= 8) {
        double xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 - u;
            if (k >= 0) {
                xv[u] = readlane_d(b * dinv, k);
                b = fma(-a[k], xv[u], b);
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 - u >= 0) sv[64 + k0 - u] = xv[u];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    wave_sync();
    const double x = lane < NP ? sv[64 + lane] : 0.0;
    wave_sync();   // the next call overwrites sv
    return x;
}

template <int NP>
__device__ __forceinline__ void build_matrix(const MechDev *__restrict__ Mp,
                                             double *__restrict__ J, double diag,
                                             double (&a)[NP]) {
    asm volatile("" ::: "memory");
    const MechDev &M = *Mp;
    int lane = lane_id();
    asm volatile("" : "+v"(lane));
    // n is made opaque here so that the per-column tests of the general case
    // are formed at each build: hoisted out of the step loop they held some
    // 160 scalar registers, spilled to vector lanes and read back each attempt
    int n = M.n;
    asm volatile("" : "+s"(n));
    const bool row_ok = lane < n;
    double *Jl = J + (row_ok ? lane : 0) * M.ldj;
    if (n == NP) {
        // every row and column is the mechanism's.  The diagonal is shifted in
        // place (x - diag, then negated, rounds as diag - x) and put back
        // after the reads, so the columns need no per-lane test; rows past
        // the matrix get zeros.
        double d = 0.0;
        if (row_ok) {
            d = Jl[lane];
            Jl[lane] = d - diag;
        }
        const double sc = row_ok ? -1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < NP; ++c) a[c] = Jl[c] * sc;
        if (row_ok) Jl[lane] = d;
        return;
    }
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        const double x = Jl[c < n ? c : 0];
        double v = (row_ok && c < n) ? -x : 0.0;
        if (c == lane) v += row_ok ? diag : 1.0;
        a[c] = v;
    }
}

// One Rodas4 attempt of size h from y (f0 = f(y), J in the wavefront's slot,
// which is given back once the iteration matrix is built).  Returns false
// when M is singular.  ynew and err are per lane.
template <int NP, bool LT, bool FO>
__device__ __forceinline__ bool rodas_attempt(const MechDev *__restrict__ M, double p, double y,
                                              double f0, double h, double *lds, JacSlot &js,
                                              double &ynew, double &err) {
    double a[NP];
    build_matrix<NP>(M, js.J, 1.0 / (kGamma * h), a);
    js.release();
    int pk;
    double dinv;
    const bool ok = lu_factor<NP>(a, dinv, pk);
    if (!ok) return false;
    const double hinv = 1.0 / h;
    double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0, u4 = 0.0, u5 = 0.0, ys = y;
#pragma unroll 1
    for (int s = 0; s < 6; ++s) {
        double rv = f0;
        if (s > 0) {
            ys = y;
            ys += kRodasA[s][0] * u0;
            ys += kRodasA[s][1] * u1;
            ys += kRodasA[s][2] * u2;
            ys += kRodasA[s][3] * u3;
            ys += kRodasA[s][4] * u4;
            rv = rhs_eval<NP, false, LT, FO>(M, p, ys, lds, nullptr);
            rv += (kRodasC[s][0] * hinv) * u0;
            rv += (kRodasC[s][1] * hinv) * u1;
            rv += (kRodasC[s][2] * hinv) * u2;
            rv += (kRodasC[s][3] * hinv) * u3;
            rv += (kRodasC[s][4] * hinv) * u4;
        }
        const double us = lu_solve<NP>(a, dinv, pk, rv, lds + M->off_sv);
        u0 = s == 0 ? us : u0;
        u1 = s == 1 ? us : u1;
        u2 = s == 2 ? us : u2;
        u3 = s == 3 ? us : u3;
        u4 = s == 4 ? us : u4;
        u5 = s == 5 ? us : u5;
    }
    ynew = ys + u5;
    err = u5;
    return true;
}

// Per-wavefront LDS: the small region (returned) and the Jacobian slot.
// Without LT (static launch: one wavefront per workgroup, records read from
// global memory) the workgroup's LDS is [Jacobian][small region].  With LT
// the whole workgroup first copies the species and reaction records into the
// shared table (once per launch), and the LDS is [table][locks][jslots
// Jacobian slots][one small region per wavefront]; jslots <= 0 or >= the
// wavefronts of the workgroup gives every wavefront a private slot.
template <bool LT>
__device__ __forceinline__ double *init_lds(const MechDev *Mp, int jslots, JacSlot &js) {
    const MechDev &M = *Mp;
    const int jd = M.n * M.ldj;
    js.jdoubles = jd;
    js.held = -1;
    double *lds;
    if (!LT) {
        js.J = lds_all;
        js.pool = nullptr;
        js.locks = nullptr;
        js.nslots = 0;
        lds = lds_all + jd;
    } else {
        const int wpb = (int)(blockDim.x >> 6), w = (int)(threadIdx.x >> 6);
        const int ns = M.N * SPC_STRIDE, nr = M.R * RXN_FIELDS;
        const auto *spc = gbl(M.spc);
        const double *rxd = reinterpret_cast<const double *>(M.rxn);
        for (int i = threadIdx.x; i < ns; i += blockDim.x) {
            const int k = i / SPC_STRIDE, f = i - k * SPC_STRIDE;
            lds_all[f * M.N + k] = spc[i];
        }
        for (int i = threadIdx.x; i < nr; i += blockDim.x)
            lds_all[ns + (i & (RXN_FIELDS - 1)) * M.R + (i / RXN_FIELDS)] = gbl(rxd)[i];
        int *locks = reinterpret_cast<int *>(lds_all + ns + nr);
        const bool priv = jslots <= 0 || jslots >= wpb;
        const int nslot = priv ? wpb : jslots;
        if (threadIdx.x < 2 * kLockDoubles) locks[threadIdx.x] = 0;
        double *pool = lds_all + ns + nr + kLockDoubles;
        js.pool = pool;
        js.locks = locks;
        js.nslots = priv ? 0 : nslot;
        js.J = priv ? pool + (size_t)w * jd : pool;
        __syncthreads();
        lds = pool + (size_t)nslot * jd + (size_t)w * M.lds_doubles;
    }
    if (lane_id() == 0) {
        lds[M.off_C + M.N] = 1.0;
        lds[M.off_g + M.N] = 1.0;
        lds[M.off_gi + M.N] = 1.0;
        lds[M.off_h + M.N] = 0.0;
    }
    wave_sync();
    return lds;
}

// -----------------------------------------------------------------------------
// Adaptive integration of one cell over [0, dt]
// -----------------------------------------------------------------------------
template <int NP, bool LT, bool FO>
__device__ __forceinline__ void integrate_cell(const MechDev *__restrict__ M, const IntParams &P,
                                               int64_t cell, double *lds, JacSlot &js) {
    const int lane = lane_id();
    const int n = M->n, N = M->N;
    const double dt = P.dt;
    const double p = P.p[cell];
    double y = 0.0;
    if (lane == 0) y = P.T[cell];
    else if (lane <= N) y = P.Y[(int64_t)(lane - 1) * P.ncells + cell];
    const double T0 = readlane_d(y, 0);
    const bool bad_in = wave_any(lane < n && !isfinite(y)) || !(T0 > 0.0) || !(p > 0.0) ||
                        !isfinite(p);
    if (bad_in) {
        if (lane == 0) {
            if (P.status) P.status[cell] = 4;
            if (P.ref_status && P.flags && P.flags[cell] == 1) *P.ref_status = 4;
            if (P.steps) { P.steps[2 * cell] = 0; P.steps[2 * cell + 1] = 0; }
            if (P.cost) P.cost[cell] = 0;
            atomicAdd(&P.stats[0], 1ull);
            atomicAdd(&P.stats[3], 1ull);
        }
        return;
    }
    double h = P.h ? P.h[cell] : 0.0;
    if (!(h > 0.0)) h = dt;
    h = uniform_d(h);
    double hnext = h, t = 0.0;
    int nacc = 0, nrej = 0, status = 0;
    bool rej_last = false;
    // jac: the Jacobian of y is in the slot (a pooled slot is given back
    // after each matrix build, so a rejected step assembles it again; the
    // same y gives the same bits)
    js.acquire();
    double f0 = rhs_eval<NP, true, LT, FO>(M, p, y, lds, js.J);
    bool jac = true;
    while (t < dt) {
        if (nacc + nrej >= P.max_steps) { status = 1; break; }
        bool last = false;
        if (h >= dt - t) { h = dt - t; last = true; }
        if (h < P.hmin_frac * dt) { status = 2; break; }
        if (!jac) {
            js.acquire();
            f0 = rhs_eval<NP, true, LT, FO>(M, p, y, lds, js.J);
        }
        double ynew = 0.0, ev = 0.0;
        const bool ok = rodas_attempt<NP, LT, FO>(M, p, y, f0, h, lds, js, ynew, ev);
        jac = !js.pooled();
        double e = 0.0;
        bool bad = !ok;
        if (ok) {
            const double sc = P.atol + P.rtol * fmax(fabs(y), fabs(ynew));
            const double r = lane < n ? fabs(ev) / sc : 0.0;
            bad = wave_any(r != r);
            if constexpr (NP <= 16) e = uniform_d(wave_max_row0(r));
            else e = uniform_d(wave_max(r));
        }
        if (!bad && e <= 1.0) {
            double fac = (e == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * rsqrt(sqrt(e))));
            if (rej_last) fac = fmin(fac, 1.0);
            y = ynew;
            t = last ? dt : t + h;
            ++nacc;
            hnext = uniform_d(h * fac);
            h = hnext;
            rej_last = false;
            if (t < dt) {
                js.acquire();
                f0 = rhs_eval<NP, true, LT, FO>(M, p, y, lds, js.J);
                jac = true;
            }
        } else {
            const double fac = bad ? 0.2 : fmax(0.2, 0.9 * rsqrt(sqrt(e)));
            h = uniform_d(h * fac);
            ++nrej;
            rej_last = true;
        }
    }
    js.release();
    if (status == 0 && wave_any(lane < n && !isfinite(y))) status = 3;
    if (lane == 0) P.T[cell] = y;
    else if (lane <= N) P.Y[(int64_t)(lane - 1) * P.ncells + cell] = y;
    if (lane == 0) {
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
}

// Static launch: workgroup i (one wavefront) integrates cell i, reading the
// records from global memory (an LDS copy per cell would cost more than it
// saves).
template <int NP, bool FO>
__global__ __launch_bounds__(64) void k_integrate_plain(const MechDev *__restrict__ M, IntParams P) {
    JacSlot js;
    double *lds = init_lds<false>(M, 0, js);
    const int64_t cell = blockIdx.x;
    if (P.flags && P.flags[cell] >= 2) return;
    integrate_cell<NP, false, FO>(M, P, cell, lds, js);
}

// Persistent wavefronts draw cells from NSEG segments of the heavy-first queue
// (segment x holds sorted positions x, x + NSEG, ...); wavefront w starts on
// segment w % NSEG and steals from the next segments once its own is drained.
// Every wavefront exits after NSEG consecutive empty segments.
// Workgroups of up to eight wavefronts (four from 56 unknowns on, where
// larger Jacobian slots leave room for fewer): with at most 256 registers per
// lane, two wavefronts share each SIMD.
__host__ __device__ constexpr int max_wpb(int NP) { return NP <= 54 ? 8 : 4; }

template <int NP, bool FO>
__global__ __launch_bounds__(64 * max_wpb(NP)) void k_integrate_queue(const MechDev *__restrict__ M,
                                                                      IntParams P) {
    JacSlot js;
    double *lds = init_lds<true>(M, P.jslots, js);
    const int wpb = (int)(blockDim.x >> 6);
    const int wave = (int)blockIdx.x * wpb + (int)(threadIdx.x >> 6);
    // P.block_static: wavefront w owns cells [w B, (w + 1) B) and integrates
    // them in index order (static partition, no balancing); otherwise cells
    // come from the work queue in chunks, segment by segment with stealing.
    const bool stat = P.block_static != 0;
    int64_t sb = 0, se = 0;
    if (stat) {
        const int64_t nw = (int64_t)gridDim.x * wpb;
        const int64_t B = (P.ncells + nw - 1) / nw;
        sb = wave * B;
        se = sb + B < P.ncells ? sb + B : P.ncells;
    }
    const int nact = stat ? 0 : uniform_i(*P.n_active);
    const int chunk = P.chunk;
    int seg = wave % NSEG;
    int first = 0, q = chunk;
    while (true) {
        int64_t cell;
        if (stat) {
            if (sb >= se) break;
            cell = sb++;
            if (P.flags && P.flags[cell] >= 2) continue;
        } else {
            if (q >= chunk || first + NSEG * q >= nact) {
                bool got = false;
                for (int probes = 0; probes < NSEG;) {
                    int c = 0;
                    if (lane_id() == 0) c = atomicAdd(&P.seg_ctr[seg], chunk);
                    c = uniform_i(__shfl(c, 0));
                    first = seg + NSEG * c;
                    if (first < nact) { got = true; break; }
                    seg = seg + 1 == NSEG ? 0 : seg + 1;
                    ++probes;
                }
                if (!got) break;
                q = 0;
            }
            cell = P.queue[first + NSEG * q];
            ++q;
        }
        integrate_cell<NP, true, FO>(M, P, cell, lds, js);
    }
}

// f(y) and J(y) per cell (kernel-level parity check of the rate/Jacobian code)
template <int NP>
__global__ __launch_bounds__(64) void k_eval_rhs_jac(const MechDev *__restrict__ M, IntParams P,
                                                     double *fout, double *Jout) {
    JacSlot js;
    double *lds = init_lds<true>(M, 0, js);
    const int64_t cell = blockIdx.x;
    const int lane = lane_id(), n = M->n, N = M->N;
    double y = 0.0;
    if (lane == 0) y = P.T[cell];
    else if (lane <= N) y = P.Y[(int64_t)(lane - 1) * P.ncells + cell];
    const double f = rhs_eval<NP, true, true, true>(M, P.p[cell], y, lds, js.J);
    if (fout && lane < n) fout[cell * n + lane] = f;
    if (Jout)
        for (int i = lane; i < n * n; i += 64)
            Jout[cell * n * n + i] = js.J[(i / n) * M->ldj + (i % n)];
}

template <int NP>
__global__ __launch_bounds__(64) void k_rodas_step(const MechDev *__restrict__ M, IntParams P,
                                                   double h, double *ynew_out, double *err_out) {
    JacSlot js;
    double *lds = init_lds<true>(M, 0, js);
    const int64_t cell = blockIdx.x;
    const int lane = lane_id(), n = M->n, N = M->N;
    double y = 0.0;
    if (lane == 0) y = P.T[cell];
    else if (lane <= N) y = P.Y[(int64_t)(lane - 1) * P.ncells + cell];
    const double p = P.p[cell];
    const double f0 = rhs_eval<NP, true, true, true>(M, p, y, lds, js.J);
    double ynew = 0.0, err = 0.0;
    const bool ok = rodas_attempt<NP, true, true>(M, p, y, f0, h, lds, js, ynew, err);
    if (!ok) { ynew = NAN; err = NAN; }
    if (lane < n) {
        ynew_out[cell * n + lane] = ynew;
        err_out[cell * n + lane] = err;
    }
}

// -----------------------------------------------------------------------------
// host-side launchers, one instantiation per padded size
// -----------------------------------------------------------------------------
#define CHEM_NP_LIST(X) X(12) X(16) X(24) X(32) X(40) X(48) X(54) X(56) X(64)

// The host side is built as two translation units that compile in parallel:
// part 0 (this file) instantiates the kernels for mechanisms with plain
// kinetics and holds the dispatch; part 1 (integrate_fo.hip, which includes
// this file) instantiates the fall-off / PLOG kernels and the single-call
// test kernels.
#ifndef CHEM_INTEGRATE_PART
#define CHEM_INTEGRATE_PART 0
#endif

int pick_np(int n);
int wave_kernel_wpb(const MechDev &M);
hipError_t launch_integrate_fo(int NP, const MechDev &M, const MechDev *Md, const IntParams &P,
                               int schedule, int grid, hipStream_t s);

#if CHEM_INTEGRATE_PART == 0
int pick_np(int n) {
#define PICK(v) if (n <= v) return v;
    CHEM_NP_LIST(PICK)
#undef PICK
    return -1;
}

#endif

// Queue-kernel workgroup shape: the most wavefronts (up to max_wpb) whose
// small regions fit in one CU's LDS next to the record table together with
// Jacobian slots for at least half of them, and as many slots as then fit
// (one per wavefront at most, which makes every slot private).  For the
// 53-species mechanism: 8 wavefronts, 4 slots (27 KB of records, 8 x 4 KB,
// 4 x 23 KB).
static constexpr size_t kLdsCap = 160 * 1024;
struct WaveLayout {
    int wpb, jslots;
};
static WaveLayout wave_layout(const MechDev &M) {
    const int np = pick_np(M.n);
    if (np < 0) return {0, 0};
    const size_t cap = kLdsCap / sizeof(double);
    const size_t head = (size_t)table_doubles(M) + kLockDoubles, jd = (size_t)M.n * M.ldj;
    for (int w = max_wpb(np); w >= 1; w /= 2) {
        const size_t base = head + (size_t)w * M.lds_doubles;
        if (base > cap) continue;
        size_t js = (cap - base) / jd;
        if (js < (size_t)(w + 1) / 2) continue;
        if (js > (size_t)w) js = (size_t)w;
        return {w, (int)js};
    }
    return {0, 0};
}
#if CHEM_INTEGRATE_PART == 0
int wave_kernel_wpb(const MechDev &M) { return wave_layout(M).wpb; }
#endif
static size_t lds_bytes(const MechDev &M, const WaveLayout &L) {
    return sizeof(double) * ((size_t)table_doubles(M) + kLockDoubles +
                             (size_t)L.jslots * M.n * M.ldj + (size_t)L.wpb * M.lds_doubles);
}

// Host launchers: M is the host copy (sizes), Md the device copy the kernels read.

// Fall-off reactions get their own instantiation (FO), so that mechanisms
// without them run code with no trace of the fall-off branch.
template <int NP, bool FO>
static hipError_t launch_integrate_np(const MechDev &M, const MechDev *Md, const IntParams &P,
                                      int schedule, int grid, hipStream_t s) {
    if (schedule == 0) {
        const size_t sh1 = sizeof(double) * ((size_t)M.n * M.ldj + (size_t)M.lds_doubles);
        hipFuncSetAttribute((const void *)k_integrate_plain<NP, FO>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh1);
        hipLaunchKernelGGL((k_integrate_plain<NP, FO>), dim3((unsigned)P.ncells), dim3(64), sh1, s, Md, P);
    } else {
        const WaveLayout L = wave_layout(M);
        if (L.wpb == 0 || L.jslots > 2 * kLockDoubles) return hipErrorInvalidConfiguration;
        const size_t sh = lds_bytes(M, L);
        IntParams Q = P;
        Q.jslots = L.jslots;
        hipFuncSetAttribute((const void *)k_integrate_queue<NP, FO>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        hipLaunchKernelGGL((k_integrate_queue<NP, FO>), dim3((unsigned)grid), dim3(64 * L.wpb), sh, s, Md, Q);
    }
    return hipGetLastError();
}

#if CHEM_INTEGRATE_PART == 0
hipError_t launch_integrate(int NP, const MechDev &M, const MechDev *Md, const IntParams &P,
                            int schedule, int grid, hipStream_t s) {
    if (M.has_fo) return launch_integrate_fo(NP, M, Md, P, schedule, grid, s);
    switch (NP) {
#define CASE(v) case v: return launch_integrate_np<v, false>(M, Md, P, schedule, grid, s);
        CHEM_NP_LIST(CASE)
#undef CASE
    }
    return hipErrorInvalidValue;
}

// Workgroups of the queue kernel that fit on one CU.
int queue_occupancy(int NP, const MechDev &M) {
    int blocks = 0;
    const WaveLayout L = wave_layout(M);
    if (L.wpb == 0) return 0;
    const size_t sh = lds_bytes(M, L);
    const int wpb = L.wpb;
    switch (NP) {
#define CASE(v)                                                                                 \
    case v:                                                                                     \
        hipFuncSetAttribute((const void *)k_integrate_queue<v, false>,                          \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);               \
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_integrate_queue<v, false>, 64 * wpb, sh); \
        break;
        CHEM_NP_LIST(CASE)
#undef CASE
    }
    return blocks;
}

#else
hipError_t launch_integrate_fo(int NP, const MechDev &M, const MechDev *Md, const IntParams &P,
                               int schedule, int grid, hipStream_t s) {
    switch (NP) {
#define CASE(v) case v: return launch_integrate_np<v, true>(M, Md, P, schedule, grid, s);
        CHEM_NP_LIST(CASE)
#undef CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_eval_rhs_jac(int NP, const MechDev &M, const MechDev *Md, const IntParams &P,
                               double *f, double *J, hipStream_t s) {
    const size_t sh = lds_bytes(M, WaveLayout{1, 1});
    switch (NP) {
#define CASE(v)                                                                                 \
    case v:                                                                                     \
        hipFuncSetAttribute((const void *)k_eval_rhs_jac<v>,                                    \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);               \
        hipLaunchKernelGGL(k_eval_rhs_jac<v>, dim3((unsigned)P.ncells), dim3(64), sh, s, Md, P, f, J); \
        return hipGetLastError();
        CHEM_NP_LIST(CASE)
#undef CASE
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rodas_step(int NP, const MechDev &M, const MechDev *Md, const IntParams &P,
                             double h, double *ynew, double *err, hipStream_t s) {
    const size_t sh = lds_bytes(M, WaveLayout{1, 1});
    switch (NP) {
#define CASE(v)                                                                                 \
    case v:                                                                                     \
        hipFuncSetAttribute((const void *)k_rodas_step<v>,                                      \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);               \
        hipLaunchKernelGGL(k_rodas_step<v>, dim3((unsigned)P.ncells), dim3(64), sh, s, Md, P, h, ynew, err); \
        return hipGetLastError();
        CHEM_NP_LIST(CASE)
#undef CASE
    }
    return hipErrorInvalidValue;
}
#endif

}  // namespace chem
