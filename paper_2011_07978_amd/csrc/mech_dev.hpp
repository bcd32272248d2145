// Device-resident mechanism tables and per-call parameters shared between the
// host API and the kernels.  All pointers are device pointers.
#pragma once
#include <stdint.h>

namespace chem {

constexpr double RU_J = 8.314462618;   // J/(mol K), for Ea/(R T)
constexpr double RU_ERG = 8.314462618e7;  // erg/(mol K)
constexpr double P_ATM = 1.01325e6;    // dyn/cm^2
constexpr double kLnPatmRu = -4.4074185890025276;   // ln(P_ATM / RU_ERG)
constexpr int NSEG = 8;                // work-queue segments (one per XCD)
constexpr int NBUCKET = 32;            // heavy-first cost buckets

// Species record (18 doubles): a1..a7, a2/2, a3/3, a4/4, a5/5, a3/2, a4/3,
// a5/4, W, 1/W, then two unused slots.
constexpr int SPC_STRIDE = 18;

// Reaction record (64 bytes).  idx[0] = r0 | r1 << 16, idx[1] = p0 | p1 << 16,
// idx[2] = p2 | tb << 16, idx[3] = (sum_nu + 8) | es0 << 8 | es1 << 16 | es2 << 24.
// Bit 15 of tb (TB_FALLOFF) marks a fall-off reaction, whose parameters are
// in MechDev::fo at the reaction's slot; bit 14 (TB_PLOG) a reaction with
// tabulated pressure dependence, whose table is in MechDev::plog.
// Missing slots hold the sentinel species N.  tb = 0: no third body;
// tb = 1: third body with up to three listed efficiencies stored inline
// (alpha - 1 in eff[], species es0..es2, unused ones eff = 0, es = N);
// tb >= 2: third body whose efficiencies are in the list tb_ptr[tb - 2].
struct RxnRec {
    double lnA, b, EaR;
    double eff[3];
    int idx[4];
};
constexpr int TB_NONE = 0, TB_INLINE = 1, TB_LIST0 = 2;
constexpr int TB_FALLOFF = 0x8000, TB_PLOG = 0x4000, TB_CODE = 0x3fff;

// Fall-off parameters of one reaction slot (8 doubles): ln A0, b0, Ea0 / R,
// Troe a, T3, T1, T2 (<= 0: no T2 term), form (1 Lindemann, 2 Troe).
constexpr int FO_STRIDE = 8;

// Fall-off factor (Lindemann, Troe) and its derivatives.  The rate constant is
// k_inf G with Pr = k0 [M] / k_inf and G = Pr / (1 + Pr) F; F = 1 (Lindemann)
// or Troe's broadening factor:
//   Fcent = (1 - a) exp(-T/T3) + a exp(-T/T1) + exp(-T2/T),
//   c = -0.4 - 0.67 log10 Fcent, n = 0.75 - 1.27 log10 Fcent, d = 0.14,
//   f1 = x / (n - d x), x = log10 Pr + c,  log10 F = log10 Fcent / (1 + f1^2).
// dGdM = dG/d[M]; dlnGdT = d ln G / dT at fixed [M] (dlnkinf = d ln k_inf / dT).
__device__ __forceinline__ void falloff_eval(const double *__restrict__ f, double T, double invT,
                                             double lnT, double kinf, double dlnkinf, double M,
                                             double &G, double &dGdM, double &dlnGdT) {
    const double k0 = exp(f[0] + f[1] * lnT - f[2] * invT);
    const double r = k0 / kinf;
    const double Pr = r * M;
    const double inv1p = 1.0 / (1.0 + Pr);
    double F = 1.0, S = 0.0, dlnF_dT = 0.0;
    if (f[7] == 2.0) {
        const double e3 = exp(-T / f[4]), e1 = exp(-T / f[5]);
        const double e2 = f[6] > 0.0 ? exp(-f[6] * invT) : 0.0;
        const double Fc = (1.0 - f[3]) * e3 + f[3] * e1 + e2;
        const double dFc = -(1.0 - f[3]) / f[4] * e3 - f[3] / f[5] * e1 + f[6] * invT * invT * e2;
        const double ln10 = 2.302585092994045684;
        const double lFc = log(Fc) / ln10;
        const double c = -0.4 - 0.67 * lFc, n = 0.75 - 1.27 * lFc;
        const double x = log(Pr) / ln10 + c;
        const double den = n - 0.14 * x;
        const double f1 = x / den;
        const double q = 1.0 / (1.0 + f1 * f1);
        F = exp(ln10 * lFc * q);
        S = -2.0 * lFc * f1 * q * q * n / (den * den);                 // d ln F / d ln Pr
        const double df1_dlFc = (1.27 * x - 0.67 * n) / (den * den);
        const double dlF_dlFc = q - 2.0 * lFc * f1 * q * q * df1_dlFc;
        dlnF_dT = dlF_dlFc * dFc / Fc;                                 // at fixed Pr
    }
    G = Pr * inv1p * F;
    dGdM = F * inv1p * (inv1p + S) * r;
    const double dlnk0 = f[1] * invT + f[2] * invT * invT;
    dlnGdT = (inv1p + S) * (dlnk0 - dlnkinf) + dlnF_dT;
}

// Tabulated pressure dependence (PLOG) of one reaction slot (PLOG_STRIDE
// doubles): the number of entries (2..8), then per entry ln p_i (p in
// dyn/cm^2, increasing), ln A_i, b_i, Ea_i / R.
constexpr int PLOG_STRIDE = 33;

// Arrhenius parameters of a PLOG reaction at the cell's pressure: ln k is
// linear in ln p between the two tabulated pressures around p, and equals the
// end entry's outside the table.  At a fixed p this is the Arrhenius form
// whose ln A, b and Ea/R are interpolated with the same weight.
__device__ __forceinline__ void plog_arrhenius(const double *__restrict__ t, double lnp, double &lnA,
                                               double &b, double &EaR) {
    const int cnt = (int)t[0];
    const double *e = t + 1;
    int i = 0;
    while (i + 2 < cnt && lnp >= e[4 * (i + 1)]) ++i;
    const double *lo = e + 4 * i, *hi = lo + 4;
    const double w = (lnp - lo[0]) / (hi[0] - lo[0]);
    if (w <= 0.0) {
        lnA = lo[1]; b = lo[2]; EaR = lo[3];
    } else if (w >= 1.0) {
        lnA = hi[1]; b = hi[2]; EaR = hi[3];
    } else {
        lnA = lo[1] + w * (hi[1] - lo[1]);
        b = lo[2] + w * (hi[2] - lo[2]);
        EaR = lo[3] + w * (hi[3] - lo[3]);
    }
}

// Loads through this cast are global-memory loads (not flat), so they do not
// share a wait counter with LDS traffic.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gbl(const T *p) {
    return (const __attribute__((address_space(1))) T *)p;
}

struct MechDev {
    int N, R, n;            // species, reactions, unknowns n = N + 1
    int ldj;                // LDS row stride of the Jacobian (odd)
    const double *spc;      // [N][SPC_STRIDE] species records
    const RxnRec *rxn;      // [R]
    // species, structure of arrays
    const double *nasa_t;   // [14][N]: a1..a7, a2/2, a3/3, a4/4, a5/5, a3/2, a4/3, a5/4
    const double *W, *invW; // [N]
    const int *tb_ptr;      // efficiency lists of third-body reactions with > 3 entries
    const int *eff_sp;
    const double *eff_am1;  // alpha - 1
    const double *fo;       // [R][FO_STRIDE] fall-off parameters by reaction slot
    const double *plog;     // [R][PLOG_STRIDE] PLOG tables by reaction slot
    int has_fo;             // any fall-off or PLOG reaction
    // per-wavefront LDS region (offsets in doubles); the Jacobian (n rows of
    // stride ldj) has a slot of its own
    int off_q, off_C, off_g, off_gi, off_h, off_e, off_cp, off_tb, off_sv, lds_doubles;
};

struct IntParams {
    double rtol, atol, hmin_frac, dt;
    int max_steps;
    int64_t ncells;
    double *T;
    const double *p;
    double *Y;
    double *h;              // nullable
    uint32_t *cost;         // nullable
    uint8_t *status;        // nullable
    int32_t *steps;         // nullable [2*ncells]
    const uint8_t *flags;   // nullable (plain schedule skips flags 2 and 3)
    // queue schedule
    const int *queue;       // sorted active cells
    int *seg_ctr;           // [NSEG] consumed items per segment
    const int *n_active;    // device scalar
    int chunk;
    int block_static;       // persistent launch, contiguous block of cells per slot
    unsigned long long *stats;  // [8] device counters
    int *ref_status;        // nullable: receives the status of the reference cell (flag 1)
    int jslots;             // Jacobian slots of a queue workgroup (set by the launcher)
};

}  // namespace chem
