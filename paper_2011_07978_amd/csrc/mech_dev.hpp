// Device-resident mechanism tables and per-call parameters shared between the
// host API and the kernels.  All pointers are device pointers.
#pragma once
#include <stdint.h>

namespace chem {

constexpr double RU_J = 8.314462618;   // J/(mol K), for Ea/(R T)
constexpr double RU_ERG = 8.314462618e7;  // erg/(mol K)
constexpr double P_ATM = 1.01325e6;    // dyn/cm^2
constexpr int NSEG = 8;                // work-queue segments (one per XCD)
constexpr int NBUCKET = 32;            // heavy-first cost buckets

// Species record (18 doubles): a1..a7, a2/2, a3/3, a4/4, a5/5, a3/2, a4/3,
// a5/4, W, 1/W, then the species' CSR range (two ints) and a pad.
// Reaction record: ln A, b, Ea/R, pad, then the index word.
constexpr int SPC_STRIDE = 18;
struct RxnRec {
    double lnA, b, EaR, pad;
    int4 idx;               // (r0 | r1 << 16, p0 | p1 << 16, p2 | tb << 16, sum_nu)
};

struct MechDev {
    int N, R, n;            // species, reactions, unknowns n = N + 1
    int ldj;                // LDS row stride of the Jacobian (odd)
    const double *spc;      // [N][SPC_STRIDE] species records
    const RxnRec *rxn;      // [R]
    // species, structure of arrays
    const double *nasa_t;   // [14][N]: a1..a7, a2/2, a3/3, a4/4, a5/5, a3/2, a4/3, a5/4
    const double *W, *invW; // [N]
    const int *sp_ptr;      // [N+1] species -> reactions (CSR)
    const int *sp_ent;      // entries: (reaction << 3) | (nu + 4)
    const int *tb_ptr;      // [ntb+1] into eff arrays
    const int *eff_sp;      // [neff]
    const double *eff_am1;  // [neff] alpha - 1
    // LDS layout (offsets in doubles)
    int off_J, off_q, off_C, off_g, off_h, off_e, off_cp, off_tb, lds_doubles;
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
    const uint8_t *flags;   // nullable (plain schedule skips flag 2)
    // queue schedule
    const int *queue;       // sorted active cells
    int *seg_ctr;           // [NSEG] consumed items per segment
    const int *n_active;    // device scalar
    int chunk;
    unsigned long long *stats;  // [8] device counters
};

}  // namespace chem
