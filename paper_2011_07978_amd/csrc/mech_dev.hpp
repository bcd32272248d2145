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
// a5/4, W, 1/W, then two unused slots.
constexpr int SPC_STRIDE = 18;

// Reaction record (64 bytes).  idx[0] = r0 | r1 << 16, idx[1] = p0 | p1 << 16,
// idx[2] = p2 | tb << 16, idx[3] = (sum_nu + 8) | es0 << 8 | es1 << 16 | es2 << 24.
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
    // LDS layout (offsets in doubles)
    int off_J, off_q, off_C, off_g, off_h, off_e, off_cp, off_tb, off_sv, lds_doubles;
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
};

}  // namespace chem
