/*
 * libchem — per-cell stiff chemistry integration on one MI355X (gfx950).
 *
 * The paper (DLBFoam, arXiv 2011.07978) splits a reacting-flow step so that
 * every finite-volume cell's chemistry becomes an independent stiff reactor
 * ODE dPhi/dt = f(Phi) over one flow time step (Sec. 1, Sec. 2.1).  It balances
 * these per-cell problems across MPI ranks (Sec. 2.2, Algorithm 1) and lets
 * cells whose mixture fraction (and optionally temperature) lies within
 * tolerance of a reference cell reuse the reference's solution (Sec. 2.3).
 * This library is that hot path on one GPU: reference mapping, an on-device
 * work queue ordered heavy-first by the previous call's per-cell cost (the
 * analogue of the paper's CPU-time load measure), and FP64 Rosenbrock (Rodas4)
 * integration with an analytic Jacobian and batched LU, all in hand-written
 * HIP kernels.
 *
 * Conventions for every entry point:
 *  - Array arguments marked "device" are device pointers (HIP global memory,
 *    FP64 unless stated), contiguous, owned by the caller, and must stay valid
 *    until the work enqueued on the context's stream has finished.
 *  - Species mass fractions are species-major: Y[k * n_cells + i] is species k
 *    of cell i.
 *  - Work is enqueued asynchronously on the context's HIP stream.  A non-NULL
 *    host `stats` argument makes the call wait for its own work.
 *  - Units: CGS.  T in K, p in dyn/cm^2, dt and h in s, molar masses in g/mol,
 *    pre-exponential factors in (cm^3/mol)^(order-1)/s, Ea in J/mol.
 *  - Return value: 0 success; negative CHEM_E_* error (nothing was written);
 *    for chem_integrate a positive k means k cells failed and their status
 *    bytes say why.  chem_last_error() gives a message for the last failure.
 *  - One context per host thread; calls on one context are not re-entrant.
 */
#ifndef LIBCHEM_CHEM_H
#define LIBCHEM_CHEM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CHEM_OK = 0,
    CHEM_E_INVALID_ARG = -1,
    CHEM_E_NO_MECHANISM = -2,
    CHEM_E_HIP = -3,
    CHEM_E_OOM = -4,
    CHEM_E_UNIMPL = -5,
    CHEM_E_CAPTURE_UNSAFE = -6,
    CHEM_E_BAD_MECHANISM = -7
};

/* per-cell status bytes written by chem_integrate */
enum {
    CHEM_CELL_OK = 0,
    CHEM_CELL_MAX_STEPS = 1,   /* attempted-step limit reached */
    CHEM_CELL_H_UNDERFLOW = 2, /* step fell below hmin_frac * dt */
    CHEM_CELL_NONFINITE = 3,   /* accepted state not finite */
    CHEM_CELL_BAD_INPUT = 4,   /* T <= 0, p <= 0 or non-finite input; cell untouched */
    CHEM_CELL_MAPPED = 5,      /* cell took the reference's increment */
    CHEM_CELL_SURROGATE = 6,   /* cell was advanced by the learned surrogate */
    CHEM_CELL_REF_FAILED = 7   /* mapped cell left unchanged: the reference cell's own
                                  integration failed, so there is no increment to copy */
};

/* routing flags (uint8 per cell) */
enum {
    CHEM_FLAG_SOLVE = 0,       /* integrate (the surrogate may take it) */
    CHEM_FLAG_REFERENCE = 1,   /* reference cell of the mapping: always integrated */
    CHEM_FLAG_MAPPED = 2,      /* takes the reference's increment */
    CHEM_FLAG_SURROGATE = 3    /* advanced by the surrogate; not integrated */
};

/* scheduling of cells onto wavefronts */
enum {
    CHEM_SCHED_PLAIN = 0,  /* one static launch, cell i on workgroup i */
    CHEM_SCHED_QUEUE = 1,  /* persistent kernel, atomic work queue + stealing */
    CHEM_SCHED_BLOCKS = 2  /* persistent kernel, slot s owns one contiguous block of
                              cells (static partition, the unbalanced baseline of
                              the load-balancing benchmark, Sec. 3) */
};

typedef struct chem_ctx chem_ctx;

/* Mechanism description (host arrays, deep-copied by chem_set_mechanism).
 * Reactions are reversible mass-action reactions with 1-2 reactant and 1-3
 * product slots (-1 = unused slot; a species may fill two slots); reverse rate
 * constants follow from equilibrium constants of the NASA-7 style single-range
 * thermodynamics.  Third-body reactions multiply the rate by
 * [M] = sum_k alpha_k C_k with alpha_k = 1 unless listed in eff_*.
 * Fall-off reactions (third-body reactions with falloff[j] = 1 Lindemann or
 * 2 Troe) use instead the rate constant k_inf G: A, b, Ea give the
 * high-pressure limit k_inf, falloff_params[7j..7j+6] = A0, b0, Ea0 (J/mol)
 * the low-pressure limit k0, then Troe's a, T3, T1, T2 (K; T2 <= 0: no T2
 * term), and with Pr = k0 [M] / k_inf, G = Pr / (1 + Pr) F, F = 1 (Lindemann)
 * or log10 F = log10 Fcent / (1 + f1^2), f1 = x / (n - 0.14 x),
 * x = log10 Pr - 0.4 - 0.67 log10 Fcent, n = 0.75 - 1.27 log10 Fcent,
 * Fcent = (1 - a) exp(-T/T3) + a exp(-T/T1) + exp(-T2/T) (Troe).  The
 * reverse rate carries the same G.
 * Reactions with tabulated pressure dependence (PLOG; plog_count[j] = 2..8,
 * reactions without a third body) ignore A, b, Ea: plog_params[32j + 4i ..]
 * = p_i (dyn/cm^2, strictly increasing), A_i, b_i, Ea_i (J/mol) give rate
 * expressions k_i(T) at the pressures p_i, and at the cell's pressure p,
 * ln k = ln k_i + (ln p - ln p_i) / (ln p_i+1 - ln p_i) (ln k_i+1 - ln k_i)
 * for p_i <= p < p_i+1, k_1 below p_1 and k_last from p_last on (the usual
 * PLOG form of kinetics input; the paper's chemistry model, Sec. 2.1, takes
 * its rates from such input). */
typedef struct {
    int32_t n_elements, n_species, n_reactions;
    const double *elem_mass;     /* [E] g/mol */
    const int32_t *composition;  /* [N*E] atom counts, row = species */
    const double *W;             /* [N] molar masses, must equal sum_e a_ek m_e */
    const double *nasa;          /* [N*7] a1..a7: cp/R = a1 + a2 T + ... + a5 T^4,
                                    H/RT adds a6/T, S/R adds a7 */
    const int32_t *reactants;    /* [R*2] species indices, -1 padded */
    const int32_t *products;     /* [R*3] species indices, -1 padded */
    const double *A;             /* [R] pre-exponential factor (> 0) */
    const double *b;             /* [R] temperature exponent */
    const double *Ea;            /* [R] activation energy J/mol */
    const int32_t *third_body;   /* [R] 0/1 */
    int32_t n_eff;               /* number of non-default efficiencies */
    const int32_t *eff_reaction; /* [n_eff] reaction index (must be third-body) */
    const int32_t *eff_species;  /* [n_eff] species index */
    const double *eff_value;     /* [n_eff] efficiency alpha */
    const int32_t *falloff;      /* [R] nullable: 0 none, 1 Lindemann, 2 Troe */
    const double *falloff_params;/* [R*7] nullable (required with falloff) */
    const int32_t *plog_count;   /* [R] nullable: 0, or 2..8 tabulated pressures */
    const double *plog_params;   /* [R*32] nullable (required with plog_count) */
} chem_mech_desc;

typedef struct {
    double rtol;          /* relative tolerance (default 1e-8) */
    double atol;          /* absolute tolerance (default 1e-12) */
    int32_t max_steps;    /* attempted-step limit per cell and call (default 100000) */
    double hmin_frac;     /* fail when h < hmin_frac * dt (default 1e-14) */
    int32_t schedule;     /* CHEM_SCHED_PLAIN, _QUEUE or _BLOCKS (default QUEUE) */
    int32_t queue_chunk;  /* cells per atomic grab; 0 = tuned value (default 0) */
    int32_t slots_per_cu; /* persistent workgroups per CU; 0 = tuned value */
    int32_t order_by_cost;/* 1: heavy-first queue order from `cost` (default 1) */
} chem_options;

/* Reference-mapping parameters (Sec. 2.3).  Mixture fraction
 * Z = (beta - beta_ox) / (beta_fuel - beta_ox), beta(Y) = sum_k w_k Y_k with
 * w_k = sum_e c_e a_ek m_e / W_k and c_e = (Z_e(Y_fuel) - Z_e(Y_ox)) / m_e,
 * Z_e(Y) = sum_k a_ek m_e Y_k / W_k (a Bilger-type coupling of all elements). */
typedef struct {
    double Z_tol;          /* cells with Z < Z_tol are candidates (strict) */
    double T_tol;          /* and, if use_T, |T - T_ref| < T_tol (strict) */
    int32_t use_T;
    const double *Y_fuel;  /* host [N] fuel-stream mass fractions */
    const double *Y_ox;    /* host [N] oxidiser-stream mass fractions */
} chem_map_params;

typedef struct {
    int64_t cells_integrated; /* cells that ran the Rosenbrock solver */
    int64_t cells_mapped;     /* cells that took the reference increment */
    int64_t cells_failed;     /* status not OK/MAPPED */
    int64_t steps_accepted;
    int64_t steps_rejected;
    int32_t max_cell_steps;   /* largest accepted+rejected count of any cell */
    int32_t reserved;
    double ms_total;          /* GPU time of the whole call (HIP events on its stream) */
    double ms_integrate;      /* GPU time of the integration kernel alone */
    int64_t cells_surrogate;  /* cells the surrogate advanced (gate passed) */
    int64_t cells_rejected;   /* cells the gate sent back to the Rosenbrock solver */
    double ms_surrogate;      /* GPU time of the surrogate pass (inference + gate) */
} chem_stats;

/* Learned surrogate (not part of the paper; its relatives there are the
 * tabulation methods ISAT/TDAC of Sec. 1 and Sec. 5).  A multilayer
 * perceptron advances a cell by dt:
 *   features x = (ln T, ln p, Y_1..Y_N, ln dt), normalised with the training
 *     set's mean and standard deviation, zero-padded to 64;
 *   four hidden layers of 256 with GELU (erf form); output 64, of which the
 *     first N+1 are the normalised increments in an inverse hyperbolic-sine
 *     scale: t = o sd_o + mu_o, dY_k = 1e-12 sinh(t_k), dT = 1e-6 K sinh(t_N)
 *     (error relative to each increment's size across its many decades).
 * Weights and activations are bfloat16 (round to nearest even), products
 * accumulate in FP32 on the matrix cores, biases and GELU in FP32.
 * Parameter blob (float32, chem_surrogate_param_count() entries): layer by
 * layer W_l [out x in] row-major then b_l [out] (dims 64-256-256-256-256-64),
 * then six blocks of 64: mu_x, sd_x (feature normalisation), mu_o, sd_o
 * (output de-normalisation), xmin, xmax (training range of the raw features).
 * The predicted state is clipped at zero, Y1 = max(Y + dY, 0), and element
 * conservation restored by the correction smallest in the metric weighted by
 * 1/Y1: Y' = Y1 - Y1 (E^T lam), (E diag(Y1) E^T) lam = E (Y1 - Y),
 * E_ek = a_ek / W_k (species at zero stay there; corrections are proportional
 * to each species' mass fraction).  T' solves h(T', Y') = h(T, Y).  The gate
 * (chem_gate_params) sends a cell back to the Rosenbrock solver unless
 * T <= T_max, every raw feature lies in [xmin - margin*(xmax - xmin), xmax +
 * margin*(xmax - xmin)], |dT| <= max_dT, E diag(Y1) E^T is invertible, every
 * Y'_k >= y_min and |T + dT - T'| <= tau_T.
 * Available for N <= 61 species and E <= 8 elements with E E^T invertible
 * (otherwise the surrogate entry points return CHEM_E_UNIMPL). */
typedef struct {
    int32_t epochs;       /* passes over the samples (default 8) */
    int32_t batch;        /* rows per Adam step: multiple of 64, <= 65536 (default 4096) */
    double lr_max;        /* cosine learning-rate schedule from lr_max ... (default 2e-3) */
    double lr_min;        /* ... to lr_min at the last step (default 2e-5) */
    uint64_t seed;        /* weight initialisation and shuffling (default 0) */
    int32_t verbose;      /* 1: loss of every epoch on stderr */
} chem_train_params;

typedef struct {
    double tau_T;         /* K (default 0.5) */
    double y_min;         /* (default -1e-10) */
    double margin;        /* fraction of each feature's training span (default 0.01: a
                             species the conservation step clipped to zero sits
                             just below the training minimum, and must not send
                             the cell back to the solver next step) */
    double max_dT;        /* K: cells whose predicted |dT| exceeds it go to the
                             solver (default 1: the surrogate takes slowly
                             changing cells; igniting cells stay on the FP64
                             path) */
    double T_max;         /* K: cells hotter than this go to the solver (default
                             1000: above it chemistry is fast, and a relative
                             error of the network on the large increments
                             exceeds the 1 K accuracy target) */
} chem_gate_params;

/* Create a context on HIP device `hip_device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  *out receives the
 * context, owned by the caller until chem_destroy. */
int chem_create(chem_ctx **out, int hip_device, void *hip_stream);
void chem_destroy(chem_ctx *ctx);
int chem_set_stream(chem_ctx *ctx, void *hip_stream);
const char *chem_last_error(const chem_ctx *ctx);

/* Validate and upload a mechanism (the per-cell reactor the paper leaves to
 * the standard chemistry model, program summary and Sec. 2.1).  Rejects:
 * N < 1 or N > 160, R < 1 or R > 4096, element-unbalanced reactions (integer
 * check), W inconsistent with the composition, cp <= 0 anywhere on
 * [200, 10000] K, A <= 0, indices out of range, efficiencies on
 * non-third-body reactions (CHEM_E_BAD_MECHANISM).  Synchronous. */
int chem_set_mechanism(chem_ctx *ctx, const chem_mech_desc *m);
/* The validation of chem_set_mechanism alone, on the host: no context and
 * no device are needed, nothing is uploaded.  Returns CHEM_OK, or
 * CHEM_E_BAD_MECHANISM / CHEM_E_INVALID_ARG with the reason written to msg
 * (host, nullable, msg_len bytes including the terminating zero; an empty
 * string on success). */
int chem_validate_mechanism(const chem_mech_desc *m, char *msg, int32_t msg_len);
/* Largest species count the integrator handles: 137 (138 unknowns).  Up to
 * 63 species a wavefront integrates a cell with its iteration matrix in
 * registers; above that a workgroup of four wavefronts integrates a cell with
 * the n x n matrix in LDS (n^2 doubles plus ~9 n, which must fit in one CU's
 * LDS: chem_set_mechanism's integrator calls return CHEM_E_UNIMPL when it does
 * not on the device at hand) and a blocked LU on the FP64 matrix cores. */
int chem_max_species(void);

int chem_set_options(chem_ctx *ctx, const chem_options *o);
int chem_get_options(const chem_ctx *ctx, chem_options *o);
void chem_default_options(chem_options *o);

/* Number of cells integrated at once by the persistent launches
 * (CHEM_SCHED_QUEUE and CHEM_SCHED_BLOCKS) for the current mechanism and
 * options, before capping by the cell count: CUs x workgroups per CU x cells
 * per workgroup (wavefronts per workgroup for up to 63 species, 1 above).
 * Under CHEM_SCHED_BLOCKS slot s owns cells [s B, (s + 1) B) with
 * B = ceil(n_cells / min(slots, n_cells)).  These slots play the role of the processes of the paper's load-balancing
 * benchmark (Sec. 3).  Requires a mechanism (CHEM_E_INVALID_ARG otherwise). */
int chem_query_slots(const chem_ctx *ctx, int64_t *slots);

/* Preallocate workspace for up to max_cells cells so that later calls with
 * n_cells <= max_cells allocate nothing (required before stream capture). */
int chem_reserve(chem_ctx *ctx, int64_t max_cells);

/* Reference mapping, Sec. 2.3: computes Z for every cell, picks the first cell
 * (lowest index) with Z < Z_tol as reference and flags every later candidate
 * that also passes the optional temperature test.
 *   T [n] device, p [n] device (unused by the criterion, validated only),
 *   Y [N*n] device, flags [n] device uint8 out (0 solve, 1 reference,
 *   2 mapped), ref_index device int64 out (-1 if no candidate).
 * n_cells = 0 is allowed (ref = -1).  Asynchronous. */
int chem_map_reference(chem_ctx *ctx, int64_t n_cells, const double *T, const double *p,
                       const double *Y, const chem_map_params *mp, uint8_t *flags,
                       int64_t *ref_index);

/* Advance every cell by dt: a constant-pressure adiabatic reactor in
 * (T, Y_1..Y_N) integrated by adaptive Rodas4 with max-norm error control
 * (the per-cell stiff ODE of Sec. 1; solution tagged with its cell, Sec. 2.2).
 *   T [n] device in/out, p [n] device, Y [N*n] device in/out.
 *   flags [n] device (nullable): cells flagged 2 are not integrated; they take
 *     Y += Y_ref(after) - Y_ref(before) and T from enthalpy conservation, with
 *     the reference cell *ref_index (device int64, required with flags).
 *     Cells flagged 3 (surrogate) are left alone.
 *   h [n] device in/out (nullable): initial step (<= 0 means dt); on return the
 *     step size proposed after each cell's last accepted step.
 *   cost [n] device uint32 in/out (nullable): in, the previous call's per-cell
 *     cost, used to order the queue heavy-first; out, attempted steps.
 *   status [n] device uint8 out (nullable): CHEM_CELL_* per cell.
 *   steps [2n] device int32 out (nullable): accepted (2i) and rejected (2i+1).
 *   stats host (nullable): totals; makes the call synchronous.
 * Returns the number of failed cells when stats is given, else 0 (or <0). */
int chem_integrate(chem_ctx *ctx, int64_t n_cells, double *T, const double *p, double *Y,
                   double dt, const uint8_t *flags, const int64_t *ref_index, double *h,
                   uint32_t *cost, uint8_t *status, int32_t *steps, chem_stats *stats);

/* chem_integrate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, hosts that forbid allocation): the
 * same arguments, kernels and results, but the call allocates nothing.  Its
 * scratch (heavy-first queue, counters, statistics, the reference cell's
 * snapshot and increment) is a fixed device array inside the library, one
 * per device, 8 MiB + 8 KiB, held until the process ends; the caller passes
 * the state, as for chem_integrate.  Limits: n_cells <= 2097152 (larger n
 * returns CHEM_E_INVALID_ARG, nothing enqueued), mechanisms of up to 63
 * species (the wavefront integrator; larger ones return CHEM_E_UNIMPL).
 * Every call on a device shares that device's array and re-initialises what
 * it reads; calls that overlap in time on one device (several contexts or
 * streams) race and must be serialised by the caller.  A context must exist
 * on the device (chem_create resolves the array's device address there). */
int chem_integrate_noalloc(chem_ctx *ctx, int64_t n_cells, double *T, const double *p, double *Y,
                           double dt, const uint8_t *flags, const int64_t *ref_index, double *h,
                           uint32_t *cost, uint8_t *status, int32_t *steps, chem_stats *stats);

/* chem_integrate with the learned surrogate first (not in the paper; the
 * learned relative of the tabulation methods of Sec. 1 and Sec. 5): every cell whose flag is
 * CHEM_FLAG_SOLVE is offered to the surrogate; cells the gate accepts are
 * updated in place and flagged CHEM_FLAG_SURROGATE (flags is device in/out
 * and required; zero-fill it when no mapping is used), all other cells are
 * handled as by chem_integrate.  ref_index may be NULL when no flag is 1 or 2.
 * Status CHEM_CELL_SURROGATE marks surrogate cells; their cost entry is set
 * to 0x7fffffff (unknown), which queues them first should a later call send
 * them to the solver.  Requires parameters
 * (chem_surrogate_train, _set_params or _load).  With a warm workspace (a
 * previous call with at least min(n, 262144) cells) it allocates nothing. */
int chem_integrate_surrogate(chem_ctx *ctx, int64_t n_cells, double *T, const double *p, double *Y,
                             double dt, uint8_t *flags, const int64_t *ref_index,
                             const chem_gate_params *gate, double *h, uint32_t *cost,
                             uint8_t *status, int32_t *steps, chem_stats *stats);

void chem_default_train_params(chem_train_params *t);
void chem_default_gate_params(chem_gate_params *g);
int64_t chem_surrogate_param_count(void);

/* Train the surrogate on n solver-generated pairs (T0, Y0) -> (T1, Y1) over
 * per-sample steps dt (all device arrays: T0, p, dt, T1 [n]; Y0, Y1 [N*n]
 * species-major).  Computes the normalisation and box from the data, draws
 * the initial weights from seed, then runs epochs x floor(n / batch) Adam
 * steps (beta 0.9/0.999, FP32 master weights) on the mean-squared error of
 * the normalised outputs.  loss_history (host, nullable) receives the mean
 * loss of each epoch.  Synchronous; allocates. */
int chem_surrogate_train(chem_ctx *ctx, int64_t n, const double *T0, const double *p,
                         const double *Y0, const double *dt, const double *T1, const double *Y1,
                         const chem_train_params *tp, float *loss_history);
/* Copy the parameter blob to / from host memory (synchronous).  set_params
 * rejects non-finite entries and non-positive normalisation scales. */
int chem_surrogate_get_params(chem_ctx *ctx, float *host);
int chem_surrogate_set_params(chem_ctx *ctx, const float *host);
/* Parameter file: 8-byte magic "LCHSUR01", int32 N, int32 E, int64 count,
 * then the float32 blob (host byte order).  load checks N and E. */
int chem_surrogate_save(chem_ctx *ctx, const char *path);
int chem_surrogate_load(chem_ctx *ctx, const char *path);
/* Raw network outputs (normalised) for n cells: out [n][64] float32 device,
 * row-major.  dt [n] device.  Kernel-level check of inference. */
int chem_surrogate_forward(chem_ctx *ctx, int64_t n, const double *T, const double *p,
                           const double *Y, const double *dt, float *out);
/* The same outputs from the fused inference kernel that
 * chem_integrate_surrogate runs (the whole network per tile of 64 rows in one
 * workgroup, activations kept in LDS), every row selected: same arguments and
 * layout as chem_surrogate_forward.  Its products accumulate in the same
 * order, so the two entry points agree bit for bit; kernel-level check. */
int chem_surrogate_forward_fused(chem_ctx *ctx, int64_t n, const double *T, const double *p,
                                 const double *Y, const double *dt, float *out);
/* Mean-squared-error loss and its gradient (host, float32, blob layout, the
 * normalisation blocks left at zero) over n pairs (64 <= n <= 65536, n a
 * multiple of 64) with the current parameters and normalisation.
 * Kernel-level check of backpropagation. */
int chem_surrogate_loss_grad(chem_ctx *ctx, int64_t n, const double *T0, const double *p,
                             const double *Y0, const double *dt, const double *T1,
                             const double *Y1, float *grad, double *loss);

/* ---- graph capture and launch tuning.  The paper keeps the balancing
 * overhead (preprocessing, balancing and update stages) below 1 % of the
 * chemistry time (Appendix B); on one GPU that overhead is the host-side
 * launch cost of the mapping and queue kernels, which replaying a recorded
 * HIP graph removes, and the queue's launch shape, which chem_autotune picks. */
typedef struct chem_graph chem_graph;

/* Record, instead of run, the calls made on ctx until chem_graph_end
 * (chem_map_reference, chem_integrate and chem_integrate_surrogate without
 * stats).  The context's stream must be a created stream, not the null
 * stream.  Everything those calls allocate must exist beforehand:
 * chem_reserve(n), one eager chem_map_reference with the same streams, and for
 * the surrogate one eager call with at least min(n, 262144) cells; a call that
 * would allocate or synchronise returns CHEM_E_CAPTURE_UNSAFE and
 * chem_graph_end then fails. */
int chem_graph_begin(chem_ctx *ctx);
/* End the recording and instantiate it; *out is owned by the caller. */
int chem_graph_end(chem_ctx *ctx, chem_graph **out);
/* Replay the recorded work on the context's stream (asynchronous).  The
 * graph reads and writes the very device arrays the recorded calls named. */
int chem_graph_launch(chem_ctx *ctx, const chem_graph *g);
void chem_graph_destroy(chem_graph *g);

typedef struct {
    int32_t schedule, queue_chunk, slots_per_cu;
    double ms;            /* GPU time of one chem_integrate call with these options */
} chem_tune_entry;

/* Time launch configurations on copies of a sample state and keep the fastest
 * in the context's options: the plain launch, and the work queue with
 * queue_chunk in {1, 2, 4, 8} and slots_per_cu in {occupancy / 2, occupancy}
 * (occupancy = workgroups of the integration kernel that fit on one CU; one
 * slot choice when they are equal).  One untimed pass first records the
 * per-cell cost that orders the queue.
 * T, p, Y, flags, ref_index as for chem_integrate (device, read only).
 * results (host, nullable) receives up to max_results entries in the order
 * above, *n_results (nullable) their count.  Synchronous; allocates scratch
 * for one copy of the state.
 * The timings are kept for the life of the process, keyed by the device's
 * architecture, the mechanism's species and reaction counts, the integration
 * kernel (wavefront or workgroup, with or without fall-off/PLOG code),
 * whether flags is given, and n_cells rounded down to a power of two.  A later
 * call with the same key, from any context, reports the kept timings and sets
 * the options from them without launching anything. */
int chem_autotune(chem_ctx *ctx, int64_t n_cells, const double *T, const double *p, const double *Y,
                  double dt, const uint8_t *flags, const int64_t *ref_index,
                  chem_tune_entry *results, int32_t max_results, int32_t *n_results);
/* Drop every kept autotune timing, so that the next chem_autotune measures. */
void chem_autotune_forget(void);

/* Evaluate f(y) and the analytic Jacobian for n cells (kernel-level check of
 * the rate and Jacobian code of the integrator: the chemistry model of
 * Sec. 2.1, the analytic Jacobian Sec. 5 names).  T, p [n], Y [N*n] device;
 * f [(N+1)*n] device out (row-major per cell: f[i*(N+1) + r]),
 * J [(N+1)^2 * n] device out (row-major per cell), either nullable. */
int chem_eval_rhs_jac(chem_ctx *ctx, int64_t n_cells, const double *T, const double *p,
                      const double *Y, double *f, double *J);

/* One Rodas4 step of fixed size h per cell with the analytic Jacobian
 * (no step control; the implicit per-cell integration of Sec. 1): y_new and the embedded error estimate, both
 * [(N+1)*n] device out, row-major per cell. */
int chem_rodas_step(chem_ctx *ctx, int64_t n_cells, const double *T, const double *p,
                    const double *Y, double h, double *ynew, double *err);

/* ---------------------------------------------------------------------------
 * Load-balancing plan across processes (Algorithm 1, Sec. 2.2).  Host only:
 * no device, context or mechanism needed.  On one GPU the work queue does the
 * balancing; this plan is what the paper's processes (or several GPUs,
 * sharding cells by cost) would exchange.
 *
 * n_proc processes; process k holds n_prob[k] problems whose costs (e.g. CPU
 * time or attempted steps of the previous step) are t_cost[off_k ..
 * off_k + n_prob[k]), off_k = n_prob[0] + ... + n_prob[k-1], in its own list
 * order.  The plan brings every process towards the mean load L (the sum of
 * all costs over n_proc), pairing the lightest remaining receivers with the
 * heaviest remaining senders as the paper's algorithm does:
 *   - receivers (load below L, lightest first, ties by index) and senders
 *     (load above L, heaviest first) are laid out as consecutive intervals of
 *     their deficits and surpluses; each overlap of a receiver's interval with
 *     a sender's is one transfer of that planned load (where a receiver and a
 *     sender end together to within 1e-12 L, the receiver is retired first);
 *   - a transfer whose planned load is below min_frac * L (the paper uses
 *     0.01) is dropped;
 *   - a kept transfer moves the fewest of the sender's problems, in its list
 *     order from where its previous transfer stopped, whose cost reaches the
 *     planned load (all that remain if none do).
 * ops (host) receives up to max_ops operations in the order found (n_ops: how
 * many were emitted, possibly more than max_ops, in which case
 * CHEM_E_INVALID_ARG is returned after filling max_ops); loads_after (host,
 * nullable, n_proc) the loads once the emitted operations move their
 * problems.  Errors: n_proc < 1, negative counts, non-finite or negative
 * costs, null arrays (CHEM_E_INVALID_ARG). */
typedef struct {
    int32_t sender, receiver;
    int64_t first;     /* index in the sender's list of the first problem sent */
    int64_t count;     /* problems sent: first .. first + count - 1 */
    double load;       /* their summed cost */
    double planned;    /* the planned load of this transfer */
} chem_balance_op;

int chem_plan_balance(int32_t n_proc, const int64_t *n_prob, const double *t_cost, double min_frac,
                      chem_balance_op *ops, int64_t max_ops, int64_t *n_ops, double *loads_after);

#ifdef __cplusplus
}
#endif
#endif
