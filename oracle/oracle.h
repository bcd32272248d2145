/*
 * CPU oracle for per-cell stiff chemistry integration — TEST INFRASTRUCTURE.
 *
 * A plain, serial, FP64 reference of everything the HIP path computes.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code with the HIP library.
 *
 * The paper (DLBFoam) treats each finite-volume cell's chemistry as an
 * independent homogeneous reactor ODE dPhi/dt = f(Phi) that is stiff and needs
 * an implicit integrator (Sec. 1); it delegates the chemistry itself to a
 * standard chemistry model (program summary).  The formulas here are the
 * textbook ones that such a model integrates:
 *   - NASA-7 style single-range thermodynamics,
 *   - mass-action kinetics, reverse rates from equilibrium constants,
 *     third-body enhanced reactions,
 *   - a constant-pressure adiabatic reactor in (T, Y_1..Y_N),
 *   - the Rodas4 Rosenbrock method (Hairer & Wanner, Solving ODEs II, Sec. IV.7)
 *     with an embedded order-3 error estimate and max-norm step control,
 *   - Doolittle LU with partial pivoting,
 *   - reference mapping by mixture fraction and temperature (Sec. 2.3).
 *
 * Units: CGS (mol/cm^3, cm^3/mol/s, dyn/cm^2, erg), activation energy in J/mol.
 */
#ifndef CHEM_ORACLE_H
#define CHEM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_RU_ERG 8.314462618e7     /* erg / (mol K) */
#define ORC_RU_J   8.314462618       /* J / (mol K)   */
#define ORC_P_ATM  1.01325e6         /* dyn / cm^2    */

/* status codes of one cell's integration */
enum { ORC_OK = 0, ORC_MAX_STEPS = 1, ORC_H_UNDERFLOW = 2, ORC_NONFINITE = 3, ORC_BAD_INPUT = 4 };

typedef struct omech {
    int E, N, R;
    double *elem_mass;   /* [E] */
    int    *comp;        /* [N*E] atom counts, row = species */
    double *W;           /* [N] */
    double *nasa;        /* [N*7] */
    int    *reac;        /* [R*2], -1 padded */
    int    *prod;        /* [R*3], -1 padded */
    double *lnA, *b, *Ea;/* [R] */
    int    *tb;          /* [R] third-body flag */
    double *alpha;       /* [R*N] third-body efficiencies (1 unless listed) */
    int    *sum_nu;      /* [R] (#product slots) - (#reactant slots) */
    int    *fo_type;     /* [R] fall-off form: 0 none, 1 Lindemann, 2 Troe */
    double *fo;          /* [R*7] A0, b0, Ea0 (J/mol), a, T3, T1, T2 (T2 <= 0: no T2 term) */
    int    has_falloff;
    int    *plog_n;      /* [R] pressure-dependent (PLOG) reactions: number of tabulated pressures, else 0 */
    double *plog;        /* [R*32] up to 8 entries p_i (dyn/cm^2, increasing), A_i, b_i, Ea_i (J/mol) */
    int    has_plog;
} omech;

typedef struct {
    double rtol, atol;
    int    max_steps;    /* limit on attempted steps (accepted + rejected) */
    double hmin_frac;    /* fail when h < hmin_frac * dt */
    int    use_cs_jac;   /* 1: drive the stepper with the complex-step Jacobian */
} oopts;

typedef struct {
    int n_accept, n_reject, n_jac, n_lu, n_rhs;
    int status;
} ostats;

/* mechanism ----------------------------------------------------------------*/
int  orc_mech_create(omech **out, int E, int N, int R,
                     const double *elem_mass, const int32_t *comp, const double *W,
                     const double *nasa, const int32_t *reac, const int32_t *prod,
                     const double *A, const double *b, const double *Ea,
                     const int32_t *tb, int n_eff, const int32_t *eff_r,
                     const int32_t *eff_s, const double *eff_v,
                     const int32_t *fo_type, const double *fo_params);
void orc_mech_destroy(omech *m);
/* tabulated pressure dependence (PLOG) of the reactions with count[j] > 0:
 * count[j] in 2..8 entries params[32j + 4i ..] = p_i, A_i, b_i, Ea_i */
int  orc_mech_set_plog(omech *m, const int32_t *count, const double *params);
/* ln k_f of reaction j at (T, p) (Arrhenius, or interpolated for PLOG) */
double orc_ln_kf(const omech *m, int j, double T, double p);
/* fall-off factor G(T, [M]) of reaction j: its rate constant is k_inf G */
double orc_falloff_factor(const omech *m, int j, double T, double M);

/* thermo (per species, nondimensional) */
void orc_thermo(const omech *m, double T, double *cp_R, double *h_RT, double *s_R);

/* kinetics at (T, p, Y): rate constants, rates of progress, production rates */
void orc_kinetics(const omech *m, double T, double p, const double *Y,
                  double *kf, double *kr, double *q, double *omega);

/* right-hand side f(y), y = (T, Y_1..Y_N) */
void orc_rhs(const omech *m, double p, const double *y, double *f);
/* analytic Jacobian, row-major n x n, J[i*n + j] = d f_i / d y_j (for
 * mechanisms with fall-off or PLOG reactions: the complex-step Jacobian) */
void orc_jac(const omech *m, double p, const double *y, double *J);
/* complex-step Jacobian (step 1e-30 i), same layout */
void orc_jac_cs(const omech *m, double p, const double *y, double *J);
/* imaginary part of f(y + i*hstep*v) / hstep, for tests of the complex path */
void orc_rhs_cs_dir(const omech *m, double p, const double *y, const double *v,
                    double hstep, double *fre, double *fim);

/* mixture helpers (mass specific, erg/g and erg/(g K)) */
double orc_enthalpy_mass(const omech *m, double T, const double *Y);
double orc_cp_mass(const omech *m, double T, const double *Y);
double orc_density(const omech *m, double T, double p, const double *Y);

/* dense LU with partial pivoting (ties to the lowest row); returns 0 or k+1 if
 * column k has no nonzero pivot */
int  orc_lu(int n, double *A, int *piv);
void orc_lu_solve(int n, const double *LU, const int *piv, double *b);

/* Rodas4 coefficient table (transformed form: a[6][6], c[6][6], gamma) */
void orc_rodas4_coeffs(double *a36, double *c36, double *gamma);
/* one Rodas4 step of fixed size h at y with Jacobian J; ynew and err out */
int  orc_rodas4_step(const omech *m, double p, const double *y, const double *f0,
                     const double *J, double h, double *ynew, double *err);
/* adaptive integration of one cell over [0, dt]; y in/out; h_io in: initial
 * step (<=0: dt), out: proposed next step */
int  orc_integrate_cell(const omech *m, double p, double *y, double dt,
                        const oopts *o, double *h_io, ostats *st);
/* batch over cells (OpenMP), Y species-major [N][cells].  flags (nullable):
 * cells with flag 2 are skipped.  schedule: 0 static, 1 dynamic(16). */
void orc_integrate_batch(const omech *m, int64_t ncells, double *T, const double *p,
                         double *Y, double dt, const oopts *o, double *h,
                         const uint8_t *flags, uint8_t *status, int32_t *n_acc,
                         int32_t *n_rej, int threads, int schedule);

/* classical RK4 with a fixed number of steps (brute-force check) */
void orc_rk4(const omech *m, double p, double *y, double t_end, int64_t nsteps);

/* reference mapping (Sec. 2.3) -------------------------------------------*/
void orc_map_weights(const omech *m, const double *Yfuel, const double *Yox,
                     double *w, double *beta_f, double *beta_ox);
void orc_mixture_fraction(const omech *m, int64_t ncells, const double *Y,
                          const double *w, double beta_f, double beta_ox, double *Z);
/* flags: 0 solve, 1 reference, 2 mapped; returns reference index or -1 */
int64_t orc_map_reference(const omech *m, int64_t ncells, const double *T,
                          const double *Y, const double *w, double beta_f,
                          double beta_ox, double Z_tol, double T_tol, int use_T,
                          uint8_t *flags);
/* mapped-cell update: Y += dY_ref, T from h(T', Y') = h(T, Y) by Newton */
void orc_map_scatter(const omech *m, int64_t ncells, double *T, double *Y,
                     const uint8_t *flags, const double *Yref_old,
                     const double *Yref_new);
double orc_temperature_from_enthalpy(const omech *m, double h, const double *Y,
                                     double T_guess, int *iters);

/* learned surrogate (see mlp.c) ------------------------------------------*/
int64_t orc_mlp_param_count(void);
double orc_bf16(double x);
void orc_mlp_features(int N, double T, double p, const double *Y, double dt, double *x);
void orc_mlp_forward(const float *P, int64_t n, int nfeat, const double *X, int bf16,
                     double *out, double *acts, double *pre);
double orc_mlp_loss_grad(const float *P, int64_t n, int nfeat, int nout, const double *X,
                         const double *target, int bf16, double *grad);
int orc_conserve(const omech *m, const double *Y0, double *Y1);
int orc_surrogate_cell(const omech *m, const float *P, double p, double *T, double *Y, double dt,
                       double tau_T, double y_min, double margin, double max_dT, double T_max);

#ifdef __cplusplus
}
#endif
#endif
