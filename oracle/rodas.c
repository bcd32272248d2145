/* Oracle LU, Rodas4 stepper, adaptive integration — TEST INFRASTRUCTURE.
 *
 * The paper requires an implicit integrator for the stiff per-cell ODE (Sec. 1)
 * at given relative/absolute tolerances (Sec. 4.1) and names analytic
 * Jacobians and problem-tailored linear algebra as the way to speed it up
 * (Sec. 5).  The method here is Rodas4 (Hairer & Wanner, Solving ODEs II,
 * Sec. IV.7): 6 stages, order 4, embedded order 3, stiffly accurate and
 * L-stable, written in the form that needs no Jacobian-vector products:
 *   (I/(gamma h) - J) u_i = f(y + sum_{j<i} a_ij u_j) + sum_{j<i} (c_ij / h) u_j
 *   y_new = y + sum_{j<5} a_6j u_j + u_5 + u_6,   error estimate = u_6.
 * Step control: err = max_i |e_i| / (atol + rtol max(|y_i|, |y_new,i|));
 * accept iff err <= 1; h <- h * min(5, max(0.2, 0.9 err^(-1/4))), with the
 * factor capped at 1 right after a rejection. */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- LU ---- */
int orc_lu(int n, double *A, int *piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double amax = fabs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(A[(size_t)i * n + k]);
            if (v > amax) { amax = v; p = i; }
        }
        piv[k] = p;
        if (amax == 0.0) return k + 1;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                double t = A[(size_t)k * n + j];
                A[(size_t)k * n + j] = A[(size_t)p * n + j];
                A[(size_t)p * n + j] = t;
            }
        for (int i = k + 1; i < n; ++i) {
            double l = A[(size_t)i * n + k] / A[(size_t)k * n + k];
            A[(size_t)i * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
        }
    }
    return 0;
}

void orc_lu_solve(int n, const double *LU, const int *piv, double *b)
{
    for (int k = 0; k < n; ++k) {
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    }
    for (int i = 0; i < n; ++i) {
        double acc = b[i];
        for (int j = 0; j < i; ++j) acc -= LU[(size_t)i * n + j] * b[j];
        b[i] = acc;
    }
    for (int i = n - 1; i >= 0; --i) {
        double acc = b[i];
        for (int j = i + 1; j < n; ++j) acc -= LU[(size_t)i * n + j] * b[j];
        b[i] = acc / LU[(size_t)i * n + i];
    }
}

/* ------------------------------------------------------ coefficients ---- */
/* Rodas4 (Hairer & Wanner 1996, Sec. IV.7, transformed coefficients). */
static const double GAMMA = 0.25;
static const double A21 = 1.544, A31 = 0.9466785280815826, A32 = 0.2557011698983284,
    A41 = 3.314825187068521, A42 = 2.896124015972201, A43 = 0.9986419139977817,
    A51 = 1.221224509226641, A52 = 6.019134481288629, A53 = 12.53708332932087,
    A54 = -0.6878860361058950;
static const double C21 = -5.6688, C31 = -2.430093356833875, C32 = -0.2063599157091915,
    C41 = -0.1073529058151375, C42 = -9.594562251023355, C43 = -20.47028614809616,
    C51 = 7.496443313967647, C52 = -10.24680431464352, C53 = -33.99990352819905,
    C54 = 11.70890893206160, C61 = 8.083246795921522, C62 = -7.981132988064893,
    C63 = -31.52159432874371, C64 = 16.31930543123136, C65 = -6.058818238834054;

static void coeffs(double a[6][6], double c[6][6])
{
    memset(a, 0, sizeof(double) * 36);
    memset(c, 0, sizeof(double) * 36);
    a[1][0] = A21;
    a[2][0] = A31; a[2][1] = A32;
    a[3][0] = A41; a[3][1] = A42; a[3][2] = A43;
    a[4][0] = A51; a[4][1] = A52; a[4][2] = A53; a[4][3] = A54;
    a[5][0] = A51; a[5][1] = A52; a[5][2] = A53; a[5][3] = A54; a[5][4] = 1.0;
    c[1][0] = C21;
    c[2][0] = C31; c[2][1] = C32;
    c[3][0] = C41; c[3][1] = C42; c[3][2] = C43;
    c[4][0] = C51; c[4][1] = C52; c[4][2] = C53; c[4][3] = C54;
    c[5][0] = C61; c[5][1] = C62; c[5][2] = C63; c[5][3] = C64; c[5][4] = C65;
}

void orc_rodas4_coeffs(double *a36, double *c36, double *gamma)
{
    double a[6][6], c[6][6];
    coeffs(a, c);
    memcpy(a36, a, sizeof a);
    memcpy(c36, c, sizeof c);
    *gamma = GAMMA;
}

/* ------------------------------------------------------------- step ---- */
/* One step: M = I/(gamma h) - J is factored here.  Returns 0, or 1 if M is
 * singular (then the step counts as rejected). */
static int rodas_step(const omech *m, double p, const double *y, const double *f0,
                      const double *J, double h, double *ynew, double *err, int *n_rhs)
{
    const int n = m->N + 1;
    double a[6][6], c[6][6];
    coeffs(a, c);
    double *M = (double *)malloc(sizeof(double) * n * n);
    double *u = (double *)malloc(sizeof(double) * 6 * n);
    double *ys = (double *)malloc(sizeof(double) * n);
    double *rhs = (double *)malloc(sizeof(double) * n);
    int *piv = (int *)malloc(sizeof(int) * n);
    const double diag = 1.0 / (GAMMA * h);
    for (int i = 0; i < n * n; ++i) M[i] = -J[i];
    for (int i = 0; i < n; ++i) M[(size_t)i * n + i] += diag;
    int sing = orc_lu(n, M, piv);
    if (!sing) {
        for (int i = 0; i < n; ++i) u[i] = f0[i];
        orc_lu_solve(n, M, piv, u);
        for (int s = 1; s < 6; ++s) {
            for (int i = 0; i < n; ++i) {
                double acc = y[i];
                for (int j = 0; j < s; ++j) acc += a[s][j] * u[(size_t)j * n + i];
                ys[i] = acc;
            }
            orc_rhs(m, p, ys, rhs);
            ++*n_rhs;
            for (int i = 0; i < n; ++i) {
                double acc = rhs[i];
                for (int j = 0; j < s; ++j) acc += (c[s][j] / h) * u[(size_t)j * n + i];
                u[(size_t)s * n + i] = acc;
            }
            orc_lu_solve(n, M, piv, u + (size_t)s * n);
        }
        /* ys holds the stage-6 input y + sum a_6j u_j */
        for (int i = 0; i < n; ++i) {
            ynew[i] = ys[i] + u[(size_t)5 * n + i];
            err[i] = u[(size_t)5 * n + i];
        }
    }
    free(M); free(u); free(ys); free(rhs); free(piv);
    return sing ? 1 : 0;
}

int orc_rodas4_step(const omech *m, double p, const double *y, const double *f0,
                    const double *J, double h, double *ynew, double *err)
{
    int nr = 0;
    return rodas_step(m, p, y, f0, J, h, ynew, err, &nr);
}

static int all_finite(int n, const double *v)
{
    for (int i = 0; i < n; ++i) if (!isfinite(v[i])) return 0;
    return 1;
}

/* --------------------------------------------------------- integrate ---- */
int orc_integrate_cell(const omech *m, double p, double *y, double dt,
                       const oopts *o, double *h_io, ostats *st)
{
    const int n = m->N + 1;
    memset(st, 0, sizeof *st);
    if (!(p > 0.0) || !isfinite(p) || !(y[0] > 0.0) || !all_finite(n, y) || !(dt > 0.0)) {
        st->status = ORC_BAD_INPUT;
        return st->status;
    }
    double *f0 = (double *)malloc(sizeof(double) * n);
    double *J = (double *)malloc(sizeof(double) * n * n);
    double *ynew = (double *)malloc(sizeof(double) * n);
    double *err = (double *)malloc(sizeof(double) * n);

    double h = (h_io && *h_io > 0.0) ? *h_io : dt;
    double t = 0.0, h_next = h;
    int reject_last = 0;
    orc_rhs(m, p, y, f0); st->n_rhs++;
    if (o->use_cs_jac) orc_jac_cs(m, p, y, J); else orc_jac(m, p, y, J);
    st->n_jac++;
    st->status = ORC_OK;
    while (t < dt) {
        if (st->n_accept + st->n_reject >= o->max_steps) { st->status = ORC_MAX_STEPS; break; }
        int last = 0;
        if (h >= dt - t) { h = dt - t; last = 1; }
        if (h < o->hmin_frac * dt) { st->status = ORC_H_UNDERFLOW; break; }
        int sing = rodas_step(m, p, y, f0, J, h, ynew, err, &st->n_rhs);
        st->n_lu++;
        double e = 0.0;
        int bad = sing;
        if (!sing) {
            for (int i = 0; i < n; ++i) {
                double sc = o->atol + o->rtol * fmax(fabs(y[i]), fabs(ynew[i]));
                double r = fabs(err[i]) / sc;
                if (!(r <= e)) e = r;            /* NaN propagates into e */
            }
            if (isnan(e)) bad = 1;
        }
        if (!bad && e <= 1.0) {
            double fac = (e == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(e, -0.25)));
            if (reject_last) fac = fmin(fac, 1.0);
            memcpy(y, ynew, sizeof(double) * n);
            t = last ? dt : t + h;
            st->n_accept++;
            h_next = h * fac;
            h = h_next;
            reject_last = 0;
            if (t < dt) {
                orc_rhs(m, p, y, f0); st->n_rhs++;
                if (o->use_cs_jac) orc_jac_cs(m, p, y, J); else orc_jac(m, p, y, J);
                st->n_jac++;
            }
        } else {
            double fac = bad ? 0.2 : fmax(0.2, 0.9 * pow(e, -0.25));
            h = h * fac;
            st->n_reject++;
            reject_last = 1;
        }
    }
    if (st->status == ORC_OK && !all_finite(n, y)) st->status = ORC_NONFINITE;
    if (h_io) *h_io = h_next;
    free(f0); free(J); free(ynew); free(err);
    return st->status;
}

void orc_integrate_batch(const omech *m, int64_t ncells, double *T, const double *p,
                         double *Y, double dt, const oopts *o, double *h,
                         const uint8_t *flags, uint8_t *status, int32_t *n_acc,
                         int32_t *n_rej, int threads, int schedule)
{
    const int N = m->N;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
#define ORC_CELL_BODY                                                            \
    {                                                                            \
        if (flags && flags[c] == 2) {                                            \
            if (status) status[c] = 0;                                           \
            if (n_acc) n_acc[c] = 0;                                             \
            if (n_rej) n_rej[c] = 0;                                             \
        } else {                                                                 \
            double y[N + 1];                                                     \
            y[0] = T[c];                                                         \
            for (int k = 0; k < N; ++k) y[1 + k] = Y[(size_t)k * ncells + c];    \
            ostats st;                                                           \
            double hc = h ? h[c] : 0.0;                                          \
            orc_integrate_cell(m, p[c], y, dt, o, &hc, &st);                     \
            if (st.status != ORC_BAD_INPUT) {                                    \
                T[c] = y[0];                                                     \
                for (int k = 0; k < N; ++k) Y[(size_t)k * ncells + c] = y[1 + k]; \
            }                                                                    \
            if (h) h[c] = hc;                                                    \
            if (status) status[c] = (uint8_t)st.status;                          \
            if (n_acc) n_acc[c] = st.n_accept;                                   \
            if (n_rej) n_rej[c] = st.n_reject;                                   \
        }                                                                        \
    }
    if (schedule == 1) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t c = 0; c < ncells; ++c) ORC_CELL_BODY
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < ncells; ++c) ORC_CELL_BODY
    }
#undef ORC_CELL_BODY
}

/* --------------------------------------------------------------- RK4 ---- */
void orc_rk4(const omech *m, double p, double *y, double t_end, int64_t nsteps)
{
    const int n = m->N + 1;
    const double h = t_end / (double)nsteps;
    double k1[n], k2[n], k3[n], k4[n], yt[n];
    for (int64_t s = 0; s < nsteps; ++s) {
        orc_rhs(m, p, y, k1);
        for (int i = 0; i < n; ++i) yt[i] = y[i] + 0.5 * h * k1[i];
        orc_rhs(m, p, yt, k2);
        for (int i = 0; i < n; ++i) yt[i] = y[i] + 0.5 * h * k2[i];
        orc_rhs(m, p, yt, k3);
        for (int i = 0; i < n; ++i) yt[i] = y[i] + h * k3[i];
        orc_rhs(m, p, yt, k4);
        for (int i = 0; i < n; ++i) y[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
}
