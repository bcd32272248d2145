/* Oracle reference mapping — TEST INFRASTRUCTURE.
 *
 * Sec. 2.3: a cell reuses the reference cell's chemistry when
 *   Z_i < Z_tol   and (optionally) |T_i - T_ref| < T_tol,
 * with Z a Bilger-type mixture fraction; the reference is the first cell found
 * that meets the criterion, and its solution is mapped to the later ones.
 *
 * Mixture fraction for arbitrary elements (the paper uses Bilger's definition,
 * which is specific to C/H/O): with element mass fractions
 *   Z_e(Y) = sum_k a_ek W_e Y_k / W_k,
 * coupling weights c_e = (Z_e(Y_fuel) - Z_e(Y_ox)) / W_e and
 *   beta(Y) = sum_e c_e Z_e(Y) = sum_k w_k Y_k,  w_k = sum_e c_e a_ek W_e / W_k,
 * the mixture fraction is Z = (beta - beta_ox) / (beta_fuel - beta_ox).
 * Every sum runs in ascending index with separately rounded multiply and add
 * (this file is compiled without floating-point contraction), so Z, and the
 * flags derived from it, are reproducible bit for bit.
 *
 * A mapped cell receives the reference's increment, Y_i' = Y_i + (Y_ref' - Y_ref),
 * and its temperature from enthalpy conservation, h(T_i', Y_i') = h(T_i, Y_i),
 * solved by Newton's method to |dT| < 1e-10 K. */
#include <math.h>
#include <stdlib.h>
#include "oracle.h"

void orc_map_weights(const omech *m, const double *Yfuel, const double *Yox,
                     double *w, double *beta_f, double *beta_ox)
{
    const int E = m->E, N = m->N;
    double c[8];
    for (int e = 0; e < E; ++e) {
        double zf = 0.0, zo = 0.0;
        for (int k = 0; k < N; ++k) {
            double t = (double)m->comp[k * E + e] * m->elem_mass[e];
            double tf = t * Yfuel[k];
            tf = tf / m->W[k];
            zf = zf + tf;
            double to = t * Yox[k];
            to = to / m->W[k];
            zo = zo + to;
        }
        c[e] = (zf - zo) / m->elem_mass[e];
    }
    for (int k = 0; k < N; ++k) {
        double acc = 0.0;
        for (int e = 0; e < E; ++e) {
            double t = c[e] * (double)m->comp[k * E + e];
            t = t * m->elem_mass[e];
            t = t / m->W[k];
            acc = acc + t;
        }
        w[k] = acc;
    }
    double bf = 0.0, bo = 0.0;
    for (int k = 0; k < N; ++k) {
        double t = w[k] * Yfuel[k];
        bf = bf + t;
        t = w[k] * Yox[k];
        bo = bo + t;
    }
    *beta_f = bf;
    *beta_ox = bo;
}

void orc_mixture_fraction(const omech *m, int64_t ncells, const double *Y,
                          const double *w, double beta_f, double beta_ox, double *Z)
{
    const int N = m->N;
    for (int64_t i = 0; i < ncells; ++i) {
        double beta = 0.0;
        for (int k = 0; k < N; ++k) {
            double t = w[k] * Y[(size_t)k * ncells + i];
            beta = beta + t;
        }
        Z[i] = (beta - beta_ox) / (beta_f - beta_ox);
    }
}

int64_t orc_map_reference(const omech *m, int64_t ncells, const double *T,
                          const double *Y, const double *w, double beta_f,
                          double beta_ox, double Z_tol, double T_tol, int use_T,
                          uint8_t *flags)
{
    double *Z = (double *)malloc(sizeof(double) * (ncells > 0 ? ncells : 1));
    orc_mixture_fraction(m, ncells, Y, w, beta_f, beta_ox, Z);
    int64_t ref = -1;
    for (int64_t i = 0; i < ncells; ++i) {
        flags[i] = 0;
        if (ref < 0 && Z[i] < Z_tol) ref = i;
    }
    if (ref >= 0) {
        flags[ref] = 1;
        for (int64_t i = ref + 1; i < ncells; ++i) {
            if (!(Z[i] < Z_tol)) continue;
            if (use_T && !(fabs(T[i] - T[ref]) < T_tol)) continue;
            flags[i] = 2;
        }
    }
    free(Z);
    return ref;
}

double orc_temperature_from_enthalpy(const omech *m, double h, const double *Y,
                                     double T_guess, int *iters)
{
    double T = T_guess;
    int it = 0;
    for (; it < 50; ++it) {
        double F = orc_enthalpy_mass(m, T, Y) - h;
        double dT = F / orc_cp_mass(m, T, Y);
        T -= dT;
        if (fabs(dT) < 1e-10) { ++it; break; }
    }
    if (iters) *iters = it;
    return T;
}

void orc_map_scatter(const omech *m, int64_t ncells, double *T, double *Y,
                     const uint8_t *flags, const double *Yref_old,
                     const double *Yref_new)
{
    const int N = m->N;
    double y[N], ynew[N];
    for (int64_t i = 0; i < ncells; ++i) {
        if (flags[i] != 2) continue;
        for (int k = 0; k < N; ++k) {
            y[k] = Y[(size_t)k * ncells + i];
            ynew[k] = y[k] + (Yref_new[k] - Yref_old[k]);
        }
        double h = orc_enthalpy_mass(m, T[i], y);
        T[i] = orc_temperature_from_enthalpy(m, h, ynew, T[i], NULL);
        for (int k = 0; k < N; ++k) Y[(size_t)k * ncells + i] = ynew[k];
    }
}
