/* Oracle mechanism storage — TEST INFRASTRUCTURE (see oracle.h). */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

int orc_mech_create(omech **out, int E, int N, int R,
                    const double *elem_mass, const int32_t *comp, const double *W,
                    const double *nasa, const int32_t *reac, const int32_t *prod,
                    const double *A, const double *b, const double *Ea,
                    const int32_t *tb, int n_eff, const int32_t *eff_r,
                    const int32_t *eff_s, const double *eff_v,
                    const int32_t *fo_type, const double *fo_params)
{
    omech *m = (omech *)calloc(1, sizeof(omech));
    if (!m) return -1;
    m->E = E; m->N = N; m->R = R;
    m->elem_mass = (double *)malloc(sizeof(double) * E);
    m->comp = (int *)malloc(sizeof(int) * N * E);
    m->W = (double *)malloc(sizeof(double) * N);
    m->nasa = (double *)malloc(sizeof(double) * N * 7);
    m->reac = (int *)malloc(sizeof(int) * R * 2);
    m->prod = (int *)malloc(sizeof(int) * R * 3);
    m->lnA = (double *)malloc(sizeof(double) * R);
    m->b = (double *)malloc(sizeof(double) * R);
    m->Ea = (double *)malloc(sizeof(double) * R);
    m->tb = (int *)malloc(sizeof(int) * R);
    m->alpha = (double *)malloc(sizeof(double) * R * N);
    m->sum_nu = (int *)malloc(sizeof(int) * R);
    m->fo_type = (int *)calloc((size_t)R, sizeof(int));
    m->fo = (double *)calloc((size_t)R * 7, sizeof(double));
    m->has_falloff = 0;
    for (int e = 0; e < E; ++e) m->elem_mass[e] = elem_mass[e];
    for (int i = 0; i < N * E; ++i) m->comp[i] = comp[i];
    for (int k = 0; k < N; ++k) m->W[k] = W[k];
    for (int i = 0; i < N * 7; ++i) m->nasa[i] = nasa[i];
    for (int j = 0; j < R; ++j) {
        int ns = 0;
        for (int s = 0; s < 2; ++s) { m->reac[2 * j + s] = reac[2 * j + s]; ns -= reac[2 * j + s] >= 0; }
        for (int s = 0; s < 3; ++s) { m->prod[3 * j + s] = prod[3 * j + s]; ns += prod[3 * j + s] >= 0; }
        m->sum_nu[j] = ns;
        m->lnA[j] = log(A[j]);
        m->b[j] = b[j];
        m->Ea[j] = Ea[j];
        m->tb[j] = tb[j];
        for (int k = 0; k < N; ++k) m->alpha[(size_t)j * N + k] = 1.0;
    }
    for (int i = 0; i < n_eff; ++i)
        m->alpha[(size_t)eff_r[i] * N + eff_s[i]] = eff_v[i];
    if (fo_type && fo_params)
        for (int j = 0; j < R; ++j) {
            m->fo_type[j] = fo_type[j];
            for (int c = 0; c < 7; ++c) m->fo[(size_t)j * 7 + c] = fo_params[(size_t)j * 7 + c];
            if (fo_type[j]) m->has_falloff = 1;
        }
    *out = m;
    return 0;
}

int orc_mech_set_plog(omech *m, const int32_t *count, const double *params)
{
    const int R = m->R;
    free(m->plog_n); free(m->plog);
    m->plog_n = (int *)calloc((size_t)R, sizeof(int));
    m->plog = (double *)calloc((size_t)R * 32, sizeof(double));
    if (!m->plog_n || !m->plog) return -1;
    m->has_plog = 0;
    for (int j = 0; j < R; ++j) {
        if (!count[j]) continue;
        if (count[j] < 2 || count[j] > 8) return -1;
        m->plog_n[j] = count[j];
        for (int c = 0; c < 4 * count[j]; ++c) m->plog[(size_t)32 * j + c] = params[(size_t)32 * j + c];
        m->has_plog = 1;
    }
    return 0;
}

void orc_mech_destroy(omech *m)
{
    if (!m) return;
    free(m->plog_n); free(m->plog);
    free(m->elem_mass); free(m->comp); free(m->W); free(m->nasa);
    free(m->reac); free(m->prod); free(m->lnA); free(m->b); free(m->Ea);
    free(m->tb); free(m->alpha); free(m->sum_nu); free(m->fo_type); free(m->fo);
    free(m);
}
