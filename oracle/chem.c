/* Oracle thermochemistry, kinetics, RHS and Jacobians — TEST INFRASTRUCTURE.
 * Formulas are stated in rhs_body.h; the reactor is the per-cell homogeneous
 * reaction system the paper solves in every CFD cell (Sec. 1, Sec. 2.1). */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define SC double
#define SC_EXP exp
#define SC_LOG log
#define FN_RHS rhs_real
#define FN_FALLOFF falloff_real
#define FN_LNKF lnkf_real
#include "rhs_body.h"
#undef SC
#undef SC_EXP
#undef SC_LOG
#undef FN_RHS
#undef FN_FALLOFF
#undef FN_LNKF

#define SC double complex
#define SC_EXP cexp
#define SC_LOG clog
#define FN_RHS rhs_cplx
#define FN_FALLOFF falloff_cplx
#define FN_LNKF lnkf_cplx
#include "rhs_body.h"
#undef SC
#undef SC_EXP
#undef SC_LOG
#undef FN_RHS
#undef FN_FALLOFF
#undef FN_LNKF

double orc_ln_kf(const omech *m, int j, double T, double p)
{
    return lnkf_real(m, j, p, T, log(T));
}

double orc_falloff_factor(const omech *m, int j, double T, double M)
{
    if (!m->fo_type[j]) return M;
    const double lnT = log(T);
    const double kinf = exp(m->lnA[j] + m->b[j] * lnT - m->Ea[j] / (ORC_RU_J * T));
    return falloff_real(m, j, T, lnT, kinf, M);
}

void orc_rhs(const omech *m, double p, const double *y, double *f)
{
    rhs_real(m, p, y, f);
}

void orc_rhs_cs_dir(const omech *m, double p, const double *y, const double *v,
                    double hstep, double *fre, double *fim)
{
    const int n = m->N + 1;
    double complex yc[n], fc[n];
    for (int i = 0; i < n; ++i) yc[i] = y[i] + I * hstep * v[i];
    rhs_cplx(m, p, yc, fc);
    for (int i = 0; i < n; ++i) { fre[i] = creal(fc[i]); fim[i] = cimag(fc[i]) / hstep; }
}

void orc_jac_cs(const omech *m, double p, const double *y, double *J)
{
    const int n = m->N + 1;
    const double hs = 1e-30;
    double complex yc[n], fc[n];
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) yc[i] = y[i];
        yc[j] = y[j] + I * hs;
        rhs_cplx(m, p, yc, fc);
        for (int i = 0; i < n; ++i) J[(size_t)i * n + j] = cimag(fc[i]) / hs;
    }
}

void orc_thermo(const omech *m, double T, double *cp_R, double *h_RT, double *s_R)
{
    const double lnT = log(T);
    for (int k = 0; k < m->N; ++k) {
        const double *a = m->nasa + 7 * k;
        cp_R[k] = a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
        h_RT[k] = a[0] + a[1] * T / 2.0 + a[2] * T * T / 3.0 + a[3] * T * T * T / 4.0
                + a[4] * T * T * T * T / 5.0 + a[5] / T;
        s_R[k] = a[0] * lnT + a[1] * T + a[2] * T * T / 2.0 + a[3] * T * T * T / 3.0
               + a[4] * T * T * T * T / 4.0 + a[6];
    }
}

/* d(cp/R)/dT */
static double dcpR_dT(const double *a, double T)
{
    return a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T * T + 4.0 * a[4] * T * T * T;
}

double orc_density(const omech *m, double T, double p, const double *Y)
{
    double s = 0.0;
    for (int k = 0; k < m->N; ++k) s += Y[k] / m->W[k];
    return p * (1.0 / s) / (ORC_RU_ERG * T);
}

double orc_enthalpy_mass(const omech *m, double T, const double *Y)
{
    const int N = m->N;
    double cp[N], h[N], s[N];
    orc_thermo(m, T, cp, h, s);
    double acc = 0.0;
    for (int k = 0; k < N; ++k) acc += Y[k] * h[k] * ORC_RU_ERG * T / m->W[k];
    return acc;
}

double orc_cp_mass(const omech *m, double T, const double *Y)
{
    const int N = m->N;
    double cp[N], h[N], s[N];
    orc_thermo(m, T, cp, h, s);
    double acc = 0.0;
    for (int k = 0; k < N; ++k) acc += Y[k] * cp[k] * ORC_RU_ERG / m->W[k];
    return acc;
}

void orc_kinetics(const omech *m, double T, double p, const double *Y,
                  double *kf, double *kr, double *q, double *omega)
{
    const int N = m->N, R = m->R;
    double cp[N], h[N], s[N], g[N], C[N];
    orc_thermo(m, T, cp, h, s);
    for (int k = 0; k < N; ++k) g[k] = h[k] - s[k];
    const double rho = orc_density(m, T, p, Y);
    for (int k = 0; k < N; ++k) { C[k] = rho * Y[k] / m->W[k]; omega[k] = 0.0; }
    const double lnT = log(T), ln_patm_RT = log(ORC_P_ATM / (ORC_RU_ERG * T));
    for (int j = 0; j < R; ++j) {
        const int *rs = m->reac + 2 * j, *ps = m->prod + 3 * j;
        double ln_kf = lnkf_real(m, j, p, T, lnT);
        double dG = 0.0, Pf = 1.0, Pr = 1.0;
        for (int s2 = 0; s2 < 2; ++s2) if (rs[s2] >= 0) { dG -= g[rs[s2]]; Pf *= C[rs[s2]]; }
        for (int s3 = 0; s3 < 3; ++s3) if (ps[s3] >= 0) { dG += g[ps[s3]]; Pr *= C[ps[s3]]; }
        double ln_Kc = -dG + (double)m->sum_nu[j] * ln_patm_RT;
        kf[j] = exp(ln_kf);
        kr[j] = exp(ln_kf - ln_Kc);
        double mj = 1.0;
        if (m->tb[j]) {
            mj = 0.0;
            for (int k = 0; k < N; ++k) mj += m->alpha[(size_t)j * N + k] * C[k];
        }
        if (m->fo_type[j]) mj = falloff_real(m, j, T, lnT, kf[j], mj);
        q[j] = mj * (kf[j] * Pf - kr[j] * Pr);
        for (int s2 = 0; s2 < 2; ++s2) if (rs[s2] >= 0) omega[rs[s2]] -= q[j];
        for (int s3 = 0; s3 < 3; ++s3) if (ps[s3] >= 0) omega[ps[s3]] += q[j];
    }
}

/* Analytic Jacobian by the chain rule through C_k(T, Y):
 *   dC_k/dY_i = rho delta_ki / W_k - C_k Wbar / W_i,   dC_k/dT = -C_k / T
 *   d ln k_f/dT = b/T + Ea/(R T^2),   d ln Kc/dT = (sum_k nu_k H_k/RT - sum nu)/T
 * First the concentration Jacobian JC = d omega / dC at fixed T and
 * JCT = d omega / dT at fixed C, then the transformation to (T, Y). */
void orc_jac(const omech *m, double p, const double *y, double *J)
{
    if (m->has_falloff || m->has_plog) {
        orc_jac_cs(m, p, y, J);
        return;
    }
    const int N = m->N, R = m->R, n = N + 1;
    const double T = y[0];
    const double *Y = y + 1;
    double cp[N], h[N], s[N], g[N], C[N], omega[N], fY[N], sk[N];
    double *JC = (double *)calloc((size_t)N * N, sizeof(double));
    double *JCT = (double *)calloc((size_t)N, sizeof(double));
    double dq[N];

    orc_thermo(m, T, cp, h, s);
    for (int k = 0; k < N; ++k) g[k] = h[k] - s[k];
    double sumYW = 0.0;
    for (int k = 0; k < N; ++k) sumYW += Y[k] / m->W[k];
    const double Wbar = 1.0 / sumYW;
    const double rho = p * Wbar / (ORC_RU_ERG * T);
    for (int k = 0; k < N; ++k) { C[k] = rho * Y[k] / m->W[k]; omega[k] = 0.0; }
    const double lnT = log(T), ln_patm_RT = log(ORC_P_ATM / (ORC_RU_ERG * T));

    for (int j = 0; j < R; ++j) {
        const int *rs = m->reac + 2 * j, *ps = m->prod + 3 * j;
        double ln_kf = m->lnA[j] + m->b[j] * lnT - m->Ea[j] / (ORC_RU_J * T);
        double dG = 0.0, dH = 0.0, Pf = 1.0, Pr = 1.0;
        for (int a = 0; a < 2; ++a) if (rs[a] >= 0) { dG -= g[rs[a]]; dH -= h[rs[a]]; Pf *= C[rs[a]]; }
        for (int a = 0; a < 3; ++a) if (ps[a] >= 0) { dG += g[ps[a]]; dH += h[ps[a]]; Pr *= C[ps[a]]; }
        const double sum_nu = (double)m->sum_nu[j];
        double ln_Kc = -dG + sum_nu * ln_patm_RT;
        double kf = exp(ln_kf), kr = exp(ln_kf - ln_Kc);
        double dlnkf = m->b[j] / T + m->Ea[j] / (ORC_RU_J * T * T);
        double dlnKc = (dH - sum_nu) / T;
        double dlnkr = dlnkf - dlnKc;
        double mj = 1.0;
        if (m->tb[j]) {
            mj = 0.0;
            for (int k = 0; k < N; ++k) mj += m->alpha[(size_t)j * N + k] * C[k];
        }
        double Delta = kf * Pf - kr * Pr;
        double q = mj * Delta;
        double dqdT = mj * (kf * dlnkf * Pf - kr * dlnkr * Pr);

        /* dq/dC_i for every i */
        for (int i = 0; i < N; ++i) dq[i] = m->tb[j] ? m->alpha[(size_t)j * N + i] * Delta : 0.0;
        for (int a = 0; a < 2; ++a) {
            if (rs[a] < 0) continue;
            double other = 1.0;
            for (int b2 = 0; b2 < 2; ++b2) if (b2 != a && rs[b2] >= 0) other *= C[rs[b2]];
            dq[rs[a]] += mj * kf * other;
        }
        for (int a = 0; a < 3; ++a) {
            if (ps[a] < 0) continue;
            double other = 1.0;
            for (int b3 = 0; b3 < 3; ++b3) if (b3 != a && ps[b3] >= 0) other *= C[ps[b3]];
            dq[ps[a]] -= mj * kr * other;
        }
        /* scatter nu_kj * (dq, dqdT, q) to the reactant and product rows */
        for (int a = 0; a < 5; ++a) {
            int k = a < 2 ? rs[a] : ps[a - 2];
            if (k < 0) continue;
            double nu = a < 2 ? -1.0 : 1.0;
            omega[k] += nu * q;
            JCT[k] += nu * dqdT;
            for (int i = 0; i < N; ++i) JC[(size_t)k * N + i] += nu * dq[i];
        }
    }

    double cpm = 0.0, dcpm = 0.0;
    for (int k = 0; k < N; ++k) {
        cpm += Y[k] * cp[k] * ORC_RU_ERG / m->W[k];
        dcpm += Y[k] * dcpR_dT(m->nasa + 7 * k, T) * ORC_RU_ERG / m->W[k];
    }
    double heat = 0.0;
    for (int k = 0; k < N; ++k) {
        fY[k] = m->W[k] * omega[k] / rho;
        heat += (h[k] * ORC_RU_ERG * T / m->W[k]) * fY[k];
    }
    const double fT = -heat / cpm;
    for (int k = 0; k < N; ++k) {
        double acc = 0.0;
        for (int l = 0; l < N; ++l) acc += JC[(size_t)k * N + l] * C[l];
        sk[k] = acc;
    }
    /* species rows */
    for (int k = 0; k < N; ++k) {
        double *row = J + (size_t)(1 + k) * n;
        row[0] = m->W[k] / rho * (JCT[k] - sk[k] / T) + fY[k] / T;
        for (int i = 0; i < N; ++i)
            row[1 + i] = (m->W[k] / m->W[i]) * JC[(size_t)k * N + i]
                       - (m->W[k] * Wbar / (rho * m->W[i])) * sk[k]
                       + fY[k] * Wbar / m->W[i];
    }
    /* temperature row */
    {
        double acc = 0.0, acc2 = 0.0;
        for (int k = 0; k < N; ++k) {
            double e = h[k] * ORC_RU_ERG * T / m->W[k];
            acc += e * J[(size_t)(1 + k) * n + 0];
            acc2 += (cp[k] * ORC_RU_ERG / m->W[k]) * fY[k];
        }
        J[0] = -(acc2 + acc) / cpm - fT * dcpm / cpm;
        for (int i = 0; i < N; ++i) {
            double a2 = 0.0;
            for (int k = 0; k < N; ++k)
                a2 += (h[k] * ORC_RU_ERG * T / m->W[k]) * J[(size_t)(1 + k) * n + 1 + i];
            J[1 + i] = -a2 / cpm - fT * (cp[i] * ORC_RU_ERG / m->W[i]) / cpm;
        }
    }
    free(JC);
    free(JCT);
}
