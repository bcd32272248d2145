/* Right-hand side of the constant-pressure adiabatic reactor — TEST INFRASTRUCTURE.
 *
 * Included twice by chem.c: once with SC = double and once with
 * SC = double complex (for the complex-step Jacobian), so both evaluate the
 * same formulas.  Required macros: SC, SC_EXP, SC_LOG, FN_RHS, FN_FALLOFF, FN_LNKF.
 *
 * State y = (T, Y_1..Y_N) at fixed pressure p.  With W-bar the mean molar
 * mass, rho = p W-bar / (R T) and C_k = rho Y_k / W_k:
 *   k_f,j  = exp(ln A_j + b_j ln T - Ea_j / (R T))
 *            or, for a pressure-dependent (PLOG) reaction with rate expressions
 *            k_i(T) tabulated at increasing pressures p_i (FN_LNKF):
 *              ln k_f = ln k_i + (ln p - ln p_i) / (ln p_i+1 - ln p_i) (ln k_i+1 - ln k_i)
 *            for p_i <= p < p_i+1, and k_1 below p_1, k_last at or above p_last
 *   ln Kc  = -sum_k nu_kj G_k/(RT) + (sum_k nu_kj) ln(p_atm / (R T))
 *   k_r,j  = exp(ln k_f,j - ln Kc,j)
 *   q_j    = m_j (k_f prod_reactants C - k_r prod_products C),
 *            m_j = [M]_j = sum_k alpha_kj C_k for third-body reactions, else 1;
 *            for fall-off reactions m_j = G([M]_j, T) instead (FN_FALLOFF):
 *            k_f is the high-pressure limit k_inf, and
 *              Pr = k0 [M] / k_inf,  k0 = A0 T^b0 exp(-Ea0 / (R T)),
 *              G  = Pr / (1 + Pr) F,
 *            F = 1 (Lindemann) or Troe's broadening factor:
 *              Fcent = (1 - a) exp(-T/T3) + a exp(-T/T1) + exp(-T2/T)  (last if T2 > 0)
 *              c = -0.4 - 0.67 log10 Fcent,  n = 0.75 - 1.27 log10 Fcent,  d = 0.14
 *              f1 = (log10 Pr + c) / (n - d (log10 Pr + c))
 *              log10 F = log10 Fcent / (1 + f1^2)
 *            (the reverse rate k_f / Kc carries the same factor)
 *   omega_k = sum_j nu_kj q_j
 *   dY_k/dt = W_k omega_k / rho
 *   dT/dt   = -sum_k H_k omega_k / (rho cp)      (cp mass specific)
 * Thermo (NASA-7 style, one range):
 *   cp/R = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4
 *   H/RT = a1 + a2 T/2 + a3 T^2/3 + a4 T^3/4 + a5 T^4/5 + a6/T
 *   S/R  = a1 ln T + a2 T + a3 T^2/2 + a4 T^3/3 + a5 T^4/4 + a7
 */

static SC FN_LNKF(const omech *m, int j, double p, SC T, SC lnT)
{
    const int cnt = m->plog_n ? m->plog_n[j] : 0;
    if (!cnt) return m->lnA[j] + m->b[j] * lnT - m->Ea[j] / (ORC_RU_J * T);
    const double *t = m->plog + (size_t)32 * j;      /* p_i, A_i, b_i, Ea_i */
    int i = 0;
    if (p >= t[4 * (cnt - 1)]) i = cnt - 1;
    else while (i + 1 < cnt && p >= t[4 * (i + 1)]) ++i;
    const SC lk = log(t[4 * i + 1]) + t[4 * i + 2] * lnT - t[4 * i + 3] / (ORC_RU_J * T);
    if (p < t[0] || i == cnt - 1) return lk;         /* outside the table: end entry */
    const SC lk1 = log(t[4 * i + 5]) + t[4 * i + 6] * lnT - t[4 * i + 7] / (ORC_RU_J * T);
    const double w = (log(p) - log(t[4 * i])) / (log(t[4 * i + 4]) - log(t[4 * i]));
    return lk + w * (lk1 - lk);
}

static SC FN_FALLOFF(const omech *m, int j, SC T, SC lnT, SC kinf, SC M)
{
    const double *fp = m->fo + (size_t)7 * j;
    const SC k0 = SC_EXP(log(fp[0]) + fp[1] * lnT - fp[2] / (ORC_RU_J * T));
    const SC Pr = k0 * M / kinf;
    SC G = Pr / (1.0 + Pr);
    if (m->fo_type[j] == 2) {
        SC Fc = (1.0 - fp[3]) * SC_EXP(-T / fp[4]) + fp[3] * SC_EXP(-T / fp[5]);
        if (fp[6] > 0.0) Fc += SC_EXP(-fp[6] / T);
        const double ln10 = log(10.0);
        const SC lFc = SC_LOG(Fc) / ln10;
        const SC c = -0.4 - 0.67 * lFc, nn = 0.75 - 1.27 * lFc;
        const SC x = SC_LOG(Pr) / ln10 + c;
        const SC f1 = x / (nn - 0.14 * x);
        G *= SC_EXP(ln10 * lFc / (1.0 + f1 * f1));
    }
    return G;
}

static void FN_RHS(const omech *m, double p, const SC *y, SC *f)
{
    const int N = m->N, R = m->R;
    const SC T = y[0];
    const SC *Y = y + 1;
    const SC lnT = SC_LOG(T);
    SC h_RT[N], g_RT[N], cp_R[N], C[N], omega[N];

    for (int k = 0; k < N; ++k) {
        const double *a = m->nasa + 7 * k;
        SC cp = a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
        SC h = a[0] + a[1] * T / 2.0 + a[2] * T * T / 3.0 + a[3] * T * T * T / 4.0
             + a[4] * T * T * T * T / 5.0 + a[5] / T;
        SC s = a[0] * lnT + a[1] * T + a[2] * T * T / 2.0 + a[3] * T * T * T / 3.0
             + a[4] * T * T * T * T / 4.0 + a[6];
        cp_R[k] = cp;
        h_RT[k] = h;
        g_RT[k] = h - s;
    }

    SC sumYW = 0.0;
    for (int k = 0; k < N; ++k) sumYW += Y[k] / m->W[k];
    const SC Wbar = 1.0 / sumYW;
    const SC rho = p * Wbar / (ORC_RU_ERG * T);
    for (int k = 0; k < N; ++k) {
        C[k] = rho * Y[k] / m->W[k];
        omega[k] = 0.0;
    }

    const SC ln_patm_RT = SC_LOG(ORC_P_ATM / (ORC_RU_ERG * T));
    for (int j = 0; j < R; ++j) {
        const int *rs = m->reac + 2 * j, *ps = m->prod + 3 * j;
        SC ln_kf = FN_LNKF(m, j, p, T, lnT);
        SC dG = 0.0;
        SC Pf = 1.0, Pr = 1.0;
        for (int s = 0; s < 2; ++s) if (rs[s] >= 0) { dG -= g_RT[rs[s]]; Pf *= C[rs[s]]; }
        for (int s = 0; s < 3; ++s) if (ps[s] >= 0) { dG += g_RT[ps[s]]; Pr *= C[ps[s]]; }
        SC ln_Kc = -dG + (double)m->sum_nu[j] * ln_patm_RT;
        SC kf = SC_EXP(ln_kf);
        SC kr = SC_EXP(ln_kf - ln_Kc);
        SC mj = 1.0;
        if (m->tb[j]) {
            mj = 0.0;
            for (int k = 0; k < N; ++k) mj += m->alpha[(size_t)j * N + k] * C[k];
        }
        if (m->fo_type[j]) mj = FN_FALLOFF(m, j, T, lnT, kf, mj);
        SC q = mj * (kf * Pf - kr * Pr);
        for (int s = 0; s < 2; ++s) if (rs[s] >= 0) omega[rs[s]] -= q;
        for (int s = 0; s < 3; ++s) if (ps[s] >= 0) omega[ps[s]] += q;
    }

    SC cp_mass = 0.0;
    for (int k = 0; k < N; ++k) cp_mass += Y[k] * cp_R[k] * ORC_RU_ERG / m->W[k];
    SC heat = 0.0;
    for (int k = 0; k < N; ++k) {
        f[1 + k] = m->W[k] * omega[k] / rho;
        heat += (h_RT[k] * ORC_RU_ERG * T / m->W[k]) * f[1 + k];
    }
    f[0] = -heat / cp_mass;
}
