/* Host driver for the sanitizer build of the CPU oracle (test infrastructure).
 *
 * Built with gcc -fsanitize=address,undefined together with the oracle's C
 * sources by tests/test_host_sanitizers.py, it reads a mechanism and a few
 * cell states from a binary file, calls every entry point of oracle.h on
 * them, and prints each result as "name count v0 v1 ..." (%.17g), so that
 * the test can compare the values with the regular build of the oracle.
 *
 * Input layout (little-endian, written by the test):
 *   int32 E, N, R, n_eff, has_plog, ncells, n_param
 *   f64 elem_mass[E]; i32 comp[N*E]; f64 W[N]; f64 nasa[N*7];
 *   i32 reac[R*2]; i32 prod[R*3]; f64 A[R], b[R], Ea[R]; i32 tb[R];
 *   i32 eff_r[n_eff], eff_s[n_eff]; f64 eff_v[n_eff];
 *   i32 fo_type[R]; f64 fo[R*7];
 *   (has_plog) i32 plog_n[R]; f64 plog[R*32];
 *   f64 p, dt; f64 T[ncells]; f64 Y[N*ncells] (species-major);
 *   f64 Yfuel[N], Yox[N]; f32 params[n_param]
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

static FILE *in_f;

static void *rd(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, in_f) != bytes) {
        fprintf(stderr, "driver: short input\n");
        exit(2);
    }
    return p;
}

static void put(const char *name, const double *v, int64_t n)
{
    printf("%s %lld", name, (long long)n);
    for (int64_t i = 0; i < n; ++i) printf(" %.17g", v[i]);
    printf("\n");
}

static void put_i(const char *name, const int *v, int64_t n)
{
    printf("%s %lld", name, (long long)n);
    for (int64_t i = 0; i < n; ++i) printf(" %d", v[i]);
    printf("\n");
}

int main(int argc, char **argv)
{
    if (argc != 2) {
        fprintf(stderr, "usage: %s input.bin\n", argv[0]);
        return 2;
    }
    in_f = fopen(argv[1], "rb");
    if (!in_f) return 2;
    int32_t *hdr = (int32_t *)rd(7 * sizeof(int32_t));
    const int E = hdr[0], N = hdr[1], R = hdr[2], n_eff = hdr[3], has_plog = hdr[4];
    const int ncells = hdr[5];
    const int64_t n_param = hdr[6];
    const int n = N + 1;

    double *elem_mass = (double *)rd(sizeof(double) * E);
    int32_t *comp = (int32_t *)rd(sizeof(int32_t) * N * E);
    double *W = (double *)rd(sizeof(double) * N);
    double *nasa = (double *)rd(sizeof(double) * N * 7);
    int32_t *reac = (int32_t *)rd(sizeof(int32_t) * R * 2);
    int32_t *prod = (int32_t *)rd(sizeof(int32_t) * R * 3);
    double *A = (double *)rd(sizeof(double) * R);
    double *b = (double *)rd(sizeof(double) * R);
    double *Ea = (double *)rd(sizeof(double) * R);
    int32_t *tb = (int32_t *)rd(sizeof(int32_t) * R);
    int32_t *eff_r = (int32_t *)rd(sizeof(int32_t) * n_eff);
    int32_t *eff_s = (int32_t *)rd(sizeof(int32_t) * n_eff);
    double *eff_v = (double *)rd(sizeof(double) * n_eff);
    int32_t *fo_type = (int32_t *)rd(sizeof(int32_t) * R);
    double *fo = (double *)rd(sizeof(double) * R * 7);
    int32_t *plog_n = NULL;
    double *plog = NULL;
    if (has_plog) {
        plog_n = (int32_t *)rd(sizeof(int32_t) * R);
        plog = (double *)rd(sizeof(double) * R * 32);
    }
    double *pdt = (double *)rd(2 * sizeof(double));
    const double p = pdt[0], dt = pdt[1];
    double *T = (double *)rd(sizeof(double) * ncells);
    double *Y = (double *)rd(sizeof(double) * (size_t)N * ncells);
    double *Yfuel = (double *)rd(sizeof(double) * N);
    double *Yox = (double *)rd(sizeof(double) * N);
    float *P = (float *)rd(sizeof(float) * n_param);
    fclose(in_f);

    omech *m = NULL;
    if (orc_mech_create(&m, E, N, R, elem_mass, comp, W, nasa, reac, prod, A, b, Ea, tb, n_eff,
                        eff_r, eff_s, eff_v, fo_type, fo) != 0) {
        fprintf(stderr, "driver: orc_mech_create failed\n");
        return 3;
    }
    if (has_plog && orc_mech_set_plog(m, plog_n, plog) != 0) {
        fprintf(stderr, "driver: orc_mech_set_plog failed\n");
        return 3;
    }

    /* the state of cell 0 */
    double *y0 = (double *)malloc(sizeof(double) * n);
    double *Y0 = y0 + 1;
    y0[0] = T[0];
    for (int k = 0; k < N; ++k) y0[1 + k] = Y[(size_t)k * ncells];

    double *cp = (double *)malloc(sizeof(double) * N);
    double *hrt = (double *)malloc(sizeof(double) * N);
    double *sr = (double *)malloc(sizeof(double) * N);
    orc_thermo(m, T[0], cp, hrt, sr);
    put("thermo_cp", cp, N);
    put("thermo_h", hrt, N);
    put("thermo_s", sr, N);

    double *lnkf = (double *)malloc(sizeof(double) * R);
    double *G = (double *)malloc(sizeof(double) * R);
    for (int j = 0; j < R; ++j) {
        lnkf[j] = orc_ln_kf(m, j, T[0], p);
        G[j] = orc_falloff_factor(m, j, T[0], 1e-5);
    }
    put("ln_kf", lnkf, R);
    put("falloff", G, R);

    double *kf = (double *)malloc(sizeof(double) * R), *kr = (double *)malloc(sizeof(double) * R);
    double *q = (double *)malloc(sizeof(double) * R), *om = (double *)malloc(sizeof(double) * N);
    orc_kinetics(m, T[0], p, Y0, kf, kr, q, om);
    put("kin_q", q, R);
    put("kin_omega", om, N);

    double *f = (double *)malloc(sizeof(double) * n);
    orc_rhs(m, p, y0, f);
    put("rhs", f, n);
    double *J = (double *)malloc(sizeof(double) * n * n);
    orc_jac(m, p, y0, J);
    put("jac", J, (int64_t)n * n);
    double *Jc = (double *)malloc(sizeof(double) * n * n);
    orc_jac_cs(m, p, y0, Jc);
    put("jac_cs", Jc, (int64_t)n * n);
    double *v = (double *)malloc(sizeof(double) * n), *fre = (double *)malloc(sizeof(double) * n);
    double *fim = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) v[i] = (i % 3 == 0) ? 1.0 : -0.5;
    orc_rhs_cs_dir(m, p, y0, v, 1e-30, fre, fim);
    put("rhs_cs_im", fim, n);

    double mix[4];
    mix[0] = orc_enthalpy_mass(m, T[0], Y0);
    mix[1] = orc_cp_mass(m, T[0], Y0);
    mix[2] = orc_density(m, T[0], p, Y0);
    int iters = 0;
    mix[3] = orc_temperature_from_enthalpy(m, mix[0], Y0, T[0] + 50.0, &iters);
    put("mixture", mix, 4);

    /* dense LU of the iteration matrix I/(gamma h) - J */
    double a36[36], c36[36], gam;
    orc_rodas4_coeffs(a36, c36, &gam);
    put("rodas_a", a36, 36);
    const double h = dt / 10.0;
    double *M = (double *)malloc(sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) M[i] = -J[i];
    for (int i = 0; i < n; ++i) M[i * n + i] += 1.0 / (gam * h);
    int *piv = (int *)malloc(sizeof(int) * n);
    const int lu_rc = orc_lu(n, M, piv);
    double *rhs_b = (double *)malloc(sizeof(double) * n);
    memcpy(rhs_b, f, sizeof(double) * n);
    if (lu_rc == 0) orc_lu_solve(n, M, piv, rhs_b);
    put("lu_solve", rhs_b, n);

    double *yn = (double *)malloc(sizeof(double) * n), *err = (double *)malloc(sizeof(double) * n);
    const int st_rc = orc_rodas4_step(m, p, y0, f, J, h, yn, err);
    put("rodas_ynew", yn, n);
    put("rodas_err", err, n);
    printf("rodas_rc 1 %d\n", st_rc);

    oopts o = {1e-8, 1e-12, 100000, 1e-14, 0};
    double *yc = (double *)malloc(sizeof(double) * n);
    memcpy(yc, y0, sizeof(double) * n);
    double h_io = 0.0;
    ostats st;
    orc_integrate_cell(m, p, yc, dt, &o, &h_io, &st);
    put("cell_y", yc, n);
    put("cell_h", &h_io, 1);
    const int cst[6] = {st.n_accept, st.n_reject, st.n_jac, st.n_lu, st.n_rhs, st.status};
    put_i("cell_stats", cst, 6);

    double *yr = (double *)malloc(sizeof(double) * n);
    memcpy(yr, y0, sizeof(double) * n);
    orc_rk4(m, p, yr, dt / 100.0, 50);
    put("rk4", yr, n);

    /* batch over every cell, static and dynamic schedules, two threads */
    double *pc = (double *)malloc(sizeof(double) * ncells);
    for (int c = 0; c < ncells; ++c) pc[c] = p;
    for (int sched = 0; sched < 2; ++sched) {
        double *Tb = (double *)malloc(sizeof(double) * ncells);
        double *Yb = (double *)malloc(sizeof(double) * (size_t)N * ncells);
        double *hb = (double *)calloc((size_t)ncells, sizeof(double));
        uint8_t *sb = (uint8_t *)calloc((size_t)ncells, 1);
        int32_t *na = (int32_t *)calloc((size_t)ncells, sizeof(int32_t));
        int32_t *nr = (int32_t *)calloc((size_t)ncells, sizeof(int32_t));
        memcpy(Tb, T, sizeof(double) * ncells);
        memcpy(Yb, Y, sizeof(double) * (size_t)N * ncells);
        orc_integrate_batch(m, ncells, Tb, pc, Yb, dt, &o, hb, NULL, sb, na, nr, 2, sched);
        put(sched ? "batch_T_dyn" : "batch_T_static", Tb, ncells);
        put(sched ? "batch_Y_dyn" : "batch_Y_static", Yb, (int64_t)N * ncells);
        int *ns = (int *)malloc(sizeof(int) * ncells);
        for (int c = 0; c < ncells; ++c) ns[c] = na[c] + nr[c] + 1000 * sb[c];
        put_i(sched ? "batch_steps_dyn" : "batch_steps_static", ns, ncells);
        free(ns);
        free(Tb); free(Yb); free(hb); free(sb); free(na); free(nr);
    }

    /* reference mapping and the mapped-cell update */
    double *w = (double *)malloc(sizeof(double) * N), bf, bo;
    orc_map_weights(m, Yfuel, Yox, w, &bf, &bo);
    double *Z = (double *)malloc(sizeof(double) * ncells);
    orc_mixture_fraction(m, ncells, Y, w, bf, bo, Z);
    put("mix_frac", Z, ncells);
    uint8_t *flags = (uint8_t *)calloc((size_t)ncells, 1);
    const int64_t ref = orc_map_reference(m, ncells, T, Y, w, bf, bo, 1e-2, 1.0, 0, flags);
    int *fl = (int *)malloc(sizeof(int) * (ncells + 1));
    for (int c = 0; c < ncells; ++c) fl[c] = flags[c];
    fl[ncells] = (int)ref;
    put_i("map_flags", fl, ncells + 1);
    double *Tm = (double *)malloc(sizeof(double) * ncells);
    double *Ym = (double *)malloc(sizeof(double) * (size_t)N * ncells);
    memcpy(Tm, T, sizeof(double) * ncells);
    memcpy(Ym, Y, sizeof(double) * (size_t)N * ncells);
    for (int c = 0; c < ncells; ++c) flags[c] = (uint8_t)(c % 2 ? 2 : 0);
    orc_map_scatter(m, ncells, Tm, Ym, flags, Y0, yc + 1);
    put("map_T", Tm, ncells);
    put("map_Y", Ym, (int64_t)N * ncells);

    /* surrogate: features, forward (both arithmetic modes, with the
     * activation buffers), loss gradient, conservation, gate */
    if (orc_mlp_param_count() != n_param) {
        fprintf(stderr, "driver: parameter count mismatch\n");
        return 4;
    }
    double *X = (double *)calloc((size_t)ncells * 64, sizeof(double));
    for (int c = 0; c < ncells; ++c) {
        double *Yc = (double *)malloc(sizeof(double) * N);
        for (int k = 0; k < N; ++k) Yc[k] = Y[(size_t)k * ncells + c];
        orc_mlp_features(N, T[c], p, Yc, dt, X + (size_t)c * 64);
        free(Yc);
    }
    put("mlp_x", X, (int64_t)ncells * 64);
    double *out = (double *)calloc((size_t)ncells * 64, sizeof(double));
    double *acts = (double *)calloc((size_t)ncells * 4 * 256, sizeof(double));
    double *pre = (double *)calloc((size_t)ncells * 5 * 256, sizeof(double));
    orc_mlp_forward(P, ncells, N + 3, X, 1, out, acts, pre);
    put("mlp_out_bf16", out, (int64_t)ncells * 64);
    orc_mlp_forward(P, ncells, N + 3, X, 0, out, NULL, NULL);
    put("mlp_out_f64", out, (int64_t)ncells * 64);
    double *target = (double *)calloc((size_t)ncells * 64, sizeof(double));
    double *grad = (double *)calloc((size_t)n_param, sizeof(double));
    double loss = orc_mlp_loss_grad(P, ncells, N + 3, N + 1, X, target, 0, grad);
    put("mlp_loss", &loss, 1);
    double gsum = 0.0;
    for (int64_t i = 0; i < n_param; ++i) gsum += grad[i] * grad[i];
    put("mlp_grad_sq", &gsum, 1);

    double *Y1 = (double *)malloc(sizeof(double) * N);
    memcpy(Y1, yc + 1, sizeof(double) * N);
    const int crc = orc_conserve(m, Y0, Y1);
    put("conserve", Y1, N);
    printf("conserve_rc 1 %d\n", crc);
    int *gate = (int *)malloc(sizeof(int) * ncells);
    double *Tg = (double *)malloc(sizeof(double) * ncells);
    for (int c = 0; c < ncells; ++c) {
        double Tc = T[c];
        double *Yc = (double *)malloc(sizeof(double) * N);
        for (int k = 0; k < N; ++k) Yc[k] = Y[(size_t)k * ncells + c];
        gate[c] = orc_surrogate_cell(m, P, p, &Tc, Yc, dt, 0.5, -1e-10, 0.0, 1.0, 1000.0);
        Tg[c] = Tc;
        free(Yc);
    }
    put_i("gate", gate, ncells);
    put("gate_T", Tg, ncells);

    double bfv[3] = {orc_bf16(1.0 / 3.0), orc_bf16(-2.5e-3), orc_bf16(7.0e5)};
    put("bf16", bfv, 3);

    orc_mech_destroy(m);
    free(hdr); free(elem_mass); free(comp); free(W); free(nasa); free(reac); free(prod);
    free(A); free(b); free(Ea); free(tb); free(eff_r); free(eff_s); free(eff_v); free(fo_type);
    free(fo); free(plog_n); free(plog); free(pdt); free(T); free(Y); free(Yfuel); free(Yox);
    free(P); free(y0); free(cp); free(hrt); free(sr); free(lnkf); free(G); free(kf); free(kr);
    free(q); free(om); free(f); free(J); free(Jc); free(v); free(fre); free(fim); free(M);
    free(piv); free(rhs_b); free(yn); free(err); free(yc); free(yr); free(pc); free(w); free(Z);
    free(flags); free(fl); free(Tm); free(Ym); free(X); free(out); free(acts); free(pre);
    free(target); free(grad); free(Y1); free(gate); free(Tg);
    return 0;
}
