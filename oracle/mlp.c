/* Oracle of the learned surrogate — TEST INFRASTRUCTURE (see oracle.h).
 *
 * Not part of the paper, whose closest relative is tabulation (ISAT/TDAC,
 * Sec. 1, Sec. 5).  The surrogate advances one cell by dt with a multilayer
 * perceptron:
 *   features  x = (ln T, ln p, Y_1..Y_N, ln dt), normalised (x - mu_x)/sd_x,
 *             padded with zeros to IN_PAD,
 *   layers    h_{l} = GELU(W_l h_{l-1} + b_l), four hidden layers of width H,
 *             GELU(z) = z/2 (1 + erf(z / sqrt 2)),
 *   output    o = W_5 h_4 + b_5: the normalised increments in an inverse
 *             hyperbolic-sine scale, t = o * sd_o + mu_o,
 *             dY_k = S_Y sinh(t_k), dT = S_T sinh(t_N), S_Y = 1e-12, S_T = 1e-6 K,
 *             so that the network's error is relative to each increment's own
 *             size over the many decades the increments span (linear below
 *             S_Y and S_T, logarithmic above).
 * With bf16 emulation on, inputs, weights and hidden activations are rounded
 * to bfloat16 (round to nearest even) before each product, as the GPU path
 * stores them; every sum is accumulated in FP64.
 * Parameter blob (floats), layer by layer: W_l [out_pad x in_pad] then
 * b_l [out_pad]; then mu_x, sd_x, mu_o, sd_o, xmin, xmax (IN_PAD each).
 *
 * Conservation: the predicted state Y + dY is first clipped at zero, then
 * element conservation is restored by the correction that is smallest in the
 * metric weighted by the inverse of the clipped mass fractions,
 *   Y1 = max(Y + dY, 0),  delta_k = Y1_k (E^T lam)_k,
 *   (E W E^T) lam = E (Y1 - Y),  W = diag(Y1),  E_ek = a_ek / W_k,
 * so sum_k a_ek (Y1_k - delta_k - Y_k) / W_k = 0 for every element (and so
 * sum_k of the increments is 0), species clipped to zero stay at zero, and
 * each correction is proportional to the species' own mass fraction.  The
 * temperature then follows from h(T', Y') = h(T, Y) as for mapped cells. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#define IN_PAD 64
#define HID 256
#define OUT_PAD 64
#define S_Y 1e-12
#define S_T 1e-6

static const int dims[6] = {IN_PAD, HID, HID, HID, HID, OUT_PAD};

int64_t orc_mlp_param_count(void)
{
    int64_t n = 0;
    for (int l = 0; l < 5; ++l) n += (int64_t)dims[l + 1] * dims[l] + dims[l + 1];
    return n + 6 * IN_PAD;
}

/* value of the bfloat16 nearest to x (ties to even); NaN stays NaN */
double orc_bf16(double xd)
{
    float x = (float)xd;
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return xd;
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    float r;
    memcpy(&r, &u, 4);
    return (double)r;
}

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }
static double gelu_d(double z)
{
    return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
}

static const float *norm_block(const float *P) { return P + (orc_mlp_param_count() - 6 * IN_PAD); }

/* raw features of one cell: ln T, ln p, Y_1..Y_N, ln dt */
void orc_mlp_features(int N, double T, double p, const double *Y, double dt, double *x)
{
    for (int i = 0; i < IN_PAD; ++i) x[i] = 0.0;
    x[0] = log(T);
    x[1] = log(p);
    for (int k = 0; k < N; ++k) x[2 + k] = Y[k];
    x[2 + N] = log(dt);
}

/* forward for n cells of raw features X [n x IN_PAD]; out [n x OUT_PAD]
 * normalised outputs; acts (nullable) [n x 4 x HID] hidden activations,
 * pre [n x 5 x HID] (nullable) pre-activations */
void orc_mlp_forward(const float *P, int64_t n, int nfeat, const double *X, int bf16,
                     double *out, double *acts, double *pre)
{
    const float *nb = norm_block(P);
    const float *mu = nb, *sd = nb + IN_PAD;
    double *h = (double *)malloc(sizeof(double) * HID);
    double *hn = (double *)malloc(sizeof(double) * HID);
    for (int64_t c = 0; c < n; ++c) {
        double x[IN_PAD];
        for (int i = 0; i < IN_PAD; ++i) {
            double v = i < nfeat ? (X[c * IN_PAD + i] - mu[i]) / sd[i] : 0.0;
            x[i] = bf16 ? orc_bf16(v) : v;
        }
        const double *in = x;
        const float *Wp = P;
        for (int l = 0; l < 5; ++l) {
            const int ni = dims[l], no = dims[l + 1];
            const float *W = Wp, *b = Wp + (size_t)no * ni;
            for (int o = 0; o < no; ++o) {
                double acc = 0.0;
                for (int i = 0; i < ni; ++i) {
                    double w = bf16 ? orc_bf16(W[(size_t)o * ni + i]) : (double)W[(size_t)o * ni + i];
                    acc += w * in[i];
                }
                acc += b[o];
                if (l < 4) {
                    if (pre) pre[(c * 5 + l) * HID + o] = acc;
                    double g = gelu(acc);
                    hn[o] = bf16 ? orc_bf16(g) : g;
                } else {
                    out[c * OUT_PAD + o] = acc;
                }
            }
            if (l < 4) {
                memcpy(h, hn, sizeof(double) * HID);
                if (acts) memcpy(acts + (c * 4 + l) * HID, h, sizeof(double) * HID);
                in = h;
            }
            Wp += (size_t)no * ni + no;
        }
    }
    free(h);
    free(hn);
}

/* mean-squared error over n cells and the first nout outputs, and its
 * gradient with respect to every weight and bias (same layout as P, the
 * normalisation block left at zero).  Returns the loss. */
double orc_mlp_loss_grad(const float *P, int64_t n, int nfeat, int nout, const double *X,
                         const double *target, int bf16, double *grad)
{
    const int64_t np = orc_mlp_param_count();
    for (int64_t i = 0; i < np; ++i) grad[i] = 0.0;
    const float *nb = norm_block(P);
    const float *mu = nb, *sd = nb + IN_PAD;
    double *acts = (double *)malloc(sizeof(double) * 4 * HID);
    double *pre = (double *)malloc(sizeof(double) * 5 * HID);
    double out[OUT_PAD];
    double loss = 0.0;
    const double scale = 1.0 / ((double)n * nout);
    const float *Wl[5];
    double *Gl[5];
    {
        const float *Wp = P;
        double *Gp = grad;
        for (int l = 0; l < 5; ++l) {
            Wl[l] = Wp;
            Gl[l] = Gp;
            Wp += (size_t)dims[l + 1] * dims[l] + dims[l + 1];
            Gp += (size_t)dims[l + 1] * dims[l] + dims[l + 1];
        }
    }
    double dcur[HID], dnext[HID], x[IN_PAD];
    for (int64_t c = 0; c < n; ++c) {
        for (int i = 0; i < IN_PAD; ++i) {
            double v = i < nfeat ? (X[c * IN_PAD + i] - mu[i]) / sd[i] : 0.0;
            x[i] = bf16 ? orc_bf16(v) : v;
        }
        orc_mlp_forward(P, 1, nfeat, X + c * IN_PAD, bf16, out, acts, pre);
        /* output layer */
        for (int o = 0; o < OUT_PAD; ++o) {
            double d = 0.0;
            if (o < nout) {
                double e = out[o] - target[c * OUT_PAD + o];
                loss += e * e;
                d = 2.0 * e * scale;
            }
            dcur[o] = d;
        }
        for (int l = 4; l >= 0; --l) {
            const int ni = dims[l], no = dims[l + 1];
            const double *in = l == 0 ? x : acts + (size_t)(l - 1) * HID;
            const float *W = Wl[l];
            double *gW = Gl[l], *gb = Gl[l] + (size_t)no * ni;
            for (int o = 0; o < no; ++o) {
                gb[o] += dcur[o];
                for (int i = 0; i < ni; ++i) gW[(size_t)o * ni + i] += dcur[o] * in[i];
            }
            if (l == 0) break;
            for (int i = 0; i < ni; ++i) {
                double acc = 0.0;
                for (int o = 0; o < no; ++o) {
                    double w = bf16 ? orc_bf16(W[(size_t)o * ni + i]) : (double)W[(size_t)o * ni + i];
                    acc += dcur[o] * w;
                }
                dnext[i] = acc * gelu_d(pre[(size_t)(l - 1) * HID + i]);
            }
            memcpy(dcur, dnext, sizeof(double) * ni);
        }
    }
    free(acts);
    free(pre);
    return loss * scale;
}

/* Element conservation of a clipped prediction (see the header): Y1 (length
 * N, non-negative) is corrected in place towards conserving the elements of
 * Y0.  Returns 0, or 1 if E W E^T is singular (Y1 unchanged). */
int orc_conserve(const omech *m, const double *Y0, double *Y1)
{
    const int E = m->E, N = m->N;
    double G[64], r[8], lam[8];
    int piv[8];
    if (E > 8) return 1;
    for (int a = 0; a < E; ++a) {
        double s = 0.0;
        for (int k = 0; k < N; ++k) s += (double)m->comp[k * E + a] / m->W[k] * (Y1[k] - Y0[k]);
        r[a] = s;
        for (int b = 0; b < E; ++b) {
            double g = 0.0;
            for (int k = 0; k < N; ++k)
                g += (double)m->comp[k * E + a] / m->W[k] * Y1[k] * ((double)m->comp[k * E + b] / m->W[k]);
            G[a * E + b] = g;
        }
    }
    if (orc_lu(E, G, piv) != 0) return 1;
    memcpy(lam, r, sizeof(double) * E);
    orc_lu_solve(E, G, piv, lam);
    for (int k = 0; k < N; ++k) {
        double s = 0.0;
        for (int a = 0; a < E; ++a) s += (double)m->comp[k * E + a] / m->W[k] * lam[a];
        Y1[k] -= Y1[k] * s;
    }
    return 0;
}

/* One surrogate step for one cell (raw state in/out); returns 1 if the gate
 * accepts (state updated), 0 if the cell must go to the Rosenbrock solver.
 * Gate: T <= T_max, every raw feature inside the training box widened by
 * margin times its span, |dT| <= max_dT, E diag(Y1) E^T invertible,
 * Y' >= y_min, |T + dT - T'| <= tau_T. */
int orc_surrogate_cell(const omech *m, const float *P, double p, double *T, double *Y, double dt,
                       double tau_T, double y_min, double margin, double max_dT, double T_max)
{
    const int N = m->N;
    const float *nb = norm_block(P);
    const float *mu_o = nb + 2 * IN_PAD, *sd_o = nb + 3 * IN_PAD;
    const float *xmin = nb + 4 * IN_PAD, *xmax = nb + 5 * IN_PAD;
    double x[IN_PAD], out[OUT_PAD];
    if (!(*T <= T_max)) return 0;
    orc_mlp_features(N, *T, p, Y, dt, x);
    for (int i = 0; i < N + 3; ++i) {
        double span = (double)xmax[i] - (double)xmin[i];
        if (x[i] < xmin[i] - margin * span || x[i] > xmax[i] + margin * span) return 0;
    }
    orc_mlp_forward(P, 1, N + 3, x, 1, out, NULL, NULL);
    double Yn[N];
    for (int k = 0; k < N; ++k) {
        const double yk = Y[k] + S_Y * sinh(out[k] * sd_o[k] + mu_o[k]);
        Yn[k] = yk > 0.0 ? yk : 0.0;
    }
    const double dT = S_T * sinh(out[N] * sd_o[N] + mu_o[N]);
    if (!(fabs(dT) <= max_dT)) return 0;
    if (orc_conserve(m, Y, Yn) != 0) return 0;
    for (int k = 0; k < N; ++k)
        if (!(Yn[k] >= y_min)) return 0;
    const double h = orc_enthalpy_mass(m, *T, Y);
    const double Th = orc_temperature_from_enthalpy(m, h, Yn, *T + dT, NULL);
    if (!(fabs(*T + dT - Th) <= tau_T)) return 0;
    *T = Th;
    for (int k = 0; k < N; ++k) Y[k] = Yn[k];
    return 1;
}
