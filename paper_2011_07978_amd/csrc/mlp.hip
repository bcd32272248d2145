// Learned surrogate for the per-cell dt-advance: BF16-MFMA MLP training and
// inference, element conservation and acceptance gate.
//
// Network: features x = (ln T, ln p, Y_1..Y_N, ln dt), normalised and padded
// to 64, four hidden layers of 256 with GELU (erf form), output 64 of which
// the first N+1 are the normalised increments in an inverse hyperbolic-sine
// scale: t = o sd_o + mu_o, dY_k = S_Y sinh(t_k), dT = S_T sinh(t_N).
// Weights and activations are bfloat16, products accumulate in FP32 on the
// matrix cores (v_mfma_f32_16x16x32_bf16), biases and GELU in FP32.
// Training: mean-squared error on the normalised outputs, Adam on FP32 master
// weights.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <random>
#include <vector>

#include "mech_dev.hpp"
#include "surrogate.hpp"

namespace chem {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float gelu_f(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_df(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ------------------------------------------------------------------ GEMM ----
// C[m][n] = sum_k A[m][k] B[n][k]  (A: M x K, B: N x K, bf16, k contiguous).
// Workgroup tile 64 x 64, four waves of 32 x 32, each 2 x 2 MFMA 16x16x32 blocks.
// MFMA operand layout (gfx950, checked on hardware): lane l holds A row l%16,
// k = 8(l/16)..+7; B column l%16, same k; D rows 4(l/16)+i, column l%16.
enum { EPI_HID = 0, EPI_OUT = 1, EPI_PLAIN = 2, EPI_OUT_T = 3 };
struct GemmEpi {
    const float *bias;
    uint16_t *H; int ldh;      // bf16 GELU output
    uint16_t *HT; int ldht;    // bf16 GELU output, transposed (nullable)
    float *Z; int ldz;         // f32 pre-activation (nullable)
    float *C; int ldc;         // f32 output
};

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(const uint16_t *__restrict__ A, int lda,
                                                 const uint16_t *__restrict__ B, int ldb, int M,
                                                 int N, int K, GemmEpi e) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64 + (w >> 1) * 32, n0 = blockIdx.y * 64 + (w & 1) * 32;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    // split-K launches (gridDim.z > 1): slice z covers k in [zK, (z+1)K) and
    // writes its partial product to its own M x ldc slab of C
    A += (size_t)blockIdx.z * K;
    B += (size_t)blockIdx.z * K;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero8 = {};
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row = m0 + 16 * i + r16;
            a[i] = row < M ? *(const bf16x8 *)(A + (size_t)row * lda + k0 + kq) : zero8;
            const int col = n0 + 16 * i + r16;
            b[i] = col < N ? *(const bf16x8 *)(B + (size_t)col * ldb + k0 + kq) : zero8;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + 16 * i + 4 * (lane >> 4) + r;
                const int col = n0 + 16 * j + r16;
                if (row >= M || col >= N) continue;
                const float v = acc[i][j][r];
                if (EPI == EPI_HID) {
                    const float z = v + e.bias[col];
                    const uint16_t g = f2bf(gelu_f(z));
                    e.H[(size_t)row * e.ldh + col] = g;
                    if (e.HT) e.HT[(size_t)col * e.ldht + row] = g;
                    if (e.Z) e.Z[(size_t)row * e.ldz + col] = z;
                } else if (EPI == EPI_OUT) {
                    e.C[(size_t)row * e.ldc + col] = v + e.bias[col];
                } else if (EPI == EPI_OUT_T) {
                    e.C[(size_t)col * e.ldc + row] = v + e.bias[col];
                } else {
                    e.C[((size_t)blockIdx.z * M + row) * e.ldc + col] = v;
                }
            }
}

template <int EPI>
static void gemm(const uint16_t *A, int lda, const uint16_t *B, int ldb, int M, int N, int K,
                 const GemmEpi &e, hipStream_t s) {
    dim3 grid((M + 63) / 64, (N + 63) / 64);
    hipLaunchKernelGGL(k_gemm_nt<EPI>, grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, e);
}

// dst[i] = sum over z of part[z][i], slices added in order
__global__ __launch_bounds__(256) void k_sum_slices(const float *part, int S, int64_t n, float *dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int z = 0; z < S; ++z) s += part[(size_t)z * n + i];
    dst[i] = s;
}

// ------------------------------------------------------------- features ----
__device__ __forceinline__ double raw_feature(const FeatSrc &f, int64_t i, int c) {
    if (c == 0) return log(f.T[i]);
    if (c == 1) return log(f.p[i]);
    if (c < f.N + 2) return f.Y[(int64_t)(c - 2) * f.n + i];
    if (c == f.N + 2) return log(f.dt_scalar > 0.0 ? f.dt_scalar : f.dt[i]);
    return 0.0;
}

// per-feature sum, sum of squares, min, max (FP64), one block per feature
__global__ __launch_bounds__(256) void k_feature_moments(FeatSrc f, int ncol, double *out) {
    const int c = blockIdx.x;
    double s = 0.0, s2 = 0.0, mn = INFINITY, mx = -INFINITY;
    for (int64_t i = threadIdx.x; i < f.n; i += blockDim.x) {
        const double v = raw_feature(f, i, c);
        s += v;
        s2 += v * v;
        mn = fmin(mn, v);
        mx = fmax(mx, v);
    }
    __shared__ double sh[4][256];
    sh[0][threadIdx.x] = s; sh[1][threadIdx.x] = s2; sh[2][threadIdx.x] = mn; sh[3][threadIdx.x] = mx;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
            sh[2][threadIdx.x] = fmin(sh[2][threadIdx.x], sh[2][threadIdx.x + st]);
            sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[4 * c] = sh[0][0]; out[4 * c + 1] = sh[1][0];
        out[4 * c + 2] = sh[2][0]; out[4 * c + 3] = sh[3][0];
    }
}

// targets: the increments dY_k = Y1_k - Y0_k (k < N) and dT = T1 - T0
// Increments in the network's output scale: asinh(dY_k / S_Y), asinh(dT / S_T).
constexpr double S_Y = 1e-12, S_T = 1e-6;
__device__ __forceinline__ double raw_target(const TgtSrc &t, int64_t i, int c) {
    if (c < t.N) return asinh((t.Y1[(int64_t)c * t.n + i] - t.Y0[(int64_t)c * t.n + i]) / S_Y);
    return asinh((t.T1[i] - t.T0[i]) / S_T);
}
__global__ __launch_bounds__(256) void k_target_moments(TgtSrc t, double *out) {
    const int c = blockIdx.x;
    double s = 0.0, s2 = 0.0;
    for (int64_t i = threadIdx.x; i < t.n; i += blockDim.x) {
        const double v = raw_target(t, i, c);
        s += v;
        s2 += v * v;
    }
    __shared__ double sh[2][256];
    sh[0][threadIdx.x] = s; sh[1][threadIdx.x] = s2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[2 * c] = sh[0][0]; out[2 * c + 1] = sh[1][0]; }
}

// rows r < B of the batch from samples idx[r] (nullable: base + r):
// X[r][c] bf16 normalised features, XT[c][r] its transpose (nullable),
// Tg[r][c] normalised targets (nullable)
__global__ __launch_bounds__(256) void k_build_rows(FeatSrc f, TgtSrc t, const int *idx, int64_t base,
                                                    int B, const float *norm, uint16_t *X,
                                                    uint16_t *XT, int ldxt, float *Tg) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int c = threadIdx.x & 63;
    if (r >= B) return;
    const int64_t i = idx ? (int64_t)idx[r] : base + r;
    const int nfeat = f.N + 3;
    uint16_t v = 0;
    if (c < nfeat) v = f2bf((float)((raw_feature(f, i, c) - norm[c]) / norm[64 + c]));
    X[(size_t)r * S_IN + c] = v;
    if (XT) XT[(size_t)c * ldxt + r] = v;
    if (Tg) {
        float tv = 0.0f;
        if (c < t.N + 1) tv = (float)((raw_target(t, i, c) - norm[128 + c]) / norm[192 + c]);
        Tg[(size_t)r * S_OUT + c] = tv;
    }
}

// ------------------------------------------------------------- backward ----
// dO = 2 (out - target) / (B * nout) for the first nout columns, 0 elsewhere
__global__ __launch_bounds__(256) void k_out_grad(const float *out, const float *Tg, int B, int nout,
                                                  float *dOf, uint16_t *dZ, uint16_t *dZT, int ldt,
                                                  double *loss_part) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int c = threadIdx.x & 63;
    float g = 0.0f;
    double l2 = 0.0;
    if (r < B && c < nout) {
        const float e = out[(size_t)r * S_OUT + c] - Tg[(size_t)r * S_OUT + c];
        g = 2.0f * e / ((float)B * (float)nout);
        l2 = (double)e * e;
    }
    if (r < B) {
        dOf[(size_t)r * S_OUT + c] = g;
        const uint16_t gb = f2bf(g);
        dZ[(size_t)r * S_OUT + c] = gb;
        dZT[(size_t)c * ldt + r] = gb;
    }
    // squared errors of the block's rows, added to the block's own running sum
    for (int m = 32; m > 0; m >>= 1) l2 += __shfl_xor(l2, m);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = l2;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] += (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// loss[0] = sum of the n per-block running sums (one block, fixed order)
__global__ __launch_bounds__(256) void k_sum_loss(const double *part, int n, double *loss) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = sh[0];
}

// Column sums of src [B x ncol] (bias gradients) in two fixed-order passes:
// block (x, y) sums rows y, y + CS_CHUNKS, ... of 64 columns into part[y][c]
// (four row phases per block, combined in order); then one thread per column
// adds the CS_CHUNKS partial sums in order.
constexpr int CS_CHUNKS = 64;
// slices of a split-K weight gradient: at most 256 workgroups of 64 x 64
// outputs, so S M N <= 256 * 4096
constexpr int64_t kSplitFloats = (int64_t)256 * 4096;
__global__ __launch_bounds__(256) void k_colsum_part(const float *src, int B, int ncol, float *part) {
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
    float s = 0.0f;
    if (c < ncol)
        for (int r = blockIdx.y + CS_CHUNKS * ph; r < B; r += 4 * CS_CHUNKS) s += src[(size_t)r * ncol + c];
    __shared__ float sh[4][64];
    sh[ph][threadIdx.x & 63] = s;
    __syncthreads();
    if (ph == 0 && c < ncol)
        part[(size_t)blockIdx.y * ncol + c] = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) +
                                              (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}
// dZ = dH * GELU'(Z) of a hidden layer as bf16 (+ transpose) and the partial
// column sums of the FP32 dZ (the bias gradient): block (x, y) covers 64
// columns and visits rows in the order of k_colsum_part, so the partial sums
// are the ones k_colsum_part would form from an FP32 copy of dZ
__global__ __launch_bounds__(256) void k_gelu_back(const float *dH, const float *Z, int B,
                                                   uint16_t *dZ, uint16_t *dZT, int ldt, float *part) {
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
    float s = 0.0f;
    for (int r = blockIdx.y + CS_CHUNKS * ph; r < B; r += 4 * CS_CHUNKS) {
        const size_t t = (size_t)r * S_HID + c;
        const float g = dH[t] * gelu_df(Z[t]);
        s += g;
        const uint16_t gb = f2bf(g);
        dZ[t] = gb;
        dZT[(size_t)c * ldt + r] = gb;
    }
    __shared__ float sh[4][64];
    sh[ph][threadIdx.x & 63] = s;
    __syncthreads();
    if (ph == 0)
        part[(size_t)blockIdx.y * S_HID + c] = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) +
                                               (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}
__global__ __launch_bounds__(256) void k_colsum_final(const float *part, int ncol, float *dst) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= ncol) return;
    float s = 0.0f;
    for (int y = 0; y < CS_CHUNKS; ++y) s += part[(size_t)y * ncol + c];
    dst[c] = s;
}

// where each layer's weights sit in the FP32 blob and their bf16 copies
struct WeightCopies {
    int64_t off[5];
    int no[5], ni[5];
    uint16_t *Wb[5], *WbT[5];
};

// Adam on the FP32 masters; a weight (not a bias) is also written to its
// layer's bf16 copy Wb [no x ni] and transpose WbT [ni x no]
__global__ __launch_bounds__(256) void k_adam(float *P, const float *G, float *m, float *v, int64_t n,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2, WeightCopies wc) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float p = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    P[i] = p;
    int64_t off = wc.off[0];
    int no = wc.no[0], ni = wc.ni[0];
    uint16_t *wb = wc.Wb[0], *wbt = wc.WbT[0];
#pragma unroll
    for (int q = 1; q < 5; ++q)
        if (i >= wc.off[q]) { off = wc.off[q]; no = wc.no[q]; ni = wc.ni[q]; wb = wc.Wb[q]; wbt = wc.WbT[q]; }
    const int64_t t = i - off;
    if (t < (int64_t)no * ni) {
        const int o = (int)(t / ni), k = (int)(t % ni);
        const uint16_t b = f2bf(p);
        wb[t] = b;
        wbt[(size_t)k * no + o] = b;
    }
}

// bf16 copies of a layer's weights: Wb [no x ni] and WbT [ni x no]
__global__ __launch_bounds__(256) void k_refresh(const float *W, int no, int ni, uint16_t *Wb,
                                                 uint16_t *WbT) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= no * ni) return;
    const int o = t / ni, i = t % ni;
    const uint16_t b = f2bf(W[t]);
    Wb[t] = b;
    WbT[(size_t)i * no + o] = b;
}

// ------------------------------------------------- conservation + gate ----
struct PostParams {
    int N, nel;
    const double *E;       // [nel][N] a_ek / W_k
    const double *nasa_t;  // species thermo [14][N] (a1..a7, a2/2, a3/3, a4/4, a5/5, ...)
    const double *invW;
    const float *norm;     // mu_x, sd_x, mu_o, sd_o, xmin, xmax
    double tau_T, y_min, margin, max_dT, T_max;
};

__device__ __forceinline__ double pred_y(const PostParams &q, const float *outT, int m, int r, int k,
                                         double yk) {
    const double t = (double)outT[(size_t)k * m + r] * q.norm[192 + k] + q.norm[128 + k];
    const double v = yk + S_Y * sinh(t);
    return v > 0.0 ? v : 0.0;
}

// One cell per thread.  outT [64][m] normalised network outputs of chunk
// rows; row r is cell base + r.  The clipped prediction Y1 = max(Y + dY, 0)
// is corrected by Y1_k (E^T lam)_k with (E W E^T) lam = E (Y1 - Y), W =
// diag(Y1); T' solves h(T', Y') = h(T, Y).  Accepted cells are updated and
// flagged 3; rejected cells are left untouched.
template <int NEL>
__global__ __launch_bounds__(256) void k_surrogate_post(FeatSrc f, int64_t base, int m,
                                                        const float *outT, PostParams q, double *T,
                                                        double *Y, uint8_t *flags,
                                                        unsigned long long *stats) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    bool accept = false, tried = false;
    if (r < m) {
        const int64_t i = base + r;
        const int N = q.N;
        if (!flags || flags[i] == 0) {
            tried = true;
            bool ok = T[i] <= q.T_max;
            // out-of-distribution box on the raw features
            for (int c = 0; c < N + 3 && ok; ++c) {
                const double v = raw_feature(f, i, c);
                const double lo = q.norm[256 + c], hi = q.norm[320 + c];
                const double span = hi - lo;
                ok = v >= lo - q.margin * span && v <= hi + q.margin * span;
            }
            double lam[NEL];
            double Tn = 0.0, dT = 0.0;
            if (ok) {
                double G[NEL][NEL], rr[NEL];
#pragma unroll
                for (int a = 0; a < NEL; ++a) {
                    rr[a] = 0.0;
#pragma unroll
                    for (int b = 0; b < NEL; ++b) G[a][b] = 0.0;
                }
                for (int k = 0; k < N; ++k) {
                    const double y0 = Y[(int64_t)k * f.n + i];
                    const double y1 = pred_y(q, outT, m, r, k, y0);
                    double ek[NEL];
#pragma unroll
                    for (int a = 0; a < NEL; ++a) ek[a] = q.E[a * N + k];
#pragma unroll
                    for (int a = 0; a < NEL; ++a) {
                        rr[a] += ek[a] * (y1 - y0);
#pragma unroll
                        for (int b = 0; b < NEL; ++b) G[a][b] += ek[a] * y1 * ek[b];
                    }
                }
                // Gaussian elimination with partial pivoting
#pragma unroll
                for (int c = 0; c < NEL; ++c) {
                    int pr = c;
#pragma unroll
                    for (int a = c + 1; a < NEL; ++a)
                        if (fabs(G[a][c]) > fabs(G[pr][c])) pr = a;
#pragma unroll
                    for (int a = c + 1; a < NEL; ++a) {
                        if (a == pr) {
#pragma unroll
                            for (int b = 0; b < NEL; ++b) {
                                const double t0 = G[c][b];
                                G[c][b] = G[a][b];
                                G[a][b] = t0;
                            }
                            const double t1 = rr[c];
                            rr[c] = rr[a];
                            rr[a] = t1;
                        }
                    }
                    ok = ok && G[c][c] != 0.0;
                    const double dinv = 1.0 / G[c][c];
#pragma unroll
                    for (int a = c + 1; a < NEL; ++a) {
                        const double l = G[a][c] * dinv;
#pragma unroll
                        for (int b = c; b < NEL; ++b) G[a][b] -= l * G[c][b];
                        rr[a] -= l * rr[c];
                    }
                }
#pragma unroll
                for (int c = NEL - 1; c >= 0; --c) {
                    double s = rr[c];
#pragma unroll
                    for (int b = c + 1; b < NEL; ++b) s -= G[c][b] * lam[b];
                    lam[c] = s / G[c][c];
                }
#pragma unroll
                for (int a = 0; a < NEL; ++a) ok = ok && isfinite(lam[a]);
                dT = S_T * sinh((double)outT[(size_t)N * m + r] * q.norm[192 + N] + q.norm[128 + N]);
                ok = ok && fabs(dT) <= q.max_dT;
                // corrected state: positivity gate and the enthalpy polynomial
                double Bo[6] = {0, 0, 0, 0, 0, 0}, Bn[6] = {0, 0, 0, 0, 0, 0};
                for (int k = 0; k < N && ok; ++k) {
                    const double y0 = Y[(int64_t)k * f.n + i];
                    const double y1 = pred_y(q, outT, m, r, k, y0);
                    double s = 0.0;
#pragma unroll
                    for (int a = 0; a < NEL; ++a) s += q.E[a * N + k] * lam[a];
                    const double yn = y1 - y1 * s;
                    ok = yn >= q.y_min;
                    const double iw = q.invW[k];
                    const double c6[6] = {q.nasa_t[k], q.nasa_t[7 * N + k], q.nasa_t[8 * N + k],
                                          q.nasa_t[9 * N + k], q.nasa_t[10 * N + k], q.nasa_t[5 * N + k]};
#pragma unroll
                    for (int t = 0; t < 6; ++t) {
                        Bo[t] += y0 * iw * c6[t];
                        Bn[t] += yn * iw * c6[t];
                    }
                }
                if (ok) {
                    const double T0 = T[i];
                    const double h0 = Bo[5] + T0 * (Bo[0] + T0 * (Bo[1] + T0 * (Bo[2] + T0 * (Bo[3] + T0 * Bo[4]))));
                    Tn = T0 + dT;
                    for (int it = 0; it < 50; ++it) {
                        const double F = Bn[5] + Tn * (Bn[0] + Tn * (Bn[1] + Tn * (Bn[2] + Tn * (Bn[3] + Tn * Bn[4])))) - h0;
                        const double dF = Bn[0] + Tn * (2.0 * Bn[1] + Tn * (3.0 * Bn[2] + Tn * (4.0 * Bn[3] + Tn * 5.0 * Bn[4])));
                        const double step = F / dF;
                        Tn -= step;
                        if (fabs(step) < 1e-10) break;
                    }
                    ok = fabs(T0 + dT - Tn) <= q.tau_T && Tn > 0.0;
                }
            }
            if (ok) {
                for (int k = 0; k < N; ++k) {
                    double *yp = Y + (int64_t)k * f.n + i;
                    const double y1 = pred_y(q, outT, m, r, k, *yp);
                    double s = 0.0;
#pragma unroll
                    for (int a = 0; a < NEL; ++a) s += q.E[a * N + k] * lam[a];
                    *yp = y1 - y1 * s;
                }
                T[i] = Tn;
                if (flags) flags[i] = 3;
                accept = true;
            }
        }
    }
    const unsigned long long na = __ballot(accept), nt = __ballot(tried);
    if ((threadIdx.x & 63) == 0) {
        if (na) atomicAdd(&stats[6], (unsigned long long)__popcll(na));
        if (nt & ~na) atomicAdd(&stats[7], (unsigned long long)__popcll(nt & ~na));
    }
}

// ------------------------------------------------------ fused inference ----
// Rows offered to the surrogate (no flag, T <= T_max): their chunk positions,
// in any order, and their count (zeroed by k_zero_int first).
__global__ void k_zero_int(int *p) { if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0; }

__global__ __launch_bounds__(256) void k_sur_select(const uint8_t *flags, const double *T, int64_t base,
                                                    int m, double T_max, int *idx, int *cnt) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    bool sel = false;
    if (r < m) {
        const int64_t i = base + r;
        sel = (!flags || flags[i] == 0) && T[i] <= T_max;
    }
    const unsigned long long b = __ballot(sel);
    const int lane = threadIdx.x & 63;
    int off = 0;
    if (lane == 0 && b) off = atomicAdd(cnt, __popcll(b));
    off = __shfl(off, 0);
    if (sel) idx[off + __popcll(b & ((1ull << lane) - 1ull))] = r;
}

// The whole network for a tile of 64 selected rows in one workgroup: the
// input tile and the hidden activations stay in LDS (bf16), weights stream
// from L2.  Per layer, wavefront w computes output columns [64w, 64w + 64)
// (16 of the 64 outputs in the last layer) for all 64 rows with 16x16x32
// MFMA blocks, accumulating over k in the same order as k_gemm_nt, so the
// outputs equal the layer-by-layer path bit for bit.  Output row r goes to
// outT[c][r] (r = chunk position), as the acceptance kernel reads it.
constexpr int FT = 64;             // rows per tile
constexpr int XLD = S_IN + 8;      // LDS row strides (bf16), padded against bank conflicts
constexpr int HLD = S_HID + 8;
struct MlpW {
    const uint16_t *W[5];
    const float *b[5];
};

template <int K, int NB>
__device__ __forceinline__ void tile_layer(const uint16_t *In, int ldi, const uint16_t *__restrict__ W,
                                           int n0, f32x4 (&acc)[4][NB]) {
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a[4], b[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j)
            b[j] = *(const bf16x8 *)(W + (size_t)(n0 + 16 * j + r16) * K + k0 + kq);
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = *(const bf16x8 *)(In + (16 * i + r16) * ldi + k0 + kq);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

template <int K>
__device__ __forceinline__ void hidden_layer(const uint16_t *In, int ldi, const uint16_t *W,
                                             const float *bias, uint16_t *Out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n0 = 64 * w;
    f32x4 acc[4][4];
    tile_layer<K, 4>(In, ldi, W, n0, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + 16 * j + (lane & 15);
            const float bc = bias[col];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * i + 4 * (lane >> 4) + r;
                Out[row * HLD + col] = f2bf(gelu_f(acc[i][j][r] + bc));
            }
        }
}

__global__ __launch_bounds__(256) void k_mlp_infer(FeatSrc f, int64_t base, int m, const int *idx,
                                                   const int *cnt, const float *norm, MlpW wt,
                                                   float *outT) {
    extern __shared__ uint16_t sm16[];
    uint16_t *Xs = sm16, *Ha = Xs + FT * XLD, *Hb = Ha + FT * HLD;
    const int n_sel = *cnt;
    const int t0 = blockIdx.x * FT;
    if (t0 >= n_sel) return;                       // whole workgroup
    const int rows = n_sel - t0 < FT ? n_sel - t0 : FT;
    const int tid = threadIdx.x, c = tid & 63;
    const int nfeat = f.N + 3;
    for (int rr = tid >> 6; rr < FT; rr += 4) {
        uint16_t v = 0;
        if (rr < rows && c < nfeat)
            v = f2bf((float)((raw_feature(f, base + idx[t0 + rr], c) - norm[c]) / norm[64 + c]));
        Xs[rr * XLD + c] = v;
    }
    __syncthreads();
    hidden_layer<S_IN>(Xs, XLD, wt.W[0], wt.b[0], Ha);
    __syncthreads();
    hidden_layer<S_HID>(Ha, HLD, wt.W[1], wt.b[1], Hb);
    __syncthreads();
    hidden_layer<S_HID>(Hb, HLD, wt.W[2], wt.b[2], Ha);
    __syncthreads();
    hidden_layer<S_HID>(Ha, HLD, wt.W[3], wt.b[3], Hb);
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6;
    f32x4 acc[4][1];
    tile_layer<S_HID, 1>(Hb, HLD, wt.W[4], 16 * w, acc);
    const int col = 16 * w + (lane & 15);
    const float bc = wt.b[4][col];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * i + 4 * (lane >> 4) + r;
            if (row < rows) outT[(size_t)col * m + idx[t0 + row]] = acc[i][0][r] + bc;
        }
}
static constexpr size_t kInferLds = sizeof(uint16_t) * (size_t)FT * (XLD + 2 * HLD);

// Every row of a chunk selected, in order (the fused kernel's check entry).
__global__ __launch_bounds__(256) void k_select_all(int m, int *idx, int *cnt) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < m) idx[r] = r;
    if (r == 0) *cnt = m;
}

// out[r][c] = outT[c][r] for a chunk of m rows and 64 outputs
__global__ __launch_bounds__(256) void k_untranspose(const float *outT, int m, float *out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)m * S_OUT) return;
    const int r = (int)(i / S_OUT), c = (int)(i % S_OUT);
    out[i] = outT[(size_t)c * m + r];
}

static void launch_post(int nel, dim3 g, hipStream_t s, const FeatSrc &f, int64_t base, int m,
                        const float *outT, const PostParams &q, double *T, double *Y, uint8_t *flags,
                        unsigned long long *stats) {
    switch (nel) {
#define POST(E_)                                                                                   \
    case E_:                                                                                       \
        hipLaunchKernelGGL(k_surrogate_post<E_>, g, dim3(256), 0, s, f, base, m, outT, q, T, Y,   \
                           flags, stats);                                                          \
        break;
        POST(1) POST(2) POST(3) POST(4) POST(5) POST(6) POST(7) POST(8)
#undef POST
    }
}

// ================================================================ host ======
static int layer_in(int l) { return l == 0 ? S_IN : S_HID; }
static int layer_out(int l) { return l == 4 ? S_OUT : S_HID; }

int64_t surrogate_param_count() {
    int64_t n = 0;
    for (int l = 0; l < 5; ++l) n += (int64_t)layer_out(l) * layer_in(l) + layer_out(l);
    return n + 6 * S_IN;
}
static int64_t weights_count() { return surrogate_param_count() - 6 * S_IN; }
static int64_t layer_offset(int l) {
    int64_t o = 0;
    for (int q = 0; q < l; ++q) o += (int64_t)layer_out(q) * layer_in(q) + layer_out(q);
    return o;
}

#define SCHK(x)                                                         \
    do {                                                                \
        hipError_t e_ = (x);                                            \
        if (e_ != hipSuccess) {                                         \
            snprintf(err, 256, "%s: %s", #x, hipGetErrorString(e_));    \
            return -3;                                                  \
        }                                                               \
    } while (0)

template <class T>
static hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, std::max<size_t>(1, count) * sizeof(T));
}

Surrogate::~Surrogate() {
    for (void *p : bufs) (void)hipFree(p);
    for (void *p : ws) (void)hipFree(p);
}

int Surrogate::init(int N_, int nel_, const std::vector<double> &E_host, char *err) {
    N = N_;
    nel = nel_;
    SCHK(hipFuncSetAttribute((const void *)k_mlp_infer, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kInferLds));
    const int64_t np = surrogate_param_count();
    float *fp = nullptr;
    SCHK(dalloc(&fp, np)); bufs.push_back(fp); P = fp;
    SCHK(dalloc(&fp, np)); bufs.push_back(fp); G = fp;
    SCHK(dalloc(&fp, np)); bufs.push_back(fp); mA = fp;
    SCHK(dalloc(&fp, np)); bufs.push_back(fp); vA = fp;
    for (int l = 0; l < 5; ++l) {
        uint16_t *b = nullptr;
        SCHK(dalloc(&b, (size_t)layer_out(l) * layer_in(l))); bufs.push_back(b); Wb[l] = b;
        SCHK(dalloc(&b, (size_t)layer_out(l) * layer_in(l))); bufs.push_back(b); WbT[l] = b;
    }
    double *dp = nullptr;
    SCHK(dalloc(&dp, E_host.size())); bufs.push_back(dp); E = dp;
    SCHK(hipMemcpy(E, E_host.data(), sizeof(double) * E_host.size(), hipMemcpyHostToDevice));
    SCHK(dalloc(&dp, 1)); bufs.push_back(dp); d_loss = dp;
    return 0;
}

int Surrogate::refresh(hipStream_t s, char *err) {
    for (int l = 0; l < 5; ++l) {
        const int no = layer_out(l), ni = layer_in(l);
        hipLaunchKernelGGL(k_refresh, dim3((no * ni + 255) / 256), dim3(256), 0, s,
                           P + layer_offset(l), no, ni, Wb[l], WbT[l]);
    }
    SCHK(hipGetLastError());
    return 0;
}

int Surrogate::set_params(const float *host, hipStream_t s, char *err) {
    SCHK(hipMemcpyAsync(P, host, sizeof(float) * surrogate_param_count(), hipMemcpyHostToDevice, s));
    SCHK(hipStreamSynchronize(s));
    int rc = refresh(s, err);
    if (rc) return rc;
    trained = true;
    return 0;
}

int Surrogate::get_params(float *host, hipStream_t s, char *err) {
    SCHK(hipMemcpyAsync(host, P, sizeof(float) * surrogate_param_count(), hipMemcpyDeviceToHost, s));
    SCHK(hipStreamSynchronize(s));
    return 0;
}

// workspace for up to B rows: activations, transposes, pre-activations
int Surrogate::reserve_ws(int B, bool training, char *err) {
    if (B <= ws_rows && (!training || ws_training)) return 0;
    for (void *p : ws) (void)hipFree(p);
    ws.clear();
    auto get16 = [&](uint16_t **p, size_t n) { hipError_t e = dalloc(p, n); ws.push_back(*p); return e; };
    auto get32 = [&](float **p, size_t n) { hipError_t e = dalloc(p, n); ws.push_back(*p); return e; };
    SCHK(get16(&X, (size_t)B * S_IN));
    for (int l = 0; l < 4; ++l) SCHK(get16(&H[l], (size_t)B * S_HID));
    SCHK(get32(&out, (size_t)B * S_OUT));
    if (training) {
        SCHK(get16(&XT, (size_t)B * S_IN));
        for (int l = 0; l < 4; ++l) {
            SCHK(get16(&HT[l], (size_t)B * S_HID));
            SCHK(get32(&Z[l], (size_t)B * S_HID));
        }
        SCHK(get32(&Tg, (size_t)B * S_OUT));
        SCHK(get32(&dOf, (size_t)B * S_OUT));
        SCHK(get16(&dZ5, (size_t)B * S_OUT));
        SCHK(get16(&dZ5T, (size_t)B * S_OUT));
        SCHK(get32(&dH, (size_t)B * S_HID));
        SCHK(get16(&dZb, (size_t)B * S_HID));
        SCHK(get16(&dZbT, (size_t)B * S_HID));
        SCHK(get32(&csum, (size_t)CS_CHUNKS * S_HID));
        SCHK(get32(&kpart, (size_t)kSplitFloats));
        double *dp = nullptr;
        SCHK(dalloc(&dp, (size_t)(B + 3) / 4)); ws.push_back(dp); lpart = dp;
    }
    int *ip = nullptr;
    SCHK(dalloc(&ip, (size_t)B)); ws.push_back(ip); idx = ip;
    SCHK(dalloc(&ip, (size_t)1)); ws.push_back(ip); sel_cnt = ip;
    ws_rows = B;
    ws_training = training;
    return 0;
}

// forward of B rows already in X (inference epilogue unless training)
void Surrogate::forward(int B, bool training, bool out_transposed, hipStream_t s) {
    const uint16_t *in = X;
    int ldin = S_IN;
    for (int l = 0; l < 4; ++l) {
        GemmEpi e{};
        e.bias = P + layer_offset(l) + (int64_t)layer_out(l) * layer_in(l);
        e.H = H[l]; e.ldh = S_HID;
        if (training) { e.HT = HT[l]; e.ldht = B; e.Z = Z[l]; e.ldz = S_HID; }
        gemm<EPI_HID>(in, ldin, Wb[l], layer_in(l), B, S_HID, layer_in(l), e, s);
        in = H[l];
        ldin = S_HID;
    }
    GemmEpi e{};
    e.bias = P + layer_offset(4) + (int64_t)S_OUT * S_HID;
    e.C = out;
    if (out_transposed) {
        e.ldc = B;
        gemm<EPI_OUT_T>(in, S_HID, Wb[4], S_HID, B, S_OUT, S_HID, e, s);
    } else {
        e.ldc = S_OUT;
        gemm<EPI_OUT>(in, S_HID, Wb[4], S_HID, B, S_OUT, S_HID, e, s);
    }
}

void Surrogate::colsum(const float *src, int B, int ncol, float *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum_part, dim3((ncol + 63) / 64, CS_CHUNKS), dim3(256), 0, s, src, B, ncol,
                       csum);
    hipLaunchKernelGGL(k_colsum_final, dim3((ncol + 255) / 256), dim3(256), 0, s, csum, ncol, dst);
}

// C [M x N], leading dimension N, = A B^T for a weight gradient: M x N is a
// few tiles and K (the batch) is long, so the K range is cut into S slices
// that fill the chip; each slice writes its partial product and a second pass
// adds the slices in order
bool Surrogate::gemm_wgrad(const uint16_t *A, int lda, const uint16_t *Bm, int ldb, int M, int N,
                           int K, float *C, hipStream_t s) {
    const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
    int S = 1;
    while (tiles * 2 * S <= 256 && K % (64 * S) == 0 && K / (2 * S) >= 128 &&
           (int64_t)2 * S * M * N <= kSplitFloats)
        S *= 2;
    // launch invariants, checked on the host before anything is enqueued:
    // every slice is a whole number of 32-wide k steps inside the rows of A
    // and B, and the S slabs of M x N partial sums fit the slice buffer
    if (K % S != 0 || (K / S) % 32 != 0 || K > lda || K > ldb || (int64_t)S * M * N > kSplitFloats)
        return false;
    GemmEpi e{};
    e.ldc = N;
    if (S == 1) {
        e.C = C;
        gemm<EPI_PLAIN>(A, lda, Bm, ldb, M, N, K, e, s);
        return true;
    }
    e.C = kpart;
    hipLaunchKernelGGL(k_gemm_nt<EPI_PLAIN>, dim3((M + 63) / 64, (N + 63) / 64, S), dim3(256), 0, s,
                       A, lda, Bm, ldb, M, N, K / S, e);
    const int64_t mn = (int64_t)M * N;
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, kpart, S,
                       mn, C);
    return true;
}

// gradients of the mean-squared error for the B rows in X / Tg into G;
// false (nothing enqueued past the failing launch) if a launch would not fit
// the workspace
bool Surrogate::backward(int B, hipStream_t s) {
    const int nout = N + 1;
    if (B > ws_rows || !ws_training || B % 64 != 0) return false;
    hipLaunchKernelGGL(k_out_grad, dim3((B + 3) / 4), dim3(256), 0, s, out, Tg, B, nout, dOf, dZ5,
                       dZ5T, B, lpart);
    // output layer
    {
        if (!gemm_wgrad(dZ5T, B, HT[3], B, S_OUT, S_HID, B, G + layer_offset(4), s))   // dW5 = dZ5^T H4
            return false;
        colsum(dOf, B, S_OUT, G + layer_offset(4) + (int64_t)S_OUT * S_HID, s);
        GemmEpi e2{};
        e2.C = dH; e2.ldc = S_HID;
        gemm<EPI_PLAIN>(dZ5, S_OUT, WbT[4], S_OUT, B, S_HID, S_OUT, e2, s);    // dH4 = dZ5 W5
    }
    for (int l = 3; l >= 0; --l) {
        hipLaunchKernelGGL(k_gelu_back, dim3(S_HID / 64, CS_CHUNKS), dim3(256), 0, s, dH, Z[l], B,
                           dZb, dZbT, B, csum);
        const int ni = layer_in(l);
        const uint16_t *inT = l == 0 ? XT : HT[l - 1];
        if (!gemm_wgrad(dZbT, B, inT, B, S_HID, ni, B, G + layer_offset(l), s))   // dW = dZ^T h_{l-1}
            return false;
        hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(256), 0, s, csum, S_HID,
                           G + layer_offset(l) + (int64_t)S_HID * ni);
        if (l > 0) {
            GemmEpi e2{};
            e2.C = dH; e2.ldc = S_HID;
            gemm<EPI_PLAIN>(dZb, S_HID, WbT[l], S_HID, B, S_HID, S_HID, e2, s);   // dh = dZ W
        }
    }
    return true;
}

int Surrogate::compute_norm(const FeatSrc &f, const TgtSrc &t, hipStream_t s, char *err) {
    const int nfeat = N + 3, nout = N + 1;
    double *dm = nullptr;
    SCHK(dalloc(&dm, (size_t)4 * nfeat + 2 * nout));
    hipLaunchKernelGGL(k_feature_moments, dim3(nfeat), dim3(256), 0, s, f, nfeat, dm);
    hipLaunchKernelGGL(k_target_moments, dim3(nout), dim3(256), 0, s, t, dm + 4 * nfeat);
    std::vector<double> hm(4 * nfeat + 2 * nout);
    SCHK(hipMemcpyAsync(hm.data(), dm, sizeof(double) * hm.size(), hipMemcpyDeviceToHost, s));
    SCHK(hipStreamSynchronize(s));
    (void)hipFree(dm);
    std::vector<float> nb(6 * S_IN, 0.0f);
    const double n = (double)f.n;
    for (int c = 0; c < S_IN; ++c) { nb[64 + c] = 1.0f; nb[192 + c] = 1.0f; }
    for (int c = 0; c < nfeat; ++c) {
        const double mu = hm[4 * c] / n;
        const double var = std::max(0.0, hm[4 * c + 1] / n - mu * mu);
        const double sd = sqrt(var);
        nb[c] = (float)mu;
        nb[64 + c] = sd > 1e-30 ? (float)sd : 1.0f;
        // the stored box must contain every training feature after rounding
        float lo = (float)hm[4 * c + 2], hi = (float)hm[4 * c + 3];
        if ((double)lo > hm[4 * c + 2]) lo = nextafterf(lo, -INFINITY);
        if ((double)hi < hm[4 * c + 3]) hi = nextafterf(hi, INFINITY);
        nb[256 + c] = lo;
        nb[320 + c] = hi;
    }
    for (int c = 0; c < nout; ++c) {
        const double mu = hm[4 * nfeat + 2 * c] / n;
        const double var = std::max(0.0, hm[4 * nfeat + 2 * c + 1] / n - mu * mu);
        const double sd = sqrt(var);
        nb[128 + c] = (float)mu;
        nb[192 + c] = sd > 1e-30 ? (float)sd : 1.0f;
    }
    SCHK(hipMemcpyAsync(P + weights_count(), nb.data(), sizeof(float) * nb.size(),
                        hipMemcpyHostToDevice, s));
    SCHK(hipStreamSynchronize(s));   // nb is released on return
    return 0;
}

int Surrogate::train(const FeatSrc &f, const TgtSrc &t, int epochs, int B, double lr0, double lr1,
                     uint64_t seed, float *loss_hist, int verbose, hipStream_t s, char *err) {
    if (B % 64 != 0 || B < 64) { snprintf(err, 256, "batch must be a positive multiple of 64"); return -1; }
    const int64_t n = f.n;
    if (n < B) { snprintf(err, 256, "fewer samples than one batch"); return -1; }
    int rc = reserve_ws(B, true, err);
    if (rc) return rc;
    rc = compute_norm(f, t, s, err);
    if (rc) return rc;
    // He-style initialisation (seeded), zero biases, small output layer
    {
        std::mt19937_64 rng(seed);
        std::normal_distribution<float> nd(0.0f, 1.0f);
        std::vector<float> h(weights_count(), 0.0f);
        for (int l = 0; l < 5; ++l) {
            const int no = layer_out(l), ni = layer_in(l);
            const float sc = (l == 4 ? 0.1f : 1.0f) * sqrtf(2.0f / (float)ni);
            float *W = h.data() + layer_offset(l);
            for (int o = 0; o < no; ++o)
                for (int i = 0; i < ni; ++i) {
                    const bool live_in = l > 0 || i < N + 3;
                    const bool live_out = l < 4 || o < N + 1;
                    W[o * ni + i] = (live_in && live_out) ? sc * nd(rng) : 0.0f;
                }
        }
        SCHK(hipMemcpyAsync(P, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, s));
        SCHK(hipMemsetAsync(mA, 0, sizeof(float) * weights_count(), s));
        SCHK(hipMemsetAsync(vA, 0, sizeof(float) * weights_count(), s));
        SCHK(hipStreamSynchronize(s));   // h is released at the end of this scope
    }
    rc = refresh(s, err);
    if (rc) return rc;
    const int64_t nb = n / B;
    const int64_t total = nb * epochs;
    int *d_perm = nullptr;
    SCHK(dalloc(&d_perm, (size_t)n));
    std::vector<int> perm(n);
    std::mt19937_64 rng(seed ^ 0x9e3779b97f4a7c15ull);
    int64_t step = 0;
    const int64_t nw = weights_count();
    WeightCopies wc{};
    for (int l = 0; l < 5; ++l) {
        wc.off[l] = layer_offset(l);
        wc.no[l] = layer_out(l);
        wc.ni[l] = layer_in(l);
        wc.Wb[l] = Wb[l];
        wc.WbT[l] = WbT[l];
    }
    for (int ep = 0; ep < epochs; ++ep) {
        std::iota(perm.begin(), perm.end(), 0);
        std::shuffle(perm.begin(), perm.end(), rng);
        SCHK(hipMemcpyAsync(d_perm, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
        SCHK(hipMemsetAsync(lpart, 0, sizeof(double) * ((B + 3) / 4), s));
        for (int64_t bi = 0; bi < nb; ++bi, ++step) {
            hipLaunchKernelGGL(k_build_rows, dim3((B + 3) / 4), dim3(256), 0, s, f, t,
                               d_perm + bi * B, (int64_t)0, B, P + weights_count(), X, XT, B, Tg);
            forward(B, true, false, s);
            if (!backward(B, s)) {
                snprintf(err, 256, "backward: launch does not fit the workspace (batch %d)", B);
                return -1;
            }
            const double frac = total > 1 ? (double)step / (double)(total - 1) : 1.0;
            const float lr = (float)(lr1 + 0.5 * (lr0 - lr1) * (1.0 + cos(M_PI * frac)));
            const float b1 = 0.9f, b2 = 0.999f;
            const float c1 = 1.0f - powf(b1, (float)(step + 1)), c2 = 1.0f - powf(b2, (float)(step + 1));
            hipLaunchKernelGGL(k_adam, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, P, G, mA,
                               vA, nw, lr, b1, b2, 1e-8f, c1, c2, wc);
        }
        hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(256), 0, s, lpart, (B + 3) / 4, d_loss);
        double l = 0.0;
        SCHK(hipMemcpyAsync(&l, d_loss, sizeof(double), hipMemcpyDeviceToHost, s));
        SCHK(hipStreamSynchronize(s));
        const double mean = l / ((double)nb * B * (N + 1));
        if (loss_hist) loss_hist[ep] = (float)mean;
        if (verbose) fprintf(stderr, "[libchem] surrogate epoch %d/%d: loss %.4e\n", ep + 1, epochs, mean);
    }
    SCHK(hipGetLastError());
    (void)hipFree(d_perm);
    trained = true;
    return 0;
}

int Surrogate::loss_grad(const FeatSrc &f, const TgtSrc &t, float *grad_host, double *loss,
                         hipStream_t s, char *err) {
    const int B = (int)f.n;
    if (B % 64 != 0 || B < 64 || B > 65536) { snprintf(err, 256, "n must be a multiple of 64, <= 65536"); return -1; }
    int rc = reserve_ws(B, true, err);
    if (rc) return rc;
    SCHK(hipMemsetAsync(lpart, 0, sizeof(double) * ((B + 3) / 4), s));
    hipLaunchKernelGGL(k_build_rows, dim3((B + 3) / 4), dim3(256), 0, s, f, t, (const int *)nullptr,
                       (int64_t)0, B, P + weights_count(), X, XT, B, Tg);
    forward(B, true, false, s);
    if (!backward(B, s)) {
        snprintf(err, 256, "backward: launch does not fit the workspace (%d rows)", B);
        return -1;
    }
    hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(256), 0, s, lpart, (B + 3) / 4, d_loss);
    SCHK(hipMemcpyAsync(grad_host, G, sizeof(float) * weights_count(), hipMemcpyDeviceToHost, s));
    double l = 0.0;
    SCHK(hipMemcpyAsync(&l, d_loss, sizeof(double), hipMemcpyDeviceToHost, s));
    SCHK(hipStreamSynchronize(s));
    *loss = l / ((double)B * (N + 1));
    return 0;
}

int Surrogate::forward_rows(const FeatSrc &f, float *out_dev, hipStream_t s, char *err) {
    const int64_t n = f.n;
    const int chunk = 65536;
    int rc = reserve_ws((int)std::min<int64_t>(n, chunk), false, err);
    if (rc) return rc;
    TgtSrc t{};
    for (int64_t base = 0; base < n; base += chunk) {
        const int m = (int)std::min<int64_t>(chunk, n - base);
        hipLaunchKernelGGL(k_build_rows, dim3((m + 3) / 4), dim3(256), 0, s, f, t, (const int *)nullptr,
                           base, m, P + weights_count(), X, (uint16_t *)nullptr, 0, (float *)nullptr);
        forward(m, false, false, s);
        SCHK(hipMemcpyAsync(out_dev + base * S_OUT, out, sizeof(float) * m * S_OUT,
                            hipMemcpyDeviceToDevice, s));
    }
    SCHK(hipGetLastError());
    return 0;
}

// Raw outputs of the fused inference kernel (the one apply() runs), every row
// selected, in the row-major layout of forward_rows.
int Surrogate::forward_fused_rows(const FeatSrc &f, float *out_dev, hipStream_t s, char *err) {
    const int64_t n = f.n;
    const int chunk = 262144;
    int rc = reserve_ws((int)std::min<int64_t>(n, chunk), false, err);
    if (rc) return rc;
    MlpW wts{};
    for (int l = 0; l < 5; ++l) {
        wts.W[l] = Wb[l];
        wts.b[l] = P + layer_offset(l) + (int64_t)layer_out(l) * layer_in(l);
    }
    for (int64_t base = 0; base < n; base += chunk) {
        const int m = (int)std::min<int64_t>(chunk, n - base);
        hipLaunchKernelGGL(k_select_all, dim3((m + 255) / 256), dim3(256), 0, s, m, idx, sel_cnt);
        hipLaunchKernelGGL(k_mlp_infer, dim3((m + FT - 1) / FT), dim3(256), kInferLds, s, f, base, m,
                           idx, sel_cnt, P + weights_count(), wts, out);
        hipLaunchKernelGGL(k_untranspose, dim3((unsigned)(((int64_t)m * S_OUT + 255) / 256)), dim3(256),
                           0, s, out, m, out_dev + base * S_OUT);
    }
    SCHK(hipGetLastError());
    return 0;
}

int Surrogate::apply(const FeatSrc &f, double *T, double *Y, uint8_t *flags, const PostIn &pin,
                     unsigned long long *stats, hipStream_t s, char *err) {
    const int64_t n = f.n;
    const int chunk = 262144;
    int rc = reserve_ws((int)std::min<int64_t>(n, chunk), false, err);
    if (rc) return rc;
    MlpW wts{};
    for (int l = 0; l < 5; ++l) {
        wts.W[l] = Wb[l];
        wts.b[l] = P + layer_offset(l) + (int64_t)layer_out(l) * layer_in(l);
    }
    PostParams q{};
    q.N = N; q.nel = nel; q.E = E; q.nasa_t = pin.nasa_t; q.invW = pin.invW;
    q.norm = P + weights_count(); q.tau_T = pin.tau_T; q.y_min = pin.y_min; q.margin = pin.margin;
    q.max_dT = pin.max_dT;
    q.T_max = pin.T_max;
    TgtSrc t{};
    for (int64_t base = 0; base < n; base += chunk) {
        const int m = (int)std::min<int64_t>(chunk, n - base);
        // only offered rows go through the network (fused, one kernel)
        hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, sel_cnt);
        hipLaunchKernelGGL(k_sur_select, dim3((m + 255) / 256), dim3(256), 0, s, flags, T, base, m,
                           pin.T_max, idx, sel_cnt);
        hipLaunchKernelGGL(k_mlp_infer, dim3((m + FT - 1) / FT), dim3(256), kInferLds, s, f, base, m,
                           idx, sel_cnt, P + weights_count(), wts, out);
        launch_post(nel, dim3((m + 255) / 256), s, f, base, m, out, q, T, Y, flags, stats);
    }
    SCHK(hipGetLastError());
    return 0;
}

}  // namespace chem
