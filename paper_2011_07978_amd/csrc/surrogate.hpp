// Learned dt-advance surrogate: state shared between the host API and the
// BF16-MFMA kernels of mlp.hip.  All pointers are device pointers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace chem {

constexpr int S_IN = 64;    // padded input width (ln T, ln p, Y_1..Y_N, ln dt)
constexpr int S_HID = 256;  // hidden width
constexpr int S_OUT = 64;   // padded output width (dY_1..dY_N, dT)
constexpr int S_MAX_SPECIES = S_IN - 3;

// Raw-feature source: species-major state arrays of n samples.
struct FeatSrc {
    const double *T, *p, *Y, *dt;  // dt per sample unless dt_scalar > 0
    double dt_scalar;
    int64_t n;
    int N;
};

// Raw-target source: the state after the advance.
struct TgtSrc {
    const double *T0, *Y0, *T1, *Y1;
    int64_t n;
    int N;
};

// Mechanism data the gate needs: thermo table [14][N] and 1/W [N].
struct PostIn {
    const double *nasa_t, *invW;
    double tau_T, y_min, margin, max_dT, T_max;
};

int64_t surrogate_param_count();

struct Surrogate {
    int N = 0, nel = 0;
    bool trained = false;
    // parameters: FP32 master blob (layout of the parameter file), gradient,
    // Adam moments; bf16 copies of every weight matrix and of its transpose
    float *P = nullptr, *G = nullptr, *mA = nullptr, *vA = nullptr;
    uint16_t *Wb[5] = {}, *WbT[5] = {};
    // element conservation: E [nel][N] = a_ek / W_k
    double *E = nullptr;
    double *d_loss = nullptr;
    std::vector<void *> bufs;
    // row workspace
    int ws_rows = 0;
    bool ws_training = false;
    std::vector<void *> ws;
    uint16_t *X = nullptr, *XT = nullptr, *H[4] = {}, *HT[4] = {};
    float *Z[4] = {}, *out = nullptr, *Tg = nullptr, *dOf = nullptr, *dH = nullptr;
    uint16_t *dZ5 = nullptr, *dZ5T = nullptr, *dZb = nullptr, *dZbT = nullptr;
    float *csum = nullptr;   // partial column sums of the bias gradients
    float *kpart = nullptr;  // split-K slices of the weight gradients
    double *lpart = nullptr; // per-block running sums of the squared error
    int *idx = nullptr;
    int *sel_cnt = nullptr;  // rows selected for inference

    ~Surrogate();
    int init(int N, int nel, const std::vector<double> &E_host, char *err);
    int refresh(hipStream_t s, char *err);
    int set_params(const float *host, hipStream_t s, char *err);
    int get_params(float *host, hipStream_t s, char *err);
    int reserve_ws(int rows, bool training, char *err);
    void forward(int B, bool training, bool out_transposed, hipStream_t s);
    bool backward(int B, hipStream_t s);
    void colsum(const float *src, int B, int ncol, float *dst, hipStream_t s);
    bool gemm_wgrad(const uint16_t *A, int lda, const uint16_t *Bm, int ldb, int M, int N, int K,
                    float *C, hipStream_t s);
    int compute_norm(const FeatSrc &f, const TgtSrc &t, hipStream_t s, char *err);
    int train(const FeatSrc &f, const TgtSrc &t, int epochs, int B, double lr0, double lr1,
              uint64_t seed, float *loss_hist, int verbose, hipStream_t s, char *err);
    int loss_grad(const FeatSrc &f, const TgtSrc &t, float *grad_host, double *loss, hipStream_t s,
                  char *err);
    int forward_rows(const FeatSrc &f, float *out_dev, hipStream_t s, char *err);
    int forward_fused_rows(const FeatSrc &f, float *out_dev, hipStream_t s, char *err);
    int apply(const FeatSrc &f, double *T, double *Y, uint8_t *flags, const PostIn &pin,
              unsigned long long *stats, hipStream_t s, char *err);
};

}  // namespace chem
