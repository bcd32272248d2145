// C-ABI of libchem: validation, mechanism packing, workspace and dispatch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/chem.h"
#include "mech_dev.hpp"
#include "surrogate.hpp"

namespace chem {
int pick_np(int n);
hipError_t launch_integrate(int NP, const MechDev &M, const MechDev *Md, const IntParams &P,
                            int schedule, int grid, hipStream_t s);
int queue_occupancy(int NP, const MechDev &M);
int wave_kernel_wpb(const MechDev &M);
hipError_t launch_eval_rhs_jac(int NP, const MechDev &M, const MechDev *Md, const IntParams &P,
                               double *f, double *J, hipStream_t s);
hipError_t launch_rodas_step(int NP, const MechDev &M, const MechDev *Md, const IntParams &P,
                             double h, double *ynew, double *err, hipStream_t s);
hipError_t launch_map(int64_t ncells, int N, const double *T, const double *Y, const double *w,
                      double beta_f, double beta_ox, double Z_tol, double T_tol, int use_T,
                      uint8_t *flags, unsigned long long *ref_tmp, int64_t *ref_out, hipStream_t s);
hipError_t launch_queue_reset(int *hist, int *cursor, int *seg_ctr, int *n_active,
                              unsigned long long *stats, int *ref_status, hipStream_t s);
hipError_t launch_queue_build(int64_t ncells, const uint8_t *flags, const uint32_t *cost, int *hist,
                              int *cursor, int *n_active, int *queue, hipStream_t s);
hipError_t launch_ref_snapshot(int64_t ncells, int N, const double *T, const double *Y,
                               const int64_t *ref, double *snap, hipStream_t s);
size_t big_lds_bytes(int n);
hipError_t big_prepare(int n);
int big_occupancy(int n);
hipError_t launch_integrate_big(const MechDev &M, const MechDev *Md, const IntParams &P,
                                int schedule, int grid, double *jws, hipStream_t s);
hipError_t launch_big_rhs_jac(const MechDev &M, const MechDev *Md, const IntParams &P, double *f,
                              double *J, hipStream_t s);
hipError_t launch_big_rodas_step(const MechDev &M, const MechDev *Md, const IntParams &P, double h,
                                 double *ynew, double *err, double *jws, hipStream_t s);
hipError_t launch_map_scatter(int64_t ncells, int N, double *T, double *Y, const uint8_t *flags,
                              const int64_t *ref, const double *snap, double *delta,
                              const double *nasa_t, const double *invW, uint8_t *status,
                              uint32_t *cost, unsigned long long *stats, const int *ref_status,
                              hipStream_t s);
}  // namespace chem

using namespace chem;

struct chem_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int num_cu = 0;
    chem_options opt;
    // mechanism
    bool has_mech = false;
    int E = 0, N = 0, R = 0, NP = -1;
    std::vector<int> comp;         // [N*E]
    std::vector<double> elem_mass, W;
    MechDev M{};                   // host copy (sizes, device pointers)
    MechDev *d_mech = nullptr;     // device copy read by the kernels
    std::vector<void *> mech_bufs;
    // mapping weights (device) and the streams they were computed for
    double *d_mapw = nullptr;
    std::vector<double> map_yf, map_yo;
    double beta_f = 0.0, beta_ox = 0.0;
    // workspace
    int64_t cap = 0;
    int *d_queue = nullptr;
    int *d_small = nullptr;        // hist[32] cursor[32] seg[8] n_active[1] . ref_status[76]
    unsigned long long *d_stats = nullptr;   // [8]
    unsigned long long *d_reftmp = nullptr;
    double *d_snap = nullptr, *d_delta = nullptr;
    unsigned long long *h_stats = nullptr;   // pinned
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr, ev4 = nullptr,
               ev5 = nullptr;
    int64_t *d_refnone = nullptr;            // device -1: "no reference cell"
    int occ = 0;
    // large mechanisms (n > 64): workgroup-per-cell kernel, Jacobian slots of
    // the workgroups in flight
    bool big = false;
    double *d_jws = nullptr;
    int big_slots = 0;
    bool in_capture = false, capture_failed = false;   // chem_graph_begin .. _end
    Surrogate *sur = nullptr;                // learned surrogate (null: not available)
    std::string sur_why;                     // why it is not available
};

static int fail(chem_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    if (c && c->in_capture) c->capture_failed = true;   // the recording misses this call
    if (getenv("CHEM_LOG")) fprintf(stderr, "[libchem] %s\n", buf);
    return code;
}

#define HIPCHK(c, x)                                                                 \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess)                                                        \
            return fail(c, CHEM_E_HIP, "%s: %s", #x, hipGetErrorString(e_));         \
    } while (0)

static bool capturing(chem_ctx *c) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c->stream, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

// ---- fixed workspace of chem_integrate_noalloc ----------------------------
// For callers that cannot allocate, the integration's per-call scratch lives
// in a fixed device array of this library's code object: every device the
// library runs on holds its own copy until the process ends.  Layout (bytes):
// [0, 320) queue counters (32 bucket offsets, 32 cursors, 8 segment counters,
// the active count at int 72, the reference cell's status at int 76),
// [512, 576) call statistics (8 x u64), [1024, 2312) the reference cell's
// state before the step (<= 161 doubles), [2560, 3840) its increment
// (<= 160 doubles), [4096, 4104) the "no reference cell" index (-1), and from
// 8192 the heavy-first queue (int32 per cell).  Calls that overlap on one
// device share it and race; every call re-initialises what it reads.
constexpr int64_t kNoAllocMaxCells = (int64_t)1 << 21;
constexpr size_t kScrStats = 512, kScrSnap = 1024, kScrDelta = 2560, kScrNone = 4096,
                 kScrQueue = 8192;
constexpr size_t kScratchBytes = kScrQueue + sizeof(int) * (size_t)kNoAllocMaxCells;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, resolved once per device by
// chem_create with that device current.  In host code the array's name is
// only a stand-in: kernels and copies must use these addresses.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_dev[kMaxDevices];

static hipError_t resolve_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_scratch_dev[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_dev[device] = (unsigned char *)ptr;
    return hipSuccess;
}

static unsigned char *scratch_on(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device >= 0 && device < kMaxDevices ? g_scratch_dev[device] : nullptr;
}

__global__ void k_set_i64(int64_t *p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Exported functions take C linkage from their declarations in chem.h.

void chem_default_options(chem_options *o) {
    o->rtol = 1e-8;
    o->atol = 1e-12;
    o->max_steps = 100000;
    o->hmin_frac = 1e-14;
    o->schedule = CHEM_SCHED_QUEUE;
    o->queue_chunk = 0;
    o->slots_per_cu = 0;
    o->order_by_cost = 1;
}

int chem_max_species(void) { return 137; }

int chem_create(chem_ctx **out, int hip_device, void *hip_stream) {
    if (!out) return CHEM_E_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
        return CHEM_E_INVALID_ARG;
    chem_ctx *c = new chem_ctx();
    c->device = hip_device;
    c->stream = (hipStream_t)hip_stream;
    chem_default_options(&c->opt);
    if (hipSetDevice(hip_device) != hipSuccess ||
        hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, hip_device) !=
            hipSuccess ||
        hipHostMalloc((void **)&c->h_stats, 8 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void **)&c->d_stats, 8 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void **)&c->d_small, 80 * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&c->d_reftmp, sizeof(unsigned long long)) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreate(&c->ev2) != hipSuccess || hipEventCreate(&c->ev3) != hipSuccess ||
        hipEventCreate(&c->ev4) != hipSuccess || hipEventCreate(&c->ev5) != hipSuccess ||
        hipMalloc((void **)&c->d_refnone, sizeof(int64_t)) != hipSuccess ||
        resolve_scratch(hip_device) != hipSuccess) {
        chem_destroy(c);
        return CHEM_E_HIP;
    }
    const int64_t none = -1;
    if (hipMemcpy(c->d_refnone, &none, sizeof none, hipMemcpyHostToDevice) != hipSuccess) {
        chem_destroy(c);
        return CHEM_E_HIP;
    }
    *out = c;
    return CHEM_OK;
}

static void free_mech(chem_ctx *c) {
    for (void *p : c->mech_bufs) (void)hipFree(p);
    c->mech_bufs.clear();
    if (c->d_mapw) (void)hipFree(c->d_mapw);
    if (c->d_snap) (void)hipFree(c->d_snap);
    if (c->d_delta) (void)hipFree(c->d_delta);
    if (c->d_jws) (void)hipFree(c->d_jws);
    c->d_jws = nullptr;
    c->big = false;
    c->big_slots = 0;
    c->d_mapw = c->d_snap = c->d_delta = nullptr;
    c->d_mech = nullptr;
    delete c->sur;
    c->sur = nullptr;
    c->sur_why = "no mechanism";
    c->map_yf.clear();
    c->map_yo.clear();
    c->has_mech = false;
}

void chem_destroy(chem_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_mech(c);
    if (c->d_queue) (void)hipFree(c->d_queue);
    if (c->d_small) (void)hipFree(c->d_small);
    if (c->d_stats) (void)hipFree(c->d_stats);
    if (c->d_reftmp) (void)hipFree(c->d_reftmp);
    if (c->h_stats) (void)hipHostFree(c->h_stats);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->ev2) (void)hipEventDestroy(c->ev2);
    if (c->ev3) (void)hipEventDestroy(c->ev3);
    if (c->ev4) (void)hipEventDestroy(c->ev4);
    if (c->ev5) (void)hipEventDestroy(c->ev5);
    if (c->d_refnone) (void)hipFree(c->d_refnone);
    delete c;
}

int chem_set_stream(chem_ctx *c, void *s) {
    if (!c) return CHEM_E_INVALID_ARG;
    c->stream = (hipStream_t)s;
    return CHEM_OK;
}

const char *chem_last_error(const chem_ctx *c) { return c ? c->err.c_str() : "null context"; }

int chem_set_options(chem_ctx *c, const chem_options *o) {
    if (!c || !o) return CHEM_E_INVALID_ARG;
    if (!(o->rtol > 0.0) || !(o->atol > 0.0) || o->max_steps < 1 || !(o->hmin_frac >= 0.0) ||
        !(o->hmin_frac < 1.0) || (o->schedule != CHEM_SCHED_PLAIN && o->schedule != CHEM_SCHED_QUEUE &&
         o->schedule != CHEM_SCHED_BLOCKS) ||
        o->queue_chunk < 0 || o->queue_chunk > 4096 || o->slots_per_cu < 0 || o->slots_per_cu > 64)
        return fail(c, CHEM_E_INVALID_ARG, "invalid options");
    c->opt = *o;
    return CHEM_OK;
}

int chem_get_options(const chem_ctx *c, chem_options *o) {
    if (!c || !o) return CHEM_E_INVALID_ARG;
    *o = c->opt;
    return CHEM_OK;
}

int chem_query_slots(const chem_ctx *c, int64_t *slots) {
    if (!c || !slots || !c->has_mech) return CHEM_E_INVALID_ARG;
    if (c->big) {
        const int per_cu = c->opt.slots_per_cu > 0 ? std::min(c->opt.slots_per_cu, c->occ) : c->occ;
        *slots = (int64_t)c->num_cu * per_cu;
    } else {
        const int per_cu = c->opt.slots_per_cu > 0 ? c->opt.slots_per_cu : std::max(1, c->occ);
        *slots = (int64_t)c->num_cu * per_cu * wave_kernel_wpb(c->M);
    }
    return CHEM_OK;
}

template <class T>
static int upload(chem_ctx *c, const std::vector<T> &h, const T **dptr) {
    void *d = nullptr;
    size_t bytes = std::max<size_t>(1, h.size()) * sizeof(T);
    if (hipMalloc(&d, bytes) != hipSuccess) return fail(c, CHEM_E_OOM, "hipMalloc(%zu)", bytes);
    c->mech_bufs.push_back(d);
    if (!h.empty() && hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return fail(c, CHEM_E_HIP, "hipMemcpy mechanism");
    *dptr = (const T *)d;
    return CHEM_OK;
}

// Element-conservation data of the surrogate: E_ek = a_ek / W_k.  E E^T must
// be invertible (every element appears in some species); checked by
// Gauss-Jordan elimination with partial pivoting.
static int setup_surrogate(chem_ctx *c) {
    const int E = c->E, N = c->N;
    if (N > S_MAX_SPECIES) {
        c->sur_why = "the surrogate takes at most 61 species";
        return CHEM_OK;
    }
    if (E > 8) {
        c->sur_why = "the surrogate takes at most 8 elements";
        return CHEM_OK;
    }
    std::vector<double> Em((size_t)E * N), G((size_t)E * E, 0.0), Gi((size_t)E * E, 0.0);
    for (int e = 0; e < E; ++e)
        for (int k = 0; k < N; ++k) Em[(size_t)e * N + k] = (double)c->comp[k * E + e] / c->W[k];
    for (int a = 0; a < E; ++a)
        for (int b = 0; b < E; ++b) {
            double t = 0.0;
            for (int k = 0; k < N; ++k) t += Em[(size_t)a * N + k] * Em[(size_t)b * N + k];
            G[a * E + b] = t;
        }
    for (int a = 0; a < E; ++a) Gi[a * E + a] = 1.0;
    double gmax = 0.0;
    for (double v : G) gmax = std::max(gmax, fabs(v));
    for (int col = 0; col < E; ++col) {
        int pr = col;
        for (int r = col + 1; r < E; ++r)
            if (fabs(G[r * E + col]) > fabs(G[pr * E + col])) pr = r;
        if (!(fabs(G[pr * E + col]) > 1e-12 * gmax)) {
            c->sur_why = "element matrix is singular (an element appears in no species)";
            return CHEM_OK;
        }
        for (int q = 0; q < E; ++q) {
            std::swap(G[col * E + q], G[pr * E + q]);
            std::swap(Gi[col * E + q], Gi[pr * E + q]);
        }
        const double d = G[col * E + col];
        for (int q = 0; q < E; ++q) { G[col * E + q] /= d; Gi[col * E + q] /= d; }
        for (int r = 0; r < E; ++r) {
            if (r == col) continue;
            const double f = G[r * E + col];
            for (int q = 0; q < E; ++q) {
                G[r * E + q] -= f * G[col * E + q];
                Gi[r * E + q] -= f * Gi[col * E + q];
            }
        }
    }
    Surrogate *sp = new Surrogate();
    char err[256] = {0};
    if (sp->init(N, E, Em, err)) {
        delete sp;
        return fail(c, CHEM_E_OOM, "surrogate: %s", err);
    }
    c->sur = sp;
    c->sur_why.clear();
    return CHEM_OK;
}

// Device order of the reactions and of their species slots.  The reaction
// pass gives one reaction to each of 64 lanes and scatters its rate of
// progress with one LDS atomic per slot (r0, r1, p0, p1, p2); lanes of one
// instruction that hit the same species are serialised.  Reactions are placed
// greedily, busiest first, into the 64-wide group and slot permutation that
// adds the least to the per-group, per-slot species counts.  Present species
// stay in the leading slots (missing ones are skipped by the kernels).
// Reactions of one kind are placed in slots of their own, kind after kind
// (plain, PLOG, third-body, fall-off), so that the extra code of a PLOG rate,
// a third body (its Jacobian terms) or a fall-off rate runs in the few groups
// that hold such reactions instead of diverging in every group.  Sums change
// only by rounding order.
struct RxnSlots {
    int src;      // mechanism index
    int sp[5];    // r0 r1 p0 p1 p2, -1 missing
};
static void order_group(int N, const std::vector<int> &subset, const std::vector<int> &freq,
                        const int *rea, const int *pro, std::vector<RxnSlots> &out) {
    const int R = (int)subset.size();
    std::vector<int> byw(subset);
    auto weight = [&](int j) {
        int w = 0;
        for (int s = 0; s < 2; ++s) if (rea[2 * j + s] >= 0) w += freq[rea[2 * j + s]];
        for (int s = 0; s < 3; ++s) if (pro[3 * j + s] >= 0) w += freq[pro[3 * j + s]];
        return w;
    };
    std::stable_sort(byw.begin(), byw.end(), [&](int a, int b) { return weight(a) > weight(b); });
    const int nb = (R + 63) / 64;
    std::vector<int> fill(nb, 0), cnt((size_t)nb * 5 * N, 0);
    std::vector<std::vector<RxnSlots>> blocks(nb);
    static const int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int j : byw) {
        int rs[2], nr = 0, ps[3], np = 0;
        for (int s = 0; s < 2; ++s) if (rea[2 * j + s] >= 0) rs[nr++] = rea[2 * j + s];
        for (int s = 0; s < 3; ++s) if (pro[3 * j + s] >= 0) ps[np++] = pro[3 * j + s];
        long best = -1;
        RxnSlots pick{};
        int pick_b = -1;
        for (int b = 0; b < nb; ++b) {
            const int cap = std::min(64, R - 64 * b);
            if (fill[b] >= cap) continue;
            const int *cb = &cnt[(size_t)b * 5 * N];
            for (int ir = 0; ir < (nr == 2 ? 2 : 1); ++ir) {
                for (int ip = 0; ip < 6; ++ip) {
                    bool ok = true;
                    RxnSlots t{j, {-1, -1, -1, -1, -1}};
                    for (int s = 0; s < nr; ++s) t.sp[s] = rs[(s + ir) % nr];
                    for (int s = 0; s < np; ++s) {
                        const int q = perm3[ip][s];
                        if (q >= np) { ok = false; break; }
                        t.sp[2 + s] = ps[q];
                    }
                    if (!ok) continue;
                    long cost = 0;
                    for (int s = 0; s < 5; ++s)
                        if (t.sp[s] >= 0) cost += 2L * cb[s * N + t.sp[s]] + 1;
                    // prefer the emptier group on ties, so groups fill evenly
                    cost = cost * 128 + fill[b];
                    if (best < 0 || cost < best) { best = cost; pick = t; pick_b = b; }
                }
            }
        }
        int *cb = &cnt[(size_t)pick_b * 5 * N];
        for (int s = 0; s < 5; ++s) if (pick.sp[s] >= 0) ++cb[s * N + pick.sp[s]];
        ++fill[pick_b];
        blocks[pick_b].push_back(pick);
    }
    for (auto &bl : blocks) {
        std::sort(bl.begin(), bl.end(), [](const RxnSlots &a, const RxnSlots &b) { return a.src < b.src; });
        out.insert(out.end(), bl.begin(), bl.end());
    }
}
// kind[j]: 0 plain, 1 PLOG, 2 third-body, 3 fall-off
static std::vector<RxnSlots> order_reactions(int N, int R, const int *rea, const int *pro,
                                             const std::vector<int> &kind) {
    std::vector<int> freq(N, 0);
    for (int j = 0; j < R; ++j) {
        for (int s = 0; s < 2; ++s) if (rea[2 * j + s] >= 0) ++freq[rea[2 * j + s]];
        for (int s = 0; s < 3; ++s) if (pro[3 * j + s] >= 0) ++freq[pro[3 * j + s]];
    }
    std::vector<RxnSlots> out;
    out.reserve(R);
    for (int k = 0; k < 4; ++k) {
        std::vector<int> subset;
        for (int j = 0; j < R; ++j) if (kind[j] == k) subset.push_back(j);
        if (!subset.empty()) order_group(N, subset, freq, rea, pro, out);
    }
    return out;
}

// Facts about a validated mechanism that the packing step reuses.
struct MechFacts {
    std::vector<int> is_tb;
    std::vector<std::vector<std::pair<int, double>>> eff;   // (species, alpha - 1) per reaction
    bool any_fo = false, any_plog = false;
};

static int bad(std::string &why, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    why = buf;
    return code;
}

// Validation of a mechanism description, host only (no device).  Returns
// CHEM_OK and fills *facts, or CHEM_E_INVALID_ARG / CHEM_E_BAD_MECHANISM with
// the reason in why.
static int check_mechanism(const chem_mech_desc *m, std::string &why, MechFacts &facts) {
    const int E = m->n_elements, N = m->n_species, R = m->n_reactions;
    if (E < 1 || E > 16 || N < 1 || N > 160 || R < 1 || R > 4096)
        return bad(why, CHEM_E_BAD_MECHANISM, "sizes out of range (E=%d N=%d R=%d)", E, N, R);
    if (!m->elem_mass || !m->composition || !m->W || !m->nasa || !m->reactants || !m->products ||
        !m->A || !m->b || !m->Ea || !m->third_body || m->n_eff < 0 ||
        (m->n_eff > 0 && (!m->eff_reaction || !m->eff_species || !m->eff_value)))
        return bad(why, CHEM_E_INVALID_ARG, "null mechanism array");
    // molar masses consistent with the composition
    for (int k = 0; k < N; ++k) {
        double w = 0.0;
        for (int e = 0; e < E; ++e) {
            if (m->composition[k * E + e] < 0) return bad(why, CHEM_E_BAD_MECHANISM, "negative atom count");
            w += m->composition[k * E + e] * m->elem_mass[e];
        }
        if (!(m->W[k] > 0.0) || fabs(w - m->W[k]) > 1e-9 * m->W[k])
            return bad(why, CHEM_E_BAD_MECHANISM, "species %d: W inconsistent with composition", k);
    }
    // cp > 0 on [200, 10000] K
    for (int k = 0; k < N; ++k) {
        const double *a = m->nasa + 7 * k;
        for (int q = 0; q <= 400; ++q) {
            const double T = 200.0 + q * (9800.0 / 400.0);
            const double cp = a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
            if (!(cp > 0.0)) return bad(why, CHEM_E_BAD_MECHANISM, "species %d: cp <= 0 at %g K", k, T);
        }
        for (int i = 0; i < 7; ++i)
            if (!isfinite(a[i])) return bad(why, CHEM_E_BAD_MECHANISM, "species %d: non-finite thermo", k);
    }
    // reactions: indices, balance, parameters
    std::vector<int> is_tb(R, 0);
    for (int j = 0; j < R; ++j) {
        int nr = 0, np = 0;
        std::vector<long> bal(E, 0);
        for (int s = 0; s < 2; ++s) {
            const int k = m->reactants[2 * j + s];
            if (k < -1 || k >= N) return bad(why, CHEM_E_BAD_MECHANISM, "reaction %d: bad reactant", j);
            if (k >= 0) { ++nr; for (int e = 0; e < E; ++e) bal[e] -= m->composition[k * E + e]; }
        }
        for (int s = 0; s < 3; ++s) {
            const int k = m->products[3 * j + s];
            if (k < -1 || k >= N) return bad(why, CHEM_E_BAD_MECHANISM, "reaction %d: bad product", j);
            if (k >= 0) { ++np; for (int e = 0; e < E; ++e) bal[e] += m->composition[k * E + e]; }
        }
        if (nr == 0 || np == 0) return bad(why, CHEM_E_BAD_MECHANISM, "reaction %d: empty side", j);
        for (int e = 0; e < E; ++e)
            if (bal[e] != 0) return bad(why, CHEM_E_BAD_MECHANISM, "reaction %d: element %d unbalanced", j, e);
        if (!(m->A[j] > 0.0) || !isfinite(m->A[j]) || !isfinite(m->b[j]) || !isfinite(m->Ea[j]))
            return bad(why, CHEM_E_BAD_MECHANISM, "reaction %d: bad rate parameters", j);
        is_tb[j] = m->third_body[j] != 0;
    }
    std::vector<std::vector<std::pair<int, double>>> eff(R);
    for (int i = 0; i < m->n_eff; ++i) {
        const int j = m->eff_reaction[i], k = m->eff_species[i];
        if (j < 0 || j >= R || !is_tb[j] || k < 0 || k >= N || !(m->eff_value[i] >= 0.0) ||
            !isfinite(m->eff_value[i]))
            return bad(why, CHEM_E_BAD_MECHANISM, "bad third-body efficiency %d", i);
        for (auto &pr : eff[j])
            if (pr.first == k) return bad(why, CHEM_E_BAD_MECHANISM, "duplicate efficiency %d", i);
        eff[j].push_back({k, m->eff_value[i] - 1.0});
    }
    // fall-off forms: third-body reactions only; finite parameters, A0 > 0,
    // Troe T3, T1 > 0
    bool any_fo = false;
    if (m->falloff) {
        if (!m->falloff_params) return bad(why, CHEM_E_BAD_MECHANISM, "falloff without falloff_params");
        for (int j = 0; j < R; ++j) {
            const int t = m->falloff[j];
            if (t == 0) continue;
            const double *f = m->falloff_params + 7 * (size_t)j;
            bool ok = (t == 1 || t == 2) && is_tb[j] && f[0] > 0.0;
            for (int i = 0; i < 7; ++i) ok = ok && isfinite(f[i]);
            if (t == 2) ok = ok && f[4] > 0.0 && f[5] > 0.0;
            if (!ok) return bad(why, CHEM_E_BAD_MECHANISM, "reaction %d: bad fall-off form", j);
            any_fo = true;
        }
    }
    // third-body codes of reactions with efficiency lists must fit TB_CODE
    {
        int lists = 0;
        for (int j = 0; j < R; ++j) lists += eff[j].size() > 3;
        if (TB_LIST0 + lists - 1 > TB_CODE)
            return bad(why, CHEM_E_BAD_MECHANISM, "too many third-body efficiency lists (%d)", lists);
    }
    // PLOG tables: reactions without a third body, 2..8 entries, strictly
    // increasing positive pressures, A_i > 0, finite parameters
    bool any_plog = false;
    if (m->plog_count) {
        if (!m->plog_params) return bad(why, CHEM_E_BAD_MECHANISM, "plog_count without plog_params");
        for (int j = 0; j < R; ++j) {
            const int cnt = m->plog_count[j];
            if (cnt == 0) continue;
            bool ok = cnt >= 2 && cnt <= 8 && !is_tb[j];
            const double *t = m->plog_params + 32 * (size_t)j;
            for (int i = 0; ok && i < cnt; ++i) {
                for (int q = 0; q < 4; ++q) ok = ok && isfinite(t[4 * i + q]);
                ok = ok && t[4 * i] > 0.0 && t[4 * i + 1] > 0.0 && (i == 0 || t[4 * i] > t[4 * i - 4]);
            }
            if (!ok) return bad(why, CHEM_E_BAD_MECHANISM, "reaction %d: bad PLOG table", j);
            any_plog = true;
        }
    }

    facts.is_tb = std::move(is_tb);
    facts.eff = std::move(eff);
    facts.any_fo = any_fo;
    facts.any_plog = any_plog;
    return CHEM_OK;
}

int chem_validate_mechanism(const chem_mech_desc *m, char *msg, int32_t msg_len) {
    if (!m) return CHEM_E_INVALID_ARG;
    std::string why;
    MechFacts facts;
    const int rc = check_mechanism(m, why, facts);
    if (msg && msg_len > 0) snprintf(msg, (size_t)msg_len, "%s", rc ? why.c_str() : "");
    return rc;
}

int chem_set_mechanism(chem_ctx *c, const chem_mech_desc *m) {
    if (!c || !m) return CHEM_E_INVALID_ARG;
    MechFacts facts;
    {
        std::string why;
        const int rc = check_mechanism(m, why, facts);
        if (rc) return fail(c, rc, "%s", why.c_str());
    }
    const int E = m->n_elements, N = m->n_species, R = m->n_reactions;
    const std::vector<int> &is_tb = facts.is_tb;
    const auto &eff = facts.eff;
    const bool any_fo = facts.any_fo, any_plog = facts.any_plog;

    HIPCHK(c, hipSetDevice(c->device));
    free_mech(c);
    c->E = E; c->N = N; c->R = R;
    c->comp.assign(m->composition, m->composition + N * E);
    c->elem_mass.assign(m->elem_mass, m->elem_mass + E);
    c->W.assign(m->W, m->W + N);

    // species tables
    std::vector<double> nasa_t(14 * (size_t)N), W(N), invW(N);
    for (int k = 0; k < N; ++k) {
        const double *a = m->nasa + 7 * k;
        for (int i = 0; i < 7; ++i) nasa_t[i * N + k] = a[i];
        nasa_t[7 * N + k] = a[1] / 2.0;
        nasa_t[8 * N + k] = a[2] / 3.0;
        nasa_t[9 * N + k] = a[3] / 4.0;
        nasa_t[10 * N + k] = a[4] / 5.0;
        nasa_t[11 * N + k] = a[2] / 2.0;
        nasa_t[12 * N + k] = a[3] / 3.0;
        nasa_t[13 * N + k] = a[4] / 4.0;
        W[k] = m->W[k];
        invW[k] = 1.0 / m->W[k];
    }
    // species records
    std::vector<double> spc((size_t)N * SPC_STRIDE, 0.0);
    for (int k = 0; k < N; ++k) {
        double *r = &spc[(size_t)k * SPC_STRIDE];
        for (int i = 0; i < 14; ++i) r[i] = nasa_t[i * N + k];
        r[14] = W[k];
        r[15] = invW[k];
    }
    // reactions; efficiency lists only for third-body reactions with > 3 entries
    std::vector<RxnRec> rxn(R);
    std::vector<int> tb_ptr(1, 0), eff_sp;
    std::vector<double> eff_am1;
    std::vector<int> kind(R, 0);
    for (int j = 0; j < R; ++j)
        kind[j] = (any_fo && m->falloff[j]) ? 3 : is_tb[j] ? 2 : (any_plog && m->plog_count[j]) ? 1 : 0;
    const std::vector<RxnSlots> ord = order_reactions(N, R, m->reactants, m->products, kind);
    for (int i = 0; i < R; ++i) {
        const int j = ord[i].src;
        auto sl = [&](int s) { return ord[i].sp[s] < 0 ? N : ord[i].sp[s]; };
        const int r0 = sl(0), r1 = sl(1), p0 = sl(2), p1 = sl(3), p2 = sl(4);
        int snu = 0;
        for (int s = 0; s < 2; ++s) snu -= m->reactants[2 * j + s] >= 0;
        for (int s = 0; s < 3; ++s) snu += m->products[3 * j + s] >= 0;
        int tb = TB_NONE;
        int es[3] = {N, N, N};
        RxnRec &q = rxn[i];
        q.eff[0] = q.eff[1] = q.eff[2] = 0.0;
        if (is_tb[j]) {
            if (eff[j].size() <= 3) {
                tb = TB_INLINE;
                for (size_t i = 0; i < eff[j].size(); ++i) {
                    es[i] = eff[j][i].first;
                    q.eff[i] = eff[j][i].second;
                }
            } else {
                tb = TB_LIST0 + (int)tb_ptr.size() - 1;
                for (auto &pr : eff[j]) { eff_sp.push_back(pr.first); eff_am1.push_back(pr.second); }
                tb_ptr.push_back((int)eff_sp.size());
            }
        }
        q.idx[0] = r0 | (r1 << 16);
        q.idx[1] = p0 | (p1 << 16);
        if (any_fo && m->falloff[j]) tb |= TB_FALLOFF;
        if (any_plog && m->plog_count[j]) tb |= TB_PLOG;
        q.idx[2] = p2 | (tb << 16);
        q.idx[3] = (snu + 8) | (es[0] << 8) | (es[1] << 16) | (es[2] << 24);
        q.lnA = log(m->A[j]);
        q.b = m->b[j];
        q.EaR = m->Ea[j] / RU_J;
    }

    // fall-off parameters by reaction slot (device order)
    std::vector<double> fo(any_fo ? (size_t)R * FO_STRIDE : 1, 0.0);
    if (any_fo)
        for (int i = 0; i < R; ++i) {
            const int j = ord[i].src;
            if (!m->falloff[j]) continue;
            const double *f = m->falloff_params + 7 * (size_t)j;
            double *d = &fo[(size_t)i * FO_STRIDE];
            d[0] = log(f[0]); d[1] = f[1]; d[2] = f[2] / RU_J;
            d[3] = f[3]; d[4] = f[4]; d[5] = f[5]; d[6] = f[6];
            d[7] = (double)m->falloff[j];
        }
    // PLOG tables by reaction slot
    std::vector<double> pl(any_plog ? (size_t)R * PLOG_STRIDE : 1, 0.0);
    if (any_plog)
        for (int i = 0; i < R; ++i) {
            const int j = ord[i].src;
            const int cnt = m->plog_count[j];
            if (!cnt) continue;
            const double *t = m->plog_params + 32 * (size_t)j;
            double *d = &pl[(size_t)i * PLOG_STRIDE];
            d[0] = (double)cnt;
            for (int e = 0; e < cnt; ++e) {
                d[1 + 4 * e] = log(t[4 * e]);
                d[2 + 4 * e] = log(t[4 * e + 1]);
                d[3 + 4 * e] = t[4 * e + 2];
                d[4 + 4 * e] = t[4 * e + 3] / RU_J;
            }
        }
    MechDev &M = c->M;
    M = MechDev{};
    M.has_fo = (any_fo || any_plog) ? 1 : 0;
    M.N = N; M.R = R; M.n = N + 1;
    M.ldj = (M.n % 2) ? M.n : M.n + 1;
    int rc;
    if ((rc = upload(c, nasa_t, &M.nasa_t)) || (rc = upload(c, W, &M.W)) ||
        (rc = upload(c, invW, &M.invW)) || (rc = upload(c, spc, &M.spc)) ||
        (rc = upload(c, rxn, &M.rxn)) || (rc = upload(c, tb_ptr, &M.tb_ptr)) ||
        (rc = upload(c, eff_sp, &M.eff_sp)) || (rc = upload(c, eff_am1, &M.eff_am1)) ||
        (rc = upload(c, fo, &M.fo)) || (rc = upload(c, pl, &M.plog))) {
        free_mech(c);
        return rc;
    }
    // LDS layout (doubles)
    int off = 0;
    M.off_q = off; off += N + 1;   // production rates (+ sentinel)
    M.off_C = off; off += N + 1;
    M.off_g = off; off += N + 1;    // exp(g_k) RT/p_atm (+ sentinel 1)
    M.off_gi = off; off += N + 1;   // its reciprocal (+ sentinel 1)
    M.off_h = off; off += N + 1;
    M.off_e = off; off += N;
    M.off_cp = off; off += N;
    M.off_tb = off; off += M.n;
    M.off_sv = off; off += 128;   // triangular-solve results, by pivot step (2 x 64)
    M.lds_doubles = off;
    {
        std::vector<MechDev> one(1, M);
        const MechDev *dm = nullptr;
        if ((rc = upload(c, one, &dm))) { free_mech(c); return rc; }
        c->d_mech = const_cast<MechDev *>(dm);
    }

    if (hipMalloc((void **)&c->d_mapw, sizeof(double) * N) != hipSuccess ||
        hipMalloc((void **)&c->d_snap, sizeof(double) * (N + 1)) != hipSuccess ||
        hipMalloc((void **)&c->d_delta, sizeof(double) * N) != hipSuccess) {
        free_mech(c);
        return fail(c, CHEM_E_OOM, "hipMalloc mapping buffers");
    }
    c->NP = pick_np(M.n);
    c->occ = 0;
    if (c->NP > 0 && wave_kernel_wpb(M) > 0) c->occ = queue_occupancy(c->NP, M);
    if (c->NP < 0) {
        // workgroup-per-cell path: the iteration matrix must fit in one CU's LDS
        int max_lds = 0;
        HIPCHK(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
        if (big_lds_bytes(M.n) <= (size_t)max_lds && big_prepare(M.n) == hipSuccess) {
            const int occ = big_occupancy(M.n);
            if (occ > 0) {
                c->big = true;
                c->occ = occ;
                c->big_slots = c->num_cu * occ;
                const size_t bytes = sizeof(double) * (size_t)M.n * M.n * c->big_slots;
                if (hipMalloc((void **)&c->d_jws, bytes) != hipSuccess) {
                    free_mech(c);
                    return fail(c, CHEM_E_OOM, "hipMalloc Jacobian slots (%zu bytes)", bytes);
                }
            }
        }
    }
    if ((rc = setup_surrogate(c))) { free_mech(c); return rc; }
    c->has_mech = true;
    return CHEM_OK;
}

int chem_reserve(chem_ctx *c, int64_t max_cells) {
    if (!c || max_cells < 0 || max_cells > (int64_t)INT32_MAX) return CHEM_E_INVALID_ARG;
    if (max_cells <= c->cap) return CHEM_OK;
    if (capturing(c)) return fail(c, CHEM_E_CAPTURE_UNSAFE, "workspace growth during capture");
    HIPCHK(c, hipSetDevice(c->device));
    if (c->d_queue) {
        HIPCHK(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
        (void)hipFree(c->d_queue);
        c->d_queue = nullptr;
        c->cap = 0;
    }
    if (hipMalloc((void **)&c->d_queue, sizeof(int) * (size_t)std::max<int64_t>(1, max_cells)) != hipSuccess)
        return fail(c, CHEM_E_OOM, "hipMalloc queue (%lld cells)", (long long)max_cells);
    c->cap = max_cells;
    return CHEM_OK;
}

// Mixture-fraction weights, evaluated with separately rounded operations in a
// fixed order (see chem_map_params).
#pragma clang fp contract(off)
static void map_weights(const chem_ctx *c, const double *Yf, const double *Yo, double *w,
                        double *bf, double *bo) {
    const int E = c->E, N = c->N;
    std::vector<double> ce(E);
    for (int e = 0; e < E; ++e) {
        double zf = 0.0, zo = 0.0;
        for (int k = 0; k < N; ++k) {
            double t = (double)c->comp[k * E + e] * c->elem_mass[e];
            double tf = t * Yf[k];
            tf = tf / c->W[k];
            zf = zf + tf;
            double to = t * Yo[k];
            to = to / c->W[k];
            zo = zo + to;
        }
        ce[e] = (zf - zo) / c->elem_mass[e];
    }
    for (int k = 0; k < N; ++k) {
        double acc = 0.0;
        for (int e = 0; e < E; ++e) {
            double t = ce[e] * (double)c->comp[k * E + e];
            t = t * c->elem_mass[e];
            t = t / c->W[k];
            acc = acc + t;
        }
        w[k] = acc;
    }
    double sf = 0.0, so = 0.0;
    for (int k = 0; k < N; ++k) {
        double t = w[k] * Yf[k];
        sf = sf + t;
        t = w[k] * Yo[k];
        so = so + t;
    }
    *bf = sf;
    *bo = so;
}
#pragma clang fp contract(on)

int chem_map_reference(chem_ctx *c, int64_t n, const double *T, const double *p, const double *Y,
                       const chem_map_params *mp, uint8_t *flags, int64_t *ref_index) {
    if (!c || !mp || !ref_index || n < 0 || !mp->Y_fuel || !mp->Y_ox || !(mp->Z_tol == mp->Z_tol) ||
        (mp->use_T && !(mp->T_tol >= 0.0)))
        return fail(c, CHEM_E_INVALID_ARG, "chem_map_reference: bad arguments");
    if (n > 0 && (!T || !p || !Y || !flags)) return fail(c, CHEM_E_INVALID_ARG, "null array");
    if (!c->has_mech) return fail(c, CHEM_E_NO_MECHANISM, "no mechanism");
    HIPCHK(c, hipSetDevice(c->device));
    const int N = c->N;
    const bool same = c->map_yf.size() == (size_t)N &&
                      std::equal(c->map_yf.begin(), c->map_yf.end(), mp->Y_fuel) &&
                      std::equal(c->map_yo.begin(), c->map_yo.end(), mp->Y_ox);
    if (!same) {
        if (capturing(c)) return fail(c, CHEM_E_CAPTURE_UNSAFE, "new mapping streams during capture");
        std::vector<double> w(N);
        map_weights(c, mp->Y_fuel, mp->Y_ox, w.data(), &c->beta_f, &c->beta_ox);
        if (!(c->beta_f != c->beta_ox)) return fail(c, CHEM_E_INVALID_ARG, "fuel and oxidiser streams coincide");
        HIPCHK(c, hipMemcpy(c->d_mapw, w.data(), sizeof(double) * N, hipMemcpyHostToDevice));
        c->map_yf.assign(mp->Y_fuel, mp->Y_fuel + N);
        c->map_yo.assign(mp->Y_ox, mp->Y_ox + N);
    }
    HIPCHK(c, launch_map(n, N, T, Y, c->d_mapw, c->beta_f, c->beta_ox, mp->Z_tol, mp->T_tol,
                         mp->use_T ? 1 : 0, flags, c->d_reftmp, ref_index, c->stream));
    return CHEM_OK;
}

static int check_integrator(chem_ctx *c) {
    if (!c->has_mech) return fail(c, CHEM_E_NO_MECHANISM, "no mechanism");
    if (c->big) return CHEM_OK;
    if (c->NP < 0)
        return fail(c, CHEM_E_UNIMPL, "%d species: the iteration matrix does not fit in one CU's "
                                      "LDS", c->N);
    if (wave_kernel_wpb(c->M) == 0)
        return fail(c, CHEM_E_UNIMPL, "mechanism tables and one cell's Jacobian exceed LDS");
    return CHEM_OK;
}

// One call of the hot path: optional surrogate pass over flag-0 cells, work
// queue, Rosenbrock integration of the remaining cells, mapped-cell scatter.
// Per-call scratch of one integration call: the context's buffers (which the
// queue may grow) or the fixed array of chem_integrate_noalloc.
struct CallWork {
    int *queue;
    int *small;                  // hist[32] cursor[32] seg[8] n_active (72), ref status (76)
    unsigned long long *stats;   // [8]
    double *snap, *delta;        // reference state before the step, its increment
    int64_t *refnone;            // device -1
    bool fixed;                  // true: no allocation; nothing may grow
};

static CallWork ctx_work(chem_ctx *c) {
    return CallWork{c->d_queue, c->d_small, c->d_stats, c->d_snap, c->d_delta, c->d_refnone, false};
}

static int integrate_core(chem_ctx *c, int64_t n, double *T, const double *p, double *Y, double dt,
                          uint8_t *flags, const int64_t *ref_index, double *h, uint32_t *cost,
                          uint8_t *status, int32_t *steps, chem_stats *stats,
                          const chem_gate_params *gate, CallWork w) {
    int rc = check_integrator(c);
    if (rc) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    const bool cap = capturing(c);
    if (stats && cap) return fail(c, CHEM_E_CAPTURE_UNSAFE, "stats requested during capture");
    if (!w.fixed && c->opt.schedule == CHEM_SCHED_QUEUE && n > c->cap) {
        if ((rc = chem_reserve(c, n))) return rc;
        w.queue = c->d_queue;
    }
    if (gate && n > 0) {
        if (!c->sur || !c->sur->trained)
            return fail(c, CHEM_E_INVALID_ARG, "surrogate not available: %s",
                        c->sur ? "no parameters (train or load first)" : c->sur_why.c_str());
        if (c->sur->ws_rows < (int)std::min<int64_t>(n, 262144) && cap)
            return fail(c, CHEM_E_CAPTURE_UNSAFE, "surrogate workspace growth during capture");
    }
    hipStream_t s = c->stream;
    if (!ref_index) {
        ref_index = w.refnone;
        if (w.fixed) {
            hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, w.refnone, (int64_t)-1);
            HIPCHK(c, hipGetLastError());
        }
    }
    if (stats) HIPCHK(c, hipEventRecord(c->ev0, s));
    int *hist = w.small, *cursor = w.small + 32, *seg = w.small + 64, *nact = w.small + 72;
    int *ref_status = w.small + 76;
    HIPCHK(c, launch_queue_reset(hist, cursor, seg, nact, w.stats, ref_status, s));
    if (n > 0) {
        if (gate) {
            if (stats) HIPCHK(c, hipEventRecord(c->ev4, s));
            FeatSrc f{T, p, Y, nullptr, dt, n, c->N};
            PostIn pin{c->M.nasa_t, c->M.invW, gate->tau_T, gate->y_min, gate->margin, gate->max_dT,
                       gate->T_max};
            char err[256] = {0};
            if (c->sur->apply(f, T, Y, flags, pin, w.stats, s, err))
                return fail(c, CHEM_E_HIP, "surrogate: %s", err);
            if (stats) HIPCHK(c, hipEventRecord(c->ev5, s));
        }
        if (flags) HIPCHK(c, launch_ref_snapshot(n, c->N, T, Y, ref_index, w.snap, s));
        IntParams P{};
        P.rtol = c->opt.rtol;
        P.atol = c->opt.atol;
        P.hmin_frac = c->opt.hmin_frac;
        P.dt = dt;
        P.max_steps = c->opt.max_steps;
        P.ncells = n;
        P.T = T; P.p = p; P.Y = Y; P.h = h; P.cost = cost; P.status = status; P.steps = steps;
        P.flags = flags;
        P.stats = w.stats;
        P.ref_status = ref_status;
        int grid = 0;
        if (c->big) {
            const int per_cu = c->opt.slots_per_cu > 0 ? std::min(c->opt.slots_per_cu, c->occ) : c->occ;
            grid = (int)std::min<int64_t>(c->num_cu * per_cu, n);
        }
        if (c->opt.schedule == CHEM_SCHED_QUEUE) {
            HIPCHK(c, launch_queue_build(n, flags, c->opt.order_by_cost ? cost : nullptr, hist, cursor,
                                         nact, w.queue, s));
            P.queue = w.queue;
            P.seg_ctr = seg;
            P.n_active = nact;
            P.chunk = c->opt.queue_chunk > 0 ? c->opt.queue_chunk : 1;
            if (!c->big) {
                const int slots = c->opt.slots_per_cu > 0 ? c->opt.slots_per_cu : std::max(1, c->occ);
                grid = c->num_cu * slots;
                if (grid > n) grid = (int)n;
            }
        } else if (c->opt.schedule == CHEM_SCHED_BLOCKS) {
            P.block_static = 1;
            if (!c->big) {
                const int slots = c->opt.slots_per_cu > 0 ? c->opt.slots_per_cu : std::max(1, c->occ);
                grid = c->num_cu * slots;
                if (grid > n) grid = (int)n;
            }
        }
        if (stats) HIPCHK(c, hipEventRecord(c->ev2, s));
        if (c->big)
            HIPCHK(c, launch_integrate_big(c->M, c->d_mech, P, c->opt.schedule, grid, c->d_jws, s));
        else
            HIPCHK(c, launch_integrate(c->NP, c->M, c->d_mech, P, c->opt.schedule, grid, s));
        if (stats) HIPCHK(c, hipEventRecord(c->ev3, s));
        if (flags)
            HIPCHK(c, launch_map_scatter(n, c->N, T, Y, flags, ref_index, w.snap, w.delta,
                                         c->M.nasa_t, c->M.invW, status, cost, w.stats,
                                         ref_status, s));
    }
    if (!stats) return CHEM_OK;
    HIPCHK(c, hipEventRecord(c->ev1, s));
    HIPCHK(c, hipMemcpyAsync(c->h_stats, w.stats, 8 * sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    float ms = 0.0f, msi = 0.0f, mss = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    if (n > 0) HIPCHK(c, hipEventElapsedTime(&msi, c->ev2, c->ev3));
    if (n > 0 && gate) HIPCHK(c, hipEventElapsedTime(&mss, c->ev4, c->ev5));
    stats->cells_integrated = (int64_t)c->h_stats[0];
    stats->steps_accepted = (int64_t)c->h_stats[1];
    stats->steps_rejected = (int64_t)c->h_stats[2];
    stats->cells_failed = (int64_t)c->h_stats[3];
    stats->max_cell_steps = (int32_t)c->h_stats[4];
    stats->cells_mapped = (int64_t)c->h_stats[5];
    stats->reserved = 0;
    stats->ms_total = ms;
    stats->ms_integrate = msi;
    stats->cells_surrogate = (int64_t)c->h_stats[6];
    stats->cells_rejected = (int64_t)c->h_stats[7];
    stats->ms_surrogate = mss;
    return (int)std::min<int64_t>(stats->cells_failed, INT32_MAX);
}

int chem_integrate(chem_ctx *c, int64_t n, double *T, const double *p, double *Y, double dt,
                   const uint8_t *flags, const int64_t *ref_index, double *h, uint32_t *cost,
                   uint8_t *status, int32_t *steps, chem_stats *stats) {
    if (!c) return CHEM_E_INVALID_ARG;
    if (n < 0 || n > (int64_t)INT32_MAX || !(dt > 0.0) || !isfinite(dt))
        return fail(c, CHEM_E_INVALID_ARG, "chem_integrate: bad n or dt");
    if (n > 0 && (!T || !p || !Y)) return fail(c, CHEM_E_INVALID_ARG, "null state array");
    if (flags && !ref_index) return fail(c, CHEM_E_INVALID_ARG, "flags need ref_index");
    return integrate_core(c, n, T, p, Y, dt, const_cast<uint8_t *>(flags), ref_index, h, cost, status,
                          steps, stats, nullptr, ctx_work(c));
}

int chem_integrate_noalloc(chem_ctx *c, int64_t n, double *T, const double *p, double *Y, double dt,
                           const uint8_t *flags, const int64_t *ref_index, double *h, uint32_t *cost,
                           uint8_t *status, int32_t *steps, chem_stats *stats) {
    if (!c) return CHEM_E_INVALID_ARG;
    if (n < 0 || n > kNoAllocMaxCells || !(dt > 0.0) || !isfinite(dt))
        return fail(c, CHEM_E_INVALID_ARG,
                    "chem_integrate_noalloc: n = %lld outside [0, %lld] (the fixed workspace's "
                    "capacity) or bad dt", (long long)n, (long long)kNoAllocMaxCells);
    if (n > 0 && (!T || !p || !Y)) return fail(c, CHEM_E_INVALID_ARG, "null state array");
    if (flags && !ref_index) return fail(c, CHEM_E_INVALID_ARG, "flags need ref_index");
    if (c->has_mech && c->big)
        return fail(c, CHEM_E_UNIMPL, "chem_integrate_noalloc: mechanisms above 63 species need "
                                      "Jacobian slots sized to the device; use chem_integrate");
    if (c->has_mech && c->N + 1 > (int)((kScrDelta - kScrSnap) / sizeof(double)))
        return fail(c, CHEM_E_UNIMPL, "chem_integrate_noalloc: too many species for the fixed workspace");
    unsigned char *base = scratch_on(c->device);
    if (!base) return fail(c, CHEM_E_HIP, "chem_integrate_noalloc: workspace address not resolved");
    CallWork w{(int *)(base + kScrQueue), (int *)base, (unsigned long long *)(base + kScrStats),
               (double *)(base + kScrSnap), (double *)(base + kScrDelta), (int64_t *)(base + kScrNone),
               true};
    return integrate_core(c, n, T, p, Y, dt, const_cast<uint8_t *>(flags), ref_index, h, cost, status,
                          steps, stats, nullptr, w);
}

int chem_integrate_surrogate(chem_ctx *c, int64_t n, double *T, const double *p, double *Y,
                             double dt, uint8_t *flags, const int64_t *ref_index,
                             const chem_gate_params *gate, double *h, uint32_t *cost,
                             uint8_t *status, int32_t *steps, chem_stats *stats) {
    if (!c) return CHEM_E_INVALID_ARG;
    if (n < 0 || n > (int64_t)INT32_MAX || !(dt > 0.0) || !isfinite(dt) || !gate)
        return fail(c, CHEM_E_INVALID_ARG, "chem_integrate_surrogate: bad n, dt or gate");
    if (n > 0 && (!T || !p || !Y || !flags)) return fail(c, CHEM_E_INVALID_ARG, "null state or flags array");
    if (!(gate->tau_T >= 0.0) || !(gate->margin >= 0.0) || gate->y_min != gate->y_min ||
        !(gate->max_dT >= 0.0) || gate->T_max != gate->T_max)
        return fail(c, CHEM_E_INVALID_ARG, "bad gate parameters");
    return integrate_core(c, n, T, p, Y, dt, flags, ref_index, h, cost, status, steps, stats, gate,
                          ctx_work(c));
}

// ------------------------------------------------------------ surrogate ----
void chem_default_train_params(chem_train_params *t) {
    t->epochs = 8;
    t->batch = 4096;
    t->lr_max = 2e-3;
    t->lr_min = 2e-5;
    t->seed = 0;
    t->verbose = 0;
}

void chem_default_gate_params(chem_gate_params *g) {
    g->tau_T = 0.5;
    g->y_min = -1e-10;
    g->margin = 0.01;
    g->max_dT = 1.0;
    g->T_max = 1000.0;
}

int64_t chem_surrogate_param_count(void) { return surrogate_param_count(); }

static int check_surrogate(chem_ctx *c, bool need_trained) {
    if (!c->has_mech) return fail(c, CHEM_E_NO_MECHANISM, "no mechanism");
    if (!c->sur) return fail(c, CHEM_E_UNIMPL, "surrogate not available: %s", c->sur_why.c_str());
    if (need_trained && !c->sur->trained)
        return fail(c, CHEM_E_INVALID_ARG, "surrogate has no parameters (train or load first)");
    return CHEM_OK;
}

int chem_surrogate_train(chem_ctx *c, int64_t n, const double *T0, const double *p, const double *Y0,
                         const double *dt, const double *T1, const double *Y1,
                         const chem_train_params *tp, float *loss_history) {
    if (!c || !tp) return CHEM_E_INVALID_ARG;
    int rc = check_surrogate(c, false);
    if (rc) return rc;
    if (n < 1 || n > (int64_t)INT32_MAX || !T0 || !p || !Y0 || !dt || !T1 || !Y1 || tp->epochs < 1 ||
        tp->batch < 64 || tp->batch % 64 != 0 || tp->batch > 65536 || n < tp->batch ||
        !(tp->lr_max > 0.0) || !(tp->lr_min >= 0.0))
        return fail(c, CHEM_E_INVALID_ARG, "chem_surrogate_train: bad arguments");
    if (capturing(c)) return fail(c, CHEM_E_CAPTURE_UNSAFE, "training during capture");
    HIPCHK(c, hipSetDevice(c->device));
    FeatSrc f{T0, p, Y0, dt, 0.0, n, c->N};
    TgtSrc t{T0, Y0, T1, Y1, n, c->N};
    char err[256] = {0};
    if ((rc = c->sur->train(f, t, tp->epochs, tp->batch, tp->lr_max, tp->lr_min, tp->seed, loss_history,
                            tp->verbose, c->stream, err)))
        return fail(c, rc, "surrogate training: %s", err);
    return CHEM_OK;
}

int chem_surrogate_get_params(chem_ctx *c, float *host) {
    if (!c || !host) return CHEM_E_INVALID_ARG;
    int rc = check_surrogate(c, true);
    if (rc) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    char err[256] = {0};
    if (c->sur->get_params(host, c->stream, err)) return fail(c, CHEM_E_HIP, "%s", err);
    return CHEM_OK;
}

int chem_surrogate_set_params(chem_ctx *c, const float *host) {
    if (!c || !host) return CHEM_E_INVALID_ARG;
    int rc = check_surrogate(c, false);
    if (rc) return rc;
    const int64_t np = surrogate_param_count();
    for (int64_t i = 0; i < np; ++i)
        if (!isfinite(host[i])) return fail(c, CHEM_E_INVALID_ARG, "non-finite parameter %lld", (long long)i);
    for (int q = 0; q < S_IN; ++q)
        if (!(host[np - 5 * S_IN + q] > 0.0f) || !(host[np - 3 * S_IN + q] > 0.0f))
            return fail(c, CHEM_E_INVALID_ARG, "normalisation scales must be positive");
    HIPCHK(c, hipSetDevice(c->device));
    char err[256] = {0};
    if (c->sur->set_params(host, c->stream, err)) return fail(c, CHEM_E_HIP, "%s", err);
    return CHEM_OK;
}

static const char kSurMagic[8] = {'L', 'C', 'H', 'S', 'U', 'R', '0', '1'};

int chem_surrogate_save(chem_ctx *c, const char *path) {
    if (!c || !path) return CHEM_E_INVALID_ARG;
    const int64_t np = surrogate_param_count();
    std::vector<float> buf(np);
    int rc = chem_surrogate_get_params(c, buf.data());
    if (rc) return rc;
    FILE *fp = fopen(path, "wb");
    if (!fp) return fail(c, CHEM_E_INVALID_ARG, "cannot open %s", path);
    const int32_t hdr[2] = {c->N, c->E};
    bool ok = fwrite(kSurMagic, 1, 8, fp) == 8 && fwrite(hdr, sizeof hdr, 1, fp) == 1 &&
              fwrite(&np, sizeof np, 1, fp) == 1 && fwrite(buf.data(), sizeof(float), np, fp) == (size_t)np;
    ok = (fclose(fp) == 0) && ok;
    return ok ? CHEM_OK : fail(c, CHEM_E_INVALID_ARG, "write error on %s", path);
}

int chem_surrogate_load(chem_ctx *c, const char *path) {
    if (!c || !path) return CHEM_E_INVALID_ARG;
    int rc = check_surrogate(c, false);
    if (rc) return rc;
    FILE *fp = fopen(path, "rb");
    if (!fp) return fail(c, CHEM_E_INVALID_ARG, "cannot open %s", path);
    char magic[8];
    int32_t hdr[2];
    int64_t np = 0;
    const int64_t want = surrogate_param_count();
    std::vector<float> buf(want);
    bool ok = fread(magic, 1, 8, fp) == 8 && memcmp(magic, kSurMagic, 8) == 0 &&
              fread(hdr, sizeof hdr, 1, fp) == 1 && fread(&np, sizeof np, 1, fp) == 1 && np == want &&
              hdr[0] == c->N && hdr[1] == c->E &&
              fread(buf.data(), sizeof(float), want, fp) == (size_t)want;
    fclose(fp);
    if (!ok) return fail(c, CHEM_E_INVALID_ARG, "%s: not a surrogate file for this mechanism", path);
    return chem_surrogate_set_params(c, buf.data());
}

int chem_surrogate_forward(chem_ctx *c, int64_t n, const double *T, const double *p, const double *Y,
                           const double *dt, float *out) {
    if (!c) return CHEM_E_INVALID_ARG;
    int rc = check_surrogate(c, true);
    if (rc) return rc;
    if (n < 0 || n > (int64_t)INT32_MAX || (n > 0 && (!T || !p || !Y || !dt || !out)))
        return fail(c, CHEM_E_INVALID_ARG, "chem_surrogate_forward: bad arguments");
    if (n == 0) return CHEM_OK;
    if (capturing(c)) return fail(c, CHEM_E_CAPTURE_UNSAFE, "surrogate forward during capture");
    HIPCHK(c, hipSetDevice(c->device));
    FeatSrc f{T, p, Y, dt, 0.0, n, c->N};
    char err[256] = {0};
    if (c->sur->forward_rows(f, out, c->stream, err)) return fail(c, CHEM_E_HIP, "%s", err);
    return CHEM_OK;
}

int chem_surrogate_forward_fused(chem_ctx *c, int64_t n, const double *T, const double *p,
                                 const double *Y, const double *dt, float *out) {
    if (!c) return CHEM_E_INVALID_ARG;
    int rc = check_surrogate(c, true);
    if (rc) return rc;
    if (n < 0 || n > (int64_t)INT32_MAX || (n > 0 && (!T || !p || !Y || !dt || !out)))
        return fail(c, CHEM_E_INVALID_ARG, "chem_surrogate_forward_fused: bad arguments");
    if (n == 0) return CHEM_OK;
    if (capturing(c)) return fail(c, CHEM_E_CAPTURE_UNSAFE, "surrogate forward during capture");
    HIPCHK(c, hipSetDevice(c->device));
    FeatSrc f{T, p, Y, dt, 0.0, n, c->N};
    char err[256] = {0};
    if (c->sur->forward_fused_rows(f, out, c->stream, err)) return fail(c, CHEM_E_HIP, "%s", err);
    return CHEM_OK;
}

int chem_surrogate_loss_grad(chem_ctx *c, int64_t n, const double *T0, const double *p,
                             const double *Y0, const double *dt, const double *T1, const double *Y1,
                             float *grad, double *loss) {
    if (!c) return CHEM_E_INVALID_ARG;
    int rc = check_surrogate(c, true);
    if (rc) return rc;
    if (n < 64 || n > 65536 || n % 64 != 0 || !T0 || !p || !Y0 || !dt || !T1 || !Y1 || !grad || !loss)
        return fail(c, CHEM_E_INVALID_ARG, "chem_surrogate_loss_grad: bad arguments");
    if (capturing(c)) return fail(c, CHEM_E_CAPTURE_UNSAFE, "loss gradient during capture");
    HIPCHK(c, hipSetDevice(c->device));
    FeatSrc f{T0, p, Y0, dt, 0.0, n, c->N};
    TgtSrc t{T0, Y0, T1, Y1, n, c->N};
    char err[256] = {0};
    if (c->sur->loss_grad(f, t, grad, loss, c->stream, err)) return fail(c, CHEM_E_HIP, "%s", err);
    return CHEM_OK;
}

int chem_eval_rhs_jac(chem_ctx *c, int64_t n, const double *T, const double *p, const double *Y,
                      double *f, double *J) {
    if (!c || n < 0 || n > (int64_t)INT32_MAX || (n > 0 && (!T || !p || !Y)))
        return fail(c, CHEM_E_INVALID_ARG, "chem_eval_rhs_jac: bad arguments");
    int rc = check_integrator(c);
    if (rc) return rc;
    if (n == 0) return CHEM_OK;
    HIPCHK(c, hipSetDevice(c->device));
    IntParams P{};
    P.ncells = n;
    P.T = const_cast<double *>(T); P.p = p; P.Y = const_cast<double *>(Y);
    if (c->big) HIPCHK(c, launch_big_rhs_jac(c->M, c->d_mech, P, f, J, c->stream));
    else HIPCHK(c, launch_eval_rhs_jac(c->NP, c->M, c->d_mech, P, f, J, c->stream));
    return CHEM_OK;
}

int chem_rodas_step(chem_ctx *c, int64_t n, const double *T, const double *p, const double *Y,
                    double h, double *ynew, double *err) {
    if (!c || n < 0 || n > (int64_t)INT32_MAX || !(h > 0.0) || (n > 0 && (!T || !p || !Y || !ynew || !err)))
        return fail(c, CHEM_E_INVALID_ARG, "chem_rodas_step: bad arguments");
    int rc = check_integrator(c);
    if (rc) return rc;
    if (n == 0) return CHEM_OK;
    HIPCHK(c, hipSetDevice(c->device));
    IntParams P{};
    P.ncells = n;
    P.T = const_cast<double *>(T); P.p = p; P.Y = const_cast<double *>(Y);
    if (c->big) {
        // one Jacobian slot per cell for this check
        if (capturing(c)) return fail(c, CHEM_E_CAPTURE_UNSAFE, "chem_rodas_step allocates here");
        double *jws = nullptr;
        const size_t bytes = sizeof(double) * (size_t)c->M.n * c->M.n * (size_t)n;
        if (hipMalloc((void **)&jws, bytes) != hipSuccess)
            return fail(c, CHEM_E_OOM, "hipMalloc Jacobian slots (%zu bytes)", bytes);
        hipError_t e = launch_big_rodas_step(c->M, c->d_mech, P, h, ynew, err, jws, c->stream);
        if (e == hipSuccess) e = c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize();
        (void)hipFree(jws);
        if (e != hipSuccess) return fail(c, CHEM_E_HIP, "big rodas step: %s", hipGetErrorString(e));
        return CHEM_OK;
    }
    HIPCHK(c, launch_rodas_step(c->NP, c->M, c->d_mech, P, h, ynew, err, c->stream));
    return CHEM_OK;
}


// ---------------------------------------------------------- graphs ---------
struct chem_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int chem_graph_begin(chem_ctx *c) {
    if (!c) return CHEM_E_INVALID_ARG;
    if (!c->stream) return fail(c, CHEM_E_INVALID_ARG, "capture needs a created stream, not the null stream");
    if (capturing(c)) return fail(c, CHEM_E_CAPTURE_UNSAFE, "stream is already capturing");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->in_capture = true;
    c->capture_failed = false;
    return CHEM_OK;
}

int chem_graph_end(chem_ctx *c, chem_graph **out) {
    if (!c || !out) return CHEM_E_INVALID_ARG;
    *out = nullptr;
    if (!capturing(c)) return fail(c, CHEM_E_INVALID_ARG, "stream is not capturing");
    HIPCHK(c, hipSetDevice(c->device));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    const bool broken = c->capture_failed;
    c->in_capture = c->capture_failed = false;
    if (e != hipSuccess || !g || broken) {
        if (g) (void)hipGraphDestroy(g);
        return fail(c, CHEM_E_CAPTURE_UNSAFE, "capture invalid: %s",
                    broken ? "a recorded call failed" : hipGetErrorString(e));
    }
    chem_graph *cg = new chem_graph();
    cg->graph = g;
    e = hipGraphInstantiate(&cg->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        chem_graph_destroy(cg);
        return fail(c, CHEM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    *out = cg;
    return CHEM_OK;
}

int chem_graph_launch(chem_ctx *c, const chem_graph *g) {
    if (!c || !g || !g->exec) return CHEM_E_INVALID_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipGraphLaunch(g->exec, c->stream));
    return CHEM_OK;
}

void chem_graph_destroy(chem_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

// ---------------------------------------------------------- autotune -------
// chem_autotune's measurements, kept for the process and keyed by device
// architecture, mechanism size (species, reactions), integrator (wavefront or
// workgroup kernel, with or without fall-off / PLOG code), whether mapping
// flags take part, and the sample's size rounded down to a power of two.
static std::mutex g_tune_mu;
static std::map<std::string, std::vector<chem_tune_entry>> g_tune_cache;

static std::string tune_key(const chem_ctx *c, int64_t n, bool mapped) {
    hipDeviceProp_t prop;
    std::string arch = hipGetDeviceProperties(&prop, c->device) == hipSuccess ? prop.gcnArchName : "?";
    int lg = 0;
    while ((int64_t)2 << lg <= n) ++lg;
    char buf[160];
    snprintf(buf, sizeof buf, "%s/N%d/R%d/%s%s/%s/2^%d", arch.c_str(), c->N, c->R, c->big ? "wg" : "wave",
             c->M.has_fo ? "+fo" : "", mapped ? "mapped" : "plain", lg);
    return buf;
}

void chem_autotune_forget(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
}

int chem_autotune(chem_ctx *c, int64_t n, const double *T, const double *p, const double *Y,
                  double dt, const uint8_t *flags, const int64_t *ref_index, chem_tune_entry *res,
                  int32_t max_res, int32_t *n_res) {
    if (!c) return CHEM_E_INVALID_ARG;
    if (n < 1 || n > (int64_t)INT32_MAX || !T || !p || !Y || !(dt > 0.0) || !isfinite(dt) ||
        (flags && !ref_index) || max_res < 0 || (max_res > 0 && !res))
        return fail(c, CHEM_E_INVALID_ARG, "chem_autotune: bad arguments");
    int rc = check_integrator(c);
    if (rc) return rc;
    if (capturing(c)) return fail(c, CHEM_E_CAPTURE_UNSAFE, "autotune during capture");
    HIPCHK(c, hipSetDevice(c->device));
    const std::string key = tune_key(c, n, flags != nullptr);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            const std::vector<chem_tune_entry> &v = it->second;
            size_t b = 0;
            for (size_t i = 0; i < v.size(); ++i) {
                if (v[i].ms < v[b].ms) b = i;
                if ((int32_t)i < max_res) res[i] = v[i];
            }
            c->opt.schedule = v[b].schedule;
            c->opt.queue_chunk = v[b].queue_chunk;
            c->opt.slots_per_cu = v[b].slots_per_cu;
            if (n_res) *n_res = std::min((int32_t)v.size(), max_res);
            return CHEM_OK;
        }
    }
    if ((rc = chem_reserve(c, n))) return rc;
    const size_t nY = (size_t)c->N * n;
    double *dT = nullptr, *dY = nullptr, *dh = nullptr;
    uint32_t *dcost = nullptr, *dcost0 = nullptr;
    auto release = [&]() {
        (void)hipStreamSynchronize(c->stream);
        for (void *q : {(void *)dT, (void *)dY, (void *)dh, (void *)dcost, (void *)dcost0})
            if (q) (void)hipFree(q);
    };
    if (hipMalloc((void **)&dT, sizeof(double) * n) != hipSuccess ||
        hipMalloc((void **)&dY, sizeof(double) * nY) != hipSuccess ||
        hipMalloc((void **)&dh, sizeof(double) * n) != hipSuccess ||
        hipMalloc((void **)&dcost, sizeof(uint32_t) * n) != hipSuccess ||
        hipMalloc((void **)&dcost0, sizeof(uint32_t) * n) != hipSuccess) {
        release();
        return fail(c, CHEM_E_OOM, "chem_autotune: scratch for %lld cells", (long long)n);
    }
    hipStream_t s = c->stream;
    auto fresh = [&](const uint32_t *cost_src) -> hipError_t {
        hipError_t e;
        if ((e = hipMemcpyAsync(dT, T, sizeof(double) * n, hipMemcpyDeviceToDevice, s))) return e;
        if ((e = hipMemcpyAsync(dY, Y, sizeof(double) * nY, hipMemcpyDeviceToDevice, s))) return e;
        if ((e = hipMemsetAsync(dh, 0, sizeof(double) * n, s))) return e;
        if (cost_src) return hipMemcpyAsync(dcost, cost_src, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
        return hipMemsetAsync(dcost, 0, sizeof(uint32_t) * n, s);
    };
    const chem_options saved = c->opt;
    uint8_t *fl = const_cast<uint8_t *>(flags);
    chem_stats st{};
    // one untimed pass records the per-cell cost that orders the queue
    hipError_t e = fresh(nullptr);
    if (e != hipSuccess) { release(); return fail(c, CHEM_E_HIP, "autotune copy: %s", hipGetErrorString(e)); }
    rc = integrate_core(c, n, dT, p, dY, dt, fl, ref_index, dh, dcost, nullptr, nullptr, &st, nullptr,
                        ctx_work(c));
    if (rc < 0) { release(); return rc; }
    e = hipMemcpyAsync(dcost0, dcost, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) { release(); return fail(c, CHEM_E_HIP, "autotune copy: %s", hipGetErrorString(e)); }
    struct Cand { int sched, chunk, slots; };
    std::vector<Cand> cands;
    const int occ = std::max(1, c->occ);
    cands.push_back({CHEM_SCHED_PLAIN, 0, 0});
    std::vector<int> slot_choices{std::max(1, occ / 2)};
    if (occ != slot_choices[0]) slot_choices.push_back(occ);   // occ == 1 leaves one choice
    for (int slots : slot_choices)
        for (int chunk : {1, 2, 4, 8}) cands.push_back({CHEM_SCHED_QUEUE, chunk, slots});
    double best = INFINITY;
    chem_options best_opt = saved;
    std::vector<chem_tune_entry> measured;
    int k = 0;
    for (const Cand &cd : cands) {
        c->opt = saved;
        c->opt.schedule = cd.sched;
        c->opt.queue_chunk = cd.chunk;
        c->opt.slots_per_cu = cd.slots;
        if ((e = fresh(dcost0)) != hipSuccess) {
            c->opt = saved;
            release();
            return fail(c, CHEM_E_HIP, "autotune copy: %s", hipGetErrorString(e));
        }
        rc = integrate_core(c, n, dT, p, dY, dt, fl, ref_index, dh, dcost, nullptr, nullptr, &st, nullptr,
                        ctx_work(c));
        if (rc < 0) { c->opt = saved; release(); return rc; }
        if (k < max_res) res[k] = chem_tune_entry{cd.sched, cd.chunk, cd.slots, st.ms_total};
        measured.push_back(chem_tune_entry{cd.sched, cd.chunk, cd.slots, st.ms_total});
        ++k;
        if (st.ms_total < best) { best = st.ms_total; best_opt = c->opt; }
    }
    c->opt = best_opt;
    if (n_res) *n_res = std::min(k, max_res);
    release();
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = measured;
    }
    return CHEM_OK;
}
