// bdis_runtime.hip -- host side of the BDIS stereo library: parameter checks,
// plans, device workspace, job tables, kernel launches and the C ABI declared
// in include/bdis.h.  Paper: arXiv 2106.07136.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bdis.h"
#include "bdis_geometry.hpp"
#include "bdis_kernels.hpp"
#include "bdis_persist.hpp"
#include "bdis_search2d.hpp"
#include "bdis_lkwave.hpp"
#include "bdisnet_internal.hpp"

using namespace bdis;

// Workspace of bdis_compute_noalloc: one array per device, created when the
// library's code object is loaded on that device and kept until the process
// ends.  In host code `scratch` names a host-side stand-in, not device
// memory: the device address is looked up once per device with
// hipGetSymbolAddress (resolve_scratch) and only that address is used.
static __device__ __align__(256) char scratch[BDIS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array; `device` must be current.
hipError_t resolve_scratch(int device, char **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = static_cast<char *>(p);
    }
    *out = g_scratch[device];
    return hipSuccess;
}

constexpr int kMaxLevels = 12;
constexpr int kSupportedPatch[] = {4, 6, 8, 10, 12, 16};
constexpr int kMaxTuning = 8;
constexpr int kNetLevel = 4;  // the proposal network runs on the 1/16 pyramid level
// LK launches of at most this many blocks per CU are "small": they take the
// three-waves-per-SIMD register budget and densify the next coarser level
constexpr int kFoldBlocksPerCU = 3;
// a densification launch takes one pixel strip per thread only when the
// strips fill at least this many blocks per CU
constexpr int kStripBlocksPerCU = 4;
// A plain batch of more than kMaxJobs pairs runs as up to kMaxLanes groups
// of pairs, each on a stream of its own, so that the groups' launches overlap.
constexpr int kMaxLanes = 3;
// An LK launch (patch side <= 8) of at most this many patches per CU runs
// one wave per patch (k_lkw) instead of one lane per patch row: the same
// bits, a shorter chain per patch where the chip is far from full.
constexpr int kWavePatchesPerCU = 8;

thread_local char g_thread_err[512] = "";

void set_err(char *buf, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
}

bool patch_supported(int p) {
    for (int s : kSupportedPatch)
        if (s == p) return true;
    return false;
}

int gtab_offset(int p) {  // offset of patch p's spatial table in the packed table
    int off = 0;
    for (int s : kSupportedPatch) {
        if (s == p) return off;
        off += s * s;
    }
    return -1;
}
constexpr int kGtabFloats = 16 + 36 + 64 + 100 + 144 + 256;

bdis_status check_params(const bdis_params *p, char *err) {
    if (!p) { set_err(err, "params is NULL"); return BDIS_E_INVALID_ARG; }
    if (p->struct_size != sizeof(bdis_params)) {
        set_err(err, "params.struct_size %u != %zu", p->struct_size, sizeof(bdis_params));
        return BDIS_E_INVALID_ARG;
    }
    if (p->patch < 2 || p->patch > 64) { set_err(err, "patch %d outside [2, 64]", p->patch); return BDIS_E_INVALID_ARG; }
    if (p->stride < 1 || p->stride > p->patch) { set_err(err, "stride %d outside [1, patch]", p->stride); return BDIS_E_INVALID_ARG; }
    if (p->iters < 0 || p->iters > 1000) { set_err(err, "iters %d outside [0, 1000]", p->iters); return BDIS_E_INVALID_ARG; }
    if (!(p->sigma_r > 0.f) || !(p->sigma_s > 0.f) || !std::isfinite(p->sigma_r) || !std::isfinite(p->sigma_s)) {
        set_err(err, "sigma_r and sigma_s must be positive and finite"); return BDIS_E_INVALID_ARG;
    }
    if (p->window < 1 || p->window > 9 || (p->window % 2) == 0) { set_err(err, "window %d must be odd in [1, 9]", p->window); return BDIS_E_INVALID_ARG; }
    if (!(p->window_step >= 0.f) || !std::isfinite(p->window_step)) { set_err(err, "window_step must be >= 0"); return BDIS_E_INVALID_ARG; }
    if (!(p->gamma >= 0.f && p->gamma <= 1.f)) { set_err(err, "gamma must be in [0, 1]"); return BDIS_E_INVALID_ARG; }
    if (p->s_mode != 0 && p->s_mode != 1) { set_err(err, "s_mode must be 0 or 1"); return BDIS_E_INVALID_ARG; }
    if (p->fusion != BDIS_FUSION_BAYES && p->fusion != BDIS_FUSION_DIS) { set_err(err, "fusion must be 0 or 1"); return BDIS_E_INVALID_ARG; }
    if (p->valid_lo < 0 || p->valid_hi > 255 || p->valid_lo > p->valid_hi) { set_err(err, "need 0 <= valid_lo <= valid_hi <= 255"); return BDIS_E_INVALID_ARG; }
    if (!(p->eps_h >= 0.f) || !std::isfinite(p->eps_h)) { set_err(err, "eps_h must be >= 0"); return BDIS_E_INVALID_ARG; }
    if (!std::isfinite(p->conv_tol)) { set_err(err, "conv_tol must be finite"); return BDIS_E_INVALID_ARG; }
    if (p->precision != 0 && p->precision != 1) { set_err(err, "precision must be 0 (FP64) or 1 (FP32)"); return BDIS_E_INVALID_ARG; }
    if (p->levels < 0 || p->levels > kMaxLevels) { set_err(err, "levels %d outside [0, %d]", p->levels, kMaxLevels); return BDIS_E_INVALID_ARG; }
    if (p->levels == 0 && !(p->max_disparity > 0.f && std::isfinite(p->max_disparity))) {
        set_err(err, "levels = 0 (auto) needs max_disparity > 0"); return BDIS_E_INVALID_ARG;
    }
    if (p->init != BDIS_INIT_ZERO && p->init != BDIS_INIT_LEARNED) { set_err(err, "init must be 0 or 1"); return BDIS_E_INVALID_ARG; }
    if (p->autotune != 0 && p->autotune != 1) { set_err(err, "autotune must be 0 or 1"); return BDIS_E_INVALID_ARG; }
    if (!patch_supported(p->patch)) { set_err(err, "patch %d not built (4, 6, 8, 10, 12, 16)", p->patch); return BDIS_E_UNSUPPORTED; }
    if (p->learned_fine_levels < 1 || p->learned_fine_levels > kNetLevel) {
        set_err(err, "learned_fine_levels must be in [1, %d]", kNetLevel); return BDIS_E_INVALID_ARG;
    }
    if (p->learned_iters < 0 || p->learned_iters > 1000) { set_err(err, "learned_iters outside [0, 1000]"); return BDIS_E_INVALID_ARG; }
    if (!(p->conf_threshold >= 0.f && p->conf_threshold <= 1.f)) { set_err(err, "conf_threshold must be in [0, 1]"); return BDIS_E_INVALID_ARG; }
    return BDIS_OK;
}

int requested_levels(const bdis_params &p, float dmax) {
    if (p.levels > 0) return p.levels;
    double r = dmax / 4.0;
    int L = 1 + (r > 1.0 ? (int)std::ceil(std::log2(r) - 1e-12) : 0);
    return std::min(L, kMaxLevels);
}

// Geometry of one pair under (patch, stride).
struct Geo {
    int L;   // LK levels
    int Lp;  // pyramid levels (>= L; deeper when the network needs its level)
    int W[kMaxLevels], H[kMaxLevels], nx[kMaxLevels], ny[kMaxLevels];
    long long patches;
};

int grid_count(int n, int p, int st) { return n < p ? 0 : (n - p + st - 1) / st + 1; }

// min_pyr: pyramid levels needed beyond the LK levels (the network's level).
bool make_geo(int W, int H, int patch, int stride, int Lreq, Geo &g, int min_pyr = 0) {
    if (W < patch || H < patch) return false;
    g.L = 0;
    g.patches = 0;
    int w = W, h = H;
    for (int l = 0; l < Lreq && l < kMaxLevels; l++) {
        if (w < patch || h < patch) break;
        g.W[l] = w; g.H[l] = h;
        g.nx[l] = grid_count(w, patch, stride);
        g.ny[l] = grid_count(h, patch, stride);
        g.patches += (long long)g.nx[l] * g.ny[l];
        g.L = l + 1;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    g.Lp = g.L;
    for (int l = g.L; l < min_pyr && l < kMaxLevels; l++) {
        g.W[l] = w; g.H[l] = h;
        g.nx[l] = g.ny[l] = 0;
        g.Lp = l + 1;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    return g.L >= 1;
}

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Workspace of one pair, elements of the arithmetic type (esz bytes):
// pyramid levels >= 1 (2 images), fields U_l for LK levels l >= 1, per-level
// patch records (u, w, u0 + a status byte), and for the learned init the
// keep mask at the injection level.
struct PairWs {
    void *pyr_l[kMaxLevels], *pyr_r[kMaxLevels], *U[kMaxLevels];
    void *rec_u[kMaxLevels], *rec_w[kMaxLevels], *rec_u0[kMaxLevels];
    int8_t *rec_st[kMaxLevels];
    uint8_t *keep;
};

// inj: injection level of the learned init (0 = no learned buffers)
size_t pair_ws_bytes(const Geo &g, size_t esz, int inj = 0) {
    size_t b = 0;
    for (int l = 0; l < g.Lp; l++) {
        size_t px = (size_t)g.W[l] * g.H[l], np = (size_t)g.nx[l] * g.ny[l];
        if (l >= 1) b += 2 * align_up(px * esz);
        if (l >= 1 && l < g.L) b += align_up(px * esz);
        if (l < g.L) b += 3 * align_up(np * esz) + align_up(np);
    }
    if (inj > 0) b += align_up((size_t)g.W[inj] * g.H[inj]);
    return b;
}

void carve(char *base, const Geo &g, size_t esz, PairWs &w, int inj = 0) {
    memset(&w, 0, sizeof w);
    size_t off = 0;
    auto take = [&](size_t bytes) { char *p = base + off; off += align_up(bytes); return (void *)p; };
    for (int l = 0; l < g.Lp; l++) {
        size_t px = (size_t)g.W[l] * g.H[l], np = (size_t)g.nx[l] * g.ny[l];
        if (l >= 1) {
            w.pyr_l[l] = take(px * esz);
            w.pyr_r[l] = take(px * esz);
        }
        if (l >= 1 && l < g.L) w.U[l] = take(px * esz);
        if (l < g.L) {
            w.rec_u[l] = take(np * esz);
            w.rec_w[l] = take(np * esz);
            w.rec_u0[l] = take(np * esz);
            w.rec_st[l] = (int8_t *)take(np);
        }
    }
    if (inj > 0) w.keep = (uint8_t *)take((size_t)g.W[inj] * g.H[inj]);
}

// Same-size pairs whose network outputs share one contiguous batch.
struct NetGroup {
    int W4, H4;
    std::vector<int> pairs;  // indices into the call's pair list
    float *out = nullptr;
};

struct PairIn {
    const uint8_t *left, *right;
    float *disp;
    int W, H, pitch, dpitch;
    int patch, stride;
    float dmax;  // largest expected disparity, level-0 pixels
    Geo g;
    PairWs ws;
    int group = -1;   // learned init: network group and index in it
    int gindex = 0;
};

}  // namespace

struct bdis_ctx {
    bdis_params prm;
    int device = 0;
    char err[512] = "";
    char *ws = nullptr;
    size_t ws_bytes = 0;
    double *gtab_d = nullptr;  // spatial Gaussian tables, one per precision
    float *gtab_f = nullptr;
    bdisnet_t *net = nullptr;  // proposal network for init = BDIS_INIT_LEARNED
    bdisnet_t *owned_net = nullptr;  // created by bdis_set_net_weights (== net while attached)
    std::vector<NetGroup> groups;
    // last single-pair run, for bdis_debug_stage
    bool have_last = false;
    PairIn last;
    hipStream_t last_stream = nullptr;
    // the last plan left the level-1 field unwritten (the level-0 LK launch
    // densified level 1 for its initial shifts only); bdis_debug_stage
    // computes it on request
    bool field1_skipped = false;
    // profiling: events around each launch, resolved in bdis_get_profile
    bool profiling = false;
    struct Rec { std::string name; hipEvent_t a, b; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> spare;
    std::vector<std::string> prof_names;
    std::vector<int> prof_count;
    std::vector<double> prof_ms;
    // batch execution
    int batch_mode = 0;
    int wgs_per_cu = 0;
    // densify levels >= 1 inside the next finer level's LK launch
    bool fold_dense = true;
    // LK launches of at most this many patches per CU run k_lkw (0: never)
    int wave_patches_per_cu = kWavePatchesPerCU;
    hipStream_t cap_stream = nullptr;
    // second stream and its fork/join events (learned init: the network
    // runs beside the plain coarse levels)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    char *p_dev = nullptr;        // tasks | jobs | kparams | counters (+ error flag)
    size_t p_dev_bytes = 0;
    char *p_host = nullptr;       // pinned staging of the tables
    size_t p_host_bytes = 0;
    hipEvent_t p_upload_ev = nullptr;
    bool p_upload_pending = false;
    std::vector<char> p_last;     // last uploaded table bytes
    std::vector<char> p_key;      // batch description the tables were built for
    hipGraph_t graph = nullptr;            // persistent kernel graph (mode 2)
    hipGraphExec_t graph_exec = nullptr;
    std::vector<long long> graph_key;
    hipGraphExec_t lv_exec = nullptr;      // per-level launch graph (mode 0)
    std::vector<char> lv_key;
    int *p_err = nullptr;         // device error flag of the last persistent run
    hipStream_t last_batch_stream = nullptr;
    // streams of the pair groups a large plain batch runs side by side on
    // (lane g >= 1; lane 0 is the caller's stream), their fork/join events
    hipStream_t lanes[kMaxLanes - 1] = {};
    hipEvent_t lane_fork = nullptr, lane_join[kMaxLanes - 1] = {};
    int n_cu = 0;
    bool lane_groups = true;      // large plain batches as overlapping groups
    // this device's copy of the no-allocation scratch array (see below)
    char *scratch = nullptr;
    // autotuner table
    int ntune = 0;
    int tune_w[kMaxTuning], tune_p[kMaxTuning], tune_s[kMaxTuning];
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

#define HIPCHK(h, call)                                                              \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            set_err((h)->err, "%s failed: %s", #call, hipGetErrorString(e_));       \
            return BDIS_E_HIP;                                                       \
        }                                                                            \
    } while (0)

size_t esize(const bdis_params &p) { return p.precision == 0 ? sizeof(double) : sizeof(float); }

bdis_status fill_gtab(bdis_t *h) {
    std::vector<double> t(kGtabFloats);
    for (int p : kSupportedPatch) {
        int off = gtab_offset(p);
        double c = 0.5 * (p - 1), s = h->prm.sigma_s;
        for (int r = 0; r < p; r++)
            for (int q = 0; q < p; q++) {
                double d2 = (r - c) * (r - c) + (q - c) * (q - c);
                t[off + r * p + q] = std::exp(-d2 / (2.0 * s * s));
            }
    }
    std::vector<float> tf(t.begin(), t.end());
    HIPCHK(h, hipMemcpy(h->gtab_d, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->gtab_f, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice));
    return BDIS_OK;
}

KParams make_kparams(const bdis_params &p, int patch) {
    KParams k;
    k.iters = p.iters;
    k.window = p.window;
    k.window_step = p.window_step;
    double s = p.s_mode == 0 ? (double)p.window : (double)patch;
    k.inv_tau = 1.0 / (2.0 * (double)p.sigma_r * (double)p.sigma_r * s * s);
    // kept iff count / p^2 >= gamma, decided on integers
    int need = 0;
    while (need <= patch * patch && (double)need / ((double)patch * patch) < (double)p.gamma) need++;
    k.min_valid = need;
    k.fusion = p.fusion;
    k.vlo = p.valid_lo;
    k.vhi = p.valid_hi;
    k.eps_h = p.eps_h;
    k.conv_tol = p.conv_tol;
    return k;
}

bdis_status ensure_ws(bdis_t *h, size_t bytes) {
    if (bytes <= h->ws_bytes) return BDIS_OK;
    if (h->ws) {
        HIPCHK(h, hipDeviceSynchronize());
        (void)hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    size_t want = align_up(bytes, 1 << 20);
    if (hipMalloc(&h->ws, want) != hipSuccess) {
        (void)hipGetLastError();
        h->ws = nullptr;
        set_err(h->err, "workspace allocation of %zu bytes failed", want);
        return BDIS_E_OOM;
    }
    h->ws_bytes = want;
    return BDIS_OK;
}

// A launch: kernel kind, template selectors and its jobs (passed by value).
// K_FORK / K_JOIN launch nothing: work after a fork runs on the side stream
// (lane 1) until the join makes the main stream wait for it.  K_FORKN /
// K_JOINN do the same for the `level` group streams of a large batch.
enum Kind { K_PYR2, K_LK, K_DENSE, K_NETIN, K_NETF, K_GATE, K_FORK, K_JOIN, K_LK2, K_DENSE2, K_FORKN, K_JOINN, K_LKW };
struct Launch {
    Kind kind;
    int level;
    int patch;
    bool u8;
    bool f64;
    int blocks;
    KParams kp;
    std::vector<char> pack;  // JobPack<Job> bytes
    int lane = 0;            // 0: the caller's stream, 1: the side stream (after K_FORK)
    int ncu = 0;             // compute units the launch's build choice assumes (0: the device's)
    int group = 0;           // pair group g > 0 of a large batch: its own stream (after K_FORKN)
};

// Splits jobs into launches of at most PackCap<Job> jobs; `blocks_of` gives
// a job's block count.
template <typename Job, typename F>
void append(std::vector<Launch> &ls, Kind kind, int level, int patch, bool u8, bool f64,
            std::vector<Job> &jobs, const KParams &kp, F blocks_of) {
    constexpr size_t cap = PackCap<Job>::value;
    for (size_t s0 = 0; s0 < jobs.size(); s0 += cap) {
        JobPack<Job> pk;
        memset(&pk, 0, sizeof pk);  // padding included: packs are compared byte for byte
        pk.n = 0;
        int blocks = 0;
        for (size_t i = s0; i < jobs.size() && i < s0 + cap; i++) {
            memcpy(&pk.j[pk.n], &jobs[i], sizeof(Job));
            pk.j[pk.n].block0 = blocks;
            blocks += blocks_of(pk.j[pk.n]);
            pk.n++;
        }
        if (blocks == 0) continue;
        Launch L{kind, level, patch, u8, f64, blocks, kp, {}};
        L.pack.resize(sizeof pk);
        memcpy(L.pack.data(), &pk, sizeof pk);
        ls.push_back(std::move(L));
    }
}

int lk_bpr(int P, int nx) {
    switch (P) {
    case 4: return lk_blocks_per_row<4>(nx);
    case 6: return lk_blocks_per_row<6>(nx);
    case 8: return lk_blocks_per_row<8>(nx);
    case 10: return lk_blocks_per_row<10>(nx);
    case 12: return lk_blocks_per_row<12>(nx);
    default: return lk_blocks_per_row<16>(nx);
    }
}

// Pyramid levels 1 .. Lp-1 of every pair, two levels per launch: launch k
// writes levels 2k+1 and 2k+2 (only 2k+1 for a pair whose pyramid ends
// there).
void plan_pyramid(std::vector<Launch> &ls, const std::vector<PairIn> &pairs, int Lpmax, bool f64,
                  const KParams &kp0) {
    for (int l = 1; l < Lpmax; l += 2) {
        std::vector<Pyr2Job> jobs;
        for (const auto &p : pairs) {
            if (p.g.Lp <= l) continue;
            Pyr2Job j{};
            j.src_l = l == 1 ? (const void *)p.left : p.ws.pyr_l[l - 1];
            j.src_r = l == 1 ? (const void *)p.right : p.ws.pyr_r[l - 1];
            j.src_pitch = l == 1 ? p.pitch : p.g.W[l - 1];
            j.ws = p.g.W[l - 1]; j.hs = p.g.H[l - 1];
            j.mid_l = p.ws.pyr_l[l]; j.mid_r = p.ws.pyr_r[l];
            j.wm = p.g.W[l]; j.hm = p.g.H[l];
            j.wd = (j.wm + 1) / 2; j.hd = (j.hm + 1) / 2;
            j.has2 = p.g.Lp > l + 1 ? 1 : 0;
            if (j.has2) { j.dst_l = p.ws.pyr_l[l + 1]; j.dst_r = p.ws.pyr_r[l + 1]; }
            j.tiles_x = (j.wd + kP2X - 1) / kP2X;
            jobs.push_back(j);
        }
        append(ls, K_PYR2, l, 0, l == 1, f64, jobs, kp0,
               [](const Pyr2Job &j) { return j.tiles_x * ((j.hd + kP2Y - 1) / kP2Y); });
    }
}

bool learned(const bdis_t *h) { return h->prm.init == BDIS_INIT_LEARNED; }

// Densification of level l of pair p (the field U_l, or the output at
// level 0); keep: the learned injection level, which fills only the pixels
// the gate left.
DenseJob make_dense_job(const bdis_t *h, const PairIn &p, int l, bool keep) {
    const bool f64 = h->prm.precision == 0;
    DenseJob j{};
    j.L = l == 0 ? (const void *)p.left : p.ws.pyr_l[l];
    j.R = l == 0 ? (const void *)p.right : p.ws.pyr_r[l];
    j.pitch = l == 0 ? p.pitch : p.g.W[l];
    j.W = p.g.W[l]; j.H = p.g.H[l];
    j.patch = p.patch; j.stride = p.stride;
    j.nx = p.g.nx[l]; j.ny = p.g.ny[l];
    j.rec_u = p.ws.rec_u[l]; j.rec_w = p.ws.rec_w[l];
    j.gtab = f64 ? (const void *)(h->gtab_d + gtab_offset(p.patch))
                 : (const void *)(h->gtab_f + gtab_offset(p.patch));
    bool coarsest = l == p.g.L - 1;
    j.Uc = coarsest ? nullptr : p.ws.U[l + 1];
    j.Wc = coarsest ? 0 : p.g.W[l + 1];
    j.Hc = coarsest ? 0 : p.g.H[l + 1];
    j.mode = l == 0 ? 2 : (coarsest ? 1 : 0);
    j.U = l == 0 ? nullptr : p.ws.U[l];
    j.out = l == 0 ? p.disp : nullptr;
    j.out_pitch = p.dpitch;
    j.keep = keep ? p.ws.keep : nullptr;
    j.ppt = 1;
    // a strip of pixels per thread shares the candidate patches' records
    // (Bayesian fusion; eq. (2)'s weights depend on each pixel's residual)
    j.strip = h->prm.fusion == BDIS_FUSION_BAYES && p.stride > 1 ? p.stride : 1;
    return j;
}

// Build every launch for a set of pairs: pyramid levels 1..Lp-1, then for
// each level from the coarsest down, LK (per patch size) and the
// densification.  With the learned init, the network input, forward and
// gate run on the side stream beside the plain levels down to the injection
// level (the fallback, which needs nothing from them); the injection level's
// densification fills only the pixels the gate did not keep, and the finer
// levels use learned_iters.
void plan_launches(bdis_t *h, std::vector<PairIn> &pairs, std::vector<Launch> &ls, int ncu = 0) {
    if (ncu <= 0) ncu = h->n_cu;
    const size_t first = ls.size();
    int Lmax = 0, Lpmax = 0;
    const bool f64 = h->prm.precision == 0;
    const bool lrn = learned(h);
    const int inj = h->prm.learned_fine_levels;
    for (auto &p : pairs) {
        Lmax = std::max(Lmax, p.g.L);
        Lpmax = std::max(Lpmax, p.g.Lp);
    }
    KParams kp0 = make_kparams(h->prm, h->prm.patch);
    plan_pyramid(ls, pairs, Lpmax, f64, kp0);
    if (lrn) {
        std::vector<bdisnet::FusedJob> fused;
        std::vector<GateJob> gate;
        for (auto &p : pairs) {
            const NetGroup &G = h->groups[p.group];
            bdisnet::FusedJob j{};
            j.L = p.ws.pyr_l[kNetLevel];
            j.R = p.ws.pyr_r[kNetLevel];
            j.out = G.out + (size_t)p.gindex * G.W4 * G.H4 * 2;
            j.W = G.W4; j.H = G.H4;
            j.tiles_x = bdisnet::fused_tiles_x(G.W4);
            fused.push_back(j);
            GateJob q{};
            q.net = G.out + (size_t)p.gindex * G.W4 * G.H4 * 2;
            q.U = p.ws.U[inj];
            q.keep = p.ws.keep;
            q.W4 = G.W4; q.H4 = G.H4;
            q.Wi = p.g.W[inj]; q.Hi = p.g.H[inj];
            q.thr = h->prm.conf_threshold;
            q.sxy = 1.f / (float)(1 << (kNetLevel - inj));
            q.sd = -(float)(1 << (kNetLevel - inj));
            gate.push_back(q);
        }
        // the network, its input and the gate run on the side stream,
        // concurrently with the plain levels down to the injection level
        // (which need nothing from it); the join comes before the injection
        // level's densification, the first launch that reads the gate
        ls.push_back(Launch{K_FORK, 0, 0, false, f64, 0, kp0, {}});
        const size_t first_side = ls.size();
        // the network: input channels and the four layers in one launch per
        // pack of up to kFusedCap pairs
        for (size_t s0 = 0; s0 < fused.size(); s0 += bdisnet::kFusedCap) {
            bdisnet::FusedPack pk;
            memset(&pk, 0, sizeof pk);
            int blocks = 0;
            for (size_t i = s0; i < fused.size() && i < s0 + bdisnet::kFusedCap; i++) {
                pk.j[pk.n] = fused[i];
                pk.j[pk.n].block0 = blocks;
                blocks += bdisnet::fused_blocks(fused[i].W, fused[i].H);
                pk.n++;
            }
            Launch L{K_NETF, kNetLevel, 0, false, f64, blocks, kp0, {}};
            L.pack.resize(sizeof pk);
            memcpy(L.pack.data(), &pk, sizeof pk);
            ls.push_back(std::move(L));
        }
        append(ls, K_GATE, inj, 0, false, f64, gate, kp0,
               [](const GateJob &j) { return (j.Wi * j.Hi + kBlock - 1) / kBlock; });
        for (size_t i = first_side; i < ls.size(); i++) ls[i].lane = 1;
    }
    // Is the densification of level l + 1 of pair p folded into p's LK launch
    // at level l?  Not for the learned injection level (its densification
    // completes the gate's field) nor for eq. (2)'s fusion (it reads images).
    // Only where the LK launch is small (at most kFoldBlocksPerCU blocks per
    // CU, as for one pair): there the densify launch it saves costs more than
    // the work it adds to the LK blocks; a large batch keeps its own.
    int lk_blocks[kMaxLevels] = {0};
    for (auto &p : pairs)
        for (int l = 0; l < p.g.L; l++) lk_blocks[l] += p.g.ny[l] * lk_bpr(p.patch, p.g.nx[l]);
    auto folded = [&](const PairIn &p, int l) {
        return h->fold_dense && l >= 0 && l + 1 < p.g.L && !(lrn && l + 1 == inj) &&
               h->prm.fusion == BDIS_FUSION_BAYES && lk_blocks[l] <= kFoldBlocksPerCU * ncu;
    };
    // the level-0 LK launch densifies level 1 for its own initial shifts
    // only (no finer level reads that field)
    h->field1_skipped = pairs.size() == 1 && folded(pairs[0], 0);
    bool joined = false;
    for (int l = Lmax - 1; l >= 0; l--) {
        // With the learned init the plain levels down to the injection level
        // are the fallback.  They run whatever the gate decides (so that they
        // overlap the network); at the injection level the densification
        // fills only the pixels the gate left.
        KParams kpl = kp0;
        if (lrn && l < inj) kpl.iters = h->prm.learned_iters;
        for (int P : kSupportedPatch) {
            std::vector<LkJob> jobs;
            for (auto &p : pairs) {
                if (p.g.L <= l || p.patch != P) continue;
                LkJob j{};
                j.L = l == 0 ? (const void *)p.left : p.ws.pyr_l[l];
                j.R = l == 0 ? (const void *)p.right : p.ws.pyr_r[l];
                j.pitch = l == 0 ? p.pitch : p.g.W[l];
                j.W = p.g.W[l]; j.H = p.g.H[l];
                bool coarsest = l == p.g.L - 1;
                j.Uc = coarsest ? nullptr : p.ws.U[l + 1];
                j.Wc = coarsest ? 0 : p.g.W[l + 1];
                j.Hc = coarsest ? 0 : p.g.H[l + 1];
                j.nx = p.g.nx[l]; j.ny = p.g.ny[l]; j.stride = p.stride;
                j.reach = (int)std::ceil(std::max(0.f, p.dmax) / (float)(1 << l)) + 1;
                j.rec_u = p.ws.rec_u[l]; j.rec_w = p.ws.rec_w[l];
                j.rec_u0 = p.ws.rec_u0[l]; j.rec_st = p.ws.rec_st[l];
                if (folded(p, l)) {
                    j.rec_u1 = p.ws.rec_u[l + 1]; j.rec_w1 = p.ws.rec_w[l + 1];
                    j.gtab1 = f64 ? (const void *)(h->gtab_d + gtab_offset(p.patch))
                                  : (const void *)(h->gtab_f + gtab_offset(p.patch));
                    j.U2 = l + 2 < p.g.L ? p.ws.U[l + 2] : nullptr;
                }
                jobs.push_back(j);
            }
            KParams kpp = make_kparams(h->prm, P);
            kpp.iters = kpl.iters;
            long long npatch = 0;
            for (const LkJob &j : jobs) npatch += (long long)j.nx * j.ny;
            if (P <= 8 && npatch <= (long long)h->wave_patches_per_cu * ncu)
                append(ls, K_LKW, l, P, l == 0, f64, jobs, kpp, [](const LkJob &j) { return lkw_blocks(j.nx, j.ny); });
            else
                append(ls, K_LK, l, P, l == 0, f64, jobs, kpp,
                       [P](const LkJob &j) { return j.ny * lk_bpr(P, j.nx); });
        }
        if (lrn && l == inj) {
            ls.push_back(Launch{K_JOIN, 0, 0, false, f64, 0, kp0, {}});
            joined = true;
        }
        std::vector<DenseJob> jobs;
        for (auto &p : pairs) {
            if (p.g.L <= l || folded(p, l - 1)) continue;
            jobs.push_back(make_dense_job(h, p, l, lrn && l == inj));
        }
        // Strips pay where they still leave several blocks per CU; a small
        // densification (one pair, the coarse levels of a batch) is bound by
        // the latency of its gathers and keeps one pixel per thread.
        long long strip_threads = 0;
        for (const DenseJob &j : jobs) strip_threads += (long long)((j.W + j.strip - 1) / j.strip) * j.H;
        if (strip_threads < (long long)kStripBlocksPerCU * kBlock * ncu)
            for (DenseJob &j : jobs) j.strip = 1;
        append(ls, K_DENSE, l, 0, l == 0, f64, jobs, kp0,
               [](const DenseJob &j) { return dense_job_blocks(j); });
    }
    if (lrn && !joined) ls.push_back(Launch{K_JOIN, 0, 0, false, f64, 0, kp0, {}});  // every fork is joined
    for (size_t i = first; i < ls.size(); i++) ls[i].ncu = ncu;
}

// kernel arguments are limited to 4 KiB
static_assert(sizeof(JobPack<PyrJob>) + sizeof(KParams) <= 4000, "pyramid job pack too large");
static_assert(sizeof(JobPack<LkJob>) + sizeof(KParams) <= 4000, "LK job pack too large");
static_assert(sizeof(JobPack<DenseJob>) + sizeof(KParams) <= 4000, "densify job pack too large");
static_assert(sizeof(JobPack<NetInJob>) <= 4000 && sizeof(JobPack<GateJob>) <= 4000, "job pack too large");
static_assert(sizeof(bdisnet::FusedPack) <= 4000, "fused network job pack too large");
static_assert(sizeof(JobPack<Lk2Job>) + sizeof(KParams) <= 4000, "2-D LK job pack too large");
static_assert(sizeof(JobPack<Dense2Job>) + sizeof(KParams) <= 4000, "2-D densify job pack too large");

template <typename Job>
const JobPack<Job> &pack_of(const Launch &L) {
    return *reinterpret_cast<const JobPack<Job> *>(L.pack.data());
}

template <typename T, int P>
void launch_lk(const bdis_t *h, const Launch &L, hipStream_t s) {
    const JobPack<LkJob> &pk = pack_of<LkJob>(L);
    // one window bound per kernel (both in one kernel would cost
    // occupancy); the register-trimmed variant for launches of more than
    // three blocks per CU, where occupancy beats per-wave latency (smaller
    // launches fit at three waves per SIMD)
    const int ncu = L.ncu > 0 ? L.ncu : h->n_cu;
    const bool big = L.blocks > kFoldBlocksPerCU * ncu;
    const dim3 g(L.blocks), b(kBlock);
    if (L.kp.window <= 5) {
        if (big) {
            if (L.u8) hipLaunchKernelGGL((k_lk<T, P, true, 5, 5>), g, b, 0, s, pk, L.kp);
            else hipLaunchKernelGGL((k_lk<T, P, false, 5, 5>), g, b, 0, s, pk, L.kp);
        } else if (!L.u8 && L.blocks <= 2 * ncu) {
            // two waves per SIMD at most: room to gather the densified
            // level's first share pixel with the initial-shift taps
            hipLaunchKernelGGL((k_lk<T, P, false, 5, 2>), g, b, 0, s, pk, L.kp);
        } else {
            if (L.u8) hipLaunchKernelGGL((k_lk<T, P, true, 5, 3>), g, b, 0, s, pk, L.kp);
            else hipLaunchKernelGGL((k_lk<T, P, false, 5, 3>), g, b, 0, s, pk, L.kp);
        }
    } else {
        if (L.u8) hipLaunchKernelGGL((k_lk<T, P, true, 9, 3>), g, b, 0, s, pk, L.kp);
        else hipLaunchKernelGGL((k_lk<T, P, false, 9, 3>), g, b, 0, s, pk, L.kp);
    }
}

template <typename T, int P>
void launch_lkw(const Launch &L, hipStream_t s) {
    const JobPack<LkJob> &pk = pack_of<LkJob>(L);
    const dim3 g(L.blocks), b(kBlock);
    if (L.kp.window <= 5) {
        if (L.u8) hipLaunchKernelGGL((k_lkw<T, P, true, 5>), g, b, 0, s, pk, L.kp);
        else hipLaunchKernelGGL((k_lkw<T, P, false, 5>), g, b, 0, s, pk, L.kp);
    } else {
        if (L.u8) hipLaunchKernelGGL((k_lkw<T, P, true, 9>), g, b, 0, s, pk, L.kp);
        else hipLaunchKernelGGL((k_lkw<T, P, false, 9>), g, b, 0, s, pk, L.kp);
    }
}

template <typename T>
void launch_one(bdis_t *h, const Launch &L, hipStream_t s) {
    switch (L.kind) {
    case K_NETIN:
        hipLaunchKernelGGL(k_net_input<T>, dim3(L.blocks), dim3(kBlock), 0, s, pack_of<NetInJob>(L));
        break;
    case K_NETF: {
        bdisnet::FusedPack pk;
        memcpy(&pk, L.pack.data(), sizeof pk);
        (void)bdisnet::forward_fused(h->net, pk, L.blocks, L.f64, s);
        break;
    }
    case K_GATE:
        hipLaunchKernelGGL(k_gate<T>, dim3(L.blocks), dim3(kBlock), 0, s, pack_of<GateJob>(L));
        break;
    case K_FORK:
    case K_JOIN:
    case K_FORKN:
    case K_JOINN:
        break;  // stream ordering only (launch_all)
    case K_PYR2: {
        const JobPack<Pyr2Job> &pk = pack_of<Pyr2Job>(L);
        if (L.u8) hipLaunchKernelGGL((k_pyr2<T, true>), dim3(L.blocks), dim3(kBlock), 0, s, pk, L.kp);
        else hipLaunchKernelGGL((k_pyr2<T, false>), dim3(L.blocks), dim3(kBlock), 0, s, pk, L.kp);
        break;
    }
    case K_LK:
        switch (L.patch) {
        case 4: launch_lk<T, 4>(h, L, s); break;
        case 6: launch_lk<T, 6>(h, L, s); break;
        case 8: launch_lk<T, 8>(h, L, s); break;
        case 10: launch_lk<T, 10>(h, L, s); break;
        case 12: launch_lk<T, 12>(h, L, s); break;
        case 16: launch_lk<T, 16>(h, L, s); break;
        }
        break;
    case K_LKW:
        switch (L.patch) {
        case 4: launch_lkw<T, 4>(L, s); break;
        case 6: launch_lkw<T, 6>(L, s); break;
        case 8: launch_lkw<T, 8>(L, s); break;
        }
        break;
    case K_LK2: {
        const JobPack<Lk2Job> &pk = pack_of<Lk2Job>(L);
        const dim3 g(L.blocks), b(kBlock);
        const bool w5 = L.kp.window <= 5;
        // the build with the densification when any job densifies level + 1
        // (a pair at its coarsest level in the same launch does not)
        bool fold = false;
        for (int i = 0; i < pk.n; i++) fold = fold || pk.j[i].rec_w1 != nullptr;
#define BDIS_LK2(PP, U, WW)                                                                   \
    do {                                                                                        \
        if (fold) hipLaunchKernelGGL((k_lk2d<T, PP, U, WW, true>), g, b, 0, s, pk, L.kp);       \
        else hipLaunchKernelGGL((k_lk2d<T, PP, U, WW, false>), g, b, 0, s, pk, L.kp);           \
    } while (0)
#define BDIS_LK2_P(PP)                                                       \
    if (L.u8) { if (w5) BDIS_LK2(PP, true, 5); else BDIS_LK2(PP, true, 9); } \
    else { if (w5) BDIS_LK2(PP, false, 5); else BDIS_LK2(PP, false, 9); }
        switch (L.patch) {
        case 4: BDIS_LK2_P(4) break;
        case 6: BDIS_LK2_P(6) break;
        default: BDIS_LK2_P(8) break;
        }
#undef BDIS_LK2_P
#undef BDIS_LK2
        break;
    }
    case K_DENSE2: {
        const JobPack<Dense2Job> &pk = pack_of<Dense2Job>(L);
        if (L.u8) hipLaunchKernelGGL((k_dense2d<T, true>), dim3(L.blocks), dim3(kBlock), 0, s, pk, L.kp);
        else hipLaunchKernelGGL((k_dense2d<T, false>), dim3(L.blocks), dim3(kBlock), 0, s, pk, L.kp);
        break;
    }
    case K_DENSE: {
        const JobPack<DenseJob> &pk = pack_of<DenseJob>(L);
        if (L.u8) hipLaunchKernelGGL((k_dense<T, true>), dim3(L.blocks), dim3(kBlock), 0, s, pk, L.kp);
        else hipLaunchKernelGGL((k_dense<T, false>), dim3(L.blocks), dim3(kBlock), 0, s, pk, L.kp);
        break;
    }
    }
}

std::string launch_name(const Launch &L) {
    char buf[48];
    const char *t = L.f64 ? "f64" : "f32";
    switch (L.kind) {
    case K_PYR2: snprintf(buf, sizeof buf, "pyr2_%s_l%d", t, L.level); break;
    case K_LK: snprintf(buf, sizeof buf, "lk_%s_p%d_l%d", t, L.patch, L.level); break;
    case K_LKW: snprintf(buf, sizeof buf, "lkw_%s_p%d_l%d", t, L.patch, L.level); break;
    case K_DENSE: snprintf(buf, sizeof buf, "dense_%s_l%d", t, L.level); break;
    case K_NETIN: snprintf(buf, sizeof buf, "netin_%s", t); break;
    case K_NETF: snprintf(buf, sizeof buf, "net_forward"); break;
    case K_LK2: snprintf(buf, sizeof buf, "lk2d_%s_p%d_l%d", t, L.patch, L.level); break;
    case K_DENSE2: snprintf(buf, sizeof buf, "dense2d_%s_l%d", t, L.level); break;
    default: snprintf(buf, sizeof buf, "gate_%s", t); break;
    }
    return buf;
}

bdis_status launch_all(bdis_t *h, const std::vector<Launch> &ls, hipStream_t s);

hipEvent_t take_event(bdis_t *h) {
    if (!h->spare.empty()) {
        hipEvent_t e = h->spare.back();
        h->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// The group streams and their events (created before a graph capture too).
bdis_status ensure_lanes(bdis_t *h, int n) {
    if (!h->lane_fork) HIPCHK(h, hipEventCreateWithFlags(&h->lane_fork, hipEventDisableTiming));
    for (int g = 1; g < n && g < kMaxLanes; g++) {
        if (!h->lanes[g - 1]) HIPCHK(h, hipStreamCreateWithFlags(&h->lanes[g - 1], hipStreamNonBlocking));
        if (!h->lane_join[g - 1]) HIPCHK(h, hipEventCreateWithFlags(&h->lane_join[g - 1], hipEventDisableTiming));
    }
    return BDIS_OK;
}

bdis_status launch_all(bdis_t *h, const std::vector<Launch> &ls, hipStream_t s) {
    for (const Launch &L : ls) {
        if (L.kind == K_FORKN || L.kind == K_JOINN) {
            const int n = L.level;
            bdis_status st = ensure_lanes(h, n);
            if (st != BDIS_OK) return st;
            if (L.kind == K_FORKN) {
                HIPCHK(h, hipEventRecord(h->lane_fork, s));
                for (int g = 1; g < n; g++) HIPCHK(h, hipStreamWaitEvent(h->lanes[g - 1], h->lane_fork, 0));
            } else {
                for (int g = 1; g < n; g++) {
                    HIPCHK(h, hipEventRecord(h->lane_join[g - 1], h->lanes[g - 1]));
                    HIPCHK(h, hipStreamWaitEvent(s, h->lane_join[g - 1], 0));
                }
            }
            continue;
        }
        if (L.kind == K_FORK || L.kind == K_JOIN) {
            if (!h->side) HIPCHK(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
            if (!h->ev_fork) HIPCHK(h, hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
            if (!h->ev_join) HIPCHK(h, hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
            if (L.kind == K_FORK) {
                HIPCHK(h, hipEventRecord(h->ev_fork, s));
                HIPCHK(h, hipStreamWaitEvent(h->side, h->ev_fork, 0));
            } else {
                HIPCHK(h, hipEventRecord(h->ev_join, h->side));
                HIPCHK(h, hipStreamWaitEvent(s, h->ev_join, 0));
            }
            continue;
        }
        const hipStream_t ls_ = L.lane ? h->side : (L.group > 0 ? h->lanes[L.group - 1] : s);
        hipEvent_t a = nullptr, b = nullptr;
        if (h->profiling) {
            a = take_event(h);
            b = take_event(h);
            if (a && b) (void)hipEventRecord(a, ls_);
        }
        if (L.f64) launch_one<double>(h, L, ls_);
        else launch_one<float>(h, L, ls_);
        if (h->profiling && a && b) {
            (void)hipEventRecord(b, ls_);
            h->pending.push_back({launch_name(L), a, b});
        }
    }
    return BDIS_OK;
}

void pick_tuning(const bdis_t *h, int W, int &patch, int &stride) {
    patch = h->prm.patch;
    stride = h->prm.stride;
    if (!h->prm.autotune) return;
    for (int i = 0; i < h->ntune; i++)
        if (W <= h->tune_w[i]) { patch = h->tune_p[i]; stride = h->tune_s[i]; return; }
}

// calibration of one rectify job: finite, non-zero focal lengths
bool camera_ok(const bdis_camera &c) {
    const double v[] = {c.fx, c.fy, c.cx, c.cy, c.k1, c.k2, c.p1, c.p2, c.k3, c.nfx, c.nfy, c.ncx, c.ncy,
                        c.R[0], c.R[1], c.R[2], c.R[3], c.R[4], c.R[5], c.R[6], c.R[7], c.R[8]};
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return c.fx != 0.0 && c.fy != 0.0 && c.nfx != 0.0 && c.nfy != 0.0;
}

bdis_status check_pair(bdis_t *h, const uint8_t *L, const uint8_t *R, int W, int H, int pitch,
                       float *disp, int dpitch, int patch) {
    if (!L || !R || !disp) { set_err(h->err, "NULL image or output pointer"); return BDIS_E_INVALID_ARG; }
    if (W < patch || H < patch) { set_err(h->err, "image %dx%d smaller than the patch %d", W, H, patch); return BDIS_E_INVALID_ARG; }
    if (W > 65536 || H > 65536) { set_err(h->err, "image %dx%d too large", W, H); return BDIS_E_INVALID_ARG; }
    if (pitch < W || dpitch < W) { set_err(h->err, "pitch smaller than width"); return BDIS_E_INVALID_ARG; }
    return BDIS_OK;
}

// ---------------------------------------------------------------- persistent batch

struct PTables {
    std::vector<PTask> tasks;
    std::vector<PJob> jobs;
    std::vector<KParams> kps;
    int lds = 0;
};

// Task list of a batch in dependency order; counters live at `ctr` (device).
void build_ptables(bdis_t *h, std::vector<PairIn> &pairs, int *ctr, PTables &t) {
    const bool f64 = h->prm.precision == 0;
    const size_t esz = f64 ? sizeof(double) : sizeof(float);
    int Lmax = 0;
    for (auto &p : pairs) Lmax = std::max(Lmax, p.g.L);
    t.kps.push_back(make_kparams(h->prm, h->prm.patch));  // 0: pyramid / densify
    t.kps.push_back(make_kparams(h->prm, 8));              // 1: LK p = 8
    t.kps.push_back(make_kparams(h->prm, 12));             // 2: LK p = 12
    const int np = (int)pairs.size();
    // job index of (pair, level, kind), -1 if absent
    std::vector<int> idx((size_t)np * kMaxLevels * 3, -1);
    auto at = [&](int p, int l, int k) -> int & { return idx[((size_t)p * kMaxLevels + l) * 3 + k]; };
    auto blocks_of = [&](const PJob &j) {
        if (j.kind == PK_PYR) return pyr_blocks(j.pyr.wd, j.pyr.hd, j.pyr.ppt);
        if (j.kind == PK_LK) return j.lk.ny * lk_bpr(j.patch, j.lk.nx);
        return dense_blocks(j.dense.W, j.dense.H, j.dense.ppt);
    };
    // jobs name their dependencies by job id while the list is built; the
    // counters' device addresses are bound at the end
    std::vector<int> dep_ids;  // two per job, -1 = none
    auto add_job = [&](PJob j, int p, int l, int d0, int d1) {
        int id = (int)t.jobs.size();
        j.need0 = d0 < 0 ? 0 : blocks_of(t.jobs[d0]);
        j.need1 = d1 < 0 ? 0 : blocks_of(t.jobs[d1]);
        t.jobs.push_back(j);
        dep_ids.push_back(d0);
        dep_ids.push_back(d1);
        at(p, l, j.kind) = id;
        int nb = blocks_of(j);
        for (int b = 0; b < nb; b++) t.tasks.push_back(PTask{id, b});
    };
    for (int l = 1; l < Lmax; l++)
        for (int p = 0; p < np; p++) {
            PairIn &q = pairs[p];
            if (q.g.L <= l) continue;
            PJob j;
            memset(&j, 0, sizeof j);
            j.kind = PK_PYR; j.u8 = l == 1; j.kp = 0;
            PyrJob &y = j.pyr;
            y.src_l = l == 1 ? (const void *)q.left : q.ws.pyr_l[l - 1];
            y.src_r = l == 1 ? (const void *)q.right : q.ws.pyr_r[l - 1];
            y.src_pitch = l == 1 ? q.pitch : q.g.W[l - 1];
            y.ws = q.g.W[l - 1]; y.hs = q.g.H[l - 1];
            y.dst_l = q.ws.pyr_l[l]; y.dst_r = q.ws.pyr_r[l];
            y.wd = q.g.W[l]; y.hd = q.g.H[l];
            y.ppt = 4;
            add_job(j, p, l, l >= 2 ? at(p, l - 1, PK_PYR) : -1, -1);
        }
    for (int l = Lmax - 1; l >= 0; l--) {
        for (int p = 0; p < np; p++) {
            PairIn &q = pairs[p];
            if (q.g.L <= l) continue;
            PJob j;
            memset(&j, 0, sizeof j);
            j.kind = PK_LK; j.patch = q.patch; j.u8 = l == 0; j.kp = q.patch == 8 ? 1 : 2;
            LkJob &k = j.lk;
            k.L = l == 0 ? (const void *)q.left : q.ws.pyr_l[l];
            k.R = l == 0 ? (const void *)q.right : q.ws.pyr_r[l];
            k.pitch = l == 0 ? q.pitch : q.g.W[l];
            k.W = q.g.W[l]; k.H = q.g.H[l];
            bool coarsest = l == q.g.L - 1;
            k.Uc = coarsest ? nullptr : q.ws.U[l + 1];
            k.Wc = coarsest ? 0 : q.g.W[l + 1];
            k.Hc = coarsest ? 0 : q.g.H[l + 1];
            k.nx = q.g.nx[l]; k.ny = q.g.ny[l]; k.stride = q.stride;
            k.reach = (int)std::ceil(std::max(0.f, q.dmax) / (float)(1 << l)) + 1;
            k.rec_u = q.ws.rec_u[l]; k.rec_w = q.ws.rec_w[l];
            k.rec_u0 = q.ws.rec_u0[l]; k.rec_st = q.ws.rec_st[l];
            const int d0 = l >= 1 ? at(p, l, PK_PYR) : -1;
            const int d1 = coarsest ? -1 : at(p, l + 1, PK_DENSE);
            int lds = q.patch == 8 ? (f64 ? lk_lds_bytes<double, 8>() : lk_lds_bytes<float, 8>())
                                   : (f64 ? lk_lds_bytes<double, 12>() : lk_lds_bytes<float, 12>());
            t.lds = std::max(t.lds, lds);
            add_job(j, p, l, d0, d1);
        }
        for (int p = 0; p < np; p++) {
            PairIn &q = pairs[p];
            if (q.g.L <= l) continue;
            PJob j;
            memset(&j, 0, sizeof j);
            j.kind = PK_DENSE; j.u8 = l == 0; j.kp = 0;
            DenseJob &d = j.dense;
            d.L = l == 0 ? (const void *)q.left : q.ws.pyr_l[l];
            d.R = l == 0 ? (const void *)q.right : q.ws.pyr_r[l];
            d.pitch = l == 0 ? q.pitch : q.g.W[l];
            d.W = q.g.W[l]; d.H = q.g.H[l];
            d.patch = q.patch; d.stride = q.stride;
            d.nx = q.g.nx[l]; d.ny = q.g.ny[l];
            d.rec_u = q.ws.rec_u[l]; d.rec_w = q.ws.rec_w[l];
            d.gtab = f64 ? (const void *)(h->gtab_d + gtab_offset(q.patch))
                         : (const void *)(h->gtab_f + gtab_offset(q.patch));
            bool coarsest = l == q.g.L - 1;
            d.Uc = coarsest ? nullptr : q.ws.U[l + 1];
            d.Wc = coarsest ? 0 : q.g.W[l + 1];
            d.Hc = coarsest ? 0 : q.g.H[l + 1];
            d.mode = l == 0 ? 2 : (coarsest ? 1 : 0);
            d.U = l == 0 ? nullptr : q.ws.U[l];
            d.out = l == 0 ? q.disp : nullptr;
            d.out_pitch = q.dpitch;
            d.ppt = 4;
            add_job(j, p, l, at(p, l, PK_LK), -1);
        }
    }
    if (ctr)
        for (size_t i = 0; i < t.jobs.size(); i++) {
            PJob &j = t.jobs[i];
            j.done = ctr + i;
            j.dep0 = dep_ids[2 * i] >= 0 ? ctr + dep_ids[2 * i] : nullptr;
            j.dep1 = dep_ids[2 * i + 1] >= 0 ? ctr + dep_ids[2 * i + 1] : nullptr;
        }
}

template <typename T, int WN>
int persist_occupancy(int lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<T, WN>, kBlock, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return std::max(nb, 1);
}

bdis_status run_persistent(bdis_t *h, std::vector<PairIn> &pairs, hipStream_t s) {
    for (auto &p : pairs)
        if (!persist_patch_ok(p.patch)) {
            set_err(h->err, "the persistent batch kernel supports patch 8 and 12 (got %d)", p.patch);
            return BDIS_E_UNSUPPORTED;
        }
    const bool f64 = h->prm.precision == 0;
    // size the device area first (counter addresses go into the tables)
    PTables t;
    build_ptables(h, pairs, nullptr, t);
    const size_t njobs = t.jobs.size(), ntasks = t.tasks.size();
    const size_t o_jobs = align_up(ntasks * sizeof(PTask));
    const size_t o_kps = o_jobs + align_up(njobs * sizeof(PJob));
    const size_t o_ctr = o_kps + align_up(t.kps.size() * sizeof(KParams));
    const size_t total = o_ctr + align_up((njobs + 1) * sizeof(int));
    if (total > h->p_dev_bytes) {
        if (h->p_upload_pending) { HIPCHK(h, hipEventSynchronize(h->p_upload_ev)); h->p_upload_pending = false; }
        HIPCHK(h, hipDeviceSynchronize());
        if (h->p_dev) (void)hipFree(h->p_dev);
        if (h->p_host) (void)hipHostFree(h->p_host);
        h->p_dev = h->p_host = nullptr;
        h->p_dev_bytes = h->p_host_bytes = 0;
        size_t want = align_up(total + total / 4, 1 << 16);
        if (hipMalloc(&h->p_dev, want) != hipSuccess || hipHostMalloc(&h->p_host, want, 0) != hipSuccess) {
            (void)hipGetLastError();
            set_err(h->err, "task table allocation failed");
            return BDIS_E_OOM;
        }
        h->p_dev_bytes = h->p_host_bytes = want;
        h->p_last.clear();
        h->graph_key.clear();
    }
    int *ctr = (int *)(h->p_dev + o_ctr);
    h->p_err = ctr + njobs;
    PTables t2;
    build_ptables(h, pairs, ctr, t2);
    std::vector<char> bytes(o_ctr);
    memcpy(bytes.data(), t2.tasks.data(), ntasks * sizeof(PTask));
    memcpy(bytes.data() + o_jobs, t2.jobs.data(), njobs * sizeof(PJob));
    memcpy(bytes.data() + o_kps, t2.kps.data(), t2.kps.size() * sizeof(KParams));
    if (bytes != h->p_last) {
        if (h->p_upload_pending) { HIPCHK(h, hipEventSynchronize(h->p_upload_ev)); h->p_upload_pending = false; }
        memcpy(h->p_host, bytes.data(), bytes.size());
        HIPCHK(h, hipMemcpyAsync(h->p_dev, h->p_host, bytes.size(), hipMemcpyHostToDevice, s));
        HIPCHK(h, hipEventRecord(h->p_upload_ev, s));
        h->p_upload_pending = true;
        h->p_last = bytes;
    }
    // grid: every workgroup resident
    const bool w5 = h->prm.window <= 5;
    const int occ = f64 ? (w5 ? persist_occupancy<double, 5>(t2.lds) : persist_occupancy<double, 9>(t2.lds))
                        : (w5 ? persist_occupancy<float, 5>(t2.lds) : persist_occupancy<float, 9>(t2.lds));
    const int per_cu = h->wgs_per_cu > 0 ? std::min(h->wgs_per_cu, occ) : occ;
    const int grid = (int)std::min<long long>((long long)per_cu * h->n_cu, (long long)ntasks);
    std::vector<long long> key = {(long long)ntasks, (long long)njobs, (long long)t2.kps.size(), grid,
                                  t2.lds, f64 ? 1 : 0, w5 ? 1 : 0, (long long)(uintptr_t)h->p_dev};
    if (key != h->graph_key) {
        if (h->graph_exec) { (void)hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
        if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
        if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        const PTask *dt = (const PTask *)h->p_dev;
        const PJob *dj = (const PJob *)(h->p_dev + o_jobs);
        const KParams *dk = (const KParams *)(h->p_dev + o_kps);
        const int spin_limit = 1 << 20;
        HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        int nctr = (int)njobs + 1;
        hipLaunchKernelGGL(k_reset, dim3((nctr + kBlock - 1) / kBlock), dim3(kBlock), 0, h->cap_stream, ctr, nctr);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), t2.lds, h->cap_stream, dt, (int)ntasks, dj, dk,
                               h->p_err, spin_limit);
        };
        if (f64) {
            if (w5) go(k_persist<double, 5>);
            else go(k_persist<double, 9>);
        } else {
            if (w5) go(k_persist<float, 5>);
            else go(k_persist<float, 9>);
        }
        hipError_t e = hipStreamEndCapture(h->cap_stream, &h->graph);
        if (e != hipSuccess) { set_err(h->err, "graph capture failed: %s", hipGetErrorString(e)); return BDIS_E_HIP; }
        HIPCHK(h, hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
        h->graph_key = key;
    }
    HIPCHK(h, hipGraphLaunch(h->graph_exec, s));
    h->last_batch_stream = s;
    return BDIS_OK;
}

// Mode 0: the per-level launch sequence captured in a hipGraph, re-captured
// only when the launches (kernels, grids, job packs) change.
bdis_status run_level_graph(bdis_t *h, const std::vector<Launch> &ls, hipStream_t s) {
    std::vector<char> key;
    for (const Launch &L : ls) {
        const int hdr[9] = {(int)L.kind, L.level, L.patch, (int)L.u8, (int)L.f64, L.blocks, L.lane, L.ncu, L.group};
        key.insert(key.end(), reinterpret_cast<const char *>(hdr), reinterpret_cast<const char *>(hdr + 9));
        const char *kp = reinterpret_cast<const char *>(&L.kp);
        key.insert(key.end(), kp, kp + sizeof(KParams));
        key.insert(key.end(), L.pack.begin(), L.pack.end());
    }
    if (key != h->lv_key || !h->lv_exec) {
        if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        // the fork/join stream and events exist before the capture begins
        if (!h->side) HIPCHK(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        if (!h->ev_fork) HIPCHK(h, hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        if (!h->ev_join) HIPCHK(h, hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
        for (const Launch &L : ls)
            if (L.kind == K_FORKN) {
                bdis_status st = ensure_lanes(h, L.level);
                if (st != BDIS_OK) return st;
            }
        const bool prof = h->profiling;
        h->profiling = false;  // no event records inside the captured graph
        HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        const bdis_status la = launch_all(h, ls, h->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
        if (la != BDIS_OK) {
            if (g) (void)hipGraphDestroy(g);
            h->profiling = prof;
            return la;
        }
        h->profiling = prof;
        if (e != hipSuccess) { set_err(h->err, "graph capture failed: %s", hipGetErrorString(e)); return BDIS_E_HIP; }
        bool updated = false;
        if (h->lv_exec) {
            hipGraphExecUpdateResult res;
            hipGraphNode_t bad = nullptr;
            updated = hipGraphExecUpdate(h->lv_exec, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
            if (!updated) {
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(h->lv_exec);
                h->lv_exec = nullptr;
            }
        }
        hipError_t ie = updated ? hipSuccess : hipGraphInstantiate(&h->lv_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) { set_err(h->err, "graph instantiate failed: %s", hipGetErrorString(ie)); return BDIS_E_HIP; }
        h->lv_key.swap(key);
    }
    HIPCHK(h, hipGraphLaunch(h->lv_exec, s));
    return BDIS_OK;
}

// Shared body of bdis_compute and bdis_compute_batch.
// fixed_ws: a caller-chosen workspace of fixed_bytes (the no-allocation
// entry point); nullptr = the handle's own, grown on demand.
bdis_status run(bdis_t *h, std::vector<PairIn> &pairs, hipStream_t s, int mode = 1, char *fixed_ws = nullptr,
                size_t fixed_bytes = 0) {
    DeviceGuard dg(h->device);
    const size_t esz = esize(h->prm);
    const bool lrn = learned(h);
    const int inj = lrn ? h->prm.learned_fine_levels : 0;
    if (lrn && !h->net) { set_err(h->err, "init = learned but no network is attached (bdis_set_net)"); return BDIS_E_STATE; }
    if (lrn && mode == 2) { set_err(h->err, "the persistent batch kernel does not run the learned init"); return BDIS_E_UNSUPPORTED; }
    size_t total = 0;
    for (auto &p : pairs) {
        if (!make_geo(p.W, p.H, p.patch, p.stride, requested_levels(h->prm, p.dmax), p.g, lrn ? kNetLevel + 1 : 0)) {
            set_err(h->err, "image %dx%d smaller than patch %d", p.W, p.H, p.patch);
            return BDIS_E_INVALID_ARG;
        }
        if (lrn && (p.g.L <= inj || p.g.Lp <= kNetLevel || p.g.W[kNetLevel] < 2 || p.g.H[kNetLevel] < 2)) {
            set_err(h->err, "image %dx%d too small for the learned init (needs %d LK levels and a 1/16 level)",
                    p.W, p.H, inj + 1);
            return BDIS_E_INVALID_ARG;
        }
        total += align_up(pair_ws_bytes(p.g, esz, inj));
    }
    // network batches: pairs grouped by their 1/16-level size
    h->groups.clear();
    size_t net_bytes = 0;
    if (lrn) {
        for (size_t i = 0; i < pairs.size(); i++) {
            PairIn &p = pairs[i];
            int gi = -1;
            for (size_t k = 0; k < h->groups.size(); k++)
                if (h->groups[k].W4 == p.g.W[kNetLevel] && h->groups[k].H4 == p.g.H[kNetLevel]) gi = (int)k;
            if (gi < 0) {
                NetGroup G;
                G.W4 = p.g.W[kNetLevel];
                G.H4 = p.g.H[kNetLevel];
                h->groups.push_back(G);
                gi = (int)h->groups.size() - 1;
            }
            p.group = gi;
            p.gindex = (int)h->groups[gi].pairs.size();
            h->groups[gi].pairs.push_back((int)i);
        }
        for (const NetGroup &G : h->groups) {
            size_t px = (size_t)G.pairs.size() * G.W4 * G.H4;
            net_bytes += align_up(px * 2 * 4);
        }
    }
    char *base = fixed_ws;
    if (fixed_ws) {
        if (total + net_bytes > fixed_bytes) {
            set_err(h->err, "this request needs %zu bytes of workspace; the no-allocation scratch holds %zu",
                    total + net_bytes, fixed_bytes);
            return BDIS_E_INVALID_ARG;
        }
    } else {
        bdis_status st = ensure_ws(h, total + net_bytes);
        if (st != BDIS_OK) return st;
        base = h->ws;
    }
    size_t off = 0;
    for (auto &p : pairs) {
        carve(base + off, p.g, esz, p.ws, inj);
        off += align_up(pair_ws_bytes(p.g, esz, inj));
    }
    if (lrn) {
        for (NetGroup &G : h->groups) {
            size_t px = (size_t)G.pairs.size() * G.W4 * G.H4;
            G.out = (float *)(base + off);
            off += align_up(px * 2 * 4);
        }
    }
    if (mode == 2) return run_persistent(h, pairs, s);
    std::vector<Launch> ls;
    const int ngroups = std::min<int>(kMaxLanes, ((int)pairs.size() + kMaxJobs - 1) / kMaxJobs);
    // Pair groups are for plain batches only: the learned init's network
    // runs on the side stream, forked from and joined to the caller's stream,
    // and is not forked again from a group's stream.
    if (!lrn && h->lane_groups && ngroups > 1) {
        // Groups of pairs, each on its own stream: pairs taken largest
        // first, each to the group with the fewest pixels so far.  Every
        // group's launches are planned as for its share of the compute units.
        std::vector<int> order(pairs.size());
        for (size_t i = 0; i < order.size(); i++) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return (long long)pairs[a].W * pairs[a].H > (long long)pairs[b].W * pairs[b].H;
        });
        std::vector<std::vector<PairIn>> grp(ngroups);
        std::vector<long long> px(ngroups, 0);
        for (int i : order) {
            const int g = (int)(std::min_element(px.begin(), px.end()) - px.begin());
            grp[g].push_back(pairs[i]);
            px[g] += (long long)pairs[i].W * pairs[i].H;
        }
        const KParams kp0 = make_kparams(h->prm, h->prm.patch);
        ls.push_back(Launch{K_FORKN, ngroups, 0, false, h->prm.precision == 0, 0, kp0, {}});
        for (int g = 0; g < ngroups; g++) {
            const size_t first = ls.size();
            plan_launches(h, grp[g], ls, std::max(1, h->n_cu / ngroups));
            for (size_t i = first; i < ls.size(); i++) ls[i].group = g;
        }
        ls.push_back(Launch{K_JOINN, ngroups, 0, false, h->prm.precision == 0, 0, kp0, {}});
    } else {
        plan_launches(h, pairs, ls);
    }
    if (mode == 0) return run_level_graph(h, ls, s);
    bdis_status st2 = launch_all(h, ls, s);
    if (st2 != BDIS_OK) return st2;
    HIPCHK(h, hipGetLastError());
    return BDIS_OK;
}

// Workspace of one pair for the 2-D search: pyramid levels >= 1, the fields
// U_l and V_l of levels 1 .. L-1, and per level the records u, v, w and the
// outcome byte.
struct PairWs2 {
    void *pyr_l[kMaxLevels], *pyr_r[kMaxLevels], *U[kMaxLevels], *V[kMaxLevels];
    void *rec_u[kMaxLevels], *rec_v[kMaxLevels], *rec_w[kMaxLevels];
    int8_t *rec_st[kMaxLevels];
};

size_t pair_ws2_bytes(const Geo &g, size_t esz, PairWs2 *w, char *base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    if (w) memset(w, 0, sizeof *w);
    for (int l = 0; l < g.L; l++) {
        const size_t px = (size_t)g.W[l] * g.H[l], np = (size_t)g.nx[l] * g.ny[l];
        void *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr;
        if (l >= 1) { a = take(px * esz); b = take(px * esz); c = take(px * esz); d = take(px * esz); }
        void *ru = take(np * esz), *rv = take(np * esz), *rw = take(np * esz), *rs = take(np);
        if (w) {
            w->pyr_l[l] = a; w->pyr_r[l] = b; w->U[l] = c; w->V[l] = d;
            w->rec_u[l] = ru; w->rec_v[l] = rv; w->rec_w[l] = rw; w->rec_st[l] = (int8_t *)rs;
        }
    }
    return off;
}

// The 2-D search on a set of pairs (geometry already made, each pair's
// vertical output and pitch in vout): pyramids, then per level (coarsest
// first) the 2-D LK launch and the two-field densification of every pair
// that has the level, at most a pack of jobs per launch.
// The launches of the 2-D search for pairs ps (their workspaces ws), planned
// for ncu compute units.
void plan_2d(bdis_t *h, const std::vector<PairIn> &ps, const std::vector<PairWs2> &ws,
             const std::vector<std::pair<float *, int>> &vout, std::vector<Launch> &ls, int ncu) {
    const bdis_params &prm = h->prm;
    const bool f64 = prm.precision == 0;
    int Lmax = 0;
    for (const PairIn &p : ps) Lmax = std::max(Lmax, p.g.L);
    const KParams kp = make_kparams(prm, prm.patch);
    const size_t first = ls.size();
    plan_pyramid(ls, ps, Lmax, f64, kp);
    const void *gt = f64 ? (const void *)(h->gtab_d + gtab_offset(prm.patch))
                         : (const void *)(h->gtab_f + gtab_offset(prm.patch));
    // A small LK launch (at most kFoldBlocksPerCU blocks per CU, as the
    // coarse levels of one pair) densifies the level above it (both fields,
    // its share of them and its patches' initial-shift taps), as the 1-D
    // path's small launches do, in place of that level's densify launch.
    // The same bits either way.
    std::vector<char> fold_at(Lmax, 0);
    for (int l = 0; l < Lmax; l++) {
        long long blocks = 0;
        for (const PairIn &p : ps)
            if (p.g.L > l) blocks += lk2_blocks(p.g.nx[l], p.g.ny[l]);
        fold_at[l] = h->fold_dense && blocks <= (long long)kFoldBlocksPerCU * ncu;
    }
    for (int l = Lmax - 1; l >= 0; l--) {
        const bool fold = fold_at[l];
        std::vector<Lk2Job> lj;
        std::vector<Dense2Job> dj;
        for (size_t i = 0; i < ps.size(); i++) {
            const PairIn &p = ps[i];
            const PairWs2 &w = ws[i];
            if (p.g.L <= l) continue;
            const bool coarsest = l == p.g.L - 1;
            Lk2Job j{};
            j.L = l == 0 ? (const void *)p.left : w.pyr_l[l];
            j.R = l == 0 ? (const void *)p.right : w.pyr_r[l];
            j.Uc = coarsest ? nullptr : w.U[l + 1];
            j.Vc = coarsest ? nullptr : w.V[l + 1];
            j.rec_u = w.rec_u[l]; j.rec_v = w.rec_v[l]; j.rec_w = w.rec_w[l]; j.rec_st = w.rec_st[l];
            if (fold && !coarsest) {
                j.rec_u1 = w.rec_u[l + 1]; j.rec_v1 = w.rec_v[l + 1]; j.rec_w1 = w.rec_w[l + 1];
                j.gtab1 = gt;
                j.U2 = l + 2 < p.g.L ? w.U[l + 2] : nullptr;
                j.V2 = l + 2 < p.g.L ? w.V[l + 2] : nullptr;
            }
            j.pitch = l == 0 ? p.pitch : p.g.W[l];
            j.W = p.g.W[l]; j.H = p.g.H[l];
            j.Wc = coarsest ? 0 : p.g.W[l + 1]; j.Hc = coarsest ? 0 : p.g.H[l + 1];
            j.nx = p.g.nx[l]; j.ny = p.g.ny[l]; j.stride = p.stride;
            lj.push_back(j);
            if (l > 0 && fold_at[l - 1]) continue;  // densified by the level l - 1 LK launch
            Dense2Job d{};
            for (int f = 0; f < 2; f++) {
                DenseView &D = f == 0 ? d.du : d.dv;
                D.L = j.L; D.R = j.R;
                D.rec_u = f == 0 ? w.rec_u[l] : w.rec_v[l];
                D.rec_w = w.rec_w[l];
                D.gtab = gt;
                D.Uc = coarsest ? nullptr : (f == 0 ? w.U[l + 1] : w.V[l + 1]);
                D.pitch = j.pitch; D.W = j.W; D.H = j.H; D.patch = p.patch; D.stride = p.stride;
                D.nx = j.nx; D.ny = j.ny; D.Wc = j.Wc; D.Hc = j.Hc;
                D.mode = l == 0 ? 2 : (coarsest ? 1 : 0);
            }
            d.Uo = l == 0 ? nullptr : w.U[l];
            d.Vo = l == 0 ? nullptr : w.V[l];
            d.out_d = l == 0 ? p.disp : nullptr;
            d.out_v = l == 0 ? vout[i].first : nullptr;
            d.out_pitch = p.dpitch; d.vout_pitch = vout[i].second;
            dj.push_back(d);
        }
        append(ls, K_LK2, l, prm.patch, l == 0, f64, lj, kp,
               [](const Lk2Job &q) { return lk2_blocks(q.nx, q.ny); });
        append(ls, K_DENSE2, l, 0, l == 0, f64, dj, kp,
               [](const Dense2Job &q) { return (q.du.W * q.du.H + kBlock - 1) / kBlock; });
    }
    for (size_t i = first; i < ls.size(); i++) ls[i].ncu = ncu;
}

bdis_status run_2d(bdis_t *h, std::vector<PairIn> &ps, const std::vector<std::pair<float *, int>> &vout,
                   hipStream_t s) {
    DeviceGuard dg(h->device);
    const bdis_params &prm = h->prm;
    const size_t esz = esize(prm);
    size_t need = 0;
    for (const PairIn &p : ps) need += align_up(pair_ws2_bytes(p.g, esz, nullptr, nullptr));
    bdis_status st = ensure_ws(h, need);
    if (st != BDIS_OK) return st;
    std::vector<PairWs2> ws(ps.size());
    size_t off = 0;
    for (size_t i = 0; i < ps.size(); i++) {
        PairIn &p = ps[i];
        off += align_up(pair_ws2_bytes(p.g, esz, &ws[i], h->ws + off));
        // the pyramid pointers feed the shared pyramid planner
        memset(&p.ws, 0, sizeof p.ws);
        for (int l = 1; l < p.g.L; l++) { p.ws.pyr_l[l] = ws[i].pyr_l[l]; p.ws.pyr_r[l] = ws[i].pyr_r[l]; }
    }
    std::vector<Launch> ls;
    const int ngroups = std::min<int>(kMaxLanes, ((int)ps.size() + kMaxJobs - 1) / kMaxJobs);
    if (h->lane_groups && ngroups > 1) {
        // pair groups on streams of their own, as bdis_compute_batch's
        std::vector<int> order(ps.size());
        for (size_t i = 0; i < order.size(); i++) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return (long long)ps[a].W * ps[a].H > (long long)ps[b].W * ps[b].H;
        });
        std::vector<std::vector<int>> grp(ngroups);
        std::vector<long long> px(ngroups, 0);
        for (int i : order) {
            const int g = (int)(std::min_element(px.begin(), px.end()) - px.begin());
            grp[g].push_back(i);
            px[g] += (long long)ps[i].W * ps[i].H;
        }
        const KParams kp0 = make_kparams(prm, prm.patch);
        ls.push_back(Launch{K_FORKN, ngroups, 0, false, prm.precision == 0, 0, kp0, {}});
        for (int g = 0; g < ngroups; g++) {
            std::vector<PairIn> gp;
            std::vector<PairWs2> gw;
            std::vector<std::pair<float *, int>> gv;
            for (int i : grp[g]) { gp.push_back(ps[i]); gw.push_back(ws[i]); gv.push_back(vout[i]); }
            const size_t first = ls.size();
            plan_2d(h, gp, gw, gv, ls, std::max(1, h->n_cu / ngroups));
            for (size_t i = first; i < ls.size(); i++) ls[i].group = g;
        }
        ls.push_back(Launch{K_JOINN, ngroups, 0, false, prm.precision == 0, 0, kp0, {}});
    } else {
        plan_2d(h, ps, ws, vout, ls, h->n_cu);
    }
    if (h->batch_mode == 0 && ps.size() > 1) return run_level_graph(h, ls, s);
    st = launch_all(h, ls, s);
    if (st != BDIS_OK) return st;
    HIPCHK(h, hipGetLastError());
    return BDIS_OK;
}

// Checks that the handle's parameters suit the 2-D search.
bdis_status check_2d(bdis_t *h) {
    if (h->prm.patch > 8) {
        set_err(h->err, "the 2-D search takes patch sides up to 8 (got %d)", h->prm.patch);
        return BDIS_E_UNSUPPORTED;
    }
    if (h->prm.fusion != BDIS_FUSION_BAYES || learned(h)) {
        set_err(h->err, "the 2-D search runs the Bayesian fusion with the zero init");
        return BDIS_E_UNSUPPORTED;
    }
    return BDIS_OK;
}

// One 2-D pair's geometry: the handle's patch and stride, levels from dmax.
bdis_status make_pair_2d(bdis_t *h, PairIn &p, const uint8_t *left, const uint8_t *right, int W, int H, int pitch,
                         float *disp, int dpitch, float dmax) {
    p.left = left; p.right = right; p.disp = disp;
    p.W = W; p.H = H; p.pitch = pitch; p.dpitch = dpitch;
    p.patch = h->prm.patch; p.stride = h->prm.stride; p.dmax = dmax;
    if (!make_geo(W, H, p.patch, p.stride, requested_levels(h->prm, p.dmax), p.g)) {
        set_err(h->err, "image %dx%d smaller than patch %d", W, H, p.patch);
        return BDIS_E_INVALID_ARG;
    }
    return BDIS_OK;
}

}  // namespace

// ============================================================== C ABI

extern "C" {

void bdis_default_params(bdis_params *p) {
    if (!p) return;
    memset(p, 0, sizeof *p);
    p->struct_size = sizeof(bdis_params);
    p->levels = 5;
    p->max_disparity = 64.f;
    p->patch = 8;
    p->stride = 4;
    p->iters = 12;
    p->sigma_r = 4.f;
    p->sigma_s = 4.f;
    p->window = 5;
    p->window_step = 0.5f;
    p->gamma = 0.75f;
    p->s_mode = 0;
    p->fusion = BDIS_FUSION_BAYES;
    p->valid_lo = 1;
    p->valid_hi = 254;
    p->eps_h = 1e-6f;
    p->conv_tol = 0.05f;
    p->precision = 0;
    p->init = BDIS_INIT_ZERO;
    p->conf_threshold = 0.5f;
    p->learned_fine_levels = 2;
    p->learned_iters = 12;
    p->autotune = 0;
}

bdis_status bdis_plan(const bdis_params *p, int32_t width, int32_t height, bdis_plan_info *out) {
    bdis_status st = check_params(p, g_thread_err);
    if (st != BDIS_OK) return st;
    if (!out) { set_err(g_thread_err, "out is NULL"); return BDIS_E_INVALID_ARG; }
    Geo g;
    if (!make_geo(width, height, p->patch, p->stride, requested_levels(*p, p->max_disparity), g)) {
        set_err(g_thread_err, "image %dx%d smaller than patch %d", width, height, p->patch);
        return BDIS_E_INVALID_ARG;
    }
    memset(out, 0, sizeof *out);
    out->levels = g.L;
    for (int l = 0; l < g.L; l++) {
        out->width[l] = g.W[l]; out->height[l] = g.H[l];
        out->nx[l] = g.nx[l]; out->ny[l] = g.ny[l];
    }
    out->patches = g.patches;
    out->workspace_bytes = (int64_t)align_up(pair_ws_bytes(g, esize(*p)));
    return BDIS_OK;
}

bdis_status bdis_create(const bdis_params *p, int device, bdis_t **out) {
    if (!out) { set_err(g_thread_err, "out is NULL"); return BDIS_E_INVALID_ARG; }
    *out = nullptr;
    bdis_params def;
    bdis_default_params(&def);
    if (!p) p = &def;
    bdis_status st = check_params(p, g_thread_err);
    if (st != BDIS_OK) return st;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        set_err(g_thread_err, "no HIP device");
        return BDIS_E_NO_DEVICE;
    }
    if (device < 0 || device >= n) { set_err(g_thread_err, "device %d out of range (%d devices)", device, n); return BDIS_E_NO_DEVICE; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { set_err(g_thread_err, "hipGetDeviceProperties failed"); return BDIS_E_NO_DEVICE; }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_err(g_thread_err, "device %d is %s, this library is built for gfx950", device, prop.gcnArchName);
        return BDIS_E_NO_DEVICE;
    }
    bdis_t *h = new (std::nothrow) bdis_t();
    if (!h) { set_err(g_thread_err, "host allocation failed"); return BDIS_E_OOM; }
    h->prm = *p;
    h->device = device;
    h->n_cu = prop.multiProcessorCount;
    DeviceGuard dg(device);
    if (hipMalloc(&h->gtab_d, kGtabFloats * sizeof(double)) != hipSuccess ||
        hipMalloc(&h->gtab_f, kGtabFloats * sizeof(float)) != hipSuccess ||
        hipEventCreateWithFlags(&h->p_upload_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        set_err(g_thread_err, "device setup failed");
        bdis_destroy(h);
        return BDIS_E_HIP;
    }
    st = fill_gtab(h);
    if (st != BDIS_OK) {
        set_err(g_thread_err, "%s", h->err);
        bdis_destroy(h);
        return st;
    }
    const hipError_t se = resolve_scratch(device, &h->scratch);
    if (se != hipSuccess) {
        (void)hipGetLastError();
        set_err(g_thread_err, "hipGetSymbolAddress of the no-allocation scratch failed: %s", hipGetErrorString(se));
        bdis_destroy(h);
        return BDIS_E_HIP;
    }
    *out = h;
    return BDIS_OK;
}

bdis_status bdis_set_params(bdis_t *h, const bdis_params *p) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    bdis_status st = check_params(p, h->err);
    if (st != BDIS_OK) return st;
    DeviceGuard dg(h->device);
    HIPCHK(h, hipDeviceSynchronize());
    h->prm = *p;
    return fill_gtab(h);
}

bdis_status bdis_reserve(bdis_t *h, int32_t width, int32_t height, int32_t n_pairs) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (width < h->prm.patch || height < h->prm.patch || n_pairs < 1) {
        set_err(h->err, "bad reserve size"); return BDIS_E_INVALID_ARG;
    }
    Geo g;
    size_t worst = 0;
    int Lreq = requested_levels(h->prm, h->prm.max_disparity);
    // the learned init also needs the pyramid down to the network's level,
    // the keep mask at the injection level and the network's activations
    // (input, three hidden layers, output) for every pair
    const bool lrn = learned(h);
    const int inj = lrn ? h->prm.learned_fine_levels : 0;
    for (int p : kSupportedPatch)
        for (int s = 1; s <= p; s++)
            if (make_geo(width, height, p, s, Lreq, g, lrn ? kNetLevel + 1 : 0))
                worst = std::max(worst, align_up(pair_ws_bytes(g, sizeof(double), g.L > inj ? inj : 0)));
    size_t net = 0;
    if (lrn) {
        int w4 = width, h4 = height;
        for (int l = 0; l < kNetLevel; l++) { w4 = (w4 + 1) / 2; h4 = (h4 + 1) / 2; }
        net = align_up((size_t)n_pairs * w4 * h4 * 2 * 4);
    }
    DeviceGuard dg(h->device);
    return ensure_ws(h, worst * (size_t)n_pairs + net);
}

bdis_status bdis_compute(bdis_t *h, const uint8_t *left, const uint8_t *right, int32_t width,
                         int32_t height, int32_t pitch_bytes, float *disp, int32_t disp_pitch_elems,
                         void *stream) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    bdis_status st = check_pair(h, left, right, width, height, pitch_bytes, disp, disp_pitch_elems, h->prm.patch);
    if (st != BDIS_OK) return st;
    std::vector<PairIn> pairs(1);
    PairIn &p = pairs[0];
    p.left = left; p.right = right; p.disp = disp;
    p.W = width; p.H = height; p.pitch = pitch_bytes; p.dpitch = disp_pitch_elems;
    p.patch = h->prm.patch; p.stride = h->prm.stride;
    p.dmax = h->prm.max_disparity;
    hipStream_t s = (hipStream_t)stream;
    st = run(h, pairs, s);
    if (st != BDIS_OK) return st;
    h->have_last = true;
    h->last = pairs[0];
    h->last_stream = s;
    return BDIS_OK;
}

bdis_status bdis_compute_noalloc(bdis_t *h, const uint8_t *left, const uint8_t *right, int32_t width,
                                 int32_t height, int32_t pitch_bytes, float *disp, int32_t disp_pitch_elems,
                                 void *stream) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    bdis_status st = check_pair(h, left, right, width, height, pitch_bytes, disp, disp_pitch_elems, h->prm.patch);
    if (st != BDIS_OK) return st;
    if (learned(h)) {
        set_err(h->err, "bdis_compute_noalloc runs the plain path only (init = zero)");
        return BDIS_E_UNSUPPORTED;
    }
    if (!h->scratch) { set_err(h->err, "no scratch address for device %d", h->device); return BDIS_E_STATE; }
    std::vector<PairIn> pairs(1);
    PairIn &p = pairs[0];
    p.left = left; p.right = right; p.disp = disp;
    p.W = width; p.H = height; p.pitch = pitch_bytes; p.dpitch = disp_pitch_elems;
    p.patch = h->prm.patch; p.stride = h->prm.stride;
    p.dmax = h->prm.max_disparity;
    // direct launches without per-launch events (recording them would create events)
    const bool prof = h->profiling;
    h->profiling = false;
    st = run(h, pairs, (hipStream_t)stream, 1, h->scratch, BDIS_NOALLOC_SCRATCH_BYTES);
    h->profiling = prof;
    // the stage taps of bdis_debug_stage would point into the shared scratch
    h->have_last = false;
    return st;
}

bdis_status bdis_compute_2d(bdis_t *h, const uint8_t *left, const uint8_t *right, int32_t width, int32_t height,
                            int32_t pitch_bytes, float *disp, int32_t disp_pitch_elems, float *vdisp,
                            int32_t vdisp_pitch_elems, void *stream) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    bdis_status st = check_pair(h, left, right, width, height, pitch_bytes, disp, disp_pitch_elems, h->prm.patch);
    if (st != BDIS_OK) return st;
    if (vdisp && vdisp_pitch_elems < width) { set_err(h->err, "vertical output pitch smaller than width"); return BDIS_E_INVALID_ARG; }
    if ((st = check_2d(h)) != BDIS_OK) return st;
    std::vector<PairIn> ps(1);
    st = make_pair_2d(h, ps[0], left, right, width, height, pitch_bytes, disp, disp_pitch_elems,
                      h->prm.max_disparity);
    if (st != BDIS_OK) return st;
    std::vector<std::pair<float *, int>> vout{{vdisp, vdisp_pitch_elems}};
    st = run_2d(h, ps, vout, (hipStream_t)stream);
    h->have_last = false;
    return st;
}

bdis_status bdis_compute_batch_2d(bdis_t *h, const bdis_pair2d *pairs, int32_t n, void *stream) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!pairs || n < 1 || n > 4096) { set_err(h->err, "need 1 <= n <= 4096 pairs"); return BDIS_E_INVALID_ARG; }
    bdis_status st = check_2d(h);
    if (st != BDIS_OK) return st;
    std::vector<PairIn> ps(n);
    std::vector<std::pair<float *, int>> vout(n);
    for (int i = 0; i < n; i++) {
        const bdis_pair2d &q = pairs[i];
        st = check_pair(h, q.left, q.right, q.width, q.height, q.pitch_bytes, q.disp, q.disp_pitch_elems,
                        h->prm.patch);
        if (st != BDIS_OK) return st;
        if (q.vdisp && q.vdisp_pitch_elems < q.width) {
            set_err(h->err, "pair %d: vertical output pitch smaller than width", i);
            return BDIS_E_INVALID_ARG;
        }
        if (!(q.max_disparity >= 0.f) || !std::isfinite(q.max_disparity)) {
            set_err(h->err, "pair %d: max_disparity must be >= 0", i);
            return BDIS_E_INVALID_ARG;
        }
        st = make_pair_2d(h, ps[i], q.left, q.right, q.width, q.height, q.pitch_bytes, q.disp, q.disp_pitch_elems,
                          q.max_disparity > 0.f ? q.max_disparity : h->prm.max_disparity);
        if (st != BDIS_OK) return st;
        vout[i] = {q.vdisp, q.vdisp_pitch_elems};
    }
    st = run_2d(h, ps, vout, (hipStream_t)stream);
    h->have_last = false;
    return st;
}

bdis_status bdis_compute_batch(bdis_t *h, const bdis_pair *pairs, int32_t n, void *stream) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!pairs || n < 1 || n > 4096) { set_err(h->err, "need 1 <= n <= 4096 pairs"); return BDIS_E_INVALID_ARG; }
    std::vector<PairIn> ps(n);
    for (int i = 0; i < n; i++) {
        const bdis_pair &q = pairs[i];
        PairIn &p = ps[i];
        pick_tuning(h, q.width, p.patch, p.stride);
        bdis_status st = check_pair(h, q.left, q.right, q.width, q.height, q.pitch_bytes, q.disp,
                                    q.disp_pitch_elems, p.patch);
        if (st != BDIS_OK) return st;
        if (!(q.max_disparity >= 0.f) || !std::isfinite(q.max_disparity)) {
            set_err(h->err, "pair %d: max_disparity must be >= 0", i);
            return BDIS_E_INVALID_ARG;
        }
        p.left = q.left; p.right = q.right; p.disp = q.disp;
        p.W = q.width; p.H = q.height; p.pitch = q.pitch_bytes; p.dpitch = q.disp_pitch_elems;
        p.dmax = q.max_disparity > 0.f ? q.max_disparity : h->prm.max_disparity;
    }
    h->have_last = false;
    h->last_batch_stream = (hipStream_t)stream;
    return run(h, ps, (hipStream_t)stream, h->batch_mode);
}

bdis_status bdis_set_batch_mode(bdis_t *h, int32_t mode, int32_t wgs_per_cu) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (mode < 0 || mode > 2) { set_err(h->err, "batch mode must be 0, 1 or 2"); return BDIS_E_INVALID_ARG; }
    if (wgs_per_cu < 0 || wgs_per_cu > 64) { set_err(h->err, "wgs_per_cu must be in [0, 64]"); return BDIS_E_INVALID_ARG; }
    h->batch_mode = mode;
    if (h->wgs_per_cu != wgs_per_cu) h->graph_key.clear();
    h->wgs_per_cu = wgs_per_cu;
    return BDIS_OK;
}

bdis_status bdis_set_batch_groups(bdis_t *h, int32_t on) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (on != 0 && on != 1) { set_err(h->err, "groups must be 0 or 1"); return BDIS_E_INVALID_ARG; }
    h->lane_groups = on != 0;
    return BDIS_OK;
}

bdis_status bdis_set_wave_lk(bdis_t *h, int32_t patches_per_cu) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (patches_per_cu < 0) { set_err(h->err, "patches_per_cu must be >= 0"); return BDIS_E_INVALID_ARG; }
    h->wave_patches_per_cu = patches_per_cu;
    return BDIS_OK;
}

bdis_status bdis_set_fold_densify(bdis_t *h, int32_t on) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (on != 0 && on != 1) { set_err(h->err, "fold must be 0 or 1"); return BDIS_E_INVALID_ARG; }
    h->fold_dense = on != 0;
    return BDIS_OK;
}

bdis_status bdis_batch_error(bdis_t *h, int32_t *flag) {
    if (!h || !flag) { set_err(g_thread_err, "NULL argument"); return BDIS_E_INVALID_ARG; }
    *flag = 0;
    DeviceGuard dg(h->device);
    HIPCHK(h, hipStreamSynchronize(h->last_batch_stream));
    if (h->batch_mode == 2 && h->p_err) HIPCHK(h, hipMemcpy(flag, h->p_err, sizeof(int), hipMemcpyDeviceToHost));
    return BDIS_OK;
}

bdis_status bdis_set_net(bdis_t *h, bdisnet_t *net) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (net && bdisnet::device_of(net) != h->device) { set_err(h->err, "network is on another device"); return BDIS_E_INVALID_ARG; }
    if (h->owned_net && h->owned_net != net) {
        bdisnet_destroy(h->owned_net);  // synchronises the device first
        h->owned_net = nullptr;
    }
    h->net = net;
    h->lv_key.clear();
    return BDIS_OK;
}

bdis_status bdis_set_net_weights(bdis_t *h, const void *blob, int64_t bytes) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!blob || bytes < 32) { set_err(h->err, "checkpoint too short"); return BDIS_E_INVALID_ARG; }
    int32_t C = 0;
    memcpy(&C, static_cast<const char *>(blob) + 12, 4);
    if (C != 32 && C != 48) { set_err(h->err, "checkpoint of an unsupported network (%d channels)", C); return BDIS_E_INVALID_ARG; }
    bdisnet_t *net = nullptr;
    bdis_status st = bdisnet_create(C, h->device, &net);
    if (st != BDIS_OK) { set_err(h->err, "%s", bdisnet_last_error(nullptr)); return st; }
    st = bdisnet_load(net, blob, bytes);
    if (st != BDIS_OK) {
        set_err(h->err, "%s", bdisnet_last_error(net));
        bdisnet_destroy(net);
        return st;
    }
    st = bdis_set_net(h, net);
    if (st != BDIS_OK) { bdisnet_destroy(net); return st; }
    h->owned_net = net;
    return BDIS_OK;
}

bdis_status bdis_net_input(bdis_t *h, const bdis_pair *pairs, int32_t n, uint16_t *x, void *stream) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!pairs || n < 1 || n > 4096 || !x) { set_err(h->err, "need 1 <= n <= 4096 pairs and an output"); return BDIS_E_INVALID_ARG; }
    std::vector<PairIn> ps(n);
    for (int i = 0; i < n; i++) {
        const bdis_pair &q = pairs[i];
        PairIn &p = ps[i];
        p.patch = h->prm.patch;
        p.stride = h->prm.stride;
        bdis_status st = check_pair(h, q.left, q.right, q.width, q.height, q.pitch_bytes, q.disp ? q.disp : (float *)x,
                                    q.disp ? q.disp_pitch_elems : q.width, p.patch);
        if (st != BDIS_OK) return st;
        p.left = q.left; p.right = q.right; p.disp = q.disp;
        p.W = q.width; p.H = q.height; p.pitch = q.pitch_bytes; p.dpitch = q.disp_pitch_elems;
        p.dmax = q.max_disparity > 0.f ? q.max_disparity : h->prm.max_disparity;
        make_geo(p.W, p.H, p.patch, p.stride, 1, p.g, kNetLevel + 1);
        if (p.g.Lp <= kNetLevel || p.g.W[kNetLevel] < 2 || p.g.H[kNetLevel] < 2) {
            set_err(h->err, "pair %d too small for a 1/16 level", i);
            return BDIS_E_INVALID_ARG;
        }
        if (p.g.W[kNetLevel] != ps[0].g.W[kNetLevel] || p.g.H[kNetLevel] != ps[0].g.H[kNetLevel]) {
            set_err(h->err, "pair %d: 1/16 level size differs from pair 0", i);
            return BDIS_E_INVALID_ARG;
        }
    }
    DeviceGuard dg(h->device);
    const size_t esz = esize(h->prm);
    size_t total = 0;
    for (auto &p : ps) total += align_up(pair_ws_bytes(p.g, esz));
    bdis_status st = ensure_ws(h, total);
    if (st != BDIS_OK) return st;
    size_t off = 0;
    for (auto &p : ps) {
        carve(h->ws + off, p.g, esz, p.ws);
        off += align_up(pair_ws_bytes(p.g, esz));
    }
    const bool f64 = h->prm.precision == 0;
    KParams kp0 = make_kparams(h->prm, h->prm.patch);
    std::vector<Launch> ls;
    plan_pyramid(ls, ps, kNetLevel + 1, f64, kp0);
    std::vector<NetInJob> in;
    const size_t per = (size_t)ps[0].g.W[kNetLevel] * ps[0].g.H[kNetLevel] * kNetIn;
    for (int i = 0; i < n; i++) {
        NetInJob j{};
        j.L = ps[i].ws.pyr_l[kNetLevel];
        j.R = ps[i].ws.pyr_r[kNetLevel];
        j.x = x + per * i;
        j.W = ps[i].g.W[kNetLevel];
        j.H = ps[i].g.H[kNetLevel];
        in.push_back(j);
    }
    append(ls, K_NETIN, kNetLevel, 0, false, f64, in, kp0,
           [](const NetInJob &j) { return (j.W * j.H + kBlock - 1) / kBlock; });
    bdis_status st3 = launch_all(h, ls, (hipStream_t)stream);
    if (st3 != BDIS_OK) return st3;
    HIPCHK(h, hipGetLastError());
    return BDIS_OK;
}

bdis_status bdis_set_tuning(bdis_t *h, int32_t n, const int32_t *max_width, const int32_t *patch,
                            const int32_t *stride) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (n < 0 || n > kMaxTuning || (n > 0 && (!max_width || !patch || !stride))) {
        set_err(h->err, "bad tuning table"); return BDIS_E_INVALID_ARG;
    }
    for (int i = 0; i < n; i++) {
        if (!patch_supported(patch[i]) || stride[i] < 1 || stride[i] > patch[i] || max_width[i] < 1 ||
            (i > 0 && max_width[i] <= max_width[i - 1])) {
            set_err(h->err, "bad tuning entry %d", i); return BDIS_E_INVALID_ARG;
        }
    }
    h->ntune = n;
    for (int i = 0; i < n; i++) { h->tune_w[i] = max_width[i]; h->tune_p[i] = patch[i]; h->tune_s[i] = stride[i]; }
    return BDIS_OK;
}

bdis_status bdis_debug_stage(bdis_t *h, int32_t stage, int32_t level, void *dst, size_t bytes) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!h->have_last) { set_err(h->err, "no single-pair compute to inspect"); return BDIS_E_STATE; }
    const PairIn &p = h->last;
    if (!dst || level < 0 || level >= (stage == 8 ? p.g.Lp : p.g.L)) {
        set_err(h->err, "bad level or dst");
        return BDIS_E_INVALID_ARG;
    }
    const size_t esz = esize(h->prm);
    size_t px = (size_t)p.g.W[level] * p.g.H[level] * esz, np = (size_t)p.g.nx[level] * p.g.ny[level];
    const void *src = nullptr;
    size_t need = 0;
    switch (stage) {
    case 0: src = p.ws.pyr_l[level]; need = px; break;
    case 1: src = p.ws.pyr_r[level]; need = px; break;
    case 2: src = p.ws.rec_u[level]; need = np * esz; break;
    case 3: src = p.ws.rec_w[level]; need = np * esz; break;
    case 4: src = p.ws.rec_st[level]; need = np; break;
    case 5: src = p.ws.U[level]; need = px; break;
    case 6: src = p.ws.rec_u0[level]; need = np * esz; break;
    case 7:
        if (level == h->prm.learned_fine_levels) src = p.ws.keep;
        need = (size_t)p.g.W[level] * p.g.H[level];
        break;
    case 8:
        if (learned(h) && level == kNetLevel && p.group >= 0 && p.group < (int)h->groups.size())
            src = h->groups[p.group].out + (size_t)p.gindex * p.g.W[kNetLevel] * p.g.H[kNetLevel] * 2;
        need = (size_t)p.g.W[kNetLevel] * p.g.H[kNetLevel] * 2 * sizeof(float);
        break;
    default: set_err(h->err, "unknown stage %d", stage); return BDIS_E_INVALID_ARG;
    }
    if (!src) { set_err(h->err, "stage %d has no level %d", stage, level); return BDIS_E_INVALID_ARG; }
    if (bytes < need) { set_err(h->err, "dst holds %zu bytes, need %zu", bytes, need); return BDIS_E_INVALID_ARG; }
    DeviceGuard dg(h->device);
    if (stage == 5 && level == 1 && h->field1_skipped) {
        // the last compute never wrote this field: densify level 1 now from
        // its records and the level-2 field, which are still in place
        std::vector<Launch> ls;
        std::vector<DenseJob> jobs{make_dense_job(h, p, 1, false)};
        append(ls, K_DENSE, 1, 0, false, h->prm.precision == 0, jobs, make_kparams(h->prm, h->prm.patch),
               [](const DenseJob &j) { return dense_job_blocks(j); });
        const bool prof = h->profiling;
        h->profiling = false;
        bdis_status st = launch_all(h, ls, h->last_stream);
        h->profiling = prof;
        if (st != BDIS_OK) return st;
        HIPCHK(h, hipGetLastError());
        h->field1_skipped = false;
    }
    HIPCHK(h, hipStreamSynchronize(h->last_stream));
    HIPCHK(h, hipMemcpy(dst, src, need, hipMemcpyDeviceToHost));
    return BDIS_OK;
}

bdis_status bdis_set_profiling(bdis_t *h, int32_t on) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    DeviceGuard dg(h->device);
    if (on) {
        HIPCHK(h, hipDeviceSynchronize());
        for (auto &r : h->pending) { h->spare.push_back(r.a); h->spare.push_back(r.b); }
        h->pending.clear();
        h->prof_names.clear();
        h->prof_count.clear();
        h->prof_ms.clear();
    }
    h->profiling = on != 0;
    return BDIS_OK;
}

bdis_status bdis_get_profile(bdis_t *h, bdis_kernel_time *out, int32_t cap, int32_t *count) {
    if (!h) { set_err(g_thread_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!count || cap < 0 || (cap > 0 && !out)) { set_err(h->err, "bad output arguments"); return BDIS_E_INVALID_ARG; }
    DeviceGuard dg(h->device);
    for (auto &r : h->pending) {
        HIPCHK(h, hipEventSynchronize(r.b));
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, r.a, r.b));
        size_t i = 0;
        while (i < h->prof_names.size() && h->prof_names[i] != r.name) i++;
        if (i == h->prof_names.size()) {
            h->prof_names.push_back(r.name);
            h->prof_count.push_back(0);
            h->prof_ms.push_back(0.0);
        }
        h->prof_count[i]++;
        h->prof_ms[i] += ms;
        h->spare.push_back(r.a);
        h->spare.push_back(r.b);
    }
    h->pending.clear();
    *count = (int32_t)h->prof_names.size();
    for (int32_t i = 0; i < cap && i < *count; i++) {
        memset(&out[i], 0, sizeof out[i]);
        snprintf(out[i].name, sizeof out[i].name, "%s", h->prof_names[i].c_str());
        out[i].launches = h->prof_count[i];
        out[i].total_ms = h->prof_ms[i];
    }
    return BDIS_OK;
}

void bdis_destroy(bdis_t *h) {
    if (!h) return;
    {
        DeviceGuard dg(h->device);
        (void)hipDeviceSynchronize();
        if (h->ws) (void)hipFree(h->ws);
        if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
        if (h->graph) (void)hipGraphDestroy(h->graph);
        if (h->lv_exec) (void)hipGraphExecDestroy(h->lv_exec);
        if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
        if (h->side) (void)hipStreamDestroy(h->side);
        for (int g = 0; g < kMaxLanes - 1; g++) {
            if (h->lanes[g]) (void)hipStreamDestroy(h->lanes[g]);
            if (h->lane_join[g]) (void)hipEventDestroy(h->lane_join[g]);
        }
        if (h->lane_fork) (void)hipEventDestroy(h->lane_fork);
        if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
        if (h->ev_join) (void)hipEventDestroy(h->ev_join);
        if (h->p_dev) (void)hipFree(h->p_dev);
        if (h->p_host) (void)hipHostFree(h->p_host);
        if (h->p_upload_ev) (void)hipEventDestroy(h->p_upload_ev);
        if (h->gtab_d) (void)hipFree(h->gtab_d);
        if (h->gtab_f) (void)hipFree(h->gtab_f);
        for (auto &r : h->pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : h->spare) (void)hipEventDestroy(e);
    }
    if (h->owned_net) bdisnet_destroy(h->owned_net);
    delete h;
}

bdis_status bdis_rectify(const bdis_rectify_job *jobs, int32_t n, void *stream) {
    if (!jobs || n < 1 || n > kMaxRectifyJobs) {
        set_err(g_thread_err, "need 1 <= n <= %d rectify jobs", kMaxRectifyJobs);
        return BDIS_E_INVALID_ARG;
    }
    RectifyPack pk;
    memset(&pk, 0, sizeof pk);
    pk.n = n;
    long long blocks = 0;
    for (int i = 0; i < n; i++) {
        const bdis_rectify_job &J = jobs[i];
        if (!J.src || !J.dst) { set_err(g_thread_err, "job %d: NULL image pointer", i); return BDIS_E_INVALID_ARG; }
        if (J.src_width < 1 || J.src_height < 1 || J.dst_width < 1 || J.dst_height < 1 || J.src_width > 65536 ||
            J.src_height > 65536 || J.dst_width > 65536 || J.dst_height > 65536) {
            set_err(g_thread_err, "job %d: image sizes must be in [1, 65536]", i);
            return BDIS_E_INVALID_ARG;
        }
        if (J.src_pitch < J.src_width || J.dst_pitch < J.dst_width) {
            set_err(g_thread_err, "job %d: pitch smaller than width", i);
            return BDIS_E_INVALID_ARG;
        }
        if (!camera_ok(J.cam)) {
            set_err(g_thread_err, "job %d: calibration must be finite with non-zero focal lengths", i);
            return BDIS_E_INVALID_ARG;
        }
        pk.j[i] = J;
        pk.blocks[i] = (int)blocks;
        const long long threads = (long long)((J.dst_width + kRectPx - 1) / kRectPx) * J.dst_height;
        blocks += (threads + bdis::kBlock - 1) / bdis::kBlock;
    }
    pk.blocks[n] = (int)blocks;
    hipLaunchKernelGGL(k_rectify, dim3((unsigned)blocks), dim3(bdis::kBlock), 0, (hipStream_t)stream, pk);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_err(g_thread_err, "k_rectify launch failed: %s", hipGetErrorString(e)); return BDIS_E_HIP; }
    return BDIS_OK;
}

bdis_status bdis_depth_from_disparity(const float *disp, int32_t width, int32_t height, int32_t disp_pitch_elems,
                                      double focal_px, double baseline, float min_disparity, float *depth,
                                      int32_t depth_pitch_elems, void *stream) {
    if (!disp || !depth) { set_err(g_thread_err, "NULL disparity or depth pointer"); return BDIS_E_INVALID_ARG; }
    if (width < 1 || height < 1 || width > 65536 || height > 65536 || (long long)width * height > (1ll << 31) - 1) {
        set_err(g_thread_err, "sizes must be in [1, 65536] with fewer than 2^31 pixels");
        return BDIS_E_INVALID_ARG;
    }
    if (disp_pitch_elems < width || depth_pitch_elems < width) { set_err(g_thread_err, "pitch smaller than width"); return BDIS_E_INVALID_ARG; }
    if (!std::isfinite(focal_px) || !std::isfinite(baseline) || !std::isfinite(min_disparity) || focal_px <= 0.0 ||
        baseline <= 0.0 || min_disparity < 0.f) {
        set_err(g_thread_err, "focal length and baseline must be finite and positive, min_disparity finite and >= 0");
        return BDIS_E_INVALID_ARG;
    }
    const long long n = (long long)width * height;
    hipLaunchKernelGGL(k_depth, dim3((unsigned)((n + bdis::kBlock - 1) / bdis::kBlock)), dim3(bdis::kBlock), 0,
                       (hipStream_t)stream, disp, width, height, disp_pitch_elems, focal_px * baseline,
                       min_disparity, depth, depth_pitch_elems);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_err(g_thread_err, "k_depth launch failed: %s", hipGetErrorString(e)); return BDIS_E_HIP; }
    return BDIS_OK;
}

const char *bdis_status_string(bdis_status s) {
    switch (s) {
    case BDIS_OK: return "ok";
    case BDIS_E_INVALID_ARG: return "invalid argument";
    case BDIS_E_NO_DEVICE: return "no usable gfx950 device";
    case BDIS_E_OOM: return "out of device memory";
    case BDIS_E_HIP: return "HIP runtime error";
    case BDIS_E_UNSUPPORTED: return "unsupported request";
    case BDIS_E_STATE: return "call out of order";
    }
    return "unknown status";
}

const char *bdis_last_error(const bdis_t *h) { return h ? h->err : g_thread_err; }

}  // extern "C"
