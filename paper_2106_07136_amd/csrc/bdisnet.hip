// bdisnet.hip -- host side of the learned proposal network: parameters,
// Adam state, training buffers, launches and the bdisnet_* C ABI of
// include/bdis.h.  The network is an added serving pattern (not in the
// paper): it proposes the initial disparity of the fine BDIS levels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "bdis.h"
#include "bdisnet_fused.hpp"
#include "bdisnet_internal.hpp"
#include "bdisnet_kernels.hpp"

using namespace bdisnet;

namespace {

thread_local char g_net_err[512] = "";

void seterr(char *buf, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
}

constexpr int kLayers = 4;

}  // namespace

struct bdisnet_ctx {
    int device = 0;
    int C = 32;
    int CI[kLayers], CO[kLayers];
    long long w_off[kLayers], b_off[kLayers];
    long long nparam = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // device, nparam each
    uint16_t *ffrag[kLayers] = {}, *dfrag[kLayers] = {};
    uint16_t *f32frag[kLayers] = {};  // B fragments of the fused forward (16x16x32 MFMA)
    // training buffers for the last forward
    size_t cap_m = 0;
    uint16_t *act[kLayers] = {};  // act[0] = copy of the input, act[l] = input of layer l
    float *out = nullptr;         // last forward output (FP32, 2 channels)
    uint16_t *gz[kLayers] = {};   // gradient at each layer's pre-activation (bf16)
    float *part = nullptr;        // weight-gradient partials
    size_t part_cap = 0;
    float *scal = nullptr;        // device scalars: [0] 1/n, [1] loss, partial sums after
    int *cnt = nullptr;
    size_t red_cap = 0;
    Geo last{0, 0, 0, 0};
    bool have_fwd = false, have_gout = false;
    int step = 0;  // last Adam step taken (0: none since the weights were set)
    char err[512] = "";
};

namespace {

#define NCHK(h, call)                                                         \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            seterr((h)->err, "%s failed: %s", #call, hipGetErrorString(e_)); \
            return BDIS_E_HIP;                                                \
        }                                                                     \
    } while (0)

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) (void)hipSetDevice(d);
    }
    ~DevGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int cop(int co) { return 16 * ((co + 15) / 16); }

// ---------------------------------------------------------------- small kernels

// Weight fragments of one layer from the FP32 master weights [tap][ci][co].
__global__ void k_pack(const float *__restrict__ w, int CI, int CO, uint16_t *__restrict__ ff,
                       uint16_t *__restrict__ df) {
    const int COP = 16 * ((CO + 15) / 16);
    const int nf = 9 * CI * COP;  // both fragment arrays hold 9 * CI * COP values
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= nf) return;
    const int j = i & 3, lane = (i >> 2) & 63, rest = i >> 8;
    // forward: B[k = ci][n = co], KC = CI / 16 chunks, NT = COP / 16 tiles
    {
        const int KC = CI / 16, NT = COP / 16;
        const int nt = rest % NT, kc = (rest / NT) % KC, tap = rest / (NT * KC);
        const int ci = kc * 16 + (lane >> 4) * 4 + j, co = nt * 16 + (lane & 15);
        ff[i] = co < CO ? f2bf(w[((size_t)tap * CI + ci) * CO + co]) : (uint16_t)0;
    }
    // input gradient: B[k = co][n = ci], KC = COP / 16 chunks, NT = CI / 16 tiles
    {
        const int KC = COP / 16, NT = CI / 16;
        const int nt = rest % NT, kc = (rest / NT) % KC, tap = rest / (NT * KC);
        const int co = kc * 16 + (lane >> 4) * 4 + j, ci = nt * 16 + (lane & 15);
        df[i] = co < CO ? f2bf(w[((size_t)tap * CI + ci) * CO + co]) : (uint16_t)0;
    }
}

__global__ void k_copy16(const uint16_t *__restrict__ a, uint16_t *__restrict__ b, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// loss, pass 1: valid-pixel counts per block
__global__ __launch_bounds__(kBlock) void k_loss_count(const uint8_t *__restrict__ valid, int M, int *__restrict__ cnt) {
    __shared__ int s[kBlock];
    const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
    s[threadIdx.x] = (i < M && valid[i]) ? 1 : 0;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[blockIdx.x] = s[0];
}

// loss, pass 2 (one block): 1 / n
__global__ __launch_bounds__(kBlock) void k_loss_norm(const int *__restrict__ cnt, int nb, float *__restrict__ scal) {
    __shared__ int s[kBlock];
    int a = 0;
    for (int i = (int)threadIdx.x; i < nb; i += kBlock) a += cnt[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) scal[0] = 1.f / (float)(s[0] > 0 ? s[0] : 1);
}

// loss, pass 3: per pixel Huber(d - t) + wc * BCE(sigmoid(c), q), q = [|d - t| < tol]
// (no gradient through q); gradient / n into gz (bf16, COP = 16 channels),
// per-block loss sums into part.
__global__ __launch_bounds__(kBlock) void k_loss_grad(const float *__restrict__ out, const float *__restrict__ tgt,
                                                       const uint8_t *__restrict__ valid, int M,
                                                       const float *__restrict__ scal, float delta, float tol,
                                                       float wc, uint16_t *__restrict__ gz, float *__restrict__ part) {
    __shared__ float s[kBlock];
    const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
    float l = 0.f;
    if (i < M) {
        float gd = 0.f, gc = 0.f;
        if (valid[i]) {
            const float inv = scal[0];
            const float d = out[2 * (size_t)i], c = out[2 * (size_t)i + 1];
            const float e = d - tgt[i], a = fabsf(e);
            const float hub = a <= delta ? 0.5f * e * e : delta * (a - 0.5f * delta);
            gd = (a <= delta ? e : delta * (e > 0.f ? 1.f : (e < 0.f ? -1.f : 0.f))) * inv;
            const float q = a < tol ? 1.f : 0.f;
            const float bce = fmaxf(c, 0.f) - q * c + log1pf(expf(-fabsf(c)));
            gc = wc * (1.f / (1.f + expf(-c)) - q) * inv;
            l = (hub + wc * bce) * inv;
        }
        uint16_t *row = gz + (size_t)i * 16;
        row[0] = f2bf(gd);
        row[1] = f2bf(gc);
        for (int k = 2; k < 16; k++) row[k] = 0;
    }
    s[threadIdx.x] = l;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kBlock) void k_loss_sum(const float *__restrict__ part, int nb, float *__restrict__ loss) {
    __shared__ float s[kBlock];
    float a = 0.f;
    for (int i = (int)threadIdx.x; i < nb; i += kBlock) a += part[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = s[0];
}

// caller-supplied gradient of the output (FP32, 2 channels) -> bf16 padded
__global__ void k_gout(const float *__restrict__ g, int M, uint16_t *__restrict__ gz) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= M) return;
    uint16_t *row = gz + (size_t)i * 16;
    row[0] = f2bf(g[2 * (size_t)i]);
    row[1] = f2bf(g[2 * (size_t)i + 1]);
    for (int k = 2; k < 16; k++) row[k] = 0;
}

__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- helpers

size_t frag32_elems(int CI, int CO) { return (size_t)((9 * CI + 31) / 32) * ((CO + 15) / 16) * 64 * 8; }

bdis_status pack_all(bdisnet_t *h, hipStream_t s) {
    for (int l = 0; l < kLayers; l++) {
        const int nf = 9 * h->CI[l] * cop(h->CO[l]);
        hipLaunchKernelGGL(k_pack, dim3((nf + 255) / 256), dim3(256), 0, s, h->w + h->w_off[l], h->CI[l], h->CO[l],
                           h->ffrag[l], h->dfrag[l]);
        const int n32 = (int)frag32_elems(h->CI[l], h->CO[l]);
        hipLaunchKernelGGL(k_pack32, dim3((n32 + 255) / 256), dim3(256), 0, s, h->w + h->w_off[l], h->CI[l],
                           h->CO[l], h->f32frag[l]);
    }
    NCHK(h, hipGetLastError());
    return BDIS_OK;
}

bdis_status ensure_train(bdisnet_t *h, size_t M) {
    if (M <= h->cap_m) return BDIS_OK;
    NCHK(h, hipDeviceSynchronize());
    for (int l = 0; l < kLayers; l++) {
        if (h->act[l]) (void)hipFree(h->act[l]);
        if (h->gz[l]) (void)hipFree(h->gz[l]);
        h->act[l] = h->gz[l] = nullptr;
    }
    if (h->out) (void)hipFree(h->out);
    h->out = nullptr;
    size_t want = std::max(M, (size_t)4096);
    want = (want + 4095) / 4096 * 4096;
    for (int l = 0; l < kLayers; l++) {
        if (hipMalloc(&h->act[l], want * h->CI[l] * 2) != hipSuccess ||
            hipMalloc(&h->gz[l], want * cop(h->CO[l]) * 2) != hipSuccess) {
            (void)hipGetLastError();
            seterr(h->err, "training buffer allocation failed");
            return BDIS_E_OOM;
        }
    }
    if (hipMalloc(&h->out, want * 2 * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        seterr(h->err, "training buffer allocation failed");
        return BDIS_E_OOM;
    }
    h->cap_m = want;
    return BDIS_OK;
}

bdis_status ensure_red(bdisnet_t *h, size_t nb) {
    if (nb <= h->red_cap) return BDIS_OK;
    NCHK(h, hipDeviceSynchronize());
    if (h->scal) (void)hipFree(h->scal);
    if (h->cnt) (void)hipFree(h->cnt);
    size_t want = std::max(nb, (size_t)1024);
    if (hipMalloc(&h->scal, (want + 8) * sizeof(float)) != hipSuccess ||
        hipMalloc(&h->cnt, want * sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        seterr(h->err, "reduction buffer allocation failed");
        return BDIS_E_OOM;
    }
    h->red_cap = want;
    return BDIS_OK;
}

template <int CI, int CO, bool LAST>
void fwd_layer(const Geo &g, const uint16_t *x, const uint16_t *ff, const float *b, uint16_t *ybf, float *yf,
               hipStream_t s) {
    const int waves = (g.M + 15) / 16;
    hipLaunchKernelGGL((k_conv_fwd<CI, CO, LAST>), dim3((waves + 3) / 4), dim3(kBlock), 0, s, g, x, ff, b, ybf, yf);
}

template <int C>
void forward_t(bdisnet_t *h, const Geo &g, const uint16_t *x, uint16_t *const *acts, float *out, hipStream_t s) {
    fwd_layer<16, C, false>(g, x, h->ffrag[0], h->w + h->b_off[0], acts[1], nullptr, s);
    fwd_layer<C, C, false>(g, acts[1], h->ffrag[1], h->w + h->b_off[1], acts[2], nullptr, s);
    fwd_layer<C, C, false>(g, acts[2], h->ffrag[2], h->w + h->b_off[2], acts[3], nullptr, s);
    fwd_layer<C, 2, true>(g, acts[3], h->ffrag[3], h->w + h->b_off[3], nullptr, out, s);
}

template <int CI, int CO>
void dgrad_layer(const Geo &g, const uint16_t *gz, const uint16_t *df, const uint16_t *x, uint16_t *gzp, hipStream_t s) {
    const int waves = (g.M + 15) / 16;
    hipLaunchKernelGGL((k_conv_dgrad<CI, CO>), dim3((waves + 3) / 4), dim3(kBlock), 0, s, g, gz, df, x, gzp);
}

template <int CI, int CO>
void wgrad_layer(const Geo &g, const uint16_t *x, const uint16_t *gz, float *part, float *grad, hipStream_t s) {
    const int nchunk = (g.M + kWChunk - 1) / kWChunk;
    hipLaunchKernelGGL((k_conv_wgrad<CI, CO>), dim3(nchunk), dim3(kBlock), 0, s, g, x, gz, part);
    const int n = 9 * CI * CO + CO;
    hipLaunchKernelGGL((k_wgrad_reduce<CI, CO>), dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, part, nchunk, grad);
}

template <int C>
void backward_t(bdisnet_t *h, hipStream_t s) {
    const Geo &g = h->last;
    wgrad_layer<C, 2>(g, h->act[3], h->gz[3], h->part, h->g + h->w_off[3], s);
    dgrad_layer<C, 2>(g, h->gz[3], h->dfrag[3], h->act[3], h->gz[2], s);
    wgrad_layer<C, C>(g, h->act[2], h->gz[2], h->part, h->g + h->w_off[2], s);
    dgrad_layer<C, C>(g, h->gz[2], h->dfrag[2], h->act[2], h->gz[1], s);
    wgrad_layer<C, C>(g, h->act[1], h->gz[1], h->part, h->g + h->w_off[1], s);
    dgrad_layer<C, C>(g, h->gz[1], h->dfrag[1], h->act[1], h->gz[0], s);
    wgrad_layer<16, C>(g, h->act[0], h->gz[0], h->part, h->g + h->w_off[0], s);
}

bdis_status check_geo(bdisnet_t *h, int n, int hh, int ww) {
    if (n < 1 || hh < 1 || ww < 1 || (long long)n * hh * ww > (1LL << 28)) {
        seterr(h->err, "bad input geometry %d x %d x %d", n, hh, ww);
        return BDIS_E_INVALID_ARG;
    }
    return BDIS_OK;
}

}  // namespace

// ================================================================ internal

namespace bdisnet {

bdis_status forward_internal(bdisnet_t *h, const uint16_t *x, int n, int hh, int ww, float *out, uint16_t *const *acts,
                             hipStream_t s) {
    Geo g{n, hh, ww, n * hh * ww};
    if (h->C == 32) forward_t<32>(h, g, x, acts, out, s);
    else forward_t<48>(h, g, x, acts, out, s);
    return hipGetLastError() == hipSuccess ? BDIS_OK : BDIS_E_HIP;
}

size_t act_bytes(const bdisnet_t *h, size_t M) {  // bytes of hidden activations for M pixels
    return M * (size_t)h->C * 2;
}

template <typename T, int C>
void launch_fused(bdisnet_t *h, const FusedPack &pk, int blocks, hipStream_t s) {
    const size_t lds = (size_t)(fused_x_elems<C>() + fused_y_elems<C>()) * sizeof(uint16_t);
    hipLaunchKernelGGL((k_net_fused<T, C>), dim3(blocks), dim3(kBlock), lds, s, pk, h->f32frag[0], h->f32frag[1],
                       h->f32frag[2], h->f32frag[3], h->w + h->b_off[0], h->w + h->b_off[1], h->w + h->b_off[2],
                       h->w + h->b_off[3]);
}

bdis_status forward_fused(bdisnet_t *h, const FusedPack &pk, int blocks, bool f64, hipStream_t s) {
    if (blocks <= 0) return BDIS_OK;
    if (h->C == 32) {
        if (f64) launch_fused<double, 32>(h, pk, blocks, s);
        else launch_fused<float, 32>(h, pk, blocks, s);
    } else {
        if (f64) launch_fused<double, 48>(h, pk, blocks, s);
        else launch_fused<float, 48>(h, pk, blocks, s);
    }
    return hipGetLastError() == hipSuccess ? BDIS_OK : BDIS_E_HIP;
}

int channels(const bdisnet_t *h) { return h->C; }
int device_of(const bdisnet_t *h) { return h->device; }

}  // namespace bdisnet

// ================================================================ C ABI

extern "C" {

bdis_status bdisnet_create(int32_t channels, int device, bdisnet_t **out) {
    if (!out) { seterr(g_net_err, "out is NULL"); return BDIS_E_INVALID_ARG; }
    *out = nullptr;
    if (channels != 32 && channels != 48) { seterr(g_net_err, "channels must be 32 or 48"); return BDIS_E_INVALID_ARG; }
    int nd = 0;
    if (hipGetDeviceCount(&nd) != hipSuccess || nd <= 0 || device < 0 || device >= nd) {
        (void)hipGetLastError();
        seterr(g_net_err, "no HIP device %d", device);
        return BDIS_E_NO_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess || strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        seterr(g_net_err, "device %d is not gfx950", device);
        return BDIS_E_NO_DEVICE;
    }
    bdisnet_t *h = new (std::nothrow) bdisnet_t();
    if (!h) { seterr(g_net_err, "host allocation failed"); return BDIS_E_OOM; }
    h->device = device;
    h->C = channels;
    const int ci[kLayers] = {16, channels, channels, channels};
    const int co[kLayers] = {channels, channels, channels, 2};
    long long off = 0;
    for (int l = 0; l < kLayers; l++) {
        h->CI[l] = ci[l];
        h->CO[l] = co[l];
        h->w_off[l] = off;
        off += 9LL * ci[l] * co[l];
        h->b_off[l] = off;
        off += co[l];
    }
    h->nparam = off;
    DevGuard dg(device);
    bool ok = hipMalloc(&h->w, off * 4) == hipSuccess && hipMalloc(&h->m, off * 4) == hipSuccess &&
              hipMalloc(&h->v, off * 4) == hipSuccess && hipMalloc(&h->g, off * 4) == hipSuccess;
    for (int l = 0; ok && l < kLayers; l++) {
        size_t nf = 9ull * ci[l] * cop(co[l]);
        ok = hipMalloc(&h->ffrag[l], nf * 2) == hipSuccess && hipMalloc(&h->dfrag[l], nf * 2) == hipSuccess &&
             hipMalloc(&h->f32frag[l], frag32_elems(ci[l], co[l]) * 2) == hipSuccess;
    }
    if (ok) {
        // partials of the widest weight gradient for up to 4096 chunks
        size_t psz = 9ull * channels * channels + 48;
        h->part_cap = psz * 4096;
        ok = hipMalloc(&h->part, h->part_cap * 4) == hipSuccess;
    }
    if (!ok || hipMemset(h->w, 0, off * 4) != hipSuccess || hipMemset(h->m, 0, off * 4) != hipSuccess ||
        hipMemset(h->v, 0, off * 4) != hipSuccess || hipMemset(h->g, 0, off * 4) != hipSuccess) {
        (void)hipGetLastError();
        seterr(g_net_err, "device allocation failed");
        bdisnet_destroy(h);
        return BDIS_E_OOM;
    }
    if (pack_all(h, nullptr) != BDIS_OK || hipDeviceSynchronize() != hipSuccess) {
        seterr(g_net_err, "%s", h->err);
        bdisnet_destroy(h);
        return BDIS_E_HIP;
    }
    *out = h;
    return BDIS_OK;
}

void bdisnet_destroy(bdisnet_t *h) {
    if (!h) return;
    {
        DevGuard dg(h->device);
        (void)hipDeviceSynchronize();
        for (float *p : {h->w, h->m, h->v, h->g, h->out, h->part, h->scal})
            if (p) (void)hipFree(p);
        if (h->cnt) (void)hipFree(h->cnt);
        for (int l = 0; l < kLayers; l++) {
            for (uint16_t *p : {h->ffrag[l], h->dfrag[l], h->f32frag[l], h->act[l], h->gz[l]})
                if (p) (void)hipFree(p);
        }
    }
    delete h;
}

int64_t bdisnet_param_count(const bdisnet_t *h) { return h ? h->nparam : 0; }

bdis_status bdisnet_set_params(bdisnet_t *h, const float *host, int64_t n) {
    if (!h || !host || n != h->nparam) {
        seterr(h ? h->err : g_net_err, "need exactly %lld parameters", h ? h->nparam : 0LL);
        return BDIS_E_INVALID_ARG;
    }
    for (int64_t i = 0; i < n; i++)
        if (!std::isfinite(host[i])) { seterr(h->err, "parameter %lld is not finite", (long long)i); return BDIS_E_INVALID_ARG; }
    DevGuard dg(h->device);
    NCHK(h, hipDeviceSynchronize());
    NCHK(h, hipMemcpy(h->w, host, n * 4, hipMemcpyHostToDevice));
    NCHK(h, hipMemset(h->m, 0, n * 4));
    NCHK(h, hipMemset(h->v, 0, n * 4));
    h->step = 0;
    bdis_status st = pack_all(h, nullptr);
    if (st != BDIS_OK) return st;
    NCHK(h, hipDeviceSynchronize());
    return BDIS_OK;
}

// Checkpoint layout (little-endian): 8 magic bytes "BDISNET\0", uint32
// version 1, int32 channels, int64 parameter count n, int64 last Adam step,
// then the FP32 master weights, the first and the second Adam moments (n
// values each).
namespace {
constexpr char kMagic[8] = {'B', 'D', 'I', 'S', 'N', 'E', 'T', 0};
constexpr uint32_t kVersion = 1;
constexpr int64_t kHeader = 32;
}  // namespace

int64_t bdisnet_checkpoint_bytes(const bdisnet_t *h) { return h ? kHeader + 12 * (int64_t)h->nparam : 0; }

int32_t bdisnet_step(const bdisnet_t *h) { return h ? h->step : 0; }

bdis_status bdisnet_save(bdisnet_t *h, void *blob, int64_t bytes) {
    if (!h) { seterr(g_net_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    const int64_t need = bdisnet_checkpoint_bytes(h);
    if (!blob || bytes < need) { seterr(h->err, "checkpoint needs %lld bytes", (long long)need); return BDIS_E_INVALID_ARG; }
    char *b = static_cast<char *>(blob);
    const int32_t C = h->C;
    const int64_t n = h->nparam, step = h->step;
    memcpy(b, kMagic, 8);
    memcpy(b + 8, &kVersion, 4);
    memcpy(b + 12, &C, 4);
    memcpy(b + 16, &n, 8);
    memcpy(b + 24, &step, 8);
    DevGuard dg(h->device);
    NCHK(h, hipDeviceSynchronize());
    NCHK(h, hipMemcpy(b + kHeader, h->w, n * 4, hipMemcpyDeviceToHost));
    NCHK(h, hipMemcpy(b + kHeader + 4 * n, h->m, n * 4, hipMemcpyDeviceToHost));
    NCHK(h, hipMemcpy(b + kHeader + 8 * n, h->v, n * 4, hipMemcpyDeviceToHost));
    return BDIS_OK;
}

bdis_status bdisnet_load(bdisnet_t *h, const void *blob, int64_t bytes) {
    if (!h) { seterr(g_net_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    const char *b = static_cast<const char *>(blob);
    if (!b || bytes < kHeader) { seterr(h->err, "checkpoint too short"); return BDIS_E_INVALID_ARG; }
    uint32_t ver;
    int32_t C;
    int64_t n, step;
    memcpy(&ver, b + 8, 4);
    memcpy(&C, b + 12, 4);
    memcpy(&n, b + 16, 8);
    memcpy(&step, b + 24, 8);
    if (memcmp(b, kMagic, 8) != 0 || ver != kVersion) { seterr(h->err, "not a version-1 network checkpoint"); return BDIS_E_INVALID_ARG; }
    if (C != h->C || n != h->nparam) {
        seterr(h->err, "checkpoint of a %d-channel network (%lld parameters); this one has %d", C, (long long)n, h->C);
        return BDIS_E_INVALID_ARG;
    }
    if (bytes < kHeader + 12 * n || step < 0 || step > INT32_MAX) { seterr(h->err, "checkpoint truncated or corrupt"); return BDIS_E_INVALID_ARG; }
    for (int64_t i = 0; i < 3 * n; i++) {
        float x;
        memcpy(&x, b + kHeader + 4 * i, 4);
        if (!std::isfinite(x) || (i >= 2 * n && x < 0.f)) { seterr(h->err, "checkpoint value %lld is invalid", (long long)i); return BDIS_E_INVALID_ARG; }
    }
    DevGuard dg(h->device);
    NCHK(h, hipDeviceSynchronize());
    NCHK(h, hipMemcpy(h->w, b + kHeader, n * 4, hipMemcpyHostToDevice));
    NCHK(h, hipMemcpy(h->m, b + kHeader + 4 * n, n * 4, hipMemcpyHostToDevice));
    NCHK(h, hipMemcpy(h->v, b + kHeader + 8 * n, n * 4, hipMemcpyHostToDevice));
    h->step = (int)step;
    bdis_status st = pack_all(h, nullptr);
    if (st != BDIS_OK) return st;
    NCHK(h, hipDeviceSynchronize());
    return BDIS_OK;
}

bdis_status bdisnet_get_params(bdisnet_t *h, float *host, int64_t n) {
    if (!h || !host || n != h->nparam) { seterr(h ? h->err : g_net_err, "bad arguments"); return BDIS_E_INVALID_ARG; }
    DevGuard dg(h->device);
    NCHK(h, hipDeviceSynchronize());
    NCHK(h, hipMemcpy(host, h->w, n * 4, hipMemcpyDeviceToHost));
    return BDIS_OK;
}

bdis_status bdisnet_get_grads(bdisnet_t *h, float *host, int64_t n) {
    if (!h || !host || n != h->nparam) { seterr(h ? h->err : g_net_err, "bad arguments"); return BDIS_E_INVALID_ARG; }
    DevGuard dg(h->device);
    NCHK(h, hipDeviceSynchronize());
    NCHK(h, hipMemcpy(host, h->g, n * 4, hipMemcpyDeviceToHost));
    return BDIS_OK;
}

bdis_status bdisnet_forward(bdisnet_t *h, const uint16_t *x, int32_t n, int32_t hh, int32_t ww, float *out,
                            void *stream) {
    if (!h) { seterr(g_net_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!x || !out) { seterr(h->err, "NULL tensor"); return BDIS_E_INVALID_ARG; }
    bdis_status st = check_geo(h, n, hh, ww);
    if (st != BDIS_OK) return st;
    const size_t M = (size_t)n * hh * ww;
    DevGuard dg(h->device);
    st = ensure_train(h, M);
    if (st != BDIS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)((M * 16 + 255) / 256)), dim3(256), 0, s, x, h->act[0], M * 16);
    st = bdisnet::forward_internal(h, h->act[0], n, hh, ww, h->out, h->act, s);
    if (st != BDIS_OK) { seterr(h->err, "forward launch failed"); return st; }
    NCHK(h, hipMemcpyAsync(out, h->out, M * 2 * sizeof(float), hipMemcpyDeviceToDevice, s));
    h->last = Geo{n, hh, ww, (int)M};
    h->have_fwd = true;
    h->have_gout = false;
    return BDIS_OK;
}

bdis_status bdisnet_loss(bdisnet_t *h, const float *target, const uint8_t *valid, float delta, float conf_tol,
                         float conf_weight, float *loss, void *stream) {
    if (!h) { seterr(g_net_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!h->have_fwd) { seterr(h->err, "no forward to take the loss of"); return BDIS_E_STATE; }
    if (!target || !valid || !loss || !(delta > 0.f) || !(conf_tol > 0.f) || !(conf_weight >= 0.f)) {
        seterr(h->err, "bad loss arguments");
        return BDIS_E_INVALID_ARG;
    }
    const int M = h->last.M;
    const int nb = (M + kBlock - 1) / kBlock;
    DevGuard dg(h->device);
    bdis_status st = ensure_red(h, nb);
    if (st != BDIS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_loss_count, dim3(nb), dim3(kBlock), 0, s, valid, M, h->cnt);
    hipLaunchKernelGGL(k_loss_norm, dim3(1), dim3(kBlock), 0, s, h->cnt, nb, h->scal);
    hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(kBlock), 0, s, h->out, target, valid, M, h->scal, delta,
                       conf_tol, conf_weight, h->gz[3], h->scal + 8);
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(kBlock), 0, s, h->scal + 8, nb, loss);
    NCHK(h, hipGetLastError());
    h->have_gout = true;
    return BDIS_OK;
}

bdis_status bdisnet_set_output_grad(bdisnet_t *h, const float *gout, void *stream) {
    if (!h) { seterr(g_net_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!h->have_fwd) { seterr(h->err, "no forward"); return BDIS_E_STATE; }
    if (!gout) { seterr(h->err, "NULL gradient"); return BDIS_E_INVALID_ARG; }
    DevGuard dg(h->device);
    const int M = h->last.M;
    hipLaunchKernelGGL(k_gout, dim3((M + 255) / 256), dim3(256), 0, (hipStream_t)stream, gout, M, h->gz[3]);
    NCHK(h, hipGetLastError());
    h->have_gout = true;
    return BDIS_OK;
}

bdis_status bdisnet_backward(bdisnet_t *h, void *stream) {
    if (!h) { seterr(g_net_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!h->have_fwd || !h->have_gout) { seterr(h->err, "backward needs a forward and an output gradient"); return BDIS_E_STATE; }
    const int nchunk = (h->last.M + kWChunk - 1) / kWChunk;
    const size_t psz = 9ull * h->C * h->C + 48;
    if ((size_t)nchunk * psz > h->part_cap) { seterr(h->err, "batch too large for the gradient partials"); return BDIS_E_INVALID_ARG; }
    DevGuard dg(h->device);
    if (h->C == 32) backward_t<32>(h, (hipStream_t)stream);
    else backward_t<48>(h, (hipStream_t)stream);
    NCHK(h, hipGetLastError());
    return BDIS_OK;
}

bdis_status bdisnet_adam_step(bdisnet_t *h, float lr, float beta1, float beta2, float eps, int32_t step,
                              void *stream) {
    if (!h) { seterr(g_net_err, "handle is NULL"); return BDIS_E_INVALID_ARG; }
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) || step < 1) {
        seterr(h->err, "bad Adam arguments");
        return BDIS_E_INVALID_ARG;
    }
    DevGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((h->nparam + 255) / 256)), dim3(256), 0, s, h->w, h->m, h->v, h->g,
                       h->nparam, lr, beta1, beta2, eps, c1, c2);
    NCHK(h, hipGetLastError());
    h->step = step;
    return pack_all(h, s);
}

bdis_status bdisnet_debug_activation(bdisnet_t *h, int32_t layer, uint16_t *host, size_t elems) {
    if (!h || layer < 0 || layer >= kLayers || !host) { seterr(h ? h->err : g_net_err, "bad arguments"); return BDIS_E_INVALID_ARG; }
    if (!h->have_fwd) { seterr(h->err, "no forward"); return BDIS_E_STATE; }
    const size_t need = (size_t)h->last.M * h->CI[layer];
    if (elems < need) { seterr(h->err, "host buffer holds %zu values, need %zu", elems, need); return BDIS_E_INVALID_ARG; }
    DevGuard dg(h->device);
    NCHK(h, hipDeviceSynchronize());
    NCHK(h, hipMemcpy(host, h->act[layer], need * 2, hipMemcpyDeviceToHost));
    return BDIS_OK;
}

const char *bdisnet_last_error(const bdisnet_t *h) { return h ? h->err : g_net_err; }

}  // extern "C"
