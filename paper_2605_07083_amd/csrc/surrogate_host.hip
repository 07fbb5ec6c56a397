// surrogate_host.hip -- host side of the surrogate C ABI (include/surrogate.h):
// workspace layout, weight packing, and the launch sequence of the forward
// pass, the training step (loss, one backward kernel per layer for the input
// and weight gradients, Adam with re-quantisation) and the conversion to
// warm-start densities.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "../../include/surrogate.h"

extern "C" {
hipError_t surx_features(const float *params, __bf16 *feat, double *loss0, int X, int B, hipStream_t s);
hipError_t surx_conv_fwd(int layer, const __bf16 *in, const __bf16 *Wf, const float *bias, float *yf, __bf16 *yb,
                         int X, int B, hipStream_t s);
hipError_t surx_loss(const float *out, const float *target, __bf16 *dz, double *loss, int X, int B, hipStream_t s);
hipError_t surx_conv_bwd(int layer, const __bf16 *dz, const float *yin, const __bf16 *feat, const __bf16 *Wb,
                         __bf16 *dzprev, float *part, float *pbias, int X, int B, hipStream_t s);
int surx_wgrad_parts(int X, int B);
int surx_loss_slots(void);
hipError_t surx_reduce_adam(const float *part, const float *pbias, int P, float *wm, float *mw, float *vw, float *dw,
                            float *bias, float *mb, float *vb, float *db, __bf16 *Wf, __bf16 *Wb, int cin, int coutp,
                            int cout_real, int kp, int kpb, float lr, float b1, float b2, float eps, float c1,
                            float c2, hipStream_t s);
hipError_t surx_requant(const float *wm, __bf16 *Wf, __bf16 *Wb, int cin, int coutp, int cout_real, int kp, int kpb,
                        hipStream_t s);
hipError_t surx_to_state(const float *out, const float *params, const double *n0, double *state, int X, int B,
                         hipStream_t s);
hipError_t surx_init_weights(float *wm, int cin, int coutp, int cout_real, int kp, uint32_t layer, uint32_t seed,
                             hipStream_t s);
hipError_t surx_to_densities(const float *out, const double *n0, double *dens, int X, int B, hipStream_t s);
hipError_t surx_unpack(const float *y, float *out, int X, int B, hipStream_t s);
}

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define SUR_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(PIC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
constexpr int CIN[SUR_LAYERS] = {16, 64, 64, 64, 64, 64};
constexpr int COUT[SUR_LAYERS] = {64, 64, 64, 64, 64, SUR_OUT};
constexpr int COUTP[SUR_LAYERS] = {64, 64, 64, 64, 64, 48};
constexpr float B1 = 0.9f, B2 = 0.999f, EPS = 1e-8f;

int pad32(int k) { return (k + 31) / 32 * 32; }

struct Layer {
    int cin, cout, coutp, kp, kpb;
    float *wm, *mw, *vw, *dw;     // [coutp][kp] FP32 (kappa = t*cin + ci)
    float *bias, *mb, *vb, *db;   // [coutp]
    __bf16 *wf;                   // [coutp][kp]
    __bf16 *wb;                   // [cin][kpb] (t*coutp + co)
};

struct Bump {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t n)
    {
        off = (off + ALIGN - 1) / ALIGN * ALIGN;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

}  // namespace

struct sur_net {
    int X = 0, bmax = 0;
    int device = -1;              // the GPU current at sur_create
    char *scratch = nullptr;      // that GPU's copy of the allocation-free forward's scratch array
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t param_bytes = 0;       // weights, moments, grads: the first bytes of ws
    Layer L[SUR_LAYERS];
    __bf16 *feat = nullptr;       // [bmax][X][16]
    float *yf[SUR_LAYERS];        // [bmax][X][coutp]
    __bf16 *yb[SUR_LAYERS - 1];   // bf16 copies of the hidden outputs
    __bf16 *dz[2];                // output gradients of a layer [bmax][X][64], ping-pong
    float *part = nullptr;        // a layer's partial weight gradients [parts][64][320]
    float *pbias = nullptr;       // and bias gradients [parts][64]
    double *loss = nullptr;       // surx_loss_slots() partial sums of the training loss
    long long t = 0;              // Adam steps taken
};

namespace {

void layout(sur_net &n, Bump &bp)
{
    const size_t P = (size_t)n.bmax * n.X;
    for (int l = 0; l < SUR_LAYERS; ++l) {
        Layer &L = n.L[l];
        L.cin = CIN[l];
        L.cout = COUT[l];
        L.coutp = COUTP[l];
        L.kp = pad32(SUR_KS * L.cin);
        L.kpb = pad32(SUR_KS * L.coutp);
        const size_t nw = (size_t)L.coutp * L.kp;
        L.wm = bp.take<float>(nw);
        L.mw = bp.take<float>(nw);
        L.vw = bp.take<float>(nw);
        L.dw = bp.take<float>(nw);
        L.bias = bp.take<float>(L.coutp);
        L.mb = bp.take<float>(L.coutp);
        L.vb = bp.take<float>(L.coutp);
        L.db = bp.take<float>(L.coutp);
        L.wf = bp.take<__bf16>(nw);
        L.wb = bp.take<__bf16>((size_t)L.cin * L.kpb);
    }
    n.loss = bp.take<double>((size_t)surx_loss_slots());
    n.param_bytes = bp.off;
    n.feat = bp.take<__bf16>(P * SUR_IN);
    for (int l = 0; l < SUR_LAYERS; ++l) n.yf[l] = bp.take<float>(P * COUTP[l]);
    for (int l = 0; l < SUR_LAYERS - 1; ++l) n.yb[l] = bp.take<__bf16>(P * COUTP[l]);
    for (int k = 0; k < 2; ++k) n.dz[k] = bp.take<__bf16>(P * SUR_HIDDEN);
    const size_t parts = (size_t)surx_wgrad_parts(n.X, n.bmax);
    n.part = bp.take<float>(parts * SUR_HIDDEN * pad32(SUR_KS * SUR_HIDDEN));
    n.pbias = bp.take<float>(parts * SUR_HIDDEN);
}

int check_shape(int batch, int cells)
{
    if (cells <= 0 || cells % 64) return fail(PIC_EINVAL, "cells must be a positive multiple of 64");
    if (batch <= 0 || (long long)batch * cells > (1ll << 28)) return fail(PIC_EINVAL, "bad batch size");
    return PIC_OK;
}

int requant_all(sur_net *n)
{
    for (int l = 0; l < SUR_LAYERS; ++l) {
        const Layer &L = n->L[l];
        SUR_TRY(surx_requant(L.wm, L.wf, L.wb, L.cin, L.coutp, L.cout, L.kp, L.kpb, n->stream));
    }
    return PIC_OK;
}

// train: also clear the loss accumulators
int forward(sur_net *n, const float *params, int B, bool train)
{
    SUR_TRY(surx_features(params, n->feat, train ? n->loss : nullptr, n->X, B, n->stream));
    for (int l = 0; l < SUR_LAYERS; ++l) {
        const __bf16 *in = l == 0 ? n->feat : n->yb[l - 1];
        __bf16 *yb = l < SUR_LAYERS - 1 ? n->yb[l] : nullptr;
        SUR_TRY(surx_conv_fwd(l, in, n->L[l].wf, n->L[l].bias, n->yf[l], yb, n->X, B, n->stream));
    }
    return PIC_OK;
}

// packed W_l[co][ci][t] <-> master [coutp][t*cin + ci]
void pack(const sur_net *n, int l, const float *m, float *packed)
{
    const Layer &L = n->L[l];
    for (int co = 0; co < L.cout; ++co)
        for (int ci = 0; ci < L.cin; ++ci)
            for (int t = 0; t < SUR_KS; ++t)
                packed[((size_t)co * L.cin + ci) * SUR_KS + t] = m[(size_t)co * L.kp + t * L.cin + ci];
}

void unpack(const sur_net *n, int l, const float *packed, float *m)
{
    const Layer &L = n->L[l];
    std::memset(m, 0, sizeof(float) * L.coutp * L.kp);
    for (int co = 0; co < L.cout; ++co)
        for (int ci = 0; ci < L.cin; ++ci)
            for (int t = 0; t < SUR_KS; ++t)
                m[(size_t)co * L.kp + t * L.cin + ci] = packed[((size_t)co * L.cin + ci) * SUR_KS + t];
}

int copy_out(sur_net *n, bool grads, float *w, float *b)
{
    if (!n || !w || !b) return fail(PIC_EINVAL, "bad arguments");
    SUR_TRY(hipStreamSynchronize(n->stream));
    size_t wo = 0, bo = 0;
    for (int l = 0; l < SUR_LAYERS; ++l) {
        const Layer &L = n->L[l];
        std::vector<float> m((size_t)L.coutp * L.kp), bb(L.coutp);
        SUR_TRY(hipMemcpy(m.data(), grads ? L.dw : L.wm, m.size() * sizeof(float), hipMemcpyDeviceToHost));
        SUR_TRY(hipMemcpy(bb.data(), grads ? L.db : L.bias, bb.size() * sizeof(float), hipMemcpyDeviceToHost));
        pack(n, l, m.data(), w + wo);
        std::memcpy(b + bo, bb.data(), sizeof(float) * L.cout);
        wo += (size_t)L.cout * L.cin * SUR_KS;
        bo += L.cout;
    }
    return PIC_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free forward pass (sur_forward_noalloc): one
// file-scope device array, so that the call needs no device memory beyond
// the handle's weights and the caller's inputs and outputs.  Every GPU the
// library runs on holds its own copy until the process ends.  In host code
// the array's name is not a device address: its address on a GPU comes from
// hipGetSymbolAddress with that GPU current (scratch_on_current_device).
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = (size_t)12 << 20;
// per sample and cell: features (16 bf16), a hidden output in FP32 (64,
// overwritten layer after layer), the last layer's FP32 output (48 padded
// channels) and two bf16 ping-pong copies of the hidden activations (64 each)
constexpr size_t SCRATCH_PER_POSITION = 16 * 2 + 64 * 4 + 48 * 4 + 2 * 64 * 2;

}  // namespace

static __device__ __align__(256) char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[MAX_DEVICES] = {};

// The scratch array's address on the current GPU, looked up once per GPU.
int scratch_on_current_device(int *device, char **ptr)
{
    int dev = -1;
    SUR_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(PIC_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PIC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *device = dev;
    *ptr = g_scratch_ptr[dev];
    return PIC_OK;
}

}  // namespace

extern "C" {

int sur_workspace_size(int max_batch, int cells, size_t *bytes)
{
    if (!bytes) return fail(PIC_EINVAL, "null argument");
    int rc = check_shape(max_batch, cells);
    if (rc) return rc;
    sur_net n;
    n.X = cells;
    n.bmax = max_batch;
    Bump bp{nullptr};
    layout(n, bp);
    *bytes = (bp.off + ALIGN - 1) / ALIGN * ALIGN;
    return PIC_OK;
}

int sur_create(int max_batch, int cells, void *dev_workspace, size_t bytes, void *hip_stream, uint32_t seed,
               sur_net **out)
{
    if (!out || !dev_workspace) return fail(PIC_EINVAL, "bad arguments");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN) return fail(PIC_EINVAL, "workspace not 256-byte aligned");
    size_t need;
    int rc = sur_workspace_size(max_batch, cells, &need);
    if (rc) return rc;
    if (bytes < need) return fail(PIC_ENOSPACE, "workspace too small");
    sur_net *n = new (std::nothrow) sur_net;
    if (!n) return fail(PIC_ENOSPACE, "host allocation failed");
    n->X = cells;
    n->bmax = max_batch;
    n->ws = static_cast<char *>(dev_workspace);
    n->stream = static_cast<hipStream_t>(hip_stream);
    Bump bp{n->ws};
    layout(*n, bp);
    auto cleanup = [&](int code) { delete n; return code; };
    // the allocation-free forward's scratch on this GPU (set-up, once per GPU)
    if ((rc = scratch_on_current_device(&n->device, &n->scratch))) return cleanup(rc);
    if (hipMemsetAsync(n->ws, 0, n->param_bytes, n->stream) != hipSuccess)
        return cleanup(fail(PIC_EHIP, "hipMemsetAsync failed"));
    for (int l = 0; l < SUR_LAYERS; ++l) {
        const Layer &L = n->L[l];
        if (surx_init_weights(L.wm, L.cin, L.coutp, L.cout, L.kp, (uint32_t)l, seed, n->stream) != hipSuccess)
            return cleanup(fail(PIC_EHIP, "weight init launch failed"));
    }
    rc = requant_all(n);
    if (rc) return cleanup(rc);
    *out = n;
    return PIC_OK;
}

int sur_set_weights(sur_net *n, const float *w, const float *b)
{
    if (!n || !w || !b) return fail(PIC_EINVAL, "bad arguments");
    SUR_TRY(hipStreamSynchronize(n->stream));
    SUR_TRY(hipMemsetAsync(n->ws, 0, n->param_bytes, n->stream));
    size_t wo = 0, bo = 0;
    for (int l = 0; l < SUR_LAYERS; ++l) {
        const Layer &L = n->L[l];
        std::vector<float> m((size_t)L.coutp * L.kp), bb(L.coutp, 0.0f);
        unpack(n, l, w + wo, m.data());
        std::memcpy(bb.data(), b + bo, sizeof(float) * L.cout);
        SUR_TRY(hipMemcpyAsync(L.wm, m.data(), m.size() * sizeof(float), hipMemcpyHostToDevice, n->stream));
        SUR_TRY(hipMemcpyAsync(L.bias, bb.data(), bb.size() * sizeof(float), hipMemcpyHostToDevice, n->stream));
        SUR_TRY(hipStreamSynchronize(n->stream));   // the staging vectors die at the end of this iteration
        wo += (size_t)L.cout * L.cin * SUR_KS;
        bo += L.cout;
    }
    n->t = 0;
    int rc = requant_all(n);
    if (rc) return rc;
    SUR_TRY(hipStreamSynchronize(n->stream));
    return PIC_OK;
}

int sur_get_weights(sur_net *n, float *w, float *b) { return copy_out(n, false, w, b); }

int sur_get_grads(sur_net *n, float *w, float *b) { return copy_out(n, true, w, b); }

int sur_forward(sur_net *n, const float *dev_params, int batch, float *dev_out)
{
    if (!n || !dev_params || !dev_out) return fail(PIC_EINVAL, "bad arguments");
    if (batch < 1 || batch > n->bmax) return fail(PIC_EINVAL, "batch exceeds the workspace's max_batch");
    int rc = forward(n, dev_params, batch, false);
    if (rc) return rc;
    SUR_TRY(surx_unpack(n->yf[SUR_LAYERS - 1], dev_out, n->X, batch, n->stream));
    return PIC_OK;
}

int sur_forward_noalloc(sur_net *n, const float *dev_params, int batch, float *dev_out)
{
    if (!n || !dev_params || !dev_out) return fail(PIC_EINVAL, "bad arguments");
    if (batch < 1) return fail(PIC_EINVAL, "batch must be positive");
    const size_t per_sample = SCRATCH_PER_POSITION * (size_t)n->X;
    const int chunk = (int)std::min<size_t>(SCRATCH_BYTES / per_sample, (size_t)batch);
    if (chunk < 1)
        return fail(PIC_EINVAL, "cells beyond the scratch array: at most " +
                                    std::to_string(SCRATCH_BYTES / SCRATCH_PER_POSITION) + " per sample");
    int dev = -1;
    SUR_TRY(hipGetDevice(&dev));
    if (dev != n->device) return fail(PIC_EINVAL, "the handle's GPU is not the current device");
    char *base = n->scratch;     // the array's address on this GPU, never its host-side name
    const size_t P = (size_t)chunk * n->X;
    __bf16 *feat = reinterpret_cast<__bf16 *>(base);
    float *yf = reinterpret_cast<float *>(base + P * 16 * 2);
    float *yout = reinterpret_cast<float *>(base + P * (16 * 2 + 64 * 4));
    __bf16 *yb[2] = {reinterpret_cast<__bf16 *>(base + P * (16 * 2 + 64 * 4 + 48 * 4)),
                     reinterpret_cast<__bf16 *>(base + P * (16 * 2 + 64 * 4 + 48 * 4 + 64 * 2))};
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        const int nb = std::min(chunk, batch - b0);
        SUR_TRY(surx_features(dev_params + (size_t)4 * b0, feat, nullptr, n->X, nb, n->stream));
        for (int l = 0; l < SUR_LAYERS; ++l) {
            const __bf16 *in = l == 0 ? feat : yb[(l - 1) & 1];
            const bool last = l == SUR_LAYERS - 1;
            SUR_TRY(surx_conv_fwd(l, in, n->L[l].wf, n->L[l].bias, last ? yout : yf, last ? nullptr : yb[l & 1], n->X,
                                  nb, n->stream));
        }
        SUR_TRY(surx_unpack(yout, dev_out + (size_t)b0 * SUR_OUT * n->X, n->X, nb, n->stream));
    }
    return PIC_OK;
}

int sur_train_step(sur_net *n, const float *dev_params, const float *dev_target, int batch, float lr, double *loss)
{
    if (!n || !dev_params || !dev_target) return fail(PIC_EINVAL, "bad arguments");
    if (batch < 1 || batch > n->bmax) return fail(PIC_EINVAL, "batch exceeds the workspace's max_batch");
    if (!(lr > 0.0f)) return fail(PIC_EINVAL, "learning rate must be positive");
    const int X = n->X;
    // the forward pass zeroes the loss accumulators (features kernel)
    int rc = forward(n, dev_params, batch, true);
    if (rc) return rc;
    SUR_TRY(surx_loss(n->yf[SUR_LAYERS - 1], dev_target, n->dz[0], n->loss, X, batch, n->stream));
    n->t += 1;
    const float c1 = (float)(1.0 - std::pow((double)B1, (double)n->t));
    const float c2 = (float)(1.0 - std::pow((double)B2, (double)n->t));
    const int parts = surx_wgrad_parts(X, batch);
    // per layer, last to first: the input gradient (with this layer's weights
    // before their update) and the partial weight gradients in one kernel,
    // then the layer's gradient summed from the partials, its Adam update and
    // BF16 copies
    int cur = 0;
    for (int l = SUR_LAYERS - 1; l >= 0; --l) {
        const Layer &L = n->L[l];
        if (l > 0)
            SUR_TRY(surx_conv_bwd(l, n->dz[cur], n->yf[l - 1], nullptr, L.wb, n->dz[cur ^ 1], n->part, n->pbias, X,
                                  batch, n->stream));
        else
            SUR_TRY(surx_conv_bwd(0, n->dz[cur], nullptr, n->feat, nullptr, nullptr, n->part, n->pbias, X, batch,
                                  n->stream));
        cur ^= 1;
        SUR_TRY(surx_reduce_adam(n->part, n->pbias, parts, L.wm, L.mw, L.vw, L.dw, L.bias, L.mb, L.vb, L.db, L.wf,
                                 L.wb, L.cin, L.coutp, L.cout, L.kp, L.kpb, lr, B1, B2, EPS, c1, c2, n->stream));
    }
    if (loss) {
        std::vector<double> parts((size_t)surx_loss_slots());
        SUR_TRY(hipMemcpyAsync(parts.data(), n->loss, parts.size() * sizeof(double), hipMemcpyDeviceToHost,
                               n->stream));
        SUR_TRY(hipStreamSynchronize(n->stream));
        double sum = 0.0;
        for (double v : parts) sum += v;
        *loss = sum;
    }
    return PIC_OK;
}

int sur_densities(sur_net *n, const float *dev_params, const double *dev_n0, int batch, double *dev_dens)
{
    if (!n || !dev_params || !dev_n0 || !dev_dens) return fail(PIC_EINVAL, "bad arguments");
    if (batch < 1 || batch > n->bmax) return fail(PIC_EINVAL, "batch exceeds the workspace's max_batch");
    int rc = forward(n, dev_params, batch, false);
    if (rc) return rc;
    SUR_TRY(surx_to_densities(n->yf[SUR_LAYERS - 1], dev_n0, dev_dens, n->X, batch, n->stream));
    return PIC_OK;
}

int sur_state(sur_net *n, const float *dev_params, const double *dev_n0, int batch, double *dev_state)
{
    if (!n || !dev_params || !dev_n0 || !dev_state) return fail(PIC_EINVAL, "bad arguments");
    if (batch < 1 || batch > n->bmax) return fail(PIC_EINVAL, "batch exceeds the workspace's max_batch");
    int rc = forward(n, dev_params, batch, false);
    if (rc) return rc;
    SUR_TRY(surx_to_state(n->yf[SUR_LAYERS - 1], dev_params, dev_n0, dev_state, n->X, batch, n->stream));
    return PIC_OK;
}

const char *sur_last_error(void) { return g_err.c_str(); }

void sur_destroy(sur_net *n) { delete n; }

}  // extern "C"
