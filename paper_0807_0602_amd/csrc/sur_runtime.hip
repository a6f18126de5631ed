// Host runtime of the surrogate network (scf_sur_* in include/scf.h): workspace plan, passes
// over explicit batches, graph-captured training steps on random minibatches, inference with
// the training-hull test.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "scf.h"
#include "sur_internal.h"

namespace scf {
// shared with the LBM runtime (scf_runtime.hip)
int set_error(int code, const std::string& msg);
}  // namespace scf

namespace {

using scf::set_error;

#define SUR_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return set_error(SCF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t al(size_t v) { return (v + 255) / 256 * 256; }

// ---------------------------------------------------------------------------------------------
// Scratch of the allocation-free prediction (scf_sur_predict_noalloc): the normalised inputs and
// two layers of activations of one call, carved as in noalloc_bytes.  A device array: each GPU
// the library runs on holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in); it uses the per-device
// address that scratch_address fetches with hipGetSymbolAddress, once per device, at
// scf_sur_create with that device current.
// ---------------------------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)20 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kMaxDevices] = {};

hipError_t scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_at[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_at[dev] = p;
    }
    *out = g_scratch_at[dev];
    return hipSuccess;
}

// Scratch bytes of a prediction over `rows` (a multiple of 64) rows: normalised inputs, then
// two (FP32 pre-activation, BF16 activation, BF16 transposed activation) layer slots.
size_t noalloc_bytes(int64_t rows, int d_in, int width) {
    const size_t r = (size_t)rows, w = (size_t)width;
    return al(4 * r * d_in) + 2 * (al(4 * r * w) + 2 * al(2 * r * w));
}

struct Plan {
    size_t total = 0;
    size_t theta, grad, m1, m2, wb, wbt, mean, stdv, lo, hi, Xd, Td, wd, Xs, Ts, wsb, Xn, Tb, wbb,
        Z, H, HT, dZ, dZb, dZbT, Y, dY, rowloss, loss, step, inhull, lr;
    int64_t P = 0;
    std::vector<int64_t> woff, boff;   // per layer, in floats
};

bool cfg_ok(const scf_sur_cfg* c, std::string* why) {
    if (!c) { *why = "cfg is NULL"; return false; }
    if (c->d_in < 1 || c->d_in > scf::sur::kMaxIn) { *why = "d_in must be in [1, 32]"; return false; }
    if (c->width < 64 || c->width % 64) { *why = "width must be a positive multiple of 64"; return false; }
    if (c->depth < 1 || c->depth > 16) { *why = "depth must be in [1, 16]"; return false; }
    if (c->max_batch < 64 || c->max_batch % 64) { *why = "max_batch must be a positive multiple of 64"; return false; }
    if (c->max_data < 1) { *why = "max_data must be >= 1"; return false; }
    if (!(c->lr > 0.0f) || !(c->beta1 >= 0.0f && c->beta1 < 1.0f) || !(c->beta2 >= 0.0f && c->beta2 < 1.0f) ||
        !(c->eps > 0.0f)) {
        *why = "bad Adam hyper-parameters";
        return false;
    }
    return true;
}

Plan plan(const scf_sur_cfg& c) {
    Plan p;
    const int W = c.width, D = c.depth, B = c.max_batch, din = c.d_in;
    // parameters: layer 0 (W x din), hidden layers 1..D-1 (W x W), output (2 x W)
    int64_t off = 0;
    for (int l = 0; l <= D; ++l) {
        const int o = l == D ? 2 : W, i = l == 0 ? din : W;
        p.woff.push_back(off);
        off += (int64_t)o * i;
        p.boff.push_back(off);
        off += o;
    }
    p.P = off;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = al(o + bytes); return r; };
    p.theta = take(4 * p.P);
    p.grad = take(4 * p.P);
    p.m1 = take(4 * p.P);
    p.m2 = take(4 * p.P);
    p.wb = take(2 * (size_t)W * W * std::max(1, D - 1));
    p.wbt = take(2 * (size_t)W * W * std::max(1, D - 1));
    p.mean = take(4 * din);
    p.stdv = take(4 * din);
    p.lo = take(4 * din);
    p.hi = take(4 * din);
    p.Xd = take(4 * (size_t)c.max_data * din);
    p.Td = take(8 * (size_t)c.max_data);
    p.wd = take(4 * (size_t)c.max_data);
    p.Xs = take(4 * (size_t)B * din);
    p.Ts = take(8 * (size_t)B);
    p.wsb = take(4 * (size_t)B);
    p.Xn = take(4 * (size_t)B * din);
    p.Tb = take(8 * (size_t)B);
    p.wbb = take(4 * (size_t)B);
    p.Z = take(4 * (size_t)B * W * D);
    p.H = take(2 * (size_t)B * W * D);
    p.HT = take(2 * (size_t)B * W * D);
    p.dZ = take(4 * (size_t)B * W);
    p.dZb = take(2 * (size_t)B * W * 2);
    p.dZbT = take(2 * (size_t)B * W * 2);
    p.Y = take(8 * (size_t)B);
    p.dY = take(8 * (size_t)B);
    p.rowloss = take(4 * (size_t)B);
    p.loss = take(4);
    p.step = take(8);
    p.inhull = take((size_t)B);
    p.lr = take(4);
    p.total = o;
    return p;
}

}  // namespace

struct scf_sur {
    scf_sur_cfg cfg;
    Plan p;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    int64_t n_data = 0;
    bool have_stats = false;
    hipGraphExec_t train_graph = nullptr;
    int train_rows = 0;
    void* scratch_dev = nullptr;     // this device's address of `scratch` (NULL: see scratch_err)
    std::string scratch_err;

    template <class T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    float* theta() const { return at<float>(p.theta); }
    float* grad() const { return at<float>(p.grad); }
    float* W(int l) const { return theta() + p.woff[l]; }
    float* b(int l) const { return theta() + p.boff[l]; }
    float* gW(int l) const { return grad() + p.woff[l]; }
    float* gb(int l) const { return grad() + p.boff[l]; }
    __bf16* Wb(int l) const { return at<__bf16>(p.wb) + (size_t)(l - 1) * cfg.width * cfg.width; }
    __bf16* WbT(int l) const { return at<__bf16>(p.wbt) + (size_t)(l - 1) * cfg.width * cfg.width; }
    float* Z(int l) const { return at<float>(p.Z) + (size_t)l * cfg.max_batch * cfg.width; }
    __bf16* H(int l) const { return at<__bf16>(p.H) + (size_t)l * cfg.max_batch * cfg.width; }
    __bf16* HT(int l) const { return at<__bf16>(p.HT) + (size_t)l * cfg.max_batch * cfg.width; }
    __bf16* dZb(int q) const { return at<__bf16>(p.dZb) + (size_t)q * cfg.max_batch * cfg.width; }
    __bf16* dZbT(int q) const { return at<__bf16>(p.dZbT) + (size_t)q * cfg.max_batch * cfg.width; }
    int64_t* step() const { return at<int64_t>(p.step); }

    ~scf_sur() {
        if (train_graph) (void)hipGraphExecDestroy(train_graph);
        if (cap) (void)hipStreamDestroy(cap);
    }

    hipError_t shadows(hipStream_t s) const {
        for (int l = 1; l < cfg.depth; ++l) {
            hipError_t e = scf::sur::shadow(W(l), cfg.width, cfg.width, Wb(l), WbT(l), s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }

    // Forward pass over `rows` normalised rows in Xn; with targets also the backward pass into
    // grad and the mean loss.  Layer 0 and the output layer in FP32, the others on MFMA.
    hipError_t pass(int rows, bool train, float inv_n, hipStream_t s) const {
        const int Wd = cfg.width, D = cfg.depth;
        const float* Xn = at<float>(p.Xn);
        hipError_t e = scf::sur::first_forward(Xn, cfg.d_in, W(0), b(0), Wd, rows, Z(0), H(0), HT(0), s);
        for (int l = 1; l < D && e == hipSuccess; ++l)
            e = scf::sur::gemm_forward(H(l - 1), Wb(l), b(l), rows, Wd, Z(l), H(l), HT(l), s);
        if (e != hipSuccess) return e;
        int q = 0;
        e = scf::sur::output_layer(Z(D - 1), Wd, rows, W(D), b(D), train ? at<float>(p.Tb) : nullptr,
                                   at<float>(p.wbb), inv_n, at<float>(p.Y), at<float>(p.dY),
                                   at<float>(p.rowloss), at<float>(p.dZ), dZb(q), dZbT(q), s);
        if (e != hipSuccess || !train) return e;
        e = scf::sur::output_grad(Z(D - 1), Wd, rows, at<float>(p.dY), gW(D), gb(D), s);
        for (int l = D - 1; l >= 1 && e == hipSuccess; --l) {
            e = scf::sur::colsum(at<float>(p.dZ), Wd, rows, gb(l), s);
            if (e == hipSuccess) e = scf::sur::gemm_weight_grad(dZbT(q), HT(l - 1), rows, Wd, gW(l), s);
            if (e == hipSuccess)
                e = scf::sur::gemm_backward(dZb(q), WbT(l), Z(l - 1), rows, Wd, at<float>(p.dZ), dZb(q ^ 1),
                                            dZbT(q ^ 1), s);
            q ^= 1;
        }
        if (e == hipSuccess) e = scf::sur::first_grad(at<float>(p.dZ), Xn, cfg.d_in, Wd, rows, gW(0), gb(0), s);
        if (e == hipSuccess) e = scf::sur::loss_sum(at<float>(p.rowloss), rows, inv_n, at<float>(p.loss), s);
        return e;
    }

    hipError_t adam_and_shadows(hipStream_t s) const {
        hipError_t e = scf::sur::adam(theta(), grad(), at<float>(p.m1), at<float>(p.m2), p.P, step(),
                                      at<float>(p.lr), cfg.beta1, cfg.beta2, cfg.eps, s);
        return e == hipSuccess ? shadows(s) : e;
    }

    // Copy an explicit batch (host, n rows) into the staging area, padded to a multiple of 64
    // rows with zero-weight rows, and normalise it.
    int stage(const float* X, const float* T, const float* w, int n, int* rows_out) {
        const int rows = (n + 63) / 64 * 64;
        if (n < 1 || rows > cfg.max_batch) return set_error(SCF_EINVAL, "batch must have 1..max_batch rows");
        std::vector<float> x((size_t)rows * cfg.d_in, 0.0f), t((size_t)rows * 2, 0.0f), ww(rows, 0.0f);
        std::memcpy(x.data(), X, sizeof(float) * (size_t)n * cfg.d_in);
        if (T) std::memcpy(t.data(), T, sizeof(float) * (size_t)n * 2);
        if (w) std::memcpy(ww.data(), w, sizeof(float) * n);
        else std::fill(ww.begin(), ww.begin() + n, 1.0f);
        SUR_TRY(hipMemcpyAsync(at<float>(p.Xs), x.data(), sizeof(float) * x.size(), hipMemcpyHostToDevice, stream));
        SUR_TRY(hipMemcpyAsync(at<float>(p.Ts), t.data(), sizeof(float) * t.size(), hipMemcpyHostToDevice, stream));
        SUR_TRY(hipMemcpyAsync(at<float>(p.wsb), ww.data(), sizeof(float) * ww.size(), hipMemcpyHostToDevice, stream));
        SUR_TRY(scf::sur::gather(at<float>(p.Xs), at<float>(p.Ts), at<float>(p.wsb), rows, cfg.d_in, rows,
                                 at<float>(p.mean), at<float>(p.stdv), at<float>(p.Xn), at<float>(p.Tb),
                                 at<float>(p.wbb), 0, 0, step(), stream));
        SUR_TRY(hipStreamSynchronize(stream));   // the host vectors go out of scope
        *rows_out = rows;
        return SCF_OK;
    }
};

extern "C" {

size_t scf_sur_workspace_bytes(const scf_sur_cfg* cfg) {
    std::string why;
    if (!cfg_ok(cfg, &why)) return 0;
    return plan(*cfg).total;
}

int scf_sur_create(scf_sur** out, const scf_sur_cfg* cfg, void* dev_ws, size_t ws_bytes, void* hip_stream) {
    if (!out) return set_error(SCF_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!cfg_ok(cfg, &why)) return set_error(SCF_EINVAL, why);
    if (!dev_ws || reinterpret_cast<uintptr_t>(dev_ws) % 256) return set_error(SCF_EINVAL, "workspace NULL or not 256-byte aligned");
    Plan p = plan(*cfg);
    if (ws_bytes < p.total) return set_error(SCF_EINVAL, "workspace too small: need " + std::to_string(p.total) + " bytes");
    scf_sur* s = new (std::nothrow) scf_sur();
    if (!s) return set_error(SCF_ENOMEM, "out of host memory");
    s->cfg = *cfg;
    s->p = p;
    s->ws = static_cast<char*>(dev_ws);
    s->stream = static_cast<hipStream_t>(hip_stream);
    hipStream_t st = s->stream;
    auto fail = [&](const char* what, hipError_t e) {
        delete s;
        return set_error(SCF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t e = hipMemsetAsync(s->ws, 0, p.total, st);
    if (e != hipSuccess) return fail("hipMemsetAsync", e);
    // identity normalisation until data are loaded
    std::vector<float> ones(cfg->d_in, 1.0f);
    e = hipMemcpyAsync(s->at<float>(p.stdv), ones.data(), sizeof(float) * cfg->d_in, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail("hipMemcpyAsync", e);
    e = hipMemcpyAsync(s->at<float>(p.lr), &cfg->lr, sizeof(float), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail("hipMemcpyAsync", e);
    e = hipStreamSynchronize(st);   // the host sources above go out of scope
    if (e != hipSuccess) return fail("hipStreamSynchronize", e);
    for (int l = 0; l <= cfg->depth && e == hipSuccess; ++l) {
        const int o = l == cfg->depth ? 2 : cfg->width, i = l == 0 ? cfg->d_in : cfg->width;
        e = scf::sur::init_params(s->theta(), p.woff[l], o, i, cfg->seed * 1000003ull + (uint64_t)l, st);
    }
    if (e == hipSuccess) e = s->shadows(st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail("surrogate initialisation", e);
    // address of the allocation-free prediction's scratch on the current device (the one that
    // holds the workspace); a failure only disables scf_sur_predict_noalloc
    int dev = -1;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        s->scratch_err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    } else if (dev < 0 || dev >= kMaxDevices) {
        s->scratch_err = "device index " + std::to_string(dev) + " beyond the scratch table";
    } else {
        e = scratch_address(dev, &s->scratch_dev);
        if (e != hipSuccess) {
            s->scratch_dev = nullptr;
            s->scratch_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        }
    }
    *out = s;
    return SCF_OK;
}

int64_t scf_sur_param_count(const scf_sur* s) { return s ? s->p.P : -1; }

int scf_sur_get_params(scf_sur* s, float* out) {
    if (!s || !out) return set_error(SCF_EINVAL, "NULL argument");
    SUR_TRY(hipMemcpyAsync(out, s->theta(), sizeof(float) * s->p.P, hipMemcpyDeviceToHost, s->stream));
    SUR_TRY(hipStreamSynchronize(s->stream));
    return SCF_OK;
}

int scf_sur_set_params(scf_sur* s, const float* in) {
    if (!s || !in) return set_error(SCF_EINVAL, "NULL argument");
    SUR_TRY(hipMemcpyAsync(s->theta(), in, sizeof(float) * s->p.P, hipMemcpyHostToDevice, s->stream));
    SUR_TRY(s->shadows(s->stream));
    SUR_TRY(hipStreamSynchronize(s->stream));
    return SCF_OK;
}

int scf_sur_set_lr(scf_sur* s, float lr) {
    if (!s) return set_error(SCF_EINVAL, "NULL argument");
    if (!(lr > 0.0f)) return set_error(SCF_EINVAL, "lr must be > 0");
    SUR_TRY(hipMemcpyAsync(s->at<float>(s->p.lr), &lr, sizeof(float), hipMemcpyHostToDevice, s->stream));
    SUR_TRY(hipStreamSynchronize(s->stream));
    return SCF_OK;
}

int scf_sur_reset_optimizer(scf_sur* s) {
    if (!s) return set_error(SCF_EINVAL, "NULL argument");
    SUR_TRY(hipMemsetAsync(s->at<float>(s->p.m1), 0, sizeof(float) * s->p.P, s->stream));
    SUR_TRY(hipMemsetAsync(s->at<float>(s->p.m2), 0, sizeof(float) * s->p.P, s->stream));
    SUR_TRY(hipMemsetAsync(s->step(), 0, sizeof(int64_t), s->stream));
    SUR_TRY(hipStreamSynchronize(s->stream));
    return SCF_OK;
}

int scf_sur_set_data(scf_sur* s, const float* X, const float* T, const float* w, int64_t n) {
    if (!s || !X || !T) return set_error(SCF_EINVAL, "NULL argument");
    if (n < 1 || n > s->cfg.max_data) return set_error(SCF_EINVAL, "n must be in [1, max_data]");
    const int din = s->cfg.d_in;
    SUR_TRY(hipMemcpyAsync(s->at<float>(s->p.Xd), X, sizeof(float) * n * din, hipMemcpyHostToDevice, s->stream));
    SUR_TRY(hipMemcpyAsync(s->at<float>(s->p.Td), T, sizeof(float) * n * 2, hipMemcpyHostToDevice, s->stream));
    if (w) {
        SUR_TRY(hipMemcpyAsync(s->at<float>(s->p.wd), w, sizeof(float) * n, hipMemcpyHostToDevice, s->stream));
    } else {
        std::vector<float> ones((size_t)n, 1.0f);
        SUR_TRY(hipMemcpyAsync(s->at<float>(s->p.wd), ones.data(), sizeof(float) * n, hipMemcpyHostToDevice, s->stream));
        SUR_TRY(hipStreamSynchronize(s->stream));
    }
    SUR_TRY(scf::sur::stats(s->at<float>(s->p.Xd), din, n, s->at<float>(s->p.mean), s->at<float>(s->p.stdv),
                            s->at<float>(s->p.lo), s->at<float>(s->p.hi), s->stream));
    SUR_TRY(hipStreamSynchronize(s->stream));
    s->n_data = n;
    s->have_stats = true;
    if (s->train_graph) {
        (void)hipGraphExecDestroy(s->train_graph);
        s->train_graph = nullptr;
    }
    return SCF_OK;
}

int scf_sur_get_norm(scf_sur* s, float* mean, float* stdv, float* lo, float* hi) {
    if (!s) return set_error(SCF_EINVAL, "NULL argument");
    const size_t nb = sizeof(float) * s->cfg.d_in;
    if (mean) SUR_TRY(hipMemcpyAsync(mean, s->at<float>(s->p.mean), nb, hipMemcpyDeviceToHost, s->stream));
    if (stdv) SUR_TRY(hipMemcpyAsync(stdv, s->at<float>(s->p.stdv), nb, hipMemcpyDeviceToHost, s->stream));
    if (lo) SUR_TRY(hipMemcpyAsync(lo, s->at<float>(s->p.lo), nb, hipMemcpyDeviceToHost, s->stream));
    if (hi) SUR_TRY(hipMemcpyAsync(hi, s->at<float>(s->p.hi), nb, hipMemcpyDeviceToHost, s->stream));
    SUR_TRY(hipStreamSynchronize(s->stream));
    return SCF_OK;
}

int scf_sur_set_norm(scf_sur* s, const float* mean, const float* stdv, const float* lo, const float* hi) {
    if (!s || !mean || !stdv || !lo || !hi) return set_error(SCF_EINVAL, "NULL argument");
    for (int k = 0; k < s->cfg.d_in; ++k)
        if (!(stdv[k] > 0.0f)) return set_error(SCF_EINVAL, "stdv must be > 0");
    const size_t nb = sizeof(float) * s->cfg.d_in;
    SUR_TRY(hipMemcpyAsync(s->at<float>(s->p.mean), mean, nb, hipMemcpyHostToDevice, s->stream));
    SUR_TRY(hipMemcpyAsync(s->at<float>(s->p.stdv), stdv, nb, hipMemcpyHostToDevice, s->stream));
    SUR_TRY(hipMemcpyAsync(s->at<float>(s->p.lo), lo, nb, hipMemcpyHostToDevice, s->stream));
    SUR_TRY(hipMemcpyAsync(s->at<float>(s->p.hi), hi, nb, hipMemcpyHostToDevice, s->stream));
    SUR_TRY(hipStreamSynchronize(s->stream));
    s->have_stats = true;
    return SCF_OK;
}

int scf_sur_grad(scf_sur* s, const float* X, const float* T, const float* w, int32_t n, float* loss, float* grad) {
    if (!s || !X || !T) return set_error(SCF_EINVAL, "NULL argument");
    int rows = 0;
    int rc = s->stage(X, T, w, n, &rows);
    if (rc) return rc;
    SUR_TRY(s->pass(rows, true, 1.0f / (float)n, s->stream));
    if (loss) SUR_TRY(hipMemcpyAsync(loss, s->at<float>(s->p.loss), sizeof(float), hipMemcpyDeviceToHost, s->stream));
    if (grad) SUR_TRY(hipMemcpyAsync(grad, s->grad(), sizeof(float) * s->p.P, hipMemcpyDeviceToHost, s->stream));
    SUR_TRY(hipStreamSynchronize(s->stream));
    return SCF_OK;
}

int scf_sur_step(scf_sur* s, const float* X, const float* T, const float* w, int32_t n, float* loss) {
    if (!s || !X || !T) return set_error(SCF_EINVAL, "NULL argument");
    int rows = 0;
    int rc = s->stage(X, T, w, n, &rows);
    if (rc) return rc;
    SUR_TRY(s->pass(rows, true, 1.0f / (float)n, s->stream));
    SUR_TRY(s->adam_and_shadows(s->stream));
    if (loss) SUR_TRY(hipMemcpyAsync(loss, s->at<float>(s->p.loss), sizeof(float), hipMemcpyDeviceToHost, s->stream));
    SUR_TRY(hipStreamSynchronize(s->stream));
    return SCF_OK;
}

int scf_sur_train(scf_sur* s, int64_t steps, int32_t batch, float* last_loss) {
    if (!s) return set_error(SCF_EINVAL, "NULL argument");
    if (s->n_data < 1) return set_error(SCF_ESTATE, "no training data (scf_sur_set_data)");
    if (batch < 64 || batch % 64 || batch > s->cfg.max_batch) return set_error(SCF_EINVAL, "batch must be a multiple of 64 up to max_batch");
    if (steps < 0) return set_error(SCF_EINVAL, "negative step count");
    if (!s->train_graph || s->train_rows != batch) {
        if (s->train_graph) {
            (void)hipGraphExecDestroy(s->train_graph);
            s->train_graph = nullptr;
        }
        if (!s->cap) SUR_TRY(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        SUR_TRY(hipStreamBeginCapture(s->cap, hipStreamCaptureModeRelaxed));
        hipError_t e = scf::sur::gather(s->at<float>(s->p.Xd), s->at<float>(s->p.Td), s->at<float>(s->p.wd),
                                        s->n_data, s->cfg.d_in, batch, s->at<float>(s->p.mean),
                                        s->at<float>(s->p.stdv), s->at<float>(s->p.Xn), s->at<float>(s->p.Tb),
                                        s->at<float>(s->p.wbb), 1, s->cfg.seed, s->step(), s->cap);
        if (e == hipSuccess) e = s->pass(batch, true, 1.0f / (float)batch, s->cap);
        if (e == hipSuccess) e = s->adam_and_shadows(s->cap);
        hipError_t end = hipStreamEndCapture(s->cap, &g);
        if (e != hipSuccess || end != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return set_error(SCF_EDEVICE, std::string("capture of the training step: ") +
                                              hipGetErrorString(e != hipSuccess ? e : end));
        }
        hipError_t inst = hipGraphInstantiate(&s->train_graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (inst != hipSuccess) return set_error(SCF_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(inst));
        s->train_rows = batch;
    }
    for (int64_t i = 0; i < steps; ++i) SUR_TRY(hipGraphLaunch(s->train_graph, s->stream));
    if (last_loss) SUR_TRY(hipMemcpyAsync(last_loss, s->at<float>(s->p.loss), sizeof(float), hipMemcpyDeviceToHost, s->stream));
    SUR_TRY(hipStreamSynchronize(s->stream));
    return SCF_OK;
}

int scf_sur_predict(scf_sur* s, const float* X, int64_t n, float* Y, uint8_t* in_hull) {
    if (!s || !X || !Y) return set_error(SCF_EINVAL, "NULL argument");
    if (n < 0) return set_error(SCF_EINVAL, "negative row count");
    const int din = s->cfg.d_in;
    for (int64_t r0 = 0; r0 < n; r0 += s->cfg.max_batch) {
        const int m = (int)std::min<int64_t>(s->cfg.max_batch, n - r0);
        int rows = 0;
        int rc = s->stage(X + r0 * din, nullptr, nullptr, m, &rows);
        if (rc) return rc;
        SUR_TRY(s->pass(rows, false, 1.0f, s->stream));
        SUR_TRY(hipMemcpyAsync(Y + 2 * r0, s->at<float>(s->p.Y), sizeof(float) * 2 * m, hipMemcpyDeviceToHost, s->stream));
        if (in_hull) {
            SUR_TRY(scf::sur::hull(s->at<float>(s->p.Xs), din, m, s->at<float>(s->p.lo), s->at<float>(s->p.hi),
                                   s->at<uint8_t>(s->p.inhull), s->stream));
            SUR_TRY(hipMemcpyAsync(in_hull + r0, s->at<uint8_t>(s->p.inhull), (size_t)m, hipMemcpyDeviceToHost, s->stream));
        }
        SUR_TRY(hipStreamSynchronize(s->stream));
    }
    if (in_hull && !s->have_stats)
        for (int64_t i = 0; i < n; ++i) in_hull[i] = 0;
    return SCF_OK;
}

int scf_sur_predict_noalloc(scf_sur* s, const float* X, int64_t n, float* Y, uint8_t* in_hull) {
    if (!s) return set_error(SCF_EINVAL, "NULL network");
    if (n < 0) return set_error(SCF_EINVAL, "negative row count");
    if (n == 0) return SCF_OK;
    if (!X || !Y) return set_error(SCF_EINVAL, "NULL input or output");
    const int din = s->cfg.d_in, Wd = s->cfg.width, D = s->cfg.depth;
    const int64_t rows = (n + 63) / 64 * 64;
    if (rows > (1 << 30) || noalloc_bytes(rows, din, Wd) > kNoAllocScratchBytes)
        return set_error(SCF_EINVAL, std::to_string(n) + " rows need " +
                                         std::to_string(noalloc_bytes(std::min<int64_t>(rows, 1 << 30), din, Wd)) +
                                         " bytes of scratch; the allocation-free prediction has " +
                                         std::to_string(kNoAllocScratchBytes) + " (split the rows over calls)");
    if (!s->scratch_dev) return set_error(SCF_EDEVICE, "no scratch on this device: " + s->scratch_err);
    char* base = static_cast<char*>(s->scratch_dev);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base + off;
        off = al(off + bytes);
        return p;
    };
    float* Xn = reinterpret_cast<float*>(take(4 * (size_t)rows * din));
    float* Z[2];
    __bf16* H[2];
    __bf16* HT[2];
    for (int q = 0; q < 2; ++q) {
        Z[q] = reinterpret_cast<float*>(take(4 * (size_t)rows * Wd));
        H[q] = reinterpret_cast<__bf16*>(take(2 * (size_t)rows * Wd));
        HT[q] = reinterpret_cast<__bf16*>(take(2 * (size_t)rows * Wd));
    }
    hipStream_t st = s->stream;
    // the same layer kernels as scf_sur_predict, activations alternating between two slots
    SUR_TRY(scf::sur::normalise(X, n, din, (int)rows, s->at<float>(s->p.mean), s->at<float>(s->p.stdv), Xn, st));
    SUR_TRY(scf::sur::first_forward(Xn, din, s->W(0), s->b(0), Wd, (int)rows, Z[0], H[0], HT[0], st));
    for (int l = 1; l < D; ++l)
        SUR_TRY(scf::sur::gemm_forward(H[(l - 1) & 1], s->Wb(l), s->b(l), (int)rows, Wd, Z[l & 1], H[l & 1],
                                       HT[l & 1], st));
    // output rows m < n straight into the caller's Y (inference: no targets)
    SUR_TRY(scf::sur::output_layer(Z[(D - 1) & 1], Wd, (int)n, s->W(D), s->b(D), nullptr, nullptr, 1.0f, Y,
                                   nullptr, nullptr, nullptr, nullptr, nullptr, st));
    if (in_hull) {
        if (s->have_stats)
            SUR_TRY(scf::sur::hull(X, din, (int)n, s->at<float>(s->p.lo), s->at<float>(s->p.hi), in_hull, st));
        else
            SUR_TRY(scf::sur::fill_u8(in_hull, n, 0, st));
    }
    return SCF_OK;
}

void scf_sur_destroy(scf_sur* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    delete s;
}

}  // extern "C"
