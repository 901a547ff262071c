// C-ABI entry points of the edge-scoring MLP (declared in include/geonet.h).
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace geonet;

struct net_mlp {
    MlpDevice d;
    DevAllocator al;           // the allocator current at net_mlp_create
    int64_t adam_t = 0;
    bool broken = false;
    bool grad_clear = false;   // d.grad is all zero (Adam clears it after use)
    // training workspace of net_mlp_train_epoch: one permuted batch
    float* xs = nullptr;       // [xs_cap][64]
    float* ys = nullptr;       // [xs_cap]
    int64_t xs_cap = 0;
    // column statistics of net_mlp_fit_input_norm: FP64 partial sums
    double* stat_part = nullptr;
    int64_t stat_cap = 0;
};

namespace {

thread_local std::string m_error;

net_status mfail(net_status st, const std::string& msg) {
    m_error = msg;
    return st;
}

net_status mdev(net_mlp* m, hipError_t e, const char* where) {
    if (m) m->broken = true;
    return mfail(NET_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Allocation through the handle's allocator; hipSuccess or hipErrorOutOfMemory.
template <typename T>
hipError_t alloc(const net_mlp* m, T** p, size_t n, hipStream_t s = nullptr) {
    *p = static_cast<T*>(m->al.get((n ? n : 1) * sizeof(T), s));
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

template <typename T>
void drop(const net_mlp* m, T** p, hipStream_t s = nullptr) {
    m->al.put(*p, s);
    *p = nullptr;
}

void release(net_mlp* m) {
    MlpDevice& d = m->d;
    void* ps[] = {d.params, d.adam_m, d.adam_v, d.grad,     d.w1b,  d.w2b,      d.w2c,      d.w1t,      d.w2p,
                  d.H1bits, d.dH2,    d.Xbt,    d.H1t,      d.dH2t, d.dH1t,
                  d.logits, d.loss,   d.in_shift, d.in_scale, d.head_part, m->xs, m->ys,      m->stat_part};
    for (void* p : ps) m->al.put(p, nullptr);
    d = MlpDevice{};
    m->xs = m->ys = nullptr;
    m->stat_part = nullptr;
    m->xs_cap = m->stat_cap = 0;
}

// Grow the activation workspace to hold `rows` rows (waits for the stream).
net_status reserve(net_mlp* m, int64_t rows, hipStream_t s) {
    if (rows <= m->d.cap) return NET_OK;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return mdev(m, e, "net_mlp: workspace");
    m->d.cap = 0;
    const size_t rp = static_cast<size_t>(mlp_ldt(rows));
    uint16_t** bufs[] = {&m->d.dH2, &m->d.H1t, &m->d.dH2t, &m->d.dH1t};
    for (uint16_t** b : bufs) {
        drop(m, b, s);
        if (alloc(m, b, rp * kMlpH, s) != hipSuccess) return mfail(NET_E_OOM, "net_mlp: workspace");
    }
    uint16_t** ibufs[] = {&m->d.Xbt};
    for (uint16_t** b : ibufs) {
        drop(m, b, s);
        if (alloc(m, b, rp * kMlpIn, s) != hipSuccess) return mfail(NET_E_OOM, "net_mlp: workspace");
    }
    drop(m, &m->d.H1bits, s);
    if (alloc(m, &m->d.H1bits, rp * (kMlpH / 32), s) != hipSuccess) return mfail(NET_E_OOM, "net_mlp: workspace");
    drop(m, &m->d.logits, s);
    if (alloc(m, &m->d.logits, static_cast<size_t>(rows), s) != hipSuccess) return mfail(NET_E_OOM, "net_mlp: workspace");
    m->d.cap = rows;
    return NET_OK;
}

net_status check(const net_mlp* m, int64_t rows, const void* x) {
    if (!m) return mfail(NET_E_ARG, "net_mlp: handle is NULL");
    if (m->broken) return mfail(NET_E_STATE, "net_mlp: handle unusable after a device error");
    if (rows < 1 || rows > (int64_t(1) << 26)) return mfail(NET_E_ARG, "net_mlp: rows must be in 1 .. 2^26");
    if (!x) return mfail(NET_E_ARG, "net_mlp: features are NULL");
    return NET_OK;
}

}  // namespace

extern "C" {

const char* net_mlp_last_error(void) { return m_error.c_str(); }

net_status net_mlp_create(net_mlp_t** out) {
    if (!out) return mfail(NET_E_ARG, "net_mlp_create: out is NULL");
    *out = nullptr;
    net_mlp* m = new net_mlp();
    m->al = current_allocator();
    MlpDevice& d = m->d;
    if (alloc(m, &d.params, kMlpParams) != hipSuccess || alloc(m, &d.adam_m, kMlpParams) != hipSuccess ||
        alloc(m, &d.adam_v, kMlpParams) != hipSuccess || alloc(m, &d.grad, kMlpParams) != hipSuccess ||
        alloc(m, &d.w1b, kMlpW1) != hipSuccess || alloc(m, &d.w2b, kMlpW2) != hipSuccess ||
        alloc(m, &d.w1t, kMlpW1) != hipSuccess || alloc(m, &d.w2p, kMlpW2) != hipSuccess ||
        alloc(m, &d.w2c, kMlpW2) != hipSuccess ||
        alloc(m, &d.loss, 1) != hipSuccess || alloc(m, &d.head_part, kHeadReplicas * kHeadPart) != hipSuccess ||
        alloc(m, &d.in_shift, kMlpIn) != hipSuccess || alloc(m, &d.in_scale, kMlpIn) != hipSuccess) {
        release(m);
        delete m;
        return mfail(NET_E_OOM, "net_mlp_create: device allocation failed");
    }
    hipError_t e = hipMemset(d.params, 0, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMemset(d.head_part, 0, kHeadReplicas * kHeadPart * sizeof(float));
    if (e == hipSuccess) e = hipMemset(d.adam_m, 0, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMemset(d.adam_v, 0, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = mlp_refresh_bf16(d, nullptr);
    if (e == hipSuccess) {
        const std::vector<float> zero(kMlpIn, 0.0f), one(kMlpIn, 1.0f);
        e = hipMemcpy(d.in_shift, zero.data(), kMlpIn * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d.in_scale, one.data(), kMlpIn * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        release(m);
        delete m;
        return mfail(NET_E_DEVICE, std::string("net_mlp_create: ") + hipGetErrorString(e));
    }
    *out = m;
    return NET_OK;
}

net_status net_mlp_set_params(net_mlp_t* m, const float* host_params, int64_t n) {
    if (!m || !host_params) return mfail(NET_E_ARG, "net_mlp_set_params: NULL argument");
    if (n != kMlpParams) return mfail(NET_E_ARG, "net_mlp_set_params: expected 82689 parameters");
    if (m->broken) return mfail(NET_E_STATE, "net_mlp_set_params: handle unusable");
    hipError_t e = hipMemcpy(m->d.params, host_params, kMlpParams * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->d.adam_m, 0, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->d.adam_v, 0, kMlpParams * sizeof(float));
    if (e == hipSuccess) e = mlp_refresh_bf16(m->d, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return mdev(m, e, "net_mlp_set_params");
    m->adam_t = 0;
    return NET_OK;
}

net_status net_mlp_set_input_norm(net_mlp_t* m, const float* shift, const float* scale) {
    if (!m || !shift || !scale) return mfail(NET_E_ARG, "net_mlp_set_input_norm: NULL argument");
    if (m->broken) return mfail(NET_E_STATE, "net_mlp_set_input_norm: handle unusable");
    hipError_t e = hipMemcpy(m->d.in_shift, shift, kMlpIn * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d.in_scale, scale, kMlpIn * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return mdev(m, e, "net_mlp_set_input_norm");
    return NET_OK;
}

net_status net_mlp_get_params(const net_mlp_t* m, float* host_params, int64_t n) {
    if (!m || !host_params) return mfail(NET_E_ARG, "net_mlp_get_params: NULL argument");
    if (n != kMlpParams) return mfail(NET_E_ARG, "net_mlp_get_params: expected 82689 parameters");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(host_params, m->d.params, kMlpParams * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return mfail(NET_E_DEVICE, std::string("net_mlp_get_params: ") + hipGetErrorString(e));
    return NET_OK;
}

net_status net_mlp_forward(net_mlp_t* m, const float* x_dev, int64_t rows, float* logits_dev, void* stream) {
    net_status st = check(m, rows, x_dev);
    if (st != NET_OK) return st;
    if (!logits_dev) return mfail(NET_E_ARG, "net_mlp_forward: logits are NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // one fused kernel: no activation workspace
    hipError_t e = mlp_forward_fused(m->d, x_dev, rows, logits_dev, s);
    if (e != hipSuccess) return mdev(m, e, "net_mlp_forward");
    return NET_OK;
}

static net_status grad_impl(net_mlp* m, const float* x, const float* y, int64_t rows, float* loss_out,
                            hipStream_t s) {
    net_status st = check(m, rows, x);
    if (st != NET_OK) return st;
    if (!y) return mfail(NET_E_ARG, "net_mlp: labels are NULL");
    if ((st = reserve(m, rows, s)) != NET_OK) return st;
    hipError_t e = hipSuccess;
    if (!m->grad_clear) e = hipMemsetAsync(m->d.grad, 0, kMlpParams * sizeof(float), s);
    m->grad_clear = false;
    if (e == hipSuccess) e = mlp_forward(m->d, x, rows, y, s);
    if (e == hipSuccess) e = mlp_backward(m->d, rows, loss_out, s);
    if (e != hipSuccess) return mdev(m, e, "net_mlp: gradient");
    return NET_OK;
}

net_status net_mlp_grad(net_mlp_t* m, const float* x_dev, const float* y_dev, int64_t rows, float* grad_dev,
                        float* loss_dev, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    net_status st = grad_impl(m, x_dev, y_dev, rows, loss_dev, s);
    if (st != NET_OK) return st;
    hipError_t e = hipSuccess;
    if (grad_dev) e = hipMemcpyAsync(grad_dev, m->d.grad, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return mdev(m, e, "net_mlp_grad");
    return NET_OK;
}

net_status net_mlp_train_step(net_mlp_t* m, const float* x_dev, const float* y_dev, int64_t rows, float lr,
                              float* loss_dev, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!(lr > 0.0f)) return mfail(NET_E_ARG, "net_mlp_train_step: lr must be > 0");
    net_status st = grad_impl(m, x_dev, y_dev, rows, loss_dev, s);
    if (st != NET_OK) return st;
    m->adam_t += 1;
    hipError_t e = mlp_adam(m->d, lr, 0.9f, 0.999f, 1e-8f, m->adam_t, s);
    if (e != hipSuccess) return mdev(m, e, "net_mlp_train_step");
    m->grad_clear = true;
    return NET_OK;
}

net_status net_mlp_fit_input_norm(net_mlp_t* m, const float* x_dev, int64_t rows, void* stream) {
    if (!m || !x_dev) return mfail(NET_E_ARG, "net_mlp_fit_input_norm: NULL argument");
    if (m->broken) return mfail(NET_E_STATE, "net_mlp_fit_input_norm: handle unusable");
    if (rows < 1 || rows > (int64_t(1) << 31)) return mfail(NET_E_ARG, "net_mlp_fit_input_norm: rows must be in 1 .. 2^31");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!m->stat_part) {
        m->stat_cap = static_cast<int64_t>(kStatBlocks + 1) * kMlpIn;
        if (alloc(m, &m->stat_part, static_cast<size_t>(m->stat_cap), s) != hipSuccess) {
            m->stat_cap = 0;
            return mfail(NET_E_OOM, "net_mlp_fit_input_norm: workspace");
        }
    }
    hipError_t e = mlp_input_stats(x_dev, rows, m->stat_part, m->d.in_shift, m->d.in_scale, s);
    if (e != hipSuccess) return mdev(m, e, "net_mlp_fit_input_norm");
    return NET_OK;
}

net_status net_mlp_get_input_norm(const net_mlp_t* m, float* shift, float* scale) {
    if (!m || !shift || !scale) return mfail(NET_E_ARG, "net_mlp_get_input_norm: NULL argument");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(shift, m->d.in_shift, kMlpIn * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(scale, m->d.in_scale, kMlpIn * sizeof(float), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return mfail(NET_E_DEVICE, std::string("net_mlp_get_input_norm: ") + hipGetErrorString(e));
    return NET_OK;
}

net_status net_mlp_train_epoch(net_mlp_t* m, const float* x_dev, const float* y_dev, int64_t rows, int64_t batch,
                               float lr, uint64_t shuffle_seed, uint32_t epoch, float* loss_dev, void* stream) {
    if (!m || !x_dev || !y_dev) return mfail(NET_E_ARG, "net_mlp_train_epoch: NULL argument");
    if (m->broken) return mfail(NET_E_STATE, "net_mlp_train_epoch: handle unusable");
    if (rows < 1 || rows > (int64_t(1) << 31)) return mfail(NET_E_ARG, "net_mlp_train_epoch: rows must be in 1 .. 2^31");
    if (batch < 1 || batch > (int64_t(1) << 26)) return mfail(NET_E_ARG, "net_mlp_train_epoch: batch must be in 1 .. 2^26");
    if (!(lr > 0.0f)) return mfail(NET_E_ARG, "net_mlp_train_epoch: lr must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t b = std::min(batch, rows);
    if (b > m->xs_cap) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return mdev(m, e, "net_mlp_train_epoch: workspace");
        drop(m, &m->xs, s);
        drop(m, &m->ys, s);
        m->xs_cap = 0;
        if (alloc(m, &m->xs, static_cast<size_t>(b) * kMlpIn, s) != hipSuccess ||
            alloc(m, &m->ys, static_cast<size_t>(b), s) != hipSuccess)
            return mfail(NET_E_OOM, "net_mlp_train_epoch: workspace");
        m->xs_cap = b;
    }
    int64_t k = 0;
    for (int64_t a0 = 0; a0 < rows; a0 += b, ++k) {
        const int64_t count = std::min(b, rows - a0);
        hipError_t e = gather_shuffled(x_dev, y_dev, rows, shuffle_seed, epoch, a0, count, m->xs, m->ys, s);
        if (e != hipSuccess) return mdev(m, e, "net_mlp_train_epoch: gather");
        net_status st = net_mlp_train_step(m, m->xs, m->ys, count, lr, loss_dev ? loss_dev + k : nullptr, stream);
        if (st != NET_OK) return st;
    }
    return NET_OK;
}

net_status net_shuffle_indices(int64_t n, uint64_t seed, uint32_t epoch, int64_t* out_dev, void* stream) {
    if (n < 0 || n > (int64_t(1) << 31)) return mfail(NET_E_ARG, "net_shuffle_indices: n must be in 0 .. 2^31");
    if (n == 0) return NET_OK;
    if (!out_dev) return mfail(NET_E_ARG, "net_shuffle_indices: output is NULL");
    hipError_t e = shuffle_indices(n, seed, epoch, out_dev, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return mfail(NET_E_DEVICE, std::string("net_shuffle_indices: ") + hipGetErrorString(e));
    return NET_OK;
}

void net_mlp_free(net_mlp_t* m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    release(m);
    delete m;
}

}  // extern "C"
