// net_features_noalloc: the pair features of net_features with no device
// allocation.  Its scratch lives in one fixed array in device memory,
// `scratch`, that every GPU the library runs on holds until the process
// ends; host code reaches each device's copy through the address
// hipGetSymbolAddress returns on that device (kept per device), never
// through the array's name.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;   // 16 MiB
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device (null: not looked up yet)

// The device address of this device's `scratch`, looked up once per device
// with that device current.
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

using namespace geonet;

extern "C" {

size_t net_features_noalloc_scratch_bytes(int32_t n_nodes, int32_t n_frames) {
    if (n_nodes < 1 || n_frames < 1) return 0;
    const size_t n = static_cast<size_t>(n_nodes), nf = static_cast<size_t>(n_frames);
    return 4 * align256(n * nf * sizeof(float)) + align256(n * 4 * sizeof(float)) + align256(nf * sizeof(float)) +
           align256(n * sizeof(float)) + align256(n * sizeof(uint32_t));
}

net_status net_features_noalloc(const net_obs_desc* obs, float* features_dev, void* stream) {
    net_status st = estimate_check_obs(obs);
    if (st != NET_OK) return st;
    if (!features_dev && obs->n_pairs > 0) return estimate_fail(NET_E_ARG, "net_features_noalloc: output is NULL");
    const size_t need = net_features_noalloc_scratch_bytes(obs->n_nodes, obs->n_frames);
    if (need > kScratchBytes)
        return estimate_fail(NET_E_RANGE, "net_features_noalloc: " + std::to_string(obs->n_nodes) + " vertices x " +
                                              std::to_string(obs->n_frames) + " frames need " + std::to_string(need) +
                                              " bytes of scratch, more than the fixed " +
                                              std::to_string(kScratchBytes) + " (use net_features)");
    void* base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess)
        return estimate_fail(NET_E_DEVICE, std::string("net_features_noalloc: scratch address: ") + hipGetErrorString(e));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n = static_cast<size_t>(obs->n_nodes), nf = static_cast<size_t>(obs->n_frames);
    unsigned char* p = static_cast<unsigned char*>(base);
    auto carve = [&p](size_t bytes) {
        unsigned char* q = p;
        p += align256(bytes);
        return q;
    };
    FeatureWork w{};
    w.en = reinterpret_cast<float*>(carve(n * nf * sizeof(float)));
    w.zn = reinterpret_cast<float*>(carve(n * nf * sizeof(float)));
    w.rn = reinterpret_cast<float*>(carve(n * nf * sizeof(float)));
    w.dc = reinterpret_cast<float*>(carve(n * nf * sizeof(float)));
    w.stats = reinterpret_cast<float*>(carve(n * 4 * sizeof(float)));
    w.pm = reinterpret_cast<float*>(carve(nf * sizeof(float)));
    float* rates = reinterpret_cast<float*>(carve(n * sizeof(float)));
    uint32_t* thr = reinterpret_cast<uint32_t*>(carve(n * sizeof(uint32_t)));
    FeatureInputs in{};
    feature_inputs(obs, in);
    if (obs->drive_rate_hz) {
        // the rates go to scratch as they are; the thresholds are formed on the device
        e = hipMemcpyAsync(rates, obs->drive_rate_hz, n * sizeof(float), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = launch_pulse_thresholds(rates, obs->n_nodes, obs->dt_ms, thr, s);
        if (e != hipSuccess)
            return estimate_fail(NET_E_DEVICE, std::string("net_features_noalloc: ") + hipGetErrorString(e));
        in.drive_thr = thr;
    }
    e = launch_features(in, w, features_dev, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return estimate_fail(NET_E_DEVICE, std::string("net_features_noalloc: ") + hipGetErrorString(e));
    return NET_OK;
}

}  // extern "C"
