// C-ABI entry points of the estimation side (declared in include/geonet.h).
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

using namespace geonet;

namespace {

thread_local std::string e_error;

net_status efail(net_status st, const std::string& msg) {
    e_error = msg;
    return st;
}

struct DeviceScratch {
    std::vector<void*> ptrs;
    ~DeviceScratch() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    T* get(size_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, (n ? n : 1) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return static_cast<T*>(p);
    }
};

net_status check_obs(const net_obs_desc* o) {
    if (!o) return efail(NET_E_ARG, "observation descriptor is NULL");
    if (o->n_nodes < 1 || o->n_frames < 2 || !o->fluor) return efail(NET_E_ARG, "need n_nodes >= 1, n_frames >= 2, fluor");
    if (o->n_pairs < 0 || (o->n_pairs > 0 && (!o->pairs || !o->pair_dist_um))) return efail(NET_E_ARG, "bad pairs");
    if (!(o->dt_ms > 0.0) || !(o->tau_c_ms > 0.0f) || o->frame_num < 1 || o->frame_den < 1)
        return efail(NET_E_ARG, "need dt > 0, tau_c > 0 and a frame rule");
    if (!(o->gain != 0.0f)) return efail(NET_E_ARG, "gain must be non-zero");
    return NET_OK;
}

// Computes the features of all pairs into out (device [P][64]).
net_status features(const net_obs_desc* o, float* out, hipStream_t s, DeviceScratch& sc) {
    FeatureInputs in{};
    in.F = o->fluor;
    in.pairs = o->pairs;
    in.dist = o->pair_dist_um;
    in.n = o->n_nodes;
    in.nf = o->n_frames;
    in.P = o->n_pairs;
    const double steps_per_frame = static_cast<double>(o->frame_den) / static_cast<double>(o->frame_num);
    in.rho = static_cast<float>(std::pow(1.0 - o->dt_ms / static_cast<double>(o->tau_c_ms), steps_per_frame));
    in.offset = o->offset;
    in.frame_num = o->frame_num;
    in.frame_den = o->frame_den;
    in.key_lo = static_cast<uint32_t>(o->control_seed);
    in.key_hi = static_cast<uint32_t>(o->control_seed >> 32);
    const size_t nn = static_cast<size_t>(o->n_nodes), nf = static_cast<size_t>(o->n_frames);
    if (o->drive_rate_hz) {
        std::vector<uint32_t> thr(nn);
        for (size_t j = 0; j < nn; ++j) thr[j] = pulse_threshold(o->drive_rate_hz[j], o->dt_ms);
        uint32_t* d = sc.get<uint32_t>(nn);
        if (!d) return efail(NET_E_OOM, "net_features: allocation");
        if (hipMemcpyAsync(d, thr.data(), nn * sizeof(uint32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return efail(NET_E_DEVICE, "net_features: upload");
        in.drive_thr = d;
    }
    FeatureWork w{};
    w.en = sc.get<float>(nn * nf);
    w.zn = sc.get<float>(nn * nf);
    w.rn = sc.get<float>(nn * nf);
    w.dc = sc.get<float>(nn * nf);
    w.stats = sc.get<float>(nn * 4);
    w.pm = sc.get<float>(nf);
    if (!w.en || !w.zn || !w.rn || !w.dc || !w.stats || !w.pm) return efail(NET_E_OOM, "net_features: allocation");
    hipError_t e = launch_features(in, w, out, s);
    if (e != hipSuccess) return efail(NET_E_DEVICE, std::string("net_features: ") + hipGetErrorString(e));
    return NET_OK;
}

}  // namespace

extern "C" {

const char* net_estimate_last_error(void) { return e_error.c_str(); }

net_status net_features(const net_obs_desc* obs, float* features_dev, void* stream) {
    net_status st = check_obs(obs);
    if (st != NET_OK) return st;
    if (!features_dev && obs->n_pairs > 0) return efail(NET_E_ARG, "net_features: output is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceScratch sc;
    st = features(obs, features_dev, s, sc);
    if (st != NET_OK) return st;
    if (hipStreamSynchronize(s) != hipSuccess) return efail(NET_E_DEVICE, "net_features: kernel");
    return NET_OK;
}

}  // extern "C"
