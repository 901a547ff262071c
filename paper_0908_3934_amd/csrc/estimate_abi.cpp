// C-ABI entry points of the estimation side (declared in include/geonet.h).
#include <algorithm>
#include <cmath>
#include <numeric>
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

// Scratch of one call, taken from the allocator installed by
// net_set_allocator (with PyTorch's caching allocator the blocks are reused
// from call to call) and handed back, ordered on the call's stream, when the
// call returns.
struct DeviceScratch {
    DevAllocator al = current_allocator();
    hipStream_t s;
    std::vector<void*> ptrs;
    explicit DeviceScratch(hipStream_t stream) : s(stream) {}
    ~DeviceScratch() {
        for (void* p : ptrs) al.put(p, s);
    }
    template <typename T>
    T* get(size_t n) {
        void* p = al.get((n ? n : 1) * sizeof(T), s);
        if (!p) return nullptr;
        ptrs.push_back(p);
        return static_cast<T*>(p);
    }
};

}  // namespace

namespace geonet {
net_status estimate_fail(net_status st, const std::string& msg) { return efail(st, msg); }
}  // namespace geonet

namespace {

net_status check_obs(const net_obs_desc* o) {
    if (!o) return efail(NET_E_ARG, "observation descriptor is NULL");
    if (o->n_nodes < 1 || o->n_frames < 2 || !o->fluor) return efail(NET_E_ARG, "need n_nodes >= 1, n_frames >= 2, fluor");
    if (o->n_pairs < 0 || (o->n_pairs > 0 && (!o->pairs || !o->pair_dist_um))) return efail(NET_E_ARG, "bad pairs");
    if (!(o->dt_ms > 0.0) || !(o->tau_c_ms > 0.0f) || o->frame_num < 1 || o->frame_den < 1)
        return efail(NET_E_ARG, "need dt > 0, tau_c > 0 and a frame rule");
    if (!(o->gain != 0.0f)) return efail(NET_E_ARG, "gain must be non-zero");
    return NET_OK;
}

}  // namespace

namespace geonet {

net_status estimate_check_obs(const net_obs_desc* o) { return check_obs(o); }

void feature_inputs(const net_obs_desc* o, FeatureInputs& in) {
    in = FeatureInputs{};
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
}

}  // namespace geonet

namespace {

// Computes the features of all pairs into out (device [P][64]).
net_status features(const net_obs_desc* o, float* out, hipStream_t s, DeviceScratch& sc) {
    FeatureInputs in{};
    feature_inputs(o, in);
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

template <typename T>
bool to_host(std::vector<T>& h, const T* d, size_t n, hipStream_t s) {
    h.resize(n);
    return n == 0 || (hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s) == hipSuccess &&
                      hipStreamSynchronize(s) == hipSuccess);
}

template <typename T>
bool to_dev(T* d, const std::vector<T>& h, hipStream_t s) {
    return h.empty() || (hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s) == hipSuccess &&
                         hipStreamSynchronize(s) == hipSuccess);
}

// Simulation-based fit; scores in the caller's pair order into out (device).
net_status simfit(const net_obs_desc* o, const net_simfit_opts* opts, float* out, hipStream_t s) {
    const int K = opts && opts->realisations ? opts->realisations : 8;
    const int sweeps = opts ? opts->sweeps : 2;
    const double init_frac = opts && opts->init_fraction > 0.0f ? opts->init_fraction : 0.3;
    const double min_gain = opts && opts->min_gain > 0.0f ? opts->min_gain : 1e-3;
    if (K < 1 || K > 64 || (64 % K) != 0) return efail(NET_E_ARG, "simfit: realisations must divide 64");
    if (sweeps < 0 || sweeps > 64) return efail(NET_E_ARG, "simfit: sweeps in 0..64");
    const int64_t P = o->n_pairs, n = o->n_nodes, nf = o->n_frames;
    DeviceScratch sc(s);
    // candidate pairs sorted by target (stable in source)
    std::vector<int32_t> hp;
    std::vector<float> hd;
    if (!to_host(hp, o->pairs, static_cast<size_t>(2 * P), s) || !to_host(hd, o->pair_dist_um, static_cast<size_t>(P), s))
        return efail(NET_E_DEVICE, "simfit: pair download");
    for (int64_t p = 0; p < P; ++p)
        if (hp[2 * p] < 0 || hp[2 * p] >= n || hp[2 * p + 1] < 0 || hp[2 * p + 1] >= n || hp[2 * p] == hp[2 * p + 1])
            return efail(NET_E_ARG, "simfit: pair index out of range or self pair");
    std::vector<int64_t> perm(P);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return hp[2 * a + 1] < hp[2 * b + 1]; });
    std::vector<int32_t> sp(2 * P);
    std::vector<float> sdist(P);
    std::vector<int64_t> row(n + 1, 0);
    for (int64_t q = 0; q < P; ++q) {
        sp[2 * q] = hp[2 * perm[q]];
        sp[2 * q + 1] = hp[2 * perm[q] + 1];
        sdist[q] = hd[perm[q]];
        row[sp[2 * q + 1] + 1]++;
    }
    for (int64_t j = 0; j < n; ++j) row[j + 1] += row[j];
    int32_t* dpairs = sc.get<int32_t>(2 * P);
    float* ddist = sc.get<float>(P);
    FitWork w{};
    const int64_t t_end = (nf * o->frame_den + o->frame_num - 1) / o->frame_num;
    w.words = static_cast<int32_t>((t_end + 31) / 32);
    w.e = sc.get<float>(n * nf);
    w.pulses = sc.get<uint32_t>(n * static_cast<int64_t>(w.words));
    w.base = sc.get<double>(n * nf);
    w.member = sc.get<uint8_t>(P);
    w.row = sc.get<int64_t>(n + 1);
    w.ll = sc.get<double>(P + n);
    float* feat = sc.get<float>(64 * P);
    if (!dpairs || !ddist || !w.e || !w.pulses || !w.base || !w.member || !w.row || !w.ll || !feat)
        return efail(NET_E_OOM, "simfit: allocation");
    if (!to_dev(dpairs, sp, s) || !to_dev(ddist, sdist, s) || !to_dev(w.row, row, s))
        return efail(NET_E_DEVICE, "simfit: upload");
    // initial graph: top init_frac of each target's candidates by the lag-0 plus
    // lag-1 correlation of activity (features 8 and 9)
    net_obs_desc os = *o;
    os.pairs = dpairs;
    os.pair_dist_um = ddist;
    net_status st = features(&os, feat, s, sc);
    if (st != NET_OK) return st;
    std::vector<float> hf;
    if (!to_host(hf, feat, static_cast<size_t>(64 * P), s)) return efail(NET_E_DEVICE, "simfit: feature download");
    std::vector<uint8_t> member(P, 0);
    for (int64_t j = 0; j < n; ++j) {
        std::vector<int64_t> c;
        for (int64_t q = row[j]; q < row[j + 1]; ++q) c.push_back(q);
        std::stable_sort(c.begin(), c.end(), [&](int64_t a, int64_t b) {
            return hf[64 * a + 8] + hf[64 * a + 9] > hf[64 * b + 8] + hf[64 * b + 9];
        });
        // ceil(f n); the margin keeps f = 0.3 given as a float (0.30000001)
        // from taking an extra candidate when f n is an integer
        const size_t take = static_cast<size_t>(std::ceil(init_frac * static_cast<double>(c.size()) - 1e-6));
        for (size_t k = 0; k < take && k < c.size(); ++k) member[c[k]] = 1;
    }
    FitInputs in{};
    in.F = o->fluor;
    std::vector<uint32_t> thr;
    if (o->drive_rate_hz) {
        thr.resize(n);
        for (int64_t j = 0; j < n; ++j) thr[j] = pulse_threshold(o->drive_rate_hz[j], o->dt_ms);
        uint32_t* dthr = sc.get<uint32_t>(n);
        if (!dthr || !to_dev(dthr, thr, s)) return efail(NET_E_DEVICE, "simfit: upload");
        in.drive_thr = dthr;
    }
    in.pairs = dpairs;
    in.n = static_cast<int32_t>(n);
    in.nf = static_cast<int32_t>(nf);
    in.K = K;
    in.n_ref = o->n_ref;
    in.P = P;
    in.t_end = t_end;
    in.frame_num = o->frame_num;
    in.frame_den = o->frame_den;
    const double spf = static_cast<double>(o->frame_den) / static_cast<double>(o->frame_num);
    in.rho = static_cast<float>(std::pow(1.0 - o->dt_ms / static_cast<double>(o->tau_c_ms), spf));
    in.offset = o->offset;
    in.inv_jump = static_cast<float>(1.0 / (static_cast<double>(o->gain) * o->dt_ms));
    {
        std::vector<float> ws(static_cast<size_t>(n), o->w_assumed);
        if (o->w_source)
            for (int64_t i = 0; i < n; ++i) {
                ws[i] = o->w_source[i];
                if (!std::isfinite(ws[i])) return efail(NET_E_ARG, "simfit: w_source holds a non-finite weight");
            }
        float* dws = sc.get<float>(n);
        if (!dws) return efail(NET_E_OOM, "simfit: allocation");
        if (!to_dev(dws, ws, s)) return efail(NET_E_DEVICE, "simfit: upload");
        in.w_src = dws;
    }
    in.decay = o->dt_ms / static_cast<double>(o->tau_ms);
    in.v_rest = o->v_rest;
    in.v_reset = o->v_reset;
    in.v_th = o->v_th;
    in.sigma = o->noise_sigma;
    in.drive_amp = o->drive_amp;
    in.gamma = o->gamma;
    in.dt = o->dt_ms;
    in.tau_c = o->tau_c_ms;
    in.gain = o->gain;
    in.ctl_lo = static_cast<uint32_t>(o->control_seed);
    in.ctl_hi = static_cast<uint32_t>(o->control_seed >> 32);
    const uint64_t fs = opts ? opts->fit_seed : 0x5EEDF17ull;
    in.fit_lo = static_cast<uint32_t>(fs);
    in.fit_hi = static_cast<uint32_t>(fs >> 32);
    hipError_t e = fit_prep(in, w, s);
    if (e != hipSuccess) return efail(NET_E_DEVICE, std::string("simfit: ") + hipGetErrorString(e));
    std::vector<double> ll;
    for (int sw = 0; sw <= sweeps; ++sw) {
        if (!to_dev(w.member, member, s)) return efail(NET_E_DEVICE, "simfit: upload");
        e = fit_eval(in, w, s);
        if (e != hipSuccess) return efail(NET_E_DEVICE, std::string("simfit: ") + hipGetErrorString(e));
        if (!to_host(ll, w.ll, static_cast<size_t>(P + n), s)) return efail(NET_E_DEVICE, "simfit: evaluation");
        if (sw == sweeps) break;
        // per target, apply the single toggle that raises its likelihood most,
        // if by more than min_gain (coordinate ascent: every sweep improves
        // each target or leaves it; gains below min_gain are noise of the
        // K-realisation estimate)
        for (int64_t j = 0; j < n; ++j) {
            int64_t best = -1;
            double gain = min_gain;
            for (int64_t q = row[j]; q < row[j + 1]; ++q)
                if (ll[q] - ll[P + j] > gain) {
                    gain = ll[q] - ll[P + j];
                    best = q;
                }
            if (best >= 0) member[best] ^= 1;
        }
    }
    std::vector<float> score(P);
    for (int64_t q = 0; q < P; ++q) {
        const double cur = ll[P + sp[2 * q + 1]], tog = ll[q];
        score[perm[q]] = static_cast<float>(member[q] ? cur - tog : tog - cur);   // LL(G+e) - LL(G-e)
    }
    if (hipMemcpyAsync(out, score.data(), P * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return efail(NET_E_DEVICE, "simfit: output");
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
    DeviceScratch sc(s);
    st = features(obs, features_dev, s, sc);
    if (st != NET_OK) return st;
    if (hipStreamSynchronize(s) != hipSuccess) return efail(NET_E_DEVICE, "net_features: kernel");
    return NET_OK;
}

net_status net_estimate(const net_obs_desc* obs, int32_t method, net_mlp_t* scorer, const net_simfit_opts* opts,
                        float* scores_dev, void* stream) {
    net_status st = check_obs(obs);
    if (st != NET_OK) return st;
    if (!scores_dev && obs->n_pairs > 0) return efail(NET_E_ARG, "net_estimate: scores are NULL");
    if (obs->n_pairs == 0) return NET_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (method == NET_EST_AUTO) method = scorer ? NET_EST_SCORER : NET_EST_SIMFIT;
    if (method == NET_EST_SCORER) {
        if (!scorer) return efail(NET_E_ARG, "net_estimate: the scorer needs a trained MLP");
        DeviceScratch sc(s);
        float* feat = sc.get<float>(64 * obs->n_pairs);
        if (!feat) return efail(NET_E_OOM, "net_estimate: allocation");
        if ((st = features(obs, feat, s, sc)) != NET_OK) return st;
        st = net_mlp_forward(scorer, feat, obs->n_pairs, scores_dev, stream);
        if (st != NET_OK) return efail(st, std::string("net_estimate: ") + net_mlp_last_error());
        if (hipStreamSynchronize(s) != hipSuccess) return efail(NET_E_DEVICE, "net_estimate: scorer");
        return NET_OK;
    }
    if (method == NET_EST_SIMFIT) {
        if (!(obs->tau_ms > 0.0f) || obs->n_ref < 0) return efail(NET_E_ARG, "net_estimate: the fit needs the vertex model");
        return simfit(obs, opts, scores_dev, s);
    }
    return efail(NET_E_ARG, "net_estimate: unknown method");
}

}  // extern "C"
