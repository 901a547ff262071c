// Observation-side kernels for the inverse problem (Sections 1 and 4 of the
// paper: estimating functional connectivity from calcium observations).
//
//   prep_kernel      per vertex: deconvolved activity e(f) = max(0, (F(f+1)-b)
//                    - rho (F(f)-b)) (the calcium model of Section 3.3 sampled
//                    at frame rate, rho = (1 - dt/tau_c)^(steps per frame)),
//                    standardised e and F, and the number of control pulses per
//                    frame (the experimenter's own drive schedule, Philox x0).
//   popmean_kernel   mean standardised activity over vertices per frame and the
//                    residual activity after removing it.
//   features_kernel  64 features per candidate pair (i -> j): lagged
//                    correlations of activity and fluorescence, responses of j
//                    to i's control pulses and the reverse, activity levels,
//                    distance.  Feature k is described in featureNames() of the
//                    Python binding.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "internal.h"
#include "philox.h"

namespace geonet {
namespace {

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct PrepArgs {
    const float* F;           // [nf][n]
    const uint32_t* drive_thr;  // [n] or null
    float* en;                // [n][nf] standardised activity
    float* zn;                // [n][nf] standardised fluorescence
    float* dc;                // [n][nf] control pulses per frame
    float* stats;             // [n][4]: mean e, std F, pulses, unused
    int32_t n, nf;
    float rho, offset;
    int64_t frame_num, frame_den;
    uint32_t key_lo, key_hi;
};

// One wave per vertex.
__global__ void __launch_bounds__(256) prep_kernel(PrepArgs a) {
    const int lane = threadIdx.x & 63;
    const int j = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (j >= a.n) return;
    float se = 0.f, see = 0.f, sf = 0.f, sff = 0.f, sp = 0.f;
    for (int f = lane; f < a.nf; f += 64) {
        const float x = a.F[static_cast<int64_t>(f) * a.n + j];
        const float e = f + 1 < a.nf
                            ? fmaxf(0.0f, (a.F[static_cast<int64_t>(f + 1) * a.n + j] - a.offset) - a.rho * (x - a.offset))
                            : 0.0f;
        a.en[static_cast<int64_t>(j) * a.nf + f] = e;
        se += e;
        see += e * e;
        sf += x;
        sff += x * x;
        // control pulses of vertex j in frame f (steps first(f) .. first(f+1)-1)
        float pulses = 0.0f;
        const uint32_t thr = a.drive_thr ? a.drive_thr[j] : 0u;
        if (thr != 0u) {
            const int64_t t0 = (static_cast<int64_t>(f) * a.frame_den + a.frame_num - 1) / a.frame_num;
            const int64_t t1 = (static_cast<int64_t>(f + 1) * a.frame_den + a.frame_num - 1) / a.frame_num;
            for (int64_t t = t0; t < t1; ++t) {
                const uint4 r = philox4x32_10(make_uint4(static_cast<uint32_t>(j), static_cast<uint32_t>(t),
                                                      static_cast<uint32_t>(static_cast<uint64_t>(t) >> 32), 0u),
                                           a.key_lo, a.key_hi);
                pulses += r.x < thr ? 1.0f : 0.0f;
            }
        }
        a.dc[static_cast<int64_t>(j) * a.nf + f] = pulses;
        sp += pulses;
    }
    se = wave_sum(se);
    see = wave_sum(see);
    sf = wave_sum(sf);
    sff = wave_sum(sff);
    sp = wave_sum(sp);
    const float inv = 1.0f / static_cast<float>(a.nf);
    const float me = se * inv, mf = sf * inv;
    const float ve = fmaxf(see * inv - me * me, 0.0f), vf = fmaxf(sff * inv - mf * mf, 0.0f);
    const float ie = ve > 1e-12f ? rsqrtf(ve) : 0.0f, iz = vf > 1e-12f ? rsqrtf(vf) : 0.0f;
    for (int f = lane; f < a.nf; f += 64) {
        const int64_t k = static_cast<int64_t>(j) * a.nf + f;
        a.en[k] = (a.en[k] - me) * ie;
        a.zn[k] = (a.F[static_cast<int64_t>(f) * a.n + j] - mf) * iz;
    }
    if (lane == 0) {
        a.stats[j * 4 + 0] = me;
        a.stats[j * 4 + 1] = sqrtf(vf);
        a.stats[j * 4 + 2] = sp;
        a.stats[j * 4 + 3] = 0.0f;
    }
}

// Population mean of the standardised activity per frame, then the
// standardised residual r_j(f) = std(e_j(f) - mean_f) per vertex.
__global__ void __launch_bounds__(256) popmean_kernel(const float* en, float* pm, int32_t n, int32_t nf) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    float s = 0.0f;
    for (int j = 0; j < n; ++j) s += en[static_cast<int64_t>(j) * nf + f];
    pm[f] = s / static_cast<float>(n);
}

__global__ void __launch_bounds__(256) residual_kernel(const float* en, const float* pm, float* rn, int32_t n,
                                                       int32_t nf) {
    const int lane = threadIdx.x & 63;
    const int j = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (j >= n) return;
    float s = 0.f, ss = 0.f;
    for (int f = lane; f < nf; f += 64) {
        const float r = en[static_cast<int64_t>(j) * nf + f] - pm[f];
        s += r;
        ss += r * r;
    }
    s = wave_sum(s);
    ss = wave_sum(ss);
    const float m = s / nf, v = fmaxf(ss / nf - m * m, 0.0f), iv = v > 1e-12f ? rsqrtf(v) : 0.0f;
    for (int f = lane; f < nf; f += 64) {
        const int64_t k = static_cast<int64_t>(j) * nf + f;
        rn[k] = (en[k] - pm[f] - m) * iv;
    }
}

struct FeatArgs {
    const float* en;
    const float* zn;
    const float* rn;
    const float* dc;
    const float* stats;
    const int32_t* pairs;     // [P][2] (i, j)
    const float* dist;        // [P]
    float* out;               // [P][64]
    int64_t P;
    int32_t nf;
};

// mean over valid f of a(f) * b(f + L)
__device__ __forceinline__ float lagcorr(const float* a, const float* b, int nf, int L, int lane) {
    float s = 0.0f;
    const int f0 = L < 0 ? -L : 0, f1 = L > 0 ? nf - L : nf;
    for (int f = f0 + lane; f < f1; f += 64) s += a[f] * b[f + L];
    s = wave_sum(s);
    return f1 > f0 ? s / static_cast<float>(f1 - f0) : 0.0f;
}

// response of b after the pulses of a: sum_f pa(f) b(f+L) / max(1, sum pa)
__device__ __forceinline__ float pulse_resp(const float* pa, float npulse, const float* b, int nf, int L, int lane) {
    float s = 0.0f;
    for (int f = lane; f + L < nf; f += 64) s += pa[f] * b[f + L];
    s = wave_sum(s);
    return s / fmaxf(1.0f, npulse);
}

// One wave per pair.
__global__ void __launch_bounds__(256) features_kernel(FeatArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (p >= a.P) return;
    const int i = a.pairs[2 * p], j = a.pairs[2 * p + 1];
    const int nf = a.nf;
    const float* ei = a.en + static_cast<int64_t>(i) * nf;
    const float* ej = a.en + static_cast<int64_t>(j) * nf;
    const float* zi = a.zn + static_cast<int64_t>(i) * nf;
    const float* zj = a.zn + static_cast<int64_t>(j) * nf;
    const float* ri = a.rn + static_cast<int64_t>(i) * nf;
    const float* rj = a.rn + static_cast<int64_t>(j) * nf;
    const float* di = a.dc + static_cast<int64_t>(i) * nf;
    const float* dj = a.dc + static_cast<int64_t>(j) * nf;
    const float npi = a.stats[i * 4 + 2], npj = a.stats[j * 4 + 2];
    float* o = a.out + p * 64;
    // every value below is wave-uniform after the reduction; lane 0 stores it
#define GEONET_PUT(k, expr)              \
    {                                    \
        const float val_ = (expr);       \
        if (lane == 0) o[(k)] = val_;    \
    }
    for (int L = -8; L <= 8; ++L) GEONET_PUT(L + 8, lagcorr(ei, ej, nf, L, lane))             // 0..16
    for (int L = -2; L <= 2; ++L) GEONET_PUT(19 + L, lagcorr(zi, zj, nf, L, lane))            // 17..21
    for (int L = 0; L < 6; ++L) GEONET_PUT(22 + L, pulse_resp(di, npi, ej, nf, L, lane))      // 22..27
    for (int L = 0; L < 4; ++L) GEONET_PUT(28 + L, pulse_resp(dj, npj, ei, nf, L, lane))      // 28..31
    GEONET_PUT(32, log1pf(npi))
    GEONET_PUT(33, log1pf(npj))
    GEONET_PUT(34, a.stats[i * 4 + 0])
    GEONET_PUT(35, a.stats[j * 4 + 0])
    GEONET_PUT(36, a.stats[i * 4 + 1])
    GEONET_PUT(37, a.stats[j * 4 + 1])
    GEONET_PUT(38, a.dist[p] * (1.0f / 150.0f))
    for (int L = 0; L < 4; ++L) GEONET_PUT(39 + L, lagcorr(ri, rj, nf, L, lane))              // 39..42
    for (int L = 0; L < 8; ++L) GEONET_PUT(43 + L, lagcorr(ei, zj, nf, L, lane))              // 43..50
    for (int L = 0; L < 8; ++L) GEONET_PUT(51 + L, lagcorr(zi, ej, nf, L, lane))              // 51..58
    for (int k = 59; k < 64; ++k) GEONET_PUT(k, 0.0f)
#undef GEONET_PUT
}

}  // namespace

namespace {
__global__ void __launch_bounds__(256) pulse_threshold_kernel(const float* rates, int32_t n, double dt_ms,
                                                              uint32_t* thr) {
    const int32_t j = static_cast<int32_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    // the same double-precision rule as pulse_threshold on the host
    const double t = floor(static_cast<double>(rates[j]) * (dt_ms * 1e-3) * 4294967296.0);
    thr[j] = !(t > 0.0) ? 0u : (t >= 4294967295.0 ? 0xFFFFFFFFu : static_cast<uint32_t>(t));
}
}  // namespace

hipError_t launch_pulse_thresholds(const float* rates, int32_t n, double dt_ms, uint32_t* thr, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(pulse_threshold_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, rates,
                       n, dt_ms, thr);
    return hipGetLastError();
}

hipError_t launch_features(const FeatureInputs& in, const FeatureWork& w, float* out, hipStream_t s) {
    PrepArgs pa;
    pa.F = in.F;
    pa.drive_thr = in.drive_thr;
    pa.en = w.en;
    pa.zn = w.zn;
    pa.dc = w.dc;
    pa.stats = w.stats;
    pa.n = in.n;
    pa.nf = in.nf;
    pa.rho = in.rho;
    pa.offset = in.offset;
    pa.frame_num = in.frame_num;
    pa.frame_den = in.frame_den;
    pa.key_lo = in.key_lo;
    pa.key_hi = in.key_hi;
    const int64_t th = static_cast<int64_t>(in.n) * 64;
    hipLaunchKernelGGL(prep_kernel, dim3(static_cast<unsigned>((th + 255) / 256)), dim3(256), 0, s, pa);
    hipLaunchKernelGGL(popmean_kernel, dim3(static_cast<unsigned>((in.nf + 255) / 256)), dim3(256), 0, s, w.en, w.pm,
                       in.n, in.nf);
    hipLaunchKernelGGL(residual_kernel, dim3(static_cast<unsigned>((th + 255) / 256)), dim3(256), 0, s, w.en, w.pm,
                       w.rn, in.n, in.nf);
    FeatArgs fa;
    fa.en = w.en;
    fa.zn = w.zn;
    fa.rn = w.rn;
    fa.dc = w.dc;
    fa.stats = w.stats;
    fa.pairs = in.pairs;
    fa.dist = in.dist;
    fa.out = out;
    fa.P = in.P;
    fa.nf = in.nf;
    const int64_t tp = in.P * 64;
    if (in.P > 0)
        hipLaunchKernelGGL(features_kernel, dim3(static_cast<unsigned>((tp + 255) / 256)), dim3(256), 0, s, fa);
    return hipGetLastError();
}

}  // namespace geonet
