// Simulation-based fit of functional edges (the paper's inverse problem,
// Sections 1 and 4; its own estimator is left to later work, so this is the
// plain fit used to judge the learned scorer).
//
// For target vertex j and a hypothesised in-neighbour set G, vertex j is
// simulated with the model of the forward path (LIF Euler step, refractory
// hold, control pulses, state noise, calcium transition of Section 3.3),
// driven by its sources' activity estimated from their own observations:
// input per step in frame f = sum_{i in G} w_i e_i(f) / S(f), e_i the
// deconvolved activity in spikes, S(f) the steps of frame f.  K noise
// realisations give the mean and variance of j's frame-averaged calcium,
// and the observed fluorescence is scored with the Gaussian observation
// model F = n*cbar + b + N(0, gamma^2) (Section 3.3):
//   LL_j(G) = -1/2 sum_f [ (F_j(f) - mu(f))^2 / s2(f) + log s2(f) ],
//   mu = n*mean_k cbar + b,  s2 = gamma^2 + n^2 var_k cbar.
//
//   fitprep_kernel   e_i(f) in spikes and the control-pulse bits of every vertex
//   fitbase_kernel   per (j, f): sum_{i in G_j} w_i e_i(f) / S(f)
//   fiteval_kernel   one lane per (variant, realisation); a variant is target j
//                    with G_j, or with one candidate toggled; K adjacent lanes
//                    hold the realisations of a variant.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "internal.h"
#include "philox.h"

namespace geonet {
namespace {

// Box-Muller in FP64 (the fit's vertex state is FP64 too): the 24-bit
// uniforms are exact, and log, sqrt and cos are correctly rounded or within
// an ulp, so a realisation's noise agrees with any other FP64 evaluation to
// about 1e-16 and cannot move a threshold crossing in practice.
__device__ __forceinline__ double gauss_fit(uint32_t a, uint32_t b) {
    const double u1 = (static_cast<double>(a >> 8) + 0.5) * 0x1p-24;
    const double u2 = (static_cast<double>(b >> 8) + 0.5) * 0x1p-24;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * 3.141592653589793 * u2);
}

__device__ __forceinline__ int64_t first_step(int64_t f, int64_t num, int64_t den) { return (f * den + num - 1) / num; }

struct FitPrepArgs {
    const float* F;            // [nf][n]
    const uint32_t* drive_thr; // [n] or null
    float* e;                  // [n][nf] activity in spikes
    uint32_t* pulses;          // [n][words] bit t: control pulse at step t
    int32_t n, nf, words;
    float rho, offset, inv_jump;   // inv_jump = 1 / (gain * dt)
    int64_t frame_num, frame_den, t_end;
    uint32_t key_lo, key_hi;
};

// One thread per (vertex, 32-step word) for the pulse bits; threads with a
// word index below nf also compute e(f) for f = word index.
__global__ void __launch_bounds__(256) fitprep_kernel(FitPrepArgs a) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = a.words > a.nf ? a.words : a.nf;
    if (idx >= static_cast<int64_t>(a.n) * per) return;
    const int j = static_cast<int>(idx / per), w = static_cast<int>(idx % per);
    if (w < a.nf) {
        const int f = w;
        const float x = a.F[static_cast<int64_t>(f) * a.n + j];
        const float e = f + 1 < a.nf
                            ? fmaxf(0.0f, (a.F[static_cast<int64_t>(f + 1) * a.n + j] - a.offset) - a.rho * (x - a.offset))
                            : 0.0f;
        a.e[static_cast<int64_t>(j) * a.nf + f] = e * a.inv_jump;
    }
    if (w < a.words) {
        uint32_t bits = 0;
        const uint32_t thr = a.drive_thr ? a.drive_thr[j] : 0u;
        if (thr != 0u) {
            for (int b = 0; b < 32; ++b) {
                const int64_t t = static_cast<int64_t>(w) * 32 + b;
                if (t >= a.t_end) break;
                const uint4 r = philox4x32_10(make_uint4(static_cast<uint32_t>(j), static_cast<uint32_t>(t),
                                                      static_cast<uint32_t>(static_cast<uint64_t>(t) >> 32), 0u),
                                           a.key_lo, a.key_hi);
                bits |= (r.x < thr ? 1u : 0u) << b;
            }
        }
        a.pulses[static_cast<int64_t>(j) * a.words + w] = bits;
    }
}

struct FitBaseArgs {
    const float* e;           // [n][nf]
    const int32_t* pairs;     // [P][2]
    const int64_t* row;       // [n+1] pairs of target j are [row[j], row[j+1]) (pairs sorted by target)
    const uint8_t* member;    // [P] 1 if the pair is in G
    const float* w_src;       // [n] assumed weight of the edges out of each vertex
    double* base;             // [n][nf]
    int32_t n, nf;
    int64_t frame_num, frame_den;
};

__global__ void __launch_bounds__(256) fitbase_kernel(FitBaseArgs a) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= static_cast<int64_t>(a.n) * a.nf) return;
    const int j = static_cast<int>(idx / a.nf), f = static_cast<int>(idx % a.nf);
    double s = 0.0;
    for (int64_t p = a.row[j]; p < a.row[j + 1]; ++p)
        if (a.member[p]) {
            const int i = a.pairs[2 * p];
            s += static_cast<double>(a.w_src[i]) * static_cast<double>(a.e[static_cast<int64_t>(i) * a.nf + f]);
        }
    const double steps = static_cast<double>(first_step(f + 1, a.frame_num, a.frame_den) -
                                             first_step(f, a.frame_num, a.frame_den));
    a.base[idx] = s / steps;
}

struct FitEvalArgs {
    const float* F;           // [nf][n] observed
    const float* e;           // [n][nf]
    const double* base;       // [n][nf]
    const uint32_t* pulses;   // [n][words]
    const int32_t* pairs;     // [P][2]
    const uint8_t* member;    // [P]
    const float* w_src;       // [n]
    double* ll;               // [P + n]: variant v < P toggles pair v; v = P + j is G_j itself
    int64_t P;
    int32_t n, nf, words, K;
    float sigma;
    double decay, v_rest, v_reset, v_th, drive_amp;
    int32_t n_ref;
    double dt, tau_c, gain, offset, gamma2;
    int64_t frame_num, frame_den;
    uint32_t key_lo, key_hi;  // fit noise key (realisation k mixed into the counter)
};

__global__ void __launch_bounds__(256) fiteval_kernel(FitEvalArgs a) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int K = a.K;
    const int64_t nvar = a.P + a.n;
    const int64_t v = r / K;
    const int k = static_cast<int>(r % K);
    const bool valid = v < nvar;
    int j = 0;
    int src = -1;
    double sign = 0.0;
    if (valid) {
        if (v < a.P) {
            j = a.pairs[2 * v + 1];
            src = a.pairs[2 * v];
            sign = (a.member[v] ? -1.0 : 1.0) * static_cast<double>(a.w_src[src]);
        } else {
            j = static_cast<int>(v - a.P);
        }
    }
    const double* bj = a.base + static_cast<int64_t>(j) * a.nf;
    const float* es = src >= 0 ? a.e + static_cast<int64_t>(src) * a.nf : nullptr;
    const uint32_t* pj = a.pulses + static_cast<int64_t>(j) * a.words;
    // V in FP64: the likelihood depends on V only through spike times, and
    // FP64 keeps threshold decisions aligned with the FP64 reference
    double V = a.v_rest;
    uint32_t age = 255u;
    double c = 0.0, acc = 0.0, ll = 0.0;
    const int group = lane - (lane % K);      // first lane of this variant's realisations
    int64_t t = 0;
    for (int f = 0; f < a.nf; ++f) {
        const int64_t t1 = first_step(f + 1, a.frame_num, a.frame_den);
        const double steps = static_cast<double>(t1 - t);
        double u = bj[f];
        if (es) u += sign * static_cast<double>(es[f]) / steps;
        uint32_t pw = pj[t >> 5];
        for (; t < t1; ++t) {
            if ((t & 31) == 0) pw = pj[t >> 5];
            acc += c;
            const bool spike = V >= a.v_th;
            c = c + a.dt * (-c / a.tau_c + (spike ? 1.0 : 0.0));
            if (spike) {
                V = a.v_reset;
                age = 1u;
                continue;
            }
            const bool held = age >= 1u && age <= static_cast<uint32_t>(a.n_ref);
            age = age >= 255u ? 255u : age + 1u;
            if (held) {
                V = a.v_reset;
                continue;
            }
            double in = u + (((pw >> (t & 31)) & 1u) ? a.drive_amp : 0.0);
            if (a.sigma != 0.0f) {
                const uint4 q = philox4x32_10(make_uint4(static_cast<uint32_t>(j), static_cast<uint32_t>(t),
                                                      static_cast<uint32_t>(static_cast<uint64_t>(t) >> 32),
                                                      2u + static_cast<uint32_t>(k)),
                                           a.key_lo, a.key_hi);
                in += static_cast<double>(a.sigma) * gauss_fit(q.y, q.z);
            }
            V = V + a.decay * (a.v_rest - V) + in;
        }
        // frame mean of this realisation, then mean/variance over the K lanes
        const double cbar = acc / steps;
        acc = 0.0;
        double s1 = 0.0, s2 = 0.0;
        for (int q = 0; q < K; ++q) {
            const double x = __shfl(cbar, group + q, 64);
            s1 += x;
            s2 += x * x;
        }
        const double mean = s1 / K, var = fmax(s2 / K - mean * mean, 0.0);
        const double mu = a.gain * mean + a.offset;
        const double s2f = a.gamma2 + a.gain * a.gain * var;
        const double dF = static_cast<double>(a.F[static_cast<int64_t>(f) * a.n + j]) - mu;
        ll += -0.5 * (dF * dF / s2f + log(s2f));
    }
    if (valid && k == 0) a.ll[v] = ll;
}

}  // namespace

hipError_t fit_prep(const FitInputs& in, const FitWork& w, hipStream_t s) {
    FitPrepArgs a;
    a.F = in.F;
    a.drive_thr = in.drive_thr;
    a.e = w.e;
    a.pulses = w.pulses;
    a.n = in.n;
    a.nf = in.nf;
    a.words = w.words;
    a.rho = in.rho;
    a.offset = in.offset;
    a.inv_jump = in.inv_jump;
    a.frame_num = in.frame_num;
    a.frame_den = in.frame_den;
    a.t_end = in.t_end;
    a.key_lo = in.ctl_lo;
    a.key_hi = in.ctl_hi;
    const int64_t per = w.words > in.nf ? w.words : in.nf;
    const int64_t tot = static_cast<int64_t>(in.n) * per;
    hipLaunchKernelGGL(fitprep_kernel, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t fit_eval(const FitInputs& in, const FitWork& w, hipStream_t s) {
    FitBaseArgs b;
    b.e = w.e;
    b.pairs = in.pairs;
    b.row = w.row;
    b.member = w.member;
    b.w_src = in.w_src;
    b.base = w.base;
    b.n = in.n;
    b.nf = in.nf;
    b.frame_num = in.frame_num;
    b.frame_den = in.frame_den;
    const int64_t nb = static_cast<int64_t>(in.n) * in.nf;
    hipLaunchKernelGGL(fitbase_kernel, dim3(static_cast<unsigned>((nb + 255) / 256)), dim3(256), 0, s, b);
    FitEvalArgs a;
    a.F = in.F;
    a.e = w.e;
    a.base = w.base;
    a.pulses = w.pulses;
    a.pairs = in.pairs;
    a.member = w.member;
    a.w_src = in.w_src;
    a.ll = w.ll;
    a.P = in.P;
    a.n = in.n;
    a.nf = in.nf;
    a.words = w.words;
    a.K = in.K;
    a.decay = in.decay;
    a.v_rest = in.v_rest;
    a.v_reset = in.v_reset;
    a.v_th = in.v_th;
    a.sigma = in.sigma;
    a.drive_amp = in.drive_amp;
    a.n_ref = in.n_ref;
    a.dt = in.dt;
    a.tau_c = in.tau_c;
    a.gain = in.gain;
    a.offset = in.offset;
    a.gamma2 = static_cast<double>(in.gamma) * static_cast<double>(in.gamma);
    a.frame_num = in.frame_num;
    a.frame_den = in.frame_den;
    a.key_lo = in.fit_lo;
    a.key_hi = in.fit_hi;
    const int64_t reps = (in.P + in.n) * in.K;
    hipLaunchKernelGGL(fiteval_kernel, dim3(static_cast<unsigned>((reps + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace geonet
