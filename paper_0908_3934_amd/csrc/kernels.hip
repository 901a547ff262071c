// Device kernels of the geonet library (gfx950, wave64).
//
//   deliver_kernel      I_j(t) = sum over in-edges i -> j of w_ij * s_i(t - d_ij)
//                       (Section 3.2, Eq. izpsc last term) over the CSR-by-target
//                       slot list; a one-bit-per-vertex "fired within the last
//                       W steps" summary, staged in LDS, filters the edges
//                       whose sources' two last spike ages are gathered; the
//                       ages (and, rarely, the history ring) decide exactly.
//   node_update_kernel  spike test (Eq. spd), LIF Euler transition with the
//                       refractory hold (Section 3.1), control and noise
//                       (Philox4x32-10 + Box-Muller), spike-history ring,
//                       recent-spike summary, calcium and camera frames
//                       (Section 3.3).
//   step_kernel         one step in one launch: each workgroup delivers the
//                       in-edges of its own vertex segment into LDS (the
//                       same candidate test as deliver_kernel) and then runs
//                       the vertex update on that segment.
//   observe_kernel      fluorescence n*cbar + b + gamma*xi (Section 3.3) and
//                       state read-outs.
//   ensemble_kernel     many small networks, all steps of a call in one
//                       launch, each network's state resident in LDS.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "internal.h"
#include "philox.h"

namespace geonet {
namespace {

// Standard normal from two 32-bit draws (Box-Muller on 24-bit uniforms).
__device__ __forceinline__ float gaussian(uint32_t a, uint32_t b) {
    const float u1 = (static_cast<float>(a >> 8) + 0.5f) * 0x1p-24f;
    const float u2 = (static_cast<float>(b >> 8) + 0.5f) * 0x1p-24f;
    return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

// The same draw in FP64 (the Izhikevich vertex keeps its state in FP64).
__device__ __forceinline__ double gaussian_d(uint32_t a, uint32_t b) {
    const double u1 = (static_cast<double>(a >> 8) + 0.5) * 0x1p-24;
    const double u2 = (static_cast<double>(b >> 8) + 0.5) * 0x1p-24;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * 3.141592653589793 * u2);
}

// One step of the Izhikevich vertex (Section 3.1, Eq. izsimple) with its
// post-synaptic current (Section 3.2, Eqs. simplepsc, alphapsc, izpsc), from
// the state at t; `spike` is spd(V(t)), `in` the delivered sum (an impulse
// into r or p, or into V without a PSC), `u` the control current and `noise`
// sigma*xi.  The expressions are evaluated in the order the header states.
struct IzhState {
    double v, w, r, p;
};

__device__ __forceinline__ IzhState izh_step(const NetParams& p, const IzhState& s, bool spike, double in, double u,
                                             double noise) {
    IzhState n = s;
    if (p.psc == NET_PSC_EXP) {
        n.r = s.r - p.dt_d * p.psc_a * s.r + in;
    } else if (p.psc == NET_PSC_ALPHA) {
        n.r = s.r + p.dt_d * s.p;
        n.p = s.p + p.dt_d * (-p.psc_a * p.psc_a * s.r - 2.0 * p.psc_a * s.p) + in;
    }
    if (spike) {
        n.v = static_cast<double>(p.v_reset);
        n.w = s.w + p.iz_d;
    } else {
        const double syn = p.psc == NET_PSC_NONE ? 0.0 : s.r;
        const double cur = p.iz_k * (s.v - p.iz_vr) * (s.v - p.iz_vt) - s.w + syn + u;
        double vn = s.v + p.dt_d * p.iz_inv_c * cur;
        if (p.psc == NET_PSC_NONE) vn = vn + in;
        n.v = vn + noise;
        n.w = s.w + p.dt_d * p.iz_a * (p.iz_b * (s.v - p.iz_vr) - s.w);
    }
    return n;
}

// Hodgkin-Huxley vertex (Section 3.1's four-state model), one Euler step
// from the state at t: the rate functions of the standard squid-axon set
// (alpha_m, alpha_n at their limits where the denominator vanishes), the PSC
// kinds as for the Izhikevich vertex.  vprev keeps V(t) for the crossing
// test of the next step.
struct HhState {
    double v, vprev, m, n, h, r, p;
};

__device__ __forceinline__ double hh_am(double V) {
    const double x = V + 40.0;
    return x == 0.0 ? 1.0 : 0.1 * x / (1.0 - exp(-x / 10.0));
}
__device__ __forceinline__ double hh_bm(double V) { return 4.0 * exp(-(V + 65.0) / 18.0); }
__device__ __forceinline__ double hh_ah(double V) { return 0.07 * exp(-(V + 65.0) / 20.0); }
__device__ __forceinline__ double hh_bh(double V) { return 1.0 / (1.0 + exp(-(V + 35.0) / 10.0)); }
__device__ __forceinline__ double hh_an(double V) {
    const double x = V + 55.0;
    return x == 0.0 ? 0.1 : 0.01 * x / (1.0 - exp(-x / 10.0));
}
__device__ __forceinline__ double hh_bn(double V) { return 0.125 * exp(-(V + 65.0) / 80.0); }

__device__ __forceinline__ HhState hh_step(const NetParams& p, const HhState& s, double in, double u, double noise) {
    HhState n = s;
    if (p.psc == NET_PSC_EXP) {
        n.r = s.r - p.dt_d * p.psc_a * s.r + in;
    } else if (p.psc == NET_PSC_ALPHA) {
        n.r = s.r + p.dt_d * s.p;
        n.p = s.p + p.dt_d * (-p.psc_a * p.psc_a * s.r - 2.0 * p.psc_a * s.p) + in;
    }
    const double syn = p.psc == NET_PSC_NONE ? 0.0 : s.r;
    const double i_na = p.hh_gna * s.m * s.m * s.m * s.h * (s.v - p.hh_ena);
    const double i_k = p.hh_gk * s.n * s.n * s.n * s.n * (s.v - p.hh_ek);
    const double i_l = p.hh_gl * (s.v - p.hh_el);
    double vn = s.v + p.dt_d * p.hh_inv_c * (-i_na - i_k - i_l + syn + u);
    if (p.psc == NET_PSC_NONE) vn = vn + in;
    n.v = vn + noise;
    n.vprev = s.v;
    n.m = s.m + p.dt_d * (hh_am(s.v) * (1.0 - s.m) - hh_bm(s.v) * s.m);
    n.h = s.h + p.dt_d * (hh_ah(s.v) * (1.0 - s.h) - hh_bh(s.v) * s.h);
    n.n = s.n + p.dt_d * (hh_an(s.v) * (1.0 - s.n) - hh_bn(s.v) * s.n);
    return n;
}

__device__ __forceinline__ float half_bits_to_float(uint32_t bits) {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(bits)));
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

// Number of set bits of `bits` (8 per lane) in all lanes below this one:
// one ballot per bit position, counted below the lane with mbcnt, so no
// cross-lane data movement through LDS.
__device__ __forceinline__ uint32_t wave_bits_before(uint32_t bits) {
    uint32_t n = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t m = __ballot((bits >> b) & 1u);
        n += __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
    }
    return n;
}

// As wave_bits_before, also returning the wave's total (wave-uniform).
__device__ __forceinline__ uint32_t wave_bits_before_total(uint32_t bits, uint32_t* total) {
    uint32_t n = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t m = __ballot((bits >> b) & 1u);
        n += __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
        tot += static_cast<uint32_t>(__builtin_popcountll(m));
    }
    *total = tot;
    return n;
}

struct DeliverArgs {
    const int32_t* __restrict__ src;
    const uint16_t* __restrict__ w;
    const uint8_t* __restrict__ d;
    const uint32_t* __restrict__ sd;   // source | delay << 24 per slot (packed two-kernel variant)
    const uint16_t* __restrict__ s_lo;      // fused step: low 16 source bits per slot
    const uint32_t* __restrict__ dl_pair;   // fused step: delays per chunk pair and lane (4 words)
    const uint32_t* __restrict__ hi_pair;   // fused step: source >> 16 nibbles per chunk pair and lane (2 words)
    const uint8_t* __restrict__ rowstart;
    const int32_t* __restrict__ chunk_row0;
    const uint32_t* __restrict__ summary;
    const uint32_t* __restrict__ ring;
    const uint16_t* __restrict__ ages;   // per vertex: steps since its last spike | since the one before << 8
    float* __restrict__ I;
    int64_t n_chunks;
    int32_t summary_vec4;   // summary size in 16-byte units
    uint32_t t;             // step index modulo 2^32 (only t mod 256 matters)
    uint32_t n_pad;         // ring row length: word (slot/32, vertex) is at slot/32*n_pad + vertex
    uint32_t window;        // summary window W: bit set iff the vertex fired in the last W steps
    uint32_t sum_shift;     // summary bit of vertex s: s >> sum_shift (0, or 1: one bit per vertex pair)
    int32_t stage_vec4;     // compacted mode: the per-wave candidate stages start here in LDS (16-byte units)
    uint32_t age_sentinel;  // index of the ages entry that stays (255, 255): gathered by non-candidate edges
};

// One wave handles 512 consecutive slots per iteration: lane L owns slots
// 8L .. 8L+7 of the chunk, loaded as 2x16 B (sources) and 8 B (delays).
// Workgroups take contiguous chunk ranges; ranges of the workgroups that
// share an XCD (blockIdx % 8) are adjacent, so the history words they gather
// for neighbouring targets meet in that XCD's L2.
//
// A weight is needed only when its edge delivers a spike (a few in 10^4
// edges at physiological rates), so by default weights are not streamed: a
// wave that has an arrival loads the 16 B of weights of each lane then, and
// the stream is 5 B per edge instead of 7.  kWStream = true streams the
// weights with the chunk instead.
//
// Loop variants (same results): kMode 0 one chunk per wave iteration,
// kMode 1 two, kMode 2 one with the next chunk's stream loads issued while
// this chunk's gathers return, kMode 3 one with the candidates compacted
// across the wave before they are resolved (compact_resolve).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

struct ChunkRegs {
    u32x4 s_lo, s_hi;
    u32x4 wq;
    u32x2 dq;
};

// The fused step's chunk: one word per edge, source in bits 0..23 and delay
// in bits 24..31, so that the stream is 4 B per edge (2x16 B per lane).
struct PackedChunk {
    u32x4 lo, hi;
};

__device__ __forceinline__ uint32_t comp4(const u32x4& v, int k) {
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}
__device__ __forceinline__ uint32_t edge_src(const ChunkRegs& x, int k) {
    return k < 4 ? comp4(x.s_lo, k) : comp4(x.s_hi, k - 4);
}
__device__ __forceinline__ uint32_t edge_delay(const ChunkRegs& x, int k) {
    return ((k < 4 ? x.dq.x : x.dq.y) >> (8 * (k & 3))) & 0xFFu;
}
__device__ __forceinline__ uint32_t edge_src(const PackedChunk& x, int k) {
    return (k < 4 ? comp4(x.lo, k) : comp4(x.hi, k - 4)) & 0xFFFFFFu;
}
__device__ __forceinline__ uint32_t edge_delay(const PackedChunk& x, int k) {
    return (k < 4 ? comp4(x.lo, k) : comp4(x.hi, k - 4)) >> 24;
}

// One chunk of the fused step's 3.5 B-per-slot stream: the lane's 8 low
// source halves, 8 delay bytes and 8 high source nibbles.
struct NarrowChunk {
    u32x4 lo;
    u32x2 dl;
    uint32_t hi;
};
__device__ __forceinline__ uint32_t edge_src(const NarrowChunk& x, int k) {
    return ((comp4(x.lo, k >> 1) >> (16 * (k & 1))) & 0xFFFFu) | (((x.hi >> (4 * k)) & 0xFu) << 16);
}
__device__ __forceinline__ uint32_t edge_delay(const NarrowChunk& x, int k) {
    return ((k < 4 ? x.dl.x : x.dl.y) >> (8 * (k & 3))) & 0xFFu;
}

// Chunks c and c + 1 (c even) of the narrow stream: four loads per lane
// (16 B of low halves per chunk, 16 B of delays and 8 B of nibbles per pair).
__device__ __forceinline__ void load_narrow_pair(NarrowChunk* x, const DeliverArgs& a, int64_t c, int lane) {
    const int64_t e0 = c * kChunkEdges + lane * kEdgesPerLane;
    x[0].lo = *reinterpret_cast<const u32x4*>(a.s_lo + e0);
    x[1].lo = *reinterpret_cast<const u32x4*>(a.s_lo + e0 + kChunkEdges);
    const int64_t rec = (c >> 1) * 64 + lane;
    const u32x4 dl = *reinterpret_cast<const u32x4*>(a.dl_pair + rec * 4);
    const u32x2 hi = *reinterpret_cast<const u32x2*>(a.hi_pair + rec * 2);
    x[0].dl = u32x2{dl.x, dl.y};
    x[1].dl = u32x2{dl.z, dl.w};
    x[0].hi = hi.x;
    x[1].hi = hi.y;
}

__device__ __forceinline__ void load_packed_chunk(PackedChunk& x, const uint32_t* sd, int64_t c, int lane) {
    const int64_t e0 = c * kChunkEdges + lane * kEdgesPerLane;
    x.lo = *reinterpret_cast<const u32x4*>(sd + e0);
    x.hi = *reinterpret_cast<const u32x4*>(sd + e0 + 4);
}

// Stream loads of one chunk (optionally non-temporal).
template <bool kWStream, bool kNT>
__device__ __forceinline__ void load_chunk(ChunkRegs& x, const DeliverArgs& a, int64_t c, int lane) {
    const int64_t e0 = c * kChunkEdges + lane * kEdgesPerLane;
    if (kNT) {
        x.s_lo = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(a.src + e0));
        x.s_hi = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(a.src + e0 + 4));
        if (kWStream) x.wq = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(a.w + e0));
        x.dq = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(a.d + e0));
    } else {
        x.s_lo = *reinterpret_cast<const u32x4*>(a.src + e0);
        x.s_hi = *reinterpret_cast<const u32x4*>(a.src + e0 + 4);
        if (kWStream) x.wq = *reinterpret_cast<const u32x4*>(a.w + e0);
        x.dq = *reinterpret_cast<const u32x2*>(a.d + e0);
    }
}

// Summary test of one chunk and a gather of two spike ages per candidate
// edge (a 2 B word per vertex, 2 MiB at N = 2^20, which stays in L2).  A
// candidate edge (its source fired within the summary window, or the edge is
// longer than the window) gathers its source's ages; every other edge takes
// the ages (255, 255), which can match no delay of a non-candidate (those are
// at most the window, below 255), so the resolution below needs no candidate
// mask.  `shift` is the summary resolution (0: one bit per vertex).
template <bool kLdsSummary, class Chunk>
__device__ __forceinline__ void gather_chunk(const Chunk& x, const DeliverArgs& a, const uint32_t* lds_summary,
                                             uint32_t shift, uint32_t* aw) {
    uint32_t sv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) sv[k] = edge_src(x, k);
    const char* ages = reinterpret_cast<const char*>(a.ages);
    uint32_t sw[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t sb = sv[k] >> shift;
        sw[k] = kLdsSummary ? lds_summary[sb >> 5] : a.summary[sb >> 5];
    }
    // Only candidate lanes issue the gather (the texture path's cost grows
    // with the active lanes); the others keep the sentinel ages.
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t dk = edge_delay(x, k);
        const bool cand = (__builtin_amdgcn_ubfe(sw[k], sv[k] >> shift, 1) != 0u) | (dk > a.window);   // bit mod 32
        uint32_t v = 0xFFFFu;
        if (cand) v = *reinterpret_cast<const uint16_t*>(ages + (sv[k] << 1));
        aw[k] = v;
    }
}

// With a1 <= a2 the ages of the source's last two spikes (255 = "255 or
// more"), the source fired at t - d only if d == a1 or d >= a2; most chunks
// have no such edge and skip the resolution (wave-uniform).
template <class Chunk>
__device__ __forceinline__ bool chunk_may_fire(const Chunk& x, const uint32_t* aw) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t dk = edge_delay(x, k);
        any = any | (dk == (aw[k] & 0xFFu)) | (dk >= ((aw[k] >> 8) & 0xFFu));
    }
    return wave_ballot(any) != 0;
}

// Exact arrival test.  For d < a2 the only spike within d steps is the one at
// a1 (exact, since a1 < a2 <= 255), so the source fired at t - d iff d == a1.
// For d >= a2 (an older spike may sit at t - d, or a2 = d = 255 is saturated)
// the history ring decides.
template <class Chunk>
__device__ __forceinline__ uint32_t fired_bits(const Chunk& x, const DeliverArgs& a, uint32_t t,
                                               const uint32_t* aw) {
    uint32_t fired = 0, need = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t dk = edge_delay(x, k);
        const uint32_t a1 = aw[k] & 0xFFu, a2 = (aw[k] >> 8) & 0xFFu;
        const bool ring = dk >= a2;
        fired |= (!ring && dk == a1 ? 1u : 0u) << k;
        need |= (ring ? 1u : 0u) << k;
    }
    if (wave_ballot(need != 0)) {
        uint32_t slot[8], word[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t dk = edge_delay(x, k);
            slot[k] = (t - dk) & 0xFFu;
            word[k] = a.ring[((need >> k) & 1u) ? (slot[k] >> 5) * a.n_pad + edge_src(x, k) : 0u];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) fired |= (((need >> k) & (word[k] >> (slot[k] & 31))) & 1u) << k;
    }
    return fired;
}

// Compacted resolution of one chunk (kMode 3).  The summary test marks the
// candidates (~5 % of edges); instead of every lane resolving its 8 edges,
// the wave writes its candidates (source | delay << 24) to its own LDS stage
// at slots counted with one ballot per edge position, then resolves them 64
// at a time, one candidate per lane (one age gather per lane, the ring read
// for the rare three-spike case), and returns each arrival to the lane that
// owns the edge through a ballot.  Sources must be below 2^24.
template <bool kLdsSummary>
__device__ __forceinline__ uint32_t compact_resolve(const ChunkRegs& x, const DeliverArgs& a,
                                                    const uint32_t* lds_summary, uint32_t t, uint32_t* stage,
                                                    int lane) {
    const uint32_t sv[8] = {x.s_lo.x, x.s_lo.y, x.s_lo.z, x.s_lo.w, x.s_hi.x, x.s_hi.y, x.s_hi.z, x.s_hi.w};
    uint32_t dv[8], cand = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t s = sv[k];
        const uint32_t sb = s >> a.sum_shift;
        const uint32_t sw = kLdsSummary ? lds_summary[sb >> 5] : a.summary[sb >> 5];
        dv[k] = ((k < 4 ? x.dq.x : x.dq.y) >> (8 * (k & 3))) & 0xFFu;
        cand |= (((sw >> (sb & 31)) & 1u) | (dv[k] > a.window ? 1u : 0u)) << k;
    }
    uint32_t slot[8], total = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint64_t m = wave_ballot((cand >> k) & 1u);
        slot[k] = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                            __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), total));
        total += static_cast<uint32_t>(__builtin_popcountll(m));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if ((cand >> k) & 1u) stage[slot[k]] = sv[k] | (dv[k] << 24);
    uint32_t fired = 0;
    for (uint32_t r = 0; r < total; r += 64) {
        const uint32_t q = r + static_cast<uint32_t>(lane);
        const bool valid = q < total;
        const uint32_t e = valid ? stage[q] : 0u;
        const uint32_t s = e & 0xFFFFFFu, d = e >> 24;
        const uint32_t aw = a.ages[s];
        const uint32_t a1 = aw & 0xFFu, a2 = aw >> 8;
        bool f = valid && d < 255u && (d == a1 || d == a2);
        const bool need = valid && !f && (d == 255u || d > a2);
        if (wave_ballot(need)) {
            const uint32_t sl = (t - d) & 0xFFu;
            const uint32_t w = a.ring[need ? (sl >> 5) * a.n_pad + s : 0u];
            f = f || (need && ((w >> (sl & 31u)) & 1u));
        }
        const uint64_t R = wave_ballot(f);
        if (R != 0) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t p = slot[k] - r;
                if (((cand >> k) & 1u) && p < 64u) fired |= static_cast<uint32_t>((R >> p) & 1u) << k;
            }
        }
    }
    return fired;
}

// Arrivals of one chunk (called by the whole wave when any lane has one).
// Row of each fired slot from the row-start bits (position 0 of the chunk
// belongs to chunk_row0 whether or not it opens a row), then one exact FP32
// atomic add per arrival.  All partial sums of a row are exact in FP32, so
// the order of these additions does not change the result.  The row-start
// byte, the chunk's first row and (unless streamed) the weights are loaded
// together, and the prefix count of row starts needs no LDS round trip.
template <bool kWStream>
__device__ __forceinline__ void deliver_fired(const DeliverArgs& a, int64_t c, int lane, uint32_t fired,
                                              const u32x4& wq_stream) {
    const int64_t e0 = c * kChunkEdges + lane * kEdgesPerLane;
    const uint32_t rs = a.rowstart[c * 64 + lane];
    const int32_t first_row = a.chunk_row0[c];
    u32x4 wq = wq_stream;
    if (!kWStream) {
        // only lanes with an arrival load their 16 B of weights
        wq = u32x4{0u, 0u, 0u, 0u};
        if (fired) wq = *reinterpret_cast<const u32x4*>(a.w + e0);
    }
    const uint32_t bits = lane == 0 ? (rs & ~1u) : rs;
    const int32_t row0 = first_row + static_cast<int32_t>(wave_bits_before(bits));
    const uint32_t wv[4] = {wq.x, wq.y, wq.z, wq.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if ((fired >> k) & 1u) {
            const int32_t row = row0 + __popc(bits & ((2u << k) - 1u));
            unsafeAtomicAdd(a.I + row, half_bits_to_float((wv[k >> 1] >> (16 * (k & 1))) & 0xFFFFu));
        }
    }
}

template <bool kLdsSummary, bool kWStream, bool kNT, int kMode>
__global__ void __launch_bounds__(1024) deliver_kernel(DeliverArgs a) {
    extern __shared__ uint4 lds_summary4[];
    const uint32_t* lds_summary = reinterpret_cast<const uint32_t*>(lds_summary4);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform chunk index
    const int nwaves = blockDim.x >> 6;
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const int lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int64_t c_begin = static_cast<int64_t>(lb) * a.n_chunks / nb;
    const int64_t c_end = static_cast<int64_t>(lb + 1) * a.n_chunks / nb;
    const uint32_t t = a.t;
    constexpr int kPer = (kMode == 1 || kMode == 4) ? 2 : 1;   // chunks per iteration
    const int64_t stride = static_cast<int64_t>(nwaves) * kPer;

    if (kLdsSummary) {
        const uint4* g = reinterpret_cast<const uint4*>(a.summary);
        for (int i = threadIdx.x; i < a.summary_vec4; i += blockDim.x) lds_summary4[i] = g[i];
        __syncthreads();
    }

    int64_t c = c_begin + static_cast<int64_t>(wave) * kPer;
    if (kMode == 4) {
        // two packed chunks per iteration; the next pair's stream loads are
        // issued right after this pair's gathers (unconditional: past the
        // range they re-read this pair, which L2 still holds), so waiting
        // for the gathers never waits for them
        PackedChunk cur[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) load_packed_chunk(cur[u], a.sd, c + u < c_end ? c + u : c_begin, lane);
        for (; c < c_end; c += stride) {
            uint32_t aw[2][8];
#pragma unroll
            for (int u = 0; u < 2; ++u) gather_chunk<kLdsSummary>(cur[u], a, lds_summary, a.sum_shift, aw[u]);
            const int64_t cn = c + stride;
            PackedChunk nxt[2];
#pragma unroll
            for (int u = 0; u < 2; ++u)
                load_packed_chunk(nxt[u], a.sd, cn + u < c_end ? cn + u : (c + u < c_end ? c + u : c), lane);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (c + u < c_end && chunk_may_fire(cur[u], aw[u])) {
                    const uint32_t fired = fired_bits(cur[u], a, t, aw[u]);
                    if (wave_ballot(fired != 0)) deliver_fired<false>(a, c + u, lane, fired, u32x4{0u, 0u, 0u, 0u});
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) cur[u] = nxt[u];
        }
    } else if (kMode == 3) {
        uint32_t* stage = reinterpret_cast<uint32_t*>(lds_summary4 + a.stage_vec4) + wave * kChunkEdges;
        for (; c < c_end; c += stride) {
            ChunkRegs cur;
            load_chunk<kWStream, kNT>(cur, a, c, lane);
            const uint32_t fired = compact_resolve<kLdsSummary>(cur, a, lds_summary, t, stage, lane);
            if (wave_ballot(fired != 0)) deliver_fired<kWStream>(a, c, lane, fired, cur.wq);
        }
    } else if (kMode == 2) {
        ChunkRegs cur;
        if (c < c_end) load_chunk<kWStream, kNT>(cur, a, c, lane);
        for (; c < c_end; c += stride) {
            uint32_t aw[8];
            gather_chunk<kLdsSummary>(cur, a, lds_summary, a.sum_shift, aw);
            const ChunkRegs now = cur;
            // the next chunk's stream is in flight while the gathers return
            // (unconditional, so waiting for the gathers never waits for it;
            // the last iteration reloads its own chunk)
            load_chunk<kWStream, kNT>(cur, a, c + stride < c_end ? c + stride : c, lane);
            if (chunk_may_fire(now, aw)) {
                const uint32_t fired = fired_bits(now, a, t, aw);
                if (wave_ballot(fired != 0)) deliver_fired<kWStream>(a, c, lane, fired, now.wq);
            }
        }
    } else {
        for (; c < c_end; c += stride) {
            // chunks beyond the range repeat the last one and are masked below
            ChunkRegs cur[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u)
                load_chunk<kWStream, kNT>(cur[u], a, c + u < c_end ? c + u : c_end - 1, lane);
            uint32_t aw[kPer][8];
#pragma unroll
            for (int u = 0; u < kPer; ++u) gather_chunk<kLdsSummary>(cur[u], a, lds_summary, a.sum_shift, aw[u]);
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                if (c + u < c_end && chunk_may_fire(cur[u], aw[u])) {
                    const uint32_t fired = fired_bits(cur[u], a, t, aw[u]);
                    if (wave_ballot(fired != 0)) deliver_fired<kWStream>(a, c + u, lane, fired, cur[u].wq);
                }
            }
        }
    }
}

struct NodeArgs {
    float* __restrict__ V;
    const uint16_t* __restrict__ age;    // ages read (step t)
    uint16_t* __restrict__ age_out;      // ages written (for step t + 1); may equal age
    float* __restrict__ I;
    uint32_t* __restrict__ ring;
    uint32_t* __restrict__ summary;
    const NetParams* __restrict__ params;
    const int32_t* __restrict__ net_id;
    const uint32_t* __restrict__ drive_thr;
    const float* __restrict__ i_ext;
    double* __restrict__ calcium;
    double* __restrict__ frame_acc;
    float* __restrict__ frames;
    uint64_t* __restrict__ rec_raster;
    float* __restrict__ rec_v;
    float* __restrict__ rec_input;
    double* __restrict__ Vd;      // Izhikevich state (null without Izhikevich networks)
    double* __restrict__ Wd;
    double* __restrict__ psc_r;
    double* __restrict__ psc_p;
    double* __restrict__ hh_m;    // Hodgkin-Huxley gates and V(t-1) (null without HH networks)
    double* __restrict__ hh_n;
    double* __restrict__ hh_h;
    double* __restrict__ hh_vprev;
    int32_t* __restrict__ spk_hist;   // plastic networks: last kStdpHist spike steps per vertex
    int32_t* __restrict__ spk_cnt;
    // push delivery (else null): out-edges of each source and the input ring
    // (slot s at push_ring + s * n_pad) the spikes of this step add into
    const uint32_t* __restrict__ out_off;
    const uint2* __restrict__ out_edge;
    float* __restrict__ push_ring;
    uint32_t push_mask;
    const int32_t* __restrict__ caller_of;   // renumbered networks: caller's index of each vertex (else null)
    // graph replays (else null): the step is *t_dev + t_off, and the frame
    // bookkeeping follows from it (frame_num > 0: observation on)
    const uint64_t* __restrict__ t_dev;
    uint32_t t_off;
    int32_t frame_num, frame_den;
    int64_t n_total, n_pad, rec_row, raster_words, frame_index;
    uint32_t t_lo, t_hi;
    int32_t d_sum, frame_flush, frame_steps, frame_cap, sum_shift;
    NetParams p0;
};

// State a vertex update reads from memory (besides the input), loaded ahead
// of the update by the fused step.
// (Four registers per vertex: the fused step keeps several per thread.)
struct VertexState {
    float v;
    uint32_t ages;   // the two spike ages; vertex_random adds the drive pulse as bit 16
    uint32_t aux;    // the drive threshold (0: not driven); vertex_random replaces it by the noise's bits
    uint32_t ring;   // the history word that holds this step's bit
};

// In a graph replay the step comes from the device counter: its Philox
// counter words and, with observation on, whether the camera frame closes
// this step (frame(t) = floor(t num / den); a frame of steps first(f) ..
// first(f+1) - 1, first(f) = ceil(f den / num)).
__device__ __forceinline__ void apply_device_step(NodeArgs& a) {
    if (!a.t_dev) return;
    const uint64_t t = *a.t_dev + a.t_off;
    a.t_lo = static_cast<uint32_t>(t);
    a.t_hi = static_cast<uint32_t>(t >> 32);
    if (a.push_ring) a.I = a.push_ring + static_cast<int64_t>(a.t_lo & a.push_mask) * a.n_pad;   // this step's slot
    if (a.frame_num > 0) {
        const int64_t num = a.frame_num, den = a.frame_den;
        const int64_t ti = static_cast<int64_t>(t);
        const int64_t f = ti * num / den, f1 = (ti + 1) * num / den;
        a.frame_index = f;
        a.frame_flush = f1 != f ? 1 : 0;
        a.frame_steps = static_cast<int32_t>(((f + 1) * den + num - 1) / num - (f * den + num - 1) / num);
    }
}

__device__ __forceinline__ VertexState load_vertex_state(const NodeArgs& a, int64_t j, int64_t j_end) {
    const int64_t jj = j < j_end ? j : 0;
    VertexState st;
    st.v = a.V[jj];
    st.ages = a.age[jj];
    st.aux = a.drive_thr ? a.drive_thr[jj] : 0u;
    st.ring = a.out_edge ? 0u : a.ring[((a.t_lo & 0xFFu) >> 5) * a.n_pad + jj];   // (push delivery keeps no ring)
    return st;
}

// Control input and state noise of step t for vertex j: the drive pulse is
// an integer compare of the first Philox word with the rate threshold, the
// noise a Box-Muller draw from the next two (Section 3.1 control and noise).
// Used only where the vertex is neither spiking nor held.
template <bool kMulti>
__device__ __forceinline__ void vertex_random(const NodeArgs& a, int64_t j, int64_t j_end, VertexState& st) {
    const int64_t jj = j < j_end ? j : 0;
    const NetParams p = kMulti ? a.params[a.net_id[jj]] : a.p0;
    const uint32_t thr = st.aux;
    float noise = 0.0f;
    uint32_t pulse = 0;
    if (thr != 0u || p.sigma != 0.0f) {
        const uint32_t jl = static_cast<uint32_t>((a.caller_of ? a.caller_of[jj] : jj) - p.node_off);
        const uint4 r = philox4x32_10(make_uint4(jl, a.t_lo, a.t_hi, 0u), p.key_lo, p.key_hi);
        pulse = r.x < thr ? 1u : 0u;
        if (p.sigma != 0.0f) noise = p.sigma * gaussian(r.y, r.z);
    }
    st.ages |= pulse << 16;
    st.aux = __float_as_uint(noise);
}

// Vertex update of step t for vertex j with delivered input `in` (all lanes
// of a wave call it together, on 64 consecutive vertices starting at a
// multiple of 64).  Vertices j >= j_end are not this caller's; the wave's
// raster and summary words are written only when their first vertex is below
// word_end.  `st` is the vertex's state as load_vertex_state returns it,
// completed by vertex_random.
template <bool kMulti, bool kModels = false>
__device__ __forceinline__ void vertex_update(const NodeArgs& a, int64_t j, int64_t j_end, int64_t word_end, float in,
                                              bool clear_input, const VertexState& st) {
    const int lane = threadIdx.x & 63;
    const bool valid = j < j_end;
    const int64_t jj = valid ? j : 0;
    const NetParams p = kMulti ? a.params[a.net_id[jj]] : a.p0;
    const bool izh = kModels && p.model == NET_MODEL_IZHIKEVICH;
    const bool hh = kModels && p.model == NET_MODEL_HODGKIN_HUXLEY;
    IzhState zs{};
    HhState hs{};
    if (izh) zs = IzhState{a.Vd[jj], a.Wd[jj], a.psc_r[jj], a.psc_p[jj]};
    if (hh) hs = HhState{a.Vd[jj], a.hh_vprev[jj], a.hh_m[jj], a.hh_n[jj], a.hh_h[jj], a.psc_r[jj], a.psc_p[jj]};
    const float v = izh ? static_cast<float>(zs.v) : (hh ? static_cast<float>(hs.v) : st.v);
    const uint32_t ages = st.ages & 0xFFFFu;
    const uint32_t age = ages & 0xFFu, age2 = ages >> 8;
    const double vth = static_cast<double>(p.v_th);
    const bool spike = valid && (izh ? zs.v >= vth : (hh ? (hs.v >= vth && hs.vprev < vth) : v >= p.v_th));

    const uint64_t spikes = wave_ballot(spike);
    if (a.rec_raster && lane == 0 && j < word_end && j < a.n_total)
        a.rec_raster[a.rec_row * a.raster_words + (j >> 6)] = spikes;
    if (a.out_edge && spikes != 0) {
        // push delivery: the wave walks the out-edges of each of its spiking
        // vertices, 64 at a time, adding each weight into the ring slot of its
        // arrival step t + d (never slot t, which this step reads: the ring
        // has more slots than the largest delay).  The sums are exact, so the
        // order of the atomics changes no bit.
        // Two rounds of 64 edges are loaded before their atomics are issued.
        const int64_t j0 = j - lane;
        for (uint64_t m = spikes; m != 0; m &= m - 1) {
            const int64_t src = j0 + __builtin_ctzll(m);
            const uint32_t e1 = a.out_off[src + 1];
            for (uint32_t e = a.out_off[src] + static_cast<uint32_t>(lane); e < e1; e += 128u) {
                const bool second = e + 64u < e1;
                const uint2 ed0 = a.out_edge[e];
                const uint2 ed1 = second ? a.out_edge[e + 64u] : make_uint2(0u, 0u);
                atomicAdd(a.push_ring + static_cast<int64_t>((a.t_lo + (ed0.y >> 16)) & a.push_mask) * a.n_pad + ed0.x,
                          half_bits_to_float(ed0.y & 0xFFFFu));
                if (second)
                    atomicAdd(a.push_ring + static_cast<int64_t>((a.t_lo + (ed1.y >> 16)) & a.push_mask) * a.n_pad + ed1.x,
                              half_bits_to_float(ed1.y & 0xFFFFu));
            }
        }
    }
    if (valid) {
        if (a.rec_v) a.rec_v[a.rec_row * a.n_total + j] = v;
        if (a.rec_input) a.rec_input[a.rec_row * a.n_total + j] = in;
        if (clear_input) a.I[j] = 0.0f;
        // spike-history ring: bit (t mod 256) of vertex j (other slots of the
        // word are only read elsewhere in this step); written only when it
        // changes
        const uint32_t slot = a.t_lo & 0xFFu;
        const uint32_t m = 1u << (slot & 31);
        if (!a.out_edge && ((st.ring & m) != 0u) != spike) a.ring[(slot >> 5) * a.n_pad + j] = st.ring ^ m;
    }

    float vn;
    uint32_t age_n;
    const bool held = age >= 1u && age <= static_cast<uint32_t>(p.n_ref);
    if (izh) {
        age_n = spike ? 1u : (age >= static_cast<uint32_t>(kAgeNever) ? kAgeNever : age + 1u);
        double u = 0.0, noise = 0.0;
        if (!spike) {
            const uint32_t thr = a.drive_thr ? a.drive_thr[jj] : 0u;
            u = a.i_ext ? static_cast<double>(a.i_ext[jj]) : 0.0;
            if (thr != 0u || p.sigma != 0.0f) {
                const uint32_t jl = static_cast<uint32_t>((a.caller_of ? a.caller_of[jj] : jj) - p.node_off);
                const uint4 r = philox4x32_10(make_uint4(jl, a.t_lo, a.t_hi, 0u), p.key_lo, p.key_hi);
                if (r.x < thr) u = u + static_cast<double>(p.drive_amp);
                noise = static_cast<double>(p.sigma) * gaussian_d(r.y, r.z);
            }
        }
        zs = izh_step(p, zs, spike, static_cast<double>(in), u, noise);
        vn = static_cast<float>(zs.v);
    } else if (hh) {
        age_n = spike ? 1u : (age >= static_cast<uint32_t>(kAgeNever) ? kAgeNever : age + 1u);
        const uint32_t thr = a.drive_thr ? a.drive_thr[jj] : 0u;
        double u = a.i_ext ? static_cast<double>(a.i_ext[jj]) : 0.0, noise = 0.0;
        if (thr != 0u || p.sigma != 0.0f) {
            const uint32_t jl = static_cast<uint32_t>((a.caller_of ? a.caller_of[jj] : jj) - p.node_off);
            const uint4 r = philox4x32_10(make_uint4(jl, a.t_lo, a.t_hi, 0u), p.key_lo, p.key_hi);
            if (r.x < thr) u = u + static_cast<double>(p.drive_amp);
            noise = static_cast<double>(p.sigma) * gaussian_d(r.y, r.z);
        }
        hs = hh_step(p, hs, static_cast<double>(in), u, noise);
        vn = static_cast<float>(hs.v);
    } else if (spike) {
        vn = p.v_reset;
        age_n = 1u;
    } else {
        age_n = age >= static_cast<uint32_t>(kAgeNever) ? kAgeNever : age + 1u;
        if (held) {
            vn = p.v_reset;
        } else {
            float u = a.i_ext ? a.i_ext[jj] : 0.0f;
            if ((st.ages >> 16) & 1u) u += p.drive_amp;
            vn = v + p.decay * (p.v_rest - v) + in + u + __uint_as_float(st.aux);
        }
    }
    // recent-spike summary for the next step: last spike within d_sum steps
    const uint64_t recent = wave_ballot(valid && age_n <= static_cast<uint32_t>(a.d_sum));
    if (lane == 0 && j < word_end && !a.out_edge) {   // (push delivery needs no summary)
        if (a.sum_shift == 0) {
            reinterpret_cast<uint64_t*>(a.summary)[j >> 6] = recent;
        } else {
            // one bit per vertex pair: OR the pairs, then pack the even bits
            uint64_t x = (recent | (recent >> 1)) & 0x5555555555555555ull;
            x = (x | (x >> 1)) & 0x3333333333333333ull;
            x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
            x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
            x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
            x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
            a.summary[j >> 6] = static_cast<uint32_t>(x);
        }
    }

    if (valid) {
        a.V[j] = vn;
        if (kModels && spike && a.spk_hist) {
            // plasticity: the step of this spike joins the vertex's recent spike times
            const int32_t c = a.spk_cnt[j];
            a.spk_hist[j * kStdpHist + (c % kStdpHist)] = static_cast<int32_t>(a.t_lo);
            a.spk_cnt[j] = c + 1;
        }
        if (izh) {
            a.Vd[j] = zs.v;
            a.Wd[j] = zs.w;
            a.psc_r[j] = zs.r;
            a.psc_p[j] = zs.p;
        }
        if (hh) {
            a.Vd[j] = hs.v;
            a.hh_vprev[j] = hs.vprev;
            a.hh_m[j] = hs.m;
            a.hh_n[j] = hs.n;
            a.hh_h[j] = hs.h;
            a.psc_r[j] = hs.r;
            a.psc_p[j] = hs.p;
        }
        // the previous last spike becomes the one before the last
        const uint32_t older = spike ? age : age2;
        const uint32_t age2_n = older >= static_cast<uint32_t>(kAgeNever) ? kAgeNever : older + 1u;
        a.age_out[j] = static_cast<uint16_t>(age_n | (age2_n << 8));
        if (a.calcium) {
            // calcium and its frame sum in FP64: tau_c / dt is thousands of steps
            const double c = a.calcium[j];
            double acc = a.frame_acc[j] + c;
            if (a.frame_flush) {
                if (a.frame_index < a.frame_cap)
                    a.frames[a.frame_index * a.n_pad + j] = static_cast<float>(acc / static_cast<double>(a.frame_steps));
                acc = 0.0;
            }
            a.frame_acc[j] = acc;
            a.calcium[j] = c + p.dt_d * (-c / p.tau_c_d + (spike ? 1.0 : 0.0));
        }
    }
}

template <bool kMulti, bool kModels>
__global__ void __launch_bounds__(256) node_update_kernel(NodeArgs a) {
    apply_device_step(a);
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const float in = a.I[j < a.n_total ? j : 0];
    VertexState st = load_vertex_state(a, j, a.n_total);
    // the Izhikevich vertex draws its own (FP64) noise inside vertex_update
    if (!kModels || (kMulti ? a.params[a.net_id[j < a.n_total ? j : 0]] : a.p0).model == NET_MODEL_LIF)
        vertex_random<kMulti>(a, j, a.n_total, st);
    vertex_update<kMulti, kModels>(a, j, a.n_total, a.n_pad, in, true, st);
}

// ---------------------------------------------------------------------------
// Ensemble kernel: one launch advances every network of an ensemble by
// n_steps.  Each workgroup owns a packed set of networks and keeps their whole
// state in LDS (V, input accumulator, age, a 32- or 256-step history ring,
// calcium); per step it runs the delivery of all its networks, one barrier,
// the vertex update of all its networks, one barrier.  Networks never share a
// workgroup's data with other workgroups, so no grid-wide synchronisation is
// needed.  Edges stream from global memory (L2/MALL resident for ensembles).
// The arithmetic per vertex and per edge is the same as in node_update_kernel
// and deliver_kernel.
// ---------------------------------------------------------------------------
struct EnsembleArgs {
    const int32_t* __restrict__ src;
    const uint16_t* __restrict__ w;
    const uint8_t* __restrict__ d;
    const uint8_t* __restrict__ rowstart;
    const int32_t* __restrict__ chunk_row0;
    const NetMeta* __restrict__ meta;
    const int32_t* __restrict__ wg_nets;
    const int32_t* __restrict__ wg_off;
    const NetParams* __restrict__ params;
    const uint32_t* __restrict__ drive_thr;
    const float* __restrict__ i_ext;
    float* __restrict__ V;
    uint16_t* __restrict__ age;
    uint32_t* __restrict__ ring;
    uint32_t* __restrict__ summary;
    double* __restrict__ calcium;
    double* __restrict__ frame_acc;
    float* __restrict__ frames;
    uint64_t* __restrict__ rec_raster;
    float* __restrict__ rec_v;
    float* __restrict__ rec_input;
    double* __restrict__ Vd;      // Izhikevich state in global memory (null without Izhikevich networks)
    double* __restrict__ Wd;
    double* __restrict__ psc_r;
    double* __restrict__ psc_p;
    double* __restrict__ hh_m;    // Hodgkin-Huxley gates and V(t-1) in global memory
    double* __restrict__ hh_n;
    double* __restrict__ hh_h;
    double* __restrict__ hh_vprev;
    const int32_t* __restrict__ caller_of;   // renumbered networks (else null)
    const uint64_t* __restrict__ t_dev;      // graph replays: the first step (else null: t0)
    const uint16_t* __restrict__ ls;         // 2 B per slot: source within its network, or with
                                             // sbits < 16 source | delay << sbits
    const uint32_t* __restrict__ push_off;   // out-edge tables of the networks with a spike log
    const uint32_t* __restrict__ push_edge;
    const uint2* __restrict__ drv;           // driven vertices (index | counter index << 16, threshold)
    int64_t t0, n_total, n_pad, raster_words;
    int32_t n_steps, frame_cap, frame_num, frame_den, d_sum, sbits;
};

struct NetLds {
    double* c;      // first: 8-byte aligned (lds_off is a multiple of 16)
    double* acc;
    float* V;
    float* I;
    uint32_t* age;
    uint32_t* ring;
};

__device__ __forceinline__ NetLds carve(uint8_t* base, const NetMeta& nm, bool obs) {
    NetLds L;
    const int n = nm.n_nodes;
    L.c = reinterpret_cast<double*>(base + nm.lds_off);
    L.acc = obs ? L.c + n : L.c;
    L.V = reinterpret_cast<float*>(obs ? L.acc + n : L.c);
    L.I = L.V + n;
    L.age = reinterpret_cast<uint32_t*>(L.I + n);
    L.ring = L.age + n;
    return L;
}

// Write the 64 bits `bits` of local vertices [u0, u0+64) (union numbering
// u0 = first vertex) into a bit array of 64-bit words shared with other
// networks: clear this network's positions (mask), then set its bits.
__device__ __forceinline__ void put_bits_shared(uint64_t* words, int64_t u0, uint64_t bits, uint64_t mask) {
    const int64_t w0 = u0 >> 6;
    const int sh = static_cast<int>(u0 & 63);
    atomicAnd(reinterpret_cast<unsigned long long*>(words + w0), ~(mask << sh));
    atomicOr(reinterpret_cast<unsigned long long*>(words + w0), (bits & mask) << sh);
    if (sh != 0 && (mask >> (64 - sh)) != 0) {
        atomicAnd(reinterpret_cast<unsigned long long*>(words + w0 + 1), ~(mask >> (64 - sh)));
        atomicOr(reinterpret_cast<unsigned long long*>(words + w0 + 1), (bits & mask) >> (64 - sh));
    }
}

// Delivery of one chunk of a network held in LDS: arrival test against the
// LDS history ring (sl: each slot's source within its network, dk: its
// delay), then each arrival's FP16 weight added into the LDS input of its
// row.  With `held`, the chunk's weights, row-start bits and first row come
// from registers (loaded once for all steps), else they are loaded when the
// chunk has an arrival.
__device__ __forceinline__ void ens_deliver_chunk(const EnsembleArgs& a, const NetMeta& nm, const NetLds& L,
                                                  uint32_t rmask, int64_t t, int c, int lane, const uint32_t (&sl)[8],
                                                  const uint32_t (&dk)[8], bool held, const u32x4& h_w,
                                                  uint32_t h_rs, int32_t h_row0) {
    const int64_t e0 = static_cast<int64_t>(c) * kChunkEdges + lane * kEdgesPerLane;
    uint32_t fired = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t slot = (static_cast<uint32_t>(t) - dk[k]) & rmask;
        const uint32_t word = L.ring[sl[k] * static_cast<uint32_t>(nm.words) + (slot >> 5)];
        fired |= ((word >> (slot & 31u)) & 1u) << k;
    }
    if (wave_ballot(fired != 0)) {
        const uint32_t rs = held ? h_rs : a.rowstart[static_cast<int64_t>(c) * 64 + lane];
        const uint32_t bits = lane == 0 ? (rs & ~1u) : rs;
        const int32_t row0 = (held ? h_row0 : a.chunk_row0[c]) - nm.node_off + static_cast<int32_t>(wave_bits_before(bits));
        uint32_t wb[8];
        if (held) {
            const uint32_t hw[4] = {h_w.x, h_w.y, h_w.z, h_w.w};
#pragma unroll
            for (int k = 0; k < 8; ++k) wb[k] = (hw[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) wb[k] = ((fired >> k) & 1u) ? a.w[e0 + k] : 0u;   // arrivals only
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if ((fired >> k) & 1u) {
                const int32_t row = row0 + __popc(bits & ((2u << k) - 1u));
                atomicAdd(L.I + row, half_bits_to_float(wb[k]));
            }
        }
    }
}

// A network's spike log in LDS: bucket b (= step mod 32) counts the
// vertices that fired at its step and lists the first log_cap of them.
struct NetLog {
    uint32_t* cnt;
    uint16_t* ids;
};

__device__ __forceinline__ NetLog log_of(uint8_t* base, const NetMeta& nm) {
    NetLog g;
    g.cnt = reinterpret_cast<uint32_t*>(base + nm.log_off);
    g.ids = reinterpret_cast<uint16_t*>(base + nm.log_off + 128);
    return g;
}

// Wave-uniform: every spike of the last maxd steps is listed in the log
// (else the step is delivered by the pull over the in-edges).
__device__ __forceinline__ bool log_complete(const NetLog& g, const NetMeta& nm, int64_t t, int lane) {
    const bool over = lane >= 1 && lane <= nm.maxd &&
                      g.cnt[(static_cast<uint32_t>(t) - static_cast<uint32_t>(lane)) & 31u] >
                          static_cast<uint32_t>(nm.log_cap);
    return wave_ballot(over) == 0;
}

// Delivery of step t by one wave from the spike log: the spike of source s
// at step t - d reaches, at step t, the out-edges of s with delay d, one
// (s, d) group per lane, its edges read four at a time.
__device__ __forceinline__ void ens_push(const EnsembleArgs& a, const NetMeta& nm, const NetLds& L, const NetLog& g,
                                         int64_t t, int lane) {
    const uint32_t cap = static_cast<uint32_t>(nm.log_cap);
    const uint32_t tt = static_cast<uint32_t>(t);
    uint32_t total = 0;
    for (int d = 1; d <= nm.maxd; ++d) total += min(g.cnt[(tt - static_cast<uint32_t>(d)) & 31u], cap);
    for (uint32_t first = 0; first < total; first += 64) {
        const uint32_t idx = first + static_cast<uint32_t>(lane);
        int my_d = 0;
        uint32_t my_i = 0, pre = 0;
        for (int d = 1; d <= nm.maxd; ++d) {
            const uint32_t c = min(g.cnt[(tt - static_cast<uint32_t>(d)) & 31u], cap);
            if (idx >= pre && idx < pre + c) {
                my_d = d;
                my_i = idx - pre;
            }
            pre += c;
        }
        if (my_d == 0) continue;
        const uint32_t src = g.ids[((tt - static_cast<uint32_t>(my_d)) & 31u) * cap + my_i];
        const int64_t o = static_cast<int64_t>(nm.po_base) + static_cast<int64_t>(src) * nm.maxd + my_d - 1;
        const uint32_t e0 = a.push_off[o], e1 = a.push_off[o + 1];
        for (uint32_t e = e0; e < e1; e += 4) {
            uint32_t v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = e + k < e1 ? a.push_edge[e + k] : 0u;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (e + k < e1) atomicAdd(L.I + (v[k] & 0xFFFFu), half_bits_to_float(v[k] >> 16));
        }
    }
}

// kModels: 0 for LIF networks only, 1 with Izhikevich networks, 2 with
// Hodgkin-Huxley networks too (the FP64 branches a kernel cannot meet are
// compiled out: the LIF kernel needs no register spills).  kStream: how a
// wave reads its chunks.  kEnsHeld: the plan gives every workgroup one
// network of at most one chunk per wave, whose chunk then stays in
// registers (a separate instantiation, so that the registers it holds do
// not weigh on the streaming kernels).  kEnsLocal: each step streams the
// 2-byte local sources and the delay bytes (3 B per slot); kEnsPacked: the
// 2-byte slots carry the delay too (2 B per slot), when every network's
// vertex count and largest delay fit in 16 bits together.  A held FP64
// model kernel runs at most 512 threads per workgroup, which gives it twice
// the registers and no spills; the streaming ones keep 1024 threads (more
// waves for large networks' edges) at the cost of some spills.
template <int kModels, int kStream>
__global__ void __launch_bounds__((kModels == 0 || kStream != kEnsHeld) ? 1024 : 512) ensemble_kernel(EnsembleArgs a) {
    const int64_t t0 = a.t_dev ? static_cast<int64_t>(*a.t_dev) : a.t0;   // graph replays read the step
    extern __shared__ uint4 lds4[];
    uint8_t* lds = reinterpret_cast<uint8_t*>(lds4);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = blockDim.x >> 6;
    const int q_begin = a.wg_off[blockIdx.x], q_end = a.wg_off[blockIdx.x + 1];
    const bool obs = a.calcium != nullptr;

    // ---- spike logs: cleared, then refilled from the history ring below
    if (kStream != kEnsHeld) {
        for (int q = q_begin; q < q_end; ++q) {
            const NetMeta nm = a.meta[a.wg_nets[q]];
            if (nm.log_cap > 0 && tid < 32) log_of(lds, nm).cnt[tid] = 0u;
        }
        __syncthreads();
    }
    // ---- load the state of every network of this workgroup into LDS
    for (int q = q_begin; q < q_end; ++q) {
        const NetMeta nm = a.meta[a.wg_nets[q]];
        const NetLds L = carve(lds, nm, obs);
        for (int j = tid; j < nm.n_nodes; j += blockDim.x) {
            const int64_t u = nm.node_off + j;
            L.V[j] = a.V[u];
            L.I[j] = 0.0f;
            L.age[j] = a.age[u] & 0xFFu;
            if (obs) {
                L.c[j] = a.calcium[u];
                L.acc[j] = a.frame_acc[u];
            }
            const uint32_t* gr = a.ring + u;          // word b of vertex u at gr[b * n_pad]
            if (nm.words == kRingWords) {
#pragma unroll
                for (int k = 0; k < kRingWords; ++k) L.ring[j * kRingWords + k] = gr[k * a.n_pad];
            } else {
                // steps t0-32 .. t0-1 into one word, bit = step mod 32
                const uint32_t q32 = static_cast<uint32_t>(t0) & 31u;
                const uint32_t hi = gr[((static_cast<uint32_t>(t0 - 1) & 255u) >> 5) * a.n_pad];
                const uint32_t lo = gr[((static_cast<uint32_t>(t0 - 32) & 255u) >> 5) * a.n_pad];
                const uint32_t m = (1u << q32) - 1u;
                const uint32_t r = q32 == 0 ? hi : ((hi & m) | (lo & ~m));
                L.ring[j] = r;
                if (kStream != kEnsHeld && nm.log_cap > 0) {
                    // bit b of the word is the step congruent to b mod 32: its bucket
                    const NetLog g = log_of(lds, nm);
                    for (uint32_t bits = r; bits != 0u; bits &= bits - 1u) {
                        const uint32_t b = static_cast<uint32_t>(__builtin_ctz(bits));
                        const uint32_t pos = atomicAdd(g.cnt + b, 1u);
                        if (pos < static_cast<uint32_t>(nm.log_cap)) g.ids[b * nm.log_cap + pos] = static_cast<uint16_t>(j);
                    }
                }
            }
        }
    }
    __syncthreads();

    // A workgroup that holds one network of at most one chunk per wave keeps
    // that chunk (sources, delays, weights, row starts) in registers for all
    // its steps: no load on the per-step path.
    constexpr bool held = kStream == kEnsHeld;
    u32x4 h_lo = u32x4{0u, 0u, 0u, 0u}, h_hi = h_lo, h_w = h_lo;
    u32x2 h_d = u32x2{0u, 0u};
    uint32_t h_rs = 0u;
    int32_t h_row0 = 0;
    if (held) {
        const NetMeta nm = a.meta[a.wg_nets[q_begin]];
        const int c = nm.chunk_begin + wave;
        if (c < nm.chunk_end) {
            const int64_t e = static_cast<int64_t>(c) * kChunkEdges + lane * kEdgesPerLane;
            h_lo = *reinterpret_cast<const u32x4*>(a.src + e);
            h_hi = *reinterpret_cast<const u32x4*>(a.src + e + 4);
            h_d = *reinterpret_cast<const u32x2*>(a.d + e);
            h_w = *reinterpret_cast<const u32x4*>(a.w + e);
            h_rs = a.rowstart[static_cast<int64_t>(c) * 64 + lane];
            h_row0 = a.chunk_row0[c];
        }
    }

    for (int s = 0; s < a.n_steps; ++s) {
        const int64_t t = t0 + s;
        // ---- delivery: I_j(t) = sum of w over in-edges whose source fired at t - d
        for (int q = q_begin; q < q_end; ++q) {
            const NetMeta nm = a.meta[a.wg_nets[q]];
            const NetLds L = carve(lds, nm, obs);
            const uint32_t rmask = 32u * static_cast<uint32_t>(nm.words) - 1u;
            if (held) {
                const int c = nm.chunk_begin + wave;
                if (c < nm.chunk_end) {
                    const uint32_t sv[8] = {h_lo.x, h_lo.y, h_lo.z, h_lo.w, h_hi.x, h_hi.y, h_hi.z, h_hi.w};
                    uint32_t sl[8], dk[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        sl[k] = sv[k] - static_cast<uint32_t>(nm.node_off);
                        dk[k] = ((k < 4 ? h_d.x : h_d.y) >> (8 * (k & 3))) & 0xFFu;
                    }
                    ens_deliver_chunk(a, nm, L, rmask, t, c, lane, sl, dk, true, h_w, h_rs, h_row0);
                }
                continue;
            }
            if (nm.log_cap > 0) {
                const NetLog g = log_of(lds, nm);
                if (tid == 0) g.cnt[static_cast<uint32_t>(t) & 31u] = 0u;   // refilled by this step's update
                if (log_complete(g, nm, t, lane)) continue;                    // pushed below
            }
            // the next kDepth - 1 chunks' slots are in flight while this chunk
            // is resolved (a register ring of this wave's chunks c, c + nwaves,
            // ...); weights and row starts are read only for chunks with an
            // arrival (streaming them too measured slower)
            constexpr bool packed = kStream == kEnsPacked;
            constexpr int kDepth = packed ? 4 : 3;
            const uint32_t smask = (1u << a.sbits) - 1u;
            int c = nm.chunk_begin + wave;
            u32x4 q_s[kDepth];
            u32x2 q_d[kDepth];
#pragma unroll
            for (int u = 0; u < kDepth; ++u) {
                q_s[u] = u32x4{0u, 0u, 0u, 0u};
                q_d[u] = u32x2{0u, 0u};
                if (c + u * nwaves < nm.chunk_end) {
                    const int64_t e = static_cast<int64_t>(c + u * nwaves) * kChunkEdges + lane * kEdgesPerLane;
                    q_s[u] = *reinterpret_cast<const u32x4*>(a.ls + e);
                    if (!packed) q_d[u] = *reinterpret_cast<const u32x2*>(a.d + e);
                }
            }
            for (; c < nm.chunk_end; c += nwaves) {
                const int64_t e0 = static_cast<int64_t>(c) * kChunkEdges + lane * kEdgesPerLane;
                const u32x4 sq = q_s[0];
                const u32x2 dq = q_d[0];
#pragma unroll
                for (int u = 0; u + 1 < kDepth; ++u) {
                    q_s[u] = q_s[u + 1];
                    q_d[u] = q_d[u + 1];
                }
                if (c + kDepth * nwaves < nm.chunk_end) {
                    const int64_t e = e0 + static_cast<int64_t>(kDepth * nwaves) * kChunkEdges;
                    q_s[kDepth - 1] = *reinterpret_cast<const u32x4*>(a.ls + e);
                    if (!packed) q_d[kDepth - 1] = *reinterpret_cast<const u32x2*>(a.d + e);
                }
                uint32_t sl[8], dk[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t v = (comp4(sq, k >> 1) >> (16 * (k & 1))) & 0xFFFFu;
                    sl[k] = packed ? (v & smask) : v;
                    dk[k] = packed ? (v >> a.sbits) : (((k < 4 ? dq.x : dq.y) >> (8 * (k & 3))) & 0xFFu);
                }
                ens_deliver_chunk(a, nm, L, rmask, t, c, lane, sl, dk, false, h_w, 0u, 0);
            }
        }
        // drive pulses of noise-free LIF networks: the Philox draw only for the
        // driven vertices, its outcome as bit 16 of the vertex's LDS age word
        // (the update of this step reads and clears it)
        if (a.drv) {
            for (int q = q_begin; q < q_end; ++q) {
                const int m = a.wg_nets[q];
                const NetMeta nm = a.meta[m];
                if (nm.drv_end == nm.drv_begin || a.params[m].model != NET_MODEL_LIF || a.params[m].sigma != 0.0f)
                    continue;
                const NetLds L = carve(lds, nm, obs);
                const uint32_t key_lo = a.params[m].key_lo, key_hi = a.params[m].key_hi;
                for (int i = nm.drv_begin + tid; i < nm.drv_end; i += blockDim.x) {
                    const uint2 dv = a.drv[i];
                    const uint4 r = philox4x32_10(make_uint4(dv.x >> 16, static_cast<uint32_t>(t),
                                                             static_cast<uint32_t>(static_cast<uint64_t>(t) >> 32), 0u),
                                                  key_lo, key_hi);
                    if (r.x < dv.y) L.age[dv.x & 0xFFFFu] |= 1u << 16;
                }
            }
        }
        // networks whose logs hold every recent spike: one wave each pushes
        // the spikes along their out-edges
        if (!held) {
            for (int q = q_begin + wave; q < q_end; q += nwaves) {
                const NetMeta nm = a.meta[a.wg_nets[q]];
                if (nm.log_cap == 0) continue;
                const NetLog g = log_of(lds, nm);
                if (log_complete(g, nm, t, lane)) ens_push(a, nm, carve(lds, nm, obs), g, t, lane);
            }
        }
        __syncthreads();
        // ---- vertex update (same rules as node_update_kernel)
        for (int q = q_begin; q < q_end; ++q) {
            const int m = a.wg_nets[q];
            const NetMeta nm = a.meta[m];
            const NetParams p = a.params[m];
            const NetLds L = carve(lds, nm, obs);
            const uint32_t rmask = 32u * static_cast<uint32_t>(nm.words) - 1u;
            for (int base = 0; base < nm.n_nodes; base += blockDim.x) {
                const int j = base + tid;
                const bool valid = j < nm.n_nodes;
                const int jj = valid ? j : 0;
                const int64_t u = nm.node_off + jj;
                const bool izh = kModels >= 1 && p.model == NET_MODEL_IZHIKEVICH;
                const bool hh = kModels >= 2 && p.model == NET_MODEL_HODGKIN_HUXLEY;
                IzhState zs{};
                HhState hs{};
                if (izh) zs = IzhState{a.Vd[u], a.Wd[u], a.psc_r[u], a.psc_p[u]};
                if (hh) hs = HhState{a.Vd[u], a.hh_vprev[u], a.hh_m[u], a.hh_n[u], a.hh_h[u], a.psc_r[u], a.psc_p[u]};
                const float v = izh ? static_cast<float>(zs.v) : (hh ? static_cast<float>(hs.v) : L.V[jj]);
                const uint32_t age_word = L.age[jj];   // bit 16: a precomputed drive pulse
                const uint32_t age = age_word & 0xFFFFu;
                const float in = L.I[jj];
                const double vth = static_cast<double>(p.v_th);
                const bool spike =
                    valid && (izh ? zs.v >= vth : (hh ? (hs.v >= vth && hs.vprev < vth) : v >= p.v_th));
                const uint64_t spikes = wave_ballot(spike);
                const uint64_t alive = wave_ballot(valid);
                if (a.rec_raster && lane == 0 && alive != 0)
                    put_bits_shared(a.rec_raster + s * a.raster_words, nm.node_off + base + wave * 64, spikes, alive);
                if (kStream != kEnsHeld && nm.log_cap > 0 && spikes != 0) {
                    // this step's spikes into bucket t mod 32 (one atomic per wave)
                    const NetLog g = log_of(lds, nm);
                    const uint32_t b = static_cast<uint32_t>(t) & 31u;
                    const int leader = __builtin_ctzll(spikes);
                    uint32_t first = 0;
                    if (lane == leader) first = atomicAdd(g.cnt + b, static_cast<uint32_t>(__popcll(spikes)));
                    first = __shfl(first, leader, 64);
                    if (spike) {
                        const uint32_t pos = first + __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(spikes >> 32),
                                                                               __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(spikes), 0u));
                        if (pos < static_cast<uint32_t>(nm.log_cap)) g.ids[b * nm.log_cap + pos] = static_cast<uint16_t>(j);
                    }
                }
                float vn;
                uint32_t age_n;
                const bool held = age >= 1u && age <= static_cast<uint32_t>(p.n_ref);
                if (izh) {
                    age_n = spike ? 1u : (age >= static_cast<uint32_t>(kAgeNever) ? kAgeNever : age + 1u);
                    double uu = 0.0, noise = 0.0;
                    if (!spike) {
                        const uint32_t thr = a.drive_thr ? a.drive_thr[u] : 0u;
                        uu = a.i_ext ? static_cast<double>(a.i_ext[u]) : 0.0;
                        if (thr != 0u || p.sigma != 0.0f) {
                            const uint4 r = philox4x32_10(make_uint4(static_cast<uint32_t>(a.caller_of ? a.caller_of[u] - nm.node_off : jj), static_cast<uint32_t>(t),
                                                                     static_cast<uint32_t>(static_cast<uint64_t>(t) >> 32), 0u),
                                                          p.key_lo, p.key_hi);
                            if (r.x < thr) uu = uu + static_cast<double>(p.drive_amp);
                            noise = static_cast<double>(p.sigma) * gaussian_d(r.y, r.z);
                        }
                    }
                    zs = izh_step(p, zs, spike, static_cast<double>(in), uu, noise);
                    vn = static_cast<float>(zs.v);
                    if (valid) {
                        a.Vd[u] = zs.v;
                        a.Wd[u] = zs.w;
                        a.psc_r[u] = zs.r;
                        a.psc_p[u] = zs.p;
                    }
                } else if (hh) {
                    age_n = spike ? 1u : (age >= static_cast<uint32_t>(kAgeNever) ? kAgeNever : age + 1u);
                    const uint32_t thr = a.drive_thr ? a.drive_thr[u] : 0u;
                    double uu = a.i_ext ? static_cast<double>(a.i_ext[u]) : 0.0, noise = 0.0;
                    if (thr != 0u || p.sigma != 0.0f) {
                        const uint4 r = philox4x32_10(make_uint4(static_cast<uint32_t>(a.caller_of ? a.caller_of[u] - nm.node_off : jj), static_cast<uint32_t>(t),
                                                                 static_cast<uint32_t>(static_cast<uint64_t>(t) >> 32), 0u),
                                                      p.key_lo, p.key_hi);
                        if (r.x < thr) uu = uu + static_cast<double>(p.drive_amp);
                        noise = static_cast<double>(p.sigma) * gaussian_d(r.y, r.z);
                    }
                    hs = hh_step(p, hs, static_cast<double>(in), uu, noise);
                    vn = static_cast<float>(hs.v);
                    if (valid) {
                        a.Vd[u] = hs.v;
                        a.hh_vprev[u] = hs.vprev;
                        a.hh_m[u] = hs.m;
                        a.hh_n[u] = hs.n;
                        a.hh_h[u] = hs.h;
                        a.psc_r[u] = hs.r;
                        a.psc_p[u] = hs.p;
                    }
                } else if (spike) {
                    vn = p.v_reset;
                    age_n = 1u;
                } else {
                    age_n = age >= static_cast<uint32_t>(kAgeNever) ? kAgeNever : age + 1u;
                    if (held) {
                        vn = p.v_reset;
                    } else {
                        float uu = a.i_ext ? a.i_ext[u] : 0.0f;
                        float noise = 0.0f;
                        if (a.drv && p.sigma == 0.0f) {
                            if ((age_word >> 16) & 1u) uu += p.drive_amp;   // drawn in the delivery phase
                        } else {
                            const uint32_t thr = a.drive_thr ? a.drive_thr[u] : 0u;
                            if (thr != 0u || p.sigma != 0.0f) {
                                const uint4 r = philox4x32_10(make_uint4(static_cast<uint32_t>(a.caller_of ? a.caller_of[u] - nm.node_off : jj), static_cast<uint32_t>(t),
                                                                  static_cast<uint32_t>(static_cast<uint64_t>(t) >> 32), 0u),
                                                       p.key_lo, p.key_hi);
                                if (r.x < thr) uu += p.drive_amp;
                                if (p.sigma != 0.0f) noise = p.sigma * gaussian(r.y, r.z);
                            }
                        }
                        vn = v + p.decay * (p.v_rest - v) + in + uu + noise;
                    }
                }
                if (valid) {
                    if (a.rec_v) a.rec_v[s * a.n_total + u] = v;
                    if (a.rec_input) a.rec_input[s * a.n_total + u] = in;
                    L.I[j] = 0.0f;
                    const uint32_t slot = static_cast<uint32_t>(t) & rmask;
                    uint32_t* wp = L.ring + j * nm.words + (slot >> 5);
                    const uint32_t mb = 1u << (slot & 31u);
                    *wp = spike ? (*wp | mb) : (*wp & ~mb);
                    L.V[j] = vn;
                    L.age[j] = age_n;
                    if (obs) {
                        const double c = L.c[j];
                        double acc = L.acc[j] + c;
                        const int64_t f_now = t * a.frame_num / a.frame_den;
                        const int64_t f_next = (t + 1) * a.frame_num / a.frame_den;
                        if (f_next != f_now) {
                            const int64_t first = (f_now * a.frame_den + a.frame_num - 1) / a.frame_num;
                            const int64_t next = ((f_now + 1) * a.frame_den + a.frame_num - 1) / a.frame_num;
                            if (f_now < a.frame_cap)
                                a.frames[f_now * a.n_pad + u] = static_cast<float>(acc / static_cast<double>(next - first));
                            acc = 0.0;
                        }
                        L.acc[j] = acc;
                        L.c[j] = c + p.dt_d * (-c / p.tau_c_d + (spike ? 1.0 : 0.0));
                    }
                }
            }
        }
        __syncthreads();
    }

    // ---- write the state back (global ring in the 256-step layout, summary)
    const int64_t t1 = t0 + a.n_steps;
    for (int q = q_begin; q < q_end; ++q) {
        const NetMeta nm = a.meta[a.wg_nets[q]];
        const NetLds L = carve(lds, nm, obs);
        for (int base = 0; base < nm.n_nodes; base += blockDim.x) {
            const int j = base + tid;
            const bool valid = j < nm.n_nodes;
            const int64_t u = nm.node_off + (valid ? j : 0);
            const uint32_t age = valid ? L.age[j] : 255u;
            const uint64_t recent = wave_ballot(valid && age <= static_cast<uint32_t>(a.d_sum));
            const uint64_t alive = wave_ballot(valid);
            if (lane == 0 && alive != 0)
                put_bits_shared(reinterpret_cast<uint64_t*>(a.summary), nm.node_off + base + wave * 64, recent, alive);
            if (!valid) continue;
            a.V[u] = L.V[j];
            // the single-launch kernel keeps no second age: 0 sends every
            // per-step delivery of these sources to the history ring
            a.age[u] = static_cast<uint16_t>(age);
            if (obs) {
                a.calcium[u] = L.c[j];
                a.frame_acc[u] = L.acc[j];
            }
            uint32_t* gr = a.ring + u;
            if (nm.words == kRingWords) {
#pragma unroll
                for (int k = 0; k < kRingWords; ++k) gr[k * a.n_pad] = L.ring[j * kRingWords + k];
            } else {
                const uint32_t q32 = static_cast<uint32_t>(t1) & 31u;
                const uint32_t r = L.ring[j];
                const int64_t ihi = ((static_cast<uint32_t>(t1 - 1) & 255u) >> 5) * a.n_pad;
                const int64_t ilo = ((static_cast<uint32_t>(t1 - 32) & 255u) >> 5) * a.n_pad;
                if (q32 == 0) {
                    gr[ihi] = r;
                } else {
                    const uint32_t m = (1u << q32) - 1u;
                    gr[ihi] = (gr[ihi] & ~m) | (r & m);
                    gr[ilo] = (gr[ilo] & m) | (r & ~m);
                }
            }
        }
    }
}

struct ObserveArgs {
    const float* __restrict__ V;
    const uint16_t* __restrict__ age;
    const double* __restrict__ calcium;
    const float* __restrict__ frames;
    const NetParams* __restrict__ params;
    const int32_t* __restrict__ net_id;
    const int32_t* __restrict__ internal_of;   // renumbered networks: internal index of each caller's vertex
    void* out;
    int64_t n_total, n_pad, n_frames;
    int32_t what, multi;
    float gain, offset, gamma;
};

__global__ void __launch_bounds__(256) observe_kernel(ObserveArgs a) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t rows = (a.what == NET_OBS_FRAMES || a.what == NET_OBS_FLUOR) ? a.n_frames : 1;
    if (idx >= rows * a.n_total) return;
    // output element (f, jc) in the caller's numbering; j is where that vertex lives
    const int64_t f = idx / a.n_total, jc = idx - f * a.n_total;
    const int64_t j = a.internal_of ? a.internal_of[jc] : jc;
    const NetParams& p = a.params[a.multi ? a.net_id[j] : 0];
    switch (a.what) {
        case NET_OBS_V:
            static_cast<float*>(a.out)[jc] = a.V[j];
            break;
        case NET_OBS_REF: {
            const int32_t age = a.age[j] & 0xFF;
            static_cast<int32_t*>(a.out)[jc] = (age >= 1 && age <= p.n_ref) ? p.n_ref + 1 - age : 0;
            break;
        }
        case NET_OBS_CALCIUM:
            static_cast<float*>(a.out)[jc] = static_cast<float>(a.calcium[j]);
            break;
        case NET_OBS_FRAMES:
            static_cast<float*>(a.out)[idx] = a.frames[f * a.n_pad + j];
            break;
        case NET_OBS_FLUOR: {
            const uint32_t jl = static_cast<uint32_t>(jc - p.node_off);
            const uint4 r = philox4x32_10(make_uint4(jl, static_cast<uint32_t>(f), static_cast<uint32_t>(f >> 32), 1u),
                                   p.key_lo, p.key_hi);
            const double F = static_cast<double>(a.gain) * a.frames[f * a.n_pad + j] + static_cast<double>(a.offset) +
                             static_cast<double>(a.gamma) * static_cast<double>(gaussian(r.x, r.y));
            static_cast<float*>(a.out)[idx] = static_cast<float>(F);
            break;
        }
        default:
            break;
    }
}

// ---------------------------------------------------------------------------
// Fused step: one workgroup per segment (a 64-aligned vertex range whose
// slots start on a chunk boundary, so the workgroup owns whole rows).  The
// workgroup delivers its chunks into an input array in LDS (two chunks per
// wave iteration, as deliver_kernel), waits for its own waves, then updates
// its vertices.  Other workgroups still read this step's ages and summary as
// sources, so the update writes the next step's copies (age_out, summary);
// the ring is written in place: step t sets only bit t, which no delivery of
// step t reads (delays are >= 1).
// ---------------------------------------------------------------------------
struct StepArgs {
    DeliverArgs d;
    NodeArgs n;
    const int32_t* seg_vertex;
    const int32_t* seg_chunk;
    int32_t queue_off;   // arrival queues start this many floats after the segment inputs' start in LDS
};

// Arrivals found in a chunk are queued in the wave's LDS queue (slot
// indices) instead of being added at once: the row and weight of an arrival
// need loads from memory, and a wave that issued them per chunk would wait
// for each.  The queue is resolved in one pass when full and at the end.
constexpr uint32_t kStepQueue = 128;   // entries per wave
constexpr int kStepPrefetch = kStepMaxSegment / 1024;   // vertices per thread whose state the step loads ahead

// Row and weight of each queued slot, then an exact FP32 add into the
// segment's LDS inputs.  The row of slot p of chunk c is chunk_row0[c] plus
// the row starts among positions 1..p of the chunk (64 bytes of row-start
// bits, bit p of the chunk's 512).
__device__ __forceinline__ void flush_arrivals(const DeliverArgs& a, const uint32_t* q, uint32_t qn, int lane,
                                               float* lds_in, int32_t v0) {
    for (uint32_t i = 0; i < qn; i += 64) {
        const uint32_t k = i + static_cast<uint32_t>(lane);
        if (k < qn) {
            const uint32_t e = q[k];
            const uint32_t c = e >> 9, p = e & 511u;
            const u32x4* rs = reinterpret_cast<const u32x4*>(a.rowstart + static_cast<uint64_t>(c) * 64);
            const u32x4 r0 = rs[0], r1 = rs[1], r2 = rs[2], r3 = rs[3];
            const uint32_t wbits = a.w[e];
            const int32_t row0 = a.chunk_row0[c];
            const uint32_t words[16] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w,
                                        r2.x, r2.y, r2.z, r2.w, r3.x, r3.y, r3.z, r3.w};
            const uint32_t pw = p >> 5, pb = p & 31u;
            int32_t cnt = -static_cast<int32_t>(r0.x & 1u);   // position 0 belongs to row0
#pragma unroll
            for (uint32_t j = 0; j < 16; ++j) {
                const uint32_t m = j < pw ? 0xFFFFFFFFu : (j == pw ? (pb == 31u ? 0xFFFFFFFFu : (2u << pb) - 1u) : 0u);
                cnt += __popc(words[j] & m);
            }
            atomicAdd(lds_in + (row0 + cnt - v0), half_bits_to_float(wbits));
        }
    }
}

__device__ __forceinline__ void deliver_fired_lds(const DeliverArgs& a, int64_t c, int lane, uint32_t fired,
                                                  float* lds_in, int32_t v0) {
    const int64_t e0 = c * kChunkEdges + lane * kEdgesPerLane;
    const uint32_t rs = a.rowstart[c * 64 + lane];
    const int32_t first_row = a.chunk_row0[c];
    u32x4 wq = u32x4{0u, 0u, 0u, 0u};
    if (fired) wq = *reinterpret_cast<const u32x4*>(a.w + e0);
    const uint32_t bits = lane == 0 ? (rs & ~1u) : rs;
    const int32_t row0 = first_row + static_cast<int32_t>(wave_bits_before(bits)) - v0;
    const uint32_t wv[4] = {wq.x, wq.y, wq.z, wq.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if ((fired >> k) & 1u) {
            const int32_t row = row0 + __popc(bits & ((2u << k) - 1u));
            atomicAdd(lds_in + row, half_bits_to_float((wv[k >> 1] >> (16 * (k & 1))) & 0xFFFFu));
        }
    }
}

// One workgroup per segment.  Waves take units of two chunks: unit `wave`
// first, then the next unclaimed one from an LDS counter (claimed one
// iteration ahead), so that waves the hardware serves later do not hold the
// workgroup's barrier.  The next unit's stream loads are issued right after
// this unit's age gathers, so the two latencies overlap (loads complete in
// issue order: the resolution waits for the gathers only).
__global__ void __launch_bounds__(1024) step_kernel(StepArgs s) {
    apply_device_step(s.n);
    // the summary at a fixed LDS address (its reads need no base), the
    // segment's inputs, the arrival queues and the unit counter after it
    __shared__ uint4 lds4[kStepSummaryBytes / 16];
    extern __shared__ float lds_in[];
    const uint32_t* lds_summary = reinterpret_cast<const uint32_t*>(lds4);
    constexpr int kPer = 2;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const int lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int32_t v0 = s.seg_vertex[lb], v1 = s.seg_vertex[lb + 1];
    const int64_t c_begin = s.seg_chunk[lb], c_end = s.seg_chunk[lb + 1];
    const uint32_t t = s.d.t;
    uint32_t* queue = reinterpret_cast<uint32_t*>(lds_in + s.queue_off) + wave * kStepQueue;
    uint32_t* unit_counter = reinterpret_cast<uint32_t*>(lds_in + s.queue_off) + nwaves * kStepQueue;
    // Start-up: the summary's loads first, then the first chunks, then the
    // vertex state, so that only the summary is waited for before the
    // barrier (which waits for LDS, not for global loads).  Every thread
    // stages 8 x 16 B of the summary in registers; the LDS array has room
    // for the largest summary, so the copy needs no branch (words past a
    // smaller summary are never read).
    const u32x4* g = reinterpret_cast<const u32x4*>(s.d.summary);
    constexpr int kSumPer = kStepSummaryBytes / 16 / 1024;
    u32x4 sreg[kSumPer];
#pragma unroll
    for (int i = 0; i < kSumPer; ++i) {
        const int idx = i * 1024 + threadIdx.x;
        sreg[i] = g[idx < s.d.summary_vec4 ? idx : s.d.summary_vec4 - 1];
    }
    __builtin_amdgcn_sched_barrier(0);   // issued first: waits count loads in issue order
    int64_t c = c_begin + static_cast<int64_t>(wave) * kPer;
    // a segment is a whole number of chunk pairs starting on an even chunk;
    // units beyond it reload its last pair and are skipped below
    NarrowChunk cur[kPer];
    load_narrow_pair(cur, s.d, c < c_end ? c : c_end - kPer, lane);
    __builtin_amdgcn_sched_barrier(0);
    // the state of this workgroup's vertices (segments hold at most
    // kStepPrefetch * 1024) arrives while the edges stream; issued after the
    // first chunks, which are then not kept waiting for it
    VertexState pre[kStepPrefetch];
#pragma unroll
    for (int i = 0; i < kStepPrefetch; ++i)
        pre[i] = load_vertex_state(s.n, v0 + static_cast<int64_t>(i) * 1024 + threadIdx.x, v1);
#pragma unroll
    for (int i = 0; i < kSumPer; ++i) reinterpret_cast<u32x4*>(lds4)[i * 1024 + threadIdx.x] = sreg[i];
    for (int i = threadIdx.x; i < v1 - v0; i += blockDim.x) lds_in[i] = 0.0f;
    if (threadIdx.x == 0) *unit_counter = static_cast<uint32_t>(nwaves);
    __syncthreads();

    uint32_t qn = 0;   // wave-uniform
    while (c < c_end) {
        uint32_t claim = 0;
        if (lane == 0) claim = atomicAdd(unit_counter, 1u);
        uint32_t aw[kPer][8];
#pragma unroll
        for (int u = 0; u < kPer; ++u) gather_chunk<true>(cur[u], s.d, lds_summary, 0u, aw[u]);
        // the next unit's stream loads go out behind this unit's gathers (past
        // the range they re-read this unit's chunks, which L2 still holds)
        const int64_t cn = c_begin + static_cast<int64_t>(__builtin_amdgcn_readfirstlane(claim)) * kPer;
        NarrowChunk nxt[kPer];
        load_narrow_pair(nxt, s.d, cn < c_end ? cn : c, lane);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            if (c + u < c_end && chunk_may_fire(cur[u], aw[u])) {
                const uint32_t fired = fired_bits(cur[u], s.d, t, aw[u]);
                uint32_t total;
                const uint32_t before = wave_bits_before_total(fired, &total);
                if (total > kStepQueue) {
                    deliver_fired_lds(s.d, c + u, lane, fired, lds_in, v0);
                } else if (total > 0) {
                    if (qn + total > kStepQueue) {
                        flush_arrivals(s.d, queue, qn, lane, lds_in, v0);
                        qn = 0;
                    }
                    uint32_t at = qn + before;
                    const uint32_t e0 = static_cast<uint32_t>(c + u) * kChunkEdges + static_cast<uint32_t>(lane) * kEdgesPerLane;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        if ((fired >> k) & 1u) queue[at++] = e0 + static_cast<uint32_t>(k);
                    }
                    qn += total;
                }
            }
        }
        c = cn;
#pragma unroll
        for (int u = 0; u < kPer; ++u) cur[u] = nxt[u];
    }
    if (qn) flush_arrivals(s.d, queue, qn, lane, lds_in, v0);
    // the random draws need no input: a wave computes them while the
    // workgroup's other waves finish their deliveries
#pragma unroll
    for (int i = 0; i < kStepPrefetch; ++i) {
        const int64_t base = v0 + static_cast<int64_t>(i) * 1024;
        if (base < v1) vertex_random<false>(s.n, base + threadIdx.x, v1, pre[i]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kStepPrefetch; ++i) {
        const int64_t base = v0 + static_cast<int64_t>(i) * 1024;
        if (base < v1) {
            const int64_t j = base + threadIdx.x;
            const float in = j < v1 ? lds_in[j - v0] : 0.0f;
            vertex_update<false>(s.n, j, v1, v1, in, false, pre[i]);
        }
    }
}

}  // namespace

hipError_t configure_deliver(DeviceGraph& g, const net_build_opts* opts, LaunchConfig& lc) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int n_cu = 0, lds_max = 0;
    if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess) return e;
    const int flags = opts ? opts->flags : 0;
    g.sum_shift = (flags & NET_BUILD_SUMMARY_HALF) ? 1 : 0;
    const size_t summary_bytes = static_cast<size_t>(g.n_pad / 8) >> g.sum_shift;
    const bool want_lds = !(flags & NET_BUILD_NO_LDS_SUMMARY);
    lc.lds_summary = want_lds && summary_bytes <= static_cast<size_t>(lds_max);
    lc.stream_weights = (flags & NET_BUILD_DELIVER_STREAM_WEIGHTS) != 0;
    lc.nontemporal = (flags & NET_BUILD_DELIVER_NONTEMPORAL) != 0;
    lc.mode = (flags & NET_BUILD_DELIVER_UNROLL2) ? 1 : ((flags & NET_BUILD_DELIVER_PIPELINE) ? 2 : 0);
    if ((flags & NET_BUILD_DELIVER_COMPACT) && g.n_pad <= (int64_t(1) << 24)) lc.mode = 3;
    if ((flags & NET_BUILD_DELIVER_PACKED) && lc.mode != 3) {
        lc.mode = g.sd ? 4 : 1;
        if (g.sd) lc.stream_weights = lc.nontemporal = false;   // the packed loop streams neither
    }
    // Workgroups per CU limited by the summary (and, compacted, the per-wave
    // candidate stages) held in LDS (160 KiB per CU).
    int threads = 1024, per_cu = 8;
    if (opts && opts->block_threads) threads = opts->block_threads;
    const size_t stage_per_wave = static_cast<size_t>(kChunkEdges) * sizeof(uint32_t);
    auto lds_need = [&](int thr) {
        return (lc.lds_summary ? summary_bytes : 0) +
               (lc.mode == 3 ? static_cast<size_t>(thr / 64) * stage_per_wave : 0);
    };
    if (lc.mode == 3 && lds_need(threads) > static_cast<size_t>(lds_max)) lc.mode = 1;   // stages do not fit
    lc.lds_bytes = lds_need(threads);
    if (lc.lds_bytes > 0) {
        per_cu = static_cast<int>((160 * 1024) / lc.lds_bytes);
        per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
    }
    if (!(opts && opts->block_threads)) {
        // up to 32 waves per CU: 1024 threads for one or two workgroups per CU
        threads = per_cu <= 2 ? 1024 : (per_cu <= 4 ? 512 : 256);
        lc.lds_bytes = lds_need(threads);
    }
    if (opts && opts->blocks_per_cu) per_cu = opts->blocks_per_cu;
    if (lc.lds_bytes > 0) {
        const void* fns[] = {
#define GEONET_DELIVER_FN(L, W, N, M) reinterpret_cast<const void*>(&deliver_kernel<L, W, N, M>),
#define GEONET_DELIVER_FNS(L, M) GEONET_DELIVER_FN(L, false, false, M) GEONET_DELIVER_FN(L, false, true, M) \
                                 GEONET_DELIVER_FN(L, true, false, M) GEONET_DELIVER_FN(L, true, true, M)
            GEONET_DELIVER_FNS(true, 0) GEONET_DELIVER_FNS(true, 1) GEONET_DELIVER_FNS(true, 2)
            GEONET_DELIVER_FNS(true, 3) GEONET_DELIVER_FNS(false, 3)
            GEONET_DELIVER_FN(true, false, false, 4)
#undef GEONET_DELIVER_FNS
#undef GEONET_DELIVER_FN
        };
        for (const void* f : fns) {
            e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lc.lds_bytes));
            if (e != hipSuccess) return e;
        }
    }
    int64_t blocks = static_cast<int64_t>(n_cu) * per_cu;
    const int64_t waves_needed = g.n_chunks;                 // at least one chunk per wave
    const int64_t max_blocks = (waves_needed + (threads / 64) - 1) / (threads / 64);
    if (blocks > max_blocks) blocks = max_blocks < 1 ? 1 : max_blocks;
    if (blocks >= 8) blocks = blocks / 8 * 8;
    lc.deliver_blocks = static_cast<int>(blocks);
    lc.deliver_threads = threads;
    // Fused step: one 1024-thread workgroup per segment, the summary and the
    // segment's inputs in LDS.
    lc.fused = false;
    // (queued arrivals are 32-bit slot indices: at most 2^23 chunks)
    if ((flags & NET_BUILD_FUSED_STEP) && g.seg_vertex && g.s_lo && g.n_seg > 0 && lc.lds_summary && g.sum_shift == 0 &&
        summary_bytes <= static_cast<size_t>(kStepSummaryBytes) && g.n_chunks <= (int64_t(1) << 23)) {
        const size_t in_bytes = (static_cast<size_t>(g.seg_max) * sizeof(float) + 15) / 16 * 16;
        const size_t need = in_bytes + kStepQueueBytes + 16;   // beyond the summary: inputs, queues, counter
        lc.queue_off = static_cast<int32_t>(in_bytes / sizeof(float));
        if (need + kStepSummaryBytes <= static_cast<size_t>(lds_max) && g.seg_max <= kStepMaxSegment) {
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&step_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    static_cast<int>(need));
            if (e != hipSuccess) return e;
            lc.fused = true;
            lc.mode = 1;
            lc.stream_weights = false;
            lc.nontemporal = false;
            lc.lds_bytes = need;
            lc.deliver_threads = 1024;
            lc.deliver_blocks = g.n_seg;
        }
    }
    return hipSuccess;
}

static DeliverArgs deliver_args(const DeviceGraph& g, const LaunchConfig& lc, int64_t t) {
    DeliverArgs a;
    a.src = g.src;
    a.w = g.w;
    a.d = g.d;
    a.sd = g.sd;
    a.s_lo = g.s_lo;
    a.dl_pair = g.dl_pair;
    a.hi_pair = g.hi_pair;
    a.rowstart = g.rowstart;
    a.chunk_row0 = g.chunk_row0;
    a.summary = g.summary;
    a.ring = g.ring;
    a.ages = g.age;
    a.I = g.I;
    a.n_chunks = g.n_chunks;
    a.summary_vec4 = static_cast<int32_t>((g.n_pad >> g.sum_shift) / 128);
    a.sum_shift = static_cast<uint32_t>(g.sum_shift);
    a.stage_vec4 = lc.lds_summary ? a.summary_vec4 : 0;
    a.t = static_cast<uint32_t>(t);
    a.n_pad = static_cast<uint32_t>(g.n_pad);
    a.window = static_cast<uint32_t>(g.d_sum);
    a.age_sentinel = static_cast<uint32_t>(g.n_pad);
    return a;
}

hipError_t launch_deliver(const DeviceGraph& g, const LaunchConfig& lc, int64_t t, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1) {
    const DeliverArgs a = deliver_args(g, lc, t);
    const dim3 grid(lc.deliver_blocks), block(lc.deliver_threads);
    const int v = lc.mode * 8 + (lc.lds_summary ? 4 : 0) + (lc.stream_weights ? 2 : 0) + (lc.nontemporal ? 1 : 0);
    const size_t shared = lc.lds_bytes;
    switch (v) {
#define GEONET_DELIVER_CASE(M, L, W, N)                                                            \
    case M * 8 + (L ? 4 : 0) + (W ? 2 : 0) + (N ? 1 : 0):                                          \
        hipExtLaunchKernelGGL((deliver_kernel<L, W, N, M>), grid, block, shared, s, ev0, ev1, 0,          \
                              a);                                                                  \
        break;
#define GEONET_DELIVER_CASES(M)              \
    GEONET_DELIVER_CASE(M, false, false, false) \
    GEONET_DELIVER_CASE(M, false, false, true)  \
    GEONET_DELIVER_CASE(M, false, true, false)  \
    GEONET_DELIVER_CASE(M, false, true, true)   \
    GEONET_DELIVER_CASE(M, true, false, false)  \
    GEONET_DELIVER_CASE(M, true, false, true)   \
    GEONET_DELIVER_CASE(M, true, true, false)   \
    GEONET_DELIVER_CASE(M, true, true, true)
        GEONET_DELIVER_CASES(0)
        GEONET_DELIVER_CASES(1)
        GEONET_DELIVER_CASES(2)
        GEONET_DELIVER_CASES(3)
        GEONET_DELIVER_CASE(4, false, false, false)
        GEONET_DELIVER_CASE(4, true, false, false)
#undef GEONET_DELIVER_CASES
#undef GEONET_DELIVER_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static NodeArgs node_args(const DeviceGraph& g, int64_t t, int64_t rec_row, const net_record* rec,
                          int32_t frame_flush, int64_t frame_index, int32_t frame_steps) {
    NodeArgs a;
    a.V = g.V;
    a.age = g.age;
    a.age_out = g.age;
    a.I = g.I;
    a.ring = g.ring;
    a.summary = g.summary;
    a.params = g.params;
    a.net_id = g.net_id;
    a.drive_thr = g.drive_thr;
    a.i_ext = g.i_ext;
    a.calcium = g.calcium;
    a.frame_acc = g.frame_acc;
    a.frames = g.frames;
    a.rec_raster = rec ? rec->raster : nullptr;
    a.rec_v = rec ? rec->v : nullptr;
    a.rec_input = rec ? rec->input : nullptr;
    a.n_total = g.n_total;
    a.n_pad = g.n_pad;
    a.rec_row = rec_row;
    a.raster_words = (g.n_total + 63) / 64;
    a.frame_index = frame_index;
    a.t_lo = static_cast<uint32_t>(t);
    a.t_hi = static_cast<uint32_t>(static_cast<uint64_t>(t) >> 32);
    a.d_sum = g.d_sum;
    a.sum_shift = g.sum_shift;
    a.frame_flush = frame_flush;
    a.frame_steps = frame_steps;
    a.frame_cap = g.frame_cap;
    a.p0 = g.p0;
    a.Vd = g.Vd;
    a.Wd = g.Wd;
    a.psc_r = g.psc_r;
    a.psc_p = g.psc_p;
    a.hh_m = g.hh_m;
    a.hh_n = g.hh_n;
    a.hh_h = g.hh_h;
    a.hh_vprev = g.hh_vprev;
    a.spk_hist = g.spk_hist;
    a.spk_cnt = g.spk_cnt;
    a.out_off = nullptr;
    a.out_edge = nullptr;
    a.push_ring = nullptr;
    a.push_mask = 0;
    if (g.in_ring) {
        // push delivery: the input is the ring slot of step t (read and cleared
        // by the update), and the update pushes its own spikes
        a.I = g.in_ring + static_cast<int64_t>(static_cast<uint64_t>(t) & g.in_ring_mask) * g.n_pad;
        a.out_off = g.out_off;
        a.out_edge = g.out_edge;
        a.push_ring = g.in_ring;
        a.push_mask = g.in_ring_mask;
    }
    a.caller_of = g.caller_of;
    a.t_dev = g.t_dev;
    a.t_off = static_cast<uint32_t>(t);
    a.frame_num = g.t_dev ? g.frame_num : 0;
    a.frame_den = g.frame_den;
    return a;
}

hipError_t launch_node_update(const DeviceGraph& g, int64_t t, int64_t rec_row, const net_record* rec,
                              int32_t frame_flush, int64_t frame_index, int32_t frame_steps, hipStream_t s,
                              hipEvent_t ev0, hipEvent_t ev1) {
    const NodeArgs a = node_args(g, t, rec_row, rec, frame_flush, frame_index, frame_steps);
    const int threads = 256;
    const int64_t blocks = g.n_pad / threads + ((g.n_pad % threads) ? 1 : 0);
    if (g.Vd || g.spk_hist) {
        if (g.n_nets > 1)
            hipExtLaunchKernelGGL((node_update_kernel<true, true>), dim3(blocks), dim3(threads), 0, s, ev0, ev1, 0, a);
        else
            hipExtLaunchKernelGGL((node_update_kernel<false, true>), dim3(blocks), dim3(threads), 0, s, ev0, ev1, 0, a);
    } else if (g.n_nets > 1) {
        hipExtLaunchKernelGGL((node_update_kernel<true, false>), dim3(blocks), dim3(threads), 0, s, ev0, ev1, 0, a);
    } else {
        hipExtLaunchKernelGGL((node_update_kernel<false, false>), dim3(blocks), dim3(threads), 0, s, ev0, ev1, 0, a);
    }
    return hipGetLastError();
}

namespace {

struct PlasticArgs {
    const int32_t* __restrict__ src;
    const uint8_t* __restrict__ d;
    int32_t* __restrict__ wq;
    const int32_t* __restrict__ slot_orig;
    const int32_t* __restrict__ row_first;
    const uint32_t* __restrict__ ring;
    const uint32_t* __restrict__ summary;   // bit i: vertex i fired within the last `window` steps
    const uint16_t* __restrict__ ages;      // steps since the last two spikes (a1 | a2 << 8, 255 saturates)
    const float* __restrict__ V;
    const int32_t* __restrict__ spk_hist;
    const int32_t* __restrict__ spk_cnt;
    float* __restrict__ I;
    int64_t n_total, n_pad, t;
    uint32_t window;
    float v_th;
    double dt, alpha, beta;
};

// s_k(u): time since vertex k's last spike before step u (0 for u <= 0,
// u*dt before any spike), from its last kStdpHist spike steps.
__device__ __forceinline__ double since_last(const PlasticArgs& a, int64_t k, int64_t u) {
    if (u <= 0) return 0.0;
    const int32_t cnt = a.spk_cnt[k];
    const int32_t have = cnt < kStdpHist ? cnt : kStdpHist;
    int64_t best = -1;
    for (int q = 0; q < have; ++q) {
        const int64_t ts = a.spk_hist[k * kStdpHist + q];
        if (ts < u && ts > best) best = ts;
    }
    return best < 0 ? static_cast<double>(u) * a.dt : static_cast<double>(u - best - 1) * a.dt;
}

// One wave per target row j: the delivered sum of step t with the weights as
// they are (integers, so the order of additions cannot change it), then the
// plasticity update of every edge of the row whose spike arrives now or
// whose target fires now: w += round((dt alpha sign(q) exp(-beta |q|)) / 2^-20).
// An edge's arrival is found as in the delivery kernels: a source that did
// not fire within the summary window (one bit per vertex, a small array that
// stays in the caches) cannot arrive over an edge no longer than the window;
// the others gather the source's two spike ages (d == a1 fires; d >= a2 asks
// the history ring).  A weight is read only for an edge that is delivered or
// updated.
__global__ void __launch_bounds__(256) plastic_deliver_kernel(PlasticArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (j >= a.n_total) return;
    const bool post = a.V[j] >= a.v_th;
    const int64_t first = a.row_first[j], last = a.row_first[j + 1];
    int64_t acc = 0;
    // an edge whose ages were gathered (ag = 0xFFFF for non-candidates)
    auto edge = [&](int64_t e, int32_t i, uint32_t dl, uint32_t ag) {
        bool arrive = false;
        if (a.t - static_cast<int64_t>(dl) >= 0) {
            const uint32_t a1 = ag & 0xFFu, a2 = ag >> 8;
            if (dl >= a2) {
                // an older spike may sit at t - d (non-candidates never get here:
                // their delay is at most the window, below 255)
                const uint32_t slot = static_cast<uint32_t>(a.t - dl) & 255u;
                arrive = ((a.ring[(slot >> 5) * a.n_pad + i] >> (slot & 31u)) & 1u) != 0u;
            } else {
                arrive = dl == a1;
            }
        }
        if (arrive || post) {
            const int32_t w = a.wq[e];
            if (arrive) acc += w;
            if (a.slot_orig[e] >= 0) {
                const double q = since_last(a, i, a.t - dl) - since_last(a, j, a.t);
                const double sg = q > 0.0 ? 1.0 : (q < 0.0 ? -1.0 : 0.0);
                const double dw = a.dt * a.alpha * sg * exp(-a.beta * fabs(q));
                a.wq[e] = w + static_cast<int32_t>(rint(dw * 1048576.0));
            }
        }
    };
    // two edges per lane per pass, their loads issued together
    for (int64_t e = first + lane; e < last; e += 128) {
        const int64_t e2 = e + 64;
        const bool two = e2 < last;
        const int32_t i0 = a.src[e], i1 = a.src[two ? e2 : e];
        const uint32_t d0 = a.d[e], d1 = a.d[two ? e2 : e];
        const uint32_t sw0 = a.summary[i0 >> 5], sw1 = a.summary[i1 >> 5];
        const bool c0 = ((sw0 >> (i0 & 31)) & 1u) != 0u || d0 > a.window;
        const bool c1 = two && (((sw1 >> (i1 & 31)) & 1u) != 0u || d1 > a.window);
        const uint32_t ag0 = c0 ? static_cast<uint32_t>(a.ages[i0]) : 0xFFFFu;
        const uint32_t ag1 = c1 ? static_cast<uint32_t>(a.ages[i1]) : 0xFFFFu;
        edge(e, i0, d0, ag0);
        if (two) edge(e2, i1, d1, ag1);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) a.I[j] = static_cast<float>(static_cast<double>(acc) * (1.0 / 1048576.0));
}

__global__ void __launch_bounds__(256) weights_out_kernel(const int32_t* wq, const int32_t* slot_orig, int64_t slots,
                                                          float* out) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= slots) return;
    const int32_t o = slot_orig[s];
    if (o >= 0) out[o] = static_cast<float>(static_cast<double>(wq[s]) * (1.0 / 1048576.0));
}

}  // namespace

namespace {

// dst[r][caller_of[k]] = src[r][k] for 4-byte values
__global__ void __launch_bounds__(256) to_caller_rows_kernel(const uint32_t* src, uint32_t* dst,
                                                             const int32_t* caller_of, int64_t n, int64_t rows) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n * rows) return;
    const int64_t r = i / n, k = i - r * n;
    dst[r * n + caller_of[k]] = src[i];
}

// raster word (r, w) in the caller's numbering: bit b is the internal
// vertex internal_of[64 w + b]'s bit
__global__ void __launch_bounds__(256) to_caller_raster_kernel(const uint64_t* src, uint64_t* dst,
                                                               const int32_t* internal_of, int64_t n, int64_t words,
                                                               int64_t rows) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= words * rows) return;
    const int64_t r = i / words, w = i - r * words;
    uint64_t out = 0;
    for (int b = 0; b < 64; ++b) {
        const int64_t jc = w * 64 + b;
        if (jc >= n) break;
        const int64_t k = internal_of[jc];
        out |= ((src[r * words + (k >> 6)] >> (k & 63)) & 1ull) << b;
    }
    dst[i] = out;
}

}  // namespace

hipError_t launch_records_to_caller(const DeviceGraph& g, const net_record* rec, int64_t rows, void* tmp,
                                    hipStream_t s) {
    const int64_t n = g.n_total, words = (n + 63) / 64;
    if (rec->raster) {
        hipError_t e = hipMemcpyAsync(tmp, rec->raster, static_cast<size_t>(rows * words) * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(to_caller_raster_kernel, dim3(static_cast<unsigned>((rows * words + 255) / 256)), dim3(256), 0,
                           s, static_cast<const uint64_t*>(tmp), rec->raster, g.internal_of, n, words, rows);
    }
    float* recs[2] = {rec->v, rec->input};
    for (float* r : recs) {
        if (!r) continue;
        hipError_t e = hipMemcpyAsync(tmp, r, static_cast<size_t>(rows * n) * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(to_caller_rows_kernel, dim3(static_cast<unsigned>((rows * n + 255) / 256)), dim3(256), 0, s,
                           static_cast<const uint32_t*>(tmp), reinterpret_cast<uint32_t*>(r), g.caller_of, n, rows);
    }
    return hipGetLastError();
}

hipError_t launch_plastic_deliver(const DeviceGraph& g, int64_t t, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    PlasticArgs a;
    a.src = g.src;
    a.d = g.d;
    a.wq = g.wq;
    a.slot_orig = g.slot_orig;
    a.row_first = g.row_first;
    a.ring = g.ring;
    a.summary = g.summary;
    a.ages = g.age;
    a.V = g.V;
    a.spk_hist = g.spk_hist;
    a.spk_cnt = g.spk_cnt;
    a.I = g.I;
    a.n_total = g.n_total;
    a.n_pad = g.n_pad;
    a.t = t;
    a.window = static_cast<uint32_t>(g.d_sum);
    a.v_th = g.p0.v_th;
    a.dt = g.p0.dt_d;
    a.alpha = g.stdp_alpha;
    a.beta = g.stdp_beta;
    const int64_t threads = g.n_total * 64;
    hipExtLaunchKernelGGL(plastic_deliver_kernel, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0, s,
                          ev0, ev1, 0, a);
    return hipGetLastError();
}

hipError_t launch_weights_out(const DeviceGraph& g, float* out, hipStream_t s) {
    hipLaunchKernelGGL(weights_out_kernel, dim3(static_cast<unsigned>((g.e_slots + 255) / 256)), dim3(256), 0, s, g.wq,
                       g.slot_orig, g.e_slots, out);
    return hipGetLastError();
}

hipError_t launch_observe(const DeviceGraph& g, int32_t what, const net_fluor_params* fp, void* out, int64_t n_frames,
                          hipStream_t s) {
    ObserveArgs a;
    a.V = g.V;
    a.age = g.age;
    a.calcium = g.calcium;
    a.frames = g.frames;
    a.params = g.params;
    a.net_id = g.net_id;
    a.internal_of = g.internal_of;
    a.out = out;
    a.n_total = g.n_total;
    a.n_pad = g.n_pad;
    a.n_frames = n_frames;
    a.what = what;
    a.multi = g.n_nets > 1 ? 1 : 0;
    a.gain = fp ? fp->gain : 1.0f;
    a.offset = fp ? fp->offset : 0.0f;
    a.gamma = fp ? fp->gamma : 0.0f;
    const int64_t rows = (what == NET_OBS_FRAMES || what == NET_OBS_FLUOR) ? n_frames : 1;
    const int64_t total = rows * g.n_total;
    if (total == 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(observe_kernel, dim3((total + threads - 1) / threads), dim3(threads), 0, s, a);
    return hipGetLastError();
}


hipError_t launch_ensemble(const DeviceGraph& g, const EnsemblePlan& plan, int64_t t0, int32_t n_steps,
                           const net_record* rec, int32_t frame_num, int32_t frame_den, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
    EnsembleArgs a;
    a.src = g.src;
    a.w = g.w;
    a.d = g.d;
    a.rowstart = g.rowstart;
    a.chunk_row0 = g.chunk_row0;
    a.meta = plan.meta;
    a.wg_nets = plan.wg_nets;
    a.wg_off = plan.wg_off;
    a.params = g.params;
    a.drive_thr = g.drive_thr;
    a.i_ext = g.i_ext;
    a.V = g.V;
    a.age = g.age;
    a.ring = g.ring;
    a.summary = g.summary;
    a.calcium = (g.calcium && frame_num > 0) ? g.calcium : nullptr;
    a.frame_acc = g.frame_acc;
    a.frames = g.frames;
    a.rec_raster = rec ? rec->raster : nullptr;
    a.rec_v = rec ? rec->v : nullptr;
    a.rec_input = rec ? rec->input : nullptr;
    a.Vd = g.Vd;
    a.Wd = g.Wd;
    a.psc_r = g.psc_r;
    a.psc_p = g.psc_p;
    a.hh_m = g.hh_m;
    a.hh_n = g.hh_n;
    a.hh_h = g.hh_h;
    a.hh_vprev = g.hh_vprev;
    a.caller_of = g.caller_of;
    a.t_dev = g.t_dev;
    a.t0 = t0;
    a.n_total = g.n_total;
    a.n_pad = g.n_pad;
    a.raster_words = (g.n_total + 63) / 64;
    a.n_steps = n_steps;
    a.frame_cap = g.frame_cap;
    a.frame_num = frame_num > 0 ? frame_num : 1;
    a.frame_den = frame_den > 0 ? frame_den : 1;
    a.d_sum = g.d_sum;
    a.ls = g.ens_ls;
    a.sbits = g.ens_sbits;
    a.push_off = g.push_off;
    a.push_edge = g.push_edge;
    a.drv = g.ens_drv;
    const int m = g.hh_m ? 2 : (g.Vd ? 1 : 0);
    const int k = plan.held ? kEnsHeld : (g.ens_sbits < 16 ? kEnsPacked : kEnsLocal);
    if (k != kEnsHeld && !g.ens_ls) return hipErrorInvalidValue;
    const dim3 grid(plan.blocks), block(plan.threads);
#define GEONET_ENS(M, K) hipExtLaunchKernelGGL((ensemble_kernel<M, K>), grid, block, plan.lds_bytes, s, ev0, ev1, 0, a)
    if (k == kEnsHeld) {
        if (m == 2) GEONET_ENS(2, kEnsHeld);
        else if (m == 1) GEONET_ENS(1, kEnsHeld);
        else GEONET_ENS(0, kEnsHeld);
    } else if (k == kEnsLocal) {
        if (m == 2) GEONET_ENS(2, kEnsLocal);
        else if (m == 1) GEONET_ENS(1, kEnsLocal);
        else GEONET_ENS(0, kEnsLocal);
    } else {
        if (m == 2) GEONET_ENS(2, kEnsPacked);
        else if (m == 1) GEONET_ENS(1, kEnsPacked);
        else GEONET_ENS(0, kEnsPacked);
    }
#undef GEONET_ENS
    return hipGetLastError();
}

hipError_t enable_ensemble_lds(size_t bytes) {
    const void* fns[] = {reinterpret_cast<const void*>(&ensemble_kernel<0, kEnsHeld>),
                         reinterpret_cast<const void*>(&ensemble_kernel<1, kEnsHeld>),
                         reinterpret_cast<const void*>(&ensemble_kernel<2, kEnsHeld>),
                         reinterpret_cast<const void*>(&ensemble_kernel<0, kEnsLocal>),
                         reinterpret_cast<const void*>(&ensemble_kernel<1, kEnsLocal>),
                         reinterpret_cast<const void*>(&ensemble_kernel<2, kEnsLocal>),
                         reinterpret_cast<const void*>(&ensemble_kernel<0, kEnsPacked>),
                         reinterpret_cast<const void*>(&ensemble_kernel<1, kEnsPacked>),
                         reinterpret_cast<const void*>(&ensemble_kernel<2, kEnsPacked>)};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
__global__ void set_counter_kernel(uint64_t* t_dev, uint64_t t) { *t_dev = t; }
__global__ void advance_counter_kernel(uint64_t* t_dev, uint64_t k) { *t_dev += k; }
}  // namespace

hipError_t launch_set_counter(uint64_t* t_dev, uint64_t t, hipStream_t s) {
    hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(1), 0, s, t_dev, t);
    return hipGetLastError();
}

hipError_t launch_advance_counter(uint64_t* t_dev, uint64_t k, hipStream_t s) {
    hipLaunchKernelGGL(advance_counter_kernel, dim3(1), dim3(1), 0, s, t_dev, k);
    return hipGetLastError();
}

hipError_t launch_step(const DeviceGraph& g, const LaunchConfig& lc, int64_t t, int64_t rec_row, const net_record* rec,
                       int32_t frame_flush, int64_t frame_index, int32_t frame_steps, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1) {
    if (!lc.fused || !g.seg_vertex || !g.age_alt || !g.summary_alt) return hipErrorInvalidValue;
    StepArgs a;
    a.d = deliver_args(g, lc, t);
    a.n = node_args(g, t, rec_row, rec, frame_flush, frame_index, frame_steps);
    a.n.age_out = g.age_alt;
    a.n.summary = g.summary_alt;
    a.n.I = nullptr;
    a.seg_vertex = g.seg_vertex;
    a.seg_chunk = g.seg_chunk;
    a.queue_off = lc.queue_off;
    hipExtLaunchKernelGGL(step_kernel, dim3(g.n_seg), dim3(lc.deliver_threads), lc.lds_bytes, s, ev0, ev1, 0, a);
    return hipGetLastError();
}

}  // namespace geonet
