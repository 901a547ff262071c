// Internal declarations of the geonet library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/geonet.h"

namespace geonet {

// Edges are processed in chunks of 512 slots: 64 lanes x 8 consecutive edges.
constexpr int kEdgesPerLane = 8;
constexpr int kChunkEdges = 64 * kEdgesPerLane;
constexpr int kRingSlots = 256;       // spike history per vertex, bits
constexpr int kRingWords = kRingSlots / 32;
constexpr int kNodeAlign = 256;       // vertex arrays padded to this many entries (one update workgroup)
constexpr uint8_t kAgeNever = 255;    // "no spike within the last 254 steps"
// The ages arrays hold this many entries past n_pad; entry n_pad stays
// (kAgeNever, kAgeNever) and is what delivery gathers for non-candidate edges.
constexpr int kAgePad = 64;
// How the single-launch ensemble kernel reads its chunks: held in registers
// for all steps, or streamed each step as 2-byte sources within the network
// plus the delay bytes, or as 2-byte slots that pack both.
constexpr int kEnsHeld = 0, kEnsLocal = 1, kEnsPacked = 2;
// The fused step kernel keeps the recent-spike summary in a fixed 128 KiB of
// LDS (one bit per vertex, up to 2^20 vertices) and its segment's inputs
// after it.
constexpr int kStepSummaryBytes = 128 * 1024;
// ... and per wave (16 per workgroup) a queue of 128 arrival slot indices,
// then a 16-byte work counter.
constexpr int kStepQueueBytes = 16 * 128 * 4;
// Vertices per fused-step segment at most (6 per thread of its workgroup).
constexpr int kStepMaxSegment = 6 * 1024;
// Spike times kept per vertex for plasticity: with at least 17 held steps
// after a spike, 16 spikes span more than the 255-step delay window.
constexpr int kStdpHist = 16;
constexpr int kStdpMinRef = 17;

// Every device allocation of the library (network handles, MLP handles and
// the scratch of the estimation calls) goes through the allocator installed
// by net_set_allocator, or hipMalloc/hipFree when none is installed.  A
// handle keeps the allocator that was current when it was created.
struct DevAllocator {
    void* (*alloc)(size_t, void*, void*) = nullptr;
    void (*release)(void*, void*, void*) = nullptr;
    void* ctx = nullptr;
    // 256-byte multiple (at least 256 bytes); null on failure
    void* get(size_t bytes, hipStream_t s) const;
    void put(void* p, hipStream_t s) const;
};
DevAllocator current_allocator();

// Per-network constants used by the vertex kernels.
struct NetParams {
    float decay;        // dt / tau
    float v_rest, v_reset, v_th;
    float sigma, drive_amp;
    int32_t n_ref;
    uint32_t key_lo, key_hi;
    int32_t node_off;   // first vertex of the network in the ensemble numbering
    double dt_d, tau_c_d;   // calcium transition in double precision
    // Izhikevich vertex (model 1; FP64 state): V_peak = v_th, c = v_reset
    int32_t model, psc;     // NET_MODEL_*, NET_PSC_*
    double iz_inv_c, iz_k, iz_vr, iz_vt, iz_a, iz_b, iz_d, psc_a;   // iz_inv_c = 1 / C
    // Hodgkin-Huxley vertex (model 2; FP64 state): hh_inv_c = 1 / C
    double hh_inv_c, hh_gna, hh_gk, hh_gl, hh_ena, hh_ek, hh_el;
};

// Per-network description used by the ensemble kernel.
struct NetMeta {
    int32_t node_off, n_nodes;
    int32_t chunk_begin, chunk_end;
    int32_t words;      // history words per vertex in LDS: 1 (32 steps) or 8 (256 steps)
    int32_t lds_off;    // byte offset of the network's state in its workgroup's LDS
    int32_t maxd;       // largest delay of the network
    // spike log (networks with words == 1 and out-edge tables, else log_cap = 0):
    // byte offset in LDS of 32 counts and 32 x log_cap vertex ids (bucket
    // t mod 32 lists the vertices that fired at step t), and the first entry
    // of the network's out-edge offsets
    int32_t log_off, log_cap, po_base;
    // driven vertices of the network in the ensemble's drive list [drv_begin, drv_end)
    int32_t drv_begin, drv_end;
};

// Spike-log capacity per step bucket of a network of n vertices, and its LDS bytes.
inline int ens_log_cap(int64_t n) {
    const int64_t c = (n / 16 + 7) / 8 * 8;
    return static_cast<int>(c < 16 ? 16 : (c > 64 ? 64 : c));
}
inline size_t ens_log_bytes(int cap) { return cap > 0 ? 128 + 64 * static_cast<size_t>(cap) : 0; }

// Host-side result of graph construction (before upload).
struct HostGraph {
    int64_t n_total = 0, n_pad = 0;
    int64_t n_edges = 0;          // real edges
    int64_t e_slots = 0;          // stored slots incl. empty-row placeholders and padding
    int64_t n_chunks = 0;
    int32_t max_delay = 1;
    int32_t window = 1;           // recent-spike summary window (steps)
    bool exact = true;
    std::vector<int32_t> src;     // [e_slots]
    std::vector<uint16_t> w;      // [e_slots] FP16 bits
    std::vector<uint8_t> d;       // [e_slots]
    std::vector<uint8_t> rowstart;  // [e_slots / 8] bit k of byte b: slot 8b+k opens a row
    std::vector<int32_t> chunk_row0;  // [n_chunks] row of each chunk's first slot
    std::vector<int64_t> node_off;    // [n_nets + 1]
    std::vector<int64_t> net_chunk_begin, net_chunk_end;  // [n_nets] chunk range of each network
    // segments for the fused step (one workgroup each): first vertex (a
    // multiple of 64) and first chunk of segment k at [k]; [n_seg] = end
    std::vector<int32_t> seg_vertex, seg_chunk;
    int32_t seg_max = 0;                                  // most vertices in one segment
    std::vector<int32_t> net_max_delay;                   // [n_nets]
    std::vector<NetParams> params;    // [n_nets]
    // per-vertex arrays [n_pad]
    std::vector<float> v0;
    std::vector<uint32_t> drive_thr;
    std::vector<float> i_ext;
    std::vector<int32_t> net_id;
    bool any_drive = false, any_iext = false;
    bool any_izh = false;             // some network uses the Izhikevich vertex
    std::vector<double> w0;           // [n_pad] initial W (Izhikevich vertices)
    // plastic weights (one network): weight of each slot in units of 2^-20,
    // the caller's index of each slot's edge (-1 for placeholders), and the
    // first slot of every row
    bool plastic = false;
    double stdp_alpha = 0.0, stdp_beta = 0.0;
    std::vector<int32_t> wq, slot_orig, row_first;
    bool any_hh = false;              // some network uses the Hodgkin-Huxley vertex
    std::vector<double> hh_m0, hh_n0, hh_h0;   // [n_pad] gates at their steady state for V(0)
    double dt_ms = 0.0;
    int32_t frame_num = 0, frame_den = 1;
};

// Spatial renumbering (NET_BUILD_REORDER): copies of the descriptors with
// every network's vertices renumbered along a Morton (Z-order) curve of
// their positions; caller_of[k] is the caller's global index of internal
// vertex k and internal_of its inverse.  The store keeps the arrays the
// copies point to.
struct ReorderStore {
    std::vector<std::vector<double>> pos;
    std::vector<std::vector<int32_t>> src, dst;
    std::vector<std::vector<float>> rate, iext, v0, w0;
};
void reorder_descs(const net_desc* in, int32_t n_nets, std::vector<net_desc>& out, ReorderStore& store,
                   std::vector<int32_t>& caller_of, std::vector<int32_t>& internal_of);

// Builds the CSR-by-target edge list and per-vertex arrays.  Returns a
// status and fills `err` on failure.
// seg_count > 0 (one network only): also cut the vertices into at most
// seg_count segments of at most seg_cap vertices, each starting on a
// 64-vertex boundary with its slots starting on a chunk boundary; leaves
// seg_vertex empty if that is not possible.
net_status build_host_graph(const net_desc* descs, int32_t n_nets, HostGraph& g, std::string& err,
                            int32_t seg_count = 0, int32_t seg_cap = 0);

// Device-side handle contents.
struct DeviceGraph {
    int64_t n_total, n_pad, e_slots, n_chunks;
    int32_t n_nets, max_delay, d_sum;   // d_sum: summary window W <= max_delay
    int32_t sum_shift = 0;        // summary bit b covers vertices [b << sum_shift, (b + 1) << sum_shift)
    const int32_t* src;
    const uint16_t* w;
    const uint8_t* d;
    const uint32_t* sd = nullptr;   // packed two-kernel variant: source | delay << 24 per slot
    // fused step's stream, 3.5 B per slot (sources below 2^20; chunks in
    // pairs 2p, 2p+1): s_lo[slot] = source & 0xFFFF; per pair and lane, 16
    // delay bytes (dl_pair, 4 words: the lane's 8 slots of chunk 2p, then of
    // chunk 2p+1) and 16 nibbles of source >> 16 (hi_pair, 2 words, same order)
    const uint16_t* s_lo = nullptr;
    const uint32_t* dl_pair = nullptr;
    const uint32_t* hi_pair = nullptr;
    // single-launch ensemble kernel's stream, 2 B per slot: the source's
    // index within its network (ens_sbits = 16; delays from d), or that
    // index | delay << ens_sbits (ens_sbits < 16)
    const uint16_t* ens_ls = nullptr;
    int32_t ens_sbits = 16;
    // single-launch ensemble kernel's out-edge tables (networks with delays
    // up to 31 steps): the out-edges of each source grouped by delay, as
    // target within the network | FP16 weight << 16, and per network
    // n x maxd + 1 offsets, entry s * maxd + d - 1 opening group (s, d)
    const uint32_t* push_off = nullptr;
    const uint32_t* push_edge = nullptr;
    // single-launch ensemble kernel: the driven vertices of every network,
    // (index within the network | Philox counter index << 16, threshold)
    const uint2* ens_drv = nullptr;
    // push delivery of the per-step update (NET_BUILD_PUSH): out-edges of
    // each source (target, FP16 weight | delay << 16) from out_off[source];
    // the input ring [in_ring_mask + 1][n_pad] (slot t & in_ring_mask holds
    // the inputs arriving at step t)
    const uint32_t* out_off = nullptr;
    const uint2* out_edge = nullptr;
    float* in_ring = nullptr;
    uint32_t in_ring_mask = 0;
    const uint8_t* rowstart;
    const int32_t* chunk_row0;
    const NetParams* params;
    const int32_t* net_id;        // null for one network
    const uint32_t* drive_thr;    // null when no vertex is driven
    const float* i_ext;           // null when all zero
    float* V;
    uint16_t* age;     // low byte: steps since the last spike, high byte: steps since the one
                       // before it (both saturate at 255; delivery at step t reads t - t_spike)
    float* I;
    uint32_t* ring;               // [kRingWords][n_pad]: bit (s mod 32) of word (s mod 256)/32 = spike at step s
    uint32_t* summary;            // [n_pad / 32] words, of which (n_pad >> sum_shift) / 32 are used
    // fused step: second buffers (the step reads age/summary and writes
    // these; the host swaps them after each step) and the segments
    uint16_t* age_alt = nullptr;
    uint32_t* summary_alt = nullptr;
    const int32_t* seg_vertex = nullptr;   // [n_seg + 1]
    const int32_t* seg_chunk = nullptr;    // [n_seg + 1]
    int32_t n_seg = 0, seg_max = 0;
    // Izhikevich networks (null otherwise): FP64 V and W, PSC states r and
    // p; V is also kept in FP32 in `V` for records and read-outs
    double* Vd = nullptr;
    double* Wd = nullptr;
    double* psc_r = nullptr;
    double* psc_p = nullptr;
    // Hodgkin-Huxley networks (null otherwise): gates and V(t-1); V is in Vd
    double* hh_m = nullptr;
    double* hh_n = nullptr;
    double* hh_h = nullptr;
    double* hh_vprev = nullptr;
    // plastic weights (null otherwise): see HostGraph; the last kStdpHist
    // spike steps of every vertex (ring, [n_pad][kStdpHist]) and their count
    int32_t* wq = nullptr;
    const int32_t* slot_orig = nullptr;
    const int32_t* row_first = nullptr;   // [n_total + 1]
    int32_t* spk_hist = nullptr;
    int32_t* spk_cnt = nullptr;
    double stdp_alpha = 0.0, stdp_beta = 0.0;
    // graph replays: the device step counter (null outside a captured
    // graph's launches) and the frame rule for the in-kernel bookkeeping
    const uint64_t* t_dev = nullptr;
    int32_t frame_num = 0, frame_den = 1;
    // spatial renumbering (null without NET_BUILD_REORDER): caller's global
    // index of each internal vertex [n_total], and the inverse
    const int32_t* caller_of = nullptr;
    const int32_t* internal_of = nullptr;
    double* calcium;              // null when observation is off
    double* frame_acc;
    float* frames;                // [frame_cap][n_pad]
    int32_t frame_cap;
    NetParams p0;                 // parameters of network 0 (fast path)
};

struct LaunchConfig {
    int deliver_blocks = 0;
    int deliver_threads = 0;
    bool lds_summary = false;
    bool stream_weights = false;
    bool nontemporal = false;
    int mode = 0;                  // delivery loop: 0 one chunk, 1 two chunks, 2 pipelined, 3 compacted,
                                   // 4 two packed chunks with the next pair prefetched
    bool fused = false;            // one kernel per step (delivery + vertex update), see launch_step
    bool push = false;             // push delivery (NET_BUILD_PUSH): the update kernel alone, per step
    int32_t queue_off = 0;         // fused step: arrival queues' offset in LDS (floats after the inputs)
    size_t lds_bytes = 0;
};

// Plan of the ensemble kernel: networks packed onto workgroups.
struct EnsemblePlan {
    bool enabled = false;
    int blocks = 0, threads = 0;
    size_t lds_bytes = 0;           // per workgroup (max over workgroups)
    NetMeta* meta = nullptr;        // device [n_nets] (lds_off filled per network)
    int32_t* wg_nets = nullptr;     // device: networks of workgroup b at [wg_off[b], wg_off[b+1])
    int32_t* wg_off = nullptr;      // device [blocks + 1]
    bool held = false;              // every workgroup holds one network of at most one chunk per wave
};

// LDS bytes one network needs in the ensemble kernel.
inline size_t ensemble_lds_bytes(int64_t n_nodes, int words, bool observe) {
    const size_t per = 4 * 3 + 4 * static_cast<size_t>(words) + (observe ? 16 : 0);   // V, I, age, ring, c, acc
    return (static_cast<size_t>(n_nodes) * per + 15) / 16 * 16;
}

// Kernel launchers (kernels.hip).
// ev0/ev1: optional events bound to the kernel's start and end (timing).
hipError_t launch_deliver(const DeviceGraph& g, const LaunchConfig& lc, int64_t t, hipStream_t s,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_node_update(const DeviceGraph& g, int64_t t, int64_t rec_row, const net_record* rec,
                              int32_t frame_flush, int64_t frame_index, int32_t frame_steps,
                              hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Fused step (lc.fused): delivery and vertex update of step t in one launch;
// reads g.age / g.summary and writes g.age_alt / g.summary_alt (swap after).
hipError_t launch_step(const DeviceGraph& g, const LaunchConfig& lc, int64_t t, int64_t rec_row, const net_record* rec,
                       int32_t frame_flush, int64_t frame_index, int32_t frame_steps, hipStream_t s,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_observe(const DeviceGraph& g, int32_t what, const net_fluor_params* fp, void* out,
                          int64_t n_frames, hipStream_t s);
// Plastic networks: delivery of step t with the weights as they are, then
// the plasticity update of step t (one wave per target row).
hipError_t launch_plastic_deliver(const DeviceGraph& g, int64_t t, hipStream_t s, hipEvent_t ev0 = nullptr,
                                  hipEvent_t ev1 = nullptr);
// Current weights in the caller's edge order (out[orig[slot]]); FP16 weights
// for networks that are not plastic.
hipError_t launch_weights_out(const DeviceGraph& g, float* out, hipStream_t s);
// Device step counter of graph replays: set it, or add k to it.
hipError_t launch_set_counter(uint64_t* t_dev, uint64_t t, hipStream_t s);
hipError_t launch_advance_counter(uint64_t* t_dev, uint64_t k, hipStream_t s);
// Renumbered networks: records of `rows` steps written in the internal
// numbering, copied to `tmp` (as large as the largest record) and put back in
// the caller's numbering.
hipError_t launch_records_to_caller(const DeviceGraph& g, const net_record* rec, int64_t rows, void* tmp,
                                    hipStream_t s);
hipError_t configure_deliver(DeviceGraph& g, const net_build_opts* opts, LaunchConfig& lc);   // sets g.sum_shift
hipError_t enable_ensemble_lds(size_t bytes);
hipError_t launch_ensemble(const DeviceGraph& g, const EnsemblePlan& plan, int64_t t0, int32_t n_steps,
                           const net_record* rec, int32_t frame_num, int32_t frame_den, hipStream_t s,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// ---------------------------------------------------------------------------
// Edge-scoring MLP 64 -> 256 -> 256 -> 1: flat FP32 parameter layout.
// ---------------------------------------------------------------------------
constexpr int kMlpIn = 64, kMlpH = 256;
constexpr int kMlpW1Off = 0, kMlpW1 = kMlpIn * kMlpH;          // W1[k][n]
constexpr int kMlpB1Off = kMlpW1Off + kMlpW1;                   // b1[256]
constexpr int kMlpW2Off = kMlpB1Off + kMlpH, kMlpW2 = kMlpH * kMlpH;   // W2[k][n]
constexpr int kMlpB2Off = kMlpW2Off + kMlpW2;                   // b2[256]
constexpr int kMlpW3Off = kMlpB2Off + kMlpH;                    // w3[256]
constexpr int kMlpB3Off = kMlpW3Off + kMlpH;                    // b3
constexpr int kMlpParams = kMlpB3Off + 1;                        // 82,689
// The head's gradient sums (w3[256], b2[256], b3, loss) are spread over
// replicas so that few workgroups add into any one address.
constexpr int kHeadReplicas = 32, kHeadPart = 3 * kMlpH + 8;   // w3, b2 sums; loss, b3; b1 sums at 2 * kMlpH + 8

struct MlpDevice {
    float* params = nullptr;      // FP32 master weights
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    float* grad = nullptr;
    uint16_t* w1b = nullptr;      // BF16 copies: W1 transposed ([n][k]), W2 row-major and transposed
    uint16_t* w2b = nullptr;
    uint16_t* w2c = nullptr;
    uint16_t* w1t = nullptr;      // BF16 W1 and W2 as the fused forward kernel holds them in LDS
    uint16_t* w2p = nullptr;      // (transposed, k reordered, 16-byte groups swizzled)
    uint32_t* H1bits = nullptr;   // [cap x 8] bits of H1 > 0 (the ReLU mask of dH1)
    uint16_t* dH2 = nullptr;      // [cap x 256] BF16, row-major
    uint16_t* Xbt = nullptr;      // transposed copies for the weight gradients: [64 x ldt], [256 x ldt]
    uint16_t* H1t = nullptr;      // (ldt = the batch rows rounded up to 8, at most cap rounded up)
    uint16_t* dH2t = nullptr;
    uint16_t* dH1t = nullptr;
    float* logits = nullptr;      // [cap]
    float* loss = nullptr;        // [1]
    float* head_part = nullptr;   // [kHeadReplicas][kHeadPart] head gradient partial sums (zero between steps)
    float* in_shift = nullptr;    // [64] input standardisation: x' = (x - shift) * scale
    float* in_scale = nullptr;    // [64]
    int64_t cap = 0;
};

// Observation-side inputs of the feature extractor.
struct FeatureInputs {
    const float* F;             // device [nf][n] fluorescence
    const uint32_t* drive_thr;  // device [n] control pulse thresholds, or null
    const int32_t* pairs;       // device [P][2]
    const float* dist;          // device [P]
    int32_t n, nf;
    int64_t P;
    float rho, offset;          // frame-to-frame calcium decay, observation offset
    int64_t frame_num, frame_den;
    uint32_t key_lo, key_hi;    // control schedule key
};
struct FeatureWork {
    float *en, *zn, *rn, *dc, *stats, *pm;
};
hipError_t launch_features(const FeatureInputs& in, const FeatureWork& w, float* out, hipStream_t s);
// Drive thresholds floor(rate * dt * 2^32) (as pulse_threshold) of n device rates.
hipError_t launch_pulse_thresholds(const float* rates, int32_t n, double dt_ms, uint32_t* thr, hipStream_t s);
// Shared by the estimation entry points: the descriptor check (NET_OK or
// NET_E_ARG with the text in net_estimate_last_error), the feature inputs
// of a descriptor (drive_thr left null) and the error setter.
net_status estimate_check_obs(const net_obs_desc* o);
void feature_inputs(const net_obs_desc* o, FeatureInputs& in);
net_status estimate_fail(net_status st, const std::string& msg);
uint32_t pulse_threshold(double rate_hz, double dt_ms);
// Steady-state gates (m, n, h) of the Hodgkin-Huxley vertex at V.
void hh_steady_gates(double V, double* m, double* n, double* h);

// Simulation-based fit.
struct FitInputs {
    const float* F;             // device [nf][n]
    const uint32_t* drive_thr;  // device [n] or null
    const int32_t* pairs;       // device [P][2], sorted by target
    const float* w_src;         // device [n]: assumed weight of the edges out of each vertex
    int32_t n, nf, K, n_ref;
    int64_t P, t_end, frame_num, frame_den;
    float rho, offset, inv_jump, sigma, gamma;
    double decay, v_rest, v_reset, v_th, drive_amp;   // the fit's vertex model runs in FP64
    double dt, tau_c, gain;
    uint32_t ctl_lo, ctl_hi, fit_lo, fit_hi;
};
struct FitWork {
    float* e;          // [n][nf]
    uint32_t* pulses;  // [n][words]
    double* base;      // [n][nf]
    uint8_t* member;   // [P]
    int64_t* row;      // [n+1]
    double* ll;        // [P + n]
    int32_t words;
};
hipError_t fit_prep(const FitInputs& in, const FitWork& w, hipStream_t s);
hipError_t fit_eval(const FitInputs& in, const FitWork& w, hipStream_t s);

int64_t mlp_ldt(int64_t B);
hipError_t mlp_forward(const MlpDevice& d, const float* X, int64_t B, const float* y, hipStream_t s);
hipError_t mlp_backward(const MlpDevice& d, int64_t B, float* loss_out, hipStream_t s);
// (also clears d.grad for the next accumulation)
hipError_t mlp_adam(const MlpDevice& d, float lr, float beta1, float beta2, float eps, int64_t t, hipStream_t s);
hipError_t mlp_refresh_bf16(const MlpDevice& d, hipStream_t s);
hipError_t mlp_forward_fused(const MlpDevice& d, const float* X, int64_t B, float* logits, hipStream_t s);
// Input standardisation statistics of X [rows][64]: shift = column mean,
// scale = 1 / column standard deviation (unbiased; 0 for a constant column),
// computed in FP64.  work: (kStatBlocks + 1) * 64 doubles.
constexpr int kStatBlocks = 512;
hipError_t mlp_input_stats(const float* X, int64_t rows, double* work, float* shift, float* scale, hipStream_t s);
// Rows [a0, a0 + count) of the order given by the keyed permutation of
// [0, rows) for (seed, epoch), gathered into xs [count][64] and ys [count].
hipError_t gather_shuffled(const float* X, const float* y, int64_t rows, uint64_t seed, uint32_t epoch, int64_t a0,
                           int64_t count, float* xs, float* ys, hipStream_t s);
// out[i] = permutation(i) for i < n.
hipError_t shuffle_indices(int64_t n, uint64_t seed, uint32_t epoch, int64_t* out, hipStream_t s);

}  // namespace geonet
