// C-ABI entry points of the geonet library (declared in include/geonet.h).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

using namespace geonet;

struct net {
    DeviceGraph g{};
    LaunchConfig lc{};
    std::vector<void*> blocks;
    std::vector<int64_t> node_off;
    int64_t n_edges = 0;
    int64_t t = 0;
    int64_t frames_done = 0;
    int64_t acc_steps = 0;
    int64_t device_bytes = 0;
    int32_t frame_num = 0, frame_den = 1;
    bool exact = true;
    bool broken = false;
    void* (*alloc)(size_t, void*, void*) = nullptr;
    void (*release)(void*, void*, void*) = nullptr;
    void* alloc_ctx = nullptr;
    hipStream_t last_stream = nullptr;
    // kernel timing: events [2 * launch] = start/end; kind 0 deliver, 1 update, 2 ensemble, 3 fused step
    std::vector<hipEvent_t> tev;
    std::vector<int32_t> tkind;
    std::vector<int64_t> tsteps;
    int64_t t_cap = 0, t_used = 0;
    int64_t t_every = 1;          // time one launch of each kind in t_every
    int64_t t_seen[4] = {0, 0, 0, 0};
    EnsemblePlan plan;
    std::vector<int32_t> push_base;   // per network: first entry of its out-edge offsets, -1 if none
    std::vector<int32_t> drv_off;     // [n_nets + 1] each network's range of the ensemble's drive list
    bool autotuned = false;
    // graph replays (NET_BUILD_GRAPH): device step counter, a private capture
    // stream, the 256-step graph of the per-step kernels and the ensemble
    // graphs by chunk length
    bool graph = false;
    uint64_t* t_dev = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t step_graph = nullptr;
    std::vector<std::pair<int32_t, hipGraphExec_t>> ens_graphs;
};

namespace {
constexpr int32_t kGraphSteps = 256;   // one replay: a whole turn of the history ring, an even number of steps
}

namespace {

thread_local std::string t_error;

struct AllocatorState {
    void* (*alloc)(size_t, void*, void*) = nullptr;
    void (*release)(void*, void*, void*) = nullptr;
    void* ctx = nullptr;
};
AllocatorState g_alloc;
std::mutex g_alloc_mu;

net_status fail(net_status st, const std::string& msg) {
    t_error = msg;
    return st;
}

}  // namespace

namespace geonet {

DevAllocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    DevAllocator a;
    a.alloc = g_alloc.alloc;
    a.release = g_alloc.release;
    a.ctx = g_alloc.ctx;
    return a;
}

void* DevAllocator::get(size_t bytes, hipStream_t s) const {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) / 256 * 256;
    void* p = nullptr;
    if (alloc) {
        p = alloc(bytes, s, ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    return p;
}

void DevAllocator::put(void* p, hipStream_t s) const {
    if (!p) return;
    if (release)
        release(p, s, ctx);
    else
        (void)hipFree(p);
}

}  // namespace geonet

namespace {

net_status device_fail(net* h, hipError_t e, const char* where) {
    if (h) h->broken = true;
    return fail(NET_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

void* dev_alloc(net* h, size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) / 256 * 256;
    void* p = nullptr;
    if (h->alloc) {
        p = h->alloc(bytes, s, h->alloc_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) {
        h->blocks.push_back(p);
        h->device_bytes += static_cast<int64_t>(bytes);
    }
    return p;
}

void release_all(net* h) {
    for (void* p : h->blocks) {
        if (h->release)
            h->release(p, h->last_stream, h->alloc_ctx);
        else
            (void)hipFree(p);
    }
    h->blocks.clear();
}

template <typename T>
net_status upload(net* h, T** dst, const std::vector<T>& src, size_t count, hipStream_t s, const char* what) {
    void* p = dev_alloc(h, count * sizeof(T), s);
    if (!p) return fail(NET_E_OOM, std::string("net_build: device allocation failed for ") + what);
    *dst = static_cast<T*>(p);
    if (!src.empty()) {
        hipError_t e = hipMemcpyAsync(p, src.data(), std::min(src.size(), count) * sizeof(T), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return device_fail(h, e, "net_build: upload");
    }
    return NET_OK;
}

template <typename T>
net_status zeros(net* h, T** dst, size_t count, hipStream_t s, const char* what, int byte = 0) {
    void* p = dev_alloc(h, count * sizeof(T), s);
    if (!p) return fail(NET_E_OOM, std::string("net_build: device allocation failed for ") + what);
    *dst = static_cast<T*>(p);
    hipError_t e = hipMemsetAsync(p, byte, count * sizeof(T), s);
    if (e != hipSuccess) return device_fail(h, e, "net_build: clear");
    return NET_OK;
}

// Next pair of timing events (or nulls when not timing).
void next_events(net* h, int32_t kind, int64_t steps, hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    if (h->t_used >= h->t_cap) return;
    if (h->t_seen[kind & 3]++ % h->t_every != 0) return;   // a uniform sample of the launches
    const int64_t k = h->t_used++;
    *e0 = h->tev[2 * k];
    *e1 = h->tev[2 * k + 1];
    h->tkind[k] = kind;
    h->tsteps[k] = steps;
}

// Longest-processing-time packing of networks onto workgroups under an LDS
// budget per workgroup.  Returns false if some network does not fit.
bool plan_ensemble(net* h, const HostGraph& hg, int n_cu, int wgs_per_cu, int threads, bool observe,
                   std::vector<NetMeta>& meta, std::vector<int32_t>& wg_nets, std::vector<int32_t>& wg_off,
                   size_t& lds_max) {
    const int n_nets = h->g.n_nets;
    const size_t budget = (160u * 1024u) / static_cast<size_t>(wgs_per_cu);
    meta.resize(n_nets);
    std::vector<int64_t> cost(n_nets);
    std::vector<size_t> need(n_nets);
    for (int m = 0; m < n_nets; ++m) {
        NetMeta& nm = meta[m];
        nm.node_off = static_cast<int32_t>(hg.node_off[m]);
        nm.n_nodes = static_cast<int32_t>(hg.node_off[m + 1] - hg.node_off[m]);
        nm.chunk_begin = static_cast<int32_t>(hg.net_chunk_begin[m]);
        nm.chunk_end = static_cast<int32_t>(hg.net_chunk_end[m]);
        nm.words = hg.net_max_delay[m] <= 31 ? 1 : kRingWords;
        nm.maxd = hg.net_max_delay[m];
        const bool push = nm.words == 1 && m < static_cast<int>(h->push_base.size()) && h->push_base[m] >= 0;
        nm.log_cap = push ? ens_log_cap(nm.n_nodes) : 0;
        nm.po_base = push ? h->push_base[m] : 0;
        const bool drv = m + 1 < static_cast<int>(h->drv_off.size());
        nm.drv_begin = drv ? h->drv_off[m] : 0;
        nm.drv_end = drv ? h->drv_off[m + 1] : 0;
        need[m] = ensemble_lds_bytes(nm.n_nodes, nm.words, observe) + ens_log_bytes(nm.log_cap);
        if (need[m] > budget) return false;
        // per-step cost model: edge slots + vertices + a fixed share of the barriers
        cost[m] = int64_t(nm.chunk_end - nm.chunk_begin) * kChunkEdges + 8 * int64_t(nm.n_nodes) + 2048;
    }
    const int n_wg = std::max(1, std::min(n_nets, n_cu * wgs_per_cu));
    std::vector<int> order(n_nets);
    for (int m = 0; m < n_nets; ++m) order[m] = m;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] != cost[y] ? cost[x] > cost[y] : x < y; });
    std::vector<int64_t> load(n_wg, 0);
    std::vector<size_t> used(n_wg, 0);
    std::vector<std::vector<int32_t>> lists(n_wg);
    for (int m : order) {
        int best = -1;
        for (int b = 0; b < n_wg; ++b)
            if (used[b] + need[m] <= budget && (best < 0 || load[b] < load[best])) best = b;
        if (best < 0) return false;
        meta[m].lds_off = static_cast<int32_t>(used[best]);
        meta[m].log_off = static_cast<int32_t>(used[best] + ensemble_lds_bytes(meta[m].n_nodes, meta[m].words, observe));
        used[best] += need[m];
        load[best] += cost[m];
        lists[best].push_back(m);
    }
    wg_off.assign(n_wg + 1, 0);
    wg_nets.clear();
    lds_max = 16;
    for (int b = 0; b < n_wg; ++b) {
        wg_off[b] = static_cast<int32_t>(wg_nets.size());
        for (int32_t m : lists[b]) wg_nets.push_back(m);
        lds_max = std::max(lds_max, used[b]);
    }
    wg_off[n_wg] = static_cast<int32_t>(wg_nets.size());
    (void)threads;
    return true;
}

// Plans the single-launch kernel for one shape and uploads the plan into the
// handle's plan buffers (allocated once, for the largest shape).
bool load_plan(net* h, const HostGraph& hg, int n_cu, int per_cu, int threads, bool observe, hipStream_t s) {
    std::vector<NetMeta> meta;
    std::vector<int32_t> wg_nets, wg_off;
    size_t lds_max = 0;
    if (!plan_ensemble(h, hg, n_cu, per_cu, threads, observe, meta, wg_nets, wg_off, lds_max)) return false;
    EnsemblePlan& pl = h->plan;
    if (hipMemcpyAsync(pl.meta, meta.data(), meta.size() * sizeof(NetMeta), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(pl.wg_nets, wg_nets.data(), wg_nets.size() * sizeof(int32_t), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(pl.wg_off, wg_off.data(), wg_off.size() * sizeof(int32_t), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return false;
    pl.blocks = static_cast<int>(wg_off.size()) - 1;
    pl.threads = threads;
    pl.lds_bytes = lds_max;
    // every workgroup one network of at most one chunk per wave: the kernel
    // that keeps the chunks in registers (for FP64 models at most 512 threads)
    pl.held = threads <= 512 || !(hg.any_izh || hg.any_hh);
    for (int b = 0; b < pl.blocks && pl.held; ++b) {
        const int q = wg_off[b];
        pl.held = wg_off[b + 1] - q == 1 && meta[wg_nets[q]].chunk_end - meta[wg_nets[q]].chunk_begin <= threads / 64;
    }
    if (!pl.held && !h->g.ens_ls) return false;   // the streaming kernels read the 2-byte stream
    return enable_ensemble_lds(lds_max) == hipSuccess;
}

// Graph replays: the executable graph of a captured launch sequence.
// `body` enqueues the launches on the capture stream; the counter is then
// advanced by `advance` steps inside the graph.
template <typename F>
hipError_t capture_graph(net* h, F body, uint64_t advance, hipGraphExec_t* out) {
    hipError_t e = hipSuccess;
    if (!h->cap_stream) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t eb = body(h->cap_stream);
    if (eb == hipSuccess) eb = launch_advance_counter(h->t_dev, advance, h->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->cap_stream, &g);
    if (eb != hipSuccess) e = eb;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

// The 256-step graph of the per-step kernels, from a step t with t % 256 == 0.
hipError_t step_graph(net* h, hipGraphExec_t* out) {
    if (h->step_graph) {
        *out = h->step_graph;
        return hipSuccess;
    }
    DeviceGraph gc = h->g;
    gc.t_dev = h->t_dev;
    const LaunchConfig lc = h->lc;
    auto body = [&](hipStream_t cs) -> hipError_t {
        for (int32_t k = 0; k < kGraphSteps; ++k) {
            hipError_t e;
            if (lc.fused) {
                e = launch_step(gc, lc, k, 0, nullptr, 0, 0, 0, cs);
                std::swap(gc.age, gc.age_alt);
                std::swap(gc.summary, gc.summary_alt);
            } else {
                e = lc.push ? hipSuccess : launch_deliver(gc, lc, k, cs);   // (push: the update delivers)
                if (e == hipSuccess) e = launch_node_update(gc, k, 0, nullptr, 0, 0, 0, cs);
            }
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipError_t e = capture_graph(h, body, kGraphSteps, &h->step_graph);
    *out = h->step_graph;
    return e;
}

hipError_t ensemble_graph(net* h, int32_t n_steps, hipGraphExec_t* out) {
    for (auto& p : h->ens_graphs)
        if (p.first == n_steps) {
            *out = p.second;
            return hipSuccess;
        }
    DeviceGraph gc = h->g;
    gc.t_dev = h->t_dev;
    hipGraphExec_t ex = nullptr;
    auto body = [&](hipStream_t cs) -> hipError_t {
        return launch_ensemble(gc, h->plan, 0, n_steps, nullptr, h->frame_num, h->frame_den, cs);
    };
    hipError_t e = capture_graph(h, body, static_cast<uint64_t>(n_steps), &ex);
    if (e != hipSuccess) return e;
    if (h->ens_graphs.size() >= 8) {            // keep a few lengths
        (void)hipGraphExecDestroy(h->ens_graphs.front().second);
        h->ens_graphs.erase(h->ens_graphs.begin());
    }
    h->ens_graphs.push_back({n_steps, ex});
    *out = ex;
    return hipSuccess;
}

// Host-side frame bookkeeping of steps t0 .. t0 + n - 1 run by a graph.
void advance_frames(net* h, int64_t t0, int64_t n) {
    if (!(h->g.frame_cap > 0 && h->frame_num > 0)) return;
    for (int64_t t = t0; t < t0 + n; ++t) {
        const int64_t frame = t * h->frame_num / h->frame_den;
        const int64_t next = (t + 1) * h->frame_num / h->frame_den;
        h->acc_steps += 1;
        if (next != frame) {
            h->acc_steps = 0;
            h->frames_done = std::max(h->frames_done, frame + 1);
        }
    }
}

void release_graphs(net* h) {
    if (h->step_graph) (void)hipGraphExecDestroy(h->step_graph);
    h->step_graph = nullptr;
    for (auto& p : h->ens_graphs) (void)hipGraphExecDestroy(p.second);
    h->ens_graphs.clear();
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    h->cap_stream = nullptr;
}

// Renumbered networks: records back into the caller's numbering (a
// temporary copy of the largest record, from the handle's allocator).
net_status records_to_caller(net* h, const net_record* rec, int64_t rows, hipStream_t s) {
    if (!h->g.caller_of || !rec || rows <= 0 || (!rec->raster && !rec->v && !rec->input)) return NET_OK;
    const size_t words = static_cast<size_t>((h->g.n_total + 63) / 64);
    size_t bytes = rec->raster ? static_cast<size_t>(rows) * words * 8 : 0;
    if (rec->v || rec->input) bytes = std::max(bytes, static_cast<size_t>(rows) * static_cast<size_t>(h->g.n_total) * 4);
    DevAllocator al;
    al.alloc = h->alloc;
    al.release = h->release;
    al.ctx = h->alloc_ctx;
    void* tmp = al.get(bytes, s);
    if (!tmp) return fail(NET_E_OOM, "net_step_n: no memory to renumber the records");
    hipError_t e = launch_records_to_caller(h->g, rec, rows, tmp, s);
    al.put(tmp, s);
    if (e != hipSuccess) return device_fail(h, e, "net_step_n: records");
    return NET_OK;
}

// The per-step kernels for n_steps steps (records optional), then the
// step counter and the records' numbering.
net_status step_loop(net* h, int64_t n_steps, const net_record* rec, hipStream_t s, bool observe) {
    for (int64_t k = 0; k < n_steps; ++k) {
        const int64_t t = h->t + k;
        hipEvent_t d0 = nullptr, d1 = nullptr, u0, u1;
        if (!h->lc.push) next_events(h, h->lc.fused ? 3 : 0, 1, &d0, &d1);   // (push: no delivery kernel)
        if (h->g.wq) {
            hipError_t e = launch_plastic_deliver(h->g, t, s, d0, d1);
            if (e != hipSuccess) return device_fail(h, e, "net_step_n: plastic delivery launch");
        } else if (!h->lc.fused && !h->lc.push) {
            hipError_t e = launch_deliver(h->g, h->lc, t, s, d0, d1);
            if (e != hipSuccess) return device_fail(h, e, "net_step_n: delivery launch");
        }
        int32_t flush = 0, steps = 0;
        int64_t frame = 0;
        if (observe) {
            frame = t * h->frame_num / h->frame_den;
            const int64_t next = (t + 1) * h->frame_num / h->frame_den;
            h->acc_steps += 1;
            if (next != frame) {
                flush = 1;
                steps = static_cast<int32_t>(h->acc_steps);
                h->acc_steps = 0;
                h->frames_done = std::max(h->frames_done, frame + 1);
            }
        }
        if (h->lc.fused) {
            hipError_t e = launch_step(h->g, h->lc, t, k, rec, flush, frame, steps, s, d0, d1);
            if (e != hipSuccess) return device_fail(h, e, "net_step_n: step launch");
            std::swap(h->g.age, h->g.age_alt);          // the step wrote the next ages and summary
            std::swap(h->g.summary, h->g.summary_alt);
            continue;
        }
        next_events(h, 1, 0, &u0, &u1);
        hipError_t e = launch_node_update(h->g, t, k, rec, flush, frame, steps, s, u0, u1);
        if (e != hipSuccess) return device_fail(h, e, "net_step_n: update launch");
    }
    h->t += n_steps;
    return records_to_caller(h, rec, n_steps, s);
}

net_status step_plain(net* h, int64_t n_steps, hipStream_t s, bool observe) {
    return n_steps > 0 ? step_loop(h, n_steps, nullptr, s, observe) : NET_OK;
}

// Back to the state right after build: V = v0, every other state array zero
// (age = never fired).
net_status reset_state(net* h, const HostGraph& hg, hipStream_t s) {
    DeviceGraph& g = h->g;
    const size_t np = static_cast<size_t>(g.n_pad);
    hipError_t e = hipMemcpyAsync(g.V, hg.v0.data(), std::min(hg.v0.size(), np) * sizeof(float),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(g.age, kAgeNever, (np + kAgePad) * sizeof(uint16_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(g.I, 0, np * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(g.ring, 0, np * kRingWords * sizeof(uint32_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(g.summary, 0, np / 32 * sizeof(uint32_t), s);
    if (e == hipSuccess && g.age_alt) e = hipMemsetAsync(g.age_alt, kAgeNever, (np + kAgePad) * sizeof(uint16_t), s);
    if (e == hipSuccess && g.summary_alt) e = hipMemsetAsync(g.summary_alt, 0, np / 32 * sizeof(uint32_t), s);
    if (e == hipSuccess && g.calcium) e = hipMemsetAsync(g.calcium, 0, np * sizeof(double), s);
    if (e == hipSuccess && g.Vd) {
        std::vector<double> vd(hg.v0.begin(), hg.v0.end());
        const size_t nb = std::min(vd.size(), np) * sizeof(double);
        e = hipMemcpyAsync(g.Vd, vd.data(), nb, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && g.Wd) e = hipMemcpyAsync(g.Wd, hg.w0.data(), nb, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && g.hh_m) e = hipMemcpyAsync(g.hh_m, hg.hh_m0.data(), nb, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && g.hh_n) e = hipMemcpyAsync(g.hh_n, hg.hh_n0.data(), nb, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && g.hh_h) e = hipMemcpyAsync(g.hh_h, hg.hh_h0.data(), nb, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && g.hh_vprev) e = hipMemcpyAsync(g.hh_vprev, vd.data(), nb, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(g.psc_r, 0, np * sizeof(double), s);
        if (e == hipSuccess) e = hipMemsetAsync(g.psc_p, 0, np * sizeof(double), s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);     // `vd` is freed below
    }
    if (e == hipSuccess && g.frame_acc) e = hipMemsetAsync(g.frame_acc, 0, np * sizeof(double), s);
    if (e == hipSuccess && g.frames)
        e = hipMemsetAsync(g.frames, 0, np * static_cast<size_t>(g.frame_cap) * sizeof(float), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? NET_OK : device_fail(h, e, "net_build: state reset");
}

// Autotuning results of this process, keyed by a fingerprint of what the
// timing depends on: a later build of an ensemble with the same networks
// (sizes, edge chunks, ring words, models, observation) on a device with the
// same CU count reuses the chosen shape instead of timing the trials again.
std::mutex g_tune_mutex;
std::vector<std::pair<uint64_t, std::pair<int, int>>> g_tune_cache;

uint64_t fnv(uint64_t h, uint64_t v) {
    for (int b = 0; b < 8; ++b) {
        h ^= (v >> (8 * b)) & 0xFFu;
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t ensemble_fingerprint(const HostGraph& hg, const net_desc* descs, int32_t n_nets, int n_cu, bool observe) {
    uint64_t h = 14695981039346656037ull;
    h = fnv(h, static_cast<uint64_t>(n_cu));
    h = fnv(h, observe ? 1u : 0u);
    h = fnv(h, static_cast<uint64_t>(hg.node_off.size()));
    for (size_t m = 0; m + 1 < hg.node_off.size(); ++m) {
        h = fnv(h, static_cast<uint64_t>(hg.node_off[m + 1] - hg.node_off[m]));
        h = fnv(h, static_cast<uint64_t>(hg.net_chunk_end[m] - hg.net_chunk_begin[m]));
        h = fnv(h, static_cast<uint64_t>(hg.net_max_delay[m]));
        h = fnv(h, static_cast<uint64_t>(static_cast<int32_t>(m) < n_nets ? descs[m].model : 0));
    }
    return h;
}

// Milliseconds of `steps` steps from the current state with the handle's
// current launch shape: the single-launch kernel if planned, else the sum of
// the per-step delivery kernels (the part the variants change).
bool trial_ms(net* h, int64_t t0, int32_t steps, hipStream_t s, double* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return false;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return false;
    }
    bool ok = true;
    double total = 0.0;
    if (h->plan.enabled) {
        ok = launch_ensemble(h->g, h->plan, t0, steps, nullptr, h->frame_num, h->frame_den, s, e0, e1) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess;
        float m = 0.0f;
        ok = ok && hipEventElapsedTime(&m, e0, e1) == hipSuccess;
        total = m;
    } else {
        for (int32_t k = 0; ok && k < steps; ++k) {
            ok = launch_deliver(h->g, h->lc, t0 + k, s, e0, e1) == hipSuccess &&
                 launch_node_update(h->g, t0 + k, 0, nullptr, 0, 0, 0, s, nullptr, nullptr) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess;
            float m = 0.0f;
            ok = ok && hipEventElapsedTime(&m, e0, e1) == hipSuccess;
            total += m;
        }
    }
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = total;
    return ok;
}

}  // namespace

extern "C" {

const char* net_last_error(void) { return t_error.c_str(); }

net_status net_set_allocator(void* (*alloc)(size_t, void*, void*), void (*release)(void*, void*, void*), void* ctx) {
    if ((alloc == nullptr) != (release == nullptr))
        return fail(NET_E_ARG, "net_set_allocator: give both functions or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.release = release;
    g_alloc.ctx = ctx;
    return NET_OK;
}

net_status net_build(const net_desc* descs, int32_t n_nets, const net_build_opts* opts, void* stream, net_t** out) {
    if (!out) return fail(NET_E_ARG, "net_build: out is NULL");
    *out = nullptr;
    if (opts && (opts->frame_capacity < 0 || opts->block_threads < 0 || opts->blocks_per_cu < 0 ||
                 (opts->block_threads && (opts->block_threads % 64 || opts->block_threads > 1024))))
        return fail(NET_E_ARG, "net_build: invalid options");
    HostGraph hg;
    std::string err;
    // fused step: one segment per CU, sized to fit next to the summary in LDS
    int32_t seg_count = 0, seg_cap = 0;
    if (opts && (opts->flags & NET_BUILD_FUSED_STEP) && n_nets == 1 && descs && descs[0].n_nodes > 0 &&
        descs[0].model == NET_MODEL_LIF && !descs[0].plastic) {
        int dev = 0, n_cu = 0, lds_max = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess) {
            const int64_t n_pad = (static_cast<int64_t>(descs[0].n_nodes) + kNodeAlign - 1) / kNodeAlign * kNodeAlign;
            const int64_t room = (static_cast<int64_t>(lds_max) - kStepSummaryBytes - kStepQueueBytes - 16) / 4;
            if (!(opts->flags & NET_BUILD_SUMMARY_HALF) && n_pad / 8 <= kStepSummaryBytes && room >= 64) {
                seg_count = n_cu;
                seg_cap = static_cast<int32_t>(std::min<int64_t>(room, kStepMaxSegment));
            }
        }
    }
    // spatial renumbering: the graph is built from renumbered copies
    std::vector<net_desc> rdescs;
    ReorderStore rstore;
    std::vector<int32_t> caller_of, internal_of;
    const bool reorder = opts && (opts->flags & NET_BUILD_REORDER) && descs && n_nets >= 1;
    if (reorder) reorder_descs(descs, n_nets, rdescs, rstore, caller_of, internal_of);
    net_status st = build_host_graph(reorder ? rdescs.data() : descs, n_nets, hg, err, seg_count, seg_cap);
    if (st != NET_OK) return fail(st, err);

    hipStream_t s = static_cast<hipStream_t>(stream);
    net* h = new net();
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        h->alloc = g_alloc.alloc;
        h->release = g_alloc.release;
        h->alloc_ctx = g_alloc.ctx;
    }
    h->last_stream = s;
    h->node_off = hg.node_off;
    h->n_edges = hg.n_edges;
    h->exact = hg.exact;
    h->frame_num = hg.frame_num;
    h->frame_den = hg.frame_den;
    DeviceGraph& g = h->g;
    g.n_total = hg.n_total;
    g.n_pad = hg.n_pad;
    g.e_slots = hg.e_slots;
    g.n_chunks = hg.n_chunks;
    g.n_nets = n_nets;
    g.max_delay = hg.max_delay;
    g.d_sum = hg.window;
    g.p0 = hg.params[0];
    const int32_t frame_cap = opts ? opts->frame_capacity : 0;
    g.frame_cap = frame_cap;

    auto bail = [&](net_status code) {
        (void)hipStreamSynchronize(s);
        release_all(h);
        delete h;
        return code;
    };
    const size_t np = static_cast<size_t>(g.n_pad);
    int32_t* src = nullptr;
    uint16_t* w = nullptr;
    uint8_t *d = nullptr, *rs = nullptr;
    int32_t* c0 = nullptr;
    NetParams* params = nullptr;
    if ((st = upload(h, &src, hg.src, hg.e_slots, s, "sources")) != NET_OK) return bail(st);
    if ((st = upload(h, &w, hg.w, hg.e_slots, s, "weights")) != NET_OK) return bail(st);
    if ((st = upload(h, &d, hg.d, hg.e_slots, s, "delays")) != NET_OK) return bail(st);
    if ((st = upload(h, &rs, hg.rowstart, hg.rowstart.size(), s, "row starts")) != NET_OK) return bail(st);
    if ((st = upload(h, &c0, hg.chunk_row0, hg.chunk_row0.size(), s, "chunk rows")) != NET_OK) return bail(st);
    if ((st = upload(h, &params, hg.params, hg.params.size(), s, "parameters")) != NET_OK) return bail(st);
    g.src = src;
    g.w = w;
    g.d = d;
    g.rowstart = rs;
    g.chunk_row0 = c0;
    g.params = params;
    if (n_nets > 1) {
        int32_t* nid = nullptr;
        if ((st = upload(h, &nid, hg.net_id, np, s, "network ids")) != NET_OK) return bail(st);
        g.net_id = nid;
    }
    if (hg.any_drive) {
        uint32_t* thr = nullptr;
        if ((st = upload(h, &thr, hg.drive_thr, np, s, "drive thresholds")) != NET_OK) return bail(st);
        g.drive_thr = thr;
    }
    if (hg.any_iext) {
        float* ie = nullptr;
        if ((st = upload(h, &ie, hg.i_ext, np, s, "constant inputs")) != NET_OK) return bail(st);
        g.i_ext = ie;
    }
    if ((st = upload(h, &g.V, hg.v0, np, s, "V")) != NET_OK) return bail(st);
    if ((st = zeros(h, &g.age, np + kAgePad, s, "age", kAgeNever)) != NET_OK) return bail(st);
    if ((st = zeros(h, &g.I, np, s, "input")) != NET_OK) return bail(st);
    if ((st = zeros(h, &g.ring, np * kRingWords, s, "history ring")) != NET_OK) return bail(st);
    if ((st = zeros(h, &g.summary, np / 32, s, "summary")) != NET_OK) return bail(st);
    if (hg.any_izh || hg.any_hh) {
        std::vector<double> vd(hg.v0.begin(), hg.v0.end());
        if ((st = upload(h, &g.Vd, vd, np, s, "FP64 V")) != NET_OK) return bail(st);
        if ((st = zeros(h, &g.psc_r, np, s, "PSC r")) != NET_OK) return bail(st);
        if ((st = zeros(h, &g.psc_p, np, s, "PSC p")) != NET_OK) return bail(st);
        if (hg.any_izh && (st = upload(h, &g.Wd, hg.w0, np, s, "Izhikevich W")) != NET_OK) return bail(st);
        if (hg.any_hh) {
            if ((st = upload(h, &g.hh_m, hg.hh_m0, np, s, "HH gates")) != NET_OK) return bail(st);
            if ((st = upload(h, &g.hh_n, hg.hh_n0, np, s, "HH gates")) != NET_OK) return bail(st);
            if ((st = upload(h, &g.hh_h, hg.hh_h0, np, s, "HH gates")) != NET_OK) return bail(st);
            if ((st = upload(h, &g.hh_vprev, vd, np, s, "HH V(t-1)")) != NET_OK) return bail(st);
        }
        const hipError_t se = hipStreamSynchronize(s);   // `vd` is freed below
        if (se != hipSuccess) {
            device_fail(h, se, "net_build: upload");
            return bail(NET_E_DEVICE);
        }
    }
    g.frame_num = hg.frame_num;
    g.frame_den = hg.frame_den > 0 ? hg.frame_den : 1;
    // push delivery: per-step update kernel only, and only where every sum is exact
    const bool push = opts && (opts->flags & NET_BUILD_PUSH) && !hg.plastic && hg.exact;
    if (opts && (opts->flags & NET_BUILD_GRAPH) && !hg.plastic) {
        if ((st = zeros(h, &h->t_dev, 1, s, "step counter")) != NET_OK) return bail(st);
        h->graph = true;
    }
    if (reorder) {
        int32_t *co = nullptr, *io = nullptr;
        if ((st = upload(h, &co, caller_of, caller_of.size(), s, "renumbering")) != NET_OK) return bail(st);
        if ((st = upload(h, &io, internal_of, internal_of.size(), s, "renumbering")) != NET_OK) return bail(st);
        g.caller_of = co;
        g.internal_of = io;
    }
    if (hg.plastic) {
        int32_t *wq = nullptr, *so = nullptr, *rf = nullptr;
        if ((st = upload(h, &wq, hg.wq, hg.wq.size(), s, "plastic weights")) != NET_OK) return bail(st);
        if ((st = upload(h, &so, hg.slot_orig, hg.slot_orig.size(), s, "edge order")) != NET_OK) return bail(st);
        if ((st = upload(h, &rf, hg.row_first, hg.row_first.size(), s, "rows")) != NET_OK) return bail(st);
        if ((st = zeros(h, &g.spk_hist, np * kStdpHist, s, "spike times")) != NET_OK) return bail(st);
        if ((st = zeros(h, &g.spk_cnt, np, s, "spike counts")) != NET_OK) return bail(st);
        g.wq = wq;
        g.slot_orig = so;
        g.row_first = rf;
        g.stdp_alpha = hg.stdp_alpha;
        g.stdp_beta = hg.stdp_beta;
    }
    if (frame_cap > 0) {
        if ((st = zeros(h, &g.calcium, np, s, "calcium")) != NET_OK) return bail(st);
        if ((st = zeros(h, &g.frame_acc, np, s, "frame accumulator")) != NET_OK) return bail(st);
        if ((st = zeros(h, &g.frames, np * static_cast<size_t>(frame_cap), s, "frames")) != NET_OK) return bail(st);
    }
    if (!hg.seg_vertex.empty()) {
        int32_t *sv = nullptr, *sc = nullptr;
        if ((st = upload(h, &sv, hg.seg_vertex, hg.seg_vertex.size(), s, "segments")) != NET_OK) return bail(st);
        if ((st = upload(h, &sc, hg.seg_chunk, hg.seg_chunk.size(), s, "segments")) != NET_OK) return bail(st);
        if ((st = zeros(h, &g.age_alt, np + kAgePad, s, "ages", kAgeNever)) != NET_OK) return bail(st);
        if ((st = zeros(h, &g.summary_alt, np / 32, s, "summary")) != NET_OK) return bail(st);
        g.seg_vertex = sv;
        g.seg_chunk = sc;
        g.n_seg = static_cast<int32_t>(hg.seg_vertex.size()) - 1;
        g.seg_max = hg.seg_max;
    }
    // the fused step streams 3.5 B per slot (16 low source bits, the delay
    // byte, 4 high source bits; sources below 2^20, chunks in pairs)
    if (!hg.seg_vertex.empty() && g.n_pad <= (int64_t(1) << 20) && hg.e_slots % (2 * kChunkEdges) == 0) {
        const int64_t pairs = hg.e_slots / (2 * kChunkEdges);
        std::vector<uint16_t> lo(static_cast<size_t>(hg.e_slots));
        std::vector<uint32_t> dl(static_cast<size_t>(pairs) * 64 * 4, 0u), hi(static_cast<size_t>(pairs) * 64 * 2, 0u);
        for (int64_t k = 0; k < hg.e_slots; ++k) {
            const uint32_t src = static_cast<uint32_t>(hg.src[k]);
            lo[k] = static_cast<uint16_t>(src & 0xFFFFu);
            const int64_t c = k / kChunkEdges, lane = (k % kChunkEdges) / kEdgesPerLane, j = k % kEdgesPerLane;
            const int64_t rec = (c / 2) * 64 + lane, half = c % 2;     // the lane's record in its pair
            dl[rec * 4 + half * 2 + j / 4] |= static_cast<uint32_t>(hg.d[k]) << (8 * (j % 4));
            hi[rec * 2 + half] |= (src >> 16) << (4 * j);
        }
        uint16_t* dlo = nullptr;
        uint32_t *ddl = nullptr, *dhi = nullptr;
        st = upload(h, &dlo, lo, lo.size(), s, "narrow edges");
        if (st == NET_OK) st = upload(h, &ddl, dl, dl.size(), s, "narrow edges");
        if (st == NET_OK) st = upload(h, &dhi, hi, hi.size(), s, "narrow edges");
        if (st == NET_OK) {
            const hipError_t se = hipStreamSynchronize(s);   // the host arrays are freed below
            if (se != hipSuccess) st = device_fail(h, se, "net_build: upload");
        }
        if (st != NET_OK) return bail(st);
        g.s_lo = dlo;
        g.dl_pair = ddl;
        g.hi_pair = dhi;
    }
    // the packed two-kernel delivery variant streams one word per slot,
    // source | delay << 24 (sources below 2^24)
    const int bflags = opts ? opts->flags : 0;
    if ((bflags & (NET_BUILD_DELIVER_PACKED | NET_BUILD_AUTOTUNE)) && g.n_pad < (int64_t(1) << 24)) {
        std::vector<uint32_t> packed(static_cast<size_t>(hg.e_slots));
        for (int64_t k = 0; k < hg.e_slots; ++k)
            packed[k] = static_cast<uint32_t>(hg.src[k]) | (static_cast<uint32_t>(hg.d[k]) << 24);
        uint32_t* sd = nullptr;
        st = upload(h, &sd, packed, packed.size(), s, "packed edges");
        if (st == NET_OK) {
            const hipError_t se = hipStreamSynchronize(s);   // `packed` is freed below
            if (se != hipSuccess) st = device_fail(h, se, "net_build: upload");
        }
        if (st != NET_OK) return bail(st);
        g.sd = sd;
    }
    hipError_t e = configure_deliver(g, opts, h->lc);
    if (e != hipSuccess) {
        device_fail(h, e, "net_build: configure");
        return bail(NET_E_DEVICE);
    }
    if (push) {
        // out-edges of every source (zero weights, the empty rows'
        // placeholders among them, add nothing and are left out): the target
        // of a slot is its chunk's first row plus the row starts after it
        const int64_t nv = g.n_pad;
        std::vector<uint32_t> off(static_cast<size_t>(nv) + 1, 0u);
        auto each_edge = [&](auto&& f) {
            for (int64_t c = 0; c < hg.n_chunks; ++c) {
                int64_t r = hg.chunk_row0[c];
                for (int64_t k = c * kChunkEdges; k < (c + 1) * kChunkEdges; ++k) {
                    if (k != c * kChunkEdges && ((hg.rowstart[k >> 3] >> (k & 7)) & 1u)) ++r;
                    if ((hg.w[k] & 0x7FFFu) != 0) f(k, r);
                }
            }
        };
        each_edge([&](int64_t k, int64_t) { ++off[static_cast<size_t>(hg.src[k]) + 1]; });
        for (int64_t i = 0; i < nv; ++i) off[i + 1] += off[i];
        std::vector<uint2> out(static_cast<size_t>(std::max<uint32_t>(off[nv], 1u)));
        {
            std::vector<uint32_t> fill(off.begin(), off.end() - 1);
            each_edge([&](int64_t k, int64_t r) {
                out[fill[hg.src[k]]++] = make_uint2(static_cast<uint32_t>(r),
                                                    static_cast<uint32_t>(hg.w[k]) | (static_cast<uint32_t>(hg.d[k]) << 16));
            });
        }
        uint32_t mask = 1;
        while (mask <= static_cast<uint32_t>(hg.max_delay)) mask <<= 1;   // slots > largest delay
        uint32_t* doff = nullptr;
        uint2* dout = nullptr;
        st = upload(h, &doff, off, off.size(), s, "out-edges");
        if (st == NET_OK) st = upload(h, &dout, out, out.size(), s, "out-edges");
        if (st == NET_OK) st = zeros(h, &g.in_ring, static_cast<size_t>(mask) * static_cast<size_t>(nv), s, "input ring");
        if (st == NET_OK) {
            const hipError_t se = hipStreamSynchronize(s);   // the host tables are freed below
            if (se != hipSuccess) st = device_fail(h, se, "net_build: upload");
        }
        if (st != NET_OK) return bail(st);
        g.out_off = doff;
        g.out_edge = dout;
        g.in_ring_mask = mask - 1;
        h->lc.push = true;
        h->lc.fused = false;
    }
    // a plastic network runs the per-step kernels only (trial steps would move its weights)
    const int flags = hg.plastic ? 0 : (opts ? opts->flags : 0);
    const bool autotune = (flags & NET_BUILD_AUTOTUNE) != 0;
    const bool single = !push && (n_nets > 1 || (flags & NET_BUILD_SINGLE_LAUNCH));
    if (single && !(flags & NET_BUILD_PER_STEP)) {
        // the single-launch kernel's 2-byte stream: sources within their
        // network, packed with the delay when both fit in 16 bits
        int64_t max_n = 1;
        for (int m = 0; m < n_nets; ++m) max_n = std::max(max_n, hg.node_off[m + 1] - hg.node_off[m]);
        if (max_n <= 65536) {
            int sb = 1;
            while ((int64_t(1) << sb) < max_n) ++sb;
            if (sb >= 16 || int64_t(hg.max_delay) >= (int64_t(1) << (16 - sb))) sb = 16;
            std::vector<uint16_t> ls(static_cast<size_t>(hg.e_slots), 0);
            for (int m = 0; m < n_nets; ++m) {
                const int64_t off = hg.node_off[m];
                for (int64_t k = hg.net_chunk_begin[m] * kChunkEdges; k < hg.net_chunk_end[m] * kChunkEdges; ++k) {
                    const uint32_t local = static_cast<uint32_t>(hg.src[k] - off);
                    ls[k] = static_cast<uint16_t>(sb < 16 ? (local | (static_cast<uint32_t>(hg.d[k]) << sb)) : local);
                }
            }
            uint16_t* dls = nullptr;
            st = upload(h, &dls, ls, ls.size(), s, "ensemble edges");
            if (st == NET_OK) {
                const hipError_t se = hipStreamSynchronize(s);   // `ls` is freed below
                if (se != hipSuccess) st = device_fail(h, se, "net_build: upload");
            }
            if (st != NET_OK) return bail(st);
            g.ens_ls = dls;
            g.ens_sbits = sb;
        }
        // the driven vertices of every network (index within the network, the
        // caller's index for the Philox counter, the rate threshold): noise-free
        // LIF networks draw their drive pulses for these alone
        h->drv_off.clear();
        if (hg.any_drive && max_n <= 65536) {
            std::vector<uint2> drv;
            h->drv_off.assign(n_nets + 1, 0);
            for (int m = 0; m < n_nets; ++m) {
                const int64_t off = hg.node_off[m];
                h->drv_off[m] = static_cast<int32_t>(drv.size());
                for (int64_t j = 0; j < hg.node_off[m + 1] - off; ++j) {
                    const uint32_t thr = hg.drive_thr[off + j];
                    if (thr == 0u) continue;
                    const int64_t jl = reorder ? caller_of[off + j] - off : j;
                    drv.push_back(make_uint2(static_cast<uint32_t>(j) | (static_cast<uint32_t>(jl) << 16), thr));
                }
            }
            h->drv_off[n_nets] = static_cast<int32_t>(drv.size());
            uint2* ddrv = nullptr;
            st = upload(h, &ddrv, drv, drv.size(), s, "drive list");
            if (st == NET_OK) {
                const hipError_t se = hipStreamSynchronize(s);   // `drv` is freed below
                if (se != hipSuccess) st = device_fail(h, se, "net_build: upload");
            }
            if (st != NET_OK) return bail(st);
            g.ens_drv = ddrv;
        }
        // out-edge tables for the networks whose delays fit the 32-step LDS ring:
        // each source's out-edges grouped by delay (zero weights, the empty
        // rows' placeholders among them, add nothing and are left out)
        {
            std::vector<uint32_t> po, pe;
            h->push_base.assign(n_nets, -1);
            bool fits = true;
            for (int m = 0; m < n_nets && fits; ++m) {
                const int32_t D = hg.net_max_delay[m];
                const int64_t off = hg.node_off[m], n = hg.node_off[m + 1] - off;
                if (D > 31 || n > 65536) continue;   // (targets are 16-bit in the table)
                if (static_cast<int64_t>(po.size()) + n * D + 1 > (int64_t(1) << 31) - 1) {
                    fits = false;
                    break;
                }
                const int64_t s0 = hg.net_chunk_begin[m] * kChunkEdges, s1 = hg.net_chunk_end[m] * kChunkEdges;
                // target of every slot: the chunk's first row plus the row starts after it
                std::vector<int32_t> row(static_cast<size_t>(s1 - s0));
                for (int64_t c = hg.net_chunk_begin[m]; c < hg.net_chunk_end[m]; ++c) {
                    int32_t r = hg.chunk_row0[c];
                    for (int64_t k = c * kChunkEdges; k < (c + 1) * kChunkEdges; ++k) {
                        if (k != c * kChunkEdges && ((hg.rowstart[k >> 3] >> (k & 7)) & 1u)) ++r;
                        row[k - s0] = r;
                    }
                }
                std::vector<int64_t> cnt(static_cast<size_t>(n * D) + 1, 0);
                for (int64_t k = s0; k < s1; ++k)
                    if ((hg.w[k] & 0x7FFFu) != 0) ++cnt[(hg.src[k] - off) * D + hg.d[k] - 1];
                const int64_t e_base = static_cast<int64_t>(pe.size());
                h->push_base[m] = static_cast<int32_t>(po.size());
                int64_t run = e_base;
                for (int64_t i = 0; i < n * D; ++i) {
                    po.push_back(static_cast<uint32_t>(run));
                    const int64_t c = cnt[i];
                    cnt[i] = run;
                    run += c;
                }
                po.push_back(static_cast<uint32_t>(run));
                if (run > (int64_t(1) << 32) - 1) {
                    fits = false;
                    break;
                }
                pe.resize(static_cast<size_t>(run));
                for (int64_t k = s0; k < s1; ++k)
                    if ((hg.w[k] & 0x7FFFu) != 0)
                        pe[cnt[(hg.src[k] - off) * D + hg.d[k] - 1]++] =
                            static_cast<uint32_t>(row[k - s0] - off) | (static_cast<uint32_t>(hg.w[k]) << 16);
            }
            if (!fits) h->push_base.assign(n_nets, -1);
            if (fits && !po.empty()) {
                if (pe.empty()) pe.push_back(0u);
                uint32_t *dpo = nullptr, *dpe = nullptr;
                st = upload(h, &dpo, po, po.size(), s, "out-edge tables");
                if (st == NET_OK) st = upload(h, &dpe, pe, pe.size(), s, "out-edge tables");
                if (st == NET_OK) {
                    const hipError_t se = hipStreamSynchronize(s);   // the host tables are freed below
                    if (se != hipSuccess) st = device_fail(h, se, "net_build: upload");
                }
                if (st != NET_OK) return bail(st);
                g.push_off = dpo;
                g.push_edge = dpe;
            } else {
                h->push_base.assign(n_nets, -1);
            }
        }
        int dev = 0, n_cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) {
            const bool observe = frame_cap > 0 && hg.frame_num > 0;
            // candidate shapes (workgroups per CU, threads); explicit options pin them
            std::vector<std::pair<int, int>> shapes;
            uint64_t tune_key = 0;
            bool cached = false;
            const int opt_cu = opts ? opts->blocks_per_cu : 0, opt_thr = opts ? opts->block_threads : 0;
            if (opt_cu || opt_thr) {
                const int pc = opt_cu ? opt_cu : 2;
                shapes.push_back({pc, opt_thr ? opt_thr : (pc >= 2 ? 512 : 1024)});
            } else if (autotune) {
                shapes = {{2, 512}, {1, 1024}, {1, 512}, {2, 256}, {4, 256}};
                tune_key = ensemble_fingerprint(hg, descs, n_nets, n_cu, observe);
                std::lock_guard<std::mutex> lock(g_tune_mutex);
                for (const auto& c : g_tune_cache)
                    if (c.first == tune_key) {
                        shapes = {c.second};       // tuned before in this process
                        cached = true;
                    }
            } else {
                shapes = {{2, 512}, {1, 1024}};      // the first that fits
            }
            int max_cu = 1;
            for (auto& sh : shapes) max_cu = std::max(max_cu, sh.first);
            EnsemblePlan& pl = h->plan;
            const size_t nn = static_cast<size_t>(n_nets);
            const size_t nwg = static_cast<size_t>(n_cu) * static_cast<size_t>(max_cu) + 1;
            std::vector<NetMeta> meta0(nn);
            std::vector<int32_t> zi(std::max(nn, nwg), 0);
            if ((st = upload(h, &pl.meta, meta0, nn, s, "ensemble plan")) != NET_OK) return bail(st);
            if ((st = upload(h, &pl.wg_nets, zi, nn, s, "ensemble plan")) != NET_OK) return bail(st);
            if ((st = upload(h, &pl.wg_off, zi, nwg, s, "ensemble plan")) != NET_OK) return bail(st);
            int best = -1;
            double best_ms = 0.0;
            for (size_t k = 0; k < shapes.size(); ++k) {
                if (!load_plan(h, hg, n_cu, shapes[k].first, shapes[k].second, observe, s)) continue;
                if (cached) {
                    best = static_cast<int>(k);
                    break;
                }
                if (!autotune || shapes.size() == 1) {
                    best = static_cast<int>(k);
                    break;
                }
                pl.enabled = true;
                double ms = 0.0;
                const bool ok = trial_ms(h, 0, 200, s, &ms) && trial_ms(h, 200, 200, s, &ms);
                pl.enabled = false;
                if ((st = reset_state(h, hg, s)) != NET_OK) return bail(st);
                if (!ok) {
                    (void)hipGetLastError();
                    continue;
                }
                if (best < 0 || ms < best_ms) {
                    best = static_cast<int>(k);
                    best_ms = ms;
                }
            }
            if (best >= 0) {
                if (!load_plan(h, hg, n_cu, shapes[best].first, shapes[best].second, observe, s)) {
                    device_fail(h, hipErrorUnknown, "net_build: ensemble plan");
                    return bail(NET_E_DEVICE);
                }
                pl.enabled = true;
                h->autotuned = autotune && (shapes.size() > 1 || cached);
                if (autotune && !cached && shapes.size() > 1) {
                    std::lock_guard<std::mutex> lock(g_tune_mutex);
                    if (g_tune_cache.size() >= 64) g_tune_cache.erase(g_tune_cache.begin());
                    g_tune_cache.push_back({tune_key, shapes[best]});
                }
            }
        }
    }
    if (autotune && !h->plan.enabled && !h->lc.fused && !h->lc.push) {
        // delivery variants of the per-step kernels (identical results)
        const int variants[] = {0,
                                NET_BUILD_DELIVER_PIPELINE,
                                NET_BUILD_DELIVER_UNROLL2,
                                NET_BUILD_DELIVER_NONTEMPORAL,
                                NET_BUILD_DELIVER_STREAM_WEIGHTS,
                                NET_BUILD_SUMMARY_HALF,
                                NET_BUILD_SUMMARY_HALF | NET_BUILD_DELIVER_PIPELINE,
                                NET_BUILD_SUMMARY_HALF | NET_BUILD_DELIVER_UNROLL2,
                                NET_BUILD_DELIVER_COMPACT,
                                NET_BUILD_DELIVER_COMPACT | NET_BUILD_SUMMARY_HALF,
                                NET_BUILD_DELIVER_PACKED,
                                NET_BUILD_DELIVER_PACKED | NET_BUILD_SUMMARY_HALF};
        net_build_opts o = opts ? *opts : net_build_opts{};
        const int keep = o.flags & ~(NET_BUILD_DELIVER_UNROLL2 | NET_BUILD_DELIVER_NONTEMPORAL |
                                     NET_BUILD_DELIVER_STREAM_WEIGHTS | NET_BUILD_DELIVER_PIPELINE |
                                     NET_BUILD_SUMMARY_HALF | NET_BUILD_DELIVER_COMPACT | NET_BUILD_DELIVER_PACKED);
        int best = -1;
        double best_ms = 0.0;
        for (int k = 0; k < static_cast<int>(sizeof(variants) / sizeof(variants[0])); ++k) {
            o.flags = keep | variants[k];
            if (configure_deliver(g, &o, h->lc) != hipSuccess) continue;
            // warm up into spiking activity (the initial state is silent, so
            // the history gathers, which the variants handle differently,
            // would be missing from the trial), then time
            double ms = 0.0;
            const bool ok = trial_ms(h, 0, 200, s, &ms) && trial_ms(h, 200, 64, s, &ms);
            if ((st = reset_state(h, hg, s)) != NET_OK) return bail(st);
            if (!ok) {
                (void)hipGetLastError();
                continue;
            }
            if (best < 0 || ms < best_ms) {
                best = k;
                best_ms = ms;
            }
        }
        o.flags = keep | (best >= 0 ? variants[best] : 0);
        e = configure_deliver(g, &o, h->lc);
        if (e != hipSuccess) {
            device_fail(h, e, "net_build: configure");
            return bail(NET_E_DEVICE);
        }
        h->autotuned = best >= 0;
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        device_fail(h, e, "net_build: upload");
        return bail(NET_E_DEVICE);
    }
    *out = h;
    if (!h->exact) {
        t_error = "net_build: some target's weights may not sum exactly in FP32";
        return NET_W_INEXACT;
    }
    return NET_OK;
}

net_status net_step_n(net_t* h, int64_t n_steps, const net_record* rec, void* stream) {
    if (!h) return fail(NET_E_ARG, "net_step_n: handle is NULL");
    if (h->broken) return fail(NET_E_STATE, "net_step_n: handle unusable after a device error");
    if (n_steps < 0) return fail(NET_E_ARG, "net_step_n: n_steps < 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    h->last_stream = s;
    const bool observe = h->g.frame_cap > 0 && h->frame_num > 0;
    // graph replays: no records, no kernel timing
    const bool graphs = h->graph && !rec && h->t_cap == 0 && n_steps > 0;
    if (graphs && h->plan.enabled) {
        int64_t done = 0;
        while (done < n_steps) {
            const int32_t chunk = static_cast<int32_t>(std::min<int64_t>(n_steps - done, int64_t(1) << 30));
            hipGraphExec_t ex = nullptr;
            hipError_t e = ensemble_graph(h, chunk, &ex);
            if (e == hipSuccess) e = launch_set_counter(h->t_dev, static_cast<uint64_t>(h->t + done), s);
            if (e == hipSuccess) e = hipGraphLaunch(ex, s);
            if (e != hipSuccess) return device_fail(h, e, "net_step_n: ensemble graph");
            done += chunk;
        }
        advance_frames(h, h->t, n_steps);
        h->t += n_steps;
        return NET_OK;
    }
    if (graphs) {
        // single steps up to a multiple of 256, whole 256-step graphs, single steps after
        const int64_t head = std::min<int64_t>(n_steps, (kGraphSteps - h->t % kGraphSteps) % kGraphSteps);
        const int64_t blocks = (n_steps - head) / kGraphSteps;
        if (blocks > 0) {
            if (head > 0) {
                net_status st = step_plain(h, head, s, observe);
                if (st != NET_OK) return st;
            }
            hipGraphExec_t ex = nullptr;
            hipError_t e = step_graph(h, &ex);
            if (e == hipSuccess) e = launch_set_counter(h->t_dev, static_cast<uint64_t>(h->t), s);
            for (int64_t b = 0; e == hipSuccess && b < blocks; ++b) e = hipGraphLaunch(ex, s);
            if (e != hipSuccess) return device_fail(h, e, "net_step_n: step graph");
            advance_frames(h, h->t, blocks * kGraphSteps);
            h->t += blocks * kGraphSteps;     // 256 swaps of the fused step's buffers: back where they were
            return step_plain(h, n_steps - head - blocks * kGraphSteps, s, observe);
        }
    }
    if (h->plan.enabled) {
        // one launch per (at most 2^30) steps for the whole ensemble
        int64_t done = 0;
        while (done < n_steps) {
            const int32_t chunk = static_cast<int32_t>(std::min<int64_t>(n_steps - done, int64_t(1) << 30));
            net_record sub{};
            if (rec) {
                const int64_t words = (h->g.n_total + 63) / 64;
                sub.raster = rec->raster ? rec->raster + done * words : nullptr;
                sub.v = rec->v ? rec->v + done * h->g.n_total : nullptr;
                sub.input = rec->input ? rec->input + done * h->g.n_total : nullptr;
            }
            hipEvent_t e0, e1;
            next_events(h, 2, chunk, &e0, &e1);
            hipError_t e = launch_ensemble(h->g, h->plan, h->t + done, chunk, rec ? &sub : nullptr, h->frame_num,
                                           h->frame_den, s, e0, e1);
            if (e != hipSuccess) return device_fail(h, e, "net_step_n: ensemble launch");
            done += chunk;
        }
        if (observe) {
            for (int64_t t = h->t; t < h->t + n_steps; ++t) {
                const int64_t frame = t * h->frame_num / h->frame_den;
                const int64_t next = (t + 1) * h->frame_num / h->frame_den;
                h->acc_steps += 1;
                if (next != frame) {
                    h->acc_steps = 0;
                    h->frames_done = std::max(h->frames_done, frame + 1);
                }
            }
        }
        h->t += n_steps;
        return records_to_caller(h, rec, n_steps, s);
    }
    return step_loop(h, n_steps, rec, s, observe);
}

net_status net_observe(net_t* h, int32_t what, const void* params, void* out, int64_t out_bytes, void* stream) {
    if (!h) return fail(NET_E_ARG, "net_observe: handle is NULL");
    if (h->broken) return fail(NET_E_STATE, "net_observe: handle unusable after a device error");
    if (!out) return fail(NET_E_ARG, "net_observe: out is NULL");
    const int64_t n = h->g.n_total;
    int64_t frames = 0;
    switch (what) {
        case NET_OBS_V:
        case NET_OBS_REF:
            if (out_bytes < 4 * n) return fail(NET_E_ARG, "net_observe: out_bytes too small");
            break;
        case NET_OBS_CALCIUM:
            if (h->g.frame_cap <= 0) return fail(NET_E_UNSUPPORTED, "net_observe: built without observation");
            if (out_bytes < 4 * n) return fail(NET_E_ARG, "net_observe: out_bytes too small");
            break;
        case NET_OBS_FRAMES:
        case NET_OBS_FLUOR: {
            if (h->g.frame_cap <= 0) return fail(NET_E_UNSUPPORTED, "net_observe: built without observation");
            if (out_bytes % (4 * n) != 0) return fail(NET_E_ARG, "net_observe: out_bytes must be F * 4 * n_total");
            frames = out_bytes / (4 * n);
            const int64_t avail = std::min<int64_t>(h->frames_done, h->g.frame_cap);
            if (frames > avail) return fail(NET_E_RANGE, "net_observe: more frames requested than recorded");
            if (what == NET_OBS_FLUOR && !params) return fail(NET_E_ARG, "net_observe: fluorescence needs parameters");
            break;
        }
        case NET_OBS_WEIGHTS: {
            if (!h->g.wq) return fail(NET_E_UNSUPPORTED, "net_observe: weights are read out for plastic networks");
            if (out_bytes < 4 * h->n_edges) return fail(NET_E_ARG, "net_observe: out_bytes too small");
            hipStream_t s = static_cast<hipStream_t>(stream);
            h->last_stream = s;
            hipError_t e = launch_weights_out(h->g, static_cast<float*>(out), s);
            if (e != hipSuccess) return device_fail(h, e, "net_observe");
            return NET_OK;
        }
        default:
            return fail(NET_E_ARG, "net_observe: unknown observable");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    h->last_stream = s;
    hipError_t e = launch_observe(h->g, what, static_cast<const net_fluor_params*>(params), out, frames, s);
    if (e != hipSuccess) return device_fail(h, e, "net_observe");
    return NET_OK;
}

net_status net_info(const net_t* h, net_info_t* out) {
    if (!h || !out) return fail(NET_E_ARG, "net_info: NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->n_total = h->g.n_total;
    out->n_edges = h->n_edges;
    out->n_edges_stored = h->g.e_slots;
    out->n_nets = h->g.n_nets;
    out->max_delay = h->g.max_delay;
    out->summary_window = h->g.d_sum;
    out->raster_words = (h->g.n_total + 63) / 64;
    out->t = h->t;
    out->frames_done = h->frames_done;
    out->exact = h->exact ? 1 : 0;
    out->lds_summary = h->lc.lds_summary ? 1 : 0;
    out->deliver_blocks = h->lc.deliver_blocks;
    out->deliver_threads = h->lc.deliver_threads;
    out->device_bytes = h->device_bytes;
    out->deliver_flags = (h->lc.mode == 1 ? NET_BUILD_DELIVER_UNROLL2 : 0) |
                         (h->lc.mode == 4 ? NET_BUILD_DELIVER_PACKED : 0) |
                         (h->lc.mode == 2 ? NET_BUILD_DELIVER_PIPELINE : 0) |
                         (h->lc.mode == 3 ? NET_BUILD_DELIVER_COMPACT : 0) |
                         (h->lc.fused ? NET_BUILD_FUSED_STEP : 0) | (h->lc.push ? NET_BUILD_PUSH : 0) |
                         (h->lc.nontemporal ? NET_BUILD_DELIVER_NONTEMPORAL : 0) |
                         (h->lc.stream_weights ? NET_BUILD_DELIVER_STREAM_WEIGHTS : 0) |
                         (h->g.sum_shift ? NET_BUILD_SUMMARY_HALF : 0);
    out->ensemble_blocks = h->plan.enabled ? h->plan.blocks : 0;
    out->ensemble_threads = h->plan.enabled ? h->plan.threads : 0;
    out->autotuned = h->autotuned ? 1 : 0;
    out->ensemble_stream = !h->plan.enabled ? 0 : (h->plan.held ? 1 : (h->g.ens_sbits < 16 ? 3 : 2));
    return NET_OK;
}

net_status net_node_offsets(const net_t* h, int64_t* out) {
    if (!h || !out) return fail(NET_E_ARG, "net_node_offsets: NULL argument");
    std::memcpy(out, h->node_off.data(), h->node_off.size() * sizeof(int64_t));
    return NET_OK;
}

net_status net_simulate_device_error(net_t* h) {
    if (!h) return fail(NET_E_ARG, "net_simulate_device_error: handle is NULL");
    h->broken = true;
    return NET_OK;
}

net_status net_timing_begin(net_t* h, int64_t max_launches, int32_t every) {
    if (!h) return fail(NET_E_ARG, "net_timing_begin: handle is NULL");
    if (h->broken) return fail(NET_E_STATE, "net_timing_begin: handle unusable after a device error");
    if (max_launches < 0 || max_launches > (int64_t(1) << 22))
        return fail(NET_E_ARG, "net_timing_begin: bad max_launches");
    if (every < 1) return fail(NET_E_ARG, "net_timing_begin: every must be >= 1");
    h->t_every = every;
    for (int64_t& c : h->t_seen) c = 0;
    for (hipEvent_t e : h->tev) (void)hipEventDestroy(e);
    h->tev.assign(static_cast<size_t>(2 * max_launches), nullptr);
    h->tkind.assign(static_cast<size_t>(max_launches), 0);
    h->tsteps.assign(static_cast<size_t>(max_launches), 0);
    h->t_cap = 0;
    h->t_used = 0;
    for (auto& e : h->tev) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return device_fail(h, r, "net_timing_begin");
    }
    h->t_cap = max_launches;
    return NET_OK;
}

net_status net_timing_end(net_t* h, net_timing_t* out) {
    if (!h || !out) return fail(NET_E_ARG, "net_timing_end: NULL argument");
    if (h->broken) return fail(NET_E_STATE, "net_timing_end: handle unusable after a device error");
    std::memset(out, 0, sizeof(*out));
    for (int64_t k = 0; k < h->t_used; ++k) {
        float ms = 0.0f;
        hipError_t r = hipEventSynchronize(h->tev[2 * k + 1]);
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, h->tev[2 * k], h->tev[2 * k + 1]);
        if (r != hipSuccess) return device_fail(h, r, "net_timing_end");
        switch (h->tkind[k]) {
            case 0: out->deliver_ms += ms; out->deliver_launches++; break;
            case 3: out->step_ms += ms; out->step_launches++; break;
            case 1: out->update_ms += ms; out->update_launches++; break;
            default: out->ensemble_ms += ms; out->ensemble_launches++; break;
        }
        out->steps += h->tsteps[k];
    }
    for (hipEvent_t e : h->tev) (void)hipEventDestroy(e);
    h->tev.clear();
    h->t_cap = h->t_used = 0;
    return NET_OK;
}

void net_free(net_t* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->last_stream);
    for (hipEvent_t e : h->tev) (void)hipEventDestroy(e);
    release_graphs(h);
    release_all(h);
    delete h;
}

}  // extern "C"
