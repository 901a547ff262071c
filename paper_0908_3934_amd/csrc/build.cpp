// Host-side graph construction: delays from geometry, FP16 weights and the
// CSR-by-target edge layout consumed by the delivery kernel.
//
// Layout of the stored edge list (one entry per "slot"):
//   rows are targets j in ensemble order; a row holds the in-edges of j
//   sorted by source; a target with no in-edge gets one placeholder slot
//   (weight 0, source j, delay 1) so that every row owns at least one slot;
//   the list is padded with placeholders to a multiple of 512 slots.
//   rowstart bit s is set iff slot s is the first slot of its row, and
//   chunk_row0[c] is the row of slot 512*c.  Row of slot s is then
//   chunk_row0[s/512] + (number of rowstart bits in (512*(s/512), s]).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "internal.h"

namespace geonet {
namespace {

uint16_t to_fp16_bits(float f) {
    _Float16 h = static_cast<_Float16>(f);   // IEEE round-to-nearest-even
    uint16_t b;
    std::memcpy(&b, &h, sizeof(b));
    return b;
}

// log2 of the spacing of FP16 values around |h| (h != 0, finite).
int fp16_ulp_log2(uint16_t h) {
    int e = (h >> 10) & 0x1F;
    return e == 0 ? -24 : e - 25;
}

bool fp16_finite(uint16_t h) { return ((h >> 10) & 0x1F) != 0x1F; }

double fp16_abs(uint16_t h) {
    _Float16 v;
    uint16_t a = h & 0x7FFF;
    std::memcpy(&v, &a, sizeof(a));
    return static_cast<double>(v);
}

// Delay rule of Eq. delaydist in steps: max(1, ceil(|xi - xj| / (s*dt))).
int32_t delay_from_geometry(const double* xi, const double* xj, int dims, double step_len) {
    double acc = 0.0;
    for (int k = 0; k < dims; ++k) {
        const double diff = xi[k] - xj[k];
        acc = acc + diff * diff;
    }
    const double steps = std::ceil(std::sqrt(acc) / step_len);
    if (!(steps <= 255.0)) return -1;
    return steps < 1.0 ? 1 : static_cast<int32_t>(steps);
}

}  // namespace

// Control pulse threshold: a pulse when a 32-bit draw is below floor(p * 2^32).
uint32_t pulse_threshold(double rate_hz, double dt_ms) {
    const double thr = std::floor(rate_hz * (dt_ms * 1e-3) * 4294967296.0);
    if (!(thr > 0.0)) return 0u;
    if (thr >= 4294967295.0) return 0xFFFFFFFFu;
    return static_cast<uint32_t>(thr);
}

void reorder_descs(const net_desc* in, int32_t n_nets, std::vector<net_desc>& out, ReorderStore& st,
                   std::vector<int32_t>& caller_of, std::vector<int32_t>& internal_of) {
    out.assign(in, in + n_nets);
    st = ReorderStore{};
    st.pos.resize(n_nets);
    st.src.resize(n_nets);
    st.dst.resize(n_nets);
    st.rate.resize(n_nets);
    st.iext.resize(n_nets);
    st.v0.resize(n_nets);
    st.w0.resize(n_nets);
    int64_t total = 0;
    for (int m = 0; m < n_nets; ++m) total += in[m].n_nodes;
    caller_of.assign(total, 0);
    internal_of.assign(total, 0);
    int64_t off = 0;
    for (int m = 0; m < n_nets; ++m) {
        const net_desc& d = in[m];
        net_desc& o = out[m];
        const int32_t n = d.n_nodes;
        std::vector<int32_t> order(n);   // order[k] = caller's local index of internal vertex k
        for (int32_t j = 0; j < n; ++j) order[j] = j;
        if (d.pos_um && d.dims >= 1 && d.dims <= 3 && n > 1) {
            const int D = d.dims;
            std::vector<double> lo(D, 1e308), hi(D, -1e308);
            for (int32_t j = 0; j < n; ++j)
                for (int k = 0; k < D; ++k) {
                    lo[k] = std::min(lo[k], d.pos_um[int64_t(j) * D + k]);
                    hi[k] = std::max(hi[k], d.pos_um[int64_t(j) * D + k]);
                }
            const int bits = D == 1 ? 63 : (D == 2 ? 31 : 21);
            std::vector<uint64_t> code(n, 0);
            for (int32_t j = 0; j < n; ++j) {
                for (int k = 0; k < D; ++k) {
                    const double span = hi[k] > lo[k] ? hi[k] - lo[k] : 1.0;
                    double q = (d.pos_um[int64_t(j) * D + k] - lo[k]) / span * std::ldexp(1.0, bits);
                    q = std::min(std::max(q, 0.0), std::ldexp(1.0, bits) - 1.0);
                    const uint64_t c = static_cast<uint64_t>(q);
                    for (int b = 0; b < bits; ++b) code[j] |= ((c >> b) & 1ull) << (b * D + k);
                }
            }
            std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return code[a] < code[b]; });
        }
        std::vector<int32_t> newid(n);
        for (int32_t k = 0; k < n; ++k) newid[order[k]] = k;
        for (int32_t k = 0; k < n; ++k) {
            caller_of[off + k] = static_cast<int32_t>(off + order[k]);
            internal_of[off + order[k]] = static_cast<int32_t>(off + k);
        }
        if (d.pos_um) {
            st.pos[m].resize(static_cast<size_t>(n) * d.dims);
            for (int32_t k = 0; k < n; ++k)
                for (int c = 0; c < d.dims; ++c) st.pos[m][int64_t(k) * d.dims + c] = d.pos_um[int64_t(order[k]) * d.dims + c];
            o.pos_um = st.pos[m].data();
        }
        if (d.n_edges > 0 && d.src && d.dst) {
            st.src[m].resize(d.n_edges);
            st.dst[m].resize(d.n_edges);
            for (int64_t e = 0; e < d.n_edges; ++e) {
                const bool ok = d.src[e] >= 0 && d.src[e] < n && d.dst[e] >= 0 && d.dst[e] < n;
                st.src[m][e] = ok ? newid[d.src[e]] : d.src[e];    // out-of-range indices are reported by the build
                st.dst[m][e] = ok ? newid[d.dst[e]] : d.dst[e];
            }
            o.src = st.src[m].data();
            o.dst = st.dst[m].data();
        }
        auto perm_f = [&](const float* a, std::vector<float>& v) -> const float* {
            if (!a) return nullptr;
            v.resize(n);
            for (int32_t k = 0; k < n; ++k) v[k] = a[order[k]];
            return v.data();
        };
        o.drive_rate_hz = perm_f(d.drive_rate_hz, st.rate[m]);
        o.i_ext = perm_f(d.i_ext, st.iext[m]);
        o.v0 = perm_f(d.v0, st.v0[m]);
        o.w0 = perm_f(d.w0, st.w0[m]);
        off += n;
    }
}

// Hodgkin-Huxley rate functions (the standard squid-axon set; mV, ms),
// alpha_m and alpha_n at their limits where the denominator vanishes.
void hh_steady_gates(double V, double* m, double* n, double* h) {
    const double x = V + 40.0, y = V + 55.0;
    const double am = x == 0.0 ? 1.0 : 0.1 * x / (1.0 - std::exp(-x / 10.0));
    const double bm = 4.0 * std::exp(-(V + 65.0) / 18.0);
    const double ah = 0.07 * std::exp(-(V + 65.0) / 20.0);
    const double bh = 1.0 / (1.0 + std::exp(-(V + 35.0) / 10.0));
    const double an = y == 0.0 ? 0.1 : 0.01 * y / (1.0 - std::exp(-y / 10.0));
    const double bn = 0.125 * std::exp(-(V + 65.0) / 80.0);
    *m = am / (am + bm);
    *n = an / (an + bn);
    *h = ah / (ah + bh);
}

net_status build_host_graph(const net_desc* descs, int32_t n_nets, HostGraph& g, std::string& err, int32_t seg_count,
                            int32_t seg_cap) {
    if (!descs || n_nets < 1) {
        err = "net_build: descs must hold n_nets >= 1 networks";
        return NET_E_ARG;
    }
    g.node_off.assign(n_nets + 1, 0);
    int64_t e_total = 0;
    for (int m = 0; m < n_nets; ++m) {
        const net_desc& d = descs[m];
        if (d.n_nodes < 1 || d.dims < 1 || d.dims > 3 || d.n_edges < 0) {
            err = "net_build: network " + std::to_string(m) + " needs n_nodes >= 1, dims in 1..3, n_edges >= 0";
            return NET_E_ARG;
        }
        if (d.n_edges > 0 && (!d.src || !d.dst || !d.weight)) {
            err = "net_build: network " + std::to_string(m) + " has edges but no src/dst/weight";
            return NET_E_ARG;
        }
        if (!d.delay_steps && d.n_edges > 0 && !d.pos_um) {
            err = "net_build: network " + std::to_string(m) + " needs positions or explicit delays";
            return NET_E_ARG;
        }
        if (d.model != NET_MODEL_LIF && d.model != NET_MODEL_IZHIKEVICH && d.model != NET_MODEL_HODGKIN_HUXLEY) {
            err = "net_build: network " + std::to_string(m) + " has an unknown vertex model";
            return NET_E_ARG;
        }
        if (d.model == NET_MODEL_LIF &&
            (!(d.dt_ms > 0.0) || !(d.tau_ms > 0.0) || d.n_ref < 0 || d.n_ref > 250)) {
            err = "net_build: network " + std::to_string(m) + " needs dt > 0, tau > 0, 0 <= n_ref <= 250";
            return NET_E_ARG;
        }
        if (d.plastic && (n_nets != 1 || d.model != NET_MODEL_LIF || d.n_ref < kStdpMinRef)) {
            err = "net_build: plasticity needs one network per handle, the LIF vertex and n_ref >= " +
                  std::to_string(kStdpMinRef);
            return NET_E_ARG;
        }
        if (d.model == NET_MODEL_HODGKIN_HUXLEY &&
            (!(d.dt_ms > 0.0) || d.n_ref != 0 || !(d.hh_C > 0.0f) || d.psc < NET_PSC_NONE || d.psc > NET_PSC_ALPHA ||
             (d.psc != NET_PSC_NONE && !(d.psc_rate >= 0.0f)))) {
            err = "net_build: Hodgkin-Huxley network " + std::to_string(m) +
                  " needs dt > 0, n_ref = 0, C > 0, psc in 0..2 and psc_rate >= 0";
            return NET_E_ARG;
        }
        if (d.model == NET_MODEL_IZHIKEVICH &&
            (!(d.dt_ms > 0.0) || d.n_ref != 0 || !(d.iz_C > 0.0f) || d.psc < NET_PSC_NONE || d.psc > NET_PSC_ALPHA ||
             (d.psc != NET_PSC_NONE && !(d.psc_rate >= 0.0f)))) {
            err = "net_build: Izhikevich network " + std::to_string(m) +
                  " needs dt > 0, n_ref = 0, C > 0, psc in 0..2 and psc_rate >= 0";
            return NET_E_ARG;
        }
        if (!d.delay_steps && d.n_edges > 0 && !(d.v_um_per_ms > 0.0)) {
            err = "net_build: network " + std::to_string(m) + " needs a positive conduction speed";
            return NET_E_ARG;
        }
        if (m > 0 && (d.dt_ms != descs[0].dt_ms || d.frame_num != descs[0].frame_num ||
                      d.frame_den != descs[0].frame_den)) {
            err = "net_build: all networks of an ensemble must share dt and the frame rule";
            return NET_E_ARG;
        }
        g.node_off[m + 1] = g.node_off[m] + d.n_nodes;
        e_total += d.n_edges;
    }
    g.n_total = g.node_off[n_nets];
    if (g.n_total > (int64_t(1) << 28)) {
        err = "net_build: more than 2^28 vertices";
        return NET_E_RANGE;
    }
    g.n_pad = (g.n_total + kNodeAlign - 1) / kNodeAlign * kNodeAlign;
    g.n_edges = e_total;
    g.dt_ms = descs[0].dt_ms;
    g.frame_num = descs[0].frame_num;
    g.frame_den = descs[0].frame_den > 0 ? descs[0].frame_den : 1;
    if (g.frame_num < 0) {
        err = "net_build: frame_num must be >= 0";
        return NET_E_ARG;
    }

    // In-degree per target row.
    const int64_t N = g.n_total;
    std::vector<int64_t> indeg(N + 1, 0);
    for (int m = 0; m < n_nets; ++m) {
        const net_desc& d = descs[m];
        for (int64_t e = 0; e < d.n_edges; ++e) {
            const int32_t i = d.src[e], j = d.dst[e];
            if (i < 0 || i >= d.n_nodes || j < 0 || j >= d.n_nodes) {
                err = "net_build: network " + std::to_string(m) + " edge " + std::to_string(e) +
                      " has a vertex index out of range";
                return NET_E_ARG;
            }
            if (i == j) {
                err = "net_build: network " + std::to_string(m) + " edge " + std::to_string(e) +
                      " is a self-loop (the input set excludes i == j)";
                return NET_E_ARG;
            }
            indeg[g.node_off[m] + j]++;
        }
    }
    // Slot offsets: every row gets max(indeg, 1) slots.  In an ensemble each
    // network's slot range starts on a chunk boundary, so a chunk never mixes
    // networks (the ensemble kernel walks each network's chunks on its own).
    std::vector<int64_t> row_ptr(N + 1, 0);   // row_ptr[r] = first slot of row r
    // Segments (fused step): balance slots plus a small per-vertex update
    // cost (the update's loads overlap the delivery, so a segment's time
    // follows its slot count), cut only at multiples of 64 vertices, at most
    // seg_cap vertices each.
    std::vector<char> seg_start(N + 1, 0);
    g.seg_vertex.clear();
    g.seg_chunk.clear();
    g.seg_max = 0;
    if (seg_count > 0 && n_nets == 1 && seg_cap >= 64) {
        const int64_t kVertexCost = 1;
        int64_t total = 0;
        for (int64_t r = 0; r < N; ++r) total += std::max<int64_t>(indeg[r], 1) + kVertexCost;
        const int64_t cap = seg_cap / 64 * 64;
        std::vector<int32_t> starts{0};
        int64_t acc = 0, begin = 0;
        for (int64_t r = 0; r < N; ++r) {
            acc += std::max<int64_t>(indeg[r], 1) + kVertexCost;
            const int64_t next = r + 1;
            if (next % 64 != 0 || next == N) continue;
            const int64_t k = static_cast<int64_t>(starts.size());
            if (acc * seg_count >= total * k || next - begin >= cap) {
                starts.push_back(static_cast<int32_t>(next));
                begin = next;
            }
        }
        bool ok = static_cast<int32_t>(starts.size()) <= seg_count;
        starts.push_back(static_cast<int32_t>(N));
        for (size_t k = 0; ok && k + 1 < starts.size(); ++k) {
            const int32_t len = starts[k + 1] - starts[k];
            ok = len <= cap;
            g.seg_max = std::max(g.seg_max, len);
        }
        if (ok) {
            g.seg_vertex = starts;
            for (size_t k = 0; k + 1 < starts.size(); ++k) seg_start[starts[k]] = 1;
        } else {
            g.seg_max = 0;
        }
    }
    // segments start on even chunks and the slot array ends on one, so the
    // fused step's units (chunk pairs) never straddle two segments
    const int64_t seg_align = g.seg_vertex.empty() ? kChunkEdges : 2 * kChunkEdges;
    g.net_chunk_begin.assign(n_nets, 0);
    g.net_chunk_end.assign(n_nets, 0);
    int64_t used = 0;
    for (int m = 0; m < n_nets; ++m) {
        if (n_nets > 1) used = (used + kChunkEdges - 1) / kChunkEdges * kChunkEdges;
        g.net_chunk_begin[m] = used / kChunkEdges;
        for (int64_t r = g.node_off[m]; r < g.node_off[m + 1]; ++r) {
            if (seg_start[r]) {
                used = (used + seg_align - 1) / seg_align * seg_align;
                g.seg_chunk.push_back(static_cast<int32_t>(used / kChunkEdges));
            }
            row_ptr[r] = used;
            used += std::max<int64_t>(indeg[r], 1);
        }
        g.net_chunk_end[m] = (used + kChunkEdges - 1) / kChunkEdges;
    }
    row_ptr[N] = used;
    g.e_slots = (used + seg_align - 1) / seg_align * seg_align;
    if (g.e_slots == 0) g.e_slots = seg_align;
    if (g.e_slots > (int64_t(1) << 31) - kChunkEdges) {
        err = "net_build: more than 2^31 edge slots";
        return NET_E_RANGE;
    }
    g.n_chunks = g.e_slots / kChunkEdges;
    if (!g.seg_vertex.empty()) g.seg_chunk.push_back(static_cast<int32_t>(g.n_chunks));
    // Every slot starts as a zero-weight placeholder owned by the preceding row
    // (its source is that row's own vertex, so it stays inside its network).
    g.src.assign(g.e_slots, 0);
    g.w.assign(g.e_slots, 0);
    g.d.assign(g.e_slots, 1);
    g.rowstart.assign(g.e_slots / 8, 0);
    for (int64_t r = 0; r < N; ++r) {
        const int64_t a = row_ptr[r];
        const int64_t b = (r + 1 < N) ? row_ptr[r + 1] : g.e_slots;
        for (int64_t s = a; s < b; ++s) g.src[s] = static_cast<int32_t>(r);
    }

    // Scatter edges into their rows (stable in input order).
    std::vector<int64_t> fill(row_ptr.begin(), row_ptr.end() - 1);
    const bool track = n_nets == 1 && descs[0].plastic;   // keep each slot's edge index
    std::vector<int32_t> orig;
    if (track) orig.assign(g.e_slots, -1);
    int32_t max_delay = 1;
    g.net_max_delay.assign(n_nets, 1);
    for (int m = 0; m < n_nets; ++m) {
        const net_desc& d = descs[m];
        const int64_t off = g.node_off[m];
        const double step_len = d.v_um_per_ms * d.dt_ms;
        for (int64_t e = 0; e < d.n_edges; ++e) {
            const int32_t i = d.src[e], j = d.dst[e];
            int32_t dl;
            if (d.delay_steps) {
                dl = d.delay_steps[e] < 1 ? 1 : d.delay_steps[e];
            } else {
                dl = delay_from_geometry(d.pos_um + int64_t(i) * d.dims, d.pos_um + int64_t(j) * d.dims, d.dims,
                                         step_len);
                if (dl < 0) {
                    err = "net_build: network " + std::to_string(m) + " edge " + std::to_string(e) +
                          " needs a delay above 255 steps";
                    return NET_E_RANGE;
                }
            }
            const uint16_t wb = to_fp16_bits(d.weight[e]);
            if (!fp16_finite(wb)) {
                err = "net_build: network " + std::to_string(m) + " edge " + std::to_string(e) +
                      " has a weight outside the FP16 range";
                return NET_E_RANGE;
            }
            max_delay = std::max(max_delay, dl);
            g.net_max_delay[m] = std::max(g.net_max_delay[m], dl);
            const int64_t s = fill[off + j]++;
            g.src[s] = static_cast<int32_t>(off + i);
            g.w[s] = wb;
            g.d[s] = static_cast<uint8_t>(dl);
            if (track) orig[s] = static_cast<int32_t>(e);
        }
    }
    g.max_delay = max_delay;
    // Summary window: the smallest W with at most 0.5 % of the edges longer
    // than W (those edges bypass the recent-spike filter).  W <= 254, so an
    // edge of delay 255 always bypasses it.
    {
        std::vector<int64_t> hist(256, 0);
        for (int64_t s = 0; s < g.e_slots; ++s) hist[g.d[s]]++;
        const int64_t allow = g.e_slots / 200;
        int64_t above = 0;
        int32_t w = max_delay;
        for (int32_t d = max_delay; d >= 1; --d) {
            if (above + hist[d] > allow) break;
            above += hist[d];
            w = d - 1;
        }
        g.window = std::min(std::max(w, 1), 254);
    }
    // Placeholders for empty rows, row-start bits, per-row order and exactness.
    const double two24 = 16777216.0;
    for (int64_t r = 0; r < N; ++r) {
        const int64_t a = row_ptr[r], b = a + std::max<int64_t>(indeg[r], 1);
        g.rowstart[a >> 3] |= uint8_t(1u << (a & 7));
        if (indeg[r] == 0) {
            g.src[a] = static_cast<int32_t>(r);
            g.w[a] = 0;
            g.d[a] = 1;
            continue;
        }
        bool sorted = true;
        for (int64_t s = a + 1; s < b; ++s)
            if (g.src[s] <= g.src[s - 1]) {
                sorted = false;
                break;
            }
        if (!sorted) {
            std::vector<int64_t> idx(b - a);
            for (int64_t s = a; s < b; ++s) idx[s - a] = s;
            std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return g.src[x] < g.src[y]; });
            std::vector<int32_t> ts(b - a), to(track ? b - a : 0);
            std::vector<uint16_t> tw(b - a);
            std::vector<uint8_t> td(b - a);
            for (int64_t k = 0; k < b - a; ++k) {
                ts[k] = g.src[idx[k]];
                tw[k] = g.w[idx[k]];
                td[k] = g.d[idx[k]];
                if (track) to[k] = orig[idx[k]];
            }
            for (int64_t k = 0; k < b - a; ++k) {
                g.src[a + k] = ts[k];
                g.w[a + k] = tw[k];
                g.d[a + k] = td[k];
                if (track) orig[a + k] = to[k];
            }
            for (int64_t s = a + 1; s < b; ++s)
                if (g.src[s] == g.src[s - 1]) {
                    err = "net_build: duplicate edge into vertex " + std::to_string(r);
                    return NET_E_ARG;
                }
        }
        // FP32 exactness: every partial sum of the row is a multiple of the
        // smallest FP16 spacing q present and bounded by sum |w|.
        double sum_abs = 0.0;
        int ulp_min = 1 << 20;
        for (int64_t s = a; s < b; ++s) {
            if ((g.w[s] & 0x7FFF) == 0) continue;
            sum_abs += fp16_abs(g.w[s]);
            ulp_min = std::min(ulp_min, fp16_ulp_log2(g.w[s]));
        }
        if (sum_abs > 0.0 && sum_abs > std::ldexp(two24, ulp_min)) g.exact = false;
    }
    if (track) {
        // plastic weights: integer multiples of 2^-20 (exact sums in any order)
        g.plastic = true;
        g.stdp_alpha = descs[0].stdp_alpha;
        g.stdp_beta = descs[0].stdp_beta;
        g.wq.assign(g.e_slots, 0);
        for (int64_t s = 0; s < g.e_slots; ++s) {
            if (orig[s] < 0) continue;
            const double k = static_cast<double>(fp16_abs(g.w[s])) * 1048576.0 * ((g.w[s] & 0x8000) ? -1.0 : 1.0);
            if (!(std::fabs(k) < 2147483648.0) || k != std::floor(k)) {
                err = "net_build: plastic weights must be multiples of 2^-20 below 2048 (edge " +
                      std::to_string(orig[s]) + ")";
                return NET_E_ARG;
            }
            g.wq[s] = static_cast<int32_t>(k);
        }
        g.slot_orig = std::move(orig);
        g.row_first.assign(N + 1, 0);
        for (int64_t r = 0; r <= N; ++r) g.row_first[r] = static_cast<int32_t>(row_ptr[r]);
    }
    g.chunk_row0.assign(g.n_chunks, 0);
    {
        int64_t r = 0;
        for (int64_t c = 0; c < g.n_chunks; ++c) {
            const int64_t s = c * kChunkEdges;
            while (r + 1 < N && row_ptr[r + 1] <= s) ++r;
            g.chunk_row0[c] = static_cast<int32_t>(r);
        }
    }

    // Per-vertex arrays and per-network constants.
    g.v0.assign(g.n_pad, 0.0f);
    g.drive_thr.assign(g.n_pad, 0u);
    g.i_ext.assign(g.n_pad, 0.0f);
    g.net_id.assign(g.n_pad, n_nets - 1);
    g.w0.assign(g.n_pad, 0.0);
    g.hh_m0.assign(g.n_pad, 0.0);
    g.hh_n0.assign(g.n_pad, 0.0);
    g.hh_h0.assign(g.n_pad, 0.0);
    g.params.resize(n_nets);
    for (int m = 0; m < n_nets; ++m) {
        const net_desc& d = descs[m];
        NetParams& p = g.params[m];
        p.decay = static_cast<float>(d.dt_ms / static_cast<double>(d.tau_ms));
        p.v_rest = d.v_rest;
        p.v_reset = d.v_reset;
        p.v_th = d.v_th;
        p.sigma = d.noise_sigma;
        p.drive_amp = d.drive_amp;
        p.dt_d = d.dt_ms;
        p.tau_c_d = d.tau_c_ms > 0.0f ? static_cast<double>(d.tau_c_ms) : 1e300;
        p.n_ref = d.n_ref;
        p.key_lo = static_cast<uint32_t>(d.seed);
        p.key_hi = static_cast<uint32_t>(d.seed >> 32);
        p.node_off = static_cast<int32_t>(g.node_off[m]);
        p.model = d.model;
        p.psc = d.psc;
        if (d.model == NET_MODEL_IZHIKEVICH) {
            g.any_izh = true;
            p.decay = 0.0f;
            p.n_ref = 0;
            p.iz_inv_c = 1.0 / static_cast<double>(d.iz_C);
            p.iz_k = d.iz_k;
            p.iz_vr = d.iz_vr;
            p.iz_vt = d.iz_vt;
            p.iz_a = d.iz_a;
            p.iz_b = d.iz_b;
            p.iz_d = d.iz_d;
            p.psc_a = d.psc_rate;
        }
        if (d.model == NET_MODEL_HODGKIN_HUXLEY) {
            g.any_hh = true;
            p.decay = 0.0f;
            p.n_ref = 0;
            p.hh_inv_c = 1.0 / static_cast<double>(d.hh_C);
            p.hh_gna = d.hh_gna;
            p.hh_gk = d.hh_gk;
            p.hh_gl = d.hh_gl;
            p.hh_ena = d.hh_ena;
            p.hh_ek = d.hh_ek;
            p.hh_el = d.hh_el;
            p.psc_a = d.psc_rate;
        }
        for (int32_t j = 0; j < d.n_nodes; ++j) {
            const int64_t k = g.node_off[m] + j;
            g.v0[k] = d.v0 ? d.v0[j] : d.v_rest;
            if (d.model == NET_MODEL_IZHIKEVICH) g.w0[k] = d.w0 ? static_cast<double>(d.w0[j]) : 0.0;
            if (d.model == NET_MODEL_HODGKIN_HUXLEY)
                hh_steady_gates(static_cast<double>(g.v0[k]), &g.hh_m0[k], &g.hh_n0[k], &g.hh_h0[k]);
            if (d.drive_rate_hz) {
                g.drive_thr[k] = pulse_threshold(d.drive_rate_hz[j], d.dt_ms);
                g.any_drive |= g.drive_thr[k] != 0u;
            }
            if (d.i_ext) {
                g.i_ext[k] = d.i_ext[j];
                g.any_iext |= d.i_ext[j] != 0.0f;
            }
            g.net_id[k] = m;
        }
    }
    return NET_OK;
}

}  // namespace geonet
