/*
 * FP64 CPU oracle for geometric-network simulation -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file.  The product path (the HIP library) shares no code,
 * header, table or helper with it.
 *
 * Plain, single-threaded, obviously-correct double-precision code that
 * follows Buibas & Silva, "A framework for simulating and estimating the
 * state and functional topology of complex dynamic geometric networks":
 *   - state transition y_j(t+dt) = H_j(y_j(t), Y_j(t), u_j(t), Theta_j)
 *     (Section 2, Eq. Htrans) with the leaky integrate-and-fire vertex of
 *     Section 3.1 (voltage decays to a target, threshold, reset at the next
 *     step) integrated by the Euler rule of Section 3.1;
 *   - spike detection spd(V) = 1 iff V >= threshold (Section 3.2, Eq. spd);
 *   - delayed weighted input: the sum over in-edges k -> j of
 *     w_kj * spd(V_k(t - tau_kj)) (Section 3.2, Eq. izpsc, last term; the set
 *     Y_j of Eq. Yjset), delays tau_ij = |x_i - x_j| / s (Eq. delaydist);
 *   - calcium transition c + dt*(-c/tau_c + spd) and the camera average over
 *     the steps of one frame, fluorescence n*c + b + N(0, gamma^2)
 *     (Section 3.3);
 *   - counter-based random numbers: Philox4x32-10 from Salmon, Moraes,
 *     Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11),
 *     Gaussian variates by Box & Muller (1958).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   R1  refractory: after the spike step the vertex is held at V_reset for
 *       n_ref further steps, during which arriving input is discarded.
 *   R2  synaptic input is an instantaneous jump of V by the delivered sum
 *       (by analogy with the PSC increment r += w upon arrival).
 *   R3  delay in steps d = max(1, ceil(dist / (s*dt))); d <= 255.
 *   R4  control u_j(t) = i_ext_j + A * [Philox x0 < floor(rate*dt*2^32)].
 *   R5  state noise: sigma * xi added to V every integrated step.
 *   R6  frames: frame(t) = floor(t*num/den); a frame's value is the mean of
 *       c_j(t) over its steps.
 *
 * Delivery here is event-driven: when vertex i fires at step t its weights
 * are pushed into a per-target inbox slot (t + d) mod 256.  This is a
 * different formulation from a pull over in-edges, on purpose.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_RING 256

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, Section 3.3 of that paper).          */
/* ------------------------------------------------------------------------ */
static void philox_round(uint32_t x[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x[1] ^ k[0];
    uint32_t y2 = hi0 ^ x[3] ^ k[1];
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;   /* Weyl key schedule */
            k[1] += 0xBB67AE85u;
        }
        philox_round(x, k);
    }
    out[0] = x[0];
    out[1] = x[1];
    out[2] = x[2];
    out[3] = x[3];
}

/* Uniform in (0,1) from the top 24 bits; exact in both float and double. */
double orc_u01_24(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }

/* Box-Muller: one standard normal from two 32-bit draws. */
double orc_box_muller(uint32_t a, uint32_t b) {
    double u1 = orc_u01_24(a), u2 = orc_u01_24(b);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* Drive threshold: an event when a 32-bit draw is below floor(p * 2^32). */
uint32_t orc_drive_threshold(double rate_hz, double dt_ms) {
    double p = rate_hz * (dt_ms * 1e-3);
    double t = floor(p * 4294967296.0);
    if (!(t > 0.0)) return 0u;
    if (t >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)t;
}

/* Eq. delaydist with the step rule R3.  Returns -1 if the delay exceeds 255. */
int32_t orc_delay_steps(const double* xi, const double* xj, int dims,
                        double v_um_per_ms, double dt_ms) {
    double s2 = 0.0;
    for (int k = 0; k < dims; ++k) {
        double d = xi[k] - xj[k];
        s2 = s2 + d * d;
    }
    double dist = sqrt(s2);
    double step_len = v_um_per_ms * dt_ms;
    double q = ceil(dist / step_len);
    if (q < 1.0) q = 1.0;
    if (q > 255.0) return -1;
    return (int32_t)q;
}

/* ------------------------------------------------------------------------ */
/* Network state                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    /* out-edges of each source (adjacency for the event-driven push) */
    int64_t* out_start;     /* [n+1] */
    int32_t* out_dst;       /* [E] */
    double* out_w;          /* [E] */
    int32_t* out_d;         /* [E] */
    /* parameters */
    double dt, tau, v_rest, v_reset, v_th, drive_amp, sigma, tau_c;
    int32_t n_ref;
    uint32_t key[2];
    uint32_t* drive_thr;    /* [n] */
    double* i_ext;          /* [n] */
    int64_t frame_num, frame_den;
    /* state */
    int64_t t;
    double* V;              /* [n] */
    int32_t* ref;           /* [n] remaining refractory steps */
    double* inbox;          /* [n * 256] input arriving at (slot) */
    double* c;              /* [n] calcium */
    double* acc;            /* [n] frame accumulator */
    int64_t acc_steps;
    double* frames;         /* [cap][n] frame means */
    int64_t frames_cap, n_frames;
    int64_t delivered;      /* count of (spike, edge) deliveries pushed */
} orc_net;

static void* xcalloc(size_t n, size_t s) {
    void* p = calloc(n ? n : 1, s);
    return p;
}

/*
 * Create a network.  Edges are (src[e] -> dst[e], w[e]); delays are given
 * (delay != NULL) or computed from positions by orc_delay_steps.
 * drive_rate_hz, i_ext, v0 may be NULL.  Returns NULL on bad input or a delay
 * above 255.
 */
void* orc_create(int32_t n, int32_t dims, const double* pos, int64_t n_edges,
                 const int32_t* src, const int32_t* dst, const float* w,
                 const uint8_t* delay, double v_um_per_ms, double dt_ms,
                 double tau_ms, double v_rest, double v_reset, double v_th,
                 int32_t n_ref, const float* drive_rate_hz, double drive_amp,
                 const float* i_ext, double noise_sigma, uint64_t seed,
                 const float* v0, double tau_c_ms, int64_t frame_num,
                 int64_t frame_den, int64_t frames_cap) {
    if (n <= 0 || n_edges < 0 || dt_ms <= 0.0) return NULL;
    orc_net* h = (orc_net*)xcalloc(1, sizeof(orc_net));
    h->n = n;
    h->out_start = (int64_t*)xcalloc((size_t)n + 1, sizeof(int64_t));
    h->out_dst = (int32_t*)xcalloc((size_t)n_edges, sizeof(int32_t));
    h->out_w = (double*)xcalloc((size_t)n_edges, sizeof(double));
    h->out_d = (int32_t*)xcalloc((size_t)n_edges, sizeof(int32_t));
    for (int64_t e = 0; e < n_edges; ++e) {
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n || src[e] == dst[e]) goto fail;
        h->out_start[src[e] + 1]++;
    }
    for (int32_t i = 0; i < n; ++i) h->out_start[i + 1] += h->out_start[i];
    {
        int64_t* fill = (int64_t*)xcalloc((size_t)n, sizeof(int64_t));
        for (int32_t i = 0; i < n; ++i) fill[i] = h->out_start[i];
        for (int64_t e = 0; e < n_edges; ++e) {
            int32_t d;
            if (delay) {
                d = delay[e];
                if (d < 1) d = 1;
            } else {
                d = orc_delay_steps(pos + (int64_t)src[e] * dims, pos + (int64_t)dst[e] * dims,
                                    dims, v_um_per_ms, dt_ms);
                if (d < 0) {
                    free(fill);
                    goto fail;
                }
            }
            int64_t o = fill[src[e]]++;
            h->out_dst[o] = dst[e];
            h->out_w[o] = (double)w[e];
            h->out_d[o] = d;
        }
        free(fill);
    }
    h->dt = dt_ms;
    h->tau = tau_ms;
    h->v_rest = v_rest;
    h->v_reset = v_reset;
    h->v_th = v_th;
    h->n_ref = n_ref;
    h->drive_amp = drive_amp;
    h->sigma = noise_sigma;
    h->tau_c = tau_c_ms;
    h->key[0] = (uint32_t)seed;
    h->key[1] = (uint32_t)(seed >> 32);
    h->frame_num = frame_num;
    h->frame_den = frame_den > 0 ? frame_den : 1;
    h->drive_thr = (uint32_t*)xcalloc((size_t)n, sizeof(uint32_t));
    h->i_ext = (double*)xcalloc((size_t)n, sizeof(double));
    for (int32_t j = 0; j < n; ++j) {
        h->drive_thr[j] = drive_rate_hz ? orc_drive_threshold(drive_rate_hz[j], dt_ms) : 0u;
        h->i_ext[j] = i_ext ? (double)i_ext[j] : 0.0;
    }
    h->V = (double*)xcalloc((size_t)n, sizeof(double));
    h->ref = (int32_t*)xcalloc((size_t)n, sizeof(int32_t));
    h->inbox = (double*)xcalloc((size_t)n * ORC_RING, sizeof(double));
    h->c = (double*)xcalloc((size_t)n, sizeof(double));
    h->acc = (double*)xcalloc((size_t)n, sizeof(double));
    for (int32_t j = 0; j < n; ++j) h->V[j] = v0 ? (double)v0[j] : v_rest;
    h->frames_cap = frames_cap > 0 ? frames_cap : 0;
    h->frames = (double*)xcalloc((size_t)(h->frames_cap ? h->frames_cap : 1) * n, sizeof(double));
    return h;
fail:
    free(h->out_start);
    free(h->out_dst);
    free(h->out_w);
    free(h->out_d);
    free(h);
    return NULL;
}

void orc_free(void* p) {
    orc_net* h = (orc_net*)p;
    if (!h) return;
    free(h->out_start);
    free(h->out_dst);
    free(h->out_w);
    free(h->out_d);
    free(h->drive_thr);
    free(h->i_ext);
    free(h->V);
    free(h->ref);
    free(h->inbox);
    free(h->c);
    free(h->acc);
    free(h->frames);
    free(h);
}

/* Delay of the out-edge list entry for (src, dst), or -1 (for tests). */
int32_t orc_edge_delay(void* p, int32_t src, int32_t dst) {
    orc_net* h = (orc_net*)p;
    for (int64_t o = h->out_start[src]; o < h->out_start[src + 1]; ++o)
        if (h->out_dst[o] == dst) return h->out_d[o];
    return -1;
}

/*
 * Advance n_steps.  Optional per-step records (row t - t_start):
 *   raster [n_steps][n] uint8   spd(V_j(t))
 *   v_rec  [n_steps][n] double  V_j(t) at the start of step t
 *   i_rec  [n_steps][n] double  delivered input I_j(t)
 * force_raster (optional, [n_steps][n] uint8): when given, the spike
 * decision of each step is taken from it instead of from V (open-loop /
 * teacher-forced use); everything else is unchanged.
 */
void orc_step_n(void* p, int64_t n_steps, uint8_t* raster, double* v_rec, double* i_rec,
                const uint8_t* force_raster) {
    orc_net* h = (orc_net*)p;
    const int32_t n = h->n;
    uint8_t* s = (uint8_t*)xcalloc((size_t)n, 1);
    const double decay = h->dt / h->tau;
    for (int64_t k = 0; k < n_steps; ++k) {
        const int64_t t = h->t;
        const int slot = (int)(t % ORC_RING);
        /* Eq. spd on the state at the start of the step. */
        for (int32_t j = 0; j < n; ++j) {
            s[j] = force_raster ? (force_raster[k * n + j] ? 1 : 0) : (h->V[j] >= h->v_th ? 1 : 0);
            if (raster) raster[k * n + j] = s[j];
            if (v_rec) v_rec[k * n + j] = h->V[j];
        }
        /* Push this step's spikes to their targets' future inbox slots. */
        for (int32_t i = 0; i < n; ++i) {
            if (!s[i]) continue;
            for (int64_t o = h->out_start[i]; o < h->out_start[i + 1]; ++o) {
                int32_t dslot = (int)((t + h->out_d[o]) % ORC_RING);
                h->inbox[(int64_t)h->out_dst[o] * ORC_RING + dslot] += h->out_w[o];
                h->delivered++;
            }
        }
        /* Camera integration: accumulate c_j(t) into the current frame. */
        int64_t f_now = (t * h->frame_num) / h->frame_den;
        int64_t f_next = ((t + 1) * h->frame_num) / h->frame_den;
        for (int32_t j = 0; j < n; ++j) h->acc[j] += h->c[j];
        h->acc_steps++;
        if (f_next != f_now && h->frame_num > 0) {
            if (f_now < h->frames_cap)
                for (int32_t j = 0; j < n; ++j) h->frames[f_now * n + j] = h->acc[j] / (double)h->acc_steps;
            for (int32_t j = 0; j < n; ++j) h->acc[j] = 0.0;
            h->acc_steps = 0;
            if (f_now + 1 > h->n_frames) h->n_frames = f_now + 1;
        }
        for (int32_t j = 0; j < n; ++j) {
            /* input arriving now (all its pushes happened at earlier steps) */
            double in = h->inbox[(int64_t)j * ORC_RING + slot];
            h->inbox[(int64_t)j * ORC_RING + slot] = 0.0;
            if (i_rec) i_rec[k * n + j] = in;
            /* calcium transition, Section 3.3 */
            h->c[j] = h->c[j] + h->dt * (-h->c[j] / h->tau_c + (double)s[j]);
            /* LIF transition with refractory hold (R1) */
            if (s[j]) {
                h->V[j] = h->v_reset;
                h->ref[j] = h->n_ref;
            } else if (h->ref[j] > 0) {
                h->V[j] = h->v_reset;
                h->ref[j] -= 1;
            } else {
                uint32_t ctr[4] = {(uint32_t)j, (uint32_t)t, (uint32_t)(t >> 32), 0u};
                uint32_t r[4];
                orc_philox4x32_10(ctr, h->key, r);
                double u = h->i_ext[j] + ((r[0] < h->drive_thr[j]) ? h->drive_amp : 0.0);
                double xi = orc_box_muller(r[1], r[2]);
                h->V[j] = h->V[j] + decay * (h->v_rest - h->V[j]) + in + u + h->sigma * xi;
            }
        }
        h->t = t + 1;
    }
    free(s);
}

int64_t orc_time(void* p) { return ((orc_net*)p)->t; }
int64_t orc_delivered(void* p) { return ((orc_net*)p)->delivered; }
int64_t orc_frames_done(void* p) { return ((orc_net*)p)->n_frames; }

void orc_get_v(void* p, double* out) {
    orc_net* h = (orc_net*)p;
    memcpy(out, h->V, (size_t)h->n * sizeof(double));
}
void orc_get_ref(void* p, int32_t* out) {
    orc_net* h = (orc_net*)p;
    memcpy(out, h->ref, (size_t)h->n * sizeof(int32_t));
}
void orc_get_c(void* p, double* out) {
    orc_net* h = (orc_net*)p;
    memcpy(out, h->c, (size_t)h->n * sizeof(double));
}

/* Frame means [n_frames][n] (capped at the capacity given at creation). */
int64_t orc_get_frames(void* p, double* out, int64_t max_frames) {
    orc_net* h = (orc_net*)p;
    int64_t nf = h->n_frames < h->frames_cap ? h->n_frames : h->frames_cap;
    if (nf > max_frames) nf = max_frames;
    memcpy(out, h->frames, (size_t)(nf * h->n) * sizeof(double));
    return nf;
}

/*
 * Fluorescence observation (Section 3.3): F = n*cbar + b + gamma*xi with
 * xi from Philox counter (j, frame, 0, 1).  cbar: [n_frames][n].
 */
void orc_fluorescence(const double* cbar, int64_t n_frames, int32_t n, int64_t frame0,
                      double gain, double offset, double gamma, uint64_t seed, double* out) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t f = 0; f < n_frames; ++f) {
        int64_t fa = f + frame0;
        for (int32_t j = 0; j < n; ++j) {
            uint32_t ctr[4] = {(uint32_t)j, (uint32_t)fa, (uint32_t)(fa >> 32), 1u};
            uint32_t r[4];
            orc_philox4x32_10(ctr, key, r);
            out[f * n + j] = gain * cbar[f * n + j] + offset + gamma * orc_box_muller(r[0], r[1]);
        }
    }
}
