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
 * Izhikevich vertex (Section 3.1, Eq. izsimple; with post-synaptic current
 * states of Section 3.2, Eqs. simplepsc, alphapsc and izpsc), selected per
 * network by orc_set_izhikevich:
 *   spike when V >= V_peak (Eq. spd); then V <- c and W <- W + d;
 *   otherwise Euler: V <- V + dt*(1/C)*[k(V-Vr)(V-Vt) - W + r + U] (+ sigma*xi)
 *                    W <- W + dt*a*(b(V-Vr) - W)
 *   PSC (every step, from the state at t):
 *     none  (psc 0): the delivered sum jumps V directly (as R2);
 *     exp   (psc 1): r <- r - dt*a_s*r + I      (dr/dt = -a_s r, r += w on arrival)
 *     alpha (psc 2): r <- r + dt*p,  p <- p + dt*(-a_s^2 r - 2 a_s p) + I
 *   R16 an arriving spike is an impulse: it adds its weight to r (exp) or p
 *       (alpha) at once, as Eqs. simplepsc and alphapsc state it; Eq. izpsc's
 *       transition writes the sum inside dt*( ), which would make the PSC
 *       amplitude depend on the step, and is read as that same impulse.
 *   R17 control U = i_ext + A*pulse enters the bracket as a current; the
 *       state noise sigma*xi is added to V after it (as R5).
 * Izhikevich state is FP64 here and in the library.
 *
 * Hodgkin-Huxley vertex (Section 3.1: four states V, m, n, h; the paper's
 * benchmark steps it at dt = 0.03 ms), selected by orc_set_hodgkin_huxley,
 * Euler-stepped from the state at t, with the same PSC kinds:
 *   C dV/dt = -gNa m^3 h (V - ENa) - gK n^4 (V - EK) - gL (V - EL) + r + U
 *   dx/dt = alpha_x(V) (1 - x) - beta_x(V) x,  x in {m, h, n}, with
 *   alpha_m = 0.1 (V + 40) / (1 - exp(-(V + 40)/10)),  beta_m = 4 exp(-(V + 65)/18)
 *   alpha_h = 0.07 exp(-(V + 65)/20),  beta_h = 1 / (1 + exp(-(V + 35)/10))
 *   alpha_n = 0.01 (V + 55) / (1 - exp(-(V + 55)/10)), beta_n = 0.125 exp(-(V + 65)/80)
 *   (mV, ms, uF/cm^2, mS/cm^2, uA/cm^2; alpha_m and alpha_n take their limits
 *   1 and 0.1 where the denominator vanishes, at V = -40 and V = -55 exactly).
 *   R20 spd for this vertex is the upward crossing of V_th (V(t) >= V_th
 *       and V(t-1) < V_th): V stays above any threshold for about a
 *       millisecond, so the level test of Eq. spd would signal every step of
 *       an action potential; there is no reset.
 * HH state is FP64 here and in the library.
 *
 * Spike-timing-dependent plasticity (Section 3.2, "Plasticity"; Eqs.
 * omegatrans and Gparams), switched on per network by orc_set_stdp:
 *   s_j, the time since j's last spike: s_j(t+1) = (1 - spd(V_j(t))) (s_j(t) + dt),
 *       s_j(0) = 0, so s_j(u) = (u - t_last - 1) dt with t_last j's last
 *       spike before step u (u dt without one; 0 for u <= 0);
 *   q_ij(t) = (s_i(t - d_ij) - s_j(t)) * max(spd(V_i(t - d_ij)), spd(V_j(t)));
 *   w_ij(t+1) = w_ij(t) + dt * alpha * sign(q) * exp(-beta |q|).
 *   R21 weights are kept as integer multiples of Q = 2^-20 (the initial FP16
 *       weights are such multiples); every increment is rounded to the
 *       nearest multiple (ties to even) before it is added, so every sum of
 *       weights is exact and the delivered input does not depend on the
 *       order of additions.  A spike delivered at step t carries w(t), the
 *       weight at its arrival; the update of step t follows the delivery.
 * Delivery of a plastic network keeps per ring slot the list of edges whose
 * spike arrives then (instead of a sum of weights).
 *
 * Delivery here is event-driven: when vertex i fires at step t its weights
 * are pushed into a per-target inbox slot (t + d) mod 256.  This is a
 * different formulation from a pull over in-edges, on purpose.
 *
 * Threads: single-threaded unless orc_set_threads(k > 1) is called (tests
 * of large networks do, to finish in reasonable time).  Then only the loops
 * over vertices whose iterations touch nothing but their own vertex (the
 * spike test and the vertex transition) are split over k threads; the push
 * of spikes into the inboxes stays one serial loop in vertex order, so every
 * sum is formed in the same order and the results are bit-identical for any
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_RING 256

static int orc_threads = 1;

/* Threads for the per-vertex loops of orc_step_n (1 = plain serial code). */
void orc_set_threads(int32_t k) { orc_threads = k > 1 ? k : 1; }
int32_t orc_get_threads(void) { return orc_threads; }

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
    /* Izhikevich vertex (model 1) with an optional PSC */
    int32_t model, psc;
    double iz_C, iz_k, iz_vr, iz_vt, iz_a, iz_b, iz_d, psc_a;
    double* W;              /* [n] recovery variable */
    double* r;              /* [n] PSC current */
    double* p;              /* [n] PSC derivative (alpha) */
    /* Hodgkin-Huxley vertex (model 2) */
    double hh_C, hh_gna, hh_gk, hh_gl, hh_ena, hh_ek, hh_el;
    double *hm, *hn, *hh;   /* [n] gating variables */
    double* vprev;          /* [n] V(t-1) for the crossing test */
    /* STDP */
    int32_t plastic;
    double stdp_alpha, stdp_beta;
    int64_t n_edges;
    int64_t* wq;            /* [E] weight of out-edge o, in units of 2^-20 */
    int64_t* stamp;         /* [E] last step at which out-edge o was updated */
    int64_t* in_start;      /* [n+1] in-edges of each target ... */
    int64_t* in_list;       /* [E]   ... as out-edge indices */
    int32_t* out_src;       /* [E] source of out-edge o */
    int64_t* arr[ORC_RING]; /* out-edges whose spike arrives at slot k */
    int64_t arr_cnt[ORC_RING], arr_cap[ORC_RING];
    int64_t** spk;          /* [n] spike steps of each vertex (all of them) */
    int64_t *spk_cnt, *spk_cap;
    int64_t* qin;           /* [n] delivered sum of this step in units of 2^-20 */
} orc_net;

#define ORC_WQ 1048576.0   /* 1 / Q, Q = 2^-20 */

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
    h->n_edges = n_edges;
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

/*
 * Switch the network to the Izhikevich vertex: iz = {C, k, Vr, Vt, a, b, d}
 * (V_peak and c are the network's v_th and v_reset); psc 0 none, 1 exp,
 * 2 alpha, with rate psc_a (1/ms); w0 = initial W or NULL (0).  Returns 0,
 * or -1 for a bad argument.
 */
int32_t orc_set_izhikevich(void* ph, int32_t psc, const double* iz, double psc_a, const float* w0) {
    orc_net* h = (orc_net*)ph;
    if (!h || !iz || psc < 0 || psc > 2 || !(iz[0] > 0.0)) return -1;
    h->model = 1;
    h->psc = psc;
    h->iz_C = iz[0];
    h->iz_k = iz[1];
    h->iz_vr = iz[2];
    h->iz_vt = iz[3];
    h->iz_a = iz[4];
    h->iz_b = iz[5];
    h->iz_d = iz[6];
    h->psc_a = psc_a;
    if (!h->W) h->W = (double*)xcalloc((size_t)h->n, sizeof(double));
    if (!h->r) h->r = (double*)xcalloc((size_t)h->n, sizeof(double));
    if (!h->p) h->p = (double*)xcalloc((size_t)h->n, sizeof(double));
    for (int32_t j = 0; j < h->n; ++j) h->W[j] = w0 ? (double)w0[j] : 0.0;
    return 0;
}

/* HH rate functions (see the header). */
static double hh_alpha_m(double V) {
    const double x = V + 40.0;
    return x == 0.0 ? 1.0 : 0.1 * x / (1.0 - exp(-x / 10.0));
}
static double hh_beta_m(double V) { return 4.0 * exp(-(V + 65.0) / 18.0); }
static double hh_alpha_h(double V) { return 0.07 * exp(-(V + 65.0) / 20.0); }
static double hh_beta_h(double V) { return 1.0 / (1.0 + exp(-(V + 35.0) / 10.0)); }
static double hh_alpha_n(double V) {
    const double x = V + 55.0;
    return x == 0.0 ? 0.1 : 0.01 * x / (1.0 - exp(-x / 10.0));
}
static double hh_beta_n(double V) { return 0.125 * exp(-(V + 65.0) / 80.0); }

/*
 * Switch the network to the Hodgkin-Huxley vertex: hh = {C, gNa, gK, gL,
 * ENa, EK, EL}; the threshold of the crossing test is the network's v_th;
 * psc and psc_a as for the Izhikevich vertex.  m, n, h start at their
 * steady state for V(0); V(-1) is taken as V(0).  Returns 0 or -1.
 */
int32_t orc_set_hodgkin_huxley(void* ph, int32_t psc, const double* hh, double psc_a) {
    orc_net* h = (orc_net*)ph;
    if (!h || !hh || psc < 0 || psc > 2 || !(hh[0] > 0.0)) return -1;
    h->model = 2;
    h->psc = psc;
    h->psc_a = psc_a;
    h->hh_C = hh[0];
    h->hh_gna = hh[1];
    h->hh_gk = hh[2];
    h->hh_gl = hh[3];
    h->hh_ena = hh[4];
    h->hh_ek = hh[5];
    h->hh_el = hh[6];
    if (!h->r) h->r = (double*)xcalloc((size_t)h->n, sizeof(double));
    if (!h->p) h->p = (double*)xcalloc((size_t)h->n, sizeof(double));
    if (!h->hm) h->hm = (double*)xcalloc((size_t)h->n, sizeof(double));
    if (!h->hn) h->hn = (double*)xcalloc((size_t)h->n, sizeof(double));
    if (!h->hh) h->hh = (double*)xcalloc((size_t)h->n, sizeof(double));
    if (!h->vprev) h->vprev = (double*)xcalloc((size_t)h->n, sizeof(double));
    for (int32_t j = 0; j < h->n; ++j) {
        const double V = h->V[j];
        h->hm[j] = hh_alpha_m(V) / (hh_alpha_m(V) + hh_beta_m(V));
        h->hh[j] = hh_alpha_h(V) / (hh_alpha_h(V) + hh_beta_h(V));
        h->hn[j] = hh_alpha_n(V) / (hh_alpha_n(V) + hh_beta_n(V));
        h->vprev[j] = V;
    }
    return 0;
}

void orc_get_hh(void* ph, double* m, double* n, double* hg) {
    orc_net* h = (orc_net*)ph;
    if (!h->hm) return;
    if (m) memcpy(m, h->hm, (size_t)h->n * sizeof(double));
    if (n) memcpy(n, h->hn, (size_t)h->n * sizeof(double));
    if (hg) memcpy(hg, h->hh, (size_t)h->n * sizeof(double));
}

static void push_i64(int64_t** a, int64_t* cnt, int64_t* cap, int64_t v) {
    if (*cnt == *cap) {
        *cap = *cap ? 2 * *cap : 16;
        *a = (int64_t*)realloc(*a, (size_t)*cap * sizeof(int64_t));
    }
    (*a)[(*cnt)++] = v;
}

/*
 * Make the network's weights plastic (STDP above) with rates alpha (weight
 * per ms) and beta (1/ms).  Needs the LIF vertex, no step taken yet, and
 * every weight an integer multiple of 2^-20 below 2048 in magnitude.
 * Returns 0 or -1.
 */
int32_t orc_set_stdp(void* ph, double alpha, double beta) {
    orc_net* h = (orc_net*)ph;
    if (!h || h->model != 0 || h->t != 0) return -1;
    const int64_t E = h->n_edges;
    h->wq = (int64_t*)xcalloc((size_t)E, sizeof(int64_t));
    h->stamp = (int64_t*)xcalloc((size_t)E, sizeof(int64_t));
    for (int64_t o = 0; o < E; ++o) {
        const double k = h->out_w[o] * ORC_WQ;
        if (!(fabs(h->out_w[o]) < 2048.0) || k != floor(k)) return -1;
        h->wq[o] = (int64_t)k;
        h->stamp[o] = -1;
    }
    h->out_src = (int32_t*)xcalloc((size_t)E, sizeof(int32_t));
    for (int32_t i = 0; i < h->n; ++i)
        for (int64_t o = h->out_start[i]; o < h->out_start[i + 1]; ++o) h->out_src[o] = i;
    h->in_start = (int64_t*)xcalloc((size_t)h->n + 1, sizeof(int64_t));
    h->in_list = (int64_t*)xcalloc((size_t)E, sizeof(int64_t));
    for (int64_t o = 0; o < E; ++o) h->in_start[h->out_dst[o] + 1]++;
    for (int32_t j = 0; j < h->n; ++j) h->in_start[j + 1] += h->in_start[j];
    {
        int64_t* fill = (int64_t*)xcalloc((size_t)h->n, sizeof(int64_t));
        for (int32_t j = 0; j < h->n; ++j) fill[j] = h->in_start[j];
        for (int64_t o = 0; o < E; ++o) h->in_list[fill[h->out_dst[o]]++] = o;
        free(fill);
    }
    h->spk = (int64_t**)xcalloc((size_t)h->n, sizeof(int64_t*));
    h->spk_cnt = (int64_t*)xcalloc((size_t)h->n, sizeof(int64_t));
    h->spk_cap = (int64_t*)xcalloc((size_t)h->n, sizeof(int64_t));
    h->qin = (int64_t*)xcalloc((size_t)h->n, sizeof(int64_t));
    h->stdp_alpha = alpha;
    h->stdp_beta = beta;
    h->plastic = 1;
    return 0;
}

/* s_i(u): time since i's last spike before step u (see the header). */
static double stdp_s(const orc_net* h, int32_t i, int64_t u) {
    if (u <= 0) return 0.0;
    const int64_t* a = h->spk[i];
    int64_t lo = 0, hi = h->spk_cnt[i];          /* first index with a[k] >= u */
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (a[mid] < u) lo = mid + 1; else hi = mid;
    }
    if (lo == 0) return (double)u * h->dt;
    return (double)(u - a[lo - 1] - 1) * h->dt;
}

/* The STDP update of out-edge o at step t (q as in the header). */
static void stdp_update(orc_net* h, int64_t o, int32_t i, int64_t t) {
    const int32_t j = h->out_dst[o];
    const double q = stdp_s(h, i, t - h->out_d[o]) - stdp_s(h, j, t);
    const double sg = q > 0.0 ? 1.0 : (q < 0.0 ? -1.0 : 0.0);
    const double dw = h->dt * h->stdp_alpha * sg * exp(-h->stdp_beta * fabs(q));
    h->wq[o] += (int64_t)nearbyint(dw * ORC_WQ);
    h->stamp[o] = t;
}

/* Current weights of the edges (src[e] -> dst[e]) (plastic networks). */
void orc_get_weights(void* ph, const int32_t* src, const int32_t* dst, int64_t m, double* out) {
    orc_net* h = (orc_net*)ph;
    for (int64_t e = 0; e < m; ++e) {
        out[e] = 0.0;
        for (int64_t o = h->out_start[src[e]]; o < h->out_start[src[e] + 1]; ++o)
            if (h->out_dst[o] == dst[e]) {
                out[e] = h->plastic ? (double)h->wq[o] / ORC_WQ : h->out_w[o];
                break;
            }
    }
}

void orc_get_izh(void* ph, double* W, double* r, double* p) {
    orc_net* h = (orc_net*)ph;
    if (!h->W) return;
    if (W) memcpy(W, h->W, (size_t)h->n * sizeof(double));
    if (r) memcpy(r, h->r, (size_t)h->n * sizeof(double));
    if (p) memcpy(p, h->p, (size_t)h->n * sizeof(double));
}

void orc_free(void* p) {
    orc_net* h = (orc_net*)p;
    if (!h) return;
    free(h->W);
    free(h->r);
    free(h->p);
    free(h->hm);
    free(h->hn);
    free(h->hh);
    free(h->vprev);
    if (h->plastic) {
        for (int k = 0; k < ORC_RING; ++k) free(h->arr[k]);
        for (int32_t j = 0; j < h->n; ++j) free(h->spk[j]);
        free(h->spk);
        free(h->spk_cnt);
        free(h->spk_cap);
        free(h->qin);
        free(h->in_start);
        free(h->in_list);
        free(h->out_src);
    }
    free(h->wq);
    free(h->stamp);
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
#pragma omp parallel for schedule(static) num_threads(orc_threads) if (orc_threads > 1 && n >= 4096)
        for (int32_t j = 0; j < n; ++j) {
            if (force_raster)
                s[j] = force_raster[k * n + j] ? 1 : 0;
            else if (h->model == 2)
                s[j] = (h->V[j] >= h->v_th && h->vprev[j] < h->v_th) ? 1 : 0;   /* R20: upward crossing */
            else
                s[j] = h->V[j] >= h->v_th ? 1 : 0;
            if (raster) raster[k * n + j] = s[j];
            if (v_rec) v_rec[k * n + j] = h->V[j];
        }
        if (h->plastic) {
            /* arrivals of step t, with the weights they carry now */
            int64_t* list = h->arr[slot];
            const int64_t cnt = h->arr_cnt[slot];
            for (int64_t a = 0; a < cnt; ++a) h->qin[h->out_dst[list[a]]] += h->wq[list[a]];
            for (int32_t j = 0; j < n; ++j) {
                h->inbox[(int64_t)j * ORC_RING + slot] = (double)h->qin[j] / ORC_WQ;
                h->qin[j] = 0;
            }
            /* the update of step t: every edge whose spike arrives now, and every
               in-edge of a vertex that fires now (once per edge) */
            for (int64_t a = 0; a < cnt; ++a) {
                const int64_t o = list[a];
                if (h->stamp[o] != t) stdp_update(h, o, h->out_src[o], t);
            }
            h->arr_cnt[slot] = 0;
            for (int32_t j = 0; j < n; ++j) {
                if (!s[j]) continue;
                for (int64_t k2 = h->in_start[j]; k2 < h->in_start[j + 1]; ++k2) {
                    const int64_t o = h->in_list[k2];
                    if (h->stamp[o] == t) continue;
                    stdp_update(h, o, h->out_src[o], t);
                }
            }
            /* this step's spikes: queued for their arrival steps, and recorded */
            for (int32_t i = 0; i < n; ++i) {
                if (!s[i]) continue;
                for (int64_t o = h->out_start[i]; o < h->out_start[i + 1]; ++o) {
                    const int dslot = (int)((t + h->out_d[o]) % ORC_RING);
                    push_i64(&h->arr[dslot], &h->arr_cnt[dslot], &h->arr_cap[dslot], o);
                    h->delivered++;
                }
                push_i64(&h->spk[i], &h->spk_cnt[i], &h->spk_cap[i], t);
            }
        } else {
        /* Push this step's spikes to their targets' future inbox slots. */
        for (int32_t i = 0; i < n; ++i) {
            if (!s[i]) continue;
            for (int64_t o = h->out_start[i]; o < h->out_start[i + 1]; ++o) {
                int32_t dslot = (int)((t + h->out_d[o]) % ORC_RING);
                h->inbox[(int64_t)h->out_dst[o] * ORC_RING + dslot] += h->out_w[o];
                h->delivered++;
            }
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
#pragma omp parallel for schedule(static) num_threads(orc_threads) if (orc_threads > 1 && n >= 4096)
        for (int32_t j = 0; j < n; ++j) {
            /* input arriving now (all its pushes happened at earlier steps) */
            double in = h->inbox[(int64_t)j * ORC_RING + slot];
            h->inbox[(int64_t)j * ORC_RING + slot] = 0.0;
            if (i_rec) i_rec[k * n + j] = in;
            /* calcium transition, Section 3.3 */
            h->c[j] = h->c[j] + h->dt * (-h->c[j] / h->tau_c + (double)s[j]);
            if (h->model == 2) {
                /* Hodgkin-Huxley transition, Euler from the state at t; no reset */
                const double V = h->V[j], r = h->r[j], pp = h->p[j];
                const double m = h->hm[j], nn = h->hn[j], hg = h->hh[j];
                if (h->psc == 1) {
                    h->r[j] = r - h->dt * h->psc_a * r + in;
                } else if (h->psc == 2) {
                    h->r[j] = r + h->dt * pp;
                    h->p[j] = pp + h->dt * (-h->psc_a * h->psc_a * r - 2.0 * h->psc_a * pp) + in;
                }
                uint32_t ctr[4] = {(uint32_t)j, (uint32_t)t, (uint32_t)(t >> 32), 0u};
                uint32_t rr[4];
                orc_philox4x32_10(ctr, h->key, rr);
                const double U = h->i_ext[j] + ((rr[0] < h->drive_thr[j]) ? h->drive_amp : 0.0);
                const double xi = orc_box_muller(rr[1], rr[2]);
                const double syn = h->psc == 0 ? 0.0 : r;
                const double i_na = h->hh_gna * m * m * m * hg * (V - h->hh_ena);
                const double i_k = h->hh_gk * nn * nn * nn * nn * (V - h->hh_ek);
                const double i_l = h->hh_gl * (V - h->hh_el);
                double Vn = V + h->dt * (1.0 / h->hh_C) * (-i_na - i_k - i_l + syn + U);
                if (h->psc == 0) Vn = Vn + in;
                h->V[j] = Vn + h->sigma * xi;
                h->vprev[j] = V;
                h->hm[j] = m + h->dt * (hh_alpha_m(V) * (1.0 - m) - hh_beta_m(V) * m);
                h->hh[j] = hg + h->dt * (hh_alpha_h(V) * (1.0 - hg) - hh_beta_h(V) * hg);
                h->hn[j] = nn + h->dt * (hh_alpha_n(V) * (1.0 - nn) - hh_beta_n(V) * nn);
                continue;
            }
            if (h->model == 1) {
                /* Izhikevich transition (Eqs. izsimple and izpsc), all from the state at t */
                const double V = h->V[j], W = h->W[j], r = h->r[j], pp = h->p[j];
                if (h->psc == 1) {
                    h->r[j] = r - h->dt * h->psc_a * r + in;
                } else if (h->psc == 2) {
                    h->r[j] = r + h->dt * pp;
                    h->p[j] = pp + h->dt * (-h->psc_a * h->psc_a * r - 2.0 * h->psc_a * pp) + in;
                }
                if (s[j]) {
                    h->V[j] = h->v_reset;
                    h->W[j] = W + h->iz_d;
                } else {
                    uint32_t ctr[4] = {(uint32_t)j, (uint32_t)t, (uint32_t)(t >> 32), 0u};
                    uint32_t rr[4];
                    orc_philox4x32_10(ctr, h->key, rr);
                    const double U = h->i_ext[j] + ((rr[0] < h->drive_thr[j]) ? h->drive_amp : 0.0);
                    const double xi = orc_box_muller(rr[1], rr[2]);
                    const double syn = h->psc == 0 ? 0.0 : r;
                    const double cur = h->iz_k * (V - h->iz_vr) * (V - h->iz_vt) - W + syn + U;
                    double Vn = V + h->dt * (1.0 / h->iz_C) * cur;
                    if (h->psc == 0) Vn = Vn + in;
                    h->V[j] = Vn + h->sigma * xi;
                    h->W[j] = W + h->dt * h->iz_a * (h->iz_b * (V - h->iz_vr) - W);
                }
                continue;
            }
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
