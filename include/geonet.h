/*
 * geonet: fixed-step simulation of dynamic geometric networks on AMD
 * Instinct MI355X (gfx950).
 *
 * Model (Buibas & Silva, "A framework for simulating and estimating the
 * state and functional topology of complex dynamic geometric networks"):
 *   - every vertex j has a fixed position x_j and a state y_j(t) advanced in
 *     steps of dt by a transition function (Section 2, Eq. Htrans); here the
 *     leaky integrate-and-fire vertex of Section 3.1, Euler-integrated;
 *   - a vertex signals when V >= threshold (Section 3.2, Eq. spd) and the
 *     signal reaches target j after tau_ij = |x_i - x_j| / s (Eq. delaydist),
 *     weighted by omega_ij: the input of j at step t is the sum over in-edges
 *     i -> j of omega_ij * spd(V_i(t - tau_ij)) (Eq. izpsc, last term);
 *   - control u_j(t) per vertex (Section 2): a constant input plus Poisson
 *     pulses; state noise as allowed by the framework (Section 1);
 *   - observation (Section 3.3): calcium c + dt*(-c/tau_c + spd), averaged
 *     over the steps of one camera frame, fluorescence n*c + b + N(0, g^2).
 *
 * Step semantics, for t = 0, 1, ... (all vertices in parallel):
 *   s_j(t)   = [V_j(t) >= v_th]
 *   I_j(t)   = sum over edges (i -> j) of w_ij * s_i(t - d_ij),  d_ij >= 1
 *   if s_j(t):                 V_j(t+1) = v_reset, hold for n_ref steps
 *   else if held:              V_j(t+1) = v_reset  (input discarded)
 *   else: V_j(t+1) = V_j + (dt/tau)(v_rest - V_j) + I_j + u_j + sigma*xi_j
 *   c_j(t+1) = c_j + dt*(-c_j/tau_c + s_j)
 * with d_ij = max(1, ceil(|x_i - x_j| / (s*dt))) unless given explicitly.
 * The held steps after a spike at step t0 are t0+1 .. t0+n_ref.
 *
 * Random numbers are Philox4x32-10 (Salmon et al., SC'11) with key = seed
 * (low word first) and counter (j, t_lo, t_hi, 0) for the step of vertex j;
 * output 0 decides the Poisson pulse (pulse iff x0 < floor(rate*dt*2^32)),
 * outputs 1 and 2 give xi by Box-Muller on 24-bit uniforms ((x>>8)+0.5)/2^24.
 * Observation noise uses counter (j, frame_lo, frame_hi, 1), outputs 0, 1.
 * j is the vertex index inside its own network.
 *
 * Conventions for every entry point:
 *   - all calls return net_status; nothing throws across this boundary;
 *     net_last_error() gives the text of the last non-OK status of the
 *     calling thread;
 *   - "host" pointers are read during the call only (the library copies
 *     them); "device" pointers are caller-owned device memory written
 *     asynchronously on `stream`;
 *   - `stream` is a hipStream_t (NULL = the default stream); every device
 *     operation of a call is ordered on it and the call does not wait for it
 *     except where stated;
 *   - a device fault seen by a call is returned as NET_E_DEVICE and leaves
 *     the handle unusable (later calls return NET_E_STATE).
 */
#ifndef GEONET_H
#define GEONET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct net net_t;

typedef enum {
    NET_OK = 0,
    NET_W_INEXACT = 1,      /* build succeeded, but some row's weight sums are not
                               provably exact in FP32 (see net_build) */
    NET_E_ARG = -1,         /* invalid argument */
    NET_E_RANGE = -2,       /* a delay above 255 steps, or a size overflow */
    NET_E_OOM = -3,         /* device allocation failed */
    NET_E_DEVICE = -4,      /* HIP runtime or kernel error */
    NET_E_STATE = -5,       /* handle unusable after an earlier device error */
    NET_E_UNSUPPORTED = -6  /* request outside what the library supports */
} net_status;

/*
 * One network (Section 2: vertex set with positions, directed weighted
 * edges, delays from geometry, per-vertex parameters Theta_j and control).
 * An array of these is an ensemble of independent networks.
 */
typedef struct {
    int32_t n_nodes;              /* J, >= 1 */
    int32_t dims;                 /* dimension of x_j: 1, 2 or 3 */
    const double* pos_um;         /* host [n_nodes*dims] row-major positions (um) */
    int64_t n_edges;              /* >= 0 */
    const int32_t* src;           /* host [n_edges] source i of edge i -> j */
    const int32_t* dst;           /* host [n_edges] target j; i != j, no duplicates */
    const float* weight;          /* host [n_edges] omega_ij; rounded to FP16 (ties to
                                     even) when built; sign selects excitation/inhibition */
    const uint8_t* delay_steps;   /* host [n_edges] explicit delays (values 0 are taken
                                     as 1), or NULL to compute them from positions */
    double v_um_per_ms;           /* conduction speed s (Eq. delaydist) */
    double dt_ms;                 /* time step; equal for all networks of an ensemble */
    float tau_ms;                 /* membrane time constant */
    float v_rest, v_reset, v_th;  /* rest (decay target), reset value, threshold */
    int32_t n_ref;                /* held steps after a spike, 0..250 */
    const float* drive_rate_hz;   /* host [n_nodes] Poisson pulse rate, or NULL */
    float drive_amp;              /* pulse amplitude A added to V */
    const float* i_ext;           /* host [n_nodes] constant input per step, or NULL */
    float noise_sigma;            /* sigma of the per-step Gaussian increment */
    uint64_t seed;                /* Philox key */
    const float* v0;              /* host [n_nodes] V(0), or NULL for v_rest */
    float tau_c_ms;               /* calcium removal time constant */
    int32_t frame_num, frame_den; /* frame(t) = floor(t*num/den); equal across an ensemble */
    /* Vertex model (Section 3.1).  NET_MODEL_LIF: the leaky integrate-and-fire
       vertex above.  NET_MODEL_IZHIKEVICH: the simple model of Eq. izsimple,
       Euler-stepped with its state (V, W and the PSC states) in FP64; v_th is
       V_peak and v_reset is c (tau_ms, v_rest unused; n_ref must be 0):
         s_j(t) = [V >= V_peak];  if s: V <- c, W <- W + d
         else V <- V + dt*(1/C)*[k(V-Vr)(V-Vt) - W + r + U] (+ I for psc NONE) + sigma*xi
              W <- W + dt*a*(b(V-Vr) - W)
       with U = i_ext + drive_amp*pulse (pA) and xi drawn in FP64.  Delivered
       input (Section 3.2) as a post-synaptic current, updated every step:
         NET_PSC_NONE  I jumps V directly (no r);
         NET_PSC_EXP   r <- r - dt*psc_rate*r + I               (Eq. simplepsc)
         NET_PSC_ALPHA r <- r + dt*p;  p <- p + dt*(-a^2 r - 2a p) + I, a = psc_rate
                                                                 (Eqs. alphapsc, izpsc)
       an arrival being an impulse of its weight (pA for EXP/ALPHA, mV for
       NONE).  Units: ms, mV, pF, pA, nS. */
    int32_t model;                /* NET_MODEL_* (0 = LIF) */
    int32_t psc;                  /* NET_PSC_* (Izhikevich and Hodgkin-Huxley) */
    float iz_C, iz_k, iz_vr, iz_vt, iz_a, iz_b, iz_d;   /* Izhikevich constants */
    float psc_rate;               /* PSC decay rate a (1/ms) */
    const float* w0;              /* host [n_nodes] initial W, or NULL (0) */
    /* NET_MODEL_HODGKIN_HUXLEY: the four-state vertex of Section 3.1 (V and the
       gates m, n, h, FP64), Euler-stepped (the paper uses dt = 0.03 ms):
         V <- V + dt*(1/C)*[-gNa m^3 h (V-ENa) - gK n^4 (V-EK) - gL (V-EL) + r + U]
              (+ I for psc NONE) + sigma*xi
         x <- x + dt*(alpha_x(V)(1-x) - beta_x(V) x),  x in {m, n, h}
       with alpha_m = 0.1(V+40)/(1-exp(-(V+40)/10)), beta_m = 4 exp(-(V+65)/18),
       alpha_h = 0.07 exp(-(V+65)/20), beta_h = 1/(1+exp(-(V+35)/10)),
       alpha_n = 0.01(V+55)/(1-exp(-(V+55)/10)), beta_n = 0.125 exp(-(V+65)/80)
       (limits 1 and 0.1 at V = -40, -55).  The gates start at their steady
       state for V(0).  A spike is the upward crossing s_j(t) = [V(t) >= v_th and
       V(t-1) < v_th] (V(-1) = V(0)); there is no reset; n_ref must be 0; the
       PSC kinds are those of the Izhikevich vertex.  Units: mV, ms, uF/cm^2,
       mS/cm^2, uA/cm^2. */
    float hh_C, hh_gna, hh_gk, hh_gl, hh_ena, hh_ek, hh_el;
    /* Spike-timing-dependent plasticity (Section 3.2 "Plasticity", Eqs.
       omegatrans and Gparams), plastic != 0: with s_j the time since j's last
       spike (s_j(t+1) = (1 - s_j(t) fired) * (s_j(t) + dt), s_j(0) = 0),
         q_ij(t) = (s_i(t - d_ij) - s_j(t)) * max(spd_i(t - d_ij), spd_j(t))
         w_ij(t+1) = w_ij(t) + dt * stdp_alpha * sign(q) * exp(-stdp_beta * |q|),
       the increment rounded to a multiple of 2^-20 (weights are kept as such
       multiples, so delivered sums stay exact in any order); a spike delivers
       the weight its edge has when it arrives.  Needs the LIF vertex, one
       network per handle, n_ref >= 17 (the last 16 spike times of a vertex
       then cover the 255-step delay window) and weights that are multiples
       of 2^-20 below 2048 after FP16 rounding; the per-step kernels are used
       (build flags that select other kernels are ignored). */
    int32_t plastic;
    float stdp_alpha;             /* weight per ms */
    float stdp_beta;              /* 1/ms */
} net_desc;

enum { NET_MODEL_LIF = 0, NET_MODEL_IZHIKEVICH = 1, NET_MODEL_HODGKIN_HUXLEY = 2 };
enum { NET_PSC_NONE = 0, NET_PSC_EXP = 1, NET_PSC_ALPHA = 2 };

/* Build options; a zeroed struct (or NULL) selects the defaults. */
typedef struct {
    int32_t frame_capacity;       /* frames kept per vertex; 0 disables calcium */
    int32_t block_threads;        /* delivery workgroup size override (0 = auto) */
    int32_t blocks_per_cu;        /* delivery workgroups per CU override (0 = auto) */
    int32_t flags;                /* NET_BUILD_* */
} net_build_opts;

/* Build flags (variants that compute the same result; for tuning/measurement). */
#define NET_BUILD_NO_LDS_SUMMARY 1        /* keep the recent-spike summary in global memory */
#define NET_BUILD_DELIVER_STREAM_WEIGHTS 2 /* delivery: stream every weight with its edge
                                             (default: load a weight only when its edge
                                             delivers a spike) */
#define NET_BUILD_DELIVER_NONTEMPORAL 4   /* delivery: non-temporal edge loads */
#define NET_BUILD_PER_STEP 8              /* ensembles: per-step kernels instead of the
                                             single-launch ensemble kernel */
#define NET_BUILD_DELIVER_UNROLL2 16      /* delivery: two 512-edge chunks per wave iteration
                                             (default one) */
#define NET_BUILD_DELIVER_PIPELINE 128   /* delivery: issue the next chunk's edge loads while
                                             this chunk's history gathers are in flight */
#define NET_BUILD_SUMMARY_HALF 256        /* delivery: one recent-spike summary bit per vertex pair
                                             (half the LDS, twice the workgroups per CU; more
                                             candidates, resolved exactly) */
#define NET_BUILD_DELIVER_COMPACT 512    /* delivery: gather the candidate edges of each chunk
                                             into an LDS stage and resolve them one per lane
                                             (needs fewer than 2^24 vertices and room in LDS) */
#define NET_BUILD_FUSED_STEP 1024        /* one network: one kernel per step, each workgroup
                                             delivering into and then updating its own range of
                                             vertices (the slot list is cut into one segment per
                                             CU). Needs at most 2^20 vertices (the summary in a
                                             fixed 128 KiB of LDS), segments of at most 6,080
                                             vertices, fewer than 2^32 edge slots and the full
                                             summary (not with NET_BUILD_SUMMARY_HALF) and LIF
                                             vertices only; otherwise the two kernels are used.
                                             net_info reports which.
                                             The step streams one 32-bit word per edge slot
                                             (source | delay << 24), built at net_build: 4 B per
                                             slot of device memory more. */
#define NET_BUILD_DELIVER_PACKED 2048    /* delivery: two chunks per wave iteration, the edges
                                             streamed as one 32-bit word each (source | delay << 24:
                                             4 B per edge instead of 5) and the next pair's loads
                                             issued behind this pair's history gathers; needs fewer
                                             than 2^24 vertices (else DELIVER_UNROLL2 is used) and
                                             4 B per edge slot of device memory more */
#define NET_BUILD_SINGLE_LAUNCH 32        /* one network: run all steps of a call in one launch of
                                             the LDS-resident kernel ensembles use, when the
                                             network fits one workgroup's LDS */
#define NET_BUILD_REORDER 4096           /* renumber each network's vertices along a Morton (Z-order) curve
                                             of their positions before building, so that vertices close in
                                             space are close in memory (the gathers of delivery then meet in
                                             cache); everything at the boundary keeps the caller's numbering:
                                             records and read-outs are put back in it (records at some extra
                                             cost) and random streams use the caller's vertex index */
#define NET_BUILD_GRAPH 8192             /* run net_step_n calls without records or kernel timing as HIP
                                             graph replays: the per-step kernels of 256 steps (a whole turn
                                             of the history ring) captured once and replayed from steps that
                                             are multiples of 256, the single-launch ensemble kernel captured
                                             once per call length; the kernels then read the step from a
                                             device counter the graph advances.  Same results; steps outside
                                             whole 256-step blocks run as plain launches.  Not for plastic
                                             networks (ignored). */
#define NET_BUILD_PUSH 16384             /* deliver by pushing spikes instead of testing every in-edge: each
                                             step's update lists the vertices that fired (one atomic per wave)
                                             and a second kernel adds the weight of every out-edge of each of
                                             them into an input ring indexed by arrival step (one FP32 word per
                                             vertex and ring slot, as many slots as the next power of two above
                                             the largest delay); the update of step t reads and clears slot t.
                                             The work per step is the spikes' out-edges, not all edges.  Used
                                             only when every target's weights sum exactly (the order of the
                                             additions then changes no bit), with the per-step update kernel
                                             (NET_BUILD_GRAPH replays it too); ignored for plastic networks.
                                             net_info's deliver_flags shows whether it is in use. */
#define NET_BUILD_AUTOTUNE 64             /* time the candidate launch shapes on this graph at
                                             build (a few steps from the initial state, which is
                                             then restored) and keep the fastest: delivery
                                             variants for the per-step kernels, workgroup size and
                                             workgroups per CU for the single-launch kernel.
                                             Every candidate computes the same bits. */

/*
 * Optional per-step records for net_step_n (device pointers, may be NULL).
 * Row k holds step t0 + k where t0 is the step counter before the call.
 * Vertices are numbered across the ensemble in net_desc order.
 */
typedef struct {
    uint64_t* raster;   /* [n_steps][raster_words]: bit (j % 64) of word j / 64 = s_j(t) */
    float* v;           /* [n_steps][n_total]: V_j(t) at the start of step t */
    float* input;       /* [n_steps][n_total]: delivered input I_j(t) */
} net_record;

typedef struct {
    int64_t n_total;        /* vertices over all networks */
    int64_t n_edges;        /* edges over all networks (as given) */
    int64_t n_edges_stored; /* stored edge slots incl. padding */
    int32_t n_nets;
    int32_t max_delay;      /* largest delay in steps */
    int64_t raster_words;   /* 64-bit words per raster row */
    int64_t t;              /* steps taken so far */
    int64_t frames_done;    /* completed camera frames */
    int32_t exact;          /* 1 if every FP32 delivery sum is provably exact */
    int32_t summary_window; /* steps covered by the recent-spike filter */
    int32_t lds_summary;    /* 1 if the delivery kernel stages the summary in LDS */
    int32_t deliver_blocks, deliver_threads;
    int64_t device_bytes;   /* device memory held by the handle */
    int32_t deliver_flags;  /* NET_BUILD_DELIVER_* bits of the delivery variant in use */
    int32_t ensemble_blocks, ensemble_threads;   /* single-launch kernel shape (0: per-step kernels) */
    int32_t autotuned;      /* 1 if the launch shape was chosen by timing at build */
    int32_t ensemble_stream; /* how the single-launch kernel reads its edge slots: 0 not in use,
                                1 held in registers for all steps, 2 streamed as 2-byte sources
                                within the network plus the delay bytes (3 B per slot), 3 streamed
                                as 2-byte slots packing source and delay (every network's vertex
                                count and largest delay fit in 16 bits together) */
} net_info_t;

/*
 * Device-memory allocator used for every allocation made by net_build (the
 * Python binding registers the PyTorch caching allocator).  alloc returns
 * NULL on failure.  Passing NULL for both restores hipMalloc/hipFree.
 * Affects handles built afterwards; not thread-safe against concurrent
 * net_build calls.
 */
net_status net_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                             void (*release)(void* ptr, void* stream, void* ctx), void* ctx);

/*
 * Build n_nets >= 1 networks into one handle (Section 2 definitions; delays
 * by Eq. delaydist).  Copies all host inputs.  Computes delays in double
 * precision (R3 rule above), rounds weights to FP16, forms the edge list
 * sorted by target (CSR by target), uploads on `stream` and waits for the
 * upload.  Returns NET_E_RANGE for a delay above 255 steps, NET_E_ARG for an
 * out-of-range index, a self-loop, a duplicate edge or inconsistent
 * dt/frame settings, NET_W_INEXACT (with a valid handle) when, for some
 * target, (sum of |w|) / (smallest FP16 ulp among its weights) > 2^24.
 * *out receives the handle on NET_OK or NET_W_INEXACT, else NULL.
 */
net_status net_build(const net_desc* descs, int32_t n_nets, const net_build_opts* opts,
                     void* stream, net_t** out);

/*
 * Advance every network by n_steps >= 0 steps (semantics above), enqueued on
 * `stream` without host synchronisation.  rec may be NULL; its buffers must
 * hold n_steps rows.
 */
net_status net_step_n(net_t* h, int64_t n_steps, const net_record* rec, void* stream);

/* What net_observe returns. */
enum {
    NET_OBS_V = 1,        /* float [n_total]  current V */
    NET_OBS_REF = 2,      /* int32 [n_total]  remaining held steps */
    NET_OBS_CALCIUM = 3,  /* float [n_total]  current c */
    NET_OBS_FRAMES = 4,   /* float [F][n_total] mean c of frames 0..F-1, F = out_bytes/(4*n_total) */
    NET_OBS_FLUOR = 5,    /* float [F][n_total] n*cbar + b + gamma*xi, params = net_fluor_params */
    NET_OBS_WEIGHTS = 6   /* float [n_edges] current weights, in the order the edges were given
                             (plastic networks only; NET_E_UNSUPPORTED otherwise) */
};

typedef struct {
    float gain, offset, gamma;  /* n, b, gamma of the observation function (Section 3.3) */
    int32_t pad;
} net_fluor_params;

/*
 * Observation z_j = F_j(y_j) (Section 2, Eq. obsfun; Section 3.3).  Writes
 * `what` into device buffer `out` of out_bytes on `stream`.  Frame requests
 * need frame_capacity > 0 at build and F <= min(frames_done, capacity).
 */
net_status net_observe(net_t* h, int32_t what, const void* params, void* out, int64_t out_bytes,
                       void* stream);

/*
 * Kernel timing for measurement.  After net_timing_begin(h, max_launches,
 * every), one in `every` kernel launches of each kind made by net_step_n
 * (the first, then every every-th) is bound to HIP events (start and end of
 * the kernel itself, on the call's stream), up to max_launches in all; a
 * bound launch costs a few microseconds of issue time, so a sample keeps
 * the timed run undisturbed.  net_timing_end waits for them, fills *out with
 * the summed durations per kernel kind and the counts of timed launches and
 * of the steps they cover, and stops recording.  Timing never changes results.
 */
typedef struct {
    double deliver_ms, update_ms, ensemble_ms;         /* summed kernel durations */
    int64_t deliver_launches, update_launches, ensemble_launches;
    int64_t steps;                                     /* steps covered by timed launches */
    double step_ms;                                    /* fused step kernels (NET_BUILD_FUSED_STEP) */
    int64_t step_launches;
} net_timing_t;

net_status net_timing_begin(net_t* h, int64_t max_launches, int32_t every);
net_status net_timing_end(net_t* h, net_timing_t* out);

/* Sizes and counters of a handle (host struct). */
net_status net_info(const net_t* h, net_info_t* out);

/* First vertex index of every network: host int64 [n_nets + 1]. */
net_status net_node_offsets(const net_t* h, int64_t* out);

/* ------------------------------------------------------------------------
 * Learned edge scorer: an MLP 64 -> 256 -> 256 -> 1 (ReLU) on pair
 * features, trained with binary cross-entropy on simulated networks whose
 * edges are known; it proposes functional edges i -> j from observations
 * (the inverse problem of Sections 1 and 4).  BF16 operands on the matrix
 * cores, FP32 accumulation and master weights.  Rounding points: features,
 * W1 and W2 to BF16; H1, H2 to BF16 after bias + ReLU; dH2, dH1 to BF16
 * before they enter a matrix product; head, loss and gradients in FP32.
 *
 * Parameters are one flat FP32 vector of 82,689 values:
 *   W1[64][256] | b1[256] | W2[256][256] | b2[256] | w3[256] | b3
 * (W[k][n] row-major: input k, output n).  Features are FP32 [rows][64]
 * row-major in device memory; labels FP32 0/1 [rows].  All calls run on
 * `stream`; the activation workspace grows (with a stream synchronisation)
 * when a call needs more rows than any earlier one.
 * ------------------------------------------------------------------------ */
typedef struct net_mlp net_mlp_t;

net_status net_mlp_create(net_mlp_t** out);                 /* parameters zero */
net_status net_mlp_set_params(net_mlp_t* m, const float* host_params, int64_t n);   /* resets Adam */
net_status net_mlp_get_params(const net_mlp_t* m, float* host_params, int64_t n);
/* Input standardisation applied before the first layer: x'_k = (x_k - shift[k]) * scale[k]
   (host [64] each; default shift 0, scale 1). */
net_status net_mlp_set_input_norm(net_mlp_t* m, const float* shift, const float* scale);
/* logits_dev[r] = MLP(x_dev[r]) */
net_status net_mlp_forward(net_mlp_t* m, const float* x_dev, int64_t rows, float* logits_dev, void* stream);
/* gradient of the mean BCE over the rows into grad_dev [82,689] and loss_dev [1] (either may be NULL) */
net_status net_mlp_grad(net_mlp_t* m, const float* x_dev, const float* y_dev, int64_t rows, float* grad_dev,
                        float* loss_dev, void* stream);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the mean BCE of the rows */
net_status net_mlp_train_step(net_mlp_t* m, const float* x_dev, const float* y_dev, int64_t rows, float lr,
                              float* loss_dev, void* stream);
/* Input standardisation fitted to training features (device x_dev [rows][64], 1 <= rows <= 2^31),
   computed on the GPU in FP64: shift = column mean, scale = 1 / column standard deviation
   (unbiased), or 0 for a column whose deviation is at most 1e-6 (a constant feature is dropped).
   Replaces what net_mlp_set_input_norm set; ordered on `stream`. */
net_status net_mlp_fit_input_norm(net_mlp_t* m, const float* x_dev, int64_t rows, void* stream);
/* The current standardisation (host [64] each); waits for the device. */
net_status net_mlp_get_input_norm(const net_mlp_t* m, float* shift, float* scale);
/* One epoch of minibatch training: the rows (x_dev [rows][64], y_dev [rows]) are visited once in
   the order of a keyed permutation of [0, rows) (net_shuffle_indices with the same seed and epoch),
   in consecutive batches of `batch` rows, the last one possibly smaller; one Adam step per batch
   (as net_mlp_train_step).  loss_dev: device [ceil(rows / batch)] mean BCE of each step's batch
   (before its update), or NULL.  The permuted batch is gathered into a workspace held by the
   handle (grown, with a stream synchronisation, when a larger batch is asked for). */
net_status net_mlp_train_epoch(net_mlp_t* m, const float* x_dev, const float* y_dev, int64_t rows, int64_t batch,
                               float lr, uint64_t shuffle_seed, uint32_t epoch, float* loss_dev, void* stream);
/* out_dev[i] = pi(i), i < n <= 2^31: the permutation of [0, n) keyed by (seed, epoch) that
   net_mlp_train_epoch visits rows in (a four-round Feistel network over Philox4x32-10 with cycle
   walking).  Device int64 [n]; ordered on `stream`. */
net_status net_shuffle_indices(int64_t n, uint64_t seed, uint32_t epoch, int64_t* out_dev, void* stream);
void net_mlp_free(net_mlp_t* m);
const char* net_mlp_last_error(void);

/* ------------------------------------------------------------------------
 * Observations of one network for the inverse problem: what an experiment
 * provides (fluorescence of every vertex per camera frame, positions, the
 * experimenter's own control schedule) plus the candidate pairs to score.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_nodes, n_frames;
    const float* fluor;          /* device [n_frames][n_nodes] fluorescence F_j(f) */
    int64_t n_pairs;
    const int32_t* pairs;        /* device [n_pairs][2]: (source i, target j), i != j */
    const float* pair_dist_um;   /* device [n_pairs] |x_i - x_j| */
    float gain, offset, gamma;   /* observation model n, b, gamma (Section 3.3) */
    double dt_ms;
    float tau_c_ms;
    int32_t frame_num, frame_den;  /* frame(t) = floor(t*num/den) */
    const float* drive_rate_hz;  /* host [n_nodes] control pulse rates, or NULL */
    float drive_amp;
    uint64_t control_seed;       /* Philox key of the control pulses (output 0 only) */
    /* vertex model assumed by the simulation-based fit */
    float tau_ms, v_rest, v_reset, v_th, noise_sigma, w_assumed;
    int32_t n_ref;
    const float* w_source;       /* host [n_nodes]: the weight the fit assumes on every edge out of
                                    vertex i (negative for an inhibitory cell, whose type the
                                    experimenter knows), or NULL: w_assumed for every vertex */
} net_obs_desc;

/*
 * Pair features (device [n_pairs][64], FP32) from the observations: per
 * vertex, activity e(f) = max(0, (F(f+1)-b) - rho (F(f)-b)) with
 * rho = (1 - dt/tau_c)^(den/num) (the calcium model sampled per frame) and
 * standardised e, F; per pair, lagged correlations of e and F, responses to
 * the other vertex's control pulses, activity levels and distance.  Waits
 * for completion.
 */
net_status net_features(const net_obs_desc* obs, float* features_dev, void* stream);

/*
 * net_features for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same features (same kernels, same bits), with the
 * scratch in a fixed 16 MiB array of device memory that the library holds on
 * every GPU it runs on until the process ends, instead of memory taken from
 * the allocator.  It allocates and frees nothing.  The scratch needed,
 * net_features_noalloc_scratch_bytes(n_nodes, n_frames) (about
 * 16 * n_nodes * n_frames bytes), must not exceed 16 MiB, else NET_E_RANGE
 * with the sizes in net_estimate_last_error and nothing launched.  Every
 * call on one GPU uses that GPU's one array: calls that overlap on one GPU
 * (from several threads or streams at once) race and must be serialised by
 * the caller; each call waits for its own completion, so successive calls
 * from one thread are safe.  Nothing in the array needs to start at zero
 * (every kernel writes its scratch before reading it).
 */
net_status net_features_noalloc(const net_obs_desc* obs, float* features_dev, void* stream);
size_t net_features_noalloc_scratch_bytes(int32_t n_nodes, int32_t n_frames);

/* Options of the simulation-based fit (zeroed struct or NULL: defaults). */
typedef struct {
    int32_t realisations;   /* K noise realisations per hypothesis, divides 64 (default 8) */
    int32_t sweeps;         /* toggle sweeps (default 0 with a zeroed struct: pass 2 for the usual fit) */
    float init_fraction;    /* initial in-neighbours per target: the top ceil(f n - 1e-6) of its n
                               candidates by correlation (f = 0.3) */
    float min_gain;         /* smallest log-likelihood gain (nats) for which a toggle is applied
                               (<= 0: 1e-3) */
    uint64_t fit_seed;      /* Philox key of the fit's own noise (never the data's) */
} net_simfit_opts;

enum { NET_EST_SCORER = 1, NET_EST_SIMFIT = 2, NET_EST_AUTO = 3 };

/*
 * Scores of the candidate pairs (device [n_pairs] FP32; higher = more likely
 * an edge i -> j), from the observations only (the inverse problem of
 * Sections 1 and 4):
 *   NET_EST_SCORER  features (net_features) through the trained MLP `scorer`;
 *                   scores are logits.
 *   NET_EST_SIMFIT  simulation-based fit.  Each target j is simulated with the
 *                   vertex model of the forward path, teacher-forced by the
 *                   deconvolved activity of a hypothesised in-neighbour set G
 *                   (input w_i * e_i(f) spread over frame f, w_i from w_source,
 *                   else w_assumed), its own
 *                   control pulses and K noise realisations (fit_seed); the
 *                   observed trace is scored with the Gaussian observation
 *                   model using the realisations' mean and variance.  G starts
 *                   as the top init_fraction by lag-0 plus lag-1 correlation;
 *                   each sweep evaluates every single toggle and, per target,
 *                   applies the one that raises the likelihood most, if by more
 *                   than min_gain.
 *                   Score = LL(G + e) - LL(G - e) at the final G.
 *   NET_EST_AUTO    the scorer when `scorer` is given (the fast path, trained on
 *                   simulated networks of the same kind), else the fit.
 * Errors: NET_E_ARG for a bad descriptor, pair or option (message in
 * net_estimate_last_error), NET_E_OOM, NET_E_DEVICE.
 * Waits for completion.
 */
net_status net_estimate(const net_obs_desc* obs, int32_t method, net_mlp_t* scorer, const net_simfit_opts* opts,
                        float* scores_dev, void* stream);
const char* net_estimate_last_error(void);

/*
 * Error-handling test hook: marks the handle exactly as a device fault seen by
 * a call would (nothing runs on the device), so that callers can exercise
 * their NET_E_STATE path without faulting a GPU.  Every later call on the
 * handle except net_info, net_node_offsets and net_free returns NET_E_STATE.
 */
net_status net_simulate_device_error(net_t* h);

/* Release the handle and its device memory (waits for the handle's stream). */
void net_free(net_t* h);

/* Text of the last non-OK status of the calling thread ("" if none). */
const char* net_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GEONET_H */
