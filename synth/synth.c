/*
 * Seeded synthetic geometric-network generator (input side only).
 *
 * This file produces the *inputs* of a simulation: which ordered vertex
 * pairs (i -> j) carry an edge, given vertex positions and a
 * distance-dependent connection probability.  It holds none of the
 * simulated method's arithmetic (no delays, no dynamics, no delivery);
 * both the GPU library and the CPU oracle consume its output unchanged.
 *
 * Edge rule: an ordered pair (i, j), i != j, at Euclidean distance r gets an
 * edge with probability p(r), drawn independently per pair:
 *   kind 0 (step):   p(r) = p0            for r <  r_cut, else 0
 *   kind 1 (expdec): p(r) = p0*exp(-r/lam) for r <  r_cut, else 0
 *
 * Sampling never tests all N^2 pairs.  Vertices are binned into cubic cells
 * of side h.  For a (source cell A, target cell B) pair, every vertex pair
 * has p <= pmax(A,B) = p(box distance of A and B), so the generator jumps
 * over the |A|*|B| virtual pairs with geometric skips of parameter pmax and
 * keeps each visited pair with probability p(r)/pmax (thinning).  The result
 * has exactly the per-pair Bernoulli law above.
 *
 * Determinism: each target cell owns a private counter-based stream keyed by
 * (seed, cell), so the edge set does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* splitmix64 finaliser: a bijective 64-bit mixer (Steele, Lea, Flood 2014). */
static inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s; } stream_t;

static inline double next_u01(stream_t* st) {       /* uniform in (0, 1) */
    st->s += 0x9E3779B97F4A7C15ull;
    uint64_t z = st->s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

typedef struct {
    int64_t n, cap;
    int32_t* src;
    int32_t* dst;
} edge_buf;

static void eb_push(edge_buf* b, int32_t s, int32_t d) {
    if (b->n == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 1024;
        b->src = (int32_t*)realloc(b->src, (size_t)nc * sizeof(int32_t));
        b->dst = (int32_t*)realloc(b->dst, (size_t)nc * sizeof(int32_t));
        b->cap = nc;
    }
    b->src[b->n] = s;
    b->dst[b->n] = d;
    b->n++;
}

typedef struct {
    int64_t n_cells;
    edge_buf* per_cell;      /* edges whose target lies in each cell */
    int64_t total;
} syn_edges_handle;

static inline double p_of(int kind, double p0, double lam, double r_cut, double r) {
    if (!(r < r_cut)) return 0.0;
    if (kind == 0) return p0;
    return p0 * exp(-r / lam);
}

/* Box distance between two cells given their integer offsets. */
static inline double box_dist(const int* off, int dims, double h) {
    double s = 0.0;
    for (int k = 0; k < dims; ++k) {
        int a = off[k] < 0 ? -off[k] : off[k];
        double g = a > 0 ? (double)(a - 1) * h : 0.0;
        s += g * g;
    }
    return sqrt(s);
}

/*
 * Generate edges.  pos: [n*dims] row-major, dims in {2,3}.  ext: extent per
 * dimension (positions lie in [0, ext)).  Returns an opaque handle; read the
 * result with syn_edges_count / syn_edges_copy, then syn_edges_free.
 */
void* syn_edges(int64_t n, int dims, const double* pos, const double* ext,
                int kind, double p0, double lam, double r_cut, double h,
                uint64_t seed) {
    if (n <= 0 || dims < 1 || dims > 3 || h <= 0.0) return NULL;
    int nc[3] = {1, 1, 1};
    for (int k = 0; k < dims; ++k) {
        nc[k] = (int)ceil(ext[k] / h);
        if (nc[k] < 1) nc[k] = 1;
    }
    int64_t n_cells = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t* cell_of = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int64_t* cstart = (int64_t*)calloc((size_t)n_cells + 1, sizeof(int64_t));
    int32_t* cnodes = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        int c[3] = {0, 0, 0};
        for (int k = 0; k < dims; ++k) {
            int q = (int)floor(pos[i * dims + k] / h);
            if (q < 0) q = 0;
            if (q >= nc[k]) q = nc[k] - 1;
            c[k] = q;
        }
        int64_t id = ((int64_t)c[2] * nc[1] + c[1]) * nc[0] + c[0];
        cell_of[i] = (int32_t)id;
        cstart[id + 1]++;
    }
    for (int64_t c = 0; c < n_cells; ++c) cstart[c + 1] += cstart[c];
    {
        int64_t* fill = (int64_t*)malloc((size_t)n_cells * sizeof(int64_t));
        memcpy(fill, cstart, (size_t)n_cells * sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i) cnodes[fill[cell_of[i]]++] = (int32_t)i;
        free(fill);
    }
    int maxnc = nc[0];
    if (nc[1] > maxnc) maxnc = nc[1];
    if (nc[2] > maxnc) maxnc = nc[2];
    int R = (r_cut < 1e300) ? (int)ceil(r_cut / h) : maxnc;
    if (R > maxnc) R = maxnc;
    int Rz = dims >= 3 ? R : 0, Ry = dims >= 2 ? R : 0;

    syn_edges_handle* H = (syn_edges_handle*)calloc(1, sizeof(syn_edges_handle));
    H->n_cells = n_cells;
    H->per_cell = (edge_buf*)calloc((size_t)n_cells, sizeof(edge_buf));

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t B = 0; B < n_cells; ++B) {
        int64_t nb = cstart[B + 1] - cstart[B];
        if (nb == 0) continue;
        int bx = (int)(B % nc[0]);
        int by = (int)((B / nc[0]) % nc[1]);
        int bz = (int)(B / ((int64_t)nc[0] * nc[1]));
        stream_t st;
        st.s = mix64(seed ^ mix64((uint64_t)B + 0x51ED2701ull));
        edge_buf* eb = &H->per_cell[B];
        for (int dz = -Rz; dz <= Rz; ++dz) {
            int az = bz + dz;
            if (az < 0 || az >= nc[2]) continue;
            for (int dy = -Ry; dy <= Ry; ++dy) {
                int ay = by + dy;
                if (ay < 0 || ay >= nc[1]) continue;
                for (int dx = -R; dx <= R; ++dx) {
                    int ax = bx + dx;
                    if (ax < 0 || ax >= nc[0]) continue;
                    int off[3] = {dx, dy, dz};
                    double dmin = box_dist(off, dims, h);
                    double pmax = p_of(kind, p0, lam, r_cut, dmin);
                    if (pmax <= 0.0) continue;
                    int64_t A = ((int64_t)az * nc[1] + ay) * nc[0] + ax;
                    int64_t na = cstart[A + 1] - cstart[A];
                    if (na == 0) continue;
                    int64_t npairs = na * nb;
                    double lq = pmax < 1.0 ? log1p(-pmax) : 0.0;
                    int64_t q = -1;
                    for (;;) {
                        if (pmax < 1.0) {
                            double u = next_u01(&st);
                            double skip = floor(log(u) / lq);
                            if (skip >= (double)(npairs - q)) break;
                            q += 1 + (int64_t)skip;
                        } else {
                            q += 1;
                        }
                        if (q >= npairs) break;
                        int32_t j = cnodes[cstart[B] + q / na];
                        int32_t i = cnodes[cstart[A] + q % na];
                        if (i == j) continue;
                        double s2 = 0.0;
                        for (int k = 0; k < dims; ++k) {
                            double dd = pos[(int64_t)i * dims + k] - pos[(int64_t)j * dims + k];
                            s2 += dd * dd;
                        }
                        double r = sqrt(s2);
                        double p = p_of(kind, p0, lam, r_cut, r);
                        if (p <= 0.0) continue;
                        if (p < pmax) {
                            double u = next_u01(&st);
                            if (!(u * pmax < p)) continue;
                        }
                        eb_push(eb, i, j);
                    }
                }
            }
        }
    }
    int64_t tot = 0;
    for (int64_t c = 0; c < n_cells; ++c) tot += H->per_cell[c].n;
    H->total = tot;
    free(cell_of);
    free(cstart);
    free(cnodes);
    return H;
}

int64_t syn_edges_count(void* h) { return h ? ((syn_edges_handle*)h)->total : -1; }

/* Copy edges (grouped by target cell, deterministic order) into caller arrays. */
void syn_edges_copy(void* h, int32_t* src, int32_t* dst) {
    syn_edges_handle* H = (syn_edges_handle*)h;
    int64_t o = 0;
    for (int64_t c = 0; c < H->n_cells; ++c) {
        edge_buf* b = &H->per_cell[c];
        if (b->n) {
            memcpy(src + o, b->src, (size_t)b->n * sizeof(int32_t));
            memcpy(dst + o, b->dst, (size_t)b->n * sizeof(int32_t));
        }
        o += b->n;
    }
}

void syn_edges_free(void* h) {
    syn_edges_handle* H = (syn_edges_handle*)h;
    if (!H) return;
    for (int64_t c = 0; c < H->n_cells; ++c) {
        free(H->per_cell[c].src);
        free(H->per_cell[c].dst);
    }
    free(H->per_cell);
    free(H);
}

int syn_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
