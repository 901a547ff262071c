// Edge-scoring MLP (64 -> 256 -> 256 -> 1) on gfx950 matrix cores.
//
// BF16 operands, FP32 accumulation (v_mfma_f32_32x32x16_bf16), FP32 master
// weights and Adam state.  Rounding points (mirrored by the CPU reference):
// the input features, W1 and W2 are rounded to BF16; H1 and H2 are rounded
// to BF16 after bias + ReLU; in the backward pass dH2 and dH1 are rounded to
// BF16 before they enter a matrix product.  The head (H2 . w3 + b3), the
// binary cross-entropy with logits and all gradients are FP32.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstdint>

#include "internal.h"
#include "philox.h"

namespace geonet {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Round to nearest, ties to even; infinities stay, NaNs become quiet NaNs.
// Branch-free (a select), since it runs once per activation.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x) {
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    const uint32_t rne = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    const uint32_t qnan = (u >> 16) | 0x40u;
    return static_cast<uint16_t>((u & 0x7FFFFFFFu) > 0x7F800000u ? qnan : rne);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
    return __builtin_bit_cast(float, static_cast<uint32_t>(b) << 16);
}

// Positions of W1[k][n] and W2[k][n] in the fused forward kernel's LDS images
// (see mlp_forward_fused_kernel): row n holds column n of the weight matrix;
// within a row, W2's k order follows the layout of the first product's
// accumulators (slot q of row n holds k = 32t + 16f + 8(j/4) + 4h + j%4 for
// q = 16(2t + f) + 8h + j), and the 16-byte groups of row n are XOR-swizzled
// with n mod 8 so that 32 lanes reading one group of 32 rows spread over the
// LDS banks.
__device__ __forceinline__ int w1_image_index(int k, int n) {
    return n * kMlpIn + (((k >> 3) ^ (n & 7)) << 3) + (k & 7);
}

__device__ __forceinline__ int w2_image_index(int k, int n) {
    const int t = k >> 5, f = (k >> 4) & 1, r2 = k & 15;
    const int h = (r2 >> 2) & 1, j = 4 * (r2 >> 3) + (r2 & 3);
    const int q = 16 * (2 * t + f) + 8 * h + j;
    return n * kMlpH + (((q >> 3) ^ (n & 7)) << 3) + (q & 7);
}

// ---------------------------------------------------------------------------
// C[M x N] = op(A)[M x K] * op(B)[K x N], BF16 operands, FP32 accumulation.
// A element (m, k) at A[m*a_rs + k*a_cs]; B element (k, n) at B[k*b_rs + n*b_cs].
// Every operand has a unit stride along k or along m / n; it is read in
// 16-byte groups of 8 elements along that dimension (a k-contiguous group
// goes to LDS as is, an m- or n-contiguous one is transposed on the way,
// since LDS holds both tiles k-contiguous for the MFMA fragments).
// Block tile BM x BN, four waves of (BM/2) x (BN/2) (tiles of
// v_mfma_f32_32x32x16_bf16), K staged KS at a time (32 or 128); the next
// stage's groups are loaded into registers while the current stage's MFMAs
// run.  Split-K: blockIdx.z takes K range [z*k_chunk, min(K, (z+1)*k_chunk)).
// BF16 epilogues go through LDS: the block's output tile is staged there
// once and written with 16-byte stores, row-major into out_bf16 and/or
// transposed into out_t ([N][ldt]: column n of C is row n of out_t, its
// entries m0.. contiguous; entries M .. ldt-1 of every row are written as
// zero, so that a later product may run its K over ldt, a multiple of 8).
// ---------------------------------------------------------------------------
enum Epilogue { kBiasReluBf16 = 0, kMaskBf16 = 1, kAtomicF32 = 2, kHeadBf16 = 3, kChainBf16 = 4 };

// Head-epilogue inputs and outputs (the H2 product's epilogue).
struct HeadArgs {
    const float* w3;
    const float* b3;
    const float* y;
    float* logits;
    uint16_t* dH2;           // [B][256] row-major
    uint16_t* dH2t;          // [256][ldt] transposed, rows B .. ldt-1 zero
    float* part;             // [kHeadReplicas][kHeadPart]: w3 gradient, b2 gradient (column sums of the BF16
                             // dH2), b3 gradient, loss (sum of per-row losses / B)
    int64_t B, ldt;
};

struct GemmArgs {
    const uint16_t* A;
    const uint16_t* B;
    int64_t M, N, K, k_chunk;
    int64_t a_rs, a_cs, b_rs, b_cs;
    const float* bias;        // kBiasReluBf16: [N]
    const uint32_t* mask_bits; // kMaskBf16: [M][N/32] bits, keep where set
    uint16_t* out_bf16;       // [M x N] row-major, or null
    uint16_t* out_t;          // [N x ldt] transposed, or null (BF16 epilogues)
    int64_t ldt;              // row length of out_t (>= M, a multiple of 8)
    float* out_f32;           // [M x N] row-major (atomic add)
    HeadArgs head;            // kHeadBf16: the head that follows the product
    // optional: A given as FP32 rows (a32, [M][K], K <= KS), standardised and
    // rounded on the way in: BF16((x - a_shift[k]) * a_scale[k])
    const float* a32;
    const float* a_shift;
    const float* a_scale;
    uint16_t* a_t;            // optional: that BF16 A tile written transposed ([K][ldt], rows M .. ldt-1 zero)
    float* colsum_part;       // kMaskBf16, BN = N: BF16 column sums of the tile added into replica
                              // (row block mod kHeadReplicas) of [kHeadReplicas][kHeadPart] at offset 2N + 8
    // kChainBf16 (64 x 256 tiles): the BF16 tile, after bias + ReLU and the
    // transposed store, is the A operand of a second product with B2
    // (k-contiguous, [N2 = 256][K2]) and bias2, followed by the head; the
    // tile's nonzero pattern is written as bits (mask_out, [M][N/32])
    const uint16_t* B2;
    const float* bias2;
    int64_t K2;
    uint32_t* mask_out;
};

// LDS rows hold KS + 8 elements (padded against bank conflicts).
template <int KS>
constexpr int lds_k() { return KS + 8; }

// 16-byte groups of a BM x KS tile per thread (256 threads).
template <int BM, int BN, int KS>
struct StageRegs {
    uint4 a[BM * KS / 8 / 256];
    uint4 b[BN * KS / 8 / 256];
};

// Group e of an R-row tile: for a k-contiguous operand, tile row
// e / (KS / 8) and k offset (e % (KS / 8)) * 8; for an m/n-contiguous one, k
// offset e / (R / 8) and tile row (e % (R / 8)) * 8.
template <int R, int KS>
__device__ __forceinline__ void group_pos(int e, bool kc, int* row, int* kk) {
    *row = kc ? e / (KS / 8) : (e % (R / 8)) * 8;
    *kk = kc ? (e % (KS / 8)) * 8 : e / (R / 8);
}

template <int BM, int BN, int KS>
__device__ __forceinline__ void load_stage(StageRegs<BM, BN, KS>& r, const GemmArgs& g, bool a_kc, bool b_kc,
                                           int64_t m0, int64_t n0, int64_t k0, int64_t k_hi, int tid) {
#pragma unroll
    for (int q = 0; q < BM * KS / 8 / 256; ++q) {
        int row, kk;
        group_pos<BM, KS>(tid + 256 * q, a_kc, &row, &kk);
        const int64_t m = m0 + row, k = k0 + kk;
        uint4 va = make_uint4(0u, 0u, 0u, 0u);
        if (m < g.M && k < k_hi) {
            if (g.a32) {
                // 8 FP32 features of row m (k-contiguous), the input's rounding point
                const float4 x0 = *reinterpret_cast<const float4*>(g.a32 + m * g.a_rs + k);
                const float4 x1 = *reinterpret_cast<const float4*>(g.a32 + m * g.a_rs + k + 4);
                const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
                uint32_t w[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t f = k + 2 * j;
                    const uint32_t lo = f32_to_bf16_bits((x[2 * j] - g.a_shift[f]) * g.a_scale[f]);
                    const uint32_t hi = f32_to_bf16_bits((x[2 * j + 1] - g.a_shift[f + 1]) * g.a_scale[f + 1]);
                    w[j] = lo | (hi << 16);
                }
                va = make_uint4(w[0], w[1], w[2], w[3]);
            } else {
                va = *reinterpret_cast<const uint4*>(g.A + m * g.a_rs + k * g.a_cs);
            }
        }
        r.a[q] = va;
    }
#pragma unroll
    for (int q = 0; q < BN * KS / 8 / 256; ++q) {
        int row, kk;
        group_pos<BN, KS>(tid + 256 * q, b_kc, &row, &kk);
        const int64_t n = n0 + row, k = k0 + kk;
        uint4 vb = make_uint4(0u, 0u, 0u, 0u);
        if (n < g.N && k < k_hi) vb = *reinterpret_cast<const uint4*>(g.B + k * g.b_rs + n * g.b_cs);
        r.b[q] = vb;
    }
}

// Writes 8 BF16 of a group to LDS: along k (one 16-byte store) or down 8 rows.
template <int KS>
__device__ __forceinline__ void put_group(uint16_t (*T)[lds_k<KS>()], int row, int kk, bool kc, const uint4& v) {
    if (kc) {
        *reinterpret_cast<uint4*>(&T[row][kk]) = v;
    } else {
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            T[row + 2 * i][kk] = static_cast<uint16_t>(w[i] & 0xFFFFu);
            T[row + 2 * i + 1][kk] = static_cast<uint16_t>(w[i] >> 16);
        }
    }
}

template <int BM, int BN, int KS>
__device__ __forceinline__ void store_stage(const StageRegs<BM, BN, KS>& r, bool a_kc, bool b_kc, int tid,
                                            uint16_t (*As)[lds_k<KS>()], uint16_t (*Bs)[lds_k<KS>()]) {
#pragma unroll
    for (int q = 0; q < BM * KS / 8 / 256; ++q) {
        int row, kk;
        group_pos<BM, KS>(tid + 256 * q, a_kc, &row, &kk);
        put_group<KS>(As, row, kk, a_kc, r.a[q]);
    }
#pragma unroll
    for (int q = 0; q < BN * KS / 8 / 256; ++q) {
        int row, kk;
        group_pos<BN, KS>(tid + 256 * q, b_kc, &row, &kk);
        put_group<KS>(Bs, row, kk, b_kc, r.b[q]);
    }
}

// Block tile BM x BN (64 or 128 each), four waves in a 2 x 2 arrangement,
// each wave (BM/2) x (BN/2) = TM x TN tiles of 32 x 32.

// Head, loss and dH2 of the 64 rows m0.. whose H2 (BF16, after bias and
// ReLU) a 256-thread workgroup holds in LDS: four threads per row form the
// logit (64 products each, then two exchanges); each thread then owns one
// column for the dH2 values (rounded to BF16 in place in LDS) and that
// column's w3 and b2 gradient sums; dH2 leaves row-major and transposed with
// 16-byte stores.  The workgroup's sums go into replica (workgroup mod
// kHeadReplicas) of the partial sums; head_finish adds the replicas into
// the gradient.
__device__ __forceinline__ void head_rows(uint16_t (*Hs)[kMlpH + 8], const HeadArgs& a, int64_t m0) {
    __shared__ float dls[64], ls[64];
    const int tid = threadIdx.x;
    {
        const int r = tid >> 2, part = tid & 3;
        float s = 0.0f;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const int c = part * 64 + g * 8;
            const uint4 v = *reinterpret_cast<const uint4*>(&Hs[r][c]);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                s += bf16_bits_to_f32(static_cast<uint16_t>(w[q] & 0xFFFFu)) * a.w3[c + 2 * q];
                s += bf16_bits_to_f32(static_cast<uint16_t>(w[q] >> 16)) * a.w3[c + 2 * q + 1];
            }
        }
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        if (part == 0) {
            const int64_t m = m0 + r;
            float dl = 0.0f, l = 0.0f;
            if (m < a.B) {
                const float logit = s + a.b3[0];
                a.logits[m] = logit;
                const float inv_b = 1.0f / static_cast<float>(a.B);
                const float y = a.y[m];
                const float p = 1.0f / (1.0f + expf(-logit));
                dl = (p - y) * inv_b;
                // log(1 + exp(-|z|)) + max(z, 0) - z*y
                l = (log1pf(expf(-fabsf(logit))) + fmaxf(logit, 0.0f) - logit * y) * inv_b;
            }
            dls[r] = dl;
            ls[r] = l;
        }
    }
    __syncthreads();
    {
        const int n = tid;
        const float w3n = a.w3[n];
        float gw3 = 0.0f, gb2 = 0.0f;
        for (int r = 0; r < 64; ++r) {
            const float h = bf16_bits_to_f32(Hs[r][n]);
            const float dl = dls[r];
            const uint16_t g = f32_to_bf16_bits(h > 0.0f ? dl * w3n : 0.0f);
            Hs[r][n] = g;
            gb2 += bf16_bits_to_f32(g);
            gw3 += dl * h;
        }
        float* part = a.part + (blockIdx.y % kHeadReplicas) * kHeadPart;
        atomicAdd(part + n, gw3);
        atomicAdd(part + kMlpH + n, gb2);
        if (n < 2) {
            float acc = 0.0f;
            for (int r = 0; r < 64; ++r) acc += n == 0 ? ls[r] : dls[r];
            atomicAdd(part + 2 * kMlpH + n, acc);
        }
    }
    __syncthreads();
    for (int e = tid; e < 64 * kMlpH / 8; e += 256) {
        const int r = e / (kMlpH / 8), c = (e % (kMlpH / 8)) * 8;
        if (m0 + r < a.B) *reinterpret_cast<uint4*>(a.dH2 + (m0 + r) * kMlpH + c) = *reinterpret_cast<const uint4*>(&Hs[r][c]);
    }
    for (int e = tid; e < 64 * kMlpH / 8; e += 256) {
        const int n = e / 8, r = (e % 8) * 8;
        const int64_t m = m0 + r;
        if (m >= a.ldt) continue;
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            w[q] = static_cast<uint32_t>(Hs[r + 2 * q][n]) | (static_cast<uint32_t>(Hs[r + 2 * q + 1][n]) << 16);
        *reinterpret_cast<uint4*>(a.dH2t + n * a.ldt + m) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// B stages of the chained second product: 256 columns x 32 k of the
// k-contiguous B2 (rows of k2), four 16-byte groups per thread held in
// registers as native vectors (copies of the uint4 class become memcpys
// through a stack slot).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct StageB {
    u32x4 b[4];
};

__device__ __forceinline__ void load_b_stage(StageB& r, const uint16_t* B2, int64_t k2, int64_t k0, int tid) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int row, kk;
        group_pos<256, 32>(tid + 256 * q, true, &row, &kk);
        r.b[q] = *reinterpret_cast<const u32x4*>(B2 + static_cast<int64_t>(row) * k2 + k0 + kk);
    }
}

template <int KSL>
__device__ __forceinline__ void store_b_stage(const StageB& r, int tid, uint16_t (*Bs)[lds_k<KSL>()]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int row, kk;
        group_pos<256, 32>(tid + 256 * q, true, &row, &kk);
        *reinterpret_cast<u32x4*>(&Bs[row][kk]) = r.b[q];
    }
}

// LDS of a block: the A and B stages during the K loop; afterwards the
// output tile (and for kMaskBf16 the mask bits), rows padded by 8.  The
// chained product keeps its first tile beside the stages (the second
// product's B stages reuse them).
template <int kEpi, int BM, int BN, int KS>
constexpr int gemm_lds_elems() {
    constexpr int stage = (BM + BN) * lds_k<KS>();
    constexpr int out = BM * (BN + 8) + (kEpi == kMaskBf16 ? BM * (BN / 16) : 0);
    if (kEpi == kChainBf16) return stage + BM * (BN + 8);
    return kEpi == kAtomicF32 ? stage : (stage > out ? stage : out);
}

template <int kEpi, int BM, int BN, int KS>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
    constexpr int TM = BM / 64, TN = BN / 64;
    __shared__ __attribute__((aligned(16))) uint16_t lds[gemm_lds_elems<kEpi, BM, BN, KS>()];
    uint16_t (*As)[lds_k<KS>()] = reinterpret_cast<uint16_t (*)[lds_k<KS>()]>(lds);                      // [m][k]
    uint16_t (*Bs)[lds_k<KS>()] = reinterpret_cast<uint16_t (*)[lds_k<KS>()]>(lds + BM * lds_k<KS>());   // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = static_cast<int64_t>(blockIdx.y) * BM, n0 = static_cast<int64_t>(blockIdx.x) * BN;
    const int64_t k_lo = static_cast<int64_t>(blockIdx.z) * g.k_chunk;
    const int64_t k_hi = k_lo + g.k_chunk < g.K ? k_lo + g.k_chunk : g.K;
    const bool a_kc = g.a_cs == 1, b_kc = g.b_rs == 1;
    f32x16 acc[TM][TN];
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[tm][tn][i] = 0.0f;
    StageRegs<BM, BN, KS> r;
    if (k_lo < k_hi) load_stage<BM, BN, KS>(r, g, a_kc, b_kc, m0, n0, k_lo, k_hi, tid);
    for (int64_t k0 = k_lo; k0 < k_hi; k0 += KS) {
        store_stage<BM, BN, KS>(r, a_kc, b_kc, tid, As, Bs);
        __syncthreads();
        if (k0 + KS < k_hi) load_stage<BM, BN, KS>(r, g, a_kc, b_kc, m0, n0, k0 + KS, k_hi, tid);
#pragma unroll
        for (int ks = 0; ks < KS; ks += 16) {
            // lane supplies row (lane % 32) and k = ks + 8*(lane / 32) .. +7
            const int rr = lane & 31, kq = ks + 8 * (lane >> 5);
            bf16x8 a[TM], b[TN];
#pragma unroll
            for (int t = 0; t < TM; ++t) a[t] = *reinterpret_cast<const bf16x8*>(&As[wm * (BM / 2) + t * 32 + rr][kq]);
#pragma unroll
            for (int t = 0; t < TN; ++t) b[t] = *reinterpret_cast<const bf16x8*>(&Bs[wn * (BN / 2) + t * 32 + rr][kq]);
#pragma unroll
            for (int tm = 0; tm < TM; ++tm)
#pragma unroll
                for (int tn = 0; tn < TN; ++tn)
                    acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[tm], b[tn], acc[tm][tn], 0, 0, 0);
        }
        __syncthreads();
    }
    // acc[tm][tn][i] holds C[m][n]: n = lane % 32, m = 8*(i/4) + 4*(lane/32) + i%4 within the 32 x 32 tile
    if constexpr (kEpi == kAtomicF32) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int tn = 0; tn < TN; ++tn) {
                const int64_t n = n0 + wn * (BN / 2) + tn * 32 + (lane & 31);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int64_t m = m0 + wm * (BM / 2) + tm * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                    if (m < g.M && n < g.N) atomicAdd(g.out_f32 + m * g.N + n, acc[tm][tn][i]);
                }
            }
        return;
    }
    if (g.a_t && n0 == 0) {
        // the (single-stage) A tile is still in LDS: write it transposed,
        // column k of the tile to row k of a_t
        for (int e = tid; e < BM * KS / 8; e += 256) {
            const int k = e / (BM / 8), r = (e % (BM / 8)) * 8;
            const int64_t m = m0 + r;
            if (k >= g.K || m >= g.ldt) continue;
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t lo = m + 2 * q < g.M ? As[r + 2 * q][k] : 0u;
                const uint32_t hi = m + 2 * q + 1 < g.M ? As[r + 2 * q + 1][k] : 0u;
                w[q] = lo | (hi << 16);
            }
            *reinterpret_cast<uint4*>(g.a_t + k * g.ldt + m) = make_uint4(w[0], w[1], w[2], w[3]);
        }
        __syncthreads();
    }
    // (the K loop ended on a barrier: the stages' LDS is free)
    constexpr int CW = BN + 8;
    uint16_t (*Cs)[CW] = reinterpret_cast<uint16_t (*)[CW]>(lds + (kEpi == kChainBf16 ? (BM + BN) * lds_k<KS>() : 0));
    uint32_t* Mb = reinterpret_cast<uint32_t*>(lds + BM * CW);   // kMaskBf16: [BM][BN / 32] bits
    constexpr int groups = BM * BN / 8;          // 16-byte groups of the tile
    if constexpr (kEpi == kMaskBf16) {
        // the tile's mask bits (N is a multiple of 32, n0 of BN)
        for (int e = tid; e < BM * (BN / 32); e += 256) {
            const int r = e / (BN / 32), q = e % (BN / 32);
            const int64_t m = m0 + r;
            Mb[e] = m < g.M ? g.mask_bits[m * (g.N / 32) + n0 / 32 + q] : 0u;
        }
        __syncthreads();
    }
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            const int nl = wn * (BN / 2) + tn * 32 + (lane & 31);
            const int64_t n = n0 + nl;
            float bn = 0.0f;
            if (kEpi != kMaskBf16) bn = n < g.N ? g.bias[n] : 0.0f;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int ml = wm * (BM / 2) + tm * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                const float v = acc[tm][tn][i];
                float o;
                if (kEpi != kMaskBf16) {
                    const float h = v + bn;
                    o = h > 0.0f ? h : 0.0f;
                } else {
                    o = v * (((Mb[ml * (BN / 32) + (nl >> 5)] >> (nl & 31)) & 1u) ? 1.0f : 0.0f);
                }
                Cs[ml][nl] = f32_to_bf16_bits(o);
            }
        }
    __syncthreads();
    if constexpr (kEpi == kMaskBf16) {
        if (g.colsum_part && BN == 256) {
            // column sums of the BF16 tile (rows past M are zero), one column per thread
            const int n = tid;
            float acc = 0.0f;
            for (int r = 0; r < BM; ++r) acc += bf16_bits_to_f32(Cs[r][n]);
            atomicAdd(g.colsum_part + (blockIdx.y % kHeadReplicas) * kHeadPart + 2 * kMlpH + 8 + n, acc);
        }
    }
    if constexpr (kEpi == kHeadBf16) {
        // the whole row width is in the tile: the head follows in place
        static_assert(BM == 64 && BN == kMlpH, "the head epilogue needs 64 x 256 tiles");
        head_rows(reinterpret_cast<uint16_t (*)[kMlpH + 8]>(lds), g.head, m0);
        return;
    }
    if (g.out_bf16) {
        for (int e = tid; e < groups; e += 256) {
            const int r = e / (BN / 8), c = (e % (BN / 8)) * 8;
            const int64_t m = m0 + r, n = n0 + c;
            if (m < g.M && n < g.N)
                *reinterpret_cast<uint4*>(g.out_bf16 + m * g.N + n) = *reinterpret_cast<const uint4*>(&Cs[r][c]);
        }
    }
    if constexpr (kEpi == kChainBf16) {
        static_assert(BM == 64 && BN == kMlpH, "the chained product needs 64 x 256 tiles");
        // nonzero bits of the first tile (the ReLU mask of the later backward product)
        for (int e = tid; e < BM * (BN / 32); e += 256) {
            const int r = e / (BN / 32), q = e % (BN / 32);
            uint32_t bits = 0;
#pragma unroll 8
            for (int b = 0; b < 32; ++b) bits |= (Cs[r][32 * q + b] != 0 ? 1u : 0u) << b;
            if (m0 + r < g.M) g.mask_out[(m0 + r) * (BN / 32) + q] = bits;
        }
    }
    if (g.out_t) {
        // group e: column c of the tile, rows r .. r+7 (consecutive threads take
        // consecutive row groups of one column, so their stores are contiguous)
        for (int e = tid; e < groups; e += 256) {
            const int c = e / (BM / 8), r = (e % (BM / 8)) * 8;
            const int64_t m = m0 + r, n = n0 + c;
            if (n >= g.N || m >= g.ldt) continue;
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t lo = m + 2 * q < g.M ? Cs[r + 2 * q][c] : 0u;
                const uint32_t hi = m + 2 * q + 1 < g.M ? Cs[r + 2 * q + 1][c] : 0u;
                w[q] = lo | (hi << 16);
            }
            *reinterpret_cast<uint4*>(g.out_t + n * g.ldt + m) = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
    if constexpr (kEpi == kChainBf16) {
        // second product: tile = BF16(ReLU(Cs B2 + bias2)), Cs read in place as
        // the A operand, B2 staged KS rows of k at a time (next stage in
        // registers while the MFMAs run); then the head on the new tile
        f32x16 acc2[TN];
#pragma unroll
        for (int tn = 0; tn < TN; ++tn)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc2[tn][i] = 0.0f;
        // (stages of 32 k in the first 32 columns of Bs: fewer registers in flight)
        constexpr int KS2 = 32;
        static_assert(BN == 256 && KS2 == 32, "the chained stage holds 256 x 32");
        StageB rb;
        load_b_stage(rb, g.B2, g.K2, 0, tid);
        for (int64_t k0 = 0; k0 < g.K2; k0 += KS2) {
            store_b_stage<KS>(rb, tid, Bs);
            __syncthreads();
            // (the last pass reloads its own stage: an unconditional load keeps rb in registers)
            load_b_stage(rb, g.B2, g.K2, k0 + KS2 < g.K2 ? k0 + KS2 : k0, tid);
#pragma unroll
            for (int ks = 0; ks < KS2; ks += 16) {
                const int rr = lane & 31, kq = ks + 8 * (lane >> 5);
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&Cs[wm * (BM / 2) + rr][k0 + kq]);
#pragma unroll
                for (int tn = 0; tn < TN; ++tn) {
                    const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn * (BN / 2) + tn * 32 + rr][kq]);
                    acc2[tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc2[tn], 0, 0, 0);
                }
            }
            __syncthreads();
        }
        // every read of the first tile is done: the second one replaces it
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
            const int nl = wn * (BN / 2) + tn * 32 + (lane & 31);
            const float bn = g.bias2[nl];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int ml = wm * (BM / 2) + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                const float h = acc2[tn][i] + bn;
                Cs[ml][nl] = f32_to_bf16_bits(h > 0.0f ? h : 0.0f);
            }
        }
        __syncthreads();
        head_rows(reinterpret_cast<uint16_t (*)[kMlpH + 8]>(&Cs[0][0]), g.head, m0);
    }
}

// Column statistics of a [rows][64] FP32 feature matrix, in FP64 with a
// fixed summation order: pass 0 sums x, pass 1 sums (x - mean)^2.  Thread t
// of a workgroup owns column t % 64 and every fourth row of the workgroup's
// stride; the four partials per column are added in LDS, one row of
// partials per workgroup.
__global__ void __launch_bounds__(256) colstats_kernel(const float* X, int64_t rows, const double* mean,
                                                       double* part) {
    __shared__ double red[4][kMlpIn];
    const int c = threadIdx.x % kMlpIn, q = threadIdx.x / kMlpIn;
    const double mu = mean ? mean[c] : 0.0;
    double acc = 0.0;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + q; r < rows; r += static_cast<int64_t>(gridDim.x) * 4) {
        const double x = static_cast<double>(X[r * kMlpIn + c]) - mu;
        acc += mean ? x * x : x;
    }
    red[q][c] = acc;
    __syncthreads();
    if (q == 0) part[static_cast<int64_t>(blockIdx.x) * kMlpIn + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// Sums the partial rows in order.  pass 0: mean = sum / rows.  pass 1:
// std = sqrt(sum / (rows - 1)) (0 for one row), shift = mean,
// scale = 1/std where std > 1e-6, else 0 (a constant feature is dropped).
__global__ void __launch_bounds__(64) colstats_finish_kernel(const double* part, int blocks, int64_t rows, int pass,
                                                             double* mean, float* shift, float* scale) {
    const int c = threadIdx.x;
    double acc = 0.0;
    for (int b = 0; b < blocks; ++b) acc += part[static_cast<int64_t>(b) * kMlpIn + c];
    if (pass == 0) {
        mean[c] = acc / static_cast<double>(rows);
        return;
    }
    const double sd = rows > 1 ? sqrt(acc / static_cast<double>(rows - 1)) : 0.0;
    shift[c] = static_cast<float>(mean[c]);
    scale[c] = sd > 1e-6 ? static_cast<float>(1.0 / sd) : 0.0f;
}

// A keyed permutation of [0, n): a four-round balanced Feistel network on
// 2h bits (2^(2h) >= n, so at most 4n values) whose round function is
// Philox4x32-10 of (right half, round, epoch), walked until the value falls
// below n (cycle walking; any permutation of the larger domain restricted
// this way is a permutation of [0, n)).
struct ShufflePerm {
    uint64_t n;
    uint32_t k0, k1, epoch;
    int h;
};

__device__ __forceinline__ uint64_t shuffle_index(uint64_t i, const ShufflePerm& p) {
    const uint32_t mask = (p.h >= 32) ? 0xFFFFFFFFu : ((1u << p.h) - 1u);
    uint64_t x = i;
    do {
        uint32_t L = static_cast<uint32_t>(x >> p.h) & mask, R = static_cast<uint32_t>(x) & mask;
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
            const uint4 f = philox4x32_10(make_uint4(R, r, p.epoch, 0x53485546u), p.k0, p.k1);
            const uint32_t nr = (L ^ f.x) & mask;
            L = R;
            R = nr;
        }
        x = (static_cast<uint64_t>(L) << p.h) | R;
    } while (x >= p.n);
    return x;
}

// Rows [a0, a0 + count) of the shuffled order gathered into xs / ys.
__global__ void __launch_bounds__(256) gather_shuffled_kernel(const float* X, const float* y, ShufflePerm p,
                                                              int64_t a0, int64_t count, float* xs, float* ys) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;   // one thread per 16 floats
    const int64_t r = i / 4;
    if (r >= count) return;
    const int part = static_cast<int>(i % 4);
    const int64_t src = static_cast<int64_t>(shuffle_index(static_cast<uint64_t>(a0 + r), p));
    const float4* in = reinterpret_cast<const float4*>(X + src * kMlpIn) + 4 * part;
    float4* out = reinterpret_cast<float4*>(xs + r * kMlpIn) + 4 * part;
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = in[k];
    if (part == 0) ys[r] = y[src];
}

__global__ void __launch_bounds__(256) shuffle_index_kernel(ShufflePerm p, int64_t* out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < static_cast<int64_t>(p.n)) out[i] = static_cast<int64_t>(shuffle_index(static_cast<uint64_t>(i), p));
}

ShufflePerm make_perm(int64_t n, uint64_t seed, uint32_t epoch) {
    ShufflePerm p{};
    p.n = static_cast<uint64_t>(n);
    p.k0 = static_cast<uint32_t>(seed);
    p.k1 = static_cast<uint32_t>(seed >> 32);
    p.epoch = epoch;
    int bits = 1;
    while (bits < 63 && (uint64_t(1) << bits) < p.n) ++bits;
    p.h = (bits + 1) / 2;
    return p;
}

// The head's replicas summed in a fixed order into the gradient (w3, b2, b3)
// and the loss (also into loss_out when given), then cleared for the next
// step (one 256-thread workgroup).
__device__ __forceinline__ void head_finish(float* part, float* grad, float* loss, float* loss_out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kHeadPart; i += gridDim.x * blockDim.x) {
        if (i >= 2 * kMlpH + 2 && i < 2 * kMlpH + 8) continue;   // unused
        float v[kHeadReplicas];
#pragma unroll
        for (int r = 0; r < kHeadReplicas; ++r) v[r] = part[r * kHeadPart + i];   // all loads in flight
        float acc = 0.0f;
#pragma unroll
        for (int r = 0; r < kHeadReplicas; ++r) {
            acc += v[r];
            part[r * kHeadPart + i] = 0.0f;
        }
        if (i < kMlpH) grad[kMlpW3Off + i] += acc;
        else if (i < 2 * kMlpH) grad[kMlpB2Off + (i - kMlpH)] += acc;
        else if (i == 2 * kMlpH) {
            loss[0] = acc;
            if (loss_out) loss_out[0] = acc;
        }
        else if (i == 2 * kMlpH + 1) grad[kMlpB3Off] += acc;
        else grad[kMlpB1Off + (i - 2 * kMlpH - 8)] += acc;
    }
}

// The replicas of the head's and the b1 column sums added into the gradient
// and the loss (one thread per entry).
__global__ void __launch_bounds__(64) finish_kernel(float* part, float* grad, float* loss, float* loss_out) {
    head_finish(part, grad, loss, loss_out);
}

// Adam on the flat FP32 parameter vector; refreshes the BF16 copies of W1, W2.
struct AdamArgs {
    float* p;
    float* m;
    float* v;
    float* g;          // read, then cleared for the next step's accumulation
    uint16_t* w1b;
    uint16_t* w2b;
    uint16_t* w2c;
    uint16_t* w1t;
    uint16_t* w2p;
    int64_t n;
    float lr, b1, b2, eps, c1, c2;   // c1 = 1 - b1^t, c2 = 1 - b2^t
};

__global__ void __launch_bounds__(256) adam_kernel(AdamArgs a) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const float gi = a.g[i];
    a.g[i] = 0.0f;
    const float m = a.b1 * a.m[i] + (1.0f - a.b1) * gi;
    const float v = a.b2 * a.v[i] + (1.0f - a.b2) * gi * gi;
    a.m[i] = m;
    a.v[i] = v;
    const float p = a.p[i] - a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
    a.p[i] = p;
    if (i < kMlpW1) {
        const uint16_t b = f32_to_bf16_bits(p);
        const int k = static_cast<int>(i) / kMlpH, n = static_cast<int>(i) % kMlpH;
        a.w1b[n * kMlpIn + k] = b;
        a.w1t[w1_image_index(k, n)] = b;
    } else if (i >= kMlpW2Off && i < kMlpW2Off + kMlpW2) {
        const int e = static_cast<int>(i - kMlpW2Off);
        const uint16_t b = f32_to_bf16_bits(p);
        a.w2b[e] = b;
        a.w2c[(e % kMlpH) * kMlpH + e / kMlpH] = b;
        a.w2p[w2_image_index(e / kMlpH, e % kMlpH)] = b;
    }
}

// BF16 copies of W1 and W2 from the FP32 parameters: W1 transposed (w1b,
// [n][k]), W2 row-major (w2b) and transposed (w2c), and the fused forward
// kernel's LDS images.
__global__ void __launch_bounds__(256) weights_bf16_kernel(const float* params, uint16_t* w1b, uint16_t* w2b,
                                                           uint16_t* w2c, uint16_t* w1t, uint16_t* w2p) {
    const int i = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < kMlpW1) {
        const uint16_t b = f32_to_bf16_bits(params[kMlpW1Off + i]);
        const int k = i / kMlpH, n = i % kMlpH;
        w1b[n * kMlpIn + k] = b;
        w1t[w1_image_index(k, n)] = b;
    } else if (i < kMlpW1 + kMlpW2) {
        const int e = i - kMlpW1;
        const uint16_t b = f32_to_bf16_bits(params[kMlpW2Off + e]);
        w2b[e] = b;
        w2c[(e % kMlpH) * kMlpH + e / kMlpH] = b;
        w2p[w2_image_index(e / kMlpH, e % kMlpH)] = b;
    }
}

// ---------------------------------------------------------------------------
// Fused forward pass for inference: logits = head(BF16(ReLU(BF16(ReLU(Xb W1
// + b1)) W2 + b2))) with the same rounding points as the layered path.  Both
// products are computed transposed (H1^T = W1^T Xb^T, H2^T = W2^T H1^T) so
// that every lane owns one row (pair) from input to logit: the MFMA B
// fragments are the lane's own standardised features (read from memory) and
// then its own H1 values (straight from the first product's accumulators,
// which is why W2's image orders k as they lie there); the A fragments come
// from the weight images in LDS (32 + 128 KiB, staged once per workgroup).
// One wave per 32 rows, rows strided over the grid; the head's dot product
// ends with one exchange between the two half-waves that share a row.
// ---------------------------------------------------------------------------
struct FwdArgs {
    const float* X;
    const float* shift;
    const float* scale;
    const uint16_t* w1t;
    const uint16_t* w2p;
    const float* params;
    float* logits;
    int64_t B;
};

constexpr int kFwdThreads = 512;   // eight waves: two per SIMD

__global__ void __launch_bounds__(kFwdThreads) mlp_forward_fused_kernel(FwdArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t W1s[kMlpH * kMlpIn];
    __shared__ __attribute__((aligned(16))) uint16_t W2s[kMlpH * kMlpH];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, col = lane & 31;
    constexpr int kWaves = kFwdThreads / 64;
    const int64_t n_tiles = (a.B + 31) / 32;
    const int64_t tile_stride = static_cast<int64_t>(gridDim.x) * kWaves;
    // The lane's raw features of its next tile (row m, features 16s + 8h ..
    // 16s + 8h + 7 for s = 0..3), loaded one tile ahead; the first ones are
    // in flight while the weights are staged.
    float4 xraw[8];
    auto load_x = [&](int64_t tile) {
        const int64_t m = tile * 32 + col;
        const float* xr = a.X + (m < a.B ? m : 0) * kMlpIn;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            xraw[2 * s] = reinterpret_cast<const float4*>(xr + 16 * s + 8 * h)[0];
            xraw[2 * s + 1] = reinterpret_cast<const float4*>(xr + 16 * s + 8 * h)[1];
        }
    };
    int64_t tile = static_cast<int64_t>(blockIdx.x) * kWaves + wave;
    if (tile < n_tiles) load_x(tile);
    // weights: every thread issues all its 16-byte loads before its LDS
    // writes (a fixed count per thread, so no wait sits between the loads)
    {
        constexpr int k1 = kMlpH * kMlpIn / 8 / kFwdThreads, k2 = kMlpH * kMlpH / 8 / kFwdThreads;
        uint4 r1[k1], r2[k2];
#pragma unroll
        for (int q = 0; q < k1; ++q) r1[q] = reinterpret_cast<const uint4*>(a.w1t)[q * kFwdThreads + tid];
#pragma unroll
        for (int q = 0; q < k2; ++q) r2[q] = reinterpret_cast<const uint4*>(a.w2p)[q * kFwdThreads + tid];
#pragma unroll
        for (int q = 0; q < k1; ++q) reinterpret_cast<uint4*>(W1s)[q * kFwdThreads + tid] = r1[q];
#pragma unroll
        for (int q = 0; q < k2; ++q) reinterpret_cast<uint4*>(W2s)[q * kFwdThreads + tid] = r2[q];
    }
    __syncthreads();
    const float* b1 = a.params + kMlpB1Off;
    const float* b2 = a.params + kMlpB2Off;
    const float* w3 = a.params + kMlpW3Off;
    const float b3 = a.params[kMlpB3Off];
    for (; tile < n_tiles; tile += tile_stride) {
        const int64_t m = tile * 32 + col;
        const bool valid = m < a.B;
        // B fragments of Xb^T: step s takes features 16s + 8h .. 16s + 8h + 7
        bf16x8 xb[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int f0 = 16 * s + 8 * h;
            const float4 x0 = xraw[2 * s], x1 = xraw[2 * s + 1];
            const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
            uint32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t lo = f32_to_bf16_bits((xv[2 * j] - a.shift[f0 + 2 * j]) * a.scale[f0 + 2 * j]);
                const uint32_t hi = f32_to_bf16_bits((xv[2 * j + 1] - a.shift[f0 + 2 * j + 1]) * a.scale[f0 + 2 * j + 1]);
                w[j] = lo | (hi << 16);
            }
            xb[s] = __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
        }
        if (tile + tile_stride < n_tiles) load_x(tile + tile_stride);
        // The two products interleaved over the first's output blocks: block t
        // of H1^T (n = 32t .. 32t + 31; acc1[i] is n = 32t + 8(i/4) + 4h + i%4
        // of row m) becomes, after bias + ReLU + BF16, the lane's two B
        // fragments of k step (t, f) of the second product, which go into all
        // eight accumulators of H2^T at once (acc2[u][i] is n2 = 32u + 8(i/4)
        // + 4h + i%4 of row m).  Only acc2 lives across the blocks.
        f32x16 acc2[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc2[u][i] = 0.0f;
#pragma unroll 1
        for (int t = 0; t < 8; ++t) {
            f32x16 acc1;
#pragma unroll
            for (int i = 0; i < 16; ++i) acc1[i] = 0.0f;
            const int n = 32 * t + col;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bf16x8 av = *reinterpret_cast<const bf16x8*>(&W1s[n * kMlpIn + (((2 * s + h) ^ (n & 7)) << 3)]);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, xb[s], acc1, 0, 0, 0);
            }
            bf16x8 hb[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                // values i = 8f .. 8f + 7: n = 32t + 16f + 4h + {0..3, 8..11};
                // the bias words are wave-uniform loads of both half-waves' values
                const float* bt = b1 + 32 * t + 16 * f;
                const float4 l0 = *reinterpret_cast<const float4*>(bt), l1 = *reinterpret_cast<const float4*>(bt + 4);
                const float4 u0 = *reinterpret_cast<const float4*>(bt + 8), u1 = *reinterpret_cast<const float4*>(bt + 12);
                const float4 bl = h ? l1 : l0, bh = h ? u1 : u0;
                const float bias[8] = {bl.x, bl.y, bl.z, bl.w, bh.x, bh.y, bh.z, bh.w};
                uint32_t w[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float v0 = acc1[8 * f + 2 * j] + bias[2 * j];
                    const float v1 = acc1[8 * f + 2 * j + 1] + bias[2 * j + 1];
                    w[j] = static_cast<uint32_t>(f32_to_bf16_bits(v0 > 0.0f ? v0 : 0.0f)) |
                           (static_cast<uint32_t>(f32_to_bf16_bits(v1 > 0.0f ? v1 : 0.0f)) << 16);
                }
                hb[f] = __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
            }
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int n2 = 32 * u + col;
                    const int grp = 2 * (2 * t + f) + h;
                    const bf16x8 av = *reinterpret_cast<const bf16x8*>(&W2s[n2 * kMlpH + ((grp ^ (n2 & 7)) << 3)]);
                    acc2[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, hb[f], acc2[u], 0, 0, 0);
                }
        }
        // bias + ReLU + BF16, then the head's dot product over the lane's 128
        // values of n2 and its partner half-wave's 128
        float part = 0.0f;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // n2 = 32u + 8q + 4h + r: wave-uniform loads of both halves' words
                const float* bu = b2 + 32 * u + 8 * q;
                const float* wu = w3 + 32 * u + 8 * q;
                const float4 b_0 = *reinterpret_cast<const float4*>(bu), b_1 = *reinterpret_cast<const float4*>(bu + 4);
                const float4 w_0 = *reinterpret_cast<const float4*>(wu), w_1 = *reinterpret_cast<const float4*>(wu + 4);
                const float4 bq = h ? b_1 : b_0, wq = h ? w_1 : w_0;
                const float bb[4] = {bq.x, bq.y, bq.z, bq.w}, ww[4] = {wq.x, wq.y, wq.z, wq.w};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float x = acc2[u][4 * q + r] + bb[r];
                    part += bf16_bits_to_f32(f32_to_bf16_bits(x > 0.0f ? x : 0.0f)) * ww[r];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        part += __shfl_xor(part, 32, 64);
        if (h == 0 && valid) a.logits[m] = part + b3;
    }
}

template <int kEpi, int BM, int BN, int KS>
hipError_t gemm_tile(const GemmArgs& g, int split, hipStream_t s) {
    dim3 grid(static_cast<unsigned>((g.N + BN - 1) / BN), static_cast<unsigned>((g.M + BM - 1) / BM),
              static_cast<unsigned>(split));
    hipLaunchKernelGGL((gemm_kernel<kEpi, BM, BN, KS>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// Tile shape: 64 x 64 unless that gives more than 8,192 workgroups.  These
// products are small and each K stage waits for its loads, so many resident
// workgroups per CU hide more latency than larger tiles save (measured on
// the scorer: training step 142 us with 64 x 64, 175 us with 64 x 128, 211 us
// with 128 x 128).  K stages of 128 wherever a workgroup's K range is a
// multiple of 128 (four times the bytes in flight per wait), else 32.
// GEONET_GEMM_TILE (0: 128 x 128, 1: 64 x 128, 2: 64 x 64) fixes the tile at
// compile time.
template <int kEpi>
hipError_t gemm(const GemmArgs& g, int split, hipStream_t s) {
    // every operand must have a unit stride along k or along its row/column
    // dimension, with that extent (and the split-K chunk) a multiple of 8 so
    // that each 16-byte group is entirely in or out of range
    const bool a_kc = g.a_cs == 1, b_kc = g.b_rs == 1;
    if ((!a_kc && g.a_rs != 1) || (!b_kc && g.b_cs != 1)) return hipErrorInvalidValue;
    if ((a_kc || b_kc) && (g.K % 8 != 0 || g.k_chunk % 32 != 0)) return hipErrorInvalidValue;
    if ((!a_kc && g.M % 8 != 0) || (!b_kc && g.N % 8 != 0)) return hipErrorInvalidValue;
    const bool wide = g.k_chunk % 128 == 0;
#ifdef GEONET_GEMM_TILE
    const int tile = GEONET_GEMM_TILE;
#else
    auto blocks = [&](int64_t bm, int64_t bn) { return ((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn) * split; };
    const int tile = blocks(64, 64) > 8192 ? 0 : 2;
#endif
    if (tile == 0) return wide ? gemm_tile<kEpi, 128, 128, 128>(g, split, s) : gemm_tile<kEpi, 128, 128, 32>(g, split, s);
    if (tile == 1) return wide ? gemm_tile<kEpi, 64, 128, 128>(g, split, s) : gemm_tile<kEpi, 64, 128, 32>(g, split, s);
    return wide ? gemm_tile<kEpi, 64, 64, 128>(g, split, s) : gemm_tile<kEpi, 64, 64, 32>(g, split, s);
}

}  // namespace

// Row length of the transposed activations of a B-row batch.
int64_t mlp_ldt(int64_t B) { return (B + 7) / 8 * 8; }

// Products over the batch rows with the whole 256-wide output row in one
// tile (64 x 256, K staged 64 at a time): each row tile of A is read once,
// and the head can follow the H2 product in its epilogue.  A and B must be
// k-contiguous and K a multiple of 64.
template <int kEpi>
hipError_t gemm_rows(const GemmArgs& g, hipStream_t s) {
    if (g.N != kMlpH || g.a_cs != 1 || g.b_rs != 1 || g.K % 64 != 0 || g.k_chunk != g.K) return hipErrorInvalidValue;
    return gemm_tile<kEpi, 64, kMlpH, 64>(g, 1, s);
}

// Training forward pass for B rows of features X (FP32 [B x 64]) with
// labels y, one launch: Xbt (the rounded inputs, transposed), H1t and the
// bits of H1 > 0, the logits, dH2 (and dH2t) and the head's gradient sums;
// H1 and H2 stay in LDS.
hipError_t mlp_forward(const MlpDevice& d, const float* X, int64_t B, const float* y, hipStream_t s) {
    const float* p = d.params;
    const int64_t ldt = mlp_ldt(B);
    // H1 = BF16(ReLU(BF16(standardised X) W1 + b1)); the product rounds X on
    // the way in and writes the rounded tile transposed (Xbt) for dW1
    GemmArgs g1{};
    g1.a32 = X;
    g1.a_shift = d.in_shift;
    g1.a_scale = d.in_scale;
    g1.a_t = d.Xbt;
    g1.B = d.w1b;         // B(k, n) = W1(k, n) at w1b[n * 64 + k]
    g1.M = B;
    g1.N = kMlpH;
    g1.K = kMlpIn;
    g1.k_chunk = kMlpIn;
    g1.a_rs = kMlpIn;
    g1.a_cs = 1;
    g1.b_rs = 1;
    g1.b_cs = kMlpIn;
    g1.bias = p + kMlpB1Off;
    g1.out_bf16 = nullptr;     // H1 stays in LDS for the second product; its ReLU mask leaves as bits
    g1.out_t = d.H1t;
    g1.ldt = ldt;
    g1.mask_out = d.H1bits;
    // H2 = BF16(ReLU(H1 W2 + b2)) from the H1 tile in LDS, then the head, the
    // loss and dH2 in the same workgroup
    g1.B2 = d.w2c;             // B2(k, n) = W2(k, n) at w2c[n * 256 + k]
    g1.bias2 = p + kMlpB2Off;
    g1.K2 = kMlpH;
    g1.head.w3 = p + kMlpW3Off;
    g1.head.b3 = p + kMlpB3Off;
    g1.head.y = y;
    g1.head.logits = d.logits;
    g1.head.dH2 = d.dH2;
    g1.head.dH2t = d.dH2t;
    g1.head.part = d.head_part;
    g1.head.B = B;
    g1.head.ldt = ldt;
    return gemm_rows<kChainBf16>(g1, s);
}

// Split-K of a weight gradient (K = the batch rows, padded to ldt): chunks
// of at least `rows` rows, in multiples of 128.
static void weight_split(int64_t ldt, int64_t rows, int* split, int64_t* chunk) {
    const int64_t sp = std::max<int64_t>((ldt + rows - 1) / rows, 1);
    *chunk = ((ldt + sp - 1) / sp + 127) / 128 * 128;
    *split = static_cast<int>((ldt + *chunk - 1) / *chunk);
}

// Backward pass after mlp_forward: accumulates the gradient of the mean BCE
// into d.grad (which the caller zeroed).  Every product reads k-contiguous
// operands: the weight gradients take the transposed activations.
hipError_t mlp_backward(const MlpDevice& d, int64_t B, float* loss_out, hipStream_t s) {
    const int64_t ldt = mlp_ldt(B);
    // dW2 = H1^T dH2  (M = 256, N = 256, K = ldt): 16 tiles, chunks of 2,048
    // rows (512 workgroups at 65,536 rows; fewer chunks, fewer atomics)
    int split = 1;
    int64_t chunk = ldt;
    weight_split(ldt, 2048, &split, &chunk);
    GemmArgs w2{};
    w2.A = d.H1t;
    w2.B = d.dH2t;
    w2.M = kMlpH;
    w2.N = kMlpH;
    w2.K = ldt;
    w2.k_chunk = chunk;
    w2.a_rs = ldt;
    w2.a_cs = 1;
    w2.b_rs = 1;
    w2.b_cs = ldt;
    w2.out_f32 = d.grad + kMlpW2Off;
    hipError_t e = gemm<kAtomicF32>(w2, split, s);
    if (e != hipSuccess) return e;
    // dH1 = BF16((dH2 W2^T) * [H1 > 0])  (M = B, N = 256, K = 256), written transposed
    GemmArgs h1{};
    h1.A = d.dH2;
    h1.B = d.w2b;
    h1.M = B;
    h1.N = kMlpH;
    h1.K = kMlpH;
    h1.k_chunk = kMlpH;
    h1.a_rs = kMlpH;
    h1.a_cs = 1;
    h1.b_rs = 1;          // B(k, n) = W2(n, k)
    h1.b_cs = kMlpH;
    h1.mask_bits = d.H1bits;
    h1.out_t = d.dH1t;
    h1.ldt = ldt;
    h1.colsum_part = d.head_part;      // b1 gradient: column sums of dH1
    if ((e = gemm_rows<kMaskBf16>(h1, s)) != hipSuccess) return e;
    // dW1 = Xb^T dH1  (M = 64, N = 256, K = ldt): four tiles, chunks of 512 rows
    weight_split(ldt, 512, &split, &chunk);
    GemmArgs w1{};
    w1.A = d.Xbt;
    w1.B = d.dH1t;
    w1.M = kMlpIn;
    w1.N = kMlpH;
    w1.K = ldt;
    w1.k_chunk = chunk;
    w1.a_rs = ldt;
    w1.a_cs = 1;
    w1.b_rs = 1;
    w1.b_cs = ldt;
    w1.out_f32 = d.grad + kMlpW1Off;
    if ((e = gemm<kAtomicF32>(w1, split, s)) != hipSuccess) return e;
    // the head's and the b1 sums into the gradient
    hipLaunchKernelGGL(finish_kernel, dim3((kHeadPart + 63) / 64), dim3(64), 0, s, d.head_part, d.grad, d.loss, loss_out);
    return hipGetLastError();
}

hipError_t mlp_forward_fused(const MlpDevice& d, const float* X, int64_t B, float* logits, hipStream_t s) {
    int dev = 0, n_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    FwdArgs a;
    a.X = X;
    a.shift = d.in_shift;
    a.scale = d.in_scale;
    a.w1t = d.w1t;
    a.w2p = d.w2p;
    a.params = d.params;
    a.logits = logits;
    a.B = B;
    // one workgroup per CU (the weight images fill its LDS), fewer for small B
    const int64_t blocks = std::min<int64_t>(std::max<int64_t>((B + 32 * kFwdThreads / 64 - 1) / (32 * kFwdThreads / 64), 1), n_cu);
    hipLaunchKernelGGL(mlp_forward_fused_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kFwdThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t mlp_adam(const MlpDevice& d, float lr, float beta1, float beta2, float eps, int64_t t, hipStream_t s) {
    AdamArgs a;
    a.p = d.params;
    a.m = d.adam_m;
    a.v = d.adam_v;
    a.g = d.grad;
    a.w1b = d.w1b;
    a.w2b = d.w2b;
    a.w2c = d.w2c;
    a.w1t = d.w1t;
    a.w2p = d.w2p;
    a.n = kMlpParams;
    a.lr = lr;
    a.b1 = beta1;
    a.b2 = beta2;
    a.eps = eps;
    a.c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta1), static_cast<double>(t)));
    a.c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta2), static_cast<double>(t)));
    hipLaunchKernelGGL(adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t mlp_input_stats(const float* X, int64_t rows, double* work, float* shift, float* scale, hipStream_t s) {
    double* mean = work + static_cast<int64_t>(kStatBlocks) * kMlpIn;
    const int blocks = static_cast<int>(std::min<int64_t>(kStatBlocks, (rows + 3) / 4));
    hipLaunchKernelGGL(colstats_kernel, dim3(blocks), dim3(256), 0, s, X, rows, static_cast<const double*>(nullptr),
                       work);
    hipLaunchKernelGGL(colstats_finish_kernel, dim3(1), dim3(kMlpIn), 0, s, static_cast<const double*>(work), blocks,
                       rows, 0, mean, shift, scale);
    hipLaunchKernelGGL(colstats_kernel, dim3(blocks), dim3(256), 0, s, X, rows, static_cast<const double*>(mean), work);
    hipLaunchKernelGGL(colstats_finish_kernel, dim3(1), dim3(kMlpIn), 0, s, static_cast<const double*>(work), blocks,
                       rows, 1, mean, shift, scale);
    return hipGetLastError();
}

hipError_t gather_shuffled(const float* X, const float* y, int64_t rows, uint64_t seed, uint32_t epoch, int64_t a0,
                           int64_t count, float* xs, float* ys, hipStream_t s) {
    const ShufflePerm p = make_perm(rows, seed, epoch);
    const int64_t threads = count * 4;
    hipLaunchKernelGGL(gather_shuffled_kernel, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0, s, X,
                       y, p, a0, count, xs, ys);
    return hipGetLastError();
}

hipError_t shuffle_indices(int64_t n, uint64_t seed, uint32_t epoch, int64_t* out, hipStream_t s) {
    const ShufflePerm p = make_perm(n, seed, epoch);
    hipLaunchKernelGGL(shuffle_index_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, p, out);
    return hipGetLastError();
}

hipError_t mlp_refresh_bf16(const MlpDevice& d, hipStream_t s) {
    hipLaunchKernelGGL(weights_bf16_kernel, dim3((kMlpW1 + kMlpW2 + 255) / 256), dim3(256), 0, s, d.params, d.w1b,
                       d.w2b, d.w2c, d.w1t, d.w2p);
    return hipGetLastError();
}

}  // namespace geonet
