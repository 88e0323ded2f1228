// Forward evaluation of log psi for the 1D minGRU chain (Sec. II.C) and the
// stacked 2D snake minGRU (Sec. II.F-G), on gfx950.
//
// One workgroup = 4 waves; each wave owns NTC tiles of 16 columns, a column
// being one (sequence, site-in-row) pair.  Sequences are packed back to back
// along the workgroup's columns (a sequence row may straddle tiles and waves).
// Rows are processed one after the other (the vertical input h_V makes rows
// sequential, Sec. II.F); inside a row, for every layer:
//   1. projections  z_pre = W_z u + b_z,  htilde = W_h [u, h_V] + b_h
//      on MFMA (layer 0: the u-part is a gather from 9-entry tables, because
//      u^(0) is two one-hot spins or zeros);
//   2. gates a = z, b = (1 - z) htilde, and the affine recurrence
//      h_t = a_t h_{t-1} + b_t along the row as a chunked parallel scan:
//      Hillis-Steele over the 16 lanes of a DPP row, then a carry chain across
//      the wave's tiles, then (if a row straddles waves) across waves through LDS.
//      A row start has a = 0, which is how h_H = 0 outside the lattice enters
//      and how packed sequences stay independent (segmented scan);
//   3. h is stored as the row frontier (LDS when it fits, else a global
//      workspace; read back as the MFMA operand h_V by the next row) and
//      x = GELU(C h + D u + s) is formed on MFMA;
//   4. after the last layer, the head gives log p of the site's own spin,
//      accumulated per column with compensated (Neumaier) summation.
//
// Precision.  FP32: v_mfma_f32_16x16x4_f32.  BF16: every operand v of a dense
// projection (weights and activations alike) is carried as two bfloat16 parts,
// hi = bf16(v) and lo = bf16(v - hi), so that hi + lo holds v to about 16
// significant bits, and a product W x is formed on v_mfma_f32_16x16x32_bf16 as
// W_hi x_hi + W_lo x_hi + W_hi x_lo with FP32 accumulation (the dropped
// W_lo x_lo term is ~2^-16 of the product).  A single bfloat16 rounding of the
// operands perturbs this randomly initialised recurrence too much for the
// local energy (per-configuration ratio errors of 0.1-1 at 20x20 and above);
// the split keeps it at FP32-like accuracy for a third of the BF16 matrix rate,
// still five times the FP32 matrix rate.
#include "psr_internal.h"
#include "gelu_fit.h"

#include <type_traits>

namespace psr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int P> struct MF;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

template <> struct MF<kBF16> {
    typedef u32x8 Frag;            // dwords 0-3: 8 bfloat16 high parts; dwords 4-7: their low parts
    static constexpr int K = 32;
    static constexpr int ELT = 4;  // bytes per value (hi and lo) in the row frontier
    // c + a b with a = a_hi + a_lo, b = b_hi + b_lo:  a_hi b_hi + a_lo b_hi + a_hi b_lo
    // (The halves are taken by shufflevector: hipcc's __builtin_bit_cast of a `.hi`
    // swizzle reads the vector's first half.)
    __device__ static inline f32x4 mma(Frag a, Frag b, f32x4 c) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, __builtin_shufflevector(a, a, 0, 1, 2, 3));
        const bf16x8 al = __builtin_bit_cast(bf16x8, __builtin_shufflevector(a, a, 4, 5, 6, 7));
        const bf16x8 bh = __builtin_bit_cast(bf16x8, __builtin_shufflevector(b, b, 0, 1, 2, 3));
        const bf16x8 bl = __builtin_bit_cast(bf16x8, __builtin_shufflevector(b, b, 4, 5, 6, 7));
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    }
};
template <> struct MF<kFP32> {
    typedef float Frag;
    static constexpr int K = 4;
    static constexpr int ELT = 4;
    __device__ static inline f32x4 mma(Frag a, Frag b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// ---------------------------------------------------------------------------
// Parameter preparation: fragment-order weights and slot-order tables
// ---------------------------------------------------------------------------

__device__ __host__ inline int unit_pos(int u, int d) {
    // position of unit u in a slot-ordered vector: [g][s], unit = slot_unit(s, g)
    return ((u >> 2) & 3) * (d >> 2) + 4 * (u >> 4) + (u & 3);
}

// bfloat16 high part of v (round to nearest even) and the float it stands for
__device__ inline __bf16 bf16_hi(float v) { return (__bf16)v; }

// BF16 weight fragments, split: for output tile mt and K block kb of 32, the
// 64 lanes' 8 high parts (1 KB), then the 64 lanes' 8 low parts (1 KB).
__global__ void prep_frag_bf16(const float* __restrict__ theta, MatSrc src, int d, __bf16* __restrict__ out) {
    const int64_t n = (int64_t)d * d;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int j = (int)(e & 7);
    const int lane = (int)((e >> 3) & 63);
    const int64_t f = e >> 9;             // fragment index = mt * (d/32) + kb
    const int nkb = d / 32;
    const int kb = (int)(f % nkb), mt = (int)(f / nkb);
    const int r = 16 * mt + (lane & 15), g = lane >> 4;
    const int k = slot_unit(8 * kb + j, g);
    const float v = theta[src.base + (int64_t)r * src.ld + src.coff + k];
    const __bf16 hi = bf16_hi(v);
    const __bf16 lo = (__bf16)(v - (float)hi);
    const int64_t o = ((f * 2) * 64 + lane) * 8 + j;
    out[o] = hi;
    out[o + 512] = lo;
}

__global__ void prep_frag_f32(const float* __restrict__ theta, MatSrc src, int d, float* __restrict__ out) {
    const int64_t n = (int64_t)d * d;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int ee = (int)(e & 3);
    const int lane = (int)((e >> 2) & 63);
    const int64_t f = e >> 8;             // mt * (d/16) + kq
    const int nkq = d / 16;
    const int kq = (int)(f % nkq), mt = (int)(f / nkq);
    const int r = 16 * mt + (lane & 15), g = lane >> 4;
    const int k = slot_unit(4 * kq + ee, g);
    out[e] = theta[src.base + (int64_t)r * src.ld + src.coff + k];
}

// Layer-0 gathers.  state = 3*sH + sV with s = spin value or 2 (outside).
// snake: u^(0) = [onehot(sH), onehot(sV)];  chain: u^(0) = onehot(sH).
struct Tab0Src {
    int chain, d;
    int64_t wz, bz, wh, bh, dd;   // theta offsets of W_z^(0), b_z^(0), W_h^(0), b_h^(0), D^(0) (dd < 0: none)
    int ldz, ldh;                 // row strides of W_z^(0) and W_h^(0)
};

__global__ void prep_tab0(const float* __restrict__ theta, Tab0Src s, float* __restrict__ tz, float* __restrict__ th,
                          float* __restrict__ td) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 9 * s.d) return;
    const int st = e / s.d, u = e % s.d;
    const int sH = st / 3, sV = st % 3;
    float z = theta[s.bz + u], h = theta[s.bh + u], dv = 0.0f;
    if (sH < 2) {
        z += theta[s.wz + (int64_t)u * s.ldz + sH];
        h += theta[s.wh + (int64_t)u * s.ldh + sH];
        if (s.dd >= 0) dv += theta[s.dd + (int64_t)u * 4 + sH];
    }
    if (!s.chain && sV < 2) {
        z += theta[s.wz + (int64_t)u * s.ldz + 2 + sV];
        h += theta[s.wh + (int64_t)u * s.ldh + 2 + sV];
        if (s.dd >= 0) dv += theta[s.dd + (int64_t)u * 4 + 2 + sV];
    }
    const int p = st * s.d + unit_pos(u, s.d);
    tz[p] = z;
    th[p] = h;
    td[p] = dv;
}

// Head of the two-class log-softmax: w = W_o[0] - W_o[1] (slot order), b = b_o[0] - b_o[1].
__global__ void prep_head(const float* __restrict__ theta, int64_t src_w, int64_t src_b, int d, float* __restrict__ w,
                          float* __restrict__ b) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= d) return;
    w[unit_pos(u, d)] = theta[src_w + u] - theta[src_w + d + u];
    if (u == 0) b[0] = theta[src_b] - theta[src_b + 1];
}

__global__ void prep_vec(const float* __restrict__ theta, int64_t src, int d, int rows, float* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * d) return;
    const int r = e / d, u = e % d;
    out[r * d + unit_pos(u, d)] = theta[src + e];
}

int launch_prepare(const Geom& g, const Prepared& pl, const float* theta, uint8_t* frag, float* tab, hipStream_t st) {
    const int d = g.d;
    int64_t off[64];
    int32_t nt = 0;
    param_offsets(g, off, &nt);
    const int T = 256;
    // fragments
    for (int l = 0; l < g.nl; ++l) {
        for (int m = 0; m < 5; ++m) {
            if (!pl.frag_present[l][m]) continue;
            const int64_t fo = pl.frag[l][m];
            // tensor order per layer: W_z, b_z, W_h, b_h, C, D
            const int64_t wz = off[6 * l + 0], wh = off[6 * l + 2], cc = off[6 * l + 4], dd = off[6 * l + 5];
            const int du = (l == 0) ? 4 : d;
            MatSrc s;
            switch (m) {
                case 0: s = MatSrc{wz, du, 0}; break;
                case 1: s = MatSrc{wh, du + d, 0}; break;
                case 2: s = MatSrc{wh, du + d, du}; break;
                case 3: s = MatSrc{dd, du, 0}; break;
                default: s = MatSrc{cc, d, 0}; break;
            }
            const int64_t n = (int64_t)d * d;
            const int blocks = (int)((n + T - 1) / T);
            if (g.prec == kBF16)
                prep_frag_bf16<<<blocks, T, 0, st>>>(theta, s, d, reinterpret_cast<__bf16*>(frag + fo));
            else
                prep_frag_f32<<<blocks, T, 0, st>>>(theta, s, d, reinterpret_cast<float*>(frag + fo));
        }
    }
    // layer-0 tables
    Tab0Src s0;
    s0.chain = g.chain;
    s0.d = d;
    s0.wz = off[0];
    s0.bz = off[1];
    s0.wh = off[2];
    s0.bh = off[3];
    if (g.chain) {
        s0.dd = -1;
        s0.ldz = 2;
        s0.ldh = 2;
    } else {
        s0.dd = off[5];
        s0.ldz = 4;
        s0.ldh = 4 + d;
    }
    prep_tab0<<<(9 * d + T - 1) / T, T, 0, st>>>(theta, s0, tab + pl.t0z, tab + pl.t0h, tab + pl.t0d);
    for (int l = 1; l < g.nl; ++l) {
        prep_vec<<<(d + T - 1) / T, T, 0, st>>>(theta, off[6 * l + 1], d, 1, tab + pl.bias_z[l]);
        prep_vec<<<(d + T - 1) / T, T, 0, st>>>(theta, off[6 * l + 3], d, 1, tab + pl.bias_h[l]);
    }
    const int ih = g.chain ? 4 : 6 * g.nl;   // index of W_o in the tensor list
    prep_head<<<(d + T - 1) / T, T, 0, st>>>(theta, off[ih], off[ih + 1], d, tab + pl.head_w, tab + pl.head_b);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Lane value from `row_shr:n` within the 16-lane DPP row; lanes without a
// source read 0 (bound_ctrl), so the move folds into the consuming VALU op.
template <int CTRL>
__device__ inline float dpp0(float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, src), CTRL, 0xf, 0xf, true));
}

// Lane value from `row_shr:n`; lanes without a source read 1.
template <int CTRL>
__device__ inline float dpp1(float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, 1.0f),
                                                                 __builtin_bit_cast(int, src), CTRL, 0xf, 0xf, false));
}

// Inclusive scan of affine maps h -> A h + B over the 16 lanes of each DPP row
// (Hillis-Steele, shifts 1, 2, 4, 8) for the four slots of a lane at once:
//   (A, B) after (A', B')  =  (A A', A B' + B).
// Each step reads the neighbour's registers as the DPP source operand of the
// VALU op itself -- B += B' A (v_fmac_f32_dpp), then A *= A' (v_mul_f32_dpp) --
// so it costs two instructions per map.  Without bound_ctrl a lane whose
// source lies outside the row is not written, i.e. it composes with the
// identity map.  FULL_A = false leaves A after the last step un-updated, for
// callers that read only the inclusive B.  Hazards: a DPP read of a VGPR needs
// two wait states after the VALU write; the leading s_nop covers values written
// just before the block, inside it every DPP read is at least four instructions
// after the write, and the trailing s_nop covers DPP reads of A or B right
// after the block.
template <bool FULL_A>
__device__ inline void row_scan4(float (&A)[4], float (&B)[4]) {
#define PSR_SCAN_B(S)                                                      \
    "v_fmac_f32_dpp %0, %0, %4 row_shr:" S " row_mask:0xf bank_mask:0xf\n" \
    "v_fmac_f32_dpp %1, %1, %5 row_shr:" S " row_mask:0xf bank_mask:0xf\n" \
    "v_fmac_f32_dpp %2, %2, %6 row_shr:" S " row_mask:0xf bank_mask:0xf\n" \
    "v_fmac_f32_dpp %3, %3, %7 row_shr:" S " row_mask:0xf bank_mask:0xf\n"
#define PSR_SCAN_A(S)                                                     \
    "v_mul_f32_dpp %4, %4, %4 row_shr:" S " row_mask:0xf bank_mask:0xf\n" \
    "v_mul_f32_dpp %5, %5, %5 row_shr:" S " row_mask:0xf bank_mask:0xf\n" \
    "v_mul_f32_dpp %6, %6, %6 row_shr:" S " row_mask:0xf bank_mask:0xf\n" \
    "v_mul_f32_dpp %7, %7, %7 row_shr:" S " row_mask:0xf bank_mask:0xf\n"
    if constexpr (FULL_A)
        asm("s_nop 1\n" PSR_SCAN_B("1") PSR_SCAN_A("1") PSR_SCAN_B("2") PSR_SCAN_A("2") PSR_SCAN_B("4") PSR_SCAN_A("4")
            PSR_SCAN_B("8") PSR_SCAN_A("8") "s_nop 1"
            : "+v"(B[0]), "+v"(B[1]), "+v"(B[2]), "+v"(B[3]), "+v"(A[0]), "+v"(A[1]), "+v"(A[2]), "+v"(A[3]));
    else
        asm("s_nop 1\n" PSR_SCAN_B("1") PSR_SCAN_A("1") PSR_SCAN_B("2") PSR_SCAN_A("2") PSR_SCAN_B("4") PSR_SCAN_A("4")
            PSR_SCAN_B("8") "s_nop 1"
            : "+v"(B[0]), "+v"(B[1]), "+v"(B[2]), "+v"(B[3]), "+v"(A[0]), "+v"(A[1]), "+v"(A[2]), "+v"(A[3]));
#undef PSR_SCAN_A
#undef PSR_SCAN_B
}

// h = b + a * (B of lane - 1 in the DPP row), with the neighbour's register read
// as the DPP source of the fmac; lane 0 of a row has no source and keeps b.
// The DPP read of B follows its last write (in row_scan4) by at least the
// trailing s_nop there.
__device__ inline float carry_apply(float b, float a, float B) {
    asm("v_fmac_f32_dpp %0, %1, %2 row_shr:1 row_mask:0xf bank_mask:0xf" : "+v"(b) : "v"(B), "v"(a));
    return b;
}

// GELU(x) = x Phi(x) = max(x, 0) - |x| p(x) with the Gaussian tail
// p(x) = erfc(|x|/sqrt 2)/2 ~ t Ph(t) 2^(-C x^2), t = 1/(1 + S|x|)
// (degree-5 coefficients fitted by gen_gelu_fit.py, accurate to float32).
__device__ inline float gelu_tail(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(ax, kGeluS, 1.0f));
    float q = kGeluP[0];
#pragma unroll
    for (int k = 1; k <= 5; ++k) q = fmaf(q, t, kGeluP[k]);
    const float p = (t * q) * __builtin_amdgcn_exp2f((x * x) * -kGeluC);
    // max(x, 0) on the bit pattern: a negative float is a negative int32
    const float xp = __builtin_bit_cast(float, max(__builtin_bit_cast(int, x), 0));
    return fmaf(-ax, p, xp);
}

__device__ inline void neumaier(float& s, float& c, float v) {
    const float t = s + v;
    c += (fabsf(s) >= fabsf(v)) ? ((s - t) + v) : ((v - t) + s);
    s = t;
}

// A operand (weights) of one 16-row output tile, per lane: BF16 one K block of
// 32 per piece (8 high and 8 low parts), FP32 four K steps of 4 per piece.
template <int P, int D>
struct AOp {
    static constexpr int N = (P == kBF16) ? D / 32 : D / 16;
    typedef typename std::conditional<P == kBF16, u32x8, f32x4>::type T;
};

// The weight fragments come through buffer loads: the matrix base and the tile
// offset stay scalar and the lane offset is one constant vector register, which
// frees the registers that per-tile 64-bit addresses would hold (such kernels
// spilled without it); the descriptor bounds the matrix (an out-of-range lane
// would read zeros).  A tile is D * 64 bytes in both precisions.
template <int P, int D, class W>
__device__ inline void load_a(W& w, const uint8_t* __restrict__ mat, int mt, int lane) {
    constexpr int TILE = D * 64;
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(mat), 0, TILE * (D / 16), 0x00020000);
#pragma unroll
    for (int k = 0; k < AOp<P, D>::N; ++k) {
        if constexpr (P == kBF16) {
            const u32x4 hi = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16 + k * 2048, mt * TILE, 0));
            const u32x4 lo =
                __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16 + k * 2048 + 1024, mt * TILE, 0));
            w[k] = __builtin_shufflevector(hi, lo, 0, 1, 2, 3, 4, 5, 6, 7);
        } else {
            w[k] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16 + k * 1024, mt * TILE, 0));
        }
    }
}

// acc[c] += W(tile) * b[c] for the NTC column tiles
template <int P, int D, int NTC, class W, class B>
__device__ inline void mma_a(f32x4 (&acc)[NTC], const W& w, const B& b) {
    if constexpr (P == kBF16) {
#pragma unroll
        for (int kb = 0; kb < D / 32; ++kb)
#pragma unroll
            for (int c = 0; c < NTC; ++c) acc[c] = MF<P>::mma(w[kb], b[c][kb], acc[c]);
    } else {
#pragma unroll
        for (int kq = 0; kq < D / 16; ++kq)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int c = 0; c < NTC; ++c) acc[c] = MF<P>::mma(w[kq][e], b[c][4 * kq + e], acc[c]);
    }
}

constexpr int kWaves = 4;
// LDS for a workgroup's BF16 row frontier (and one zero row)
constexpr int kLdsFrontier = 112 * 1024;
constexpr float kNegLog2e = -1.4426950408889634f;
constexpr float kLn2 = 0.69314718055994531f;

// Gates and the chunked scan of one output tile (4 units per lane, NTC positions):
//   z = sigmoid(az), a = z (0 at a row start), b = (1 - z) htilde,
//   h = a h_prev + b along the row.
template <int NTC, bool CROSS, bool ALIGNED>
__device__ inline void scan_tile(const f32x4 (&az)[NTC], const f32x4 (&ah)[NTC], const float (&keep)[NTC],
                                 float (&h)[NTC][4], float (&xw)[2][kWaves][16][2], int mt, int wave, int g, int r16) {
    float A[NTC][4], Bv[NTC][4];   // maps of the positions, composed inside the chunk
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int c = 0; c < NTC; ++c) {
            const float z = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(az[c][i] * kNegLog2e));
            // ALIGNED: every row starts at position 0 of lane 0 of a DPP row, where the
            // carry is zero and the multiplier is never applied, so a needs no mask
            const float aa = ALIGNED ? z : z * keep[c];
            const float bb = fmaf(-z, ah[c][i], ah[c][i]);   // (1 - z) htilde
            if (c == 0) {
                A[c][i] = aa;
                Bv[c][i] = bb;
            } else {
                Bv[c][i] = fmaf(aa, Bv[c - 1][i], bb);
                A[c][i] = aa * A[c - 1][i];
            }
        }
    }
    // chunk aggregates -> inclusive over chunks 0..lane of the DPP row (in place: the
    // last column's map is not needed again, because the inclusive value is its h)
    float (&sA)[4] = A[NTC - 1];
    float (&sB)[4] = Bv[NTC - 1];
    row_scan4<CROSS>(sA, sB);
    if constexpr (!CROSS) {
        // no carry enters a wave: lane 0 of a DPP row starts a sequence row
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int c = 0; c + 1 < NTC; ++c) h[c][i] = carry_apply(Bv[c][i], A[c][i], sB[i]);
            h[NTC - 1][i] = sB[i];
        }
    } else {
        float X[4];   // carry entering this lane's chunk from the lanes before it
#pragma unroll
        for (int i = 0; i < 4; ++i) X[i] = dpp0<0x111>(sB[i]);
        const int buf = mt & 1;
        if (r16 == 15) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                xw[buf][wave][4 * g + i][0] = sA[i];
                xw[buf][wave][4 * g + i][1] = sB[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float Xa = dpp1<0x111>(sA[i]);   // product of the multipliers before this chunk
            float W = 0.0f;                        // carry entering this wave
            for (int w = 0; w < wave; ++w) W = fmaf(xw[buf][w][4 * g + i][0], W, xw[buf][w][4 * g + i][1]);
            const float Xt = fmaf(Xa, W, X[i]);
#pragma unroll
            for (int c = 0; c + 1 < NTC; ++c) h[c][i] = fmaf(A[c][i], Xt, Bv[c][i]);
            h[NTC - 1][i] = fmaf(sA[i], W, sB[i]);
        }
    }
}

// slots s, s+1 (s even) of a lane's operand array.  BF16 packs the pair's high
// parts into one dword of the fragment's first half and their low parts
// (v - hi, rounded again) into the same dword of the second half.
template <int P, int D>
__device__ inline void set_pair(typename MF<P>::Frag (&f)[D / MF<P>::K], int s, float x0, float x1) {
    if constexpr (P == kBF16) {
        bf16x2 v;
        v[0] = bf16_hi(x0);
        v[1] = bf16_hi(x1);
        const uint32_t hu = __builtin_bit_cast(uint32_t, v);
        bf16x2 w;
        w[0] = (__bf16)(x0 - __builtin_bit_cast(float, hu << 16));
        w[1] = (__bf16)(x1 - __builtin_bit_cast(float, hu & 0xFFFF0000u));
        const int q = (s & 7) >> 1;
        f[s >> 3][q] = hu;
        f[s >> 3][4 + q] = __builtin_bit_cast(uint32_t, w);
    } else {
        f[s] = x0;
        f[s + 1] = x1;
    }
}

// Keep the values of output tile mt (slots 4mt..4mt+3 of an operand array) at
// this point of the program: an empty volatile asm that reads them stops the
// compiler from sinking their computation into a later pipeline stage.
template <int P, int D>
__device__ inline void pin_tile(typename MF<P>::Frag (&f)[D / MF<P>::K], int mt) {
    if constexpr (P == kBF16) {
        const int q = 2 * (mt & 1);
        asm volatile("" ::"v"(f[mt >> 1][q]), "v"(f[mt >> 1][q + 1]), "v"(f[mt >> 1][4 + q]), "v"(f[mt >> 1][5 + q]));
    } else {
        asm volatile("" ::"v"(f[4 * mt]), "v"(f[4 * mt + 1]), "v"(f[4 * mt + 2]), "v"(f[4 * mt + 3]));
    }
}
__device__ inline void pin1(float& x) { asm volatile("" : "+v"(x)); }

// Row frontier (h of the previous row, in the projections' operand form):
// per sequence-local index qi, layer l, physical column i, lane group g, the
// lane's d/4 slots are contiguous (BF16: per fragment, the 16 bytes of high
// parts, then the 16 bytes of low parts), so a lane moves whole 16-byte pieces.
template <int ELT, int D>
__device__ inline uint8_t* col_ptr(void* base, int64_t qi, int l, int nslot, int lx, int i, int g) {
    return reinterpret_cast<uint8_t*>(base) + ((((size_t)qi * nslot + l) * lx + i) * D + (size_t)g * (D / 4)) * ELT;
}

// 16-byte pieces of a lane's operand array (BF16: half a fragment, high parts
// first; FP32: four slots)
template <int P, int D>
__device__ inline void frag_set16(typename MF<P>::Frag (&f)[D / MF<P>::K], int k, f32x4 v) {
    if constexpr (P == kBF16) {
        const u32x4 u = __builtin_bit_cast(u32x4, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) f[k >> 1][4 * (k & 1) + e] = u[e];
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) f[4 * k + e] = v[e];
    }
}
template <int P, int D>
__device__ inline f32x4 frag_get16(const typename MF<P>::Frag (&f)[D / MF<P>::K], int k) {
    if constexpr (P == kBF16) {
        const int o = 4 * (k & 1);
        return __builtin_bit_cast(f32x4, u32x4{f[k >> 1][o], f[k >> 1][o + 1], f[k >> 1][o + 2], f[k >> 1][o + 3]});
    } else {
        return f32x4{f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]};
    }
}

// 16 bytes at a uniform float base plus a per-lane byte offset that fits 32 bits
// (lets the compiler address with a scalar base and a 32-bit vector offset)
__device__ inline f32x4 ld16(const float* base, uint32_t byte_off) {
    return *reinterpret_cast<const f32x4*>(reinterpret_cast<const uint8_t*>(base) + byte_off);
}

// ---------------------------------------------------------------------------
// The fused row-recurrence forward kernel
// ---------------------------------------------------------------------------
//
// Column layout.  A wave owns 16 chunks (the 16 lanes of a DPP row; the four
// DPP rows hold four unit groups of the same columns) of NTC consecutive
// columns each (its NTC MFMA tiles).  Chunk k of the workgroup = wave*16 + lane%16
// covers flat columns k*NTC .. k*NTC+NTC-1, and sequences occupy lx consecutive
// flat columns each (a column = one site of the current row of one sequence,
// in snake order).  The in-row scan is therefore a chunked parallel scan:
//   (1) inside a lane, the NTC positions of its chunk are composed in order;
//   (2) the chunk aggregates are scanned across the 16 lanes with DPP;
//   (3) if a row continues in the next wave, wave aggregates go through LDS;
//   (4) each position applies the carry entering its chunk: h = A X + B.
// A position that starts a row has a = 0 (h_H = 0 outside the lattice), which
// also keeps sequences that share a chunk or a DPP row independent.


template <int P, int D, int NTC, bool CROSS, bool CHAIN, bool ALIGNED, bool LDSF>
__global__ void __launch_bounds__(kWaves * 64) fwd_kernel(const FwdArgs a) {
    using F = MF<P>;
    typedef typename F::Frag Frag;
    typedef typename AOp<P, D>::T AT;
    constexpr int NA = AOp<P, D>::N;
    constexpr int NK = D / F::K;   // B fragments per tile
    constexpr int NS = D / 4;      // slots per lane
    constexpr int NMT = D / 16;    // 16-unit output tiles
    constexpr int COLS = kWaves * NTC * 16;

    __shared__ float xw[2][kWaves][16][2];
    __shared__ float red[COLS][2];
    // LDSF: the row frontier lives in LDS, [seq][layer][column] rows of PITCH bytes
    // (padded by 16 B so that the 16 columns of a DPP row hit distinct banks),
    // after one zero row that stands in for the residual of layers 0 and 1
    constexpr int PITCH = D * F::ELT + 16;
    constexpr int ZOFF = D * F::ELT;
    __shared__ __attribute__((aligned(16))) uint8_t fl[LDSF ? kLdsFrontier : 16];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const Geom G = a.g;
    const int lx = G.lx, ly = G.ly, nl = G.nl;
    const int N = lx * ly;
    const int seqs = a.sh.seqs;

    int64_t q_end = a.q_begin + a.q_count;
    if (a.q_total) q_end = min(q_end, *a.q_total);
    const int64_t q0 = a.q_begin + (int64_t)blockIdx.x * seqs;
    if (q0 >= q_end) return;   // uniform across the workgroup
    if constexpr (LDSF) {
        // the zero row, and the frontier itself: row 0 reads it as h_V before it is written
        const int nw = (ZOFF + a.sh.seqs * G.nl * G.lx * PITCH) / 16;
        for (int e = threadIdx.x; e < nw; e += blockDim.x) reinterpret_cast<uint4*>(fl)[e] = uint4{0u, 0u, 0u, 0u};
    }

    // per-column constants (column = chunk position c of this lane), kept in 32-bit fields
    int t[NTC], kq[NTC], srow[NTC], flip[NTC];
    bool valid[NTC];
#pragma unroll
    for (int c = 0; c < NTC; ++c) {
        const int col = (wave * 16 + r16) * NTC + c;
        const int k = col / lx;
        kq[c] = k;
        t[c] = col - k * lx;
        const int64_t q = q0 + k;
        valid[c] = (k < seqs) && (q < q_end);
        srow[c] = valid[c] ? (int)q : (int)q0;   // packed row of the spins
        flip[c] = -1;                             // sites a | b << 16 flipped (0xFFFF: none)
        if (a.desc && valid[c]) {
            const uint32_t s0 = a.desc[2 * q], s1 = a.desc[2 * q + 1];
            srow[c] = (int)s0;
            const uint32_t fa = s1 & 0xFFFF, fb = s1 >> 16;
            flip[c] = (int)(fa | ((fb == fa ? 0xFFFFu : fb) << 16));
        }
    }
    auto spin = [&](int c, int site) -> int {
        const uint32_t* w = a.spins + (size_t)srow[c] * a.words_per_seq;
        const int v = (int)((w[site >> 5] >> (site & 31)) & 1u);
        const int fa = flip[c] & 0xFFFF, fb = (int)((uint32_t)flip[c] >> 16);
        return v ^ (int)(site == fa) ^ (int)(site == fb);
    };
    auto seq_local = [&](int c) -> int64_t { return valid[c] ? (q0 + kq[c] - a.q_begin) : 0; };
    float keep[NTC];   // 0 at a row start: h_H is zero outside the lattice
#pragma unroll
    for (int c = 0; c < NTC; ++c) keep[c] = (t[c] == 0) ? 0.0f : 1.0f;

    const float* tab = a.tab;
    const uint32_t goff = (uint32_t)(g * NS) * 4u;   // byte offset of this lane's unit group in a d-vector
    float ls[NTC], lc[NTC];
#pragma unroll
    for (int c = 0; c < NTC; ++c) ls[c] = lc[c] = 0.0f;

    Frag u[NTC][NK];    // B operand: input of the current layer (layers >= 1)
    // frontier bytes per layer
    const size_t fl_stride = LDSF ? (size_t)lx * PITCH : (size_t)lx * D * F::ELT;

    for (int j = 0; j < ly; ++j) {
        __syncthreads();   // frontier of row j-1 is complete
        int iph[NTC], st[NTC], own[NTC];
#pragma unroll
        for (int c = 0; c < NTC; ++c) {
            const int i = (j & 1) ? (lx - 1 - t[c]) : t[c];
            iph[c] = i;
            int sH = 2, sV = 2;
            const int ih = (j & 1) ? i + 1 : i - 1;
            own[c] = 0;
            if (valid[c]) {
                if (ih >= 0 && ih < lx) sH = spin(c, j * lx + ih);
                if (j > 0) sV = spin(c, (j - 1) * lx + i);
                own[c] = spin(c, j * lx + i);
            }
            st[c] = 3 * sH + sV;
        }
        const bool vert = (!CHAIN) && (j > 0);
        // this row's frontier columns (layer l adds l * fl_stride bytes)
        uint8_t* frow[NTC];
#pragma unroll
        for (int c = 0; c < NTC; ++c) {
            if constexpr (LDSF)
                frow[c] = fl + ZOFF + ((size_t)((valid[c] ? kq[c] : 0) * nl) * lx + iph[c]) * PITCH + g * (D / 4) * F::ELT;
            else
                frow[c] = col_ptr<F::ELT, D>(a.frontier, seq_local(c), 0, nl, lx, iph[c], g);
        }
        // logit difference l_0 - l_1 of the head (all a two-class log-softmax needs),
        // accumulated over the last layer's output tiles
        float l0[NTC];
#pragma unroll
        for (int c = 0; c < NTC; ++c) l0[c] = 0.0f;

        // h_V operand of the layer being computed: the previous row's frontier (0 on row 0).
        // Layer 0's is loaded here; layer l+1's is loaded while layer l forms its output.
        Frag hv[NTC][NK];
        auto load_hv = [&](int l) {
#pragma unroll
            for (int c = 0; c < NTC; ++c) {
                const f32x4* src = reinterpret_cast<const f32x4*>(frow[c] + l * fl_stride);
#pragma unroll
                for (int k = 0; k < NK * (int)sizeof(Frag) / 16; ++k) frag_set16<P, D>(hv[c], k, src[k]);
            }
        };
        if constexpr (!CHAIN) {
            if (vert) {
                load_hv(0);
            } else {
#pragma unroll
                for (int c = 0; c < NTC; ++c)
#pragma unroll
                    for (int k = 0; k < NK * (int)sizeof(Frag) / 16; ++k)
                        frag_set16<P, D>(hv[c], k, f32x4{0.f, 0.f, 0.f, 0.f});
            }
        }

        // GEMM1 operand slots (fragments and seeds of two tiles), at row scope so that a
        // layer can load the next layer's first two tiles during its last output tiles
        // layers >= 1 run the pipelined path when two slots of a tile's fragments are few registers
        constexpr bool PFK = 3 * NA * (int)sizeof(AT) <= 12 * 16;
        AT w1r[2][3][NA];
        f32x4 s1zr[2][NTC], s1hr[2][NTC];
        bool pre1 = false;   // the next layer's tiles 0 and 1 are in w1r / s1zr / s1hr

        // One layer.  FIRST: u is the one-hot layer-0 input (tables);  LAST: x feeds the head.
        // Inside a layer there is no branch between the output tiles; the operands of
        // the next tile (weight fragments, accumulator seeds) are loaded while the
        // current one is computed.
        auto layer = [&](auto first_c, auto last_c, int l) {
            constexpr bool FIRST = decltype(first_c)::value;
            constexpr bool LAST = decltype(last_c)::value;
            constexpr int NM1 = CHAIN ? 0 : (FIRST ? 1 : 3);       // GEMM1 matrices: (W_hV) or (W_z, W_hu, W_hV)
            constexpr int NM2 = CHAIN ? 1 : (FIRST ? 1 : 2);       // GEMM2 matrices: (C) or (D, C)
            // prefetch one tile ahead when the fragments of a tile are few registers
            // (decided per model, not per layer: a pipelined first layer with large tiles
            // would hold two slots of fragments for both GEMMs at once)
            constexpr bool PF = PFK;
            // layers >= 1 without the pipelined path read h_V from the LDS frontier per tile
            constexpr bool HVL = LDSF && !PF && !FIRST;
            const uint8_t* m1[3];
            const uint8_t* m2[2];
            if constexpr (FIRST) {
                m1[0] = m1[1] = m1[2] = a.frag + a.pl.frag[l][2];
                m2[0] = m2[1] = a.frag + a.pl.frag[l][4];
            } else {
                m1[0] = a.frag + a.pl.frag[l][0];
                m1[1] = a.frag + a.pl.frag[l][1];
                m1[2] = a.frag + a.pl.frag[l][2];
                m2[0] = a.frag + a.pl.frag[l][3];
                m2[1] = a.frag + a.pl.frag[l][4];
            }

            // source of the residual h^(l-1) (layers >= 2): this row's frontier of layer l-1;
            // layer 1 reads the zero row (LDS frontier) or scales what it reads by 0 (global frontier)
            const uint8_t* rsrc[NTC];
            float rs = 1.0f;
#pragma unroll
            for (int c = 0; c < NTC; ++c) {
                if constexpr (LDSF)
                    rsrc[c] = (l >= 2) ? frow[c] + (l - 1) * fl_stride : fl + g * (D / 4) * F::ELT;
                else
                    rsrc[c] = frow[c] + (l >= 1 ? l - 1 : 0) * fl_stride;
            }
            if constexpr (!LDSF) rs = (l >= 2) ? 1.0f : 0.0f;
            (void)rs;

            // GEMM1 operands of tile mt: fragments and the accumulator seeds
            // (layer 0: table rows of the site's state; else the biases)
            auto seeds1 = [&](int mt, f32x4 (&sz)[NTC], f32x4 (&sh)[NTC]) {
                if constexpr (FIRST) {
#pragma unroll
                    for (int c = 0; c < NTC; ++c) {
                        const int o = st[c] * D + g * NS;
                        sz[c] = ld16(tab + a.pl.t0z + 4 * mt, (uint32_t)o * 4u);
                        sh[c] = ld16(tab + a.pl.t0h + 4 * mt, (uint32_t)o * 4u);
                    }
                } else {
                    const f32x4 bz = ld16(tab + a.pl.bias_z[l] + 4 * mt, goff);
                    const f32x4 bh = ld16(tab + a.pl.bias_h[l] + 4 * mt, goff);
#pragma unroll
                    for (int c = 0; c < NTC; ++c) {
                        sz[c] = bz;
                        sh[c] = bh;
                    }
                }
            };
            auto fetch1 = [&](int mt, AT (&w)[3][NA], f32x4 (&sz)[NTC], f32x4 (&sh)[NTC]) {
#pragma unroll
                for (int m = 0; m < NM1; ++m) load_a<P, D>(w[m], m1[m], mt, lane);
                seeds1(mt, sz, sh);
            };
            // GEMM2 operands of tile mt: fragments, the seed (layer 0: table row of D u;
            // else the residual row, zero for layer 1) and the head rows (last layer)
            auto seeds2 = [&](int mt, f32x4 (&so)[NTC]) {
                if constexpr (!CHAIN) {
                    if constexpr (FIRST) {
#pragma unroll
                        for (int c = 0; c < NTC; ++c)
                            so[c] = ld16(tab + a.pl.t0d + 4 * mt, (uint32_t)(st[c] * D + g * NS) * 4u);
                    } else {
                        // residual h^(l-1) of this row, from the frontier (layers >= 2)
#pragma unroll
                        for (int c = 0; c < NTC; ++c) {
                            if constexpr (P == kBF16) {
                                // slots 4mt..4mt+3: two dwords of high parts and the two
                                // dwords of their low parts, 16 bytes further on
                                const uint8_t* q = rsrc[c] + (mt >> 1) * 32 + (mt & 1) * 8;
                                const uint2 vh = *reinterpret_cast<const uint2*>(q);
                                const uint2 vl = *reinterpret_cast<const uint2*>(q + 16);
                                so[c] = f32x4{__builtin_bit_cast(float, vh.x << 16) + __builtin_bit_cast(float, vl.x << 16),
                                              __builtin_bit_cast(float, vh.x & 0xFFFF0000u) +
                                                  __builtin_bit_cast(float, vl.x & 0xFFFF0000u),
                                              __builtin_bit_cast(float, vh.y << 16) + __builtin_bit_cast(float, vl.y << 16),
                                              __builtin_bit_cast(float, vh.y & 0xFFFF0000u) +
                                                  __builtin_bit_cast(float, vl.y & 0xFFFF0000u)};
                                if constexpr (!LDSF) so[c] = so[c] * rs;   // layer 1 has no residual
                            } else {
                                so[c] = *reinterpret_cast<const f32x4*>(rsrc[c] + 16 * mt) * rs;
                            }
                        }
                    }
                }
            };
            auto fetch2 = [&](int mt, AT (&w)[NM2][NA], f32x4 (&so)[NTC]) {
                if constexpr (!CHAIN) {
#pragma unroll
                    for (int m = 0; m < NM2; ++m) load_a<P, D>(w[m], m2[m], mt, lane);
                    seeds2(mt, so);
                }
            };

            // Two operand slots per phase.  With PF the phases are software-pipelined:
            // iteration mt issues the MFMAs of tile mt+1, loads the operands of tile
            // mt+2 and then runs the VALU epilogue of tile mt, so that the matrix core
            // works while the VALU forms the previous tile's outputs.
            constexpr int NSL = PF ? 2 : 1;   // accumulator slots
            // operand (fragments + seeds) slots: tile mt+NWS loads during tile mt (a third
            // slot measured slower: the extra registers become accumulator-register moves)
            constexpr int NWS = PF ? 2 : 1;
            // Without PF the fragments go through a ring of two single-matrix slots:
            // the next matrix (of this tile, the next tile or the next phase) loads
            // while the current matrix's MFMAs run.  Stage q counts matrices.
            AT wm[PF ? 1 : 2][NA];
            auto& w1 = w1r;
            auto& s1z = s1zr;
            auto& s1h = s1hr;
            AT w2[NWS][NM2][NA];
            f32x4 s2[NWS][NTC];
            f32x4 az[NSL][NTC], ah[NSL][NTC], ao[NSL][NTC];

            auto issue1 = [&](int sl, int ws) {   // accumulator slot, operand slot
#pragma unroll
                for (int c = 0; c < NTC; ++c) {
                    az[sl][c] = s1z[ws][c];
                    ah[sl][c] = s1h[ws][c];
                }
                if constexpr (FIRST) {
                    if constexpr (!CHAIN) mma_a<P, D, NTC>(ah[sl], w1[ws][0], hv);
                } else {
                    mma_a<P, D, NTC>(az[sl], w1[ws][0], u);
                    mma_a<P, D, NTC>(ah[sl], w1[ws][1], u);
                    mma_a<P, D, NTC>(ah[sl], w1[ws][2], hv);
                }
            };
            Frag hb[NTC][NK];
            auto valu1 = [&](int mt, int sl) {
                // ---- gates and the chunked scan along the row
                float h[NTC][4];
                scan_tile<NTC, CROSS, ALIGNED>(az[sl], ah[sl], keep, h, xw, mt, wave, g, r16);
                // ---- outputs of tile mt: GEMM2 operand, residual, chain head
#pragma unroll
                for (int c = 0; c < NTC; ++c) {
                    set_pair<P, D>(hb[c], 4 * mt, h[c][0], h[c][1]);
                    set_pair<P, D>(hb[c], 4 * mt + 2, h[c][2], h[c][3]);
                    pin_tile<P, D>(hb[c], mt);
                    if constexpr (CHAIN) {   // head reads h directly
                        const f32x4 w0 = ld16(tab + a.pl.head_w + 4 * mt, goff);
#pragma unroll
                        for (int i = 0; i < 4; ++i) l0[c] = fmaf(w0[i], h[c][i], l0[c]);
                    }
                }
            };

            if constexpr (PF) {
                if (!pre1) {
#pragma unroll
                    for (int t = 0; t < NWS; ++t) {
                        if (t < NMT)
                            fetch1(t, w1[t], s1z[t], s1h[t]);
                        else if constexpr (!CHAIN)
                            fetch2(t - NMT, w2[t - NMT], s2[t - NMT]);
                    }
                }
                pre1 = false;
                issue1(0, 0);
            } else if constexpr (NM1 > 0) {
                load_a<P, D>(wm[0], m1[0], 0, lane);
            }
#pragma unroll
            for (int mt = 0; mt < NMT; ++mt) {
                if constexpr (PF) {
                    const int cs = mt & 1, ns = cs ^ 1;
                    if (mt + 1 < NMT) issue1(ns, (mt + 1) % NWS);
                    // tile mt+3 reuses the operand slot of tile mt (its MFMAs are issued)
                    const int t = mt + NWS;
                    if (t < NMT)
                        fetch1(t, w1[mt % NWS], s1z[mt % NWS], s1h[mt % NWS]);
                    else if (t - NMT < NWS && t - NMT < NMT) {
                        if constexpr (!CHAIN) fetch2(t - NMT, w2[(t - NMT) % NWS], s2[(t - NMT) % NWS]);
                    }
                    valu1(mt, cs);
                    __builtin_amdgcn_sched_barrier(0);
                } else {
                    seeds1(mt, s1z[0], s1h[0]);
#pragma unroll
                    for (int c = 0; c < NTC; ++c) {
                        az[0][c] = s1z[0][c];
                        ah[0][c] = s1h[0][c];
                    }
#pragma unroll
                    for (int m = 0; m < NM1; ++m) {
                        const int sl = (mt * NM1 + m) & 1;
                        if (m + 1 < NM1)
                            load_a<P, D>(wm[sl ^ 1], m1[m + 1], mt, lane);
                        else if (mt + 1 < NMT)
                            load_a<P, D>(wm[sl ^ 1], m1[0], mt + 1, lane);
                        else if constexpr (!CHAIN)
                            load_a<P, D>(wm[sl ^ 1], m2[0], 0, lane);
                        if constexpr (FIRST)
                            mma_a<P, D, NTC>(ah[0], wm[sl], hv);
                        else if (m == 0)
                            mma_a<P, D, NTC>(az[0], wm[sl], u);
                        else if (m == 1)
                            mma_a<P, D, NTC>(ah[0], wm[sl], u);
                        else if constexpr (HVL) {
                            // h_V straight from the LDS frontier, live only for this product
                            Frag hvt[NTC][NK];
#pragma unroll
                            for (int c = 0; c < NTC; ++c) {
                                const f32x4* src = reinterpret_cast<const f32x4*>(frow[c] + l * fl_stride);
#pragma unroll
                                for (int k = 0; k < NK * (int)sizeof(Frag) / 16; ++k) frag_set16<P, D>(hvt[c], k, src[k]);
                            }
                            mma_a<P, D, NTC>(ah[0], wm[sl], hvt);
                        } else {
                            mma_a<P, D, NTC>(ah[0], wm[sl], hv);
                        }
                    }
                    if constexpr (CHAIN && NM1 == 0) (void)wm;
                    valu1(mt, 0);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if constexpr (CHAIN) return;
            else {
                // h of this row: the next row's h_V and the residual of layer l+2
#pragma unroll
                for (int c = 0; c < NTC; ++c) {
                    if (!valid[c]) continue;
                    f32x4* dst = reinterpret_cast<f32x4*>(frow[c] + l * fl_stride);
#pragma unroll
                    for (int k = 0; k < NK * (int)sizeof(Frag) / 16; ++k) dst[k] = frag_get16<P, D>(hb[c], k);
                }
                // the next layer's h_V, in flight during this layer's output (not needed when
                // the next layer reads it from the LDS frontier tile by tile)
                if constexpr (!LAST && !(LDSF && !PFK)) {
                    if (vert) load_hv(l + 1);
                }

                // ---- x = GELU(C h + D u + s); the last layer feeds the head
                Frag xn[NTC][LAST ? 1 : NK];
                auto issue2 = [&](int sl, int ws) {   // accumulator slot, operand slot
#pragma unroll
                    for (int c = 0; c < NTC; ++c) ao[sl][c] = s2[ws][c];
                    if constexpr (!FIRST) mma_a<P, D, NTC>(ao[sl], w2[ws][0], u);
                    mma_a<P, D, NTC>(ao[sl], w2[ws][NM2 - 1], hb);
                };
                auto valu2 = [&](int mt, int sl) {
                    if constexpr (!LAST) {
#pragma unroll
                        for (int c = 0; c < NTC; ++c) {
                            set_pair<P, D>(xn[c], 4 * mt, gelu_tail(ao[sl][c][0]), gelu_tail(ao[sl][c][1]));
                            set_pair<P, D>(xn[c], 4 * mt + 2, gelu_tail(ao[sl][c][2]), gelu_tail(ao[sl][c][3]));
                            pin_tile<P, D>(xn[c], mt);
                        }
                    } else {
                        const f32x4 hw0 = ld16(tab + a.pl.head_w + 4 * mt, goff);
#pragma unroll
                        for (int c = 0; c < NTC; ++c) {
#pragma unroll
                            for (int i = 0; i < 4; ++i) l0[c] = fmaf(hw0[i], gelu_tail(ao[sl][c][i]), l0[c]);
                            pin1(l0[c]);
                        }
                    }
                };
                if constexpr (PF) issue2(0, 0);
#pragma unroll
                for (int mt = 0; mt < NMT; ++mt) {
                    if constexpr (PF) {
                        const int cs = mt & 1, ns = cs ^ 1;
                        if (mt + 1 < NMT) issue2(ns, (mt + 1) % NWS);
                        if (mt + NWS < NMT) {
                            fetch2(mt + NWS, w2[mt % NWS], s2[mt % NWS]);
                        } else if constexpr (PFK && !LAST) {
                            // the next layer's tiles 0 and 1 (layer l+1 >= 1: W_z, W_hu, W_hV, biases)
                            const int t = mt + NWS - NMT;
                            const uint8_t* mn[3] = {a.frag + a.pl.frag[l + 1][0], a.frag + a.pl.frag[l + 1][1],
                                                    a.frag + a.pl.frag[l + 1][2]};
#pragma unroll
                            for (int m = 0; m < 3; ++m) load_a<P, D>(w1[t][m], mn[m], t, lane);
                            const f32x4 bz = ld16(tab + a.pl.bias_z[l + 1] + 4 * t, goff);
                            const f32x4 bh = ld16(tab + a.pl.bias_h[l + 1] + 4 * t, goff);
#pragma unroll
                            for (int c = 0; c < NTC; ++c) {
                                s1z[t][c] = bz;
                                s1h[t][c] = bh;
                            }
                            pre1 = true;
                        }
                        valu2(mt, cs);
                        __builtin_amdgcn_sched_barrier(0);
                    } else {
                        seeds2(mt, s2[0]);
#pragma unroll
                        for (int c = 0; c < NTC; ++c) ao[0][c] = s2[0][c];
#pragma unroll
                        for (int m = 0; m < NM2; ++m) {
                            const int sl = (NMT * NM1 + mt * NM2 + m) & 1;
                            if (m + 1 < NM2)
                                load_a<P, D>(wm[sl ^ 1], m2[m + 1], mt, lane);
                            else if (mt + 1 < NMT)
                                load_a<P, D>(wm[sl ^ 1], m2[0], mt + 1, lane);
                            if (FIRST || m == 1)
                                mma_a<P, D, NTC>(ao[0], wm[sl], hb);
                            else
                                mma_a<P, D, NTC>(ao[0], wm[sl], u);
                        }
                        valu2(mt, 0);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                if constexpr (!LAST) {
#pragma unroll
                    for (int c = 0; c < NTC; ++c)
#pragma unroll
                        for (int k = 0; k < NK; ++k) u[c][k] = xn[c][k];
                }
            }
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        if (CHAIN || nl == 1) {
            layer(T_{}, T_{}, 0);
        } else if constexpr (!CHAIN) {
            layer(T_{}, F_{}, 0);
            for (int l = 1; l + 1 < nl; ++l) layer(F_{}, F_{}, l);
            layer(F_{}, T_{}, nl - 1);
        }
        // head: logits = W_o x + b_o, log p of the site's own spin; with two classes the
        // log-softmax depends on the logit difference only
        const float bod = tab[a.pl.head_b];
#pragma unroll
        for (int c = 0; c < NTC; ++c) {
            float v = l0[c];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            v += bod;
            // dl = (logit of the other spin) - (logit of the own spin)
            const float dl = own[c] ? v : -v;
            // log p = -softplus(dl) = -(max(dl, 0) + ln(1 + e^-|dl|)), in base 2 on the
            // hardware exp2/log2 (1 + e rounds to 1 only where e < 2^-24)
            const float e = __builtin_amdgcn_exp2f(fabsf(dl) * kNegLog2e);
            const float lp = -(fmaxf(dl, 0.0f) + kLn2 * __builtin_amdgcn_logf(1.0f + e));
            if (valid[c]) {
                neumaier(ls[c], lc[c], lp);
                if (a.logp_site && g == 0) a.logp_site[(size_t)(q0 + kq[c]) * N + j * lx + iph[c]] = lp;
            }
        }
    }

    // per-sequence total over its columns, in column order
    __syncthreads();
    if (g == 0) {
#pragma unroll
        for (int c = 0; c < NTC; ++c) {
            const int col = (wave * 16 + r16) * NTC + c;
            red[col][0] = valid[c] ? ls[c] : 0.0f;
            red[col][1] = valid[c] ? lc[c] : 0.0f;
        }
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k < seqs && q0 + k < q_end) {
        float s = 0.0f, cc = 0.0f;
        for (int t2 = 0; t2 < lx; ++t2) {
            neumaier(s, cc, red[k * lx + t2][0]);
            cc += red[k * lx + t2][1];
        }
        // log psi = (1/2) sum log p; kept as a float pair (hi, lo), scaled exactly
        const float hi = s + cc;
        const float lo = cc - (hi - s);
        a.out_hi[q0 + k] = 0.5f * hi;
        if (a.out_lo) a.out_lo[q0 + k] = 0.5f * lo;
    }
}

// ---------------------------------------------------------------------------
// Launch shape and dispatch
// ---------------------------------------------------------------------------

// Tiles per wave, chosen so that the four register-resident operand sets
// (layer input, h_V, h, next input) fit.  A split BF16 operand takes the
// registers of an FP32 one, so both precisions use the same shapes.  The launch
// (template argument) and the host-side sizing (fwd_shape) both take it from here.
static constexpr int ntc_for(int prec, int d) {
    (void)prec;
    return d <= 32 ? 4 : (d <= 128 ? 2 : 1);
}

FwdShape fwd_shape(const Geom& g) {
    FwdShape s;
    s.ntc = ntc_for(g.prec, g.d);
    s.waves = kWaves;
    s.cols = s.waves * s.ntc * 16;
    s.seqs = s.cols / g.lx;
    const int per_wave = s.ntc * 16;
    s.cross_wave = 0;
    for (int k = 0; k < s.seqs; ++k) {
        const int c0 = k * g.lx, c1 = (k + 1) * g.lx - 1;
        if (c0 / per_wave != c1 / per_wave) s.cross_wave = 1;
    }
    // BF16 frontier rows: d values of 4 bytes (high and low parts) plus 16 bytes of padding
    const int64_t pitch = (int64_t)g.d * 4 + 16;
    s.lds_frontier = (!g.chain && g.prec == kBF16 &&
                      (int64_t)g.d * 4 + (int64_t)s.seqs * g.nl * g.lx * pitch <= kLdsFrontier) ? 1 : 0;
    return s;
}

template <int P, int D, int NTC>
static int launch_t(const FwdArgs& a, hipStream_t st) {
    const int64_t blocks = (a.q_count + a.sh.seqs - 1) / a.sh.seqs;
    if (blocks <= 0) return 0;
    const dim3 grid((unsigned)blocks), block(kWaves * 64);
    if (a.g.chain) {
        if (a.sh.cross_wave)
            fwd_kernel<P, D, NTC, true, true, false, false><<<grid, block, 0, st>>>(a);
        else
            fwd_kernel<P, D, NTC, false, true, false, false><<<grid, block, 0, st>>>(a);
    } else if (a.sh.lds_frontier) {
        if constexpr (P == kBF16) {
            if (a.sh.cross_wave)
                fwd_kernel<P, D, NTC, true, false, false, true><<<grid, block, 0, st>>>(a);
            else if (a.g.lx == 16 * NTC)
                fwd_kernel<P, D, NTC, false, false, true, true><<<grid, block, 0, st>>>(a);
            else
                fwd_kernel<P, D, NTC, false, false, false, true><<<grid, block, 0, st>>>(a);
        }
    } else {
        if (a.sh.cross_wave)
            fwd_kernel<P, D, NTC, true, false, false, false><<<grid, block, 0, st>>>(a);
        else if (a.g.lx == 16 * NTC)
            fwd_kernel<P, D, NTC, false, false, true, false><<<grid, block, 0, st>>>(a);
        else
            fwd_kernel<P, D, NTC, false, false, false, false><<<grid, block, 0, st>>>(a);
    }
    return (int)hipGetLastError();
}

int launch_forward(const FwdArgs& a, hipStream_t st) {
    const int d = a.g.d;
    if (a.sh.ntc != ntc_for(a.g.prec, d)) return (int)hipErrorInvalidValue;   // shape from another model
    if (a.g.prec == kBF16) {
        switch (d) {
            case 32: return launch_t<kBF16, 32, ntc_for(kBF16, 32)>(a, st);
            case 64: return launch_t<kBF16, 64, ntc_for(kBF16, 64)>(a, st);
            case 128: return launch_t<kBF16, 128, ntc_for(kBF16, 128)>(a, st);
            case 256: return launch_t<kBF16, 256, ntc_for(kBF16, 256)>(a, st);
        }
    } else {
        switch (d) {
            case 32: return launch_t<kFP32, 32, ntc_for(kFP32, 32)>(a, st);
            case 64: return launch_t<kFP32, 64, ntc_for(kFP32, 64)>(a, st);
            case 128: return launch_t<kFP32, 128, ntc_for(kFP32, 128)>(a, st);
            case 256: return launch_t<kFP32, 256, ntc_for(kFP32, 256)>(a, st);
        }
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace psr
