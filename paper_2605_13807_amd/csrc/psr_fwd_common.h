// Device-side helpers shared by the two forward kernels (psr_fwd.hip, psr_fwd_split.hip):
// operand formats, the MFMA products, the chunked in-row scan, GELU and the
// compensated sums.  See psr_fwd.hip for the precision scheme.
#pragma once

#include "psr_internal.h"
#include "gelu_fit.h"

#include <type_traits>

namespace psr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// The two 16-bit formats of the split paths: element and pair types, the scale
// s of the low part, and the 16x16x32 matrix product.
template <int P> struct Split;
template <> struct Split<kBF16> {
    typedef __bf16 E;
    typedef bf16x2 E2;
    typedef bf16x8 E8;
    static constexpr float kLoScale = 1.0f;
    __device__ static inline f32x4 mfma(E8 a, E8 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Split<kFP16> {
    typedef _Float16 E;
    typedef f16x2 E2;
    typedef f16x8 E8;
    static constexpr float kLoScale = 1.0f;
    __device__ static inline f32x4 mfma(E8 a, E8 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// Split operand fragments: dwords 0-3 hold 8 high parts, dwords 4-7 their 8 low parts.
template <int P> struct MF {
    typedef u32x8 Frag;
    static constexpr int K = 32;
    static constexpr int ELT = 4;  // bytes per value (hi and lo) in the row frontier
};
template <> struct MF<kFP32> {
    typedef float Frag;
    static constexpr int K = 4;
    static constexpr int ELT = 4;
};

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

// A operand (weights) of one 16-row output tile, per lane: split 16-bit one K
// block of 32 per piece (8 high and 8 low parts), FP32 four K steps of 4 per piece.
template <int P, int D>
struct AOp {
    static constexpr int N = (P != kFP32) ? D / 32 : D / 16;
    typedef typename std::conditional<P != kFP32, u32x8, f32x4>::type T;
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
        if constexpr (P != kFP32) {
            const u32x4 hi = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16 + k * 2048, mt * TILE, 0));
            const u32x4 lo =
                __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16 + k * 2048 + 1024, mt * TILE, 0));
            w[k] = __builtin_shufflevector(hi, lo, 0, 1, 2, 3, 4, 5, 6, 7);
        } else {
            w[k] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16 + k * 1024, mt * TILE, 0));
        }
    }
}

// acc[c] += W(tile) * b[c] for the NTC column tiles.  Split paths: the three
// partial products run as three independent accumulation chains (the high
// product on acc, the two low products on their own, started from zero) that
// are combined at the end, acc += s (c1 + c2).
template <int P, int D, int NTC, class W, class B>
__device__ inline void mma_a(f32x4 (&acc)[NTC], const W& w, const B& b) {
    if constexpr (P != kFP32) {
        typedef typename Split<P>::E8 E8;
        f32x4 c1[NTC], c2[NTC];
        const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < D / 32; ++kb)
#pragma unroll
            for (int c = 0; c < NTC; ++c) {
                // halves by shufflevector: hipcc's __builtin_bit_cast of a `.hi`
                // swizzle reads the vector's first half
                const u32x8 a = w[kb], v = b[c][kb];
                const E8 ah = __builtin_bit_cast(E8, __builtin_shufflevector(a, a, 0, 1, 2, 3));
                const E8 al = __builtin_bit_cast(E8, __builtin_shufflevector(a, a, 4, 5, 6, 7));
                const E8 bh = __builtin_bit_cast(E8, __builtin_shufflevector(v, v, 0, 1, 2, 3));
                const E8 bl = __builtin_bit_cast(E8, __builtin_shufflevector(v, v, 4, 5, 6, 7));
                acc[c] = Split<P>::mfma(ah, bh, acc[c]);
                c1[c] = Split<P>::mfma(al, bh, kb ? c1[c] : zero);
                c2[c] = Split<P>::mfma(ah, bl, kb ? c2[c] : zero);
            }
#pragma unroll
        for (int c = 0; c < NTC; ++c) acc[c] += (c1[c] + c2[c]) * Split<P>::kLoScale;
    } else {
#pragma unroll
        for (int kq = 0; kq < D / 16; ++kq)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int c = 0; c < NTC; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[kq][e], b[c][4 * kq + e], acc[c], 0, 0, 0);
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

// slots s, s+1 (s even) of a lane's operand array.  Split paths pack the
// pair's high parts into one dword of the fragment's first half and their low
// parts, (v - hi) / s rounded, into the same dword of the second half.
template <int P, int D>
__device__ inline void set_pair(typename MF<P>::Frag (&f)[D / MF<P>::K], int s, float x0, float x1) {
    if constexpr (P != kFP32) {
        typedef typename Split<P>::E E;
        typename Split<P>::E2 v, w;
        v[0] = (E)x0;
        v[1] = (E)x1;
        w[0] = (E)((x0 - (float)v[0]) * (1.0f / Split<P>::kLoScale));
        w[1] = (E)((x1 - (float)v[1]) * (1.0f / Split<P>::kLoScale));
        const int q = (s & 7) >> 1;
        f[s >> 3][q] = __builtin_bit_cast(uint32_t, v);
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
    if constexpr (P != kFP32) {
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
    if constexpr (P != kFP32) {
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
    if constexpr (P != kFP32) {
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

// The c4v symmetry T_k of the L-by-L lattice applied to a site s = y L + x: the
// kernels read a configuration as sigma o T_k, i.e. the spin at s is sigma(T_k(s)).
// k: identity, rotations by 90, 180, 270 degrees, reflections x -> L-1-x,
// y -> L-1-y, in the diagonal and in the anti-diagonal.
__device__ inline int xform_site(int site, int k, int L) {
    if (k == 0) return site;
    const int y = site / L, x = site - y * L;
    int xx = x, yy = y;
    switch (k) {
        case 1: xx = L - 1 - y; yy = x; break;
        case 2: xx = L - 1 - x; yy = L - 1 - y; break;
        case 3: xx = y; yy = L - 1 - x; break;
        case 4: xx = L - 1 - x; break;
        case 5: yy = L - 1 - y; break;
        case 6: xx = y; yy = x; break;
        default: xx = L - 1 - y; yy = L - 1 - x; break;
    }
    return yy * L + xx;
}

}  // namespace psr
