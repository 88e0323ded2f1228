// Forward kernel of the split 16-bit paths (BF16 or FP16 operand pairs, see
// psr_fwd.hip) for the stacked 2D snake minGRU (Sec. II.F-G) at d = 128 and 256.
//
// The workgroup's W waves share its C = 16 NTC columns (a column is one site
// of the current row of one sequence; whole sequence rows are packed back to
// back, the last columns may stay idle) and split the d units of every layer:
// wave w owns the UT = d / (16 W) output tiles of 16 units starting at tile
// w UT.  Rows run one after the other (the vertical input h_V makes them
// sequential, Sec. II.F); per row and layer:
//   GEMM1  z_pre = W_z u + b_z, htilde = W_h [u, h_V] + b_h and D u for the
//          wave's units, every column tile: the wave's weight fragments
//          (read once per workgroup and row instead of once per wave) times
//          the activations, u from LDS and h_V staged into LDS from the global
//          row frontier at the start of the layer (one load burst).
//          Layer 0's u-part comes from 9-entry gather tables (u^(0) is two
//          one-hot spins or zeros).
//   scan   gates a = z (0 at a row start), b = (1 - z) htilde and the affine
//          recurrence h_t = a_t h_{t-1} + b_t along the row for the wave's
//          units: every column of the workgroup is in the wave, so the chunked
//          scan (NTC columns composed in a lane, Hillis-Steele over the 16
//          lanes of a DPP row) needs no carry from another wave.
//   h      written as 16-bit pairs to LDS (the B operand of C h for every
//          wave) and, after the barrier that ends GEMM1, to the global row
//          frontier (the next row's h_V).
//   GEMM2  C h + D u + s (s = h^(l-1), Sec. II.G) for the wave's units, GELU,
//          written to LDS as the next layer's u; after the last layer each
//          wave's partial logit difference W_o[0] - W_o[1] is summed over the
//          waves through LDS and the first wave forms log p.
// Four barriers per layer and row (two on the first row), one more for the head.
#include "psr_fwd_common.h"

namespace psr {

// Waves and column tiles of the split kernel for width d (measured: at d = 128 four
// waves of two tiles over 64 columns ran 14 % faster than eight waves over 64 or 128).
static constexpr int split_waves(int d) { return d >= 256 ? 8 : 4; }
static constexpr int split_ntc(int d) { return d >= 128 ? 4 : 8; }

// One K block of 32 of output tile mt of a prepared split matrix: high parts in
// dwords 0-3, low parts in dwords 4-7 (layout of prep_frag_split).
template <int D>
__device__ inline u32x8 load_kb(const uint8_t* __restrict__ mat, int mt, int kb, int lane) {
    constexpr int TILE = D * 64;
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(mat), 0, TILE * (D / 16), 0x00020000);
    const u32x4 hi = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16 + kb * 2048, mt * TILE, 0));
    const u32x4 lo =
        __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16 + kb * 2048 + 1024, mt * TILE, 0));
    return __builtin_shufflevector(hi, lo, 0, 1, 2, 3, 4, 5, 6, 7);
}

// 32 bytes of one column's operand vector: high parts, then low parts, 16 each
__device__ inline u32x8 ld32(const uint8_t* p) {
    const u32x4 hi = *reinterpret_cast<const u32x4*>(p);
    const u32x4 lo = *reinterpret_cast<const u32x4*>(p + 16);
    return __builtin_shufflevector(hi, lo, 0, 1, 2, 3, 4, 5, 6, 7);
}

// c + a b with a = a_hi + s a_lo, b = b_hi + s b_lo: three 16-bit products, one chain
template <int P>
__device__ inline f32x4 mma3(u32x8 a, u32x8 b, f32x4 c) {
    typedef typename Split<P>::E8 E8;
    const E8 ah = __builtin_bit_cast(E8, __builtin_shufflevector(a, a, 0, 1, 2, 3));
    const E8 al = __builtin_bit_cast(E8, __builtin_shufflevector(a, a, 4, 5, 6, 7));
    const E8 bh = __builtin_bit_cast(E8, __builtin_shufflevector(b, b, 0, 1, 2, 3));
    const E8 bl = __builtin_bit_cast(E8, __builtin_shufflevector(b, b, 4, 5, 6, 7));
    c = Split<P>::mfma(ah, bh, c);
    c = Split<P>::mfma(al, bh, c);
    return Split<P>::mfma(ah, bl, c);
}

// Four values of one output tile (slots 4mt..4mt+3 of a lane group) as 16-bit
// pairs at p: 8 bytes of high parts at p, 8 bytes of low parts at p + 16.
template <int P>
__device__ inline void st_tile(uint8_t* p, const float (&v)[4]) {
    typedef typename Split<P>::E E;
    typename Split<P>::E2 h0, h1, l0, l1;
    h0[0] = (E)v[0];
    h0[1] = (E)v[1];
    h1[0] = (E)v[2];
    h1[1] = (E)v[3];
    l0[0] = (E)(v[0] - (float)h0[0]);
    l0[1] = (E)(v[1] - (float)h0[1]);
    l1[0] = (E)(v[2] - (float)h1[0]);
    l1[1] = (E)(v[3] - (float)h1[1]);
    *reinterpret_cast<uint2*>(p) = uint2{__builtin_bit_cast(uint32_t, h0), __builtin_bit_cast(uint32_t, h1)};
    *reinterpret_cast<uint2*>(p + 16) = uint2{__builtin_bit_cast(uint32_t, l0), __builtin_bit_cast(uint32_t, l1)};
}

// The four values of st_tile's layout back as floats (hi + lo)
template <int P>
__device__ inline f32x4 unpack4(uint2 vh, uint2 vl) {
    typedef typename Split<P>::E2 E2;
    const E2 h0 = __builtin_bit_cast(E2, vh.x), h1 = __builtin_bit_cast(E2, vh.y);
    const E2 l0 = __builtin_bit_cast(E2, vl.x), l1 = __builtin_bit_cast(E2, vl.y);
    return f32x4{(float)h0[0] + (float)l0[0], (float)h0[1] + (float)l0[1], (float)h1[0] + (float)l1[0],
                 (float)h1[1] + (float)l1[1]};
}

// XF: the spins are read through a c4v symmetry of the lattice (a.xform).
template <int P, int D, int W, int NTC, bool XF>
__global__ void __launch_bounds__(W * 64) fwd_split_kernel(const FwdArgs a) {
    static_assert(P != kFP32, "split kernel: 16-bit operand pairs only");
    static_assert(Split<P>::kLoScale == 1.0f, "split kernel: unscaled low parts");
    constexpr int NT = D / 16;           // output tiles of a layer
    constexpr int UT = NT / W;           // output tiles of one wave
    static_assert(UT >= 1 && UT * W == NT, "waves must divide the output tiles");
    constexpr int NKB = D / 32;          // K blocks of 32
    constexpr int C = 16 * NTC;          // columns of the workgroup
    constexpr int NS = D / 4;            // slots of a lane group
    constexpr int PITCH = 4 * D + 16;    // bytes of one column in the LDS activation buffers

    // u (the layer input) and h of the current layer, per column: D 16-bit pairs
    // in slot order (lane group g at g D bytes; per 32-value fragment 16 bytes of
    // high parts, then 16 of low parts), rows padded by 16 bytes.  The column
    // r16 NTC + c of a lane's chunk has LDS row c 16 + r16, so that the 16 lanes
    // of a DPP row read rows one pitch (16 bytes modulo the 256 bytes of the
    // banks) apart: no bank conflicts on the 16-byte reads.
    __shared__ __attribute__((aligned(16))) uint8_t lu[C * PITCH];
    __shared__ __attribute__((aligned(16))) uint8_t lh[C * PITCH];
    __shared__ float red[W][C];          // per-wave partial logit differences
    __shared__ float lsum[C][2];         // per-column Neumaier sum of log p (and its compensation)
    __shared__ float xw_unused[2][kWaves][16][2];

    const int lane = threadIdx.x & 63;
    // the wave index through readfirstlane: the compiler then knows it is uniform, so the
    // tile offsets of the weight loads stay scalar (no per-lane waterfall around the loads)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, r16 = lane & 15;
    const Geom G = a.g;
    const int lx = G.lx, ly = G.ly, nl = G.nl;
    const int N = lx * ly;
    const int seqs = a.sh.seqs;
    const int T0 = wave * UT;            // first output tile of this wave

    int64_t q_end = a.q_begin + a.q_count;
    if (a.q_total) q_end = min(q_end, *a.q_total);
    const int64_t q0 = a.q_begin + (int64_t)blockIdx.x * seqs;
    if (q0 >= q_end) return;   // uniform across the workgroup

    // per-column constants of this lane's chunk (columns r16 NTC + c): row position
    // t and sequence k packed as t | k << 16, the packed spin row and the flipped sites
    int tk[NTC], srow[NTC], flip[NTC];
    uint32_t vmask = 0;   // bit c: column c holds a sequence of this launch
#pragma unroll
    for (int c = 0; c < NTC; ++c) {
        const int col = r16 * NTC + c;
        const int k = col / lx;
        tk[c] = (col - k * lx) | (k << 16);
        const int64_t q = q0 + k;
        const bool v = (k < seqs) && (q < q_end);
        vmask |= v ? (1u << c) : 0u;
        srow[c] = v ? (int)q : (int)q0;   // packed row of the spins
        flip[c] = -1;                      // sites a | b << 16 flipped (0xFFFF: none)
        if (a.desc && v) {
            const uint32_t s0 = a.desc[2 * q], s1 = a.desc[2 * q + 1];
            srow[c] = (int)s0;
            const uint32_t fa = s1 & 0xFFFF, fb = s1 >> 16;
            flip[c] = (int)(fa | ((fb == fa ? 0xFFFFu : fb) << 16));
        }
    }
    auto valid = [&](int c) -> bool { return (vmask >> c) & 1u; };
    auto tpos = [&](int c) -> int { return tk[c] & 0xFFFF; };
    auto kseq = [&](int c) -> int { return tk[c] >> 16; };
    // spin at lattice site s of the configuration read as sigma o T_xform (c4v symmetry)
    auto spin = [&](int c, int site) -> int {
        if constexpr (XF) site = xform_site(site, a.xform, G.slx);
        const uint32_t* w = a.spins + (size_t)srow[c] * a.words_per_seq;
        const int v = (int)((w[site >> 5] >> (site & 31)) & 1u);
        const int fa = flip[c] & 0xFFFF, fb = (int)((uint32_t)flip[c] >> 16);
        return v ^ (int)(site == fa) ^ (int)(site == fb);
    };
    const float* tab = a.tab;
    const uint32_t goff = (uint32_t)(g * NS) * 4u;   // byte offset of this lane group in a slot-ordered d-vector
    for (int e = threadIdx.x; e < 2 * C; e += W * 64) (&lsum[0][0])[e] = 0.0f;
    // this workgroup's sequences in the frontier ([seq][layer][column][D pairs], contiguous),
    // read and written through a buffer resource with 32-bit offsets
    const uint32_t lbytes = (uint32_t)(lx * D * 4);   // one layer of one sequence
    uint8_t* const wfront = reinterpret_cast<uint8_t*>(a.frontier) + (size_t)(q0 - a.q_begin) * nl * lbytes;
    const __amdgpu_buffer_rsrc_t fr =
        __builtin_amdgcn_make_buffer_rsrc(wfront, 0, (int)(seqs * nl * lbytes), 0x00020000);

#pragma unroll 1
    for (int j = 0; j < ly; ++j) {
        // frontier offset of each column (layer 0); idle columns read (never write) sequence 0
        uint32_t fro[NTC];
#pragma unroll
        for (int c = 0; c < NTC; ++c) {
            const int i = (j & 1) ? (lx - 1 - tpos(c)) : tpos(c);
            const int kl = valid(c) ? kseq(c) : 0;
            fro[c] = (uint32_t)(kl * nl) * lbytes + (uint32_t)(i * (D * 4) + g * D);
        }
        const bool vert = j > 0;
        float l0[NTC];   // partial logit difference l_0 - l_1 over this wave's units
#pragma unroll
        for (int c = 0; c < NTC; ++c) l0[c] = 0.0f;

#pragma unroll 1
        for (int l = 0; l < nl; ++l) {
            const bool first = (l == 0), last = (l == nl - 1);
            const uint8_t* fz = a.frag + a.pl.frag[l][0];
            const uint8_t* fu = a.frag + a.pl.frag[l][1];
            const uint8_t* fv = a.frag + a.pl.frag[l][2];
            const uint8_t* fd = a.frag + a.pl.frag[l][3];
            const uint8_t* fc = a.frag + a.pl.frag[l][4];
            const uint32_t lo_l = (uint32_t)l * lbytes;   // this layer's frontier columns

            // h_V of the whole row (the previous row's h^(l)) staged into the h buffer, which is
            // free until this layer's scan: one load burst per layer instead of a dependent
            // global load per column and K block in the h_V product
            if (vert) {
                constexpr int PIECES = 4 * D / 16;   // 16-byte pieces of a column
                for (int e = threadIdx.x; e < seqs * lx * PIECES; e += W * 64) {
                    const int col = e / PIECES, piece = e - col * PIECES;
                    const int k = col / lx, t = col - k * lx;
                    if (q0 + k >= q_end) continue;   // columns past the launch keep stale, finite values
                    const int i = (j & 1) ? (lx - 1 - t) : t;
                    const uint32_t src = (uint32_t)(k * nl + l) * lbytes + (uint32_t)(i * 4 * D + piece * 16);
                    const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(fr, src, 0, 0));
                    *reinterpret_cast<u32x4*>(lh + ((col % NTC) * 16 + col / NTC) * PITCH + piece * 16) = v;
                }
                __syncthreads();
            }

            // ---- GEMM1: seeds, then the products on u (layers >= 1) and on h_V (rows >= 1)
            f32x4 az[UT][NTC], ah[UT][NTC], ad[UT][NTC];
            if (first) {
                // u^(0) = (one-hot spin at the H-pred, at the V-pred): 9-entry tables
#pragma unroll
                for (int c = 0; c < NTC; ++c) {
                    const int i = (j & 1) ? (lx - 1 - tpos(c)) : tpos(c);
                    const int ih = (j & 1) ? i + 1 : i - 1;
                    int sH = 2, sV = 2;
                    if (valid(c)) {
                        if (ih >= 0 && ih < lx) sH = spin(c, j * lx + ih);
                        if (j > 0) sV = spin(c, (j - 1) * lx + i);
                    }
                    const uint32_t o = (uint32_t)((3 * sH + sV) * D + g * NS) * 4u;
#pragma unroll
                    for (int tt = 0; tt < UT; ++tt) {
                        const int mt = T0 + tt;
                        az[tt][c] = ld16(tab + a.pl.t0z + 4 * mt, o);
                        ah[tt][c] = ld16(tab + a.pl.t0h + 4 * mt, o);
                        ad[tt][c] = ld16(tab + a.pl.t0d + 4 * mt, o);
                    }
                }
            } else {
#pragma unroll
                for (int tt = 0; tt < UT; ++tt) {
                    const int mt = T0 + tt;
                    const f32x4 bz = ld16(tab + a.pl.bias_z[l] + 4 * mt, goff);
                    const f32x4 bh = ld16(tab + a.pl.bias_h[l] + 4 * mt, goff);
#pragma unroll
                    for (int c = 0; c < NTC; ++c) {
                        az[tt][c] = bz;
                        ah[tt][c] = bh;
                        ad[tt][c] = f32x4{0.f, 0.f, 0.f, 0.f};
                    }
                }
#pragma unroll 1
                for (int kb = 0; kb < NKB; ++kb) {
                    u32x8 wz[UT], wu[UT];
#pragma unroll
                    for (int tt = 0; tt < UT; ++tt) {
                        wz[tt] = load_kb<D>(fz, T0 + tt, kb, lane);
                        wu[tt] = load_kb<D>(fu, T0 + tt, kb, lane);
                    }
#pragma unroll
                    for (int c = 0; c < NTC; ++c) {
                        const u32x8 b = ld32(lu + (c * 16 + r16) * PITCH + g * D + kb * 32);
#pragma unroll
                        for (int tt = 0; tt < UT; ++tt) {
                            az[tt][c] = mma3<P>(wz[tt], b, az[tt][c]);
                            ah[tt][c] = mma3<P>(wu[tt], b, ah[tt][c]);
                        }
                        __builtin_amdgcn_sched_barrier(0);   // one column's operands live at a time
                    }
                }
            }
            // second pass: D u (layers >= 1) and W_hV h_V (rows >= 1)
            if (!first || vert) {
#pragma unroll 1
                for (int kb = 0; kb < NKB; ++kb) {
                    u32x8 wd[UT], wv[UT];
#pragma unroll
                    for (int tt = 0; tt < UT; ++tt) {
                        if (!first) wd[tt] = load_kb<D>(fd, T0 + tt, kb, lane);
                        if (vert) wv[tt] = load_kb<D>(fv, T0 + tt, kb, lane);
                    }
#pragma unroll
                    for (int c = 0; c < NTC; ++c) {
                        if (!first) {
                            const u32x8 b = ld32(lu + (c * 16 + r16) * PITCH + g * D + kb * 32);
#pragma unroll
                            for (int tt = 0; tt < UT; ++tt) ad[tt][c] = mma3<P>(wd[tt], b, ad[tt][c]);
                        }
                        if (vert) {
                            const u32x8 b = ld32(lh + (c * 16 + r16) * PITCH + g * D + kb * 32);   // staged h_V
#pragma unroll
                            for (int tt = 0; tt < UT; ++tt) ah[tt][c] = mma3<P>(wv[tt], b, ah[tt][c]);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
            // the residual joins the GEMM2 seed: s = h^(l-1) for l >= 2 (Sec. II.G), this
            // row's h of the layer below, from the frontier (written after that layer's first barrier)
            if (l >= 2) {
#pragma unroll
                for (int tt = 0; tt < UT; ++tt) {
                    const int mt = T0 + tt;
#pragma unroll
                    for (int c = 0; c < NTC; ++c) {
                        const uint32_t o = fro[c] + lo_l - lbytes + (mt >> 1) * 32 + (mt & 1) * 8;
                        const uint2 vh = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(fr, o, 0, 0));
                        const uint2 vl = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(fr, o + 16, 0, 0));
                        ad[tt][c] += unpack4<P>(vh, vl);
                    }
                }
            }

            if (vert) __syncthreads();   // every wave is done with the staged h_V before h overwrites it
            // ---- gates and the chunked scan along the row; h to LDS
#pragma unroll
            for (int tt = 0; tt < UT; ++tt) {
                const int mt = T0 + tt;
                float h[NTC][4];
                float keep[NTC];   // 0 at a row start: h_H is zero outside the lattice
#pragma unroll
                for (int c = 0; c < NTC; ++c) keep[c] = (tpos(c) == 0) ? 0.0f : 1.0f;
                scan_tile<NTC, false, false>(az[tt], ah[tt], keep, h, xw_unused, mt, wave, g, r16);
#pragma unroll
                for (int c = 0; c < NTC; ++c)
                    st_tile<P>(lh + (c * 16 + r16) * PITCH + g * D + (mt >> 1) * 32 + (mt & 1) * 8, h[c]);
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();   // h of every unit is in LDS; every wave is past GEMM1 (u and h_V reads)
            // h is the next row's h_V: this layer's frontier columns are free now (copied from LDS)
#pragma unroll
            for (int c = 0; c < NTC; ++c) {
                if (!valid(c)) continue;
#pragma unroll
                for (int tt = 0; tt < UT; ++tt) {
                    const int mt = T0 + tt;
                    const uint8_t* src = lh + (c * 16 + r16) * PITCH + g * D + (mt >> 1) * 32 + (mt & 1) * 8;
                    uint8_t* dst = wfront + fro[c] + lo_l + (mt >> 1) * 32 + (mt & 1) * 8;
                    *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(src);
                    *reinterpret_cast<uint2*>(dst + 16) = *reinterpret_cast<const uint2*>(src + 16);
                }
            }

            // ---- GEMM2: x = GELU(C h + D u + s) for this wave's units
#pragma unroll 1
            for (int kb = 0; kb < NKB; ++kb) {
                u32x8 wc[UT];
#pragma unroll
                for (int tt = 0; tt < UT; ++tt) wc[tt] = load_kb<D>(fc, T0 + tt, kb, lane);
#pragma unroll
                for (int c = 0; c < NTC; ++c) {
                    const u32x8 b = ld32(lh + (c * 16 + r16) * PITCH + g * D + kb * 32);
#pragma unroll
                    for (int tt = 0; tt < UT; ++tt) ad[tt][c] = mma3<P>(wc[tt], b, ad[tt][c]);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if (!last) {
                // the next layer's input, in LDS (every wave finished reading u before the barrier above)
#pragma unroll
                for (int tt = 0; tt < UT; ++tt) {
                    const int mt = T0 + tt;
#pragma unroll
                    for (int c = 0; c < NTC; ++c) {
                        float x[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) x[i] = gelu_tail(ad[tt][c][i]);
                        st_tile<P>(lu + (c * 16 + r16) * PITCH + g * D + (mt >> 1) * 32 + (mt & 1) * 8, x);
                        // one column at a time: interleaving all of them costs more registers than it hides
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            } else {
#pragma unroll
                for (int tt = 0; tt < UT; ++tt) {
                    const f32x4 hw = ld16(tab + a.pl.head_w + 4 * (T0 + tt), goff);
#pragma unroll
                    for (int c = 0; c < NTC; ++c) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) l0[c] = fmaf(hw[i], gelu_tail(ad[tt][c][i]), l0[c]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
            __syncthreads();   // the next layer's u is complete; every wave is done with h in LDS
        }

        // ---- head: logit difference over all units, log p of the site's own spin
#pragma unroll
        for (int c = 0; c < NTC; ++c) {
            float v = l0[c];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (g == 0) red[wave][r16 * NTC + c] = v;
        }
        __syncthreads();
        if (wave == 0 && g == 0) {
            const float bod = tab[a.pl.head_b];
#pragma unroll
            for (int c = 0; c < NTC; ++c) {
                const int col = r16 * NTC + c;
                float v = bod;
#pragma unroll
                for (int w = 0; w < W; ++w) v += red[w][col];
                const int i = (j & 1) ? (lx - 1 - tpos(c)) : tpos(c);
                const int own = valid(c) ? spin(c, j * lx + i) : 0;
                // dl = (logit of the other spin) - (logit of the own spin); log p = -softplus(dl)
                const float dl = own ? v : -v;
                const float e = __builtin_amdgcn_exp2f(fabsf(dl) * kNegLog2e);
                const float lp = -(fmaxf(dl, 0.0f) + kLn2 * __builtin_amdgcn_logf(1.0f + e));
                if (valid(c)) {
                    neumaier(lsum[col][0], lsum[col][1], lp);
                    if (a.logp_site) a.logp_site[(size_t)(q0 + kseq(c)) * N + j * lx + i] = lp;
                }
            }
        }
        // red is rewritten only after the next row's layer barriers
    }

    // per-sequence total over its columns, in column order
    __syncthreads();
    const int k = threadIdx.x;
    if (k < seqs && q0 + k < q_end) {
        float s0 = 0.0f, cc = 0.0f;
        for (int t2 = 0; t2 < lx; ++t2) {
            neumaier(s0, cc, lsum[k * lx + t2][0]);
            cc += lsum[k * lx + t2][1];
        }
        // log psi = (1/2) sum log p; kept as a float pair (hi, lo), scaled exactly
        const float hi = s0 + cc;
        const float lo = cc - (hi - s0);
        a.out_hi[q0 + k] = 0.5f * hi;
        if (a.out_lo) a.out_lo[q0 + k] = 0.5f * lo;
    }
}

template <int P, int D>
static int launch_split_t(const FwdArgs& a, hipStream_t st) {
    constexpr int W = split_waves(D), NTC = split_ntc(D);
    if (a.sh.waves != W || a.sh.ntc != NTC) return (int)hipErrorInvalidValue;   // shape from another model
    const int64_t blocks = (a.q_count + a.sh.seqs - 1) / a.sh.seqs;
    if (blocks <= 0) return 0;
    if (a.g.sym)
        fwd_split_kernel<P, D, W, NTC, true><<<dim3((unsigned)blocks), dim3(W * 64), 0, st>>>(a);
    else
        fwd_split_kernel<P, D, W, NTC, false><<<dim3((unsigned)blocks), dim3(W * 64), 0, st>>>(a);
    return (int)hipGetLastError();
}

// d >= 128 (d = 64 keeps the lane-owns-all-units kernel of psr_fwd.hip, whose operand
// sets fit in registers there; not measured with this kernel)
bool split_kernel_applies(const Geom& g) {
    return g.prec != kFP32 && !g.chain && g.patch == 1 && g.d >= 128 && g.lx <= 16 * split_ntc(g.d);
}

void split_shape(const Geom& g, FwdShape* s) {
    s->ntc = split_ntc(g.d);
    s->waves = split_waves(g.d);
    s->cols = 16 * s->ntc;
    s->seqs = s->cols / g.lx;
    s->cross_wave = 0;
    s->lds_frontier = 0;
    s->split_kernel = 1;
}

int launch_forward_split(const FwdArgs& a, hipStream_t st) {
    if (a.g.prec == kBF16) {
        switch (a.g.d) {
            case 128: return launch_split_t<kBF16, 128>(a, st);
            case 256: return launch_split_t<kBF16, 256>(a, st);
        }
    } else if (a.g.prec == kFP16) {
        switch (a.g.d) {
            case 128: return launch_split_t<kFP16, 128>(a, st);
            case 256: return launch_split_t<kFP16, 256>(a, st);
        }
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace psr
