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
// Precision.  FP32: v_mfma_f32_16x16x4_f32.  The 16-bit paths carry every
// operand v of a dense projection (weights and activations alike) as two
// 16-bit parts, v ~ hi + s lo with hi = r(v) and lo = r((v - hi) / s), and form a
// product W x as W_hi x_hi + s (W_lo x_hi + W_hi x_lo) on the 16-bit matrix
// cores with FP32 accumulation (the dropped s^2 W_lo x_lo term is below the
// parts' own rounding):
//   BF16  r = bfloat16 rounding, s = 1: hi + lo holds ~16 significant bits;
//   FP16  r = binary16 rounding, s = 1: ~22 significant bits where the low
//         part is a normal number (|v| above ~2^-3), an absolute error below
//         2^-25 where it is subnormal; within binary16's range (|v| < 65504,
//         which the unit-scale activations and weights respect).
// (The split-operand kernel for d = 128 and 256 is psr_fwd_split.hip; this file
// keeps the FP32 path, the split paths at d = 32 and 64, and the chain.)
// A single 16-bit rounding of the operands perturbs this randomly initialised
// recurrence too much for the local energy (per-configuration log-ratio errors
// of 0.1-1 at 20x20 and above); the split keeps it at a few hundred (BF16) or a
// few (FP16) float32 ulps, for a third of the 16-bit matrix rate.
#include "psr_fwd_common.h"

namespace psr {

// ---------------------------------------------------------------------------
// Parameter preparation: fragment-order weights and slot-order tables
// ---------------------------------------------------------------------------

__device__ __host__ inline int unit_pos(int u, int d) {
    // position of unit u in a slot-ordered vector: [g][s], unit = slot_unit(s, g)
    return ((u >> 2) & 3) * (d >> 2) + 4 * (u >> 4) + (u & 3);
}

// Split weight fragments: for output tile mt and K block kb of 32, the 64
// lanes' 8 high parts (1 KB), then the 64 lanes' 8 low parts (1 KB).
template <int P>
__global__ void prep_frag_split(const float* __restrict__ theta, MatSrc src, int d, typename Split<P>::E* __restrict__ out) {
    typedef typename Split<P>::E E;
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
    const E hi = (E)v;
    const E lo = (E)((v - (float)hi) * (1.0f / Split<P>::kLoScale));
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

// Layer-0 gathers.  state = (K+1) sH + sV with s = the local state (a spin, or a
// 2x2 patch's 16-letter state) or K (outside the lattice).
// snake: u^(0) = [onehot_K(sH), onehot_K(sV)];  chain: u^(0) = onehot_2(sH).
struct Tab0Src {
    int chain, d, K;
    int64_t wz, bz, wh, bh, dd;   // theta offsets of W_z^(0), b_z^(0), W_h^(0), b_h^(0), D^(0) (dd < 0: none)
    int ldz, ldh;                 // row strides of W_z^(0) and W_h^(0)
};

__global__ void prep_tab0(const float* __restrict__ theta, Tab0Src s, float* __restrict__ tz, float* __restrict__ th,
                          float* __restrict__ td) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int K = s.K;
    if (e >= (K + 1) * (K + 1) * s.d) return;
    const int st = e / s.d, u = e % s.d;
    const int sH = st / (K + 1), sV = st % (K + 1);
    float z = theta[s.bz + u], h = theta[s.bh + u], dv = 0.0f;
    if (sH < K) {
        z += theta[s.wz + (int64_t)u * s.ldz + sH];
        h += theta[s.wh + (int64_t)u * s.ldh + sH];
        if (s.dd >= 0) dv += theta[s.dd + (int64_t)u * (2 * K) + sH];
    }
    if (!s.chain && sV < K) {
        z += theta[s.wz + (int64_t)u * s.ldz + K + sV];
        h += theta[s.wh + (int64_t)u * s.ldh + K + sV];
        if (s.dd >= 0) dv += theta[s.dd + (int64_t)u * (2 * K) + K + sV];
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

// Head of the K-class log-softmax (2x2 patches, K = 16): every row of W_o in slot order, and b_o.
__global__ void prep_head_k(const float* __restrict__ theta, int64_t src_w, int64_t src_b, int d, int K,
                            float* __restrict__ w, float* __restrict__ b) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K * d) return;
    const int cls = e / d, u = e % d;
    w[cls * d + unit_pos(u, d)] = theta[src_w + e];
    if (u == 0) b[cls] = theta[src_b + cls];
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
            const int du = (l == 0) ? 2 * n_states(g) : d;
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
                prep_frag_split<kBF16><<<blocks, T, 0, st>>>(theta, s, d, reinterpret_cast<__bf16*>(frag + fo));
            else if (g.prec == kFP16)
                prep_frag_split<kFP16><<<blocks, T, 0, st>>>(theta, s, d, reinterpret_cast<_Float16*>(frag + fo));
            else
                prep_frag_f32<<<blocks, T, 0, st>>>(theta, s, d, reinterpret_cast<float*>(frag + fo));
        }
    }
    // layer-0 tables
    Tab0Src s0;
    s0.chain = g.chain;
    s0.d = d;
    s0.K = n_states(g);
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
        s0.ldz = 2 * s0.K;
        s0.ldh = 2 * s0.K + d;
    }
    const int nst = (s0.K + 1) * (s0.K + 1);
    prep_tab0<<<(nst * d + T - 1) / T, T, 0, st>>>(theta, s0, tab + pl.t0z, tab + pl.t0h, tab + pl.t0d);
    for (int l = 1; l < g.nl; ++l) {
        prep_vec<<<(d + T - 1) / T, T, 0, st>>>(theta, off[6 * l + 1], d, 1, tab + pl.bias_z[l]);
        prep_vec<<<(d + T - 1) / T, T, 0, st>>>(theta, off[6 * l + 3], d, 1, tab + pl.bias_h[l]);
    }
    const int ih = g.chain ? 4 : 6 * g.nl;   // index of W_o in the tensor list
    if (n_states(g) == 2)
        prep_head<<<(d + T - 1) / T, T, 0, st>>>(theta, off[ih], off[ih + 1], d, tab + pl.head_w, tab + pl.head_b);
    else
        prep_head_k<<<(n_states(g) * d + T - 1) / T, T, 0, st>>>(theta, off[ih], off[ih + 1], d, n_states(g),
                                                                 tab + pl.head_w, tab + pl.head_b);
    return (int)hipGetLastError();
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


// PATCH: 2x2 patch inputs (a 16-letter alphabet per grid site, a 16-way head).
// XF: the spins are read through a c4v symmetry of the lattice (a.xform).
template <int P, int D, int NTC, bool CROSS, bool CHAIN, bool ALIGNED, bool LDSF, bool PATCH = false, bool XF = false>
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
    // spin at lattice site s of the configuration (XF: read as sigma o T_xform, a c4v symmetry)
    auto spin = [&](int c, int site) -> int {
        if constexpr (XF) site = xform_site(site, a.xform, G.slx);
        const uint32_t* w = a.spins + (size_t)srow[c] * a.words_per_seq;
        const int v = (int)((w[site >> 5] >> (site & 31)) & 1u);
        const int fa = flip[c] & 0xFFFF, fb = (int)((uint32_t)flip[c] >> 16);
        return v ^ (int)(site == fa) ^ (int)(site == fb);
    };
    // local state at grid site (i, jj): the spin, or the 16-letter state of the 2x2 patch
    // s(2i, 2jj) + 2 s(2i+1, 2jj) + 4 s(2i, 2jj+1) + 8 s(2i+1, 2jj+1)
    auto local_state = [&](int c, int i, int jj) -> int {
        if constexpr (PATCH) {
            const int s0 = (2 * jj) * G.slx + 2 * i;
            return spin(c, s0) | (spin(c, s0 + 1) << 1) | (spin(c, s0 + G.slx) << 2) | (spin(c, s0 + G.slx + 1) << 3);
        } else {
            return spin(c, jj * lx + i);
        }
    };
    constexpr int K = PATCH ? 16 : 2;   // local alphabet; K also marks 'outside the lattice'
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
            int sH = K, sV = K;
            const int ih = (j & 1) ? i + 1 : i - 1;
            own[c] = 0;
            if (valid[c]) {
                if (ih >= 0 && ih < lx) sH = local_state(c, ih, j);
                if (j > 0) sV = local_state(c, i, j - 1);
                own[c] = local_state(c, i, j);
            }
            st[c] = (K + 1) * sH + sV;
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
        // PATCH: all 16 logits (partial over this lane's units)
        float lk[PATCH ? 16 : 1][NTC];
#pragma unroll
        for (int k = 0; k < (PATCH ? 16 : 1); ++k)
#pragma unroll
            for (int c = 0; c < NTC; ++c) lk[k][c] = 0.0f;

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
                            if constexpr (P != kFP32) {
                                // slots 4mt..4mt+3: two dwords of high parts and the two
                                // dwords of their low parts, 16 bytes further on
                                typedef typename Split<P>::E2 E2;
                                const uint8_t* q = rsrc[c] + (mt >> 1) * 32 + (mt & 1) * 8;
                                const uint2 vh = *reinterpret_cast<const uint2*>(q);
                                const uint2 vl = *reinterpret_cast<const uint2*>(q + 16);
                                const E2 h0 = __builtin_bit_cast(E2, vh.x), h1 = __builtin_bit_cast(E2, vh.y);
                                const E2 l0 = __builtin_bit_cast(E2, vl.x), l1 = __builtin_bit_cast(E2, vl.y);
                                constexpr float sc = Split<P>::kLoScale;
                                so[c] = f32x4{fmaf((float)l0[0], sc, (float)h0[0]), fmaf((float)l0[1], sc, (float)h0[1]),
                                              fmaf((float)l1[0], sc, (float)h1[0]), fmaf((float)l1[1], sc, (float)h1[1])};
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
                    } else if constexpr (PATCH) {
#pragma unroll
                        for (int c = 0; c < NTC; ++c) {
                            float x[4];
#pragma unroll
                            for (int i = 0; i < 4; ++i) x[i] = gelu_tail(ao[sl][c][i]);
#pragma unroll
                            for (int k = 0; k < 16; ++k) {
                                const f32x4 hw = ld16(tab + a.pl.head_w + k * D + 4 * mt, goff);
#pragma unroll
                                for (int i = 0; i < 4; ++i) lk[k][c] = fmaf(hw[i], x[i], lk[k][c]);
                            }
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
            float lp;
            if constexpr (PATCH) {
                // log p(k_own) = l_own - max - ln sum_k exp(l_k - max) over the 16 logits
                float v[16], mx = -3.0e38f, vo = 0.0f;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    float t2 = lk[k][c];
                    t2 += __shfl_xor(t2, 16);
                    t2 += __shfl_xor(t2, 32);
                    v[k] = t2 + tab[a.pl.head_b + k];
                    mx = fmaxf(mx, v[k]);
                    vo = (k == own[c]) ? v[k] : vo;
                }
                float se = 0.0f;
#pragma unroll
                for (int k = 0; k < 16; ++k) se += __builtin_amdgcn_exp2f((v[k] - mx) * -kNegLog2e);
                lp = (vo - mx) - kLn2 * __builtin_amdgcn_logf(se);
            } else {
                float v = l0[c];
                v += __shfl_xor(v, 16);
                v += __shfl_xor(v, 32);
                v += bod;
                // dl = (logit of the other spin) - (logit of the own spin)
                const float dl = own[c] ? v : -v;
                // log p = -softplus(dl) = -(max(dl, 0) + ln(1 + e^-|dl|)), in base 2 on the
                // hardware exp2/log2 (1 + e rounds to 1 only where e < 2^-24)
                const float e = __builtin_amdgcn_exp2f(fabsf(dl) * kNegLog2e);
                lp = -(fmaxf(dl, 0.0f) + kLn2 * __builtin_amdgcn_logf(1.0f + e));
            }
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
    if (split_kernel_applies(g)) {
        split_shape(g, &s);
        return s;
    }
    s.split_kernel = 0;
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
    // split frontier rows: d values of 4 bytes (high and low parts) plus 16 bytes of padding
    const int64_t pitch = (int64_t)g.d * 4 + 16;
    // the patch and symmetry kernels are instantiated for the general layout only
    if (g.patch == 2 || g.sym) s.cross_wave = 1;
    s.lds_frontier = (!g.chain && g.prec != kFP32 && g.patch == 1 && !g.sym &&
                      (int64_t)g.d * 4 + (int64_t)s.seqs * g.nl * g.lx * pitch <= kLdsFrontier) ? 1 : 0;
    return s;
}

template <int P, int D, int NTC>
static int launch_t(const FwdArgs& a, hipStream_t st) {
    const int64_t blocks = (a.q_count + a.sh.seqs - 1) / a.sh.seqs;
    if (blocks <= 0) return 0;
    const dim3 grid((unsigned)blocks), block(kWaves * 64);
    if (a.g.patch == 2 || a.g.sym) {
        // 2x2 patches and c4v-symmetrised evaluations: the general layout (rows may straddle
        // waves, frontier in global memory)
        if (a.g.patch == 2 && a.g.sym)
            fwd_kernel<P, D, NTC, true, false, false, false, true, true><<<grid, block, 0, st>>>(a);
        else if (a.g.patch == 2)
            fwd_kernel<P, D, NTC, true, false, false, false, true, false><<<grid, block, 0, st>>>(a);
        else
            fwd_kernel<P, D, NTC, true, false, false, false, false, true><<<grid, block, 0, st>>>(a);
    } else if (a.g.chain) {
        if (a.sh.cross_wave)
            fwd_kernel<P, D, NTC, true, true, false, false><<<grid, block, 0, st>>>(a);
        else
            fwd_kernel<P, D, NTC, false, true, false, false><<<grid, block, 0, st>>>(a);
    } else if (a.sh.lds_frontier) {
        if constexpr (P != kFP32) {
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
    if (a.sh.split_kernel) return launch_forward_split(a, st);
    if (a.sh.ntc != ntc_for(a.g.prec, d)) return (int)hipErrorInvalidValue;   // shape from another model
    if (a.g.prec == kBF16) {
        switch (d) {
            case 32: return launch_t<kBF16, 32, ntc_for(kBF16, 32)>(a, st);
            case 64: return launch_t<kBF16, 64, ntc_for(kBF16, 64)>(a, st);
            case 128: return launch_t<kBF16, 128, ntc_for(kBF16, 128)>(a, st);
            case 256: return launch_t<kBF16, 256, ntc_for(kBF16, 256)>(a, st);
        }
    } else if (a.g.prec == kFP16) {
        switch (d) {
            case 32: return launch_t<kFP16, 32, ntc_for(kFP16, 32)>(a, st);
            case 64: return launch_t<kFP16, 64, ntc_for(kFP16, 64)>(a, st);
            case 128: return launch_t<kFP16, 128, ntc_for(kFP16, 128)>(a, st);
            case 256: return launch_t<kFP16, 256, ntc_for(kFP16, 256)>(a, st);
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
