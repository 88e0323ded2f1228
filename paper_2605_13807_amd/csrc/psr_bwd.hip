// Per-sample gradients O_s = d log psi(sigma_s) / d theta (reverse mode), FP32.
//
// One workgroup per sample.  Phase 0 runs the row recurrence forward and keeps
// only the row frontier h^(l) (all layers, all columns) at the start of every
// checkpoint chunk of R rows.  Phase 1 walks the chunks backwards: each chunk is
// recomputed from its checkpoint (storing its intermediates), then swept in
// reverse, row by row and layer by layer:
//   head      g_logit_t = (1/2) (onehot(sigma_t) - softmax(logits_t))
//   output    g_pre = g_x * GELU'(pre), pre = C h + D u + s
//   residual  s^(l) = h^(l-1) (l >= 2) sends g_pre^(l) to h^(l-1)
//   state     g_h = C^T g_pre + [residual] + W_hV^T g_htilde(next row, same column)
//   scan      lambda_t = g_h_t + z_{t+1} lambda_{t+1}   (the reverse of
//             h_t = z_t h_{t-1} + (1 - z_t) htilde_t along the zigzag row)
//   gates     g_z = lambda (h_{t-1} - htilde),  g_htilde = lambda (1 - z),
//             g_zpre = g_z z (1 - z)
//   input     g_u = W_z^T g_zpre + W_hu^T g_htilde + D^T g_pre
// The weight gradients of the chunk are the outer products summed over the
// chunk's sites and are added to the sample's row of O once per chunk.
#include "psr_internal.h"
#include "psr_gemm.h"

namespace psr {

namespace {

struct BwdArgs {
    Geom g;
    int R, nch;
    const float* theta;
    int64_t off[64];           // tensor offsets in theta (and in a row of O)
    const uint32_t* packed;
    int words;
    int64_t B, P;
    float* scratch;
    int64_t per_sample;
    float* O;
    float* logpsi;
};

struct Buf {
    float *ckpt, *front, *Z, *HT, *H, *PRE, *XIN, *HV, *GZP, *GHT, *GPRE, *GLOG, *GFR, *GX, *GRES, *LAM, *ROWIN;
};

__device__ inline float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }
__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_d(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.3989422804014327f * expf(-0.5f * x * x);
}

__host__ __device__ inline Buf carve(float* base, int nch, int R, int nl, int lx, int d) {
    Buf b;
    const int64_t F = (int64_t)nl * lx * d;   // one frontier
    const int64_t C = (int64_t)R * F;         // one chunk tensor
    float* p = base;
    b.ckpt = p; p += nch * F;
    b.front = p; p += F;
    b.Z = p; p += C;
    b.HT = p; p += C;
    b.H = p; p += C;
    b.PRE = p; p += C;
    b.XIN = p; p += C;
    b.HV = p; p += C;
    b.GZP = p; p += C;
    b.GHT = p; p += C;
    b.GPRE = p; p += C;
    b.GLOG = p; p += (int64_t)R * lx * 2;
    b.GFR = p; p += 2 * F;
    b.GX = p; p += (int64_t)lx * d;
    b.GRES = p; p += F;
    b.LAM = p; p += (int64_t)lx * d;
    b.ROWIN = p; p += (int64_t)lx * 2 * d;
    return b;
}

__device__ inline int spin_at(const uint32_t* w, int a) { return (int)((w[a >> 5] >> (a & 31)) & 1u); }

// Component k of the layer-0 input at column i of row j:
// u = [onehot(H-pred), onehot(V-pred)] (chain: onehot of the previous site),
// zeros outside the lattice.
__device__ inline float u0_val(const Geom& G, const uint32_t* w, int j, int i, int k) {
    if (G.chain) return (i > 0 && spin_at(w, i - 1) == k) ? 1.0f : 0.0f;
    if (k < 2) {
        const int ih = (j & 1) ? i + 1 : i - 1;
        return (ih >= 0 && ih < G.lx && spin_at(w, j * G.lx + ih) == k) ? 1.0f : 0.0f;
    }
    return (j > 0 && spin_at(w, (j - 1) * G.lx + i) == k - 2) ? 1.0f : 0.0f;
}

// ---------------------------------------------------------------------------
// Dense products on the matrix cores (FP32 MFMA 16x16x4), operands in memory
// ---------------------------------------------------------------------------
//
using namespace gemm_detail;   // MA, MB, MC, gemm (psr_gemm.h)

// Offset of the (chunk row r, layer l) slab of a chunk tensor: layer-major, so
// that the rows of one layer are contiguous ([l][r][column][unit]).
__device__ inline int64_t cidx(const BwdArgs& a, int r, int l) {
    return ((int64_t)l * a.R + r) * a.g.lx * a.g.d;
}

// One row forward for every layer.  When `r >= 0` the row's intermediates
// are stored in chunk slot r.  Updates the frontier and returns the row's
// sum of log p (thread 0 only; others return 0).
__device__ float row_forward(const BwdArgs& a, const Buf& b, const uint32_t* w, int j, int r) {
    const Geom& G = a.g;
    const int lx = G.lx, d = G.d, nl = G.nl;
    const int tid = threadIdx.x, T = blockDim.x;
    const int64_t F1 = (int64_t)lx * d;
    float logp_sum = 0.0f;
    float* X = b.ROWIN;            // [lx][d] current layer input x^(l) (layers >= 1)
    float* Hrow = b.LAM;           // [lx][d] h of this layer (row)
    const float* th = a.theta;
    for (int l = 0; l < nl; ++l) {
        const int du = G.chain ? 2 : (l == 0 ? 4 : d);
        const int64_t oWz = a.off[6 * l + 0], obz = a.off[6 * l + 1], oWh = a.off[6 * l + 2], obh = a.off[6 * l + 3];
        float* Zs = (r >= 0) ? b.Z + cidx(a, r, l) : b.GX;       // GX is free during the forward
        float* HTs = (r >= 0) ? b.HT + cidx(a, r, l) : b.GRES;
        const float* hv = b.front + l * F1;
        const bool vert = !G.chain && j > 0;
        const int ldh = G.chain ? du : du + d;   // row stride of W_h ([d][2] on the chain)
        // projections: biases and the one-hot layer-0 input here, dense parts on MFMA
        for (int e = tid; e < lx * d; e += T) {
            const int i = e / d, m = e - i * d;
            float zp = th[obz + m], hp = th[obh + m];
            if (l == 0) {
                for (int k = 0; k < du; ++k) {
                    const float uk = u0_val(G, w, j, i, k);
                    zp = fmaf(th[oWz + (int64_t)m * du + k], uk, zp);
                    hp = fmaf(th[oWh + (int64_t)m * ldh + k], uk, hp);
                }
            }
            Zs[e] = zp;
            HTs[e] = hp;
            if (r >= 0) {
                b.HV[cidx(a, r, l) + e] = vert ? hv[e] : 0.0f;
                if (l > 0) b.XIN[cidx(a, r, l) + e] = X[e];
            }
        }
        __syncthreads();
        if (l >= 1) {
            gemm(d, lx, d, MA{th + oWz, du, 1}, MB{X, 1, d}, MC{Zs, 1, d}, true);
            gemm(d, lx, d, MA{th + oWh, ldh, 1}, MB{X, 1, d}, MC{HTs, 1, d}, true);
        }
        if (vert) gemm(d, lx, d, MA{th + oWh + du, ldh, 1}, MB{hv, 1, d}, MC{HTs, 1, d}, true);
        __syncthreads();
        for (int e = tid; e < lx * d; e += T) Zs[e] = sigm(Zs[e]);
        __syncthreads();
        // sequential recurrence along the snake row, one thread per unit; the operands
        // of a block of 8 sites are loaded before the block's dependent updates
        for (int m = tid; m < d; m += T) {
            float h = 0.0f;
            for (int s0 = 0; s0 < lx; s0 += 8) {
                float zb[8], tb[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int s = min(s0 + q, lx - 1);
                    const int i = (j & 1) ? lx - 1 - s : s;
                    zb[q] = Zs[i * d + m];
                    tb[q] = HTs[i * d + m];
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int s = s0 + q;
                    if (s < lx) {
                        const int i = (j & 1) ? lx - 1 - s : s;
                        h = zb[q] * h + (1.0f - zb[q]) * tb[q];
                        Hrow[i * d + m] = h;
                    }
                }
            }
        }
        __syncthreads();
        if (G.chain) {
            // the head reads h directly
            for (int e = tid; e < lx * d; e += T) {
                if (r >= 0) b.H[cidx(a, r, l) + e] = Hrow[e];
                X[e] = Hrow[e];
            }
            __syncthreads();
            break;
        }
        // output x = GELU(C h + D u + s)
        const int64_t oC = a.off[6 * l + 4], oD = a.off[6 * l + 5];
        float* Ps = (r >= 0) ? b.PRE + cidx(a, r, l) : b.GZP;   // GZP free during the forward
        for (int e = tid; e < lx * d; e += T) {
            const int i = e / d, m = e - i * d;
            float p = 0.0f;
            if (l == 0) {
                for (int k = 0; k < 4; ++k) p = fmaf(th[oD + (int64_t)m * 4 + k], u0_val(G, w, j, i, k), p);
            }
            if (l >= 2) p += b.front[(l - 1) * F1 + e];   // h^(l-1) of this row (frontier already updated)
            Ps[e] = p;
        }
        __syncthreads();
        gemm(d, lx, d, MA{th + oC, d, 1}, MB{Hrow, 1, d}, MC{Ps, 1, d}, true);
        if (l >= 1) gemm(d, lx, d, MA{th + oD, d, 1}, MB{X, 1, d}, MC{Ps, 1, d}, true);
        __syncthreads();
        for (int e = tid; e < lx * d; e += T) {
            if (r >= 0) b.H[cidx(a, r, l) + e] = Hrow[e];
            b.front[l * F1 + e] = Hrow[e];
            X[e] = gelu(Ps[e]);
        }
        __syncthreads();
    }
    // head on X = x^(nl) (chain: h)
    const int64_t oWo = G.chain ? a.off[4] : a.off[6 * nl], obo = oWo + 2 * d;
    // logits: 8 threads per site, each a d/8 slice of the products, then a shuffle sum
    for (int i0 = 0; i0 < lx; i0 += T / 8) {
        const int i = i0 + tid / 8, part = tid % 8;
        float l0 = 0.0f, l1 = 0.0f;
        if (i < lx) {
            for (int k = part; k < d; k += 8) {
                l0 = fmaf(a.theta[oWo + k], X[i * d + k], l0);
                l1 = fmaf(a.theta[oWo + d + k], X[i * d + k], l1);
            }
        }
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
            l0 += __shfl_xor(l0, o, 8);
            l1 += __shfl_xor(l1, o, 8);
        }
        if (i >= lx || part != 0) continue;
        l0 += a.theta[obo];
        l1 += a.theta[obo + 1];
        const int own = spin_at(w, j * lx + i);
        const float mx = fmaxf(l0, l1);
        const float lse = mx + logf(expf(l0 - mx) + expf(l1 - mx));
        const float lp = (own ? l1 : l0) - lse;
        if (r >= 0) {
            const float p1 = expf(l1 - lse), p0 = expf(l0 - lse);
            b.GLOG[(r * lx + i) * 2 + 0] = 0.5f * ((own == 0 ? 1.0f : 0.0f) - p0);
            b.GLOG[(r * lx + i) * 2 + 1] = 0.5f * ((own == 1 ? 1.0f : 0.0f) - p1);
        }
        Hrow[i] = lp;   // reuse: per-site log p for the row sum below
    }
    __syncthreads();
    if (tid == 0)
        for (int i = 0; i < lx; ++i) logp_sum += Hrow[i];
    __syncthreads();
    return logp_sum;
}

__global__ void __launch_bounds__(256) bwd_kernel(const BwdArgs a) {
    const Geom& G = a.g;
    const int lx = G.lx, ly = G.ly, nl = G.nl, d = G.d;
    const int tid = threadIdx.x, T = blockDim.x;
    const int64_t s = blockIdx.x;
    const uint32_t* w = a.packed + s * a.words;
    Buf b = carve(a.scratch + s * a.per_sample, a.nch, a.R, nl, lx, d);
    const int64_t F = (int64_t)nl * lx * d, F1 = (int64_t)lx * d;
    float* Orow = a.O + s * a.P;
    const float* th = a.theta;

    // ---- phase 0: forward with checkpoints -------------------------------
    for (int64_t e = tid; e < F; e += T) b.front[e] = 0.0f;
    for (int64_t e = tid; e < a.P; e += T) Orow[e] = 0.0f;
    __syncthreads();
    float lsum = 0.0f, lcomp = 0.0f;
    for (int j = 0; j < ly; ++j) {
        if (j % a.R == 0) {
            float* ck = b.ckpt + (int64_t)(j / a.R) * F;
            for (int64_t e = tid; e < F; e += T) ck[e] = b.front[e];
            __syncthreads();
        }
        const float rs = row_forward(a, b, w, j, -1);
        if (tid == 0) {
            const float t = lsum + rs;
            lcomp += (fabsf(lsum) >= fabsf(rs)) ? ((lsum - t) + rs) : ((rs - t) + lsum);
            lsum = t;
        }
    }
    if (tid == 0 && a.logpsi) a.logpsi[s] = 0.5f * (lsum + lcomp);

    // ---- phase 1: chunks in reverse ---------------------------------------
    for (int64_t e = tid; e < 2 * F; e += T) b.GFR[e] = 0.0f;
    __syncthreads();
    int cur = 0;   // GFR[cur] holds the adjoint coming from the row below in the sweep (row j+1)
    const int64_t oWo = G.chain ? a.off[4] : a.off[6 * nl];
    for (int c = a.nch - 1; c >= 0; --c) {
        const int j0 = c * a.R, j1 = min(ly, j0 + a.R);
        const float* ck = b.ckpt + (int64_t)c * F;
        for (int64_t e = tid; e < F; e += T) b.front[e] = ck[e];
        __syncthreads();
        for (int j = j0; j < j1; ++j) row_forward(a, b, w, j, j - j0);

        for (int j = j1 - 1; j >= j0; --j) {
            const int r = j - j0;
            float* gin = b.GFR + cur * F;          // from row j+1
            float* gout = b.GFR + (1 - cur) * F;   // to row j-1
            // head adjoint into the last layer's output
            for (int e = tid; e < lx * d; e += T) {
                const int i = e / d, m = e - i * d;
                const float g0 = b.GLOG[(r * lx + i) * 2], g1 = b.GLOG[(r * lx + i) * 2 + 1];
                b.GX[e] = th[oWo + m] * g0 + th[oWo + d + m] * g1;
            }
            for (int64_t e = tid; e < F; e += T) b.GRES[e] = 0.0f;
            __syncthreads();
            for (int l = nl - 1; l >= 0; --l) {
                const int du = G.chain ? 2 : (l == 0 ? 4 : d);
                const int ldh = G.chain ? du : du + d;
                const int64_t base = cidx(a, r, l);
                float* gpre = b.GPRE + base;
                float* gzp = b.GZP + base;
                float* ght = b.GHT + base;
                const float* Z = b.Z + base;
                const float* HT = b.HT + base;
                const float* Hh = b.H + base;
                // g_pre and the direct adjoint of h: lambda = g_h(row below) + g_res + C^T g_pre
                if (!G.chain) {
                    const int64_t oC = a.off[6 * l + 4];
                    for (int e = tid; e < lx * d; e += T) {
                        const float gp = b.GX[e] * gelu_d(b.PRE[base + e]);
                        gpre[e] = gp;
                        b.LAM[e] = gin[l * F1 + e] + b.GRES[l * F1 + e];
                        if (l >= 2) b.GRES[(l - 1) * F1 + e] = gp;
                    }
                    __syncthreads();
                    gemm(d, lx, d, MA{th + oC, 1, d}, MB{gpre, 1, d}, MC{b.LAM, 1, d}, true);
                } else {
                    for (int e = tid; e < lx * d; e += T) b.LAM[e] = b.GX[e];
                }
                __syncthreads();
                // reverse scan along the snake row, one thread per unit
                for (int m = tid; m < d; m += T) {
                    float lam = 0.0f, znext = 0.0f;
                    for (int s1 = lx - 1; s1 >= 0; s1 -= 8) {
                        // operands of 8 sites (snake positions s1, s1-1, ...) first
                        float gl[8], zb[8], tb[8], hp[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int sidx = max(s1 - q, 0);
                            const int i = (j & 1) ? lx - 1 - sidx : sidx;
                            const int ip = (j & 1) ? lx - sidx : sidx - 1;   // snake predecessor
                            gl[q] = b.LAM[i * d + m];
                            zb[q] = Z[i * d + m];
                            tb[q] = HT[i * d + m];
                            hp[q] = (sidx > 0) ? Hh[ip * d + m] : 0.0f;
                        }
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int sidx = s1 - q;
                            if (sidx >= 0) {
                                const int i = (j & 1) ? lx - 1 - sidx : sidx;
                                lam = gl[q] + znext * lam;
                                const float z = zb[q];
                                const float gz = lam * (hp[q] - tb[q]);
                                ght[i * d + m] = lam * (1.0f - z);
                                gzp[i * d + m] = gz * z * (1.0f - z);
                                znext = z;
                            }
                        }
                    }
                }
                __syncthreads();
                // adjoints of the inputs: vertical (to row j-1) and, for l >= 1, the layer input
                const int64_t oWz = a.off[6 * l + 0], oWh = a.off[6 * l + 2];
                const bool vert = !G.chain && j > 0;
                if (vert) gemm(d, lx, d, MA{th + oWh + du, 1, ldh}, MB{ght, 1, d}, MC{gout + l * F1, 1, d}, false);
                if (l >= 1) {
                    const int64_t oD = a.off[6 * l + 5];
                    gemm(d, lx, d, MA{th + oWz, 1, du}, MB{gzp, 1, d}, MC{b.ROWIN, 1, d}, false);
                    gemm(d, lx, d, MA{th + oWh, 1, ldh}, MB{ght, 1, d}, MC{b.ROWIN, 1, d}, true);
                    gemm(d, lx, d, MA{th + oD, 1, du}, MB{gpre, 1, d}, MC{b.ROWIN, 1, d}, true);
                }
                __syncthreads();
                if (l >= 1) {
                    for (int e = tid; e < lx * d; e += T) b.GX[e] = b.ROWIN[e];
                    __syncthreads();
                }
            }
            cur = 1 - cur;
            __syncthreads();
        }

        // weight gradients of this chunk, added to the sample's row of O:
        // outer products summed over the chunk's sites (S of them, contiguous per layer)
        const int nrow = j1 - j0;
        const int S = nrow * lx;
        for (int l = 0; l < nl; ++l) {
            const int du = G.chain ? 2 : (l == 0 ? 4 : d);
            const int ldh = G.chain ? du : du + d;
            const int64_t oWz = a.off[6 * l + 0], obz = a.off[6 * l + 1], oWh = a.off[6 * l + 2],
                          obh = a.off[6 * l + 3];
            const int64_t L = cidx(a, 0, l);
            if (l >= 1) {
                // dW(m, k) = sum_s g(s, m) x(s, k), formed as its transpose so a lane's 4 results are contiguous
                gemm(d, d, S, MA{b.XIN + L, 1, d}, MB{b.GZP + L, d, 1}, MC{Orow + oWz, 1, du}, true);
                gemm(d, d, S, MA{b.XIN + L, 1, d}, MB{b.GHT + L, d, 1}, MC{Orow + oWh, 1, ldh}, true);
                gemm(d, d, S, MA{b.XIN + L, 1, d}, MB{b.GPRE + L, d, 1}, MC{Orow + a.off[6 * l + 5], 1, du}, true);
            } else {
                // one-hot layer-0 input (chain: previous spin): each site adds its
                // adjoints to the (at most two) input columns that are 1 there
                for (int m = tid; m < d; m += T) {
                    float gw[4] = {0.f, 0.f, 0.f, 0.f}, gz[4] = {0.f, 0.f, 0.f, 0.f}, gd[4] = {0.f, 0.f, 0.f, 0.f};
                    for (int e = 0; e < S; ++e) {
                        const int rr = e / lx, i = e - rr * lx;
                        const float vh = b.GHT[L + (int64_t)e * d + m], vz = b.GZP[L + (int64_t)e * d + m];
                        const float vp = G.chain ? 0.0f : b.GPRE[L + (int64_t)e * d + m];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            if (k < du && u0_val(G, w, j0 + rr, i, k) != 0.0f) {
                                gw[k] += vh;
                                gz[k] += vz;
                                gd[k] += vp;
                            }
                        }
                    }
                    for (int k = 0; k < du; ++k) {
                        Orow[oWh + (int64_t)m * ldh + k] += gw[k];
                        Orow[oWz + (int64_t)m * du + k] += gz[k];
                        if (!G.chain) Orow[a.off[6 * l + 5] + (int64_t)m * du + k] += gd[k];
                    }
                }
            }
            if (!G.chain) {
                gemm(d, d, S, MA{b.HV + L, 1, d}, MB{b.GHT + L, d, 1}, MC{Orow + oWh + du, 1, ldh}, true);
                gemm(d, d, S, MA{b.H + L, 1, d}, MB{b.GPRE + L, d, 1}, MC{Orow + a.off[6 * l + 4], 1, d}, true);
            }
            // biases
            for (int m = tid; m < d; m += T) {
                float sz = 0.0f, sh = 0.0f;
#pragma unroll 8
                for (int e = 0; e < S; ++e) {
                    sz += b.GZP[L + (int64_t)e * d + m];
                    sh += b.GHT[L + (int64_t)e * d + m];
                }
                Orow[obz + m] += sz;
                Orow[obh + m] += sh;
            }
            __syncthreads();
        }
        // head
        // head: per unit m both logits' rows (x computed once per site), then the biases
        {
            const int64_t Lh = cidx(a, 0, nl - 1);
            const int S = (j1 - j0) * lx;
            for (int m = tid; m < d; m += T) {
                float a0 = 0.0f, a1 = 0.0f;
#pragma unroll 4
                for (int e = 0; e < S; ++e) {
                    const float x = G.chain ? b.H[Lh + (int64_t)e * d + m] : gelu(b.PRE[Lh + (int64_t)e * d + m]);
                    a0 = fmaf(b.GLOG[e * 2], x, a0);
                    a1 = fmaf(b.GLOG[e * 2 + 1], x, a1);
                }
                Orow[oWo + m] += a0;
                Orow[oWo + d + m] += a1;
            }
            if (tid < 2) {
                float acc = 0.0f;
                for (int e = 0; e < S; ++e) acc += b.GLOG[e * 2 + tid];
                Orow[oWo + 2 * d + tid] += acc;
            }
        }
        __syncthreads();
    }
}

}  // namespace

BwdLayout bwd_layout(const Geom& g, int ckpt_rows) {
    BwdLayout bl;
    // default: about 128 sites per chunk (measured best or within 1 % of it at 10x10, 32x32, 52x52)
    int R = ckpt_rows > 0 ? ckpt_rows : (128 / g.lx > 1 ? 128 / g.lx : 1);
    if (R > g.ly) R = g.ly;
    bl.rows_per_chunk = R;
    bl.n_chunks = (g.ly + R - 1) / R;
    const int64_t F = (int64_t)g.nl * g.lx * g.d;
    bl.ws_per_sample_floats = bl.n_chunks * F + F + 9 * (int64_t)R * F + (int64_t)R * g.lx * 2 + 2 * F +
                              (int64_t)g.lx * g.d + F + (int64_t)g.lx * g.d + (int64_t)g.lx * 2 * g.d;
    bl.wt_floats = 0;
    return bl;
}

int launch_backward(const Geom& g, const BwdLayout& bl, const float* theta, const uint32_t* packed, int words,
                    int64_t B, float* wt, float* scratch, float* O, float* logpsi, hipStream_t st) {
    (void)wt;
    if (B == 0) return 0;
    BwdArgs a;
    a.g = g;
    a.R = bl.rows_per_chunk;
    a.nch = bl.n_chunks;
    a.theta = theta;
    int32_t nt = 0;
    param_offsets(g, a.off, &nt);
    a.packed = packed;
    a.words = words;
    a.B = B;
    a.P = a.off[nt];
    a.scratch = scratch;
    a.per_sample = bl.ws_per_sample_floats;
    a.O = O;
    a.logpsi = logpsi;
    bwd_kernel<<<(unsigned)B, 256, 0, st>>>(a);
    return (int)hipGetLastError();
}

}  // namespace psr
