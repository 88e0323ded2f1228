// log psi of the 1D LRU ansatz (Sec. II.B, Eq. (lru); residual with GLU, Sec. II.G).
//
// Per layer, with the layer input x_t in R^d at every site t of the chain:
//   lambda = exp(-e^nu + i e^theta),  h_t = lambda h_{t-1} + e^gamma (B x_t),  h_{-1} = 0,
//   y_t = Re(C h_t) + D x_t,  x'_t = (W_a y_t + b_a) sigmoid(W_g y_t + b_g) + [l >= 1] x_t.
// The layer-0 input at site t is the embedding E[:, sigma_{t-1}] (zero at t = 0),
// and the head is a two-way softmax on the last layer's output; log psi is half
// the sum of the sites' log p (Sec. III.B).
//
// One workgroup (8 waves) takes S sequences at a time, S N columns (S = 256 / N
// for short chains, else 1).  The activations of the group live in the
// workgroup's workspace, unit-major ([units][columns]):
//   * drive:   U = [B_re; B_im] X                 one FP32 MFMA GEMM, M = 2 d_h
//   * scan:    the recurrence is linear with a constant diagonal coefficient, so
//              each (sequence, unit) is cut into chunks that are scanned from a
//              zero state in parallel; the chunks' end states are chained with
//              lambda^len, and every element then gets lambda^(t - t0 + 1) times
//              its chunk's carry (Sec. II.B: the LRU hidden states by a parallel scan)
//   * output:  Y = D x + C_re h_re + C_im (-h_im)      two GEMM passes, K = d_h each
//   * GLU:     G = W_glu Y + b_glu                     one GEMM, M = 2 d
//   * gate, residual, then the head and a per-sequence FP64 sum.
// Every step runs in FP32; the GEMMs are the dense part of the layer.

#include <hip/hip_runtime.h>

#include "psr_gemm.h"
#include "psr_internal.h"

namespace psr {

namespace {

using namespace gemm_detail;

constexpr int kThreads = 512;
constexpr int kColTarget = 256;     // columns per group for short chains
constexpr int kR = 32;              // longest scan chunk held in registers
constexpr int kB = 8;               // elementwise loops: loads in flight per thread
constexpr int kXYLds = 2 * 64 * 256;  // floats of LDS for X and Y (128 KB)
constexpr int64_t kMaxGroupsInFlight = 1024;

struct LruArgs {
    LruGeom g;
    const float* theta;
    const int8_t* spins;   // [B][N]
    int64_t B;
    int S;                 // sequences per group
    int64_t groups;
    float* logpsi;         // [B] (log psi, or its high part when logpsi_lo is set)
    float* logpsi_lo;      // [B] low part (log psi = hi + lo, the sum kept in FP64) or null
    float* logp_site;      // [B][N] or null
    float* scratch;
    int64_t per_wg;        // floats of workspace per workgroup
};

__device__ inline float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }
__device__ inline float softplus(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }

// C (+)= A B with A [M][K] (row stride lda; weights), B [K][ldb] and C [M][ldc] (workspace),
// for K <= 4 kKQ.  A wave keeps the A fragment of its 16 output rows in registers
// (K/4 floats a lane) across all of its column tiles, and issues the next tile's B
// loads before the current tile's MFMAs.  Lane layout of the FP32 16x16x4 MFMA: a
// lane holds A(m0 + lane%16, 4j + lane/16), B(4j + lane/16, n0 + lane%16) and
// outputs rows m0 + 4 (lane/16) + i of column n0 + lane%16.  M is a multiple of 16;
// N is masked (columns past N read column N - 1 and are not stored).  With dseed,
// C = dseed[row] xseed(row, n) + A B (xseed with C's strides).  Called by the whole
// workgroup; no barrier inside.
constexpr int kKQ = 16;
__device__ inline void gemm_ws(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C,
                               int ldc, bool acc_in, const float* dseed = nullptr, const float* xseed = nullptr) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int kq = lane >> 4, r16 = lane & 15;
    const int tm = M >> 4, tn = (N + 15) >> 4, KQ = K >> 2;
    // waves -> tiles: with at least nw row tiles a wave takes every nw-th row tile and all
    // column tiles; with fewer, nw / tm waves share a row tile and split its column tiles
    int mt0 = wave, mstep = nw, nt0 = 0, nstep = 1;
    if (tm < nw) {
        const int wpm = nw / tm;
        mt0 = wave / wpm;
        mstep = nw;
        nt0 = wave % wpm;
        nstep = wpm;
    }
    for (int mt = mt0; mt < tm; mt += mstep) {
        const int m0 = mt << 4;
        float af[kKQ];
        const float* ap = A + (int64_t)(m0 + r16) * lda + kq;
#pragma unroll
        for (int j = 0; j < kKQ; ++j) af[j] = (j < KQ) ? ap[4 * j] : 0.0f;
        float bc[kKQ], bn[kKQ];
        auto loadb = [&](int nt, float* b) {
            const int n = min((nt << 4) + r16, N - 1);
            const float* bp = B + (int64_t)kq * ldb + n;
#pragma unroll
            for (int j = 0; j < kKQ; ++j) b[j] = (j < KQ) ? bp[(int64_t)4 * j * ldb] : 0.0f;
        };
        if (nt0 < tn) loadb(nt0, bc);
        for (int nt = nt0; nt < tn; nt += nstep) {
            if (nt + nstep < tn) loadb(nt + nstep, bn);
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < kKQ; ++j)
                if (j < KQ) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[j], bc[j], acc, 0, 0, 0);
            const int n = (nt << 4) + r16;
            if (n < N) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = m0 + 4 * kq + i;
                    float* cp = C + (int64_t)row * ldc + n;
                    if (dseed)   // C = dseed[row] * xseed(row, n) + A B
                        *cp = fmaf(dseed[row], xseed[(int64_t)row * ldc + n], acc[i]);
                    else
                        *cp = acc_in ? *cp + acc[i] : acc[i];
                }
            }
#pragma unroll
            for (int j = 0; j < kKQ; ++j) bc[j] = bn[j];
        }
    }
}

// GLU fused with its projections and the residual, for d <= 4 kKQ:
//   X(m, n) = [res] X(m, n) + (W_a y + b_a)(m, n) sigmoid(W_g y + b_g)(m, n),
// W = [W_a; W_g] ([2 d][d]), b = [b_a; b_g], y = Y ([d][ldb]).  A wave computes the value
// and the gate tile of the same 16 rows, so the gate is applied in registers (no B
// prefetch here: it measured no faster and spilled registers).  X is only touched at
// the element each lane writes (Y is the B operand).  Whole workgroup.
__device__ inline void gemm_glu_ws(int d, int N, const float* W, const float* b, const float* Y, int ldb, float* X,
                                   int ldc, bool res) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int kq = lane >> 4, r16 = lane & 15;
    const int tm = d >> 4, tn = (N + 15) >> 4, KQ = d >> 2;
    int mt0 = wave, mstep = nw, nt0 = 0, nstep = 1;
    if (tm < nw) {
        const int wpm = nw / tm;
        mt0 = wave / wpm;
        nt0 = wave % wpm;
        nstep = wpm;
    }
    for (int mt = mt0; mt < tm; mt += mstep) {
        const int m0 = mt << 4;
        float av[kKQ], ag[kKQ];
        const float* pv = W + (int64_t)(m0 + r16) * d + kq;
        const float* pg = pv + (int64_t)d * d;
#pragma unroll
        for (int j = 0; j < kKQ; ++j) {
            av[j] = (j < KQ) ? pv[4 * j] : 0.0f;
            ag[j] = (j < KQ) ? pg[4 * j] : 0.0f;
        }
        float bc[kKQ];
        auto loadb = [&](int nt, float* bb) {
            const int n = min((nt << 4) + r16, N - 1);
            const float* bp = Y + (int64_t)kq * ldb + n;
#pragma unroll
            for (int j = 0; j < kKQ; ++j) bb[j] = (j < KQ) ? bp[(int64_t)4 * j * ldb] : 0.0f;
        };
        for (int nt = nt0; nt < tn; nt += nstep) {
            loadb(nt, bc);
            f32x4 accv = {0.f, 0.f, 0.f, 0.f}, accg = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < kKQ; ++j)
                if (j < KQ) {
                    accv = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j], bc[j], accv, 0, 0, 0);
                    accg = __builtin_amdgcn_mfma_f32_16x16x4f32(ag[j], bc[j], accg, 0, 0, 0);
                }
            const int n = (nt << 4) + r16;
            if (n < N) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = m0 + 4 * kq + i;
                    float* xp = X + (int64_t)row * ldc + n;
                    const float v = (accv[i] + b[row]) * sigm(accg[i] + b[d + row]);
                    *xp = res ? *xp + v : v;
                }
            }
        }
    }
}

// the weights-stationary GEMM where K fits its registers, the general one otherwise
__device__ inline void gemm_lru(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C,
                                int ldc, bool acc_in) {
    if (K <= 4 * kKQ)
        gemm_ws(M, N, K, A, lda, B, ldb, C, ldc, acc_in);
    else
        gemm(M, N, K, MA{A, lda, 1}, MB{B, ldb, 1}, MC{C, ldc, 1}, acc_in);
}

// scan phase 2: the carry into chunk c of item it (unit it % dh) is the state after
// chunk c - 1; lambda^len in closed form, exp(-len e^nu) (cos, sin)(len e^theta), chains
// the chunks' end states.  Called by the whole workgroup; no barrier inside.
__device__ inline void lru_carries(const float* nu, const float* ph, int dh, int items, int nch, int Lc, int N,
                                   const float2* endst, float2* carry) {
    for (int it = threadIdx.x; it < items; it += kThreads) {
        const int u = it % dh;
        const float a_ = expf(nu[u]), b_ = expf(ph[u]);
        float cr = 0.0f, ci = 0.0f;
        for (int c = 0; c < nch; ++c) {
            carry[c * items + it] = make_float2(cr, ci);
            const int t0 = c * Lc, len = max(0, min(N, t0 + Lc) - t0);
            const float mag = expf(-(float)len * a_);
            float sn, cs;
            sincosf((float)len * b_, &sn, &cs);
            const float pr = mag * cs, pi = mag * sn;
            const float2 e = endst[c * items + it];
            const float nr = pr * cr - pi * ci + e.x;
            const float ni = pr * ci + pi * cr + e.y;
            cr = nr;
            ci = ni;
        }
    }
}

// XY_LDS: the layer input X and the output map's result Y live in LDS (the fused
// path for d, d_h <= 4 kKQ with 2 d S N <= kXYLds); otherwise in the workspace.
template <bool XY_LDS>
__global__ void __launch_bounds__(kThreads) lru_kernel(const LruArgs a) {
    const LruGeom& G = a.g;
    const int N = G.n, d = G.d, dh = G.dh, nl = G.nl, S = a.S;
    const int cols = S * N;
    const int tid = threadIdx.x;
    float* Xg = a.scratch + (int64_t)blockIdx.x * a.per_wg;  // [d][cols]
    float* U = Xg + (int64_t)d * cols;                         // [2 dh][cols]
    float* Yg = U + (int64_t)2 * dh * cols;                    // [d][cols]
    float* GL = Yg + (int64_t)d * cols;                        // [2 d][cols]
    float* X = Xg;
    float* Y = Yg;
    if constexpr (XY_LDS) {
        __shared__ float xy[kXYLds];
        X = xy;
        Y = xy + d * cols;
    }
    const float* th = a.theta;
    const int64_t lstride = lru_layer_floats(G);
    const float* Wo = th + (int64_t)2 * d + nl * lstride;
    const float* bo = Wo + 2 * d;

    __shared__ float2 endst[kThreads], carry[kThreads];
    __shared__ double red[kThreads];

    // chunks per (sequence, unit) of the scan; items * nch <= kThreads when nch > 1
    const int items = dh * S;
    const int nch = items >= kThreads ? 1 : min(N, kThreads / items);
    const int Lc = (N + nch - 1) / nch;

    for (int64_t grp = blockIdx.x; grp < a.groups; grp += gridDim.x) {
        const int64_t q0 = grp * S;
        // layer-0 input: E[:, sigma_{t-1}], zero at t = 0 and for sequences past B
        for (int e0 = tid; e0 < d * cols; e0 += kB * kThreads) {
            float xv[kB];
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                const int e = e0 + k * kThreads;
                const int m = e / cols, col = e - m * cols;
                const int s = col / N, t = col - s * N;
                const int64_t q = q0 + s;
                xv[k] = (e < d * cols && t > 0 && q < a.B) ? th[m * 2 + (a.spins[q * N + t - 1] & 1)] : 0.0f;
            }
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                const int e = e0 + k * kThreads;
                if (e < d * cols) X[e] = xv[k];
            }
        }
        __syncthreads();
        for (int l = 0; l < nl; ++l) {
            const float* Lp = th + (int64_t)2 * d + l * lstride;
            const float* nu = Lp;
            const float* ph = Lp + dh;
            const float* gm = Lp + 2 * dh;
            const float* Bm = Lp + 3 * dh;                 // [2 dh][d]
            const float* Dv = Bm + (int64_t)2 * dh * d;    // [d]
            const float* Cm = Dv + d;                      // [d][2 dh]
            const float* Wg = Cm + (int64_t)2 * dh * d;    // [2 d][d]
            const float* bg = Wg + (int64_t)2 * d * d;     // [2 d]
            // drive B x (the e^gamma scale is applied in the scan)
            gemm_lru(2 * dh, cols, d, Bm, d, X, cols, U, cols, false);
            __syncthreads();
            if (Lc <= kR) {
                // chunks of at most kR sites: each is loaded in one burst, scanned in
                // registers and, with several chunks, kept there across the carry step
                // (then items * nch <= kThreads: one chunk per thread, one pass)
                const int nwork = items * nch;
                for (int w0 = 0; w0 < nwork; w0 += kThreads) {
                    const int w = w0 + tid;
                    const bool mine = w < nwork;
                    float vr[kR], vi[kR];
                    float lr = 0.0f, li = 0.0f;
                    int len = 0;
                    float* ur = U;
                    float* ui = U;
                    if (mine) {
                        const int it = w % items, c = w / items;
                        const int u = it % dh, s = it / dh;
                        const int t0 = c * Lc;
                        len = max(0, min(N, t0 + Lc) - t0);
                        const float mag = expf(-expf(nu[u]));
                        float sn, cs;
                        sincosf(expf(ph[u]), &sn, &cs);
                        lr = mag * cs;
                        li = mag * sn;
                        const float gg = expf(gm[u]);
                        ur = U + (int64_t)u * cols + s * N + t0;
                        ui = U + (int64_t)(dh + u) * cols + s * N + t0;
#pragma unroll
                        for (int j = 0; j < kR; ++j) {
                            vr[j] = (j < len) ? ur[j] : 0.0f;
                            vi[j] = (j < len) ? ui[j] : 0.0f;
                        }
                        float hr = 0.0f, hi = 0.0f;
#pragma unroll
                        for (int j = 0; j < kR; ++j) {
                            const float nr = fmaf(lr, hr, fmaf(-li, hi, gg * vr[j]));
                            const float ni = fmaf(lr, hi, fmaf(li, hr, gg * vi[j]));
                            hr = (j < len) ? nr : hr;
                            hi = (j < len) ? ni : hi;
                            vr[j] = hr;
                            vi[j] = hi;
                        }
                        if (nch > 1) endst[w] = make_float2(hr, hi);
                    }
                    if (nch > 1) {
                        __syncthreads();
                        lru_carries(nu, ph, dh, items, nch, Lc, N, endst, carry);
                        __syncthreads();
                        if (mine) {
                            const float2 cin = carry[w];
                            float pr = lr, pi = li;
#pragma unroll
                            for (int j = 0; j < kR; ++j) {
                                vr[j] += pr * cin.x - pi * cin.y;
                                vi[j] += pr * cin.y + pi * cin.x;
                                const float np = pr * lr - pi * li;
                                pi = pr * li + pi * lr;
                                pr = np;
                            }
                        }
                    }
                    if (mine) {
#pragma unroll
                        for (int j = 0; j < kR; ++j)
                            if (j < len) {
                                ur[j] = vr[j];
                                ui[j] = -vi[j];
                            }
                    }
                }
            } else {
            // scan, phase 1: every chunk from a zero state
            for (int w = tid; w < items * nch; w += kThreads) {
                const int it = w % items, c = w / items;
                const int u = it % dh, s = it / dh;
                const int t0 = c * Lc, t1 = min(N, t0 + Lc);
                const float mag = expf(-expf(nu[u]));
                float sn, cs;
                sincosf(expf(ph[u]), &sn, &cs);
                const float lr = mag * cs, li = mag * sn, gg = expf(gm[u]);
                float* ur = U + (int64_t)u * cols + s * N;
                float* ui = U + (int64_t)(dh + u) * cols + s * N;
                float hr = 0.0f, hi = 0.0f;
                for (int t = t0; t < t1; ++t) {
                    const float nr = fmaf(lr, hr, fmaf(-li, hi, gg * ur[t]));
                    const float ni = fmaf(lr, hi, fmaf(li, hr, gg * ui[t]));
                    hr = nr;
                    hi = ni;
                    ur[t] = hr;
                    ui[t] = (nch == 1) ? -hi : hi;   // one chunk: final, -Im for the output GEMM
                }
                if (nch > 1) endst[w] = make_float2(hr, hi);
            }
            if (nch > 1) {
                __syncthreads();
                lru_carries(nu, ph, dh, items, nch, Lc, N, endst, carry);
                __syncthreads();
                // phase 3: h_t += lambda^(t - t0 + 1) carry
                for (int w = tid; w < items * nch; w += kThreads) {
                    const int it = w % items, c = w / items;
                    const int u = it % dh, s = it / dh;
                    const int t0 = c * Lc, t1 = min(N, t0 + Lc);
                    const float mag = expf(-expf(nu[u]));
                    float sn, cs;
                    sincosf(expf(ph[u]), &sn, &cs);
                    const float lr = mag * cs, li = mag * sn;
                    const float2 cin = carry[w];
                    float* ur = U + (int64_t)u * cols + s * N;
                    float* ui = U + (int64_t)(dh + u) * cols + s * N;
                    float pr = lr, pi = li;
                    for (int t = t0; t < t1; ++t) {
                        ur[t] += pr * cin.x - pi * cin.y;
                        ui[t] = -(ui[t] + pr * cin.y + pi * cin.x);
                        const float np = pr * lr - pi * li;
                        pi = pr * li + pi * lr;
                        pr = np;
                    }
                }
            }
            }
            if (XY_LDS || (d <= 4 * kKQ && dh <= 4 * kKQ)) {
                // y = D x + C_re h_re + C_im (-h_im): the seed in the first pass's epilogue,
                // the second pass accumulating (both give an element to the same lane);
                // the barrier orders the scan's stores of h before the passes read them
                __syncthreads();
                gemm_ws(d, cols, dh, Cm, 2 * dh, U, cols, Y, cols, false, Dv, X);
                gemm_ws(d, cols, dh, Cm + dh, 2 * dh, U + (int64_t)dh * cols, cols, Y, cols, true);
                __syncthreads();
                gemm_glu_ws(d, cols, Wg, bg, Y, cols, X, cols, l >= 1);
                __syncthreads();
            } else if constexpr (!XY_LDS) {
                // seeds: y = D x, and the GLU biases (loads in batches of kB, then the stores)
                for (int e0 = tid; e0 < d * cols; e0 += kB * kThreads) {
                    float xv[kB], dv[kB];
#pragma unroll
                    for (int k = 0; k < kB; ++k) {
                        const int e = e0 + k * kThreads;
                        xv[k] = (e < d * cols) ? X[e] : 0.0f;
                        dv[k] = (e < d * cols) ? Dv[e / cols] : 0.0f;
                    }
#pragma unroll
                    for (int k = 0; k < kB; ++k) {
                        const int e = e0 + k * kThreads;
                        if (e < d * cols) Y[e] = dv[k] * xv[k];
                    }
                }
                for (int e0 = tid; e0 < 2 * d * cols; e0 += kB * kThreads) {
                    float bv[kB];
#pragma unroll
                    for (int k = 0; k < kB; ++k) {
                        const int e = e0 + k * kThreads;
                        bv[k] = (e < 2 * d * cols) ? bg[e / cols] : 0.0f;
                    }
#pragma unroll
                    for (int k = 0; k < kB; ++k) {
                        const int e = e0 + k * kThreads;
                        if (e < 2 * d * cols) GL[e] = bv[k];
                    }
                }
                __syncthreads();
                // y += Re(C h) = C_re h_re + C_im (-h_im), one pass per half of C's columns (the
                // two passes give each output element to the same lane, in this order)
                gemm_lru(d, cols, dh, Cm, 2 * dh, U, cols, Y, cols, true);
                gemm_lru(d, cols, dh, Cm + dh, 2 * dh, U + (int64_t)dh * cols, cols, Y, cols, true);
                __syncthreads();
                gemm_lru(2 * d, cols, d, Wg, d, Y, cols, GL, cols, true);
                __syncthreads();
                // GLU and the residual (from the second layer on), loads in batches of kB
                for (int e0 = tid; e0 < d * cols; e0 += kB * kThreads) {
                    float gv[kB], gg[kB], xv[kB];
#pragma unroll
                    for (int k = 0; k < kB; ++k) {
                        const int e = e0 + k * kThreads;
                        const bool in = e < d * cols;
                        gv[k] = in ? GL[e] : 0.0f;
                        gg[k] = in ? GL[e + (int64_t)d * cols] : 0.0f;
                        xv[k] = (in && l >= 1) ? X[e] : 0.0f;
                    }
#pragma unroll
                    for (int k = 0; k < kB; ++k) {
                        const int e = e0 + k * kThreads;
                        if (e < d * cols) X[e] = xv[k] + gv[k] * sigm(gg[k]);
                    }
                }
                __syncthreads();
            }
        }
        // head: logit(0) - logit(1) per column; log p of the own spin into GL's first row
        for (int col = tid; col < cols; col += kThreads) {
            const int s = col / N, t = col - s * N;
            const int64_t q = q0 + s;
            float dl = bo[0] - bo[1];
            for (int m = 0; m < d; ++m) dl = fmaf(Wo[m] - Wo[d + m], X[(int64_t)m * cols + col], dl);
            float lp = 0.0f;
            if (q < a.B) {
                const int own = a.spins[q * N + t] & 1;
                lp = -softplus(own ? dl : -dl);
                if (a.logp_site) a.logp_site[q * N + t] = lp;
            }
            GL[col] = lp;
        }
        __syncthreads();
        if (S == 1) {
            double acc = 0.0;
            for (int t = tid; t < N; t += kThreads) acc += (double)GL[t];
            red[tid] = acc;
            __syncthreads();
            for (int w = kThreads / 2; w >= 1; w >>= 1) {
                if (tid < w) red[tid] += red[tid + w];
                __syncthreads();
            }
            if (tid == 0 && q0 < a.B) {
                const float hi = (float)(0.5 * red[0]);
                a.logpsi[q0] = hi;
                if (a.logpsi_lo) a.logpsi_lo[q0] = (float)(0.5 * red[0] - (double)hi);
            }
        } else if (tid < S && q0 + tid < a.B) {
            double acc = 0.0;
            for (int t = 0; t < N; ++t) acc += (double)GL[tid * N + t];
            const float hi = (float)(0.5 * acc);
            a.logpsi[q0 + tid] = hi;
            if (a.logpsi_lo) a.logpsi_lo[q0 + tid] = (float)(0.5 * acc - (double)hi);
        }
        __syncthreads();   // the next group overwrites the workspace
    }
}

// E_loc(s) = diag(s) + sum_{k < n_conn(s)} mel(s, k) exp(log psi(sigma'_k) - log psi(sigma_s))
// with the connected entries in per-sample slots (s * max_conn + k).  Both log psi
// are (hi, lo) pairs of FP64 sums, so the prefix a flip leaves unchanged (bitwise
// equal site terms) cancels in the difference.  One wave per sample, FP64
// accumulation in a fixed order.
__global__ void lru_eloc_kernel(int64_t B, int64_t max_conn, const int32_t* __restrict__ n_conn,
                                const float* __restrict__ diag, const float* __restrict__ mel,
                                const float* __restrict__ lpc, const float* __restrict__ lpc_lo,
                                const float* __restrict__ lps, const float* __restrict__ lps_lo,
                                double* __restrict__ eloc) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (s >= B) return;
    const int64_t base = s * max_conn;
    const int nc = n_conn[s];
    const double l0 = (double)lps[s] + (double)lps_lo[s];
    double acc = 0.0;
    for (int k = lane; k < nc; k += 64)
        acc += (double)mel[base + k] * exp(((double)lpc[base + k] - l0) + (double)lpc_lo[base + k]);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) eloc[s] = (double)diag[s] + acc;
}

int lru_seqs_per_group(const LruGeom& g) { return g.n >= kColTarget ? 1 : kColTarget / g.n; }

int64_t lru_per_wg_floats(const LruGeom& g) {
    const int64_t cols = (int64_t)lru_seqs_per_group(g) * g.n;
    return ((int64_t)4 * g.d + (int64_t)2 * g.dh) * cols;
}

int64_t lru_grid(const LruGeom& g, int64_t B) {
    const int S = lru_seqs_per_group(g);
    const int64_t groups = (B + S - 1) / S;
    // at most kMaxGroupsInFlight workgroups, fewer when a group's workspace is large
    // (but never fewer than one per compute unit)
    const int64_t by_mem = ((int64_t)1 << 30) / (lru_per_wg_floats(g) * (int64_t)sizeof(float));
    int64_t cap = by_mem < kMaxGroupsInFlight ? by_mem : kMaxGroupsInFlight;
    if (cap < 256) cap = 256;
    return groups < cap ? groups : cap;
}

}  // namespace

int64_t lru_param_count(const LruGeom& g) {
    return (int64_t)2 * g.d + g.nl * lru_layer_floats(g) + (int64_t)2 * g.d + 2;
}

int64_t lru_workspace_floats(const LruGeom& g, int64_t B) {
    if (B <= 0) return 0;
    return lru_grid(g, B) * lru_per_wg_floats(g);
}

int launch_lru_eloc_combine(int64_t B, int64_t max_conn, const int32_t* n_conn, const float* diag, const float* mel,
                            const float* lpc, const float* lpc_lo, const float* lps, const float* lps_lo, double* eloc,
                            hipStream_t st) {
    if (B == 0) return 0;
    lru_eloc_kernel<<<(unsigned)((B + 3) / 4), 256, 0, st>>>(B, max_conn, n_conn, diag, mel, lpc, lpc_lo, lps, lps_lo,
                                                             eloc);
    return (int)hipGetLastError();
}

int launch_lru_logpsi(const LruGeom& g, const float* theta, const int8_t* spins, int64_t B, float* logpsi,
                      float* logpsi_lo, float* logp_site, float* scratch, hipStream_t st) {
    if (B == 0) return 0;
    LruArgs a;
    a.g = g;
    a.theta = theta;
    a.spins = spins;
    a.B = B;
    a.S = lru_seqs_per_group(g);
    a.groups = (B + a.S - 1) / a.S;
    a.logpsi = logpsi;
    a.logpsi_lo = logpsi_lo;
    a.logp_site = logp_site;
    a.scratch = scratch;
    a.per_wg = lru_per_wg_floats(g);
    const bool xy_lds = g.d <= 4 * kKQ && g.dh <= 4 * kKQ && (int64_t)2 * g.d * a.S * g.n <= kXYLds;
    if (xy_lds)
        hipLaunchKernelGGL(lru_kernel<true>, dim3((unsigned)lru_grid(g, B)), dim3(kThreads), 0, st, a);
    else
        hipLaunchKernelGGL(lru_kernel<false>, dim3((unsigned)lru_grid(g, B)), dim3(kThreads), 0, st, a);
    return (int)hipGetLastError();
}

}  // namespace psr
