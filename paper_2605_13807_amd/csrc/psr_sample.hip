// Exact autoregressive sampling of the 2D snake model and the chain, in step mode.
//
// The model is autoregressive (Sec. III.B): p(sigma) = prod_t p(sigma_t | sigma_<t)
// along the snake order of Sec. II.F, so an exact sample is drawn site by site:
// run every layer of the stacked 2D minGRU (Sec. II.F, II.G) at site t on the
// spins drawn so far, read p(sigma_t = 1 | sigma_<t) off the two-way softmax
// head, and set sigma_t = 1 iff u_t < p, with u_t a caller-supplied uniform.
// The recurrence is the same cell as the forward, evaluated one site at a time
// (no scan): h = z h_H + (1 - z) htilde with h_H the previous site of the row
// (zero at a row start) and h_V the row above (zero on the first row).
//
// One workgroup (8 waves) draws kS sequences.  Per site and layer the dense products are
// FP32 MFMA GEMMs with the kS sequences as the N dimension (psr_gemm.h), over
// the workgroup's workspace -- the row frontier FR[l][i] (h^(l) of the row above
// at column i) and the horizontal state HH[l] -- and over the activations X, Z,
// HT, PRE of the site ([d][kS] each, unit-major), which stay in LDS with the
// sampled spins of the current and the previous row.  Everything runs in FP32, whatever the model's
// precision.  The chain (one layer, input the one-hot previous spin, head on h)
// takes the same path with a one-site-high lattice, no vertical input and no
// output block.

#include <hip/hip_runtime.h>

#include "psr_gemm.h"
#include "psr_internal.h"

namespace psr {

namespace {

using namespace gemm_detail;

constexpr int kS = 16;          // sequences per workgroup (the GEMM N dimension)
constexpr int kMaxD = 256;      // largest model width
constexpr int kThreads = 512;      // 8 waves: one 16-unit output tile each at d = 128
constexpr int kLanesPerSeq = kThreads / kS;   // head: threads per sequence (a power of two <= 64)
static_assert(kLanesPerSeq <= 64 && (kLanesPerSeq & (kLanesPerSeq - 1)) == 0, "head lanes per sequence");

struct SampleArgs {
    Geom g;
    const float* theta;
    int64_t off[64];            // tensor offsets in theta
    const float* u;             // [B][N] uniforms in [0, 1), lattice row-major
    int64_t B;
    int8_t* spins;              // [B][N] out, lattice row-major
    float* logpsi;              // [B] out
    float* scratch;             // per_wg floats per workgroup
    int64_t per_wg;
};

__device__ inline float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }
__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
// log(1 + e^x) without overflow
__device__ inline float softplus(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }

__global__ void __launch_bounds__(kThreads) sample_kernel(const SampleArgs a) {
    const Geom& G = a.g;
    const int lx = G.lx, ly = G.ly, d = G.d, nl = G.nl, N = lx * ly;
    const int tid = threadIdx.x;
    const int64_t q0 = (int64_t)blockIdx.x * kS;
    const int DS = d * kS;
    float* FR = a.scratch + (int64_t)blockIdx.x * a.per_wg;   // [nl][lx][d][kS]
    float* HH = FR + (int64_t)nl * lx * DS;                    // [nl][d][kS]
    // the activations of the site being drawn stay in LDS ([d][kS] each)
    __shared__ float X[kMaxD * kS], Z[kMaxD * kS], HT[kMaxD * kS], PRE[kMaxD * kS];
    const float* th = a.theta;

    extern __shared__ int8_t sp[];   // [2][lx][kS]: spins of the previous and of the current row
    __shared__ double lsum[kS];
    if (tid < kS) lsum[tid] = 0.0;
    __syncthreads();

    int cur = 0;
    for (int j = 0; j < ly; ++j) {
        const int8_t* spv = sp + (1 - cur) * lx * kS;   // row j - 1
        int8_t* spc = sp + cur * lx * kS;               // row j
        for (int t = 0; t < lx; ++t) {
            const int i = (j & 1) ? lx - 1 - t : t;     // snake: odd rows run right to left
            const int ih = (j & 1) ? i + 1 : i - 1;     // horizontal predecessor
            const bool hp = t > 0, vp = j > 0;
            // ---- layer 0: u is (one-hot spin at H-pred, one-hot spin at V-pred), so its
            //      products are column gathers (chain: the one-hot previous spin only)
            if (G.chain) {
                const int64_t oWz = a.off[0], obz = a.off[1], oWh = a.off[2], obh = a.off[3];
                for (int e = tid; e < DS; e += kThreads) {
                    const int m = e / kS, n = e % kS;
                    float cz = th[obz + m], ch = th[obh + m];
                    if (hp) {
                        const int c = spc[ih * kS + n];
                        cz += th[oWz + m * 2 + c];
                        ch += th[oWh + m * 2 + c];
                    }
                    Z[e] = cz;
                    HT[e] = ch;
                }
            } else {
                const int64_t oWz = a.off[0], obz = a.off[1], oWh = a.off[2], obh = a.off[3], oD = a.off[5];
                for (int e = tid; e < DS; e += kThreads) {
                    const int m = e / kS, n = e % kS;
                    float cz = th[obz + m], ch = th[obh + m], cd = 0.0f;
                    if (hp) {
                        const int c = spc[ih * kS + n];
                        cz += th[oWz + m * 4 + c];
                        ch += th[oWh + (int64_t)m * (4 + d) + c];
                        cd += th[oD + m * 4 + c];
                    }
                    if (vp) {
                        const int c = 2 + spv[i * kS + n];
                        cz += th[oWz + m * 4 + c];
                        ch += th[oWh + (int64_t)m * (4 + d) + c];
                        cd += th[oD + m * 4 + c];
                    }
                    Z[e] = cz;
                    HT[e] = ch;
                    PRE[e] = cd;
                }
            }
            for (int l = 0; l < nl; ++l) {
                const int du = (l == 0) ? 4 : d;
                const int ldh = du + d;
                const int64_t oWz = a.off[6 * l], obz = a.off[6 * l + 1], oWh = a.off[6 * l + 2];
                const int64_t obh = a.off[6 * l + 3], oC = a.off[6 * l + 4], oD = a.off[6 * l + 5];
                float* fr = FR + ((int64_t)l * lx + i) * DS;   // h^(l) at column i: row j-1, then row j
                float* hh = HH + (int64_t)l * DS;
                if (l >= 1) {
                    // seeds: the biases, and the residual h^(l-1) of this site for l >= 2
                    const float* hb = HH + (int64_t)(l - 1) * DS;
                    for (int e = tid; e < DS; e += kThreads) {
                        const int m = e / kS;
                        Z[e] = th[obz + m];
                        HT[e] = th[obh + m];
                        PRE[e] = (l >= 2) ? hb[e] : 0.0f;
                    }
                    __syncthreads();
                    gemm_lds_b(d, kS, d, MA{th + oWz, du, 1}, MB{X, kS, 1}, MC{Z, kS, 1}, true);
                    gemm_lds_b(d, kS, d, MA{th + oWh, ldh, 1}, MB{X, kS, 1}, MC{HT, kS, 1}, true);
                    gemm_lds_b(d, kS, d, MA{th + oD, du, 1}, MB{X, kS, 1}, MC{PRE, kS, 1}, true);
                }
                if (vp) {
                    if (l == 0) __syncthreads();
                    gemm(d, kS, d, MA{th + oWh + du, ldh, 1}, MB{fr, kS, 1}, MC{HT, kS, 1}, true);
                }
                __syncthreads();
                // gate: h = z h_H + (1 - z) htilde; it is this row's frontier and the state
                // that the next site of the row reads as h_H
                for (int e = tid; e < DS; e += kThreads) {
                    const float z = sigm(Z[e]);
                    const float hH = hp ? hh[e] : 0.0f;
                    const float h = z * hH + (1.0f - z) * HT[e];
                    hh[e] = h;
                    fr[e] = h;
                }
                __syncthreads();
                if (G.chain) break;   // one layer; the head reads h
                // x^(l+1) = GELU(C h + D u + s)
                gemm(d, kS, d, MA{th + oC, d, 1}, MB{hh, kS, 1}, MC{PRE, kS, 1}, true);
                __syncthreads();
                for (int e = tid; e < DS; e += kThreads) X[e] = gelu(PRE[e]);
                __syncthreads();
            }
            // ---- head: logits = W_o x + b_o; kLanesPerSeq threads per sequence
            {
                const int n = tid / kLanesPerSeq, r = tid % kLanesPerSeq;
                const int ih0 = G.chain ? 4 : 6 * nl;   // index of W_o in the tensor list
                const int64_t oWo = a.off[ih0], obo = a.off[ih0 + 1];
                const float* xo = G.chain ? HH : X;    // chain: the head reads h
                float l0 = 0.0f, l1 = 0.0f;
                for (int m = r; m < d; m += kLanesPerSeq) {
                    const float x = xo[m * kS + n];
                    l0 = fmaf(th[oWo + m], x, l0);
                    l1 = fmaf(th[oWo + d + m], x, l1);
                }
#pragma unroll
                for (int w = kLanesPerSeq / 2; w >= 1; w >>= 1) {
                    l0 += __shfl_xor(l0, w, kLanesPerSeq);
                    l1 += __shfl_xor(l1, w, kLanesPerSeq);
                }
                if (r == 0) {
                    const float dl = (l0 + th[obo]) - (l1 + th[obo + 1]);   // logit(0) - logit(1)
                    const float p1 = 1.0f / (1.0f + expf(dl));              // p(sigma_t = 1 | sigma_<t)
                    const int64_t q = q0 + n;
                    int s = 0;
                    if (q < a.B) {
                        const int site = j * lx + i;
                        s = (a.u[q * N + site] < p1) ? 1 : 0;
                        a.spins[q * N + site] = (int8_t)s;
                        // log p(sigma_t) = -softplus(logit(other) - logit(own))
                        lsum[n] += (double)(-softplus(s ? dl : -dl));
                    }
                    spc[i * kS + n] = (int8_t)s;
                }
            }
            __syncthreads();
        }
        cur = 1 - cur;
    }
    if (tid < kS && q0 + tid < a.B) a.logpsi[q0 + tid] = (float)(0.5 * lsum[tid]);
}

}  // namespace

int64_t sample_ws_per_wg_floats(const Geom& g) {
    const int64_t DS = (int64_t)g.d * kS;
    return (int64_t)g.nl * g.lx * DS + (int64_t)g.nl * DS;
}

int64_t sample_groups(int64_t B) { return (B + kS - 1) / kS; }

int launch_sample(const Geom& g, const float* theta, const float* u, int64_t B, int8_t* spins, float* logpsi,
                  float* scratch, hipStream_t st) {
    if (B == 0) return 0;
    SampleArgs a;
    a.g = g;
    a.theta = theta;
    int32_t nt = 0;
    param_offsets(g, a.off, &nt);
    a.u = u;
    a.B = B;
    a.spins = spins;
    a.logpsi = logpsi;
    a.scratch = scratch;
    a.per_wg = sample_ws_per_wg_floats(g);
    const size_t lds = (size_t)2 * g.lx * kS;
    hipLaunchKernelGGL(sample_kernel, dim3((unsigned)sample_groups(B)), dim3(kThreads), lds, st, a);
    return (int)hipGetLastError();
}

}  // namespace psr
