// Exact sampler and per-sample gradients of the 1D LRU ansatz (Sec. II.B Eq. (lru),
// Sec. II.G residual with GLU, Sec. III.B autoregressive sampling and VMC gradient).
//
// Per layer l with input x_t in R^d (layer 0: the embedding E[:, sigma_{t-1}],
// zero at t = 0):
//   v_t = e^gamma (B x_t)                 complex drive, B = B_re + i B_im
//   h_t = lambda h_{t-1} + v_t,           lambda = exp(-e^nu + i e^theta), h_{-1} = 0
//   y_t = Re(C h_t) + D x_t = C_re h_re - C_im h_im + D x_t
//   x'_t = a_t s_t + [l >= 1] x_t,        a = W_a y + b_a, s = sigmoid(W_g y + b_g)
// then logits W_o x + b_o and log psi = 1/2 sum_t log p(sigma_t | sigma_<t).
//
// Both kernels give one workgroup to one chain at a time (a grid-stride loop
// over the batch), in FP32 with FP32 accumulation (sums over the chain's sites).
//
// Sampler: sites one after the other (each conditional needs the spins before
// it); per site and layer the drive, the recurrence step, the output map and
// the GLU are matrix-vector products over the workgroup's threads, with the
// complex state h of every layer kept in LDS.
//
// Backward: the forward over the whole chain is recomputed and every layer's
// x, v, h, y, a and s are kept in the chain's workspace.  The reverse pass
// then goes layer by layer:
//   da = dx' s, dg = dx' a s (1 - s)         dW_a += da y^T, dW_g += dg y^T
//   dy = W_a^T da + W_g^T dg                  dD += dy x, dC_re += dy h_re^T, dC_im -= dy h_im^T
//   G_t = (C_re^T dy_t) - i (C_im^T dy_t)     the adjoint of h_t from y_t
//   Ghat_t = G_t + conj(lambda) Ghat_{t+1}    the reverse scan of the recurrence
//   dlambda = sum_t Ghat_t conj(h_{t-1}),     dnu = Re(conj(dlambda) (-e^nu lambda)),
//                                             dtheta = Re(conj(dlambda) (i e^theta lambda))
//   dgamma = sum_t Re(conj(Ghat_t) v_t),      dB_re += e^gamma Ghat_re x^T, dB_im += e^gamma Ghat_im x^T
//   dx = D dy + [l >= 1] dx' + B_re^T (e^gamma Ghat_re) + B_im^T (e^gamma Ghat_im)
// and finally dE from the layer-0 adjoint.  The weight gradients are written
// straight into the chain's row of O (the layout of the parameters).
#include "psr_internal.h"

namespace psr {
namespace {

constexpr int kT = 256;   // threads of a workgroup

// theta offsets of one layer's tensors
struct LruOff {
    int64_t nu, th, ga, B, D, C, W, b;
};

__host__ __device__ inline LruOff lru_layer_off(const LruGeom& g, int l) {
    const int64_t d = g.d, dh = g.dh;
    LruOff o;
    o.nu = 2 * d + (int64_t)l * lru_layer_floats(g);
    o.th = o.nu + dh;
    o.ga = o.th + dh;
    o.B = o.ga + dh;
    o.D = o.B + 2 * dh * d;
    o.C = o.D + d;
    o.W = o.C + d * 2 * dh;
    o.b = o.W + 2 * d * d;
    return o;
}
__host__ __device__ inline int64_t lru_head_off(const LruGeom& g) { return 2 * (int64_t)g.d + g.nl * lru_layer_floats(g); }

// Prepared per-layer values shared by all chains: transposed matrices (so that
// a thread per output reads consecutive addresses), lambda and e^gamma.
struct LruPrep {
    int64_t Bt, Ct, Wt;   // [l][d][2 dh], [l][2 dh][d], [l][d][2 d]
    int64_t lam, eg;      // [l][dh][2] (re, im), [l][dh]
    int64_t floats;
};

__host__ __device__ inline LruPrep lru_prep_layout(const LruGeom& g) {
    const int64_t d = g.d, dh = g.dh, L = g.nl;
    LruPrep p;
    int64_t t = 0;
    p.Bt = t; t += L * d * 2 * dh;
    p.Ct = t; t += L * 2 * dh * d;
    p.Wt = t; t += L * d * 2 * d;
    p.lam = t; t += L * dh * 2;
    p.eg = t; t += L * dh;
    p.floats = t;
    return p;
}

__global__ void lru_prep_kernel(const float* __restrict__ theta, LruGeom g, float* __restrict__ pw) {
    const LruPrep P = lru_prep_layout(g);
    const int d = g.d, dh = g.dh;
    const int64_t per = (int64_t)2 * dh * d + 2 * dh * d + 2 * d * d + 3 * dh;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= per * g.nl) return;
    const int l = (int)(e / per);
    int64_t r = e % per;
    const LruOff o = lru_layer_off(g, l);
    if (r < (int64_t)2 * dh * d) {   // B[k][j] -> Bt[j][k]
        const int k = (int)(r / d), j = (int)(r % d);
        pw[P.Bt + (int64_t)l * d * 2 * dh + (int64_t)j * 2 * dh + k] = theta[o.B + r];
        return;
    }
    r -= (int64_t)2 * dh * d;
    if (r < (int64_t)2 * dh * d) {   // C[i][k] -> Ct[k][i]
        const int i = (int)(r / (2 * dh)), k = (int)(r % (2 * dh));
        pw[P.Ct + (int64_t)l * 2 * dh * d + (int64_t)k * d + i] = theta[o.C + r];
        return;
    }
    r -= (int64_t)2 * dh * d;
    if (r < (int64_t)2 * d * d) {    // W[i][j] -> Wt[j][i]
        const int i = (int)(r / d), j = (int)(r % d);
        pw[P.Wt + (int64_t)l * d * 2 * d + (int64_t)j * 2 * d + i] = theta[o.W + r];
        return;
    }
    r -= (int64_t)2 * d * d;
    const int k = (int)(r / 3), what = (int)(r % 3);
    if (what == 0) {
        const float mag = expf(-expf(theta[o.nu + k])), ang = expf(theta[o.th + k]);
        pw[P.lam + ((int64_t)l * dh + k) * 2] = mag * cosf(ang);
    } else if (what == 1) {
        const float mag = expf(-expf(theta[o.nu + k])), ang = expf(theta[o.th + k]);
        pw[P.lam + ((int64_t)l * dh + k) * 2 + 1] = mag * sinf(ang);
    } else {
        pw[P.eg + (int64_t)l * dh + k] = expf(theta[o.ga + k]);
    }
}

__device__ inline float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }
__device__ inline float softplus(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }

// out[t][r] (+)= sum_k M[k * ldm + r] in[t * ldi + k] for t < n, r < R (M given as [K][R]),
// over the workgroup's threads; `scale`, if given, multiplies in[t][k] by scale[k].
__device__ inline void gemm_rows(float* __restrict__ out, int ldo, const float* __restrict__ M, int ldm,
                                 const float* __restrict__ in, int ldi, const float* __restrict__ scale, int n, int R,
                                 int K, bool accumulate) {
    const int tid = threadIdx.x;
    for (int e = tid; e < n * R; e += kT) {
        const int t = e / R, r = e - t * R;
        const float* x = in + (int64_t)t * ldi;
        float acc = accumulate ? out[(int64_t)t * ldo + r] : 0.0f;
        if (scale) {
            for (int k = 0; k < K; ++k) acc = fmaf(M[(int64_t)k * ldm + r], x[k] * scale[k], acc);
        } else {
            for (int k = 0; k < K; ++k) acc = fmaf(M[(int64_t)k * ldm + r], x[k], acc);
        }
        out[(int64_t)t * ldo + r] = acc;
    }
}

// Od[r * C + c] = sign * sum_t p[t * ldp + r] (pscale ? pscale[r] : 1) q[t * ldq + c], for r < R, c < C
__device__ inline void outer_sum(float* __restrict__ Od, const float* __restrict__ p, int ldp,
                                 const float* __restrict__ pscale, const float* __restrict__ q, int ldq, int n, int R,
                                 int C, float sign) {
    for (int e = threadIdx.x; e < R * C; e += kT) {
        const int r = e / C, c = e - r * C;
        float acc = 0.0f;
        for (int t = 0; t < n; ++t) acc = fmaf(p[(int64_t)t * ldp + r], q[(int64_t)t * ldq + c], acc);
        Od[e] = sign * acc * (pscale ? pscale[r] : 1.0f);
    }
}

// ---------------------------------------------------------------------------
// Sampler
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kT) lru_sample_kernel(const float* __restrict__ theta, const float* __restrict__ pw,
                                                         LruGeom g, const float* __restrict__ u, int64_t B,
                                                         int8_t* __restrict__ spins, float* __restrict__ logpsi) {
    const LruPrep P = lru_prep_layout(g);
    const int d = g.d, dh = g.dh, N = g.n, L = g.nl, tid = threadIdx.x;
    extern __shared__ float sm[];
    float* x = sm;                  // [d] the current layer's input
    float* v = x + d;               // [2 dh]
    float* y = v + 2 * dh;          // [d]
    float* ag = y + d;              // [2 d]
    float* hs = ag + 2 * d;         // [L][2 dh] the recurrent states
    float* red = hs + L * 2 * dh;   // [kT]
    const int64_t ho = lru_head_off(g);
    for (int64_t q = blockIdx.x; q < B; q += gridDim.x) {
        for (int e = tid; e < L * 2 * dh; e += kT) hs[e] = 0.0f;
        double lp = 0.0;
        int prev = -1;
        for (int t = 0; t < N; ++t) {
            for (int j = tid; j < d; j += kT) x[j] = prev < 0 ? 0.0f : theta[(int64_t)j * 2 + prev];
            __syncthreads();
            for (int l = 0; l < L; ++l) {
                const LruOff o = lru_layer_off(g, l);
                const float* Bt = pw + P.Bt + (int64_t)l * d * 2 * dh;
                const float* Ct = pw + P.Ct + (int64_t)l * 2 * dh * d;
                const float* Wt = pw + P.Wt + (int64_t)l * d * 2 * d;
                const float* lam = pw + P.lam + (int64_t)l * dh * 2;
                const float* eg = pw + P.eg + (int64_t)l * dh;
                float* h = hs + l * 2 * dh;
                // drive and recurrence step, one complex unit per thread
                for (int k = tid; k < dh; k += kT) {
                    float vr = 0.0f, vi = 0.0f;
                    for (int j = 0; j < d; ++j) {
                        vr = fmaf(Bt[(int64_t)j * 2 * dh + k], x[j], vr);
                        vi = fmaf(Bt[(int64_t)j * 2 * dh + dh + k], x[j], vi);
                    }
                    const float lr = lam[2 * k], li = lam[2 * k + 1];
                    const float hr = h[k], hi = h[dh + k];
                    h[k] = lr * hr - li * hi + eg[k] * vr;
                    h[dh + k] = li * hr + lr * hi + eg[k] * vi;
                }
                __syncthreads();
                // y = C_re h_re - C_im h_im + D x
                for (int i = tid; i < d; i += kT) {
                    float acc = theta[o.D + i] * x[i];
                    for (int k = 0; k < dh; ++k) {
                        acc = fmaf(Ct[(int64_t)k * d + i], h[k], acc);
                        acc = fmaf(-Ct[(int64_t)(dh + k) * d + i], h[dh + k], acc);
                    }
                    y[i] = acc;
                }
                __syncthreads();
                // GLU pre-activations
                for (int i = tid; i < 2 * d; i += kT) {
                    float acc = theta[o.b + i];
                    for (int j = 0; j < d; ++j) acc = fmaf(Wt[(int64_t)j * 2 * d + i], y[j], acc);
                    ag[i] = acc;
                }
                __syncthreads();
                for (int i = tid; i < d; i += kT) x[i] = ag[i] * sigm(ag[d + i]) + (l >= 1 ? x[i] : 0.0f);
                __syncthreads();
            }
            // head: logit difference l_1 - l_0, p(sigma_t = 1) = sigmoid of it
            float part = 0.0f;
            for (int i = tid; i < d; i += kT) part = fmaf(theta[ho + d + i] - theta[ho + i], x[i], part);
            red[tid] = part;
            __syncthreads();
            for (int w = kT / 2; w >= 1; w >>= 1) {
                if (tid < w) red[tid] += red[tid + w];
                __syncthreads();
            }
            const float dl = red[0] + (theta[ho + 2 * d + 1] - theta[ho + 2 * d]);
            const float p1 = sigm(dl);
            const int s = u[q * N + t] < p1 ? 1 : 0;
            lp += (double)(s ? -softplus(-dl) : -softplus(dl));
            if (tid == 0) spins[q * N + t] = (int8_t)s;
            prev = s;
            __syncthreads();   // red and x are reused at the next site
        }
        if (tid == 0) logpsi[q] = (float)(0.5 * lp);
    }
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------

// per-chain workspace (floats)
struct LruBwdWs {
    int64_t X, V, H, Y, A, S, DX, DX2, DY, DA, DG, G, DL;
    int64_t floats;
};

__host__ __device__ inline LruBwdWs lru_bwd_layout(const LruGeom& g) {
    const int64_t N = g.n, d = g.d, dh = g.dh, L = g.nl;
    LruBwdWs w;
    int64_t t = 0;
    w.X = t; t += (L + 1) * N * d;
    w.V = t; t += L * N * 2 * dh;
    w.H = t; t += L * N * 2 * dh;
    w.Y = t; t += L * N * d;
    w.A = t; t += L * N * d;
    w.S = t; t += L * N * d;
    w.DX = t; t += N * d;
    w.DX2 = t; t += N * d;
    w.DY = t; t += N * d;
    w.DA = t; t += N * d;
    w.DG = t; t += N * d;
    w.G = t; t += N * 2 * dh;
    w.DL = t; t += N * 2;
    w.floats = t;
    return w;
}

__global__ void __launch_bounds__(kT) lru_bwd_kernel(const float* __restrict__ theta, const float* __restrict__ pw,
                                                      LruGeom g, const int8_t* __restrict__ spins, int64_t B, int64_t P,
                                                      float* __restrict__ O, float* __restrict__ logpsi,
                                                      float* __restrict__ scratch) {
    const LruPrep PP = lru_prep_layout(g);
    const LruBwdWs WL = lru_bwd_layout(g);
    const int d = g.d, dh = g.dh, N = g.n, L = g.nl, tid = threadIdx.x;
    const int64_t ho = lru_head_off(g);
    __shared__ double red[kT];
    float* ws = scratch + (int64_t)blockIdx.x * WL.floats;
    float* X = ws + WL.X;
    float* V = ws + WL.V;
    float* Hs = ws + WL.H;
    float* Y = ws + WL.Y;
    float* A = ws + WL.A;
    float* S = ws + WL.S;
    float* DX = ws + WL.DX;
    float* DX2 = ws + WL.DX2;
    float* DY = ws + WL.DY;
    float* DA = ws + WL.DA;
    float* DG = ws + WL.DG;
    float* G = ws + WL.G;
    float* DL = ws + WL.DL;
    for (int64_t q = blockIdx.x; q < B; q += gridDim.x) {
        const int8_t* sq = spins + q * N;
        float* Oq = O + q * P;
        // ---- forward, keeping every layer's activations
        for (int e = tid; e < N * d; e += kT) {
            const int t = e / d, j = e - t * d;
            X[e] = t == 0 ? 0.0f : theta[(int64_t)j * 2 + (sq[t - 1] & 1)];
        }
        __syncthreads();
        for (int l = 0; l < L; ++l) {
            const LruOff o = lru_layer_off(g, l);
            const float* Xl = X + (int64_t)l * N * d;
            float* Vl = V + (int64_t)l * N * 2 * dh;
            float* Hl = Hs + (int64_t)l * N * 2 * dh;
            float* Yl = Y + (int64_t)l * N * d;
            float* Al = A + (int64_t)l * N * d;
            float* Sl = S + (int64_t)l * N * d;
            float* Xn = X + (int64_t)(l + 1) * N * d;
            const float* lam = pw + PP.lam + (int64_t)l * dh * 2;
            const float* eg = pw + PP.eg + (int64_t)l * dh;
            // v = e^gamma (B x): [N][2 dh], columns re then im
            gemm_rows(Vl, 2 * dh, pw + PP.Bt + (int64_t)l * d * 2 * dh, 2 * dh, Xl, d, nullptr, N, 2 * dh, d, false);
            __syncthreads();
            for (int e = tid; e < N * 2 * dh; e += kT) Vl[e] *= eg[e % dh];
            __syncthreads();
            // h_t = lambda h_{t-1} + v_t, one unit per thread
            for (int k = tid; k < dh; k += kT) {
                const float lr = lam[2 * k], li = lam[2 * k + 1];
                float hr = 0.0f, hi = 0.0f;
                for (int t = 0; t < N; ++t) {
                    const float nr = lr * hr - li * hi + Vl[(int64_t)t * 2 * dh + k];
                    const float ni = li * hr + lr * hi + Vl[(int64_t)t * 2 * dh + dh + k];
                    hr = nr;
                    hi = ni;
                    Hl[(int64_t)t * 2 * dh + k] = hr;
                    Hl[(int64_t)t * 2 * dh + dh + k] = hi;
                }
            }
            __syncthreads();
            // y = C_re h_re - C_im h_im + D x
            const float* Ct = pw + PP.Ct + (int64_t)l * 2 * dh * d;
            for (int e = tid; e < N * d; e += kT) {
                const int t = e / d, i = e - t * d;
                const float* ht = Hl + (int64_t)t * 2 * dh;
                float acc = theta[o.D + i] * Xl[e];
                for (int k = 0; k < dh; ++k) {
                    acc = fmaf(Ct[(int64_t)k * d + i], ht[k], acc);
                    acc = fmaf(-Ct[(int64_t)(dh + k) * d + i], ht[dh + k], acc);
                }
                Yl[e] = acc;
            }
            __syncthreads();
            // GLU: a = W_a y + b_a, s = sigmoid(W_g y + b_g), x' = a s + [l >= 1] x
            const float* Wt = pw + PP.Wt + (int64_t)l * d * 2 * d;
            for (int e = tid; e < N * d; e += kT) {
                const int t = e / d, i = e - t * d;
                const float* yt = Yl + (int64_t)t * d;
                float aa = theta[o.b + i], gg = theta[o.b + d + i];
                for (int j = 0; j < d; ++j) {
                    aa = fmaf(Wt[(int64_t)j * 2 * d + i], yt[j], aa);
                    gg = fmaf(Wt[(int64_t)j * 2 * d + d + i], yt[j], gg);
                }
                const float s = sigm(gg);
                Al[e] = aa;
                Sl[e] = s;
                Xn[e] = aa * s + (l >= 1 ? Xl[e] : 0.0f);
            }
            __syncthreads();
        }
        // ---- head: log p and its adjoint d log psi / d logits = 1/2 (onehot - softmax)
        const float* XL = X + (int64_t)L * N * d;
        double lp = 0.0;
        for (int t = tid; t < N; t += kT) {
            float l0 = theta[ho + 2 * d], l1 = theta[ho + 2 * d + 1];
            for (int i = 0; i < d; ++i) {
                l0 = fmaf(theta[ho + i], XL[(int64_t)t * d + i], l0);
                l1 = fmaf(theta[ho + d + i], XL[(int64_t)t * d + i], l1);
            }
            const int s = sq[t] & 1;
            const float dl = s ? l0 - l1 : l1 - l0;     // (logit of the other class) - (own)
            lp += (double)(-softplus(dl));
            const float p1 = sigm(l1 - l0);
            DL[2 * t] = 0.5f * ((s == 0 ? 1.0f : 0.0f) - (1.0f - p1));
            DL[2 * t + 1] = 0.5f * ((s == 1 ? 1.0f : 0.0f) - p1);
        }
        red[tid] = lp;
        __syncthreads();
        for (int w = kT / 2; w >= 1; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0 && logpsi) logpsi[q] = (float)(0.5 * red[0]);
        // dW_o, db_o
        outer_sum(Oq + ho, DL, 2, nullptr, XL, d, N, 2, d, 1.0f);
        for (int c = tid; c < 2; c += kT) {
            float acc = 0.0f;
            for (int t = 0; t < N; ++t) acc += DL[2 * t + c];
            Oq[ho + 2 * d + c] = acc;
        }
        // dx of the last layer's output: W_o^T dlogits
        gemm_rows(DX, d, theta + ho, d, DL, 2, nullptr, N, d, 2, false);
        __syncthreads();
        // ---- layers in reverse
        for (int l = L - 1; l >= 0; --l) {
            const LruOff o = lru_layer_off(g, l);
            const float* Xl = X + (int64_t)l * N * d;
            const float* Vl = V + (int64_t)l * N * 2 * dh;
            const float* Hl = Hs + (int64_t)l * N * 2 * dh;
            const float* Yl = Y + (int64_t)l * N * d;
            const float* Al = A + (int64_t)l * N * d;
            const float* Sl = S + (int64_t)l * N * d;
            const float* lam = pw + PP.lam + (int64_t)l * dh * 2;
            const float* eg = pw + PP.eg + (int64_t)l * dh;
            // GLU adjoints
            for (int e = tid; e < N * d; e += kT) {
                const float s = Sl[e];
                DA[e] = DX[e] * s;
                DG[e] = DX[e] * Al[e] * s * (1.0f - s);
            }
            __syncthreads();
            outer_sum(Oq + o.W, DA, d, nullptr, Yl, d, N, d, d, 1.0f);               // dW_a
            outer_sum(Oq + o.W + (int64_t)d * d, DG, d, nullptr, Yl, d, N, d, d, 1.0f);   // dW_g
            for (int i = tid; i < 2 * d; i += kT) {
                const float* src = i < d ? DA : DG;
                const int c = i < d ? i : i - d;
                float acc = 0.0f;
                for (int t = 0; t < N; ++t) acc += src[(int64_t)t * d + c];
                Oq[o.b + i] = acc;
            }
            // dy = W_a^T da + W_g^T dg  (W given as [2 d][d]: rows value then gate)
            gemm_rows(DY, d, theta + o.W, d, DA, d, nullptr, N, d, d, false);
            __syncthreads();
            gemm_rows(DY, d, theta + o.W + (int64_t)d * d, d, DG, d, nullptr, N, d, d, true);
            __syncthreads();
            // dD, dC_re, dC_im
            for (int i = tid; i < d; i += kT) {
                float acc = 0.0f;
                for (int t = 0; t < N; ++t) acc = fmaf(DY[(int64_t)t * d + i], Xl[(int64_t)t * d + i], acc);
                Oq[o.D + i] = acc;
            }
            for (int e = tid; e < d * 2 * dh; e += kT) {
                const int i = e / (2 * dh), k = e - i * 2 * dh;
                float acc = 0.0f;
                for (int t = 0; t < N; ++t) acc = fmaf(DY[(int64_t)t * d + i], Hl[(int64_t)t * 2 * dh + k], acc);
                Oq[o.C + e] = k < dh ? acc : -acc;
            }
            // G_t = C_re^T dy_t - i C_im^T dy_t  (C given as [d][2 dh])
            for (int e = tid; e < N * 2 * dh; e += kT) {
                const int t = e / (2 * dh), k = e - t * 2 * dh;
                float acc = 0.0f;
                for (int i = 0; i < d; ++i) acc = fmaf(theta[o.C + (int64_t)i * 2 * dh + k], DY[(int64_t)t * d + i], acc);
                G[e] = k < dh ? acc : -acc;
            }
            __syncthreads();
            // reverse scan Ghat_t = G_t + conj(lambda) Ghat_{t+1}; dlambda, dgamma, dnu, dtheta
            for (int k = tid; k < dh; k += kT) {
                const float lr = lam[2 * k], li = lam[2 * k + 1];
                float gr = 0.0f, gi = 0.0f, dlr = 0.0f, dli = 0.0f, dga = 0.0f;
                for (int t = N - 1; t >= 0; --t) {
                    // conj(lambda) (gr + i gi) = (lr gr + li gi) + i (lr gi - li gr)
                    const float nr = G[(int64_t)t * 2 * dh + k] + lr * gr + li * gi;
                    const float ni = G[(int64_t)t * 2 * dh + dh + k] + lr * gi - li * gr;
                    gr = nr;
                    gi = ni;
                    G[(int64_t)t * 2 * dh + k] = gr;
                    G[(int64_t)t * 2 * dh + dh + k] = gi;
                    if (t > 0) {   // Ghat_t conj(h_{t-1})
                        const float hr = Hl[(int64_t)(t - 1) * 2 * dh + k], hi = Hl[(int64_t)(t - 1) * 2 * dh + dh + k];
                        dlr += gr * hr + gi * hi;
                        dli += gi * hr - gr * hi;
                    }
                    dga += gr * Vl[(int64_t)t * 2 * dh + k] + gi * Vl[(int64_t)t * 2 * dh + dh + k];
                }
                // d lambda / d nu = -e^nu lambda, d lambda / d theta = i e^theta lambda
                const float enu = expf(theta[o.nu + k]), eth = expf(theta[o.th + k]);
                Oq[o.nu + k] = dlr * (-enu * lr) + dli * (-enu * li);
                Oq[o.th + k] = dlr * (-eth * li) + dli * (eth * lr);
                Oq[o.ga + k] = dga;
            }
            __syncthreads();
            // the drive's adjoint e^gamma Ghat (dlambda, dgamma above used Ghat itself)
            for (int e = tid; e < N * 2 * dh; e += kT) G[e] *= eg[e % dh];
            __syncthreads();
            // dB (rows re then im) = (e^gamma Ghat) x^T
            outer_sum(Oq + o.B, G, 2 * dh, nullptr, Xl, d, N, dh, d, 1.0f);
            outer_sum(Oq + o.B + (int64_t)dh * d, G + dh, 2 * dh, nullptr, Xl, d, N, dh, d, 1.0f);
            // dx = D dy + [l >= 1] dx' + B^T (e^gamma Ghat)
            for (int e = tid; e < N * d; e += kT) {
                const int i = e % d;
                DX2[e] = theta[o.D + i] * DY[e] + (l >= 1 ? DX[e] : 0.0f);
            }
            __syncthreads();
            gemm_rows(DX2, d, theta + o.B, d, G, 2 * dh, nullptr, N, d, 2 * dh, true);
            __syncthreads();
            float* tmp = DX;
            DX = DX2;
            DX2 = tmp;
        }
        // dE[j][c] = sum_{t >= 1, sigma_{t-1} = c} dx^0_t[j]
        for (int e = tid; e < 2 * d; e += kT) {
            const int j = e / 2, c = e - j * 2;
            float acc = 0.0f;
            for (int t = 1; t < N; ++t)
                if ((sq[t - 1] & 1) == c) acc += DX[(int64_t)t * d + j];
            Oq[e] = acc;
        }
        __syncthreads();   // the workspace is reused by the next chain
        // restore the buffer roles (an odd number of layers swapped them)
        if (L & 1) {
            float* tmp = DX;
            DX = DX2;
            DX2 = tmp;
        }
    }
}

}  // namespace

int64_t lru_prep_floats(const LruGeom& g) { return lru_prep_layout(g).floats; }
int64_t lru_bwd_chain_floats(const LruGeom& g) { return lru_bwd_layout(g).floats; }
// chains in flight: at most 1024, and at most 4 GiB of per-chain workspace
int64_t lru_bwd_grid(const LruGeom& g, int64_t B) {
    const int64_t by_mem = ((int64_t)1 << 30) / lru_bwd_layout(g).floats;
    int64_t cap = by_mem < 1024 ? by_mem : 1024;
    if (cap < 1) cap = 1;
    return B < cap ? B : cap;
}

int launch_lru_prep(const LruGeom& g, const float* theta, float* pw, hipStream_t st) {
    const int64_t per = (int64_t)2 * g.dh * g.d + 2 * g.dh * g.d + 2 * g.d * g.d + 3 * g.dh;
    const int64_t n = per * g.nl;
    lru_prep_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(theta, g, pw);
    return (int)hipGetLastError();
}

int launch_lru_sample(const LruGeom& g, const float* theta, const float* pw, const float* u, int64_t B, int8_t* spins,
                      float* logpsi, hipStream_t st) {
    if (B == 0) return 0;
    const size_t lds = sizeof(float) * ((size_t)g.d + 2 * g.dh + g.d + 2 * g.d + (size_t)g.nl * 2 * g.dh + kT);
    const int64_t grid = B < 2048 ? B : 2048;
    lru_sample_kernel<<<(unsigned)grid, kT, lds, st>>>(theta, pw, g, u, B, spins, logpsi);
    return (int)hipGetLastError();
}

int launch_lru_backward(const LruGeom& g, const float* theta, const float* pw, const int8_t* spins, int64_t B,
                        float* O, float* logpsi, float* scratch, hipStream_t st) {
    if (B == 0) return 0;
    lru_bwd_kernel<<<(unsigned)lru_bwd_grid(g, B), kT, 0, st>>>(theta, pw, g, spins, B, lru_param_count(g), O, logpsi,
                                                                scratch);
    return (int)hipGetLastError();
}

}  // namespace psr
