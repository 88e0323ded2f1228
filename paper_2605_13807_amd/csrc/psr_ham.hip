// Spin packing, connected-configuration enumeration (bit-exact, canonical
// order), local-energy combination and FP64 batch reductions.
//
// Hamiltonians (Sec. III.B, III.C): open-boundary nearest-neighbour bonds.
//   TFIM        diag = -J sum_<ab> s_a s_b, one single flip per site, element -h
//   Heisenberg  diag = (J/4) sum_<ab> s_a s_b, one exchange per antiparallel
//               bond, element -J/2 after the Marshall rotation (+J/2 without)
// Canonical order: sites ascending, and at each site a the bond (a, a+1)
// before the bond (a, a+lx).  The bond list is generated arithmetically from
// the bond index, so every sample walks the same order.
#include "psr_internal.h"

namespace psr {

// ---------------------------------------------------------------------------
// packing: int8 [B][N] -> uint32 [B][ceil(N/32)], bit (a % 32) of word a / 32
// ---------------------------------------------------------------------------
__global__ void pack_kernel(const int8_t* __restrict__ spins, int64_t B, int N, int words, uint32_t* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * words) return;
    const int64_t b = e / words;
    const int w = (int)(e - b * words);
    const int8_t* s = spins + b * N;
    uint32_t v = 0;
    const int a0 = 32 * w;
    const int n = min(32, N - a0);
    for (int k = 0; k < n; ++k) v |= (uint32_t)(s[a0 + k] & 1) << k;
    out[e] = v;
}

int launch_pack_spins(const int8_t* spins, int64_t B, int N, uint32_t* packed, hipStream_t st) {
    const int words = (N + 31) / 32;
    const int64_t n = B * words;
    if (n == 0) return 0;
    pack_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(spins, B, N, words, packed);
    return (int)hipGetLastError();
}

__global__ void check_kernel(const int8_t* __restrict__ s, int64_t n, int* bad) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int local = 0;
    for (; e < n; e += stride) local |= (s[e] != 0 && s[e] != 1);
    if (__any(local) && (threadIdx.x & 63) == 0) atomicOr(bad, 1);
}

int launch_check_spins(const int8_t* spins, int64_t n, int32_t* bad, hipStream_t st) {
    const hipError_t me = hipMemsetAsync(bad, 0, sizeof(int), st);
    if (me != hipSuccess) return (int)me;
    if (n > 0) check_kernel<<<1024, 256, 0, st>>>(spins, n, bad);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// bonds
// ---------------------------------------------------------------------------
__host__ __device__ inline int64_t n_bonds(int lx, int ly) {
    return (int64_t)(lx - 1) * ly + (int64_t)lx * (ly - 1);
}

// Bond number k in canonical order -> sites (a, b).  A row y < ly-1 holds
// 2*lx - 1 bonds: (x, right), (x, up) for x < lx-1 and (lx-1, up); the last
// row holds lx - 1 right bonds.
__device__ inline void bond_sites(int lx, int ly, int k, int& a, int& b) {
    const int per = 2 * lx - 1;
    const int full = (ly - 1) * per;
    if (k < full) {
        const int y = k / per, r = k - y * per;
        const int x = r >> 1;
        a = y * lx + x;
        b = (r & 1) || (x == lx - 1) ? a + lx : a + 1;
    } else {
        const int x = k - full;
        a = (ly - 1) * lx + x;
        b = a + 1;
    }
}

__device__ inline int bit_of(const int8_t* w, int a) { return (int)(w[a] & 1); }

int64_t ham_max_connected(const Ham& h) {
    return h.kind == 0 ? (int64_t)h.lx * h.ly : n_bonds(h.lx, h.ly);
}

// one wave per sample
__global__ void conn_count_kernel(Ham h, const int8_t* __restrict__ spins, int64_t B,
                                  int32_t* __restrict__ n_conn, float* __restrict__ diag) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (s >= B) return;
    const int8_t* w = spins + s * (int64_t)h.lx * h.ly;
    const int nb = (int)n_bonds(h.lx, h.ly);
    int anti = 0;
    for (int k = lane; k < nb; k += 64) {
        int a, b;
        bond_sites(h.lx, h.ly, k, a, b);
        anti += bit_of(w, a) ^ bit_of(w, b);
    }
    for (int o = 32; o > 0; o >>= 1) anti += __shfl_xor(anti, o);
    if (lane == 0) {
        const int par = nb - anti;      // sum_<ab> s_a s_b = #parallel - #antiparallel (exact integers)
        const int zz = par - anti;
        if (h.kind == 0) {
            n_conn[s] = h.lx * h.ly;
            if (diag) diag[s] = -h.J * (float)zz;
        } else {
            n_conn[s] = anti;
            if (diag) diag[s] = (h.J * 0.25f) * (float)zz;
        }
    }
}

int launch_conn_count(const Ham& h, const int8_t* spins, int64_t B, int32_t* n_conn, float* diag, hipStream_t st) {
    if (B == 0) return 0;
    conn_count_kernel<<<(unsigned)((B + 3) / 4), 256, 0, st>>>(h, spins, B, n_conn, diag);
    return (int)hipGetLastError();
}

// one wave per sample; ballot + popcount compaction keeps canonical order
__global__ void conn_write_kernel(Ham h, const int8_t* __restrict__ spins, int64_t B,
                                  const int64_t* __restrict__ offs, int64_t stride, uint32_t* __restrict__ desc,
                                  float* __restrict__ mel) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (s >= B) return;
    const int8_t* w = spins + s * (int64_t)h.lx * h.ly;
    int64_t base = offs ? offs[s] : s * stride;
    const float el = (h.kind == 0) ? -h.h : (h.marshall ? -0.5f * h.J : 0.5f * h.J);
    if (h.kind == 0) {
        const int N = h.lx * h.ly;
        for (int a = lane; a < N; a += 64) {
            if (desc) {
                desc[2 * (base + a)] = (uint32_t)s;
                desc[2 * (base + a) + 1] = (uint32_t)a | ((uint32_t)a << 16);
            }
            if (mel) mel[base + a] = el;
        }
        return;
    }
    const int nb = (int)n_bonds(h.lx, h.ly);
    for (int k0 = 0; k0 < nb; k0 += 64) {
        const int k = k0 + lane;
        int a = 0, b = 0, f = 0;
        if (k < nb) {
            bond_sites(h.lx, h.ly, k, a, b);
            f = bit_of(w, a) ^ bit_of(w, b);
        }
        const uint64_t m = __ballot(f);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (f) {
            const int64_t o = base + pre;
            if (desc) {
                desc[2 * o] = (uint32_t)s;
                desc[2 * o + 1] = (uint32_t)a | ((uint32_t)b << 16);
            }
            if (mel) mel[o] = el;
        }
        base += __popcll(m);
    }
}

// full configurations conn[s][k][N] from descriptors in per-sample layout
__global__ void conn_expand_kernel(const int8_t* __restrict__ spins, int N, int64_t B, int64_t max_conn,
                                   const int32_t* __restrict__ n_conn, const uint32_t* __restrict__ desc,
                                   int8_t* __restrict__ conn) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * max_conn * N) return;
    const int64_t sk = e / N;
    const int a = (int)(e - sk * N);
    const int64_t s = sk / max_conn, k = sk - s * max_conn;
    if (k >= n_conn[s]) return;
    const uint32_t d1 = desc[2 * sk + 1];
    const int fa = (int)(d1 & 0xFFFF), fb = (int)(d1 >> 16);
    int v = spins[s * N + a];
    if (a == fa) v ^= 1;
    if (a == fb && fb != fa) v ^= 1;
    conn[e] = (int8_t)v;
}

int launch_conn_write(const Ham& h, const int8_t* spins, int64_t B, const int64_t* offs, int64_t stride,
                      uint32_t* desc, float* mel, hipStream_t st) {
    if (B == 0) return 0;
    conn_write_kernel<<<(unsigned)((B + 3) / 4), 256, 0, st>>>(h, spins, B, offs, stride, desc, mel);
    return (int)hipGetLastError();
}

int launch_conn_expand(const int8_t* spins, int N, int64_t B, int64_t max_conn, const int32_t* n_conn,
                       const uint32_t* desc, int8_t* conn, hipStream_t st) {
    const int64_t n = B * max_conn * N;
    if (n == 0) return 0;
    conn_expand_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(spins, N, B, max_conn, n_conn, desc, conn);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan of the per-sample counts (one workgroup, deterministic)
// ---------------------------------------------------------------------------
__global__ void scan_kernel(const int32_t* __restrict__ cnt, int64_t B, int64_t* __restrict__ offs) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x, T = blockDim.x;
    const int64_t per = (B + T - 1) / T;
    const int64_t b0 = min(B, per * t), b1 = min(B, b0 + per);
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += cnt[b];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int k = 0; k < T; ++k) {
            const int64_t v = part[k];
            part[k] = acc;
            acc += v;
        }
        offs[B] = acc;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t b = b0; b < b1; ++b) {
        offs[b] = acc;
        acc += cnt[b];
    }
}

int launch_scan_counts(const int32_t* n_conn, int64_t B, int64_t* offs, hipStream_t st) {
    scan_kernel<<<1, 1024, 0, st>>>(n_conn, B, offs);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// E_loc(s) = diag(s) + sum_k mel_k exp(log psi(sigma'_k) - log psi(sigma_s))
// One wave per sample, fixed summation order (deterministic).  The difference
// of the two log psi values is taken on (hi, lo) pairs so that the common
// prefix of sigma and sigma' cancels to float precision.
// ---------------------------------------------------------------------------
__global__ void eloc_kernel(int64_t B, const int64_t* __restrict__ offs, const float* __restrict__ diag,
                            const float* __restrict__ mel, const float* __restrict__ chi, const float* __restrict__ clo,
                            const float* __restrict__ shi, const float* __restrict__ slo, double* __restrict__ eloc) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (s >= B) return;
    const int64_t k0 = offs[s], k1 = offs[s + 1];
    const float h0 = shi[s], l0 = slo[s];
    float acc = 0.0f;
    for (int64_t k = k0 + lane; k < k1; k += 64) {
        const float dl = (chi[k] - h0) + (clo[k] - l0);
        acc = fmaf(mel[k], __expf(dl), acc);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) eloc[s] = (double)(diag[s] + acc);
}

int launch_eloc_combine(int64_t B, const int64_t* offs, const float* diag, const float* mel, const float* lpc_hi,
                        const float* lpc_lo, const float* lps_hi, const float* lps_lo, double* eloc, hipStream_t st) {
    if (B == 0) return 0;
    eloc_kernel<<<(unsigned)((B + 3) / 4), 256, 0, st>>>(B, offs, diag, mel, lpc_hi, lpc_lo, lps_hi, lps_lo, eloc);
    return (int)hipGetLastError();
}

// mean and variance (1/B) in FP64, one workgroup, fixed order
__global__ void stats_kernel(const double* __restrict__ x, int64_t B, double* __restrict__ out) {
    __shared__ double part[1024];
    const int t = threadIdx.x, T = blockDim.x;
    double s = 0.0;
    for (int64_t b = t; b < B; b += T) s += x[b];
    part[t] = s;
    __syncthreads();
    for (int w = T / 2; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    const double mean = part[0] / (double)B;
    __syncthreads();
    double v = 0.0;
    for (int64_t b = t; b < B; b += T) {
        const double e = x[b] - mean;
        v += e * e;
    }
    part[t] = v;
    __syncthreads();
    for (int w = T / 2; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) {
        out[0] = mean;
        out[1] = part[0] / (double)B;
    }
}

int launch_stats(const double* x, int64_t B, double* stats, hipStream_t st) {
    stats_kernel<<<1, 1024, 0, st>>>(x, B, stats);
    return (int)hipGetLastError();
}

__global__ void vmc_w_kernel(const double* __restrict__ e, const double* __restrict__ stats, int64_t B,
                             double* __restrict__ w) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) w[b] = (2.0 / (double)B) * (e[b] - stats[0]);
}

int launch_vmc_weights(const double* eloc, const double* stats, int64_t B, double* w, hipStream_t st) {
    if (B == 0) return 0;
    vmc_w_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(eloc, stats, B, w);
    return (int)hipGetLastError();
}

__global__ void combine_kernel(const float* __restrict__ hi, const float* __restrict__ lo, int64_t B,
                               float* __restrict__ out) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) out[b] = hi[b] + lo[b];
}

// log psi_c4v = 1/2 [logsumexp_k 2 log psi(sigma o T_k) - log 8] from the eight
// (hi, lo) pairs, in FP64, kept as a (hi, lo) pair
__global__ void c4v_combine_kernel(const float* __restrict__ hi8, const float* __restrict__ lo8, int64_t n,
                                   float* __restrict__ out_hi, float* __restrict__ out_lo) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double v[8];
    double mx = -1e300;
    for (int k = 0; k < 8; ++k) {
        v[k] = 2.0 * ((double)hi8[k * n + q] + (double)lo8[k * n + q]);
        mx = fmax(mx, v[k]);
    }
    double sum = 0.0;
    for (int k = 0; k < 8; ++k) sum += exp(v[k] - mx);
    const double r = 0.5 * (mx + log(sum) - log(8.0));
    const float h = (float)r;
    out_hi[q] = h;
    if (out_lo) out_lo[q] = (float)(r - (double)h);
}

int launch_c4v_combine(const float* hi8, const float* lo8, int64_t n, float* out_hi, float* out_lo, hipStream_t st) {
    if (n <= 0) return 0;
    c4v_combine_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(hi8, lo8, n, out_hi, out_lo);
    return (int)hipGetLastError();
}

int launch_combine_logpsi(const float* hi, const float* lo, int64_t B, float* out, hipStream_t st) {
    if (B == 0) return 0;
    combine_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(hi, lo, B, out);
    return (int)hipGetLastError();
}

// g[p] = sum_s w[s] O[s][p] in FP64; one thread per parameter, samples in order
__global__ void wsum_kernel(const float* __restrict__ O, int64_t B, int64_t P, const double* __restrict__ w,
                            double* __restrict__ g) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double acc = 0.0;
    for (int64_t s = 0; s < B; ++s) acc += w[s] * (double)O[s * P + p];
    g[p] = acc;
}

int launch_weighted_sum(const float* O, int64_t B, int64_t P, const double* w, double* g, hipStream_t st) {
    if (P == 0) return 0;
    wsum_kernel<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(O, B, P, w, g);
    return (int)hipGetLastError();
}

}  // namespace psr
