// FP32 MFMA tile GEMM over operands in device memory, used by the kernels that
// keep their activations in a per-workgroup workspace (backward, sampler).
#pragma once

#include <hip/hip_runtime.h>

namespace psr {
namespace gemm_detail {

// C(m, n) (+)= sum_k A(m, k) B(k, n) with element (m, k) of A at a.p[m*a.sm + k*a.sk],
// (k, n) of B at b.p[k*b.sk + n*b.sn] and (m, n) of C at c.p[m*c.sm + n*c.sn].
// M is a multiple of 16; N and K are masked.  The workgroup's waves take the
// 16x16 output tiles in turn; a lane holds rows 4*(lane/16)..+3 of column
// lane%16 of a tile.  Must be called by the whole workgroup (no barrier inside).
typedef float f32x4 __attribute__((ext_vector_type(4)));
struct MA { const float* p; int sm, sk; };
struct MB { const float* p; int sk, sn; };
struct MC { float* p; int sm, sn; };

// Offsets are 32-bit element offsets from a workgroup-uniform base (every
// operand lives in one sample's scratch, its row of O or theta).  Operands are
// read with buffer loads: the K step of a load is a scalar offset and the lane's
// part one vector offset per tile, so no per-load address arithmetic reaches the
// vector unit.  Full K blocks run unchecked; a ragged last block zeroes A beyond
// K.  A column n >= N of B only feeds output column n, which is not stored, so
// its address is clamped instead of masked (no branches around the loads).
__device__ inline float ldbuf(__amdgpu_buffer_rsrc_t r, int voff_bytes, int soff_bytes) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff_bytes, soff_bytes, 0));
}

__device__ inline void gemm(int M, int N, int K, MA a, MB b, MC c, bool acc_in) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int tm = M >> 4, tn = (N + 15) >> 4;
    const int kq = lane >> 4, r16 = lane & 15;
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.p), 0, 0x7ffffff0, 0x00020000);
    const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(b.p), 0, 0x7ffffff0, 0x00020000);
    const int Kf = K & ~31;   // K covered by full blocks of 32
    for (int t = wave; t < tm * tn; t += nw) {
        const int m0 = (t % tm) << 4, n0 = (t / tm) << 4;
        const int n = n0 + r16;
        const bool nok = n < N;
        const int av0 = ((m0 + r16) * a.sm + kq * a.sk) * 4;        // bytes, lane part
        const int bv0 = ((nok ? n : N - 1) * b.sn + kq * b.sk) * 4;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        // K in blocks of 32: the block's 16 loads are issued together, then 8 MFMAs
        for (int k0 = 0; k0 < Kf; k0 += 32) {
            float av[8], bv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                av[q] = ldbuf(ra, av0, (k0 + 4 * q) * a.sk * 4);
                bv[q] = ldbuf(rb, bv0, (k0 + 4 * q) * b.sk * 4);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], bv[q], acc, 0, 0, 0);
        }
        if (Kf < K) {
            // last, partial block: rows k >= K of A read as zero (their addresses clamped to K - 1)
            float av[8], bv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int k = Kf + 4 * q + kq;
                const float x = ldbuf(ra, ((m0 + r16) * a.sm + min(k, K - 1) * a.sk) * 4, 0);
                av[q] = (k < K) ? x : 0.0f;
                bv[q] = ldbuf(rb, ((nok ? n : N - 1) * b.sn + min(k, K - 1) * b.sk) * 4, 0);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], bv[q], acc, 0, 0, 0);
        }
        if (nok) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float* cp = c.p + ((m0 + 4 * kq + i) * c.sm + n * c.sn);
                *cp = acc_in ? *cp + acc[i] : acc[i];
            }
        }
    }
}

// gemm() with B read by plain loads, for a B operand in LDS (buffer descriptors
// address global memory only); K must be a multiple of 32.  C goes through
// plain stores, so it may be in LDS as well.
__device__ inline void gemm_lds_b(int M, int N, int K, MA a, MB b, MC c, bool acc_in) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int tm = M >> 4, tn = (N + 15) >> 4;
    const int kq = lane >> 4, r16 = lane & 15;
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.p), 0, 0x7ffffff0, 0x00020000);
    for (int t = wave; t < tm * tn; t += nw) {
        const int m0 = (t % tm) << 4, n0 = (t / tm) << 4;
        const int n = n0 + r16;
        const bool nok = n < N;
        const int av0 = ((m0 + r16) * a.sm + kq * a.sk) * 4;
        const float* bp = b.p + (nok ? n : N - 1) * b.sn + kq * b.sk;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < K; k0 += 32) {
            float av[8], bv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                av[q] = ldbuf(ra, av0, (k0 + 4 * q) * a.sk * 4);
                bv[q] = bp[(k0 + 4 * q) * b.sk];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], bv[q], acc, 0, 0, 0);
        }
        if (nok) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float* cp = c.p + ((m0 + 4 * kq + i) * c.sm + n * c.sn);
                *cp = acc_in ? *cp + acc[i] : acc[i];
            }
        }
    }
}

}  // namespace gemm_detail
}  // namespace psr
