// Internal declarations shared by the libpsr translation units (not installed).
//
// Register layout used by every projection kernel
// ------------------------------------------------
// The dense projections are MFMA products  out[unit][column] = W[unit][k] * act[k][column]
// with the weights as the A operand and the activations as the B operand of
// v_mfma_f32_16x16x32_bf16 / _f16 (split 16-bit paths) or v_mfma_f32_16x16x4_f32 (FP32 path).
// A column is one (sequence, site) pair, so the 16 columns of an MFMA tile are
// 16 lanes of a DPP row and the scan along a lattice row runs across lanes.
//
// A 16x16 f32 accumulator puts output row 4g+i (g = lane/16, i = 0..3) of
// column lane%16 in register i of lane `lane`.  A lane in lane group g
// therefore holds, for its column, the units
//      unit(s, g) = 16*(s/4) + 4*g + (s%4),    s = 0 .. d/4-1
// when it keeps the accumulators of all d/16 output tiles as v[s = 4*mt + i].
// That vector, converted and packed in order of s, is exactly what the lane
// must supply as the B operand of the next product, provided the weights' K
// index is permuted the same way: a contraction only needs A and B to agree
// slot by slot.  So activations never leave registers between layers; the
// weights are re-laid out once per call ("fragments") in that K order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace psr {

constexpr int kFP32 = 0;
constexpr int kBF16 = 1;   // split BF16 operands (hi + lo)
constexpr int kFP16 = 2;   // split binary16 operands (hi + 2^-11 lo)

__host__ __device__ inline int slot_unit(int s, int g) { return 16 * (s >> 2) + 4 * g + (s & 3); }

// Model geometry as seen by the kernels.
struct Geom {
    int chain;     // 1: Eq. (minGRU) chain, head on h; 0: 2D snake
    int lx, ly;    // the grid the recurrence runs on: sites, or 2x2 patches (patch = 2)
    int nl, d, prec;
    int patch;     // 1: single-site inputs (K = 2); 2: 2x2 patches (K = 16)
    int slx, sly;  // the spin lattice (lx, ly times patch)
    int sym;       // 1: c4v-symmetrised log psi (eight transformed evaluations)
};
__host__ __device__ inline int n_states(const Geom& g) { return g.patch == 2 ? 16 : 2; }

// Where one GEMM matrix of the model sits inside theta: element (r, k) is
// theta[base + r * ld + coff + k] for r, k in [0, d).
struct MatSrc { int64_t base; int ld; int coff; };

// Offsets of the prepared (fragment-order) parameters.
struct Prepared {
    // per layer l: fragment offset (bytes) of each GEMM matrix, -1 if absent.
    //   index 0: W_z, 1: W_h (u part), 2: W_h (h_V part), 3: D, 4: C
    int64_t frag[8][5];
    int frag_present[8][5];    // 1 if the matrix exists (layer 0 has only W_h's h_V part and C)
    int64_t frag_bytes;        // total bytes of the fragment area
    // float offsets (in floats) into the table area
    int64_t t0z, t0h, t0d;     // layer-0 tables [9][d] in slot order (state = 3*sH + sV)
    int64_t bias_z[8], bias_h[8];   // layers >= 1: [d] in slot order
    int64_t head_w, head_b;    // W_o[0] - W_o[1] [d] slot order, b_o[0] - b_o[1]
    int64_t table_floats;
};

// Model-dependent host helpers (psr_api.hip).
int64_t param_count(const Geom& g);
void param_offsets(const Geom& g, int64_t* off, int32_t* n);
Prepared prepared_layout(const Geom& g);

// Forward-kernel launch shape chosen for a model.
struct FwdShape {
    int ntc;          // 16-column MFMA tiles per wave
    int waves;        // waves per workgroup
    int cols;         // columns per workgroup = waves * ntc * 16
    int seqs;         // sequences per workgroup = cols / lx
    int cross_wave;   // some sequence row spans a wave boundary
    int lds_frontier; // the row frontier is kept in LDS (split 16-bit paths, when it fits)
    int split_kernel; // 1: the units-split kernel of psr_fwd_split.hip runs this model
};
FwdShape fwd_shape(const Geom& g);
// The units-split kernel (split 16-bit operands, 2D, d = 128 or 256, rows within its columns).
bool split_kernel_applies(const Geom& g);
void split_shape(const Geom& g, FwdShape* s);

// Arguments of the forward kernel.
struct FwdArgs {
    Geom g;
    const uint32_t* spins;    // packed spins, words_per_seq uint32 per source row, bit a%32 of word a/32 = site a
    int words_per_seq;
    const uint32_t* desc;     // NULL: sequence q reads packed row q unflipped; else {row, a | b << 16} per q
    int64_t q_begin;          // first sequence of this launch
    int64_t q_count;          // sequences in this launch (upper bound)
    const int64_t* q_total;   // NULL or device count: sequences with index >= *q_total are skipped
    const uint8_t* frag;      // prepared fragments
    const float* tab;         // prepared tables
    Prepared pl;
    FwdShape sh;
    void* frontier;           // [q_count][nl][lx][d] h of the previous row (f32 or 16-bit pairs), indexed by q - q_begin
    float* out_hi;            // [.] log psi, high part   (indexed by q)
    float* out_lo;            // [.] log psi, low part    (indexed by q) or NULL
    float* logp_site;         // [q][N] or NULL
    int xform;                // 0..7: the spins are read as sigma o T_xform (c4v symmetry T_k)
};

// Launchers (return a hipError_t cast to int).
int launch_prepare(const Geom& g, const Prepared& pl, const float* theta, uint8_t* frag, float* tab,
                   hipStream_t st);
int launch_forward(const FwdArgs& a, hipStream_t st);
int launch_forward_split(const FwdArgs& a, hipStream_t st);
int launch_pack_spins(const int8_t* spins, int64_t B, int N, uint32_t* packed, hipStream_t st);
int launch_check_spins(const int8_t* spins, int64_t n, int32_t* bad, hipStream_t st);

// Hamiltonian descriptor as seen by the kernels.
struct Ham {
    int kind;         // 0 TFIM, 1 Heisenberg
    int lx, ly;
    int marshall;
    float J, h;
};
int64_t ham_max_connected(const Ham& h);
// count pass: n_conn[s], diag[s]
int launch_conn_count(const Ham& h, const int8_t* spins, int64_t B, int32_t* n_conn, float* diag, hipStream_t st);
int launch_conn_expand(const int8_t* spins, int N, int64_t B, int64_t max_conn, const int32_t* n_conn,
                       const uint32_t* desc, int8_t* conn, hipStream_t st);
// write pass: entries of sample s go to flat index base(s) + k, base(s) = offs ? offs[s] : s * stride
int launch_conn_write(const Ham& h, const int8_t* spins, int64_t B, const int64_t* offs, int64_t stride,
                      uint32_t* desc, float* mel, hipStream_t st);
// exclusive scan of n_conn into offs[B] and offs[B] = total (single workgroup)
int launch_scan_counts(const int32_t* n_conn, int64_t B, int64_t* offs, hipStream_t st);
// E_loc(s) = diag + sum mel * exp(lp_conn - lp_sample), per sample; then mean/var in FP64
int launch_eloc_combine(int64_t B, const int64_t* offs, const float* diag, const float* mel,
                        const float* lpc_hi, const float* lpc_lo, const float* lps_hi, const float* lps_lo,
                        double* eloc, hipStream_t st);
int launch_stats(const double* x, int64_t B, double* stats, hipStream_t st);
int launch_vmc_weights(const double* eloc, const double* stats, int64_t B, double* w, hipStream_t st);
int launch_combine_logpsi(const float* hi, const float* lo, int64_t B, float* out, hipStream_t st);
// c4v: (out_hi, out_lo)[q] = 1/2 [logsumexp_k 2 (hi + lo)[k n + q] - log 8], k = 0..7, in FP64
int launch_c4v_combine(const float* hi8, const float* lo8, int64_t n, float* out_hi, float* out_lo, hipStream_t st);

// Sampler (psr_sample.hip): workgroups of sequences, per-workgroup workspace
int64_t sample_ws_per_wg_floats(const Geom& g);
int64_t sample_groups(int64_t B);
int launch_sample(const Geom& g, const float* theta, const float* u, int64_t B, int8_t* spins, float* logpsi,
                  float* scratch, hipStream_t st);
// Backward (psr_bwd.hip)
struct BwdLayout {
    int rows_per_chunk, n_chunks;
    int64_t ws_per_sample_floats;    // per-sample scratch
    int64_t wt_floats;               // transposed weights area
};
BwdLayout bwd_layout(const Geom& g, int ckpt_rows);
int launch_backward(const Geom& g, const BwdLayout& bl, const float* theta, const uint32_t* packed, int words,
                    int64_t B, float* wt, float* scratch, float* O, float* logpsi, hipStream_t st);
int launch_weighted_sum(const float* O, int64_t B, int64_t P, const double* w, double* g, hipStream_t st);

// 1D LRU ansatz (psr_lru.hip)
struct LruGeom {
    int n, nl, d, dh;   // chain length, layers, width, hidden (complex) units
};
// floats of one layer: nu, theta, gamma [dh]; B [2 dh][d]; D [d]; C [d][2 dh]; W_glu [2 d][d]; b_glu [2 d]
__host__ __device__ inline int64_t lru_layer_floats(const LruGeom& g) {
    const int64_t d = g.d, dh = g.dh;
    return 3 * dh + 2 * dh * d + d + 2 * d * dh + 2 * d * d + 2 * d;
}
int64_t lru_param_count(const LruGeom& g);
int64_t lru_workspace_floats(const LruGeom& g, int64_t B);
// logpsi_lo (or NULL): the low part of log psi (the FP64 sum as a float pair)
int launch_lru_logpsi(const LruGeom& g, const float* theta, const int8_t* spins, int64_t B, float* logpsi,
                      float* logpsi_lo, float* logp_site, float* scratch, hipStream_t st);
// LRU sampler and backward (psr_lru_bwd.hip): a shared prepared area (transposed
// matrices, lambda, e^gamma) and, for the backward, a workspace per chain in flight
int64_t lru_prep_floats(const LruGeom& g);
int64_t lru_bwd_chain_floats(const LruGeom& g);
int64_t lru_bwd_grid(const LruGeom& g, int64_t B);
int launch_lru_prep(const LruGeom& g, const float* theta, float* pw, hipStream_t st);
int launch_lru_sample(const LruGeom& g, const float* theta, const float* pw, const float* u, int64_t B, int8_t* spins,
                      float* logpsi, hipStream_t st);
int launch_lru_backward(const LruGeom& g, const float* theta, const float* pw, const int8_t* spins, int64_t B,
                        float* O, float* logpsi, float* scratch, hipStream_t st);
// E_loc from per-sample connected slots (s * max_conn + k) and the two log psi (hi, lo) arrays
int launch_lru_eloc_combine(int64_t B, int64_t max_conn, const int32_t* n_conn, const float* diag, const float* mel,
                            const float* lpc, const float* lpc_lo, const float* lps, const float* lps_lo, double* eloc,
                            hipStream_t st);

}  // namespace psr
