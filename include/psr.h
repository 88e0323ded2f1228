/*
 * psr.h -- C ABI of libpsr, the MI355X (gfx950) hot path of the parallel-scan
 * recurrent neural quantum state (PSR-NQS): batched log psi of an
 * autoregressive 1D/2D minGRU wave function, the configurations a Hamiltonian
 * connects to each sample, the local energy E_loc and the per-sample
 * gradient d log psi / d theta.
 *
 * Paper: E. Merali, M. Hibat-Allah, M. Kohandel, R. T. Scalettar, E. Khatami,
 * "Parallel Scan Recurrent Neural Quantum States for Scalable Variational
 * Monte Carlo".  Section references below are to that paper.
 *
 * General rules
 *  - Every pointer argument named as device memory must point to HIP device
 *    memory of the current device; the caller owns it and keeps it alive until
 *    the work queued on `stream` has finished.  Pointers to descriptor structs
 *    are host pointers, read before the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Compute calls only queue work on it and return; they never synchronise,
 *    except where a call says otherwise.
 *  - Return value: PSR_OK (0) or a negative PSR_E* code.  Arguments are checked
 *    on the host before anything is queued, so an error return queues no work
 *    and writes no output.  psr_last_error() gives a message for the last
 *    failing call of the calling thread.
 *  - Spins are int8 in {0, 1}, 1 = spin up (sigma^z = +1), stored per sample
 *    in lattice row-major order: site a = y * lx + x.  Values outside {0, 1}
 *    are a precondition violation (use psr_check_spins to test a batch).
 *  - Parameters theta are float32, one flat vector in the layout given by
 *    psr_param_offsets (also the layout of every gradient row).
 */
#ifndef PSR_H
#define PSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PSR_OK            0
#define PSR_EINVAL       -1   /* invalid argument */
#define PSR_EUNSUPPORTED -2   /* valid request that this library does not support */
#define PSR_ENOMEM       -3   /* workspace too small or allocation failed */
#define PSR_EDEVICE      -4   /* HIP runtime error */
#define PSR_ECAPACITY    -5   /* max_conn smaller than a sample's connected count */
#define PSR_EDATA        -6   /* spins outside {0, 1} (psr_check_spins) */

/* ---- model ------------------------------------------------------------- */
#define PSR_CHAIN_1D   0  /* Sec. II.C, Eq. (minGRU): one layer on a chain, head on h_t */
#define PSR_SNAKE_2D   1  /* Sec. II.F-G: stacked 2D minGRU along the zigzag path */

/* Precision of the dense projections (W_z u, W_h [u, h_V], C h, D u; Sec. II.F).
 * Everything else -- gates, the in-row scan and its carries, GELU, the head,
 * log-softmax and log psi -- is FP32 in every mode.
 *   PSR_FP32  FP32 matrix cores (v_mfma_f32_16x16x4_f32).
 *   PSR_BF16  BF16 matrix cores with FP32 accumulation.  Each operand (weight or
 *             activation) is carried as two bfloat16 parts, v ~ hi + lo with
 *             hi = bf16(v), lo = bf16(v - hi) (about 16 significant bits), and a
 *             product is hi*hi + lo*hi + hi*lo: three BF16 products.
 *   PSR_FP16  FP16 matrix cores with FP32 accumulation, operands as two binary16
 *             parts v ~ hi + 2^-11 lo (about 22 significant bits), same three
 *             products.  Operands must stay below 65504 in magnitude.
 * One rounding of the operands to 16 bits moves E_loc of the randomly
 * initialised 32x32 model by several per cent; the split keeps log psi within
 * ~1e-3 (BF16) of float64 there. */
#define PSR_FP32       0
#define PSR_BF16       1
#define PSR_FP16       2

typedef struct {
    int32_t geometry;   /* PSR_CHAIN_1D or PSR_SNAKE_2D */
    int32_t lx, ly;     /* lattice sides; the chain has ly = 1 and lx = N */
    int32_t n_layers;   /* chain: 1 */
    int32_t d;          /* hidden size d = d_h; 32, 64, 128 or 256 */
    int32_t precision;  /* PSR_FP32, PSR_BF16 or PSR_FP16 (arithmetic of the dense projections) */
    int32_t ckpt_rows;  /* rows per backward checkpoint chunk; 0 = max(1, 128 / lx) */
    int32_t patch;      /* 0 or 1: single-site inputs; 2: 2x2 patches (Sec. II.F), snake only, even lx, ly */
    int32_t symmetry;   /* PSR_SYM_NONE or PSR_SYM_C4V (square snake lattices) */
} psr_model_desc;

/* Patches (patch = 2): the recurrence runs on the (lx/2)-by-(ly/2) grid of 2x2
 * patches in the same zigzag order; patch (I, J) covers the spins (2I + a, 2J + b)
 * and has the state k = s(2I,2J) + 2 s(2I+1,2J) + 4 s(2I,2J+1) + 8 s(2I+1,2J+1)
 * of a 16-letter alphabet; u^(0) is the one-hot state of the H- and V-predecessor
 * patches (du = 32 at layer 0) and the head is a 16-way softmax (W_o[16][d],
 * b_o[16]).  log psi = 1/2 sum over patches of log p(k_t | k_<t); logp_site
 * outputs are per patch, [B][(lx/2) (ly/2)] in grid row-major order.
 *
 * Symmetry (Sec. III.C: the 2D runs impose the c4v symmetry of the lattice):
 * with T_0..T_7 the eight symmetries of the L-by-L lattice acting on site
 * positions, |psi_c4v(sigma)|^2 = (1/8) sum_k |psi(sigma o T_k)|^2, i.e.
 * log psi_c4v = 1/2 [logsumexp_k 2 log psi(sigma o T_k) - log 8] (the paper
 * gives no formula; this form keeps normalisation and exact sampling).  The
 * library evaluates the eight transformed configurations with the same kernels
 * and combines them in FP64.  T_k maps (x, y) to: (x, y), (L-1-y, x),
 * (L-1-x, L-1-y), (y, L-1-x), (L-1-x, y), (x, L-1-y), (y, x), (L-1-y, L-1-x).
 * psr_logpsi_backward and psr_sample support neither patches nor symmetry
 * (PSR_EUNSUPPORTED). */
#define PSR_SYM_NONE   0
#define PSR_SYM_C4V    1

/*
 * Parameter layout (Sec. II.C for the chain, Sec. II.F-G for the snake):
 *   chain : W_z[d][2], b_z[d], W_h[d][2], b_h[d], W_o[2][d], b_o[2]
 *   snake : for each layer l = 0..n_layers-1
 *             W_z[d][du], b_z[d], W_h[d][du+d], b_h[d], C[d][d], D[d][du]
 *           with du = 2K at l = 0 (one-hot states of the two causal
 *           predecessors; K = 2 for single sites, 16 for 2x2 patches) and
 *           du = d above; then W_o[K][d], b_o[K].
 * Matrices are row-major (output index first).  W_h multiplies [u, h_V].
 */
int64_t psr_param_count(const psr_model_desc* m);  /* P, or a negative code */

/* offsets[k] = first entry of tensor k (k = 0..n-1) and offsets[n] = P.
 * `offsets` must hold at least 6 * n_layers + 3 entries; *n_tensors gets n. */
int psr_param_offsets(const psr_model_desc* m, int64_t* offsets, int32_t* n_tensors);

/* ---- Hamiltonian ------------------------------------------------------- */
#define PSR_TFIM        0  /* H = -J sum_<ab> Z_a Z_b - h sum_a X_a (Sec. III.B, open chain) */
#define PSR_HEISENBERG  1  /* H = J sum_<ab> S_a . S_b, S = sigma/2 (Sec. III.C, open square lattice) */

typedef struct {
    int32_t kind;       /* PSR_TFIM or PSR_HEISENBERG */
    int32_t lx, ly;     /* must equal the model's lattice; bonds are the open-boundary nearest neighbours */
    int32_t marshall;   /* Heisenberg only: 1 = Marshall-rotated basis (off-diagonal -J/2, Sec. III.C) */
    int32_t pbc;        /* must be 0: open boundaries, as in the paper */
    double  J, h;
} psr_hamiltonian;

/* Largest connected count of one sample: N for TFIM, the bond count 2 lx ly - lx - ly for Heisenberg. */
int64_t psr_max_connected(const psr_hamiltonian* H);

/* ---- workspace --------------------------------------------------------- */
#define PSR_OP_LOGPSI        0
#define PSR_OP_LOCAL_ENERGY  1
#define PSR_OP_BACKWARD      2
#define PSR_OP_SAMPLE        3

/* Device workspace bytes that `op` needs for a batch of `batch` samples
 * (`chunk_seqs` only matters for PSR_OP_LOCAL_ENERGY).  Negative on error. */
int64_t psr_workspace_bytes(const psr_model_desc* m, int32_t op, int64_t batch, int64_t chunk_seqs);

/* ---- compute calls ------------------------------------------------------ */

/*
 * log psi of a batch (Sec. III.B: psi is the square root of the
 * autoregressive probability, log psi = 1/2 sum_t log p(sigma_t | sigma_<t)),
 * evaluated row by row with a parallel scan along each zigzag row (Sec. II.F).
 *   theta      device, float[P]
 *   spins      device, int8[B][N]
 *   logpsi     device, float[B]                     (out)
 *   logp_site  device, float[B][N] or NULL          (out) log p of each site, row-major
 *   ws         device workspace of psr_workspace_bytes(m, PSR_OP_LOGPSI, B, 0) bytes
 */
int psr_logpsi(const psr_model_desc* m, const float* theta, const int8_t* spins, int64_t B,
               float* logpsi, float* logp_site, void* ws, size_t ws_bytes, void* stream);

/*
 * psr_logpsi without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The call allocates nothing: its scratch is a static
 * device array of psr_static_scratch_bytes() bytes (64 MiB) that each GPU holds
 * until the process ends.  Every call on one GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams, other threads) race; the caller
 * serialises them.  A batch whose workspace (psr_workspace_bytes(m,
 * PSR_OP_LOGPSI, B, 0)) exceeds the array is rejected with PSR_ENOMEM before
 * anything is queued.  Arguments and results otherwise as psr_logpsi.
 */
int64_t psr_static_scratch_bytes(void);
int psr_logpsi_static(const psr_model_desc* m, const float* theta, const int8_t* spins, int64_t B,
                      float* logpsi, float* logp_site, void* stream);

/*
 * Connected configurations of each sample (Sec. II.A: the extra forward passes
 * of the local energy), in canonical order: sites ascending; at each site a the
 * bond (a, a+1) before the bond (a, a+lx).  Heisenberg: one entry per bond
 * whose spins differ (the exchange), element -J/2 (Marshall) or +J/2.  TFIM:
 * one entry per site (single flip), element -h.
 *   spins   device int8[B][N]
 *   conn    device int8[B][max_conn][N] or NULL   (out) the configurations
 *   desc    device uint32[B][max_conn][2] or NULL (out) {sample, a | b << 16};
 *           sites a and b are flipped (a == b: one flip)
 *   mel     device float[B][max_conn] or NULL     (out) <sigma|H|sigma'>
 *   n_conn  device int32[B]                       (out)
 *   diag    device float[B] or NULL               (out) <sigma|H|sigma>
 * Entries k >= n_conn[s] of a sample are left untouched.  max_conn must be at
 * least psr_max_connected(H) (else PSR_ECAPACITY); N must be <= 65535.
 */
int psr_connected(const psr_hamiltonian* H, const int8_t* spins, int64_t B, int64_t max_conn,
                  int8_t* conn, uint32_t* desc, float* mel, int32_t* n_conn, float* diag,
                  void* stream);

/*
 * Local energies E_loc(s) = diag(s) + sum_k mel_k psi(sigma'_k) / psi(sigma_s)
 * and their batch mean and variance (1/B normaliser) accumulated in FP64.
 * The connected configurations are evaluated in chunks of `chunk_seqs`
 * sequences (0 = 32768), so device memory stays O(chunk), not O(B * N).
 *   eloc    device double[B]      (out)
 *   stats   device double[2]      (out) mean, variance
 *   logpsi  device float[B] or NULL (out) log psi of the samples
 */
int psr_local_energy(const psr_model_desc* m, const float* theta, const psr_hamiltonian* H,
                     const int8_t* spins, int64_t B, int64_t chunk_seqs,
                     double* eloc, double* stats, float* logpsi,
                     void* ws, size_t ws_bytes, void* stream);

/*
 * Per-sample gradients O_s = d log psi(sigma_s) / d theta by a reverse-mode
 * adjoint of the row recurrence (reverse scan along each zigzag row).  The
 * forward keeps only the row frontier at checkpoint-chunk boundaries and each
 * chunk is recomputed before its reverse sweep.
 *   O       device float[B][P] or NULL   (out) one gradient row per sample
 *   logpsi  device float[B] or NULL      (out)
 *   w, g    device double[B], double[P]  both NULL or both set: g = sum_s w_s O_s (FP64)
 * At least one of O and g must be set.  The backward runs in FP32 whatever
 * m->precision is: O is the gradient of the FP32 model (and logpsi its value).
 */
int psr_logpsi_backward(const psr_model_desc* m, const float* theta, const int8_t* spins, int64_t B,
                        float* O, float* logpsi, const double* w, double* g,
                        void* ws, size_t ws_bytes, void* stream);

/*
 * VMC weights of the energy-gradient estimator (Sec. III.B, stochastic energy
 * gradient with real psi): w_s = (2 / B) (E_loc(s) - mean), mean = stats[0].
 * With these weights psr_logpsi_backward's g is the gradient estimate
 * (2/B) sum_s (E_loc(s) - mean) O_s.   eloc, stats, w: device doubles.
 */
int psr_vmc_weights(const double* eloc, const double* stats, int64_t B, double* w, void* stream);

/*
 * The energy-gradient estimate (Sec. III.B) from per-sample gradient rows that
 * psr_logpsi_backward returned earlier: g[p] = sum_s w[s] O[s][p], summed in
 * FP64 in the same order as the fused path of psr_logpsi_backward (equal
 * results).  It lets O be computed before the weights are known, e.g. on a
 * second stream while psr_local_energy runs.
 *   O   device float[B][P]    w   device double[B]    g   device double[P] (out)
 */
int psr_gradient_estimate(const float* O, int64_t B, int64_t P, const double* w, double* g, void* stream);

/*
 * Exact autoregressive samples (Sec. III.B: p(sigma) = prod_t p(sigma_t | sigma_<t),
 * sites in the zigzag order of Sec. II.F): site by site, every layer of the
 * model runs at the site on the spins drawn so far and
 *     sigma_t = 1  iff  uniforms[b][t] < p(sigma_t = 1 | sigma_<t),
 * with p computed in float32 (the sampler runs in FP32 whatever m->precision
 * is).  The random numbers are the caller's: equal uniforms give equal samples.
 * Both geometries (the chain visits its sites left to right).
 *   theta      device, float[P]
 *   uniforms   device, float[B][N] in [0, 1), lattice row-major (site y * lx + x)
 *   spins      device, int8[B][N]     (out) the samples, lattice row-major
 *   logpsi     device, float[B]       (out) log psi of each sample (FP32 model)
 *   ws         device workspace of psr_workspace_bytes(m, PSR_OP_SAMPLE, B, 0) bytes
 */
int psr_sample(const psr_model_desc* m, const float* theta, const float* uniforms, int64_t B,
               int8_t* spins, float* logpsi, void* ws, size_t ws_bytes, void* stream);

/* Synchronous check of a spin batch: PSR_OK if every value is 0 or 1, PSR_EDATA otherwise.
 *   spins  device int8[n_values]
 *   flag   device int32[1], caller-owned scratch (overwritten; the call allocates nothing)
 * The call queues the check on `stream` and waits for it. */
int psr_check_spins(const int8_t* spins, int64_t n_values, int32_t* flag, void* stream);

/* ---- 1D LRU ansatz (Sec. II.B, Eq. (lru); residual with GLU, Sec. II.G) -- */

typedef struct {
    int32_t n;          /* chain length N, 1 .. 16384 */
    int32_t n_layers;   /* 1 .. 8 */
    int32_t d;          /* width of each layer's input and output: a multiple of 16 in 16 .. 256 */
    int32_t d_h;        /* complex hidden units per layer: a multiple of 16 in 16 .. 256 */
} psr_lru_desc;

/*
 * Parameter layout (one flat float vector; matrices row-major, output index first):
 *   E[d][2]                 embedding of the previous spin: the layer-0 input at
 *                           site t is E[:, sigma_{t-1}], zero at t = 0
 *   for each layer l:
 *     nu[d_h], theta[d_h], gamma[d_h]   lambda = exp(-e^nu + i e^theta); drive scale e^gamma
 *     B[2 d_h][d]           rows 0..d_h-1 the real part, then the imaginary part
 *     D[d]
 *     C[d][2 d_h]           columns 0..d_h-1 the real part, then the imaginary part
 *     W_glu[2 d][d], b_glu[2 d]   rows 0..d-1 the GLU value projection, then its gate
 *   W_o[2][d], b_o[2]       two-way softmax head on the last layer's output
 * With 3 layers and d = d_h = 64 this is 75,138 parameters (Table I: about 75,000).
 */
int64_t psr_lru_param_count(const psr_lru_desc* m);   /* P, or a negative code */

/* Device workspace bytes that psr_lru_logpsi needs for `batch` chains; negative on error. */
int64_t psr_lru_workspace_bytes(const psr_lru_desc* m, int64_t batch);

/*
 * log psi of a batch of chains under the 1D LRU ansatz.  Per layer
 *   h_t = lambda h_{t-1} + e^gamma (B x_t),  h_{-1} = 0,   y_t = Re(C h_t) + D x_t,
 *   x'_t = (W_a y_t + b_a) sigmoid(W_g y_t + b_g) + [l >= 1] x_t,
 * then log psi = 1/2 sum_t log p(sigma_t | sigma_<t) from the head (Sec. III.B).
 * The recurrence runs as a chunked parallel scan over the chain (Sec. II.B); all
 * arithmetic is FP32 (FP32 MFMA for the projections), the final sum FP64.
 *   theta      device, float[P]
 *   spins      device, int8[B][N] with values in {0, 1} (only the low bit is read;
 *              psr_check_spins validates a batch)
 *   logpsi     device, float[B]               (out)
 *   logp_site  device, float[B][N] or NULL    (out) log p of each site
 *   ws         device workspace of psr_lru_workspace_bytes(m, B) bytes, owned by the caller
 * Errors: PSR_EINVAL (descriptor or pointer), PSR_ENOMEM (workspace too small),
 * PSR_EDEVICE (launch).  The work is queued on `stream`; the call does not wait for it.
 * Forward timing (psr_timing_begin) covers this kernel's launches too.
 */
int psr_lru_logpsi(const psr_lru_desc* m, const float* theta, const int8_t* spins, int64_t B,
                   float* logpsi, float* logp_site, void* ws, size_t ws_bytes, void* stream);

/*
 * Local energies of a batch of chains under the 1D LRU ansatz (the E_loc of
 * Sec. III.B: E_loc(sigma) = sum_sigma' H(sigma, sigma') psi(sigma') / psi(sigma)),
 * with their FP64 mean and variance (1/B).  H is PSR_TFIM or PSR_HEISENBERG on an
 * open chain (lx = n, ly = 1).  The connected configurations are enumerated in the
 * order of psr_connected, written out in full, and evaluated by the kernel of
 * psr_lru_logpsi; the ratio sum runs in FP64.
 *   theta   device, float[P];  spins  device, int8[B][n] in {0, 1}
 *   eloc    device, double[B]  (out);  stats  device, double[2] = (mean, variance) (out)
 *   logpsi  device, float[B] or NULL (out) log psi of the samples
 *   ws      device workspace of psr_lru_eloc_workspace_bytes(m, H, B) bytes, owned by the caller
 *           (it holds every connected configuration: B * max_connected * n bytes among the rest)
 * Errors: PSR_EINVAL (descriptors, lattice mismatch, NULL pointer), PSR_EUNSUPPORTED
 * (periodic boundaries), PSR_ENOMEM (workspace too small), PSR_EDEVICE (launch).
 * Queued on `stream`; the call does not wait for it.
 */
int64_t psr_lru_eloc_workspace_bytes(const psr_lru_desc* m, const psr_hamiltonian* H, int64_t batch);
int psr_lru_local_energy(const psr_lru_desc* m, const float* theta, const psr_hamiltonian* H, const int8_t* spins,
                         int64_t B, double* eloc, double* stats, float* logpsi, void* ws, size_t ws_bytes,
                         void* stream);

/*
 * Device workspace bytes of an LRU call for `batch` chains: op = PSR_OP_LOGPSI
 * (psr_lru_logpsi, as psr_lru_workspace_bytes), PSR_OP_SAMPLE (psr_lru_sample)
 * or PSR_OP_BACKWARD (psr_lru_backward with O = NULL; with O given, fewer
 * bytes suffice).  Negative on error.
 */
int64_t psr_lru_op_workspace_bytes(const psr_lru_desc* m, int32_t op, int64_t batch);

/*
 * Exact autoregressive samples of chains under the LRU ansatz (Sec. III.B:
 * p(sigma) = prod_t p(sigma_t | sigma_<t), sites left to right):
 *     sigma_t = 1  iff  uniforms[b][t] < p(sigma_t = 1 | sigma_<t),
 * p from the model's two-way head in FP32.  Equal uniforms give equal samples.
 *   theta     device float[P];  uniforms  device float[B][n] in [0, 1)
 *   spins     device int8[B][n]  (out);  logpsi  device float[B]  (out)
 *   ws        device workspace of psr_lru_op_workspace_bytes(m, PSR_OP_SAMPLE, B) bytes
 * Errors: PSR_EINVAL, PSR_ENOMEM (workspace too small), PSR_EDEVICE.  Queued on `stream`.
 */
int psr_lru_sample(const psr_lru_desc* m, const float* theta, const float* uniforms, int64_t B, int8_t* spins,
                   float* logpsi, void* ws, size_t ws_bytes, void* stream);

/*
 * Per-sample gradients O_s = d log psi(sigma_s) / d theta of the LRU ansatz
 * (Sec. II.B Eq. (lru), Sec. II.G; the VMC gradient of Sec. III.B): the forward
 * over each chain is recomputed and swept in reverse, the complex recurrence by
 * the reverse scan Ghat_t = G_t + conj(lambda) Ghat_{t+1}.  FP32.
 *   spins   device int8[B][n] in {0, 1}
 *   O       device float[B][P] or NULL   (out) one gradient row per chain, parameter layout
 *   logpsi  device float[B] or NULL      (out)
 *   w, g    device double[B], double[P]  both NULL or both set: g = sum_s w_s O_s (FP64)
 *   ws      device workspace of psr_lru_op_workspace_bytes(m, PSR_OP_BACKWARD, B) bytes
 * At least one of O and g must be set.  Errors as psr_lru_sample.
 */
int psr_lru_backward(const psr_lru_desc* m, const float* theta, const int8_t* spins, int64_t B, float* O,
                     float* logpsi, const double* w, double* g, void* ws, size_t ws_bytes, void* stream);

/* ---- layout query ------------------------------------------------------- */

/*
 * Launch layout of the forward kernel for a model (for tools and tests that
 * check the kernels' addressing on the host).  shape[0..8] = columns per
 * workgroup, sequences per workgroup, 16-column tiles per wave, waves per
 * workgroup, 1 if a sequence row may straddle waves, 1 if the row frontier is
 * kept in LDS, 1 for the units-split kernel, sequences per forward launch of
 * psr_logpsi for `batch` samples, and frontier bytes per sequence.
 */
int psr_forward_shape(const psr_model_desc* m, int64_t batch, int64_t* shape);

/* ---- measurement -------------------------------------------------------- */

/* Timing of the forward (log psi) kernel, for measurement tools.  After
 * psr_timing_begin(), every forward-kernel launch that this thread queues is
 * bracketed by two HIP events recorded on the launch's stream.
 * psr_timing_end() waits for those events, returns the summed kernel time in
 * milliseconds and the number of launches, and stops recording.  Two event
 * records per launch are the only overhead. */
int psr_timing_begin(void);
int psr_timing_end(double* total_ms, int64_t* launches);

/* Message of the last failing call on this thread ("" if none). */
const char* psr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PSR_H */
