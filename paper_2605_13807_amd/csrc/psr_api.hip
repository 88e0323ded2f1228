// libpsr C ABI: argument checks, parameter/workspace layouts and dispatch.
// Every compute step runs in the kernels of psr_fwd.hip, psr_ham.hip and
// psr_bwd.hip; this file only validates, carves the caller's workspace and
// queues launches on the caller's stream.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/psr.h"
#include "psr_internal.h"

namespace psr {

static thread_local char g_err[512] = "";

static int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

static int ok() {
    g_err[0] = 0;
    return PSR_OK;
}

static int dev_check(int e, const char* what) {
    if (e != 0) return fail(PSR_EDEVICE, "%s: HIP error %d (%s)", what, e, hipGetErrorString((hipError_t)e));
    return PSR_OK;
}

// ---------------------------------------------------------------------------
// model checks and layouts
// ---------------------------------------------------------------------------

static int check_model(const psr_model_desc* m, Geom* out) {
    if (!m) return fail(PSR_EINVAL, "model descriptor is NULL");
    if (m->geometry != PSR_CHAIN_1D && m->geometry != PSR_SNAKE_2D)
        return fail(PSR_EINVAL, "geometry %d is not PSR_CHAIN_1D or PSR_SNAKE_2D", m->geometry);
    if (m->lx < 1 || m->ly < 1) return fail(PSR_EINVAL, "lattice %d x %d is empty", m->lx, m->ly);
    if ((int64_t)m->lx * m->ly > 65535) return fail(PSR_EUNSUPPORTED, "more than 65535 sites");
    if (m->geometry == PSR_CHAIN_1D && (m->ly != 1 || m->n_layers != 1))
        return fail(PSR_EINVAL, "the chain ansatz needs ly = 1 and n_layers = 1");
    if (m->n_layers < 1 || m->n_layers > 8) return fail(PSR_EINVAL, "n_layers %d outside [1, 8]", m->n_layers);
    if (m->d != 32 && m->d != 64 && m->d != 128 && m->d != 256)
        return fail(PSR_EUNSUPPORTED, "hidden size %d is not 32, 64, 128 or 256", m->d);
    if (m->precision != PSR_FP32 && m->precision != PSR_BF16 && m->precision != PSR_FP16)
        return fail(PSR_EINVAL, "precision %d is not PSR_FP32, PSR_BF16 or PSR_FP16", m->precision);
    if (m->ckpt_rows < 0) return fail(PSR_EINVAL, "ckpt_rows must be >= 0");
    const int patch = m->patch == 0 ? 1 : m->patch;
    if (patch != 1 && patch != 2) return fail(PSR_EINVAL, "patch %d is not 1 or 2", m->patch);
    if (patch == 2 && (m->geometry != PSR_SNAKE_2D || m->lx % 2 || m->ly % 2))
        return fail(PSR_EINVAL, "2x2 patches need the 2D snake on even lattice sides (got %d x %d)", m->lx, m->ly);
    if (m->symmetry != PSR_SYM_NONE && m->symmetry != PSR_SYM_C4V)
        return fail(PSR_EINVAL, "symmetry %d is not PSR_SYM_NONE or PSR_SYM_C4V", m->symmetry);
    if (m->symmetry == PSR_SYM_C4V && (m->geometry != PSR_SNAKE_2D || m->lx != m->ly))
        return fail(PSR_EINVAL, "c4v symmetry needs a square 2D lattice (got %d x %d)", m->lx, m->ly);
    Geom g;
    g.chain = (m->geometry == PSR_CHAIN_1D);
    g.patch = patch;
    g.slx = m->lx;
    g.sly = m->ly;
    g.lx = m->lx / patch;
    g.ly = m->ly / patch;
    g.nl = m->n_layers;
    g.d = m->d;
    g.prec = m->precision == PSR_BF16 ? kBF16 : (m->precision == PSR_FP16 ? kFP16 : kFP32);
    g.sym = m->symmetry == PSR_SYM_C4V ? 1 : 0;
    const FwdShape sh = fwd_shape(g);
    if (sh.seqs < 1)
        return fail(PSR_EUNSUPPORTED, "row length %d exceeds the %d columns of a workgroup at d = %d", g.lx, sh.cols,
                    g.d);
    if (out) *out = g;
    return PSR_OK;
}

int64_t param_count(const Geom& g) {
    int64_t off[64];
    int32_t n = 0;
    param_offsets(g, off, &n);
    return off[n];
}

void param_offsets(const Geom& g, int64_t* off, int32_t* n) {
    const int64_t d = g.d;
    int k = 0;
    int64_t p = 0;
    auto add = [&](int64_t sz) {
        off[k++] = p;
        p += sz;
    };
    if (g.chain) {
        add(d * 2);   // W_z
        add(d);       // b_z
        add(d * 2);   // W_h
        add(d);       // b_h
    } else {
        for (int l = 0; l < g.nl; ++l) {
            const int64_t du = (l == 0) ? 2 * n_states(g) : d;
            add(d * du);          // W_z
            add(d);               // b_z
            add(d * (du + d));    // W_h
            add(d);               // b_h
            add(d * d);           // C
            add(d * du);          // D
        }
    }
    add(n_states(g) * d);   // W_o
    add(n_states(g));       // b_o
    off[k] = p;
    *n = k;
}

Prepared prepared_layout(const Geom& g) {
    Prepared pl;
    const int64_t d = g.d;
    const int64_t mat = d * d * 4;   // FP32 values, or 16-bit high and low parts
    int64_t fb = 0;
    // absent matrices keep offset 0 (never read) so that pointer arithmetic stays in range
    for (int l = 0; l < 8; ++l)
        for (int m = 0; m < 5; ++m) {
            pl.frag[l][m] = 0;
            pl.frag_present[l][m] = 0;
        }
    if (!g.chain) {
        for (int l = 0; l < g.nl; ++l) {
            for (int m = 0; m < 5; ++m) {
                const bool present = (l == 0) ? (m == 2 || m == 4) : true;
                if (present) {
                    pl.frag[l][m] = fb;
                    pl.frag_present[l][m] = 1;
                    fb += mat;
                }
            }
        }
    }
    pl.frag_bytes = fb > 0 ? fb : 256;
    int64_t t = 0;
    const int64_t nst = (int64_t)(n_states(g) + 1) * (n_states(g) + 1);   // (H-pred, V-pred) states, 'outside' included
    pl.t0z = t; t += nst * d;
    pl.t0h = t; t += nst * d;
    pl.t0d = t; t += nst * d;
    for (int l = 0; l < 8; ++l) {
        pl.bias_z[l] = 0;
        pl.bias_h[l] = 0;
    }
    for (int l = 1; l < g.nl; ++l) {
        pl.bias_z[l] = t; t += d;
        pl.bias_h[l] = t; t += d;
    }
    // two classes: the logit difference only; 16 classes: every row of the head
    pl.head_w = t; t += (n_states(g) == 2 ? 1 : n_states(g)) * d;
    pl.head_b = t; t += n_states(g) == 2 ? 4 : n_states(g);
    pl.table_floats = t;
    return pl;
}

static int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Workspace carving: a sequence of 256-byte aligned regions.
struct Carver {
    uint8_t* base;
    int64_t used = 0;
    explicit Carver(void* b) : base(reinterpret_cast<uint8_t*>(b)) {}
    template <class T>
    T* take(int64_t count) {
        T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
        used += align256(count * (int64_t)sizeof(T));
        return p;
    }
};

// Per-sequence device scratch of the forward kernel: the row frontier h^(l)
// of every layer (the next row's h_V), in the projections' operand type.
static int64_t frontier_seq_bytes(const Geom& g) {
    return (int64_t)g.nl * g.lx * g.d * 4;   // FP32 values, or 16-bit high and low parts
}

// sequences per forward launch for psr_logpsi (bounds the frontier workspace to ~256 MB)
static int64_t logpsi_chunk(const Geom& g, int64_t B) {
    const int64_t per = frontier_seq_bytes(g);
    int64_t c = (256ll << 20) / (per > 0 ? per : 1);
    if (c < 1024) c = 1024;
    return B < c ? B : c;
}

struct LogpsiWs {
    uint32_t* packed;
    uint8_t* frag;
    float* tab;
    void* frontier;
    float* hi;
    float* lo;
    float *hi8, *lo8;   // c4v: log psi of the eight transformed batches, [8][B]
    int64_t chunk;
};

static int64_t carve_logpsi(const Geom& g, int64_t B, void* ws, LogpsiWs* w) {
    Carver c(ws);
    const Prepared pl = prepared_layout(g);
    const int words = (g.slx * g.sly + 31) / 32;
    w->chunk = logpsi_chunk(g, B);
    w->packed = c.take<uint32_t>(B * words);
    w->frag = c.take<uint8_t>(pl.frag_bytes);
    w->tab = c.take<float>(pl.table_floats);
    w->frontier = c.take<uint8_t>(w->chunk * frontier_seq_bytes(g));
    w->hi = c.take<float>(B);
    w->lo = c.take<float>(B);
    w->hi8 = g.sym ? c.take<float>(8 * B) : nullptr;
    w->lo8 = g.sym ? c.take<float>(8 * B) : nullptr;
    return c.used;
}

struct ElocWs {
    uint32_t* packed;
    uint8_t* frag;
    float* tab;
    void* frontier;
    int32_t* n_conn;
    float* diag;
    int64_t* offs;
    uint32_t* desc;
    float* mel;
    float *chi, *clo, *shi, *slo;
    float *chi8, *clo8, *shi8, *slo8;   // c4v: the eight transformed evaluations, [8][M] and [8][B]
};

static int64_t carve_eloc(const Geom& g, int64_t B, int64_t max_conn, int64_t chunk, void* ws, ElocWs* w) {
    Carver c(ws);
    const Prepared pl = prepared_layout(g);
    const int words = (g.slx * g.sly + 31) / 32;
    const int64_t M = B * max_conn;
    w->packed = c.take<uint32_t>(B * words);
    w->frag = c.take<uint8_t>(pl.frag_bytes);
    w->tab = c.take<float>(pl.table_floats);
    w->frontier = c.take<uint8_t>(chunk * frontier_seq_bytes(g));
    w->n_conn = c.take<int32_t>(B);
    w->diag = c.take<float>(B);
    w->offs = c.take<int64_t>(B + 1);
    w->desc = c.take<uint32_t>(2 * M);
    w->mel = c.take<float>(M);
    w->chi = c.take<float>(M);
    w->clo = c.take<float>(M);
    w->shi = c.take<float>(B);
    w->slo = c.take<float>(B);
    w->chi8 = g.sym ? c.take<float>(8 * M) : nullptr;
    w->clo8 = g.sym ? c.take<float>(8 * M) : nullptr;
    w->shi8 = g.sym ? c.take<float>(8 * B) : nullptr;
    w->slo8 = g.sym ? c.take<float>(8 * B) : nullptr;
    return c.used;
}

struct BwdWs {
    uint32_t* packed;
    float* scratch;
    float* O;
};

static int64_t carve_bwd(const Geom& g, int ckpt_rows, int64_t B, bool need_O, void* ws, BwdWs* w) {
    Carver c(ws);
    const BwdLayout bl = bwd_layout(g, ckpt_rows);
    const int words = (g.slx * g.sly + 31) / 32;
    w->packed = c.take<uint32_t>(B * words);
    w->scratch = c.take<float>(B * bl.ws_per_sample_floats);
    w->O = need_O ? c.take<float>(B * param_count(g)) : nullptr;
    return c.used;
}

static int check_ham(const psr_hamiltonian* H, Ham* out) {
    if (!H) return fail(PSR_EINVAL, "Hamiltonian descriptor is NULL");
    if (H->kind != PSR_TFIM && H->kind != PSR_HEISENBERG)
        return fail(PSR_EINVAL, "Hamiltonian kind %d is not PSR_TFIM or PSR_HEISENBERG", H->kind);
    if (H->lx < 1 || H->ly < 1) return fail(PSR_EINVAL, "lattice %d x %d is empty", H->lx, H->ly);
    if ((int64_t)H->lx * H->ly > 65535) return fail(PSR_EUNSUPPORTED, "more than 65535 sites");
    if (H->pbc != 0) return fail(PSR_EUNSUPPORTED, "periodic boundaries are not supported (the paper uses open ones)");
    if (!std::isfinite(H->J) || !std::isfinite(H->h)) return fail(PSR_EINVAL, "couplings must be finite");
    Ham h;
    h.kind = H->kind == PSR_TFIM ? 0 : 1;
    h.lx = H->lx;
    h.ly = H->ly;
    h.marshall = H->marshall ? 1 : 0;
    h.J = (float)H->J;
    h.h = (float)H->h;
    if (out) *out = h;
    return PSR_OK;
}

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Forward-kernel timing (psr_timing_begin / psr_timing_end).
struct TimingState {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
};
static thread_local TimingState g_tm;

static void timing_before(hipStream_t st, hipEvent_t* stop) {
    *stop = nullptr;
    if (!g_tm.on) return;
    if (g_tm.used == g_tm.ev.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);   // cleanup; the launch goes untimed
            return;
        }
        g_tm.ev.emplace_back(a, b);
    }
    auto& p = g_tm.ev[g_tm.used];
    if (hipEventRecord(p.first, st) != hipSuccess) return;   // this launch goes untimed
    ++g_tm.used;
    *stop = p.second;
}

static int run_forward(const Geom& g, const Prepared& pl, const uint32_t* packed, const uint32_t* desc,
                       int64_t q_begin, int64_t q_count, const int64_t* q_total, const uint8_t* frag, const float* tab,
                       void* frontier, float* hi, float* lo, float* logp_site, hipStream_t st, int xform = 0) {
    FwdArgs a;
    a.g = g;
    a.spins = packed;
    a.words_per_seq = (g.slx * g.sly + 31) / 32;
    a.desc = desc;
    a.q_begin = q_begin;
    a.q_count = q_count;
    a.q_total = q_total;
    a.frag = frag;
    a.tab = tab;
    a.pl = pl;
    a.sh = fwd_shape(g);
    a.frontier = frontier;
    a.out_hi = hi;
    a.out_lo = lo;
    a.logp_site = logp_site;
    a.xform = xform;
    hipEvent_t stop;
    timing_before(st, &stop);
    const int e = launch_forward(a, st);
    if (stop && hipEventRecord(stop, st) != hipSuccess) {
        // the start event of this pair is recorded but not the stop: drop the pair
        --g_tm.used;
    }
    return e;
}

// ---------------------------------------------------------------------------
// Static device scratch of psr_logpsi_static (callers that cannot allocate)
// ---------------------------------------------------------------------------

// Each GPU the library runs on holds one copy of this array until the process
// ends.  Host code must not pass its name to a kernel (that is a host-side
// stand-in, not a device address): its address on the current device comes
// from hipGetSymbolAddress, once per device, below.
constexpr size_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;   // per device, filled on the first call on that device

static int static_scratch(void** out) {
    int dev = 0;
    int r = dev_check((int)hipGetDevice(&dev), "current device");
    if (r) return r;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if ((r = dev_check((int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "static scratch address"))) return r;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PSR_OK;
}

}  // namespace psr

using namespace psr;

extern "C" {

const char* psr_last_error(void) { return g_err; }

int psr_timing_begin(void) {
    g_tm.on = true;
    g_tm.used = 0;
    return ok();
}

int psr_timing_end(double* total_ms, int64_t* launches) {
    if (!total_ms || !launches) return fail(PSR_EINVAL, "total_ms and launches must not be NULL");
    double t = 0.0;
    int r = PSR_OK;
    for (size_t k = 0; k < g_tm.used && !r; ++k) {
        float ms = 0.0f;
        r = dev_check((int)hipEventSynchronize(g_tm.ev[k].second), "timing sync");
        if (!r) r = dev_check((int)hipEventElapsedTime(&ms, g_tm.ev[k].first, g_tm.ev[k].second), "timing read");
        t += ms;
    }
    *total_ms = t;
    *launches = (int64_t)g_tm.used;
    g_tm.on = false;
    g_tm.used = 0;
    return r ? r : ok();
}

int64_t psr_param_count(const psr_model_desc* m) {
    Geom g;
    const int r = check_model(m, &g);
    if (r) return r;
    ok();
    return param_count(g);
}

int psr_param_offsets(const psr_model_desc* m, int64_t* offsets, int32_t* n_tensors) {
    Geom g;
    const int r = check_model(m, &g);
    if (r) return r;
    if (!offsets || !n_tensors) return fail(PSR_EINVAL, "offsets and n_tensors must not be NULL");
    int64_t off[64];
    int32_t n = 0;
    param_offsets(g, off, &n);
    for (int k = 0; k <= n; ++k) offsets[k] = off[k];
    *n_tensors = n;
    return ok();
}

int64_t psr_max_connected(const psr_hamiltonian* H) {
    Ham h;
    const int r = check_ham(H, &h);
    if (r) return r;
    ok();
    return ham_max_connected(h);
}

int64_t psr_workspace_bytes(const psr_model_desc* m, int32_t op, int64_t batch, int64_t chunk_seqs) {
    Geom g;
    const int r = check_model(m, &g);
    if (r) return r;
    if (batch < 0) return fail(PSR_EINVAL, "negative batch");
    if (chunk_seqs < 0) return fail(PSR_EINVAL, "negative chunk_seqs");
    ok();
    if (op == PSR_OP_LOGPSI) {
        LogpsiWs w;
        return carve_logpsi(g, batch, nullptr, &w);
    }
    if (op == PSR_OP_LOCAL_ENERGY) {
        psr_hamiltonian H;
        std::memset(&H, 0, sizeof(H));
        H.kind = PSR_HEISENBERG;
        H.lx = g.slx;
        H.ly = g.sly;
        Ham h;
        check_ham(&H, &h);
        int64_t mc = ham_max_connected(h);
        if ((int64_t)g.slx * g.sly > mc) mc = (int64_t)g.slx * g.sly;   // enough for either Hamiltonian
        ElocWs w;
        const int64_t ch = chunk_seqs > 0 ? chunk_seqs : 32768;
        return carve_eloc(g, batch, mc, ch, nullptr, &w);
    }
    if (op == PSR_OP_BACKWARD) {
        BwdWs w;
        return carve_bwd(g, m->ckpt_rows, batch, true, nullptr, &w);
    }
    if (op == PSR_OP_SAMPLE) {
        return sample_groups(batch) * sample_ws_per_wg_floats(g) * (int64_t)sizeof(float);
    }
    return fail(PSR_EINVAL, "unknown op %d", op);
}

int psr_logpsi(const psr_model_desc* m, const float* theta, const int8_t* spins, int64_t B, float* logpsi,
               float* logp_site, void* ws, size_t ws_bytes, void* stream) {
    Geom g;
    int r = check_model(m, &g);
    if (r) return r;
    if (B < 0) return fail(PSR_EINVAL, "negative batch");
    if (B == 0) return ok();
    if (!theta || !spins || !logpsi) return fail(PSR_EINVAL, "theta, spins and logpsi must not be NULL");
    if (g.sym && logp_site) return fail(PSR_EINVAL, "per-site log p is not defined for a symmetrised wave function");
    LogpsiWs w;
    const int64_t need = carve_logpsi(g, B, nullptr, &w);
    if (!ws || (int64_t)ws_bytes < need)
        return fail(PSR_ENOMEM, "workspace of %zu bytes is smaller than the %lld needed", ws_bytes, (long long)need);
    carve_logpsi(g, B, ws, &w);
    hipStream_t st = as_stream(stream);
    const Prepared pl = prepared_layout(g);
    const int N = g.slx * g.sly;   // spins per sample
    if ((r = dev_check(launch_pack_spins(spins, B, N, w.packed, st), "pack"))) return r;
    if ((r = dev_check(launch_prepare(g, pl, theta, w.frag, w.tab, st), "prepare"))) return r;
    // c4v: the batch read as sigma o T_k for k = 0..7, combined below
    const int nx = g.sym ? 8 : 1;
    for (int k = 0; k < nx; ++k) {
        float* hi = g.sym ? w.hi8 + (size_t)k * B : w.hi;
        float* lo = g.sym ? w.lo8 + (size_t)k * B : w.lo;
        for (int64_t q0 = 0; q0 < B; q0 += w.chunk) {
            const int64_t n = (B - q0 < w.chunk) ? B - q0 : w.chunk;
            if ((r = dev_check(run_forward(g, pl, w.packed, nullptr, q0, n, nullptr, w.frag, w.tab, w.frontier, hi, lo,
                                           logp_site, st, k),
                               "forward")))
                return r;
        }
    }
    if (g.sym && (r = dev_check(launch_c4v_combine(w.hi8, w.lo8, B, w.hi, w.lo, st), "c4v combine"))) return r;
    if ((r = dev_check(launch_combine_logpsi(w.hi, w.lo, B, logpsi, st), "combine"))) return r;
    return ok();
}

int psr_forward_shape(const psr_model_desc* m, int64_t batch, int64_t* shape) {
    Geom g;
    const int r = check_model(m, &g);
    if (r) return r;
    if (!shape) return fail(PSR_EINVAL, "shape must not be NULL");
    if (batch < 0) return fail(PSR_EINVAL, "negative batch");
    const FwdShape sh = fwd_shape(g);
    shape[0] = sh.cols;
    shape[1] = sh.seqs;
    shape[2] = sh.ntc;
    shape[3] = sh.waves;
    shape[4] = sh.cross_wave;
    shape[5] = sh.lds_frontier;
    shape[6] = sh.split_kernel;
    shape[7] = batch > 0 ? logpsi_chunk(g, batch) : 0;
    shape[8] = frontier_seq_bytes(g);
    return ok();
}

int64_t psr_static_scratch_bytes(void) { return (int64_t)kStaticScratchBytes; }

int psr_logpsi_static(const psr_model_desc* m, const float* theta, const int8_t* spins, int64_t B, float* logpsi,
                      float* logp_site, void* stream) {
    Geom g;
    int r = check_model(m, &g);
    if (r) return r;
    if (B < 0) return fail(PSR_EINVAL, "negative batch");
    if (B == 0) return ok();
    LogpsiWs w;
    const int64_t need = carve_logpsi(g, B, nullptr, &w);
    if (need > (int64_t)kStaticScratchBytes)
        return fail(PSR_ENOMEM, "a batch of %lld needs %lld bytes of scratch; the static scratch holds %lld",
                    (long long)B, (long long)need, (long long)kStaticScratchBytes);
    void* ws = nullptr;
    if ((r = static_scratch(&ws))) return r;
    // every region of the scratch is written before it is read (packed spins,
    // prepared weights, frontier rows, log psi halves): nothing to clear
    return psr_logpsi(m, theta, spins, B, logpsi, logp_site, ws, kStaticScratchBytes, stream);
}

int psr_connected(const psr_hamiltonian* H, const int8_t* spins, int64_t B, int64_t max_conn, int8_t* conn,
                  uint32_t* desc, float* mel, int32_t* n_conn, float* diag, void* stream) {
    Ham h;
    int r = check_ham(H, &h);
    if (r) return r;
    if (B < 0) return fail(PSR_EINVAL, "negative batch");
    if (B == 0) return ok();
    if (!spins || !n_conn) return fail(PSR_EINVAL, "spins and n_conn must not be NULL");
    if (conn && !desc) return fail(PSR_EINVAL, "conn output needs the desc output too");
    const int64_t need = ham_max_connected(h);
    if (max_conn < need)
        return fail(PSR_ECAPACITY, "max_conn %lld is below the %lld connected configurations a sample can have",
                    (long long)max_conn, (long long)need);
    hipStream_t st = as_stream(stream);
    if ((r = dev_check(launch_conn_count(h, spins, B, n_conn, diag, st), "connected count"))) return r;
    if (desc || mel) {
        if ((r = dev_check(launch_conn_write(h, spins, B, nullptr, max_conn, desc, mel, st), "connected write")))
            return r;
    }
    if (conn) {
        if ((r = dev_check(launch_conn_expand(spins, h.lx * h.ly, B, max_conn, n_conn, desc, conn, st),
                           "connected expand")))
            return r;
    }
    return ok();
}

int psr_local_energy(const psr_model_desc* m, const float* theta, const psr_hamiltonian* H, const int8_t* spins,
                     int64_t B, int64_t chunk_seqs, double* eloc, double* stats, float* logpsi, void* ws,
                     size_t ws_bytes, void* stream) {
    Geom g;
    int r = check_model(m, &g);
    if (r) return r;
    Ham h;
    if ((r = check_ham(H, &h))) return r;
    if (h.lx != g.slx || h.ly != g.sly)
        return fail(PSR_EINVAL, "Hamiltonian lattice %d x %d differs from the model's %d x %d", h.lx, h.ly, g.slx, g.sly);
    if (B < 0 || chunk_seqs < 0) return fail(PSR_EINVAL, "negative batch or chunk");
    if (B == 0) return ok();
    if (!theta || !spins || !eloc || !stats) return fail(PSR_EINVAL, "theta, spins, eloc and stats must not be NULL");
    const int64_t chunk = chunk_seqs > 0 ? chunk_seqs : 32768;
    const int64_t max_conn = ham_max_connected(h);
    ElocWs w;
    const int64_t need = carve_eloc(g, B, max_conn, chunk, nullptr, &w);
    if (!ws || (int64_t)ws_bytes < need)
        return fail(PSR_ENOMEM, "workspace of %zu bytes is smaller than the %lld needed", ws_bytes, (long long)need);
    carve_eloc(g, B, max_conn, chunk, ws, &w);
    hipStream_t st = as_stream(stream);
    const Prepared pl = prepared_layout(g);
    const int N = g.slx * g.sly;   // spins per sample
    if ((r = dev_check(launch_pack_spins(spins, B, N, w.packed, st), "pack"))) return r;
    if ((r = dev_check(launch_prepare(g, pl, theta, w.frag, w.tab, st), "prepare"))) return r;
    if ((r = dev_check(launch_conn_count(h, spins, B, w.n_conn, w.diag, st), "connected count"))) return r;
    if ((r = dev_check(launch_scan_counts(w.n_conn, B, w.offs, st), "scan"))) return r;
    if ((r = dev_check(launch_conn_write(h, spins, B, w.offs, 0, w.desc, w.mel, st), "connected write"))) return r;
    // c4v: every configuration is read as sigma o T_k for k = 0..7 and combined below
    const int nx = g.sym ? 8 : 1;
    const int64_t M = B * max_conn;
    for (int k = 0; k < nx; ++k) {
        float* shi = g.sym ? w.shi8 + (size_t)k * B : w.shi;
        float* slo = g.sym ? w.slo8 + (size_t)k * B : w.slo;
        float* chi = g.sym ? w.chi8 + (size_t)k * M : w.chi;
        float* clo = g.sym ? w.clo8 + (size_t)k * M : w.clo;
        // the samples themselves
        for (int64_t q0 = 0; q0 < B; q0 += chunk) {
            const int64_t n = (B - q0 < chunk) ? B - q0 : chunk;
            if ((r = dev_check(run_forward(g, pl, w.packed, nullptr, q0, n, nullptr, w.frag, w.tab, w.frontier, shi,
                                           slo, nullptr, st, k),
                               "forward (samples)")))
                return r;
        }
        // the connected configurations, streamed in chunks; launches past the
        // device-side total exit at once
        for (int64_t q0 = 0; q0 < M; q0 += chunk) {
            const int64_t n = (M - q0 < chunk) ? M - q0 : chunk;
            if ((r = dev_check(run_forward(g, pl, w.packed, w.desc, q0, n, w.offs + B, w.frag, w.tab, w.frontier, chi,
                                           clo, nullptr, st, k),
                               "forward (connected)")))
                return r;
        }
    }
    if (g.sym) {
        if ((r = dev_check(launch_c4v_combine(w.shi8, w.slo8, B, w.shi, w.slo, st), "c4v combine (samples)"))) return r;
        if ((r = dev_check(launch_c4v_combine(w.chi8, w.clo8, M, w.chi, w.clo, st), "c4v combine (connected)")))
            return r;
    }
    if ((r = dev_check(launch_eloc_combine(B, w.offs, w.diag, w.mel, w.chi, w.clo, w.shi, w.slo, eloc, st), "E_loc")))
        return r;
    if ((r = dev_check(launch_stats(eloc, B, stats, st), "stats"))) return r;
    if (logpsi && (r = dev_check(launch_combine_logpsi(w.shi, w.slo, B, logpsi, st), "combine"))) return r;
    return ok();
}

int psr_logpsi_backward(const psr_model_desc* m, const float* theta, const int8_t* spins, int64_t B, float* O,
                        float* logpsi, const double* w, double* gout, void* ws, size_t ws_bytes, void* stream) {
    Geom g;
    int r = check_model(m, &g);
    if (r) return r;
    if (B < 0) return fail(PSR_EINVAL, "negative batch");
    if (B == 0) return ok();
    if (!theta || !spins) return fail(PSR_EINVAL, "theta and spins must not be NULL");
    if ((w == nullptr) != (gout == nullptr)) return fail(PSR_EINVAL, "w and g must be both set or both NULL");
    if (g.patch != 1 || g.sym)
        return fail(PSR_EUNSUPPORTED, "the backward covers single-site inputs without symmetrisation");
    if (!O && !gout) return fail(PSR_EINVAL, "nothing to compute: O and g are both NULL");
    BwdWs bw;
    const int64_t need = carve_bwd(g, m->ckpt_rows, B, O == nullptr, nullptr, &bw);
    if (!ws || (int64_t)ws_bytes < need)
        return fail(PSR_ENOMEM, "workspace of %zu bytes is smaller than the %lld needed", ws_bytes, (long long)need);
    carve_bwd(g, m->ckpt_rows, B, O == nullptr, ws, &bw);
    hipStream_t st = as_stream(stream);
    const int N = g.slx * g.sly;   // spins per sample
    const int words = (N + 31) / 32;
    float* Ouse = O ? O : bw.O;
    const BwdLayout bl = bwd_layout(g, m->ckpt_rows);
    if ((r = dev_check(launch_pack_spins(spins, B, N, bw.packed, st), "pack"))) return r;
    if ((r = dev_check(launch_backward(g, bl, theta, bw.packed, words, B, nullptr, bw.scratch, Ouse, logpsi, st),
                       "backward")))
        return r;
    if (gout && (r = dev_check(launch_weighted_sum(Ouse, B, param_count(g), w, gout, st), "gradient sum"))) return r;
    return ok();
}

int psr_sample(const psr_model_desc* m, const float* theta, const float* uniforms, int64_t B, int8_t* spins,
               float* logpsi, void* ws, size_t ws_bytes, void* stream) {
    Geom g;
    int r = check_model(m, &g);
    if (r) return r;
    if (B < 0) return fail(PSR_EINVAL, "negative batch");
    if (B == 0) return ok();
    if (!theta || !uniforms || !spins || !logpsi) return fail(PSR_EINVAL, "theta, uniforms, spins and logpsi must not be NULL");
    if (g.patch != 1 || g.sym)
        return fail(PSR_EUNSUPPORTED, "the sampler covers single-site inputs without symmetrisation");
    const int64_t need = sample_groups(B) * sample_ws_per_wg_floats(g) * (int64_t)sizeof(float);
    if (!ws || (int64_t)ws_bytes < need)
        return fail(PSR_ENOMEM, "workspace of %zu bytes is smaller than the %lld needed", ws_bytes, (long long)need);
    if ((r = dev_check(launch_sample(g, theta, uniforms, B, spins, logpsi, reinterpret_cast<float*>(ws),
                                     as_stream(stream)),
                       "sample")))
        return r;
    return ok();
}

int psr_gradient_estimate(const float* O, int64_t B, int64_t P, const double* w, double* g, void* stream) {
    if (B < 0 || P < 0) return fail(PSR_EINVAL, "negative size");
    if (P == 0) return ok();
    if (!g) return fail(PSR_EINVAL, "g must not be NULL");
    if (B > 0 && (!O || !w)) return fail(PSR_EINVAL, "O and w must not be NULL");
    int r;
    if ((r = dev_check(launch_weighted_sum(O, B, P, w, g, as_stream(stream)), "gradient sum"))) return r;
    return ok();
}

int psr_vmc_weights(const double* eloc, const double* stats, int64_t B, double* w, void* stream) {
    if (B < 0) return fail(PSR_EINVAL, "negative batch");
    if (B == 0) return ok();
    if (!eloc || !stats || !w) return fail(PSR_EINVAL, "eloc, stats and w must not be NULL");
    int r;
    if ((r = dev_check(launch_vmc_weights(eloc, stats, B, w, as_stream(stream)), "weights"))) return r;
    return ok();
}

static int check_lru(const psr_lru_desc* m, LruGeom* g) {
    if (!m) return fail(PSR_EINVAL, "LRU descriptor is NULL");
    if (m->n < 1 || m->n > 16384) return fail(PSR_EINVAL, "chain length %d outside [1, 16384]", m->n);
    if (m->n_layers < 1 || m->n_layers > 8) return fail(PSR_EINVAL, "n_layers %d outside [1, 8]", m->n_layers);
    if (m->d < 16 || m->d > 256 || m->d % 16) return fail(PSR_EINVAL, "d = %d is not a multiple of 16 in [16, 256]", m->d);
    if (m->d_h < 16 || m->d_h > 256 || m->d_h % 16)
        return fail(PSR_EINVAL, "d_h = %d is not a multiple of 16 in [16, 256]", m->d_h);
    g->n = m->n;
    g->nl = m->n_layers;
    g->d = m->d;
    g->dh = m->d_h;
    return PSR_OK;
}

int64_t psr_lru_param_count(const psr_lru_desc* m) {
    LruGeom g;
    const int r = check_lru(m, &g);
    if (r) return r;
    ok();
    return lru_param_count(g);
}

int64_t psr_lru_workspace_bytes(const psr_lru_desc* m, int64_t batch) {
    LruGeom g;
    const int r = check_lru(m, &g);
    if (r) return r;
    if (batch < 0) return fail(PSR_EINVAL, "negative batch");
    ok();
    return lru_workspace_floats(g, batch) * (int64_t)sizeof(float);
}

int psr_lru_logpsi(const psr_lru_desc* m, const float* theta, const int8_t* spins, int64_t B, float* logpsi,
                   float* logp_site, void* ws, size_t ws_bytes, void* stream) {
    LruGeom g;
    int r = check_lru(m, &g);
    if (r) return r;
    if (B < 0) return fail(PSR_EINVAL, "negative batch");
    if (B == 0) return ok();
    if (!theta || !spins || !logpsi) return fail(PSR_EINVAL, "theta, spins and logpsi must not be NULL");
    const int64_t need = lru_workspace_floats(g, B) * (int64_t)sizeof(float);
    if (!ws || (int64_t)ws_bytes < need)
        return fail(PSR_ENOMEM, "workspace of %zu bytes is smaller than the %lld needed", ws_bytes, (long long)need);
    hipStream_t st = as_stream(stream);
    hipEvent_t stop;
    timing_before(st, &stop);
    const int e = launch_lru_logpsi(g, theta, spins, B, logpsi, nullptr, logp_site, static_cast<float*>(ws), st);
    if (stop && hipEventRecord(stop, st) != hipSuccess) --g_tm.used;   // drop the half-recorded pair
    if ((r = dev_check(e, "LRU forward"))) return r;
    return ok();
}

// workspace of psr_lru_local_energy: connected slots, their configurations, both log psi
// arrays and the LRU kernel's scratch for the larger of its two launches
struct LruElocWs {
    int32_t* n_conn;
    float* diag;
    uint32_t* desc;
    float* mel;
    int8_t* conn;
    float *lps, *lps_lo;
    float *lpc, *lpc_lo;
    float* scratch;
};

static int64_t carve_lru_eloc(const LruGeom& g, int64_t B, int64_t mc, void* base, LruElocWs* w) {
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o += align256(bytes);
        return base ? static_cast<char*>(base) + at : nullptr;
    };
    const int64_t M = B * mc;
    w->n_conn = reinterpret_cast<int32_t*>(take(B * 4));
    w->diag = reinterpret_cast<float*>(take(B * 4));
    w->desc = reinterpret_cast<uint32_t*>(take(M * 8));
    w->mel = reinterpret_cast<float*>(take(M * 4));
    w->conn = reinterpret_cast<int8_t*>(take(M * g.n));
    w->lps = reinterpret_cast<float*>(take(B * 4));
    w->lps_lo = reinterpret_cast<float*>(take(B * 4));
    w->lpc = reinterpret_cast<float*>(take(M * 4));
    w->lpc_lo = reinterpret_cast<float*>(take(M * 4));
    const int64_t sc = lru_workspace_floats(g, M > B ? M : B);
    w->scratch = reinterpret_cast<float*>(take(sc * 4));
    return o;
}

static int check_lru_ham(const LruGeom& g, const psr_hamiltonian* H, Ham* h) {
    int r = check_ham(H, h);
    if (r) return r;
    if (h->ly != 1 || h->lx != g.n)
        return fail(PSR_EINVAL, "Hamiltonian lattice %d x %d is not the model's chain of %d sites", h->lx, h->ly, g.n);
    return PSR_OK;
}

int64_t psr_lru_eloc_workspace_bytes(const psr_lru_desc* m, const psr_hamiltonian* H, int64_t batch) {
    LruGeom g;
    int r = check_lru(m, &g);
    if (r) return r;
    Ham h;
    if ((r = check_lru_ham(g, H, &h))) return r;
    if (batch < 0) return fail(PSR_EINVAL, "negative batch");
    ok();
    LruElocWs w;
    return carve_lru_eloc(g, batch, ham_max_connected(h), nullptr, &w);
}

int psr_lru_local_energy(const psr_lru_desc* m, const float* theta, const psr_hamiltonian* H, const int8_t* spins,
                         int64_t B, double* eloc, double* stats, float* logpsi, void* ws, size_t ws_bytes,
                         void* stream) {
    LruGeom g;
    int r = check_lru(m, &g);
    if (r) return r;
    Ham h;
    if ((r = check_lru_ham(g, H, &h))) return r;
    if (B < 0) return fail(PSR_EINVAL, "negative batch");
    if (B == 0) return ok();
    if (!theta || !spins || !eloc || !stats) return fail(PSR_EINVAL, "theta, spins, eloc and stats must not be NULL");
    const int64_t mc = ham_max_connected(h);
    LruElocWs w;
    const int64_t need = carve_lru_eloc(g, B, mc, nullptr, &w);
    if (!ws || (int64_t)ws_bytes < need)
        return fail(PSR_ENOMEM, "workspace of %zu bytes is smaller than the %lld needed", ws_bytes, (long long)need);
    carve_lru_eloc(g, B, mc, ws, &w);
    hipStream_t st = as_stream(stream);
    const int64_t M = B * mc;
    if ((r = dev_check(launch_conn_count(h, spins, B, w.n_conn, w.diag, st), "connected count"))) return r;
    if ((r = dev_check(launch_conn_write(h, spins, B, nullptr, mc, w.desc, w.mel, st), "connected write"))) return r;
    if ((r = dev_check(launch_conn_expand(spins, g.n, B, mc, w.n_conn, w.desc, w.conn, st), "connected expand")))
        return r;
    // slots past a sample's count hold unwritten bytes: the kernel reads only their low
    // bit and the combine never reads their log psi
    for (int pass = 0; pass < 2; ++pass) {
        hipEvent_t stop;
        timing_before(st, &stop);
        const int e = pass == 0 ? launch_lru_logpsi(g, theta, spins, B, w.lps, w.lps_lo, nullptr, w.scratch, st)
                                : launch_lru_logpsi(g, theta, w.conn, M, w.lpc, w.lpc_lo, nullptr, w.scratch, st);
        if (stop && hipEventRecord(stop, st) != hipSuccess) --g_tm.used;
        if ((r = dev_check(e, "LRU forward"))) return r;
    }
    if ((r = dev_check(launch_lru_eloc_combine(B, mc, w.n_conn, w.diag, w.mel, w.lpc, w.lpc_lo, w.lps, w.lps_lo, eloc,
                                               st),
                       "E_loc")))
        return r;
    if ((r = dev_check(launch_stats(eloc, B, stats, st), "stats"))) return r;
    if (logpsi && (r = dev_check(hipMemcpyAsync(logpsi, w.lps, B * sizeof(float), hipMemcpyDeviceToDevice, st),
                                 "log psi copy")))
        return r;
    return ok();
}

// LRU sampler / backward workspace: the prepared area, the per-chain workspace of
// the chains in flight (backward), and the O rows when the caller wants only g
static int64_t lru_aux_bytes(const LruGeom& g, int32_t op, int64_t B, bool need_O) {
    int64_t b = align256(lru_prep_floats(g) * 4);
    if (op == PSR_OP_BACKWARD) {
        b += align256(lru_bwd_grid(g, B > 0 ? B : 1) * lru_bwd_chain_floats(g) * 4);
        if (need_O) b += align256(B * lru_param_count(g) * 4);
    }
    return b;
}

int64_t psr_lru_op_workspace_bytes(const psr_lru_desc* m, int32_t op, int64_t batch) {
    LruGeom g;
    const int r = check_lru(m, &g);
    if (r) return r;
    if (batch < 0) return fail(PSR_EINVAL, "negative batch");
    ok();
    if (op == PSR_OP_LOGPSI) return lru_workspace_floats(g, batch) * (int64_t)sizeof(float);
    if (op == PSR_OP_SAMPLE) return lru_aux_bytes(g, op, batch, false);
    if (op == PSR_OP_BACKWARD) return lru_aux_bytes(g, op, batch, true);
    return fail(PSR_EINVAL, "op %d is not PSR_OP_LOGPSI, PSR_OP_SAMPLE or PSR_OP_BACKWARD", op);
}

int psr_lru_sample(const psr_lru_desc* m, const float* theta, const float* uniforms, int64_t B, int8_t* spins,
                   float* logpsi, void* ws, size_t ws_bytes, void* stream) {
    LruGeom g;
    int r = check_lru(m, &g);
    if (r) return r;
    if (B < 0) return fail(PSR_EINVAL, "negative batch");
    if (B == 0) return ok();
    if (!theta || !uniforms || !spins || !logpsi) return fail(PSR_EINVAL, "theta, uniforms, spins and logpsi must not be NULL");
    const int64_t need = lru_aux_bytes(g, PSR_OP_SAMPLE, B, false);
    if (!ws || (int64_t)ws_bytes < need)
        return fail(PSR_ENOMEM, "workspace of %zu bytes is smaller than the %lld needed", ws_bytes, (long long)need);
    hipStream_t st = as_stream(stream);
    float* pw = static_cast<float*>(ws);
    if ((r = dev_check(launch_lru_prep(g, theta, pw, st), "LRU prepare"))) return r;
    if ((r = dev_check(launch_lru_sample(g, theta, pw, uniforms, B, spins, logpsi, st), "LRU sample"))) return r;
    return ok();
}

int psr_lru_backward(const psr_lru_desc* m, const float* theta, const int8_t* spins, int64_t B, float* O,
                     float* logpsi, const double* w, double* gout, void* ws, size_t ws_bytes, void* stream) {
    LruGeom g;
    int r = check_lru(m, &g);
    if (r) return r;
    if (B < 0) return fail(PSR_EINVAL, "negative batch");
    if (B == 0) return ok();
    if (!theta || !spins) return fail(PSR_EINVAL, "theta and spins must not be NULL");
    if ((w == nullptr) != (gout == nullptr)) return fail(PSR_EINVAL, "w and g must be both set or both NULL");
    if (!O && !gout) return fail(PSR_EINVAL, "nothing to compute: O and g are both NULL");
    const int64_t need = lru_aux_bytes(g, PSR_OP_BACKWARD, B, O == nullptr);
    if (!ws || (int64_t)ws_bytes < need)
        return fail(PSR_ENOMEM, "workspace of %zu bytes is smaller than the %lld needed", ws_bytes, (long long)need);
    hipStream_t st = as_stream(stream);
    uint8_t* base = static_cast<uint8_t*>(ws);
    float* pw = reinterpret_cast<float*>(base);
    float* scratch = reinterpret_cast<float*>(base + align256(lru_prep_floats(g) * 4));
    float* Ouse = O ? O
                    : reinterpret_cast<float*>(base + align256(lru_prep_floats(g) * 4) +
                                               align256(lru_bwd_grid(g, B) * lru_bwd_chain_floats(g) * 4));
    if ((r = dev_check(launch_lru_prep(g, theta, pw, st), "LRU prepare"))) return r;
    if ((r = dev_check(launch_lru_backward(g, theta, pw, spins, B, Ouse, logpsi, scratch, st), "LRU backward")))
        return r;
    if (gout && (r = dev_check(launch_weighted_sum(Ouse, B, lru_param_count(g), w, gout, st), "gradient sum")))
        return r;
    return ok();
}

int psr_check_spins(const int8_t* spins, int64_t n_values, int32_t* flag, void* stream) {
    if (n_values < 0) return fail(PSR_EINVAL, "negative size");
    if (n_values == 0) return ok();
    if (!spins || !flag) return fail(PSR_EINVAL, "spins and flag must not be NULL");
    hipStream_t st = as_stream(stream);
    int host = 0;
    int r = dev_check(launch_check_spins(spins, n_values, flag, st), "check");
    if (!r) r = dev_check((int)hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, st), "copy flag");
    if (!r) r = dev_check((int)hipStreamSynchronize(st), "synchronise");
    if (r) return r;
    if (host) return fail(PSR_EDATA, "spins outside {0, 1}");
    return ok();
}

}  // extern "C"
