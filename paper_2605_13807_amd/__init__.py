"""Python binding of libpsr, the MI355X hot path of the parallel-scan recurrent
neural quantum state (PSR-NQS).

Argument marshalling only: every step of log psi, the connected
configurations, E_loc and the per-sample gradients runs in the HIP kernels of
``libpsr.so`` (see ``include/psr.h``).  PyTorch provides device memory and the
current stream.  There is no CPU fallback: if the library or a GPU is missing,
the calls raise.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = [
    "Model", "Hamiltonian", "PsrError", "lib",
    "param_count", "param_offsets", "max_connected", "workspace_bytes",
    "logpsi", "logpsi_static", "lru_sample", "lru_backward", "connected", "local_energy", "logpsi_backward", "vmc_weights", "check_spins",
    "LogPsi", "per_sample_grad", "timing_begin", "timing_end",
    "CHAIN_1D", "SNAKE_2D", "FP32", "BF16", "FP16", "SYM_NONE", "SYM_C4V", "TFIM", "HEISENBERG",
]

CHAIN_1D, SNAKE_2D = 0, 1
FP32, BF16, FP16 = 0, 1, 2
SYM_NONE, SYM_C4V = 0, 1
TFIM, HEISENBERG = 0, 1
OP_LOGPSI, OP_LOCAL_ENERGY, OP_BACKWARD, OP_SAMPLE = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsr.so")


class PsrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpsr error {code}: {msg}")
        self.code = code


class _ModelDesc(ctypes.Structure):
    _fields_ = [("geometry", ctypes.c_int32), ("lx", ctypes.c_int32), ("ly", ctypes.c_int32),
                ("n_layers", ctypes.c_int32), ("d", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ckpt_rows", ctypes.c_int32), ("patch", ctypes.c_int32), ("symmetry", ctypes.c_int32)]


class _HamDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("lx", ctypes.c_int32), ("ly", ctypes.c_int32),
                ("marshall", ctypes.c_int32), ("pbc", ctypes.c_int32), ("J", ctypes.c_double),
                ("h", ctypes.c_double)]


@dataclass(frozen=True)
class Model:
    geometry: int
    lx: int
    ly: int
    n_layers: int
    d: int
    precision: int = FP32
    ckpt_rows: int = 0
    patch: int = 1          # 2: 2x2 patch inputs (16-letter alphabet, 16-way head)
    symmetry: int = 0       # SYM_C4V: c4v-symmetrised log psi (square lattices)

    def c(self) -> _ModelDesc:
        return _ModelDesc(self.geometry, self.lx, self.ly, self.n_layers, self.d, self.precision, self.ckpt_rows,
                          self.patch, self.symmetry)

    @property
    def n_sites(self) -> int:
        return self.lx * self.ly

    @property
    def n_grid(self) -> int:
        """Sites of the grid the recurrence runs on (2x2 patches: a quarter of the spins)."""
        return (self.lx // self.patch) * (self.ly // self.patch)


@dataclass(frozen=True)
class Hamiltonian:
    kind: int
    lx: int
    ly: int
    J: float = 1.0
    h: float = 1.0
    marshall: bool = True
    pbc: bool = False

    def c(self) -> _HamDesc:
        return _HamDesc(self.kind, self.lx, self.ly, int(self.marshall), int(self.pbc), float(self.J), float(self.h))


class _LruDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_layers", ctypes.c_int32), ("d", ctypes.c_int32), ("d_h", ctypes.c_int32)]


@dataclass(frozen=True)
class LruModel:
    """The 1D LRU ansatz: chain length n, layers, width d and complex hidden units d_h."""
    n: int
    n_layers: int
    d: int
    d_h: int

    def c(self) -> _LruDesc:
        return _LruDesc(self.n, self.n_layers, self.d, self.d_h)

    @property
    def n_sites(self) -> int:
        return self.n


_lib = None
_flags: dict = {}   # per device: the int32 flag psr_check_spins writes


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2605_13807_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        L.psr_param_count.argtypes = [P(_ModelDesc)]
        L.psr_param_count.restype = i64
        L.psr_param_offsets.argtypes = [P(_ModelDesc), P(i64), P(i32)]
        L.psr_param_offsets.restype = ctypes.c_int
        L.psr_max_connected.argtypes = [P(_HamDesc)]
        L.psr_max_connected.restype = i64
        L.psr_workspace_bytes.argtypes = [P(_ModelDesc), i32, i64, i64]
        L.psr_workspace_bytes.restype = i64
        L.psr_logpsi.argtypes = [P(_ModelDesc), vp, vp, i64, vp, vp, vp, sz, vp]
        L.psr_logpsi.restype = ctypes.c_int
        L.psr_forward_shape.argtypes = [P(_ModelDesc), i64, P(i64)]
        L.psr_forward_shape.restype = ctypes.c_int
        L.psr_logpsi_static.argtypes = [P(_ModelDesc), vp, vp, i64, vp, vp, vp]
        L.psr_logpsi_static.restype = ctypes.c_int
        L.psr_static_scratch_bytes.argtypes = []
        L.psr_static_scratch_bytes.restype = i64
        L.psr_connected.argtypes = [P(_HamDesc), vp, i64, i64, vp, vp, vp, vp, vp, vp]
        L.psr_connected.restype = ctypes.c_int
        L.psr_local_energy.argtypes = [P(_ModelDesc), vp, P(_HamDesc), vp, i64, i64, vp, vp, vp, vp, sz, vp]
        L.psr_local_energy.restype = ctypes.c_int
        L.psr_logpsi_backward.argtypes = [P(_ModelDesc), vp, vp, i64, vp, vp, vp, vp, vp, sz, vp]
        L.psr_logpsi_backward.restype = ctypes.c_int
        L.psr_sample.argtypes = [P(_ModelDesc), vp, vp, i64, vp, vp, vp, sz, vp]
        L.psr_sample.restype = ctypes.c_int
        L.psr_gradient_estimate.argtypes = [vp, i64, i64, vp, vp, vp]
        L.psr_gradient_estimate.restype = ctypes.c_int
        L.psr_vmc_weights.argtypes = [vp, vp, i64, vp, vp]
        L.psr_vmc_weights.restype = ctypes.c_int
        L.psr_lru_param_count.argtypes = [P(_LruDesc)]
        L.psr_lru_param_count.restype = i64
        L.psr_lru_workspace_bytes.argtypes = [P(_LruDesc), i64]
        L.psr_lru_workspace_bytes.restype = i64
        L.psr_lru_logpsi.argtypes = [P(_LruDesc), vp, vp, i64, vp, vp, vp, sz, vp]
        L.psr_lru_logpsi.restype = ctypes.c_int
        L.psr_lru_eloc_workspace_bytes.argtypes = [P(_LruDesc), P(_HamDesc), i64]
        L.psr_lru_eloc_workspace_bytes.restype = i64
        L.psr_lru_local_energy.argtypes = [P(_LruDesc), vp, P(_HamDesc), vp, i64, vp, vp, vp, vp, sz, vp]
        L.psr_lru_local_energy.restype = ctypes.c_int
        L.psr_lru_op_workspace_bytes.argtypes = [P(_LruDesc), i32, i64]
        L.psr_lru_op_workspace_bytes.restype = i64
        L.psr_lru_sample.argtypes = [P(_LruDesc), vp, vp, i64, vp, vp, vp, sz, vp]
        L.psr_lru_sample.restype = ctypes.c_int
        L.psr_lru_backward.argtypes = [P(_LruDesc), vp, vp, i64, vp, vp, vp, vp, vp, sz, vp]
        L.psr_lru_backward.restype = ctypes.c_int
        L.psr_check_spins.argtypes = [vp, i64, vp, vp]
        L.psr_check_spins.restype = ctypes.c_int
        L.psr_timing_begin.argtypes = []
        L.psr_timing_begin.restype = ctypes.c_int
        L.psr_timing_end.argtypes = [P(ctypes.c_double), P(i64)]
        L.psr_timing_end.restype = ctypes.c_int
        L.psr_last_error.argtypes = []
        L.psr_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code: int) -> None:
    if code != 0:
        raise PsrError(code, lib().psr_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t.contiguous()


def param_count(m: Model) -> int:
    n = lib().psr_param_count(ctypes.byref(m.c()))
    _check(int(n) if n < 0 else 0)
    return int(n)


def param_offsets(m: Model) -> list[int]:
    off = (ctypes.c_int64 * 64)()
    n = ctypes.c_int32(0)
    _check(lib().psr_param_offsets(ctypes.byref(m.c()), off, ctypes.byref(n)))
    return [int(off[k]) for k in range(n.value + 1)]


def forward_shape(m: Model, batch: int) -> dict:
    """The forward kernel's launch layout for `batch` samples (psr_forward_shape)."""
    out = (ctypes.c_int64 * 9)()
    _check(lib().psr_forward_shape(ctypes.byref(m.c()), batch, out))
    keys = ("cols", "seqs", "ntc", "waves", "cross_wave", "lds_frontier", "split_kernel", "launch_seqs",
            "frontier_seq_bytes")
    return {k: int(out[i]) for i, k in enumerate(keys)}


def max_connected(h: Hamiltonian) -> int:
    n = lib().psr_max_connected(ctypes.byref(h.c()))
    _check(int(n) if n < 0 else 0)
    return int(n)


def workspace_bytes(m: Model, op: int, batch: int, chunk_seqs: int = 0) -> int:
    n = lib().psr_workspace_bytes(ctypes.byref(m.c()), op, batch, chunk_seqs)
    _check(int(n) if n < 0 else 0)
    return int(n)


def _workspace(m: Model, op: int, batch: int, device, chunk_seqs: int = 0) -> torch.Tensor:
    return torch.empty(max(1, workspace_bytes(m, op, batch, chunk_seqs)), dtype=torch.uint8, device=device)


def logpsi(m: Model, theta: torch.Tensor, spins: torch.Tensor, site_logp: bool = False, ws: torch.Tensor | None = None):
    """log psi [B] (float32), and the per-site log p [B, N] if ``site_logp``."""
    theta = _dev(theta, torch.float32, "theta")
    spins = _dev(spins, torch.int8, "spins")
    B = spins.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=spins.device)
    lps = torch.empty(B, m.n_grid, dtype=torch.float32, device=spins.device) if site_logp else None
    if ws is None:
        ws = _workspace(m, OP_LOGPSI, B, spins.device)
    _check(lib().psr_logpsi(ctypes.byref(m.c()), _ptr(theta), _ptr(spins), B, _ptr(out), _ptr(lps), _ptr(ws),
                            ws.numel(), _stream(spins.device)))
    return (out, lps) if site_logp else out


def logpsi_static(m: Model, theta: torch.Tensor, spins: torch.Tensor, site_logp: bool = False):
    """log psi through psr_logpsi_static: no workspace, the library's static device scratch
    (calls on one GPU must not overlap)."""
    theta = _dev(theta, torch.float32, "theta")
    spins = _dev(spins, torch.int8, "spins")
    B = spins.shape[0]
    out = torch.empty(B, dtype=torch.float32, device=spins.device)
    lps = torch.empty(B, m.n_grid, dtype=torch.float32, device=spins.device) if site_logp else None
    _check(lib().psr_logpsi_static(ctypes.byref(m.c()), _ptr(theta), _ptr(spins), B, _ptr(out), _ptr(lps),
                                   _stream(spins.device)))
    return (out, lps) if site_logp else out


def lru_param_count(m: LruModel) -> int:
    n = lib().psr_lru_param_count(ctypes.byref(m.c()))
    _check(int(n) if n < 0 else 0)
    return int(n)


def lru_workspace_bytes(m: LruModel, batch: int) -> int:
    n = lib().psr_lru_workspace_bytes(ctypes.byref(m.c()), batch)
    _check(int(n) if n < 0 else 0)
    return int(n)


def lru_logpsi(m: LruModel, theta: torch.Tensor, spins: torch.Tensor, site_logp: bool = False,
               ws: torch.Tensor | None = None):
    """log psi [B] (float32) of chains under the 1D LRU ansatz, and the per-site log p [B, N] if ``site_logp``."""
    theta = _dev(theta, torch.float32, "theta")
    spins = _dev(spins, torch.int8, "spins")
    B = spins.shape[0]
    if spins.dim() != 2 or spins.shape[1] != m.n:
        raise ValueError(f"spins must be [B, {m.n}], got {list(spins.shape)}")
    if theta.numel() != lru_param_count(m):
        raise ValueError(f"theta has {theta.numel()} entries, the model {lru_param_count(m)}")
    out = torch.empty(B, dtype=torch.float32, device=spins.device)
    lps = torch.empty(B, m.n, dtype=torch.float32, device=spins.device) if site_logp else None
    if ws is None:
        ws = torch.empty(max(1, lru_workspace_bytes(m, B)), dtype=torch.uint8, device=spins.device)
    _check(lib().psr_lru_logpsi(ctypes.byref(m.c()), _ptr(theta), _ptr(spins), B, _ptr(out), _ptr(lps), _ptr(ws),
                                ws.numel(), _stream(spins.device)))
    return (out, lps) if site_logp else out


def lru_local_energy(m: LruModel, theta: torch.Tensor, h: Hamiltonian, spins: torch.Tensor,
                     ws: torch.Tensor | None = None):
    """(E_loc [B] float64, stats [2] float64 = (mean, variance), log psi [B] float32) under the 1D LRU."""
    theta = _dev(theta, torch.float32, "theta")
    spins = _dev(spins, torch.int8, "spins")
    B = spins.shape[0]
    dev = spins.device
    e = torch.empty(B, dtype=torch.float64, device=dev)
    st = torch.zeros(2, dtype=torch.float64, device=dev)
    lp = torch.empty(B, dtype=torch.float32, device=dev)
    if ws is None:
        n = lib().psr_lru_eloc_workspace_bytes(ctypes.byref(m.c()), ctypes.byref(h.c()), B)
        _check(int(n) if n < 0 else 0)
        ws = torch.empty(max(1, int(n)), dtype=torch.uint8, device=dev)
    _check(lib().psr_lru_local_energy(ctypes.byref(m.c()), _ptr(theta), ctypes.byref(h.c()), _ptr(spins), B, _ptr(e),
                                      _ptr(st), _ptr(lp), _ptr(ws), ws.numel(), _stream(dev)))
    return e, st, lp


def _lru_ws(m: LruModel, op: int, B: int, device) -> torch.Tensor:
    n = lib().psr_lru_op_workspace_bytes(ctypes.byref(m.c()), op, B)
    _check(int(n) if n < 0 else 0)
    return torch.empty(max(1, int(n)), dtype=torch.uint8, device=device)


def lru_sample(m: LruModel, theta: torch.Tensor, uniforms: torch.Tensor, ws: torch.Tensor | None = None):
    """Exact autoregressive samples of LRU chains: (spins [B, n] int8, log psi [B] float32)."""
    theta = _dev(theta, torch.float32, "theta")
    u = _dev(uniforms, torch.float32, "uniforms")
    B, N = u.shape
    if N != m.n:
        raise ValueError(f"uniforms has {N} sites, the model {m.n}")
    spins = torch.empty(B, N, dtype=torch.int8, device=u.device)
    lp = torch.empty(B, dtype=torch.float32, device=u.device)
    if ws is None:
        ws = _lru_ws(m, OP_SAMPLE, B, u.device)
    _check(lib().psr_lru_sample(ctypes.byref(m.c()), _ptr(theta), _ptr(u), B, _ptr(spins), _ptr(lp), _ptr(ws),
                                ws.numel(), _stream(u.device)))
    return spins, lp


def lru_backward(m: LruModel, theta: torch.Tensor, spins: torch.Tensor, w: torch.Tensor | None = None,
                 want_O: bool = True, ws: torch.Tensor | None = None):
    """(O [B, P] float32 or None, log psi [B], g [P] float64 or None) of LRU chains, g = sum_s w_s O_s."""
    theta = _dev(theta, torch.float32, "theta")
    spins = _dev(spins, torch.int8, "spins")
    B = spins.shape[0]
    dev = spins.device
    P = lru_param_count(m)
    O = torch.empty(B, P, dtype=torch.float32, device=dev) if want_O else None
    lp = torch.empty(B, dtype=torch.float32, device=dev)
    g = None
    if w is not None:
        w = _dev(w, torch.float64, "w")
        g = torch.empty(P, dtype=torch.float64, device=dev)
    if ws is None:
        ws = _lru_ws(m, OP_BACKWARD, B, dev)
    _check(lib().psr_lru_backward(ctypes.byref(m.c()), _ptr(theta), _ptr(spins), B, _ptr(O), _ptr(lp), _ptr(w),
                                  _ptr(g), _ptr(ws), ws.numel(), _stream(dev)))
    return O, lp, g


def connected(h: Hamiltonian, spins: torch.Tensor, max_conn: int | None = None, configs: bool = False):
    """Connected configurations in canonical order (per-sample slots).

    Returns dict(n_conn [B] int32, diag [B] f32, desc [B, max_conn, 2] uint32
    stored as int32, mel [B, max_conn] f32, and conn [B, max_conn, N] int8 if
    ``configs``).
    """
    spins = _dev(spins, torch.int8, "spins")
    B, N = spins.shape
    mc = max_connected(h) if max_conn is None else int(max_conn)
    dev = spins.device
    n_conn = torch.zeros(B, dtype=torch.int32, device=dev)
    diag = torch.empty(B, dtype=torch.float32, device=dev)
    desc = torch.zeros(B, mc, 2, dtype=torch.int32, device=dev)
    mel = torch.zeros(B, mc, dtype=torch.float32, device=dev)
    conn = torch.zeros(B, mc, N, dtype=torch.int8, device=dev) if configs else None
    _check(lib().psr_connected(ctypes.byref(h.c()), _ptr(spins), B, mc, _ptr(conn), _ptr(desc), _ptr(mel),
                               _ptr(n_conn), _ptr(diag), _stream(dev)))
    out = {"n_conn": n_conn, "diag": diag, "desc": desc, "mel": mel}
    if configs:
        out["conn"] = conn
    return out


def local_energy(m: Model, theta: torch.Tensor, h: Hamiltonian, spins: torch.Tensor, chunk_seqs: int = 32768,
                 ws: torch.Tensor | None = None):
    """(E_loc [B] float64, stats [2] float64 = (mean, variance), log psi [B] float32)."""
    theta = _dev(theta, torch.float32, "theta")
    spins = _dev(spins, torch.int8, "spins")
    B = spins.shape[0]
    dev = spins.device
    eloc = torch.empty(B, dtype=torch.float64, device=dev)
    stats = torch.empty(2, dtype=torch.float64, device=dev)
    lp = torch.empty(B, dtype=torch.float32, device=dev)
    if ws is None:
        ws = _workspace(m, OP_LOCAL_ENERGY, B, dev, chunk_seqs)
    _check(lib().psr_local_energy(ctypes.byref(m.c()), _ptr(theta), ctypes.byref(h.c()), _ptr(spins), B, chunk_seqs,
                                  _ptr(eloc), _ptr(stats), _ptr(lp), _ptr(ws), ws.numel(), _stream(dev)))
    return eloc, stats, lp


def logpsi_backward(m: Model, theta: torch.Tensor, spins: torch.Tensor, w: torch.Tensor | None = None,
                    want_O: bool = True, ws: torch.Tensor | None = None):
    """(O [B, P] float32 or None, log psi [B], g [P] float64 or None) with g = sum_s w_s O_s."""
    theta = _dev(theta, torch.float32, "theta")
    spins = _dev(spins, torch.int8, "spins")
    B = spins.shape[0]
    dev = spins.device
    P = param_count(m)
    O = torch.empty(B, P, dtype=torch.float32, device=dev) if want_O else None
    lp = torch.empty(B, dtype=torch.float32, device=dev)
    g = None
    if w is not None:
        w = _dev(w, torch.float64, "w")
        g = torch.empty(P, dtype=torch.float64, device=dev)
    if ws is None:
        ws = _workspace(m, OP_BACKWARD, B, dev)
    _check(lib().psr_logpsi_backward(ctypes.byref(m.c()), _ptr(theta), _ptr(spins), B, _ptr(O), _ptr(lp), _ptr(w),
                                     _ptr(g), _ptr(ws), ws.numel(), _stream(dev)))
    return O, lp, g


def sample(m: Model, theta: torch.Tensor, uniforms: torch.Tensor, ws: torch.Tensor | None = None):
    """Exact autoregressive samples: (spins [B, N] int8, log psi [B] float32).

    ``uniforms`` [B, N] float32 in [0, 1), lattice row-major: site t takes spin 1
    iff its uniform is below p(sigma_t = 1 | sigma_<t).
    """
    theta = _dev(theta, torch.float32, "theta")
    uniforms = _dev(uniforms, torch.float32, "uniforms")
    B, N = uniforms.shape
    if N != m.n_sites:
        raise ValueError(f"uniforms has {N} sites, the model {m.n_sites}")
    dev = uniforms.device
    spins = torch.empty(B, N, dtype=torch.int8, device=dev)
    lp = torch.empty(B, dtype=torch.float32, device=dev)
    if ws is None:
        ws = _workspace(m, OP_SAMPLE, B, dev)
    _check(lib().psr_sample(ctypes.byref(m.c()), _ptr(theta), _ptr(uniforms), B, _ptr(spins), _ptr(lp), _ptr(ws),
                            ws.numel(), _stream(dev)))
    return spins, lp


def gradient_estimate(O: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """g = sum_s w_s O_s (float64 [P]) from per-sample rows O [B, P] (float32) and weights w [B] (float64)."""
    O = _dev(O, torch.float32, "O")
    w = _dev(w, torch.float64, "w")
    B, Pn = O.shape
    if w.shape != (B,):
        raise ValueError("w must be [B]")
    g = torch.empty(Pn, dtype=torch.float64, device=O.device)
    _check(lib().psr_gradient_estimate(_ptr(O), B, Pn, _ptr(w), _ptr(g), _stream(O.device)))
    return g


def vmc_weights(eloc: torch.Tensor, stats: torch.Tensor) -> torch.Tensor:
    """w_s = (2/B) (E_loc(s) - mean)."""
    eloc = _dev(eloc, torch.float64, "eloc")
    stats = _dev(stats, torch.float64, "stats")
    w = torch.empty_like(eloc)
    _check(lib().psr_vmc_weights(_ptr(eloc), _ptr(stats), eloc.numel(), _ptr(w), _stream(eloc.device)))
    return w


def check_spins(spins: torch.Tensor) -> None:
    """Raise PsrError (code PSR_EDATA) unless every value is 0 or 1 (synchronous)."""
    spins = _dev(spins, torch.int8, "spins")
    key = spins.device.index
    if key not in _flags:
        _flags[key] = torch.zeros(1, dtype=torch.int32, device=spins.device)
    _check(lib().psr_check_spins(_ptr(spins), spins.numel(), _ptr(_flags[key]), _stream(spins.device)))


def timing_begin() -> None:
    """Start bracketing every forward-kernel launch of this thread with HIP events."""
    _check(lib().psr_timing_begin())


def timing_end() -> tuple[float, int]:
    """(summed forward-kernel milliseconds, launches) since timing_begin()."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().psr_timing_end(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


class LogPsi(torch.autograd.Function):
    """log psi(theta; spins) with a backward through the reverse-scan adjoint.

    forward  -> psr_logpsi
    backward -> psr_logpsi_backward with w = grad_output: grad_theta = O^T grad_output
    """

    @staticmethod
    def forward(ctx, theta, spins, model):
        ctx.model = model
        ctx.save_for_backward(theta, spins)
        return logpsi(model, theta, spins)

    @staticmethod
    def backward(ctx, grad_out):
        theta, spins = ctx.saved_tensors
        _, _, g = logpsi_backward(ctx.model, theta, spins, w=grad_out.to(torch.float64), want_O=False)
        return g.to(theta.dtype), None, None


def per_sample_grad(m: Model, theta: torch.Tensor, spins: torch.Tensor) -> torch.Tensor:
    """O [B, P]: one row d log psi(sigma_s) / d theta per sample."""
    O, _, _ = logpsi_backward(m, theta, spins)
    return O
