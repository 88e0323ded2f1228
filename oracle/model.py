"""Oracle: the autoregressive recurrent wave function, float64, CPU.

TEST INFRASTRUCTURE -- see ``oracle/__init__.py``.

Two ansatz families are covered.

``chain``   The minGRU recurrence of Sec. II.C (Eq. minGRU) on a 1D chain:
            z_t = sigma(W_z x_{t-1} + b_z), htilde_t = W_h x_{t-1} + b_h,
            h_t = z_t * h_{t-1} + (1 - z_t) * htilde_t, with x_{t-1} the one-hot
            spin of the previous site (zero before the first site) and h_0 = 0.
            One layer; a linear two-way softmax head reads h_t.

``snake2d`` The stacked 2D minGRU of Sec. II.F and II.G on an lx-by-ly lattice
            visited in zigzag ("snake") order: row j runs left to right for
            even j and right to left for odd j (0-based rows).  Horizontal
            predecessor (i - (-1)^j, j), vertical predecessor (i, j - 1);
            anything outside the lattice is zero.  Per layer l:
              u^(0) = (x^(0) at H-pred, x^(0) at V-pred), u^(l>=1) = x^(l)
              z     = sigma(W_z u + b_z)
              htil  = W_h [u, h_V] + b_h
              h     = z * h_H + (1 - z) * htil
              xt    = C h + D u
              s     = h^(l-1) if l >= 2 else 0          (residual, Sec. II.G)
              x^(l+1) = GELU(xt + s)                   (exact erf GELU)
            and the head reads x^(n_l).

Amplitude (Sec. III.B, "formalism of" Hibat-Allah et al. 2020): the head gives
logits in R^2 at every site, log p_t = logit[sigma_t] - logsumexp(logits), the
wave function is positive and log psi = (1/2) sum_t log p_t.

Parameter layout (flat float vector, row-major matrices, in this order):
per layer  W_z[d][du], b_z[d], W_h[d][du + d], b_h[d], C[d][d], D[d][du]
(du = 2 K at l = 0, d afterwards); chain: W_z[d][2], b_z[d], W_h[d][2], b_h[d];
then the head W_o[K][d], b_o[K].  K is the size of the local alphabet: 2 for
single-site inputs, 16 for 2x2 patches.

Patches (Sec. II.F: the initial input can be a 2x2 patch of spins).  With
``patch = 2`` the recurrence runs on the (lx/2)-by-(ly/2) grid of patches in the
same zigzag order; patch (I, J) covers the spins (2I + a, 2J + b), a, b in {0, 1},
and its state is k = sigma(2I, 2J) + 2 sigma(2I+1, 2J) + 4 sigma(2I, 2J+1)
+ 8 sigma(2I+1, 2J+1) (a reading: the paper gives no encoding).  u^(0) is the
one-hot state (16 entries) of the H- and V-predecessor patches, and the head
gives the 16-way conditional of the patch's own state, so log psi = (1/2) sum
over patches of log p(k_t | k_<t).

``mode="seq"`` runs the plain sequential recurrence and is the authority.
``mode="scan"`` replaces the loop along each row by a Blelloch up-sweep /
down-sweep over the affine pairs (a_t, b_t) = (z_t, (1 - z_t) htilde_t), the
reassociation the paper relies on (Sec. II.A, II.B, II.F).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import erf, expit, logsumexp

SQRT1_2 = 0.7071067811865476


@dataclass(frozen=True)
class Model:
    """Ansatz shape.  ``geometry`` is ``"chain"`` (ly must be 1) or ``"snake2d"``."""

    geometry: str
    lx: int
    ly: int
    n_layers: int
    d: int
    patch: int = 1

    @property
    def n_sites(self) -> int:
        return self.lx * self.ly

    @property
    def px(self) -> int:
        """Columns of the grid the recurrence runs on (patches)."""
        return self.lx // self.patch

    @property
    def py(self) -> int:
        return self.ly // self.patch

    @property
    def n_states(self) -> int:
        """Size of the local alphabet K: 2 per site, 16 per 2x2 patch."""
        return 2 ** (self.patch * self.patch)

    def __post_init__(self):
        if self.geometry not in ("chain", "snake2d"):
            raise ValueError(self.geometry)
        if self.geometry == "chain" and (self.ly != 1 or self.n_layers != 1):
            raise ValueError("the chain ansatz is one minGRU layer on ly = 1")
        if min(self.lx, self.ly, self.n_layers, self.d) < 1:
            raise ValueError("sizes must be positive")
        if self.patch not in (1, 2):
            raise ValueError("patch must be 1 or 2")
        if self.patch == 2 and (self.geometry != "snake2d" or self.lx % 2 or self.ly % 2):
            raise ValueError("2x2 patches need the 2D snake on even lattice sides")


def snake_tensor_shapes(n_layers: int, d: int, du0: int = 4, n_out: int = 2):
    """Tensor shapes of the stacked 2D minGRU (Sec. II.F, II.G) plus its head.

    ``du0`` is the width of u^(0) (two predecessor inputs: 2 x 2 one-hot spins
    for single-site inputs) and ``n_out`` the size of the local alphabet the
    head predicts.  W_h acts on [u, h_V], C on h and D on u; only z and htilde
    carry biases.
    """
    out: list[tuple[str, tuple[int, ...]]] = []
    for l in range(n_layers):
        du = du0 if l == 0 else d
        out += [
            (f"Wz{l}", (d, du)),
            (f"bz{l}", (d,)),
            (f"Wh{l}", (d, du + d)),
            (f"bh{l}", (d,)),
            (f"C{l}", (d, d)),
            (f"D{l}", (d, du)),
        ]
    out += [("Wo", (n_out, d)), ("bo", (n_out,))]
    return out


def tensor_shapes(m: Model) -> list[tuple[str, tuple[int, ...]]]:
    """Names and shapes of the parameter tensors, in storage order."""
    d = m.d
    if m.geometry == "chain":
        return [("Wz0", (d, 2)), ("bz0", (d,)), ("Wh0", (d, 2)), ("bh0", (d,)),
                ("Wo", (2, d)), ("bo", (2,))]
    return snake_tensor_shapes(m.n_layers, d, du0=2 * m.n_states, n_out=m.n_states)


def n_params(m: Model) -> int:
    return int(sum(int(np.prod(s)) for _, s in tensor_shapes(m)))


def unpack(theta: np.ndarray, m: Model) -> dict[str, np.ndarray]:
    """Views of the flat vector as float64 tensors (read as float64(theta))."""
    theta = np.asarray(theta, dtype=np.float64).reshape(-1)
    if theta.size != n_params(m):
        raise ValueError(f"theta has {theta.size} entries, model needs {n_params(m)}")
    out, off = {}, 0
    for name, shape in tensor_shapes(m):
        k = int(np.prod(shape))
        out[name] = theta[off: off + k].reshape(shape)
        off += k
    return out


def gelu(x: np.ndarray) -> np.ndarray:
    """GELU with the exact Gaussian CDF (Hendrycks & Gimpel), x * Phi(x)."""
    return 0.5 * x * (1.0 + erf(x * SQRT1_2))


def snake_row(lx: int, j: int) -> list[int]:
    """Columns of row j in visiting order (0-based j: even rows left to right)."""
    return list(range(lx)) if j % 2 == 0 else list(range(lx - 1, -1, -1))


def snake_order(lx: int, ly: int) -> list[tuple[int, int]]:
    """All sites (i, j) in the order the autoregressive factorisation visits them."""
    return [(i, j) for j in range(ly) for i in snake_row(lx, j)]


def h_pred(i: int, j: int) -> tuple[int, int]:
    """Horizontal causal predecessor (i - (-1)^j, j) of site (i, j)."""
    return (i - (1 if j % 2 == 0 else -1), j)


def v_pred(i: int, j: int) -> tuple[int, int]:
    """Vertical causal predecessor (i, j - 1) of site (i, j)."""
    return (i, j - 1)


def _onehot_at(states: np.ndarray, lx: int, ly: int, i: int, j: int, k: int = 2) -> np.ndarray:
    """One-hot (k entries) of the state at grid site (i, j) for every batch row; zeros outside."""
    b = states.shape[0]
    out = np.zeros((b, k))
    if 0 <= i < lx and 0 <= j < ly:
        s = states[:, j * lx + i].astype(np.int64)
        out[np.arange(b), s] = 1.0
    return out


def patch_states(spins: np.ndarray, m: Model) -> np.ndarray:
    """Local states on the recurrence grid, [B, px * py] (grid row-major).

    patch = 1: the spins themselves.  patch = 2: patch (I, J) has state
    sigma(2I, 2J) + 2 sigma(2I+1, 2J) + 4 sigma(2I, 2J+1) + 8 sigma(2I+1, 2J+1).
    """
    spins = np.asarray(spins).astype(np.int64)
    if m.patch == 1:
        return spins
    B = spins.shape[0]
    lat = spins.reshape(B, m.ly, m.lx)             # [b, y, x]
    out = np.zeros((B, m.py, m.px), dtype=np.int64)
    for b_ in range(2):
        for a_ in range(2):
            out += lat[:, b_::2, a_::2] << (a_ + 2 * b_)
    return out.reshape(B, m.px * m.py)


# ----------------------------------------------------------------------------
# Recurrence along one row: sequential loop (authority) and Blelloch scan
# ----------------------------------------------------------------------------

def affine_seq(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """h_t = a_t * h_{t-1} + b_t along axis 1 from h_{-1} = 0 (plain loop)."""
    h = np.zeros_like(b)
    prev = np.zeros_like(b[:, 0])
    for t in range(b.shape[1]):
        prev = a[:, t] * prev + b[:, t]
        h[:, t] = prev
    return h


def _compose(p_a, p_b, q_a, q_b):
    """Pair that applies p first and q second: (q_a p_a, q_a p_b + q_b)."""
    return q_a * p_a, q_a * p_b + q_b


def affine_blelloch(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Same result as ``affine_seq`` by Blelloch's work-efficient scan (1990).

    The pairs are padded with the identity (1, 0) to a power of two; the
    up-sweep builds subtree aggregates, the root is cleared to the identity and
    the down-sweep hands every node the composition of everything to its left
    (the parent's prefix applied first, the left subtree second).  The inclusive
    prefix at t is then (exclusive prefix, then element t), and since the state
    enters at zero, h_t is the offset part of that pair.
    """
    n = b.shape[1]
    size = 1
    while size < n:
        size *= 2
    shp = (b.shape[0], size) + b.shape[2:]
    A = np.ones(shp)
    Bv = np.zeros(shp)
    A[:, :n] = a
    Bv[:, :n] = b
    stride = 1
    while stride < size:                      # up-sweep
        for k in range(2 * stride - 1, size, 2 * stride):
            left = k - stride
            A[:, k], Bv[:, k] = _compose(A[:, left], Bv[:, left], A[:, k], Bv[:, k])
        stride *= 2
    A[:, size - 1] = 1.0                      # clear the root
    Bv[:, size - 1] = 0.0
    stride = size // 2
    while stride >= 1:                        # down-sweep
        for k in range(2 * stride - 1, size, 2 * stride):
            left = k - stride
            ta, tb = A[:, left].copy(), Bv[:, left].copy()
            A[:, left], Bv[:, left] = A[:, k], Bv[:, k]
            A[:, k], Bv[:, k] = _compose(A[:, k], Bv[:, k], ta, tb)
        stride //= 2
    _, h = _compose(A[:, :n], Bv[:, :n], a, b)   # exclusive prefix, then element t
    return h


# ----------------------------------------------------------------------------
# Forward passes
# ----------------------------------------------------------------------------

def _site_logp(logits: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """log p(sigma_t) = logit[sigma_t] - logsumexp(logits), per batch row."""
    pick = logits[np.arange(logits.shape[0]), sigma.astype(np.int64)]
    return pick - logsumexp(logits, axis=1)


def _forward_chain(P, spins, m: Model, mode: str, keep_hidden: bool):
    B, N = spins.shape
    d = m.d
    # x_{t-1} for t = 0..N-1: zero before the first site, then one-hot spins
    xprev = np.zeros((B, N, 2))
    xprev[:, 1:, :] = np.eye(2)[spins[:, :-1].astype(np.int64)]
    z = expit(xprev @ P["Wz0"].T + P["bz0"])
    ht = xprev @ P["Wh0"].T + P["bh0"]
    a, b = z, (1.0 - z) * ht
    h = affine_seq(a, b) if mode == "seq" else affine_blelloch(a, b)
    logits = h @ P["Wo"].T + P["bo"]
    logp = np.empty((B, N))
    for t in range(N):
        logp[:, t] = _site_logp(logits[:, t], spins[:, t])
    hidden = [h] if keep_hidden else None
    return logp, hidden


def _forward_snake(P, spins, m: Model, mode: str, keep_hidden: bool):
    # the recurrence runs on the grid of sites (patch = 1) or of 2x2 patches
    states = patch_states(spins, m)
    B, N = states.shape
    lx, ly, d, nl, K = m.px, m.py, m.d, m.n_layers, m.n_states
    frontier = [np.zeros((B, lx, d)) for _ in range(nl)]   # h^(l) of the previous row
    logp = np.empty((B, N))
    hidden = [np.zeros((B, N, d)) for _ in range(nl)] if keep_hidden else None
    for j in range(ly):
        cols = snake_row(lx, j)                              # visiting order
        # layer-0 input at every site of the row, indexed by column i
        u = np.zeros((B, lx, 2 * K))
        for i in range(lx):
            hi, hj = h_pred(i, j)
            vi, vj = v_pred(i, j)
            u[:, i, 0:K] = _onehot_at(states, lx, ly, hi, hj, K)
            u[:, i, K:2 * K] = _onehot_at(states, lx, ly, vi, vj, K)
        h_below = None                                       # h^(l-1) of this row
        for l in range(nl):
            hV = frontier[l]
            ui = u
            z = expit(ui @ P[f"Wz{l}"].T + P[f"bz{l}"])
            ht = np.concatenate([ui, hV], axis=2) @ P[f"Wh{l}"].T + P[f"bh{l}"]
            # recurrence along the row in snake order, h_H = 0 at the row start
            a = z[:, cols]
            b = (1.0 - z[:, cols]) * ht[:, cols]
            hs = affine_seq(a, b) if mode == "seq" else affine_blelloch(a, b)
            h = np.empty_like(hs)
            h[:, cols] = hs
            xt = h @ P[f"C{l}"].T + ui @ P[f"D{l}"].T
            if l >= 2:
                xt = xt + h_below
            u = gelu(xt)
            frontier[l] = h
            h_below = h
            if keep_hidden:
                hidden[l][:, j * lx: (j + 1) * lx] = h
        logits = u @ P["Wo"].T + P["bo"]                     # [B, lx, K]
        for i in range(lx):
            logp[:, j * lx + i] = _site_logp(logits[:, i], states[:, j * lx + i])
    return logp, hidden


def forward(theta, spins, m: Model, mode: str = "seq", keep_hidden: bool = False):
    """Per-site log p in grid row-major order, and optionally hidden states.

    ``spins`` is an int array [B, N] with values in {0, 1}, row-major (site
    y * lx + x).  Returns ``(logp, hidden)``: logp is [B, px * py], one entry per
    site (patch = 1: [B, N] in lattice order) or per 2x2 patch (patch I + px J);
    ``hidden[l]`` is h^(l) on the same grid, [B, px * py, d], when
    ``keep_hidden`` is set, else ``None``.
    """
    spins = np.asarray(spins)
    if spins.ndim != 2 or spins.shape[1] != m.n_sites:
        raise ValueError("spins must be [B, lx*ly]")
    if spins.size and (spins.min() < 0 or spins.max() > 1):
        raise ValueError("spins must be 0 or 1")
    if mode not in ("seq", "scan"):
        raise ValueError(mode)
    P = unpack(theta, m)
    if m.geometry == "chain":
        return _forward_chain(P, spins, m, mode, keep_hidden)
    return _forward_snake(P, spins, m, mode, keep_hidden)


def logpsi(theta, spins, m: Model, mode: str = "seq") -> np.ndarray:
    """log psi(sigma) = (1/2) sum_t log p_t, float64 [B]."""
    logp, _ = forward(theta, spins, m, mode)
    return 0.5 * logp.sum(axis=1)


def all_configs(n: int) -> np.ndarray:
    """Every configuration of n sites, [2^n, n] int8; row k has site s = bit (n-1-s) of k."""
    k = np.arange(2 ** n, dtype=np.int64)[:, None]
    sh = np.arange(n - 1, -1, -1, dtype=np.int64)[None, :]
    return ((k >> sh) & 1).astype(np.int8)
