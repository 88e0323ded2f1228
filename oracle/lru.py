"""Oracle: the 1D LRU ansatz -- TEST INFRASTRUCTURE (see ``oracle/__init__``).

The paper's 1D model (Sec. II.B, Eq. (lru); Sec. II.G residual with GLU;
3 layers, d = d_h = 64 in Table I).  Per layer l with input sequence x_t in R^d:

    lambda = exp(-e^nu + i e^theta)                    (complex, per hidden unit)
    h_t    = lambda * h_{t-1} + e^gamma * (B x_t),     h_{-1} = 0
    y_t    = Re(C h_t) + D * x_t
    x'_t   = GLU(y_t) + [l >= 1] x_t,   GLU(y) = (W_a y + b_a) * sigmoid(W_g y + b_g)

Readings where the paper leaves a choice:
  * The shift that makes the model autoregressive is taken once, at the input:
    the layer-0 input at site t is the embedding E[:, sigma_{t-1}] of the
    previous spin, zero at t = 0 (the zero initial input and state of the
    chain).  The x_{t-1} of Eq. (lru) is read as the layer's input at the
    position whose state h_t it forms.
  * The embedding is a learned E in R^{d x 2}; the head is a linear layer and a
    two-way softmax on x^(n_layers)_t, as for the 2D model; psi = sqrt(p).
  * GLU (Shazeer) has its own value and gate projections with biases.
  With these shapes 3 layers at d = d_h = 64 have 75,138 parameters against the
  paper's figure of about 75,000 (Table I caption).

Parameter layout (flat float vector, matrices row-major, output index first):
  E[d][2]; per layer: nu[dh], theta[dh], gamma[dh], B[2 dh][d] (rows: Re then Im),
  D[d], C[d][2 dh] (columns: Re then Im), W_glu[2 d][d] (rows: value then gate),
  b_glu[2 d]; then W_o[2][d], b_o[2].

The recurrence is evaluated sequentially in complex128; there is no scan here.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class LruModel:
    n_sites: int
    n_layers: int
    d: int
    dh: int


def tensor_shapes(m: LruModel) -> list[tuple[str, tuple[int, ...]]]:
    """(name, shape) of every tensor in layout order."""
    d, dh = m.d, m.dh
    out = [("E", (d, 2))]
    for l in range(m.n_layers):
        out += [(f"nu{l}", (dh,)), (f"theta{l}", (dh,)), (f"gamma{l}", (dh,)), (f"B{l}", (2 * dh, d)),
                (f"D{l}", (d,)), (f"C{l}", (d, 2 * dh)), (f"Wglu{l}", (2 * d, d)), (f"bglu{l}", (2 * d,))]
    out += [("W_o", (2, d)), ("b_o", (2,))]
    return out


def n_params(m: LruModel) -> int:
    return int(sum(int(np.prod(s)) for _, s in tensor_shapes(m)))


def unpack(theta, m: LruModel) -> dict[str, np.ndarray]:
    th = np.asarray(theta, dtype=np.float64)
    assert th.size == n_params(m)
    out, o = {}, 0
    for name, shape in tensor_shapes(m):
        k = int(np.prod(shape))
        out[name] = th[o:o + k].reshape(shape)
        o += k
    return out


def lam(nu, theta):
    """The diagonal propagator of Eq. (lru): exp(-e^nu + i e^theta)."""
    return np.exp(-np.exp(nu) + 1j * np.exp(theta))


def sigmoid(x):
    """The logistic function, as 1/2 (1 + tanh(x/2)) (no overflow for large |x|)."""
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def layer(x, p: dict, l: int, return_h: bool = False):
    """One LRU layer with its GLU and residual on x [B, N, d]; returns x' (and h [B, N, dh])."""
    dh = p[f"nu{l}"].shape[0]
    Bc = p[f"B{l}"][:dh] + 1j * p[f"B{l}"][dh:]          # [dh, d]
    Cc = p[f"C{l}"][:, :dh] + 1j * p[f"C{l}"][:, dh:]    # [d, dh]
    lm = lam(p[f"nu{l}"], p[f"theta{l}"])
    v = np.exp(p[f"gamma{l}"]) * (x @ Bc.T)              # drive e^gamma (B x_t), [B, N, dh]
    h = np.zeros(v.shape, dtype=np.complex128)
    state = np.zeros(v[:, 0].shape, dtype=np.complex128)
    for t in range(x.shape[1]):
        state = lm * state + v[:, t]
        h[:, t] = state
    y = (h @ Cc.T).real + p[f"D{l}"] * x
    d = x.shape[2]
    W, b = p[f"Wglu{l}"], p[f"bglu{l}"]
    g = (y @ W[:d].T + b[:d]) * sigmoid(y @ W[d:].T + b[d:])
    xn = g + (x if l >= 1 else 0.0)
    return (xn, h) if return_h else xn


def site_logp(theta, spins, m: LruModel) -> np.ndarray:
    """log p(sigma_t | sigma_<t) of every site, [B, N] (Sec. III.B autoregressive factorisation)."""
    p = unpack(theta, m)
    s = np.asarray(spins).astype(np.int64)
    Bn, N = s.shape
    assert N == m.n_sites
    x = np.zeros((Bn, N, m.d))
    if N > 1:
        x[:, 1:, :] = p["E"].T[s[:, :-1]]            # E[:, sigma_{t-1}]
    for l in range(m.n_layers):
        x = layer(x, p, l)
    logits = x @ p["W_o"].T + p["b_o"]               # [B, N, 2]
    mx = logits.max(axis=2, keepdims=True)
    lse = mx[..., 0] + np.log(np.exp(logits - mx).sum(axis=2))
    own = np.take_along_axis(logits, s[..., None], axis=2)[..., 0]
    return own - lse


def logpsi(theta, spins, m: LruModel) -> np.ndarray:
    """log psi = (1/2) sum_t log p(sigma_t | sigma_<t), [B]."""
    return 0.5 * site_logp(theta, spins, m).sum(axis=1)


def conditionals(theta, spins, m: LruModel) -> np.ndarray:
    """p(sigma_t = 1 | sigma_<t) at every site, [B, N] (the two-way softmax of the head)."""
    s = np.asarray(spins)
    p_own = np.exp(site_logp(theta, s, m))
    return np.where(s == 1, p_own, 1.0 - p_own)


def sample(theta, uniforms, m: LruModel):
    """Exact samples of the LRU chain and their log psi, drawn site by site (Sec. III.B).

    sigma_t = 1 iff uniforms[b, t] < p(sigma_t = 1 | sigma_<t); the conditional at
    site t is read from a forward over the spins drawn so far (one forward per site).
    """
    u = np.asarray(uniforms, dtype=np.float64)
    B, N = u.shape
    if N != m.n_sites:
        raise ValueError("uniforms must be [B, n_sites]")
    spins = np.zeros((B, N), dtype=np.int8)
    for t in range(N):
        p1 = conditionals(theta, spins, m)[:, t]
        spins[:, t] = (u[:, t] < p1).astype(np.int8)
    return spins, logpsi(theta, spins, m)
