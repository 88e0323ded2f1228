"""Oracle: per-sample gradients of the 1D LRU ansatz -- TEST INFRASTRUCTURE
(see ``oracle/__init__``).

``per_sample_grad`` is a second forward of the LRU model of ``oracle/lru.py``
(Sec. II.B Eq. (lru), Sec. II.G GLU residual, readings as there), written
separately in torch complex128 on the CPU so that autograd can differentiate
it.  Every sample gets its own copy of theta, so one backward of sum(log psi)
yields every O_s = d log psi(sigma_s) / d theta.  It is cross-checked against
``lru.logpsi`` and against central finite differences of ``lru.logpsi``.
"""

from __future__ import annotations

import numpy as np
import torch

from . import lru as L


def _forward(theta_b: torch.Tensor, spins: torch.Tensor, m: L.LruModel) -> torch.Tensor:
    """log psi per sample; theta_b is [B, P] float64 (one parameter copy per sample)."""
    B, N = spins.shape
    d, dh = m.d, m.dh
    W, off = {}, 0
    for name, shp in L.tensor_shapes(m):
        k = int(np.prod(shp))
        W[name] = theta_b[:, off: off + k].reshape((B,) + shp)
        off += k
    sig = spins.long()
    # layer-0 input: the embedding column of the previous spin, zero at the first site
    E = W["E"]                                                    # [B, d, 2]
    prev = torch.nn.functional.one_hot(sig[:, :-1], 2).to(theta_b.dtype)   # [B, N-1, 2]
    x = torch.cat([torch.zeros(B, 1, d, dtype=theta_b.dtype), prev @ E.transpose(1, 2)], dim=1)
    for l in range(m.n_layers):
        Bm = W[f"B{l}"]                                           # [B, 2dh, d]
        Bc = torch.complex(Bm[:, :dh], Bm[:, dh:])                # [B, dh, d]
        Cm = W[f"C{l}"]                                           # [B, d, 2dh]
        Cc = torch.complex(Cm[:, :, :dh], Cm[:, :, dh:])          # [B, d, dh]
        lam = torch.exp(torch.complex(-torch.exp(W[f"nu{l}"]), torch.exp(W[f"theta{l}"])))   # [B, dh]
        drive = torch.exp(W[f"gamma{l}"]).unsqueeze(1) * (x.to(torch.complex128) @ Bc.transpose(1, 2))  # [B, N, dh]
        hs = []
        h = torch.zeros(B, dh, dtype=torch.complex128)
        for t in range(N):
            h = lam * h + drive[:, t]
            hs.append(h)
        H = torch.stack(hs, dim=1)                                # [B, N, dh]
        y = (H @ Cc.transpose(1, 2)).real + W[f"D{l}"].unsqueeze(1) * x
        Wg, bg = W[f"Wglu{l}"], W[f"bglu{l}"]
        a = y @ Wg[:, :d].transpose(1, 2) + bg[:, None, :d]
        gate = torch.sigmoid(y @ Wg[:, d:].transpose(1, 2) + bg[:, None, d:])
        x = a * gate + (x if l >= 1 else 0.0)
    logits = x @ W["W_o"].transpose(1, 2) + W["b_o"].unsqueeze(1)   # [B, N, 2]
    lp = torch.log_softmax(logits, dim=2).gather(2, sig.unsqueeze(2)).squeeze(2)
    return 0.5 * lp.sum(dim=1)


def per_sample_grad(theta, spins, m: L.LruModel):
    """(log psi [B], O [B, P]) in float64, O_s = d log psi(sigma_s) / d theta."""
    spins_t = torch.as_tensor(np.asarray(spins), dtype=torch.int64)
    B = spins_t.shape[0]
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64))
    theta_b = th.unsqueeze(0).repeat(B, 1).requires_grad_(True)
    lp = _forward(theta_b, spins_t, m)
    (g,) = torch.autograd.grad(lp.sum(), theta_b)
    return lp.detach().numpy(), g.numpy()


def finite_difference(theta, spins, m: L.LruModel, index: int, eps: float = 1e-5) -> np.ndarray:
    """Central difference of ``lru.logpsi`` with respect to theta[index], per sample."""
    th = np.asarray(theta, dtype=np.float64).copy()
    th[index] += eps
    up = L.logpsi(th, spins, m)
    th[index] -= 2 * eps
    dn = L.logpsi(th, spins, m)
    return (up - dn) / (2 * eps)
