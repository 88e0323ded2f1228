"""Oracle: per-sample gradients, finite differences and VMC batch statistics.

TEST INFRASTRUCTURE -- see ``oracle/__init__.py``.

``per_sample_grad`` is a second forward of the ansatz, written separately in
float64 torch on the CPU so that autograd can differentiate it.  Every sample
gets its own copy of theta, so one backward of sum(log psi) yields every
O_s = d log psi(sigma_s) / d theta at once.  It is cross-checked against
``model.logpsi`` and against central finite differences of ``model``.

Statistics (Sec. III.B: energy minimisation with stochastic gradient
estimates; real, positive psi):
  mean  = (1/B) sum_s E_loc(s)
  var   = (1/B) sum_s (E_loc(s) - mean)^2
  g     = (2/B) sum_s (E_loc(s) - mean) O_s
"""

from __future__ import annotations

import numpy as np
import torch

from . import model as M


def _torch_forward(theta_b: torch.Tensor, spins: torch.Tensor, m: M.Model) -> torch.Tensor:
    """log psi per sample; theta_b is [B, P] (one parameter copy per sample)."""
    B, N = spins.shape
    d = m.d
    shapes = M.tensor_shapes(m)
    W, off = {}, 0
    for name, shp in shapes:
        k = int(np.prod(shp))
        W[name] = theta_b[:, off: off + k].reshape((B,) + shp)
        off += k

    def lin(w, x):            # per-sample matrix-vector: w [B, o, i], x [B, i]
        return torch.bmm(w, x.unsqueeze(2)).squeeze(2)

    sig = spins.long()
    onehot = torch.nn.functional.one_hot(sig, 2).to(theta_b.dtype)   # [B, N, 2]
    total = torch.zeros(B, dtype=theta_b.dtype)

    def add_site(xh, t):
        nonlocal total
        logits = lin(W["Wo"], xh) + W["bo"]
        lp = torch.log_softmax(logits, dim=1).gather(1, sig[:, t: t + 1]).squeeze(1)
        total = total + lp

    if m.geometry == "chain":
        h = torch.zeros(B, d, dtype=theta_b.dtype)
        x = torch.zeros(B, 2, dtype=theta_b.dtype)
        for t in range(N):
            z = torch.sigmoid(lin(W["Wz0"], x) + W["bz0"])
            hh = lin(W["Wh0"], x) + W["bh0"]
            h = z * h + (1 - z) * hh
            add_site(h, t)
            x = onehot[:, t]
        return 0.5 * total

    lx, ly, nl = m.lx, m.ly, m.n_layers
    zero2 = torch.zeros(B, 2, dtype=theta_b.dtype)
    zero_d = torch.zeros(B, d, dtype=theta_b.dtype)
    prev_row = [[zero_d] * lx for _ in range(nl)]
    for j in range(ly):
        order = range(lx) if j % 2 == 0 else range(lx - 1, -1, -1)
        step = 1 if j % 2 == 0 else -1
        cur_row = [[None] * lx for _ in range(nl)]
        h_run = [zero_d] * nl
        for i in order:
            ih = i - step
            xh = onehot[:, j * lx + ih] if 0 <= ih < lx else zero2
            xv = onehot[:, (j - 1) * lx + i] if j >= 1 else zero2
            u = torch.cat([xh, xv], dim=1)
            below = None
            for l in range(nl):
                hv = prev_row[l][i]
                z = torch.sigmoid(lin(W[f"Wz{l}"], u) + W[f"bz{l}"])
                hh = lin(W[f"Wh{l}"], torch.cat([u, hv], dim=1)) + W[f"bh{l}"]
                h = z * h_run[l] + (1 - z) * hh
                h_run[l] = h
                cur_row[l][i] = h
                pre = lin(W[f"C{l}"], h) + lin(W[f"D{l}"], u)
                if l >= 2:
                    pre = pre + below
                u = 0.5 * pre * (1 + torch.erf(pre * M.SQRT1_2))
                below = h
            add_site(u, j * lx + i)
        prev_row = cur_row
    return 0.5 * total


def per_sample_grad(theta, spins, m: M.Model):
    """(log psi [B], O [B, P]) in float64, O_s = d log psi(sigma_s) / d theta (single-site inputs)."""
    if m.patch != 1:
        raise NotImplementedError("the autograd forward covers single-site inputs")
    spins_t = torch.as_tensor(np.asarray(spins), dtype=torch.int64)
    B = spins_t.shape[0]
    th = torch.as_tensor(np.asarray(theta, dtype=np.float64))
    theta_b = th.unsqueeze(0).repeat(B, 1).requires_grad_(True)
    lp = _torch_forward(theta_b, spins_t, m)
    (g,) = torch.autograd.grad(lp.sum(), theta_b)
    return lp.detach().numpy(), g.numpy()


def finite_difference(theta, spins, m: M.Model, index: int, eps: float = 1e-5) -> np.ndarray:
    """Central difference of ``model.logpsi`` w.r.t. theta[index], per sample."""
    th = np.asarray(theta, dtype=np.float64).copy()
    th[index] += eps
    up = M.logpsi(th, spins, m)
    th[index] -= 2 * eps
    dn = M.logpsi(th, spins, m)
    return (up - dn) / (2 * eps)


def energy_stats(eloc: np.ndarray):
    """(mean, var) with the 1/B normaliser."""
    e = np.asarray(eloc, dtype=np.float64)
    mean = e.sum() / e.size
    return mean, ((e - mean) ** 2).sum() / e.size


def gradient_estimate(eloc: np.ndarray, O: np.ndarray) -> np.ndarray:
    """g = (2/B) sum_s (E_loc(s) - mean) O_s."""
    e = np.asarray(eloc, dtype=np.float64)
    mean = e.sum() / e.size
    return (2.0 / e.size) * ((e - mean) @ np.asarray(O, dtype=np.float64))
