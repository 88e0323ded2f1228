"""Single-GPU variational Monte Carlo on top of the library (the training step of Sec. III.B).

One step: draw exact samples from |psi|^2 (``sample``), evaluate their local
energies and FP64 statistics (``local_energy``), turn them into the weights of
the energy-gradient estimator g = (2/B) sum_s (E_loc(s) - mean) d log psi(s) / d theta
(``vmc_weights``, real positive psi), get g from the per-sample backward
(``logpsi_backward``) and update theta with Adam.  Every model evaluation runs
in the HIP library; this module only strings the calls together and keeps the
optimiser state (PyTorch tensors on the same device).
"""

from __future__ import annotations

import math

import torch

from . import (OP_BACKWARD, OP_LOCAL_ENERGY, OP_SAMPLE, Hamiltonian, LruModel, Model, _lru_ws, _workspace,
               local_energy, logpsi_backward, lru_backward, lru_local_energy, lru_sample, sample, vmc_weights)


class Adam:
    """Adam (Kingma and Ba) on a flat parameter vector: m, v moments, bias-corrected step."""

    def __init__(self, n: int, device, lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8):
        self.lr, (self.b1, self.b2), self.eps = lr, betas, eps
        self.m = torch.zeros(n, dtype=torch.float64, device=device)
        self.v = torch.zeros(n, dtype=torch.float64, device=device)
        self.t = 0

    def step(self, theta: torch.Tensor, g: torch.Tensor) -> None:
        self.t += 1
        self.m.mul_(self.b1).add_(g, alpha=1.0 - self.b1)
        self.v.mul_(self.b2).addcmul_(g, g, value=1.0 - self.b2)
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        theta.sub_((self.lr * mh / (vh.sqrt() + self.eps)).to(theta.dtype))


def lr_decay(eta0: float, delta0: float):
    """Learning-rate decay of the paper's training appendix: eta(t) = eta0 / (1 + t / delta0)."""
    return lambda t: eta0 / (1.0 + t / delta0)


def n_steps(L: int, s: float, C: float, r: float, L0: int, F: float) -> int:
    """Training steps for iterative retraining at linear size L (training appendix):
    ceil(s (C exp(-r (L - L0)) + F))."""
    return int(math.ceil(s * (C * math.exp(-r * (L - L0)) + F)))


def vmc(m: Model, h: Hamiltonian, theta: torch.Tensor, steps: int, batch: int, lr=1e-3, seed: int = 0,
        log_every: int = 0):
    """Run `steps` VMC steps in place on `theta` (float32, device).  Returns [(mean E, variance)] per step.

    ``m`` is a 2D snake / chain minGRU ``Model`` or a 1D ``LruModel`` (Table I's ansatz).

    ``lr`` is a constant or a function of the step index t = 0, 1, ... (e.g.
    ``lr_decay(eta0, delta0)``).  The uniforms of the sampler come from a seeded
    torch generator on the device, so a run is reproducible for a given seed.

    Precision: the sampler and the backward run in FP32 whatever ``m.precision``
    is; only the local energies follow it.  The 16-bit paths split every
    projection operand into two parts (about 16 bits for BF16, 22 for FP16), so
    their E_loc stays within 1e-3 of the float64 model on the benchmark lattices
    (and within ~1e-5 at the small lattices a VMC run here trains) and the
    estimator pairs it with the gradient of the same model up to that error.
    """
    dev = theta.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    sched = lr if callable(lr) else (lambda t: lr)
    opt = Adam(theta.numel(), dev, lr=sched(0))
    lru = isinstance(m, LruModel)
    if lru:
        # the 1D LRU ansatz of Table I (psr_lru_* calls)
        ws_s = _lru_ws(m, OP_SAMPLE, batch, dev)
        ws_b = _lru_ws(m, OP_BACKWARD, batch, dev)
        ws_e = None
    else:
        ws_s = _workspace(m, OP_SAMPLE, batch, dev)
        ws_e = _workspace(m, OP_LOCAL_ENERGY, batch, dev)
        ws_b = _workspace(m, OP_BACKWARD, batch, dev)
    hist = []
    for k in range(steps):
        u = torch.rand(batch, m.n_sites, generator=gen, device=dev, dtype=torch.float32)
        if lru:
            spins, _ = lru_sample(m, theta, u, ws=ws_s)
            e, st, _ = lru_local_energy(m, theta, h, spins)
            w = vmc_weights(e, st)
            _, _, g = lru_backward(m, theta, spins, w=w, want_O=False, ws=ws_b)
        else:
            spins, _ = sample(m, theta, u, ws=ws_s)
            e, st, _ = local_energy(m, theta, h, spins, ws=ws_e)
            w = vmc_weights(e, st)
            _, _, g = logpsi_backward(m, theta, spins, w=w, want_O=False, ws=ws_b)
        opt.lr = sched(k)
        opt.step(theta, g)
        mean, var = (float(x) for x in st.cpu())
        hist.append((mean, var))
        if log_every and (k + 1) % log_every == 0:
            print(f"  step {k + 1}: E = {mean:.6f}, var = {var:.3e}", flush=True)
    return hist
