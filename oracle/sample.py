"""Oracle: exact autoregressive sampling -- TEST INFRASTRUCTURE (see ``oracle/__init__``).

The wave function is the square root of an autoregressive distribution
(Sec. III.B): p(sigma) = prod_t p(sigma_t | sigma_<t), the sites taken in the
order of the factorisation (the zigzag order of Sec. II.F on the 2D lattice,
left to right on the chain).  Because every conditional depends on earlier
sites only, an exact sample is drawn by visiting the sites in that order and
drawing each spin from its conditional given the spins already drawn.

The random numbers are inputs: ``uniforms[b, t]`` decides site t of sample b
(lattice row-major) by  sigma_t = 1  iff  uniforms[b, t] < p(sigma_t = 1 | sigma_<t).
"""

from __future__ import annotations

import numpy as np

from . import model as M


def visiting_order(m: M.Model) -> list[int]:
    """Lattice row-major site indices in the order of the autoregressive factorisation."""
    if m.geometry == "chain":
        return list(range(m.n_sites))
    return [j * m.lx + i for (i, j) in M.snake_order(m.lx, m.ly)]


def conditionals(theta, spins, m: M.Model) -> np.ndarray:
    """p(sigma_t = 1 | sigma_<t) at every site of every configuration, [B, N] row-major.

    The model's per-site log p is that of the spin the configuration holds, so
    the conditional of spin 1 is p itself where sigma_t = 1 and 1 - p where
    sigma_t = 0 (Sec. III.B: two-way softmax per site).
    """
    spins = np.asarray(spins)
    logp, _ = M.forward(theta, spins, m)
    p_own = np.exp(logp)
    return np.where(spins == 1, p_own, 1.0 - p_own)


def sample(theta, uniforms, m: M.Model):
    """Exact samples and their log psi, drawn site by site (Sec. III.B).

    Returns ``(spins [B, N] int8 row-major, log psi [B])``.  Site t's
    conditional is read from a forward pass over the spins drawn so far (the
    later sites do not influence it), so the cost is one forward per site.
    """
    uniforms = np.asarray(uniforms, dtype=np.float64)
    B, N = uniforms.shape
    if N != m.n_sites:
        raise ValueError("uniforms must be [B, lx*ly]")
    spins = np.zeros((B, N), dtype=np.int8)
    for t in visiting_order(m):
        p1 = conditionals(theta, spins, m)[:, t]
        spins[:, t] = (uniforms[:, t] < p1).astype(np.int8)
    return spins, M.logpsi(theta, spins, m)
