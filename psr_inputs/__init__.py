"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module only draws random numbers and builds spin configurations. It holds
none of the wave-function or Hamiltonian arithmetic, so that the reference
implementation under ``oracle/`` and the HIP library can both consume the same
inputs without sharing any of the computation they are compared on.

Conventions (shared by both sides as an interface, not as code):

* spins are ``int8`` in ``{0, 1}``; ``1`` is spin up (sigma^z = +1);
* a configuration is stored in lattice row-major order, site ``y * lx + x``;
* parameters are a flat ``float32`` vector, every entry drawn from
  N(0, 1/d) from one PCG64 stream in storage order (biases included).

The workloads stand in for the variational Monte Carlo batches of the paper
(Sec. III): the paper trains on samples drawn from |psi|^2, which cannot be
produced without trained weights, so random configurations of the same size,
magnetisation sector and structure are used instead.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "params",
    "spins_bernoulli",
    "spins_zero_mag",
    "spins_neel_like",
    "uniforms",
]


def rng(seed: int) -> np.random.Generator:
    """The one generator family used everywhere: ``Generator(PCG64(seed))``."""
    return np.random.Generator(np.random.PCG64(int(seed)))


def params(n_params: int, d: int, seed: int) -> np.ndarray:
    """Flat float32 parameter vector, entries i.i.d. N(0, 1/d), storage order."""
    g = rng(seed)
    return (g.standard_normal(int(n_params)) / np.sqrt(float(d))).astype(np.float32)


def spins_bernoulli(batch: int, n_sites: int, seed: int) -> np.ndarray:
    """i.i.d. Bernoulli(1/2) spins, shape [batch, n_sites], int8."""
    g = rng(seed)
    return g.integers(0, 2, size=(int(batch), int(n_sites)), dtype=np.int8)


def spins_zero_mag(batch: int, n_sites: int, seed: int) -> np.ndarray:
    """Zero-magnetisation spins: each row is a random permutation of N/2 ones."""
    if n_sites % 2:
        raise ValueError("zero magnetisation needs an even number of sites")
    g = rng(seed)
    base = np.zeros(n_sites, dtype=np.int8)
    base[: n_sites // 2] = 1
    out = np.empty((int(batch), int(n_sites)), dtype=np.int8)
    for b in range(int(batch)):
        out[b] = g.permutation(base)
    return out


def _nn_bonds(lx: int, ly: int) -> np.ndarray:
    """Open-boundary nearest-neighbour bonds of an lx-by-ly lattice, [n_bonds, 2].

    Listed site by site in row-major order; for each site the bond to its right
    neighbour comes before the bond to the neighbour one row up.  (Input
    construction only: used to place exchanges when building Neel-like states.)
    """
    out = []
    for y in range(ly):
        for x in range(lx):
            a = y * lx + x
            if x + 1 < lx:
                out.append((a, a + 1))
            if y + 1 < ly:
                out.append((a, a + lx))
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


def spins_neel_like(batch: int, lx: int, ly: int, seed: int, n_swaps: int | None = None) -> np.ndarray:
    """Neel state plus random exchanges of antiparallel nearest neighbours.

    Starts from sigma(x, y) = (x + y) mod 2 and applies ``n_swaps``
    (default floor(N/32)) exchanges, each on a uniformly drawn bond that is
    antiparallel at that moment.  Every state stays at zero magnetisation and
    keeps most bonds antiparallel, like the low-energy configurations that a
    trained Heisenberg wave function samples.
    """
    n = lx * ly
    if n_swaps is None:
        n_swaps = n // 32
    g = rng(seed)
    bonds = _nn_bonds(lx, ly)
    xs = np.arange(n) % lx
    ys = np.arange(n) // lx
    neel = ((xs + ys) % 2).astype(np.int8)
    out = np.empty((int(batch), n), dtype=np.int8)
    for b in range(int(batch)):
        s = neel.copy()
        done = 0
        while done < n_swaps:
            a, c = bonds[g.integers(0, len(bonds))]
            if s[a] != s[c]:
                s[a], s[c] = s[c], s[a]
                done += 1
        out[b] = s
    return out


def uniforms(batch: int, n_sites: int, seed: int) -> np.ndarray:
    """Random numbers for the sampler: float32 [batch, n_sites] in [0, 1), one per site."""
    return rng(seed).random((batch, n_sites), dtype=np.float32)
