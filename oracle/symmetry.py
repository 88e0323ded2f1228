"""Oracle: c4v symmetrisation of the wave function, float64, CPU.

TEST INFRASTRUCTURE -- see ``oracle/__init__.py``.

The 2D runs of the paper impose the point-group symmetry of the open square
lattice, c4v (Sec. III.C and the captions of Tables II and VI), without writing
out how.  The reading used here (the usual one for positive autoregressive
wave functions, which keeps both normalisation and exact sampling): with
T_0 .. T_7 the eight symmetries of the L-by-L lattice (four rotations, each
with and without a reflection) acting on site positions,

    |psi_c4v(sigma)|^2 = (1/8) sum_k |psi(sigma o T_k)|^2,
    log psi_c4v(sigma) = (1/2) [logsumexp_k 2 log psi(sigma o T_k) - log 8],

where (sigma o T_k)(s) = sigma(T_k(s)).  Summing over the whole group makes
psi_c4v invariant, and it stays normalised because every T_k permutes the basis.
An exact sample of |psi_c4v|^2 is an exact sample of |psi|^2 carried by a
uniformly drawn T_k.
"""

from __future__ import annotations

import numpy as np
from scipy.special import logsumexp

# the eight symmetries of the square as maps (x, y) -> (x', y') on an L-by-L lattice
_MAPS = (
    lambda x, y, L: (x, y),                    # identity
    lambda x, y, L: (L - 1 - y, x),            # rotation by 90 degrees
    lambda x, y, L: (L - 1 - x, L - 1 - y),    # rotation by 180 degrees
    lambda x, y, L: (y, L - 1 - x),            # rotation by 270 degrees
    lambda x, y, L: (L - 1 - x, y),            # reflection x -> L-1-x
    lambda x, y, L: (x, L - 1 - y),            # reflection y -> L-1-y
    lambda x, y, L: (y, x),                    # reflection in the diagonal
    lambda x, y, L: (L - 1 - y, L - 1 - x),    # reflection in the anti-diagonal
)


def c4v_perms(L: int) -> np.ndarray:
    """[8, L*L]: row k maps site s = y L + x to the site T_k(s)."""
    out = np.empty((8, L * L), dtype=np.int64)
    for k, f in enumerate(_MAPS):
        for y in range(L):
            for x in range(L):
                xx, yy = f(x, y, L)
                out[k, y * L + x] = yy * L + xx
    return out


def transformed(spins: np.ndarray, L: int) -> list[np.ndarray]:
    """The eight configurations sigma o T_k, each [B, L*L]."""
    spins = np.asarray(spins)
    return [spins[:, perm] for perm in c4v_perms(L)]


def logpsi_c4v(logpsi_fn, spins: np.ndarray, L: int) -> np.ndarray:
    """log psi_c4v(sigma) = (1/2) [logsumexp_k 2 log psi(sigma o T_k) - log 8], float64 [B]."""
    lp = np.stack([logpsi_fn(t) for t in transformed(spins, L)], axis=0)   # [8, B]
    return 0.5 * (logsumexp(2.0 * lp, axis=0) - np.log(8.0))
