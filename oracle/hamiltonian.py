"""Oracle: Hamiltonians, connected configurations and the local energy, float64.

TEST INFRASTRUCTURE -- see ``oracle/__init__.py``.

Models (Sec. III.B and III.C of the paper):

* transverse-field Ising, open chain:  H = -J sum_{i<N} Z_i Z_{i+1} - h sum_i X_i
  (the paper writes J = 1).  On a 2D lattice the same form is used with the
  open-boundary nearest-neighbour bonds.
* spin-1/2 Heisenberg antiferromagnet on the open square lattice:
  H = J sum_<ab> S_a . S_b with S = sigma / 2.  After the Marshall sign
  rotation the model is sign-free (stoquastic).

Basis: a configuration sigma has sigma_a in {0, 1} per site, 1 = up, and
s_a = 2 sigma_a - 1 is the Z eigenvalue.  Sites are numbered row-major,
a = y * lx + x.

Canonical order of connected configurations (a reading: the paper lists none):
sites ascending; for each site a, the bond to the right neighbour (a, a+1)
before the bond to the upper neighbour (a, a+lx).  Heisenberg keeps only bonds
whose two spins differ (the exchange swaps them); TFIM flips each site once, in
ascending order.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True)
class Hamiltonian:
    kind: str          # "tfim" | "heisenberg"
    lx: int
    ly: int
    J: float = 1.0
    h: float = 1.0     # transverse field (TFIM only)
    marshall: bool = True   # Heisenberg only: apply the Marshall sign rotation

    @property
    def n_sites(self) -> int:
        return self.lx * self.ly

    def __post_init__(self):
        if self.kind not in ("tfim", "heisenberg"):
            raise ValueError(self.kind)


def bonds(lx: int, ly: int) -> list[tuple[int, int]]:
    """Open-boundary nearest-neighbour bonds in canonical order."""
    out = []
    for a in range(lx * ly):
        x, y = a % lx, a // lx
        if x + 1 < lx:
            out.append((a, a + 1))
        if y + 1 < ly:
            out.append((a, a + lx))
    return out


def max_connected(ham: Hamiltonian) -> int:
    """Largest number of connected configurations one sample can have."""
    return ham.n_sites if ham.kind == "tfim" else len(bonds(ham.lx, ham.ly))


def connected(ham: Hamiltonian, spins: np.ndarray):
    """Off-diagonal neighbours of every sample (Sec. II.A, local energy).

    Returns a dict with
      ``diag``   [B]  diagonal element <sigma|H|sigma>,
      ``n_conn`` [B]  number of connected configurations,
      ``sample``, ``a``, ``b``, ``mel`` (flat, canonical order, sample-major):
                 the connected configuration is sigma with sites a and b
                 flipped (a == b: one site flipped), and ``mel`` is
                 <sigma|H|sigma'>.
    """
    spins = np.asarray(spins)
    B, N = spins.shape
    if N != ham.n_sites:
        raise ValueError("spins do not match the lattice")
    s = 2.0 * spins.astype(np.float64) - 1.0
    bl = bonds(ham.lx, ham.ly)
    diag = np.zeros(B)
    for a, b in bl:
        diag += s[:, a] * s[:, b]
    samp, fa, fb, mel, n_conn = [], [], [], [], np.zeros(B, dtype=np.int64)
    if ham.kind == "tfim":
        diag *= -ham.J
        for k in range(B):
            for a in range(N):
                samp.append(k)
                fa.append(a)
                fb.append(a)
                mel.append(-ham.h)
            n_conn[k] = N
    else:
        diag *= ham.J / 4.0
        off = -ham.J / 2.0 if ham.marshall else ham.J / 2.0
        for k in range(B):
            c = 0
            for a, b in bl:
                if spins[k, a] != spins[k, b]:
                    samp.append(k)
                    fa.append(a)
                    fb.append(b)
                    mel.append(off)
                    c += 1
            n_conn[k] = c
    return {
        "diag": diag,
        "n_conn": n_conn,
        "sample": np.asarray(samp, dtype=np.int64),
        "a": np.asarray(fa, dtype=np.int64),
        "b": np.asarray(fb, dtype=np.int64),
        "mel": np.asarray(mel, dtype=np.float64),
    }


def apply_flips(spins: np.ndarray, conn: dict) -> np.ndarray:
    """The connected configurations themselves, [n_total, N] int8."""
    spins = np.asarray(spins)
    out = spins[conn["sample"]].copy()
    r = np.arange(out.shape[0])
    out[r, conn["a"]] ^= 1
    two = conn["a"] != conn["b"]
    out[r[two], conn["b"][two]] ^= 1
    return out


def local_energy(logpsi_fn, ham: Hamiltonian, spins: np.ndarray) -> np.ndarray:
    """E_loc(sigma) = sum_sigma' H(sigma, sigma') psi(sigma') / psi(sigma).

    ``logpsi_fn`` maps an int8 batch [M, N] to log psi [M] (real, psi > 0).
    """
    spins = np.asarray(spins)
    conn = connected(ham, spins)
    lp = logpsi_fn(spins)
    e = conn["diag"].copy()
    if conn["sample"].size:
        lpc = logpsi_fn(apply_flips(spins, conn))
        ratio = np.exp(lpc - lp[conn["sample"]])
        np.add.at(e, conn["sample"], conn["mel"] * ratio)
    return e


# ----------------------------------------------------------------------------
# Dense / sparse Hamiltonians from Pauli Kronecker products (independent of the
# enumeration above).  Basis index n = sum_a sigma_a 2^(N-1-a): site 0 is the
# most significant factor.  Local basis order (down, up) = (sigma 0, sigma 1).
# ----------------------------------------------------------------------------

_X = np.array([[0.0, 1.0], [1.0, 0.0]])
_Y = np.array([[0.0, 1.0j], [-1.0j, 0.0]])   # sigma^y written in the (down, up) basis
_Z = np.array([[-1.0, 0.0], [0.0, 1.0]])


def _site_op(op, a: int, n: int):
    return sp.kron(sp.kron(sp.identity(2 ** a, format="csr"), sp.csr_matrix(op)),
                   sp.identity(2 ** (n - a - 1), format="csr"), format="csr")


def sparse_hamiltonian(ham: Hamiltonian):
    """H as a scipy.sparse CSR matrix (real), 2^N x 2^N."""
    n = ham.n_sites
    ops = {c: [_site_op(m, a, n) for a in range(n)] for c, m in (("x", _X), ("y", _Y), ("z", _Z))}
    H = sp.csr_matrix((2 ** n, 2 ** n), dtype=np.complex128)
    bl = bonds(ham.lx, ham.ly)
    if ham.kind == "tfim":
        for a, b in bl:
            H = H - ham.J * (ops["z"][a] @ ops["z"][b])
        for a in range(n):
            H = H - ham.h * ops["x"][a]
    else:
        for a, b in bl:
            H = H + (ham.J / 4.0) * (ops["x"][a] @ ops["x"][b] + ops["y"][a] @ ops["y"][b]
                                     + ops["z"][a] @ ops["z"][b])
        if ham.marshall:
            # U = diag((-1)^(number of up spins on sublattice A)), A = {(x + y) even}
            cfg = all_bits(n)
            xs = np.arange(n) % ham.lx
            ys = np.arange(n) // ham.lx
            on_a = ((xs + ys) % 2 == 0)
            sign = np.where(cfg[:, on_a].sum(axis=1) % 2 == 0, 1.0, -1.0)
            U = sp.diags(sign)
            H = U @ H @ U
    imag = abs(H.imag).max() if H.nnz else 0.0
    if imag > 1e-12:
        raise AssertionError("Hamiltonian is not real")
    return sp.csr_matrix(H.real)


def all_bits(n: int) -> np.ndarray:
    """Configuration of every basis index, [2^n, n] int8 (site a = bit n-1-a)."""
    k = np.arange(2 ** n, dtype=np.int64)[:, None]
    sh = np.arange(n - 1, -1, -1, dtype=np.int64)[None, :]
    return ((k >> sh) & 1).astype(np.int8)


def local_energy_dense(logpsi_all: np.ndarray, ham: Hamiltonian) -> np.ndarray:
    """E_loc for every basis state from H psi / psi (psi from log psi of all states)."""
    H = sparse_hamiltonian(ham)
    psi = np.exp(np.asarray(logpsi_all, dtype=np.float64))
    return (H @ psi) / psi


def ground_energy(ham: Hamiltonian) -> float:
    """Lowest eigenvalue of H (dense for small N, Lanczos otherwise)."""
    H = sparse_hamiltonian(ham)
    if H.shape[0] <= 4096:
        return float(np.linalg.eigvalsh(H.toarray())[0])
    from scipy.sparse.linalg import eigsh
    return float(eigsh(H, k=1, which="SA", tol=1e-12)[0][0])


def tfim_obc_exact_energy_per_site(n: int) -> float:
    """Exact ground energy per site of the open TFIM at h = J = 1 (Table I caption).

    e(N) = [1 - csc(pi / (2 (2N + 1)))] / N.
    """
    return (1.0 - 1.0 / np.sin(np.pi / (2.0 * (2 * n + 1)))) / n
