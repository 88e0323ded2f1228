"""Write the float64 oracle's local energies for the full-size workloads' sample subsets.

The GPU tests check the library at the full 32x32 and 52x52 workloads against
these stored values, because the oracle needs minutes to hours for them (each
sample has about two thousand, or five thousand, connected configurations).
Only ``oracle/`` and the seeded generators of ``psr_inputs`` are used.

Workloads (open Heisenberg lattice, Marshall basis, J = 1; 2D snake minGRU;
parameters N(0, 1/d) from PCG64(1000 + k), Neel-like samples from PCG64(2000 + k)):
  heisenberg32x32  L = 32, 3 layers, d = 128, k = 3: the first 64 samples
  heisenberg52x52  L = 52, 4 layers, d = 256, k = 4: log psi of the first 64
                   samples, E_loc of the first 2

Each output line: sample index, number of connected configurations, log psi,
E_loc (``nan`` where not computed), as ``%.17g``.

Run from the repository root:  python tests/golden/gen_fullsize_eloc.py [workload ...]
(chunks of connected configurations are spread over worker processes, one
BLAS thread each).
"""

from __future__ import annotations

import os
import sys

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("MKL_NUM_THREADS", "1")

import multiprocessing as mp  # noqa: E402

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import psr_inputs as I  # noqa: E402
from oracle import hamiltonian as OH  # noqa: E402
from oracle import model as OM  # noqa: E402

WORKLOADS = {
    "heisenberg32x32": dict(L=32, nl=3, d=128, k=3, n_logpsi=64, n_eloc=64),
    "heisenberg52x52": dict(L=52, nl=4, d=256, k=4, n_logpsi=64, n_eloc=2),
}


def _setup(name):
    w = WORKLOADS[name]
    m = OM.Model("snake2d", w["L"], w["L"], w["nl"], w["d"])
    th = I.params(OM.n_params(m), w["d"], 1000 + w["k"])
    s = I.spins_neel_like(max(w["n_logpsi"], w["n_eloc"]), w["L"], w["L"], 2000 + w["k"])
    return w, m, th, s


def _part(args):
    """Sum of mel psi(sigma')/psi(sigma) over connected configurations [i0, i1) of sample b."""
    name, b, i0, i1 = args
    w, m, th, s = _setup(name)
    oh = OH.Hamiltonian("heisenberg", w["L"], w["L"])
    one = s[b: b + 1]
    conn = OH.connected(oh, one)
    flips = OH.apply_flips(one, conn)[i0:i1]
    lp0 = OM.logpsi(th, one, m)[0]
    lpc = OM.logpsi(th, flips, m)
    return b, i0, np.asarray(conn["mel"][i0:i1] * np.exp(lpc - lp0))


def main(names):
    for name in names:
        w, m, th, s = _setup(name)
        lp = OM.logpsi(th, s[: w["n_logpsi"]], m)
        oh = OH.Hamiltonian("heisenberg", w["L"], w["L"])
        conn = OH.connected(oh, s[: w["n_eloc"]])
        chunk = 64 if w["L"] > 40 else 256
        jobs = [(name, b, i0, min(i0 + chunk, int(conn["n_conn"][b])))
                for b in range(w["n_eloc"]) for i0 in range(0, int(conn["n_conn"][b]), chunk)]
        with mp.Pool(int(os.environ.get("GEN_WORKERS", os.cpu_count() or 1))) as pool:
            parts = pool.map(_part, jobs, chunksize=1)
        eloc = {}
        for b in range(w["n_eloc"]):
            # terms in canonical connected order, summed once in float64
            terms = np.concatenate([t for bb, _, t in sorted(parts, key=lambda p: (p[0], p[1])) if bb == b])
            eloc[b] = (int(conn["n_conn"][b]), float(conn["diag"][b]) + float(np.sum(terms)))
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle_eloc.txt")
        with open(out, "w") as f:
            f.write(f"# float64 oracle, {name}: lattice {w['L']}x{w['L']}, {w['nl']} layers, d = {w['d']}, "
                    f"theta seed {1000 + w['k']}, spin seed {2000 + w['k']} (Neel-like)\n")
            f.write("# written by tests/golden/gen_fullsize_eloc.py\n")
            f.write("# sample n_conn logpsi eloc\n")
            for b in range(w["n_logpsi"]):
                n, e = eloc.get(b, (-1, float("nan")))
                f.write(f"{b} {n} {lp[b]:.17g} {e:.17g}\n")
        print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
