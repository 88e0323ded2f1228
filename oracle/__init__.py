"""Reference ("oracle") implementation of the PSR-NQS hot path -- TEST INFRASTRUCTURE.

Plain, slow, float64 CPU code written from the paper (Merali, Hibat-Allah,
Kohandel, Scalettar, Khatami, "Parallel Scan Recurrent Neural Quantum States
for Scalable Variational Monte Carlo"), used only to check the HIP library.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with ``paper_2605_13807_amd``
and imports nothing from it; the two meet only through the seeded inputs of
``psr_inputs``.

Modules
-------
``model``        geometry, parameter layout, the 1D minGRU chain and the 2D
                 snake minGRU (single sites or 2x2 patches), log psi by the
                 sequential recurrence (authority) and by an independent
                 Blelloch scan over each row.
``hamiltonian``  TFIM and (Marshall-rotated) Heisenberg: canonical connected
                 configurations, matrix elements, diagonal part, E_loc, dense
                 Hamiltonians from Pauli Kronecker products, exact spectra.
``sample``       exact autoregressive sampling with given uniforms, site by
                 site in the order of the factorisation.
``symmetry``     the eight symmetries of the square lattice (c4v) and the
                 symmetrised log psi of the 2D runs.
``lru``          the 1D LRU ansatz (complex diagonal recurrence, GLU, residual):
                 parameter layout, log psi by the sequential recurrence, and
                 exact site-by-site sampling.
``lru_grad``     per-sample d log psi / d theta of the LRU by float64 torch
                 autograd (a second, separately written complex forward) and
                 central finite differences of ``lru``.
``grad``         per-sample d log psi / d theta by float64 torch autograd on
                 the CPU (a second, separately written forward), central finite
                 differences of ``model``, and the VMC batch statistics.

Every function cites the passage of the paper it follows.  Pins (what fixes
each function other than itself) live in ``tests/test_oracle_pins.py`` and
``tests/test_oracle_lru_pins.py``.
"""

from . import model, hamiltonian, sample, lru, symmetry  # noqa: F401
