"""The C ABI on the CPU: the library loads, exports every symbol of
include/psr.h, and rejects bad arguments on the host with the documented codes
before queuing any GPU work (no compute call reaches a GPU here)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2605_13807_amd as P  # noqa: N813
    P.lib()
    return P


def test_exports_every_declared_symbol(P):
    with open(os.path.join(ROOT, "include", "psr.h")) as f:
        hdr = f.read()
    names = set(re.findall(r"\b(psr_[a-z_]+)\s*\(", hdr))
    assert len(names) >= 11
    for n in sorted(names):
        assert hasattr(P.lib(), n), n


def test_param_layout_matches_oracle(P):
    from oracle import model as OM
    for geom, lx, ly, nl, d in ((0, 16, 1, 1, 32), (1, 10, 10, 2, 64), (1, 32, 32, 3, 128), (1, 52, 52, 4, 256),
                                (1, 3, 2, 5, 32)):
        m = P.Model(geom, lx, ly, nl, d)
        om = OM.Model("chain" if geom == 0 else "snake2d", lx, ly, nl, d)
        off = P.param_offsets(m)
        shapes = OM.tensor_shapes(om)
        assert len(off) == len(shapes) + 1
        sizes = [int(np.prod(s)) for _, s in shapes]
        assert np.array_equal(np.diff(off), sizes)
        assert P.param_count(m) == OM.n_params(om)


def test_max_connected(P):
    assert P.max_connected(P.Hamiltonian(P.TFIM, 16, 1)) == 16
    for L in (4, 10, 20, 32, 52):
        assert P.max_connected(P.Hamiltonian(P.HEISENBERG, L, L)) == 2 * L * (L - 1)
    assert P.max_connected(P.Hamiltonian(P.HEISENBERG, 5, 3)) == 4 * 3 + 5 * 2


@pytest.mark.parametrize("kw,code", [
    (dict(geometry=7), -1),
    (dict(lx=0), -1),
    (dict(d=48), -2),
    (dict(n_layers=0), -1),
    (dict(n_layers=9), -1),
    (dict(precision=3), -1),
    (dict(ckpt_rows=-1), -1),
    (dict(lx=300, ly=300), -2),
    (dict(lx=70, d=256), -2),   # row longer than a workgroup's columns at d = 256
])
def test_model_validation(P, kw, code):
    base = dict(geometry=1, lx=4, ly=4, n_layers=2, d=32, precision=0, ckpt_rows=0)
    base.update(kw)
    m = P.Model(**base)
    with pytest.raises(P.PsrError) as e:
        P.param_count(m)
    assert e.value.code == code


def test_chain_shape_rules(P):
    with pytest.raises(P.PsrError):
        P.param_count(P.Model(0, 8, 2, 1, 32))
    with pytest.raises(P.PsrError):
        P.param_count(P.Model(0, 8, 1, 2, 32))


def test_hamiltonian_validation(P):
    with pytest.raises(P.PsrError) as e:
        P.max_connected(P.Hamiltonian(1, 4, 4, pbc=True))
    assert e.value.code == -2
    with pytest.raises(P.PsrError) as e:
        P.max_connected(P.Hamiltonian(5, 4, 4))
    assert e.value.code == -1


def test_compute_calls_check_arguments_before_any_launch(P):
    L = P.lib()
    m = P.Model(1, 4, 4, 2, 32).c()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails its host checks
    # NULL outputs
    assert L.psr_logpsi(ctypes.byref(m), fake, fake, 4, None, None, fake, 1 << 30, None) == -1
    # workspace too small
    assert L.psr_logpsi(ctypes.byref(m), fake, fake, 4, fake, None, fake, 16, None) == -3
    assert b"workspace" in L.psr_last_error()
    # negative batch
    assert L.psr_logpsi(ctypes.byref(m), fake, fake, -1, fake, None, fake, 1 << 30, None) == -1
    # lattice mismatch between model and Hamiltonian
    h = P.Hamiltonian(1, 5, 4).c()
    assert L.psr_local_energy(ctypes.byref(m), fake, ctypes.byref(h), fake, 4, 0, fake, fake, None, fake, 1 << 30,
                              None) == -1
    # capacity
    h4 = P.Hamiltonian(1, 4, 4).c()
    assert L.psr_connected(ctypes.byref(h4), fake, 4, 3, None, None, None, fake, None, None) == -5
    # conn without desc
    assert L.psr_connected(ctypes.byref(h4), fake, 4, 100, fake, None, None, fake, None, None) == -1
    # backward: w without g, nothing requested
    assert L.psr_logpsi_backward(ctypes.byref(m), fake, fake, 4, None, None, fake, None, fake, 1 << 30, None) == -1
    assert L.psr_logpsi_backward(ctypes.byref(m), fake, fake, 4, None, None, None, None, fake, 1 << 30, None) == -1
    # sampler: NULL outputs, workspace too small (2D and chain), negative batch
    assert L.psr_sample(ctypes.byref(m), fake, fake, 4, None, fake, fake, 1 << 30, None) == -1
    assert L.psr_sample(ctypes.byref(m), fake, fake, 4, fake, fake, fake, 16, None) == -3
    chain = P.Model(0, 16, 1, 1, 32).c()
    assert L.psr_workspace_bytes(ctypes.byref(chain), 3, 4, 0) > 0
    assert L.psr_sample(ctypes.byref(chain), fake, fake, 4, fake, fake, fake, 16, None) == -3
    assert L.psr_sample(ctypes.byref(m), fake, fake, -1, fake, fake, fake, 1 << 30, None) == -1
    assert L.psr_workspace_bytes(ctypes.byref(m), 3, 17, 0) > 0
    # empty batches are no-ops that succeed
    assert L.psr_sample(ctypes.byref(m), None, None, 0, None, None, None, 0, None) == 0
    assert L.psr_logpsi(ctypes.byref(m), None, None, 0, None, None, None, 0, None) == 0
    assert L.psr_last_error() == b""


def test_workspace_sizes_grow_with_batch(P):
    m = P.Model(1, 10, 10, 2, 64)
    for op in (0, 1, 2):
        a = P.workspace_bytes(m, op, 100, 1000)
        b = P.workspace_bytes(m, op, 200, 1000)
        assert 0 < a < b



def test_lru_layout_and_host_checks(P):
    from oracle import lru as OL
    for n, nl, d, dh in ((256, 3, 64, 64), (8, 1, 16, 32), (100, 2, 32, 16), (1, 8, 256, 256)):
        assert P.lru_param_count(P.LruModel(n, nl, d, dh)) == OL.n_params(OL.LruModel(n, nl, d, dh))
    assert P.lru_param_count(P.LruModel(64, 3, 64, 64)) == 75138
    L = P.lib()
    for bad in ((0, 1, 64, 64), (16385, 1, 64, 64), (8, 0, 64, 64), (8, 9, 64, 64), (8, 1, 24, 64),
                (8, 1, 64, 8), (8, 1, 272, 64)):
        assert L.psr_lru_param_count(ctypes.byref(P.LruModel(*bad).c())) == -1, bad
    assert L.psr_lru_param_count(None) == -1
    m = P.LruModel(256, 3, 64, 64).c()
    fake = ctypes.c_void_p(16)
    assert L.psr_lru_workspace_bytes(ctypes.byref(m), -1) == -1
    assert L.psr_lru_workspace_bytes(ctypes.byref(m), 0) == 0
    small, big = (L.psr_lru_workspace_bytes(ctypes.byref(m), b) for b in (3, 300000))
    assert 0 < small <= big
    # NULL outputs, workspace too small, negative batch: rejected before any launch
    assert L.psr_lru_logpsi(ctypes.byref(m), fake, fake, 4, None, None, fake, 1 << 40, None) == -1
    assert L.psr_lru_logpsi(ctypes.byref(m), fake, fake, 4, fake, None, fake, 16, None) == -3
    assert L.psr_lru_logpsi(ctypes.byref(m), fake, fake, 4, fake, None, None, 1 << 40, None) == -3
    assert L.psr_lru_logpsi(ctypes.byref(m), fake, fake, -1, fake, None, fake, 1 << 40, None) == -1
    assert L.psr_lru_logpsi(ctypes.byref(m), None, None, 0, None, None, None, 0, None) == 0
    assert L.psr_last_error() == b""


def test_lru_local_energy_host_checks(P):
    L = P.lib()
    fake = ctypes.c_void_p(16)
    m = P.LruModel(16, 2, 32, 32).c()
    h_ok = P.Hamiltonian(P.TFIM, 16, 1).c()
    assert L.psr_lru_eloc_workspace_bytes(ctypes.byref(m), ctypes.byref(h_ok), 10) > 0
    assert L.psr_lru_eloc_workspace_bytes(ctypes.byref(m), ctypes.byref(h_ok), -1) == -1
    for bad in (P.Hamiltonian(P.TFIM, 15, 1), P.Hamiltonian(P.HEISENBERG, 8, 2), P.Hamiltonian(P.TFIM, 16, 1, pbc=True)):
        code = L.psr_lru_local_energy(ctypes.byref(m), fake, ctypes.byref(bad.c()), fake, 4, fake, fake, None, fake,
                                      1 << 40, None)
        assert code in (-1, -2), bad
    # NULL outputs, workspace too small, empty batch
    assert L.psr_lru_local_energy(ctypes.byref(m), fake, ctypes.byref(h_ok), fake, 4, None, fake, None, fake, 1 << 40,
                                  None) == -1
    assert L.psr_lru_local_energy(ctypes.byref(m), fake, ctypes.byref(h_ok), fake, 4, fake, fake, None, fake, 64,
                                  None) == -3
    assert L.psr_lru_local_energy(ctypes.byref(m), None, ctypes.byref(h_ok), None, 0, None, None, None, None, 0,
                                  None) == 0


def test_logpsi_static_limits_on_host(P):
    """The allocation-free entry point states its scratch size and rejects a batch
    whose workspace exceeds it on the host, before touching a GPU."""
    L = P.lib()
    cap = L.psr_static_scratch_bytes()
    assert cap == 64 << 20
    m = P.Model(P.SNAKE_2D, 52, 52, 4, 256, P.BF16)
    big = 4096
    assert P.workspace_bytes(m, P.OP_LOGPSI, big) > cap
    d = m.c()
    code = L.psr_logpsi_static(ctypes.byref(d), ctypes.c_void_p(16), ctypes.c_void_p(16), big,
                               ctypes.c_void_p(16), None, None)
    assert code == -3
    assert b"static scratch" in L.psr_last_error()
    assert L.psr_logpsi_static(ctypes.byref(d), None, None, 0, None, None, None) == 0


def test_patch_and_symmetry_checks_on_host(P):
    """2x2 patches need even sides on the snake, c4v a square lattice; the backward and
    the sampler reject both; log p per site is not defined under c4v.  Parameter
    counts follow the oracle's layout."""
    from oracle import model as OM
    L = P.lib()
    m = P.Model(P.SNAKE_2D, 5, 4, 2, 32, P.FP32, 0, 2, 0)
    assert L.psr_param_count(ctypes.byref(m.c())) == -1
    m = P.Model(P.SNAKE_2D, 6, 4, 2, 32, P.FP32, 0, 1, 1)
    assert L.psr_param_count(ctypes.byref(m.c())) == -1
    m = P.Model(P.SNAKE_2D, 6, 4, 2, 32, P.FP32, 0, 3, 0)
    assert L.psr_param_count(ctypes.byref(m.c())) == -1
    for lx, ly, nl, d in ((4, 4, 2, 32), (52, 52, 3, 256), (10, 6, 6, 64)):
        m = P.Model(P.SNAKE_2D, lx, ly, nl, d, P.BF16, 0, 2, 0)
        assert P.param_count(m) == OM.n_params(OM.Model("snake2d", lx, ly, nl, d, patch=2))
    m = P.Model(P.SNAKE_2D, 4, 4, 2, 32, P.FP32, 0, 2, 1)
    d = m.c()
    p16 = ctypes.c_void_p(16)
    assert L.psr_logpsi_backward(ctypes.byref(d), p16, p16, 1, p16, None, None, None, p16, 1 << 30, None) == -2
    assert L.psr_sample(ctypes.byref(d), p16, p16, 1, p16, p16, p16, 1 << 30, None) == -2
    assert L.psr_logpsi(ctypes.byref(d), p16, p16, 1, p16, p16, p16, 1 << 30, None) == -1
