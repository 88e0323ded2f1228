"""A full single-GPU VMC loop (f3): exact samples -> E_loc -> energy gradient -> Adam.

The loop runs the library's sampler, local energy and per-sample backward;
training must reach the exact ground energy: the open TFIM chain at h = J = 1
(the exact formula of Table I's caption), with the chain model and with the 2D
snake model on a 12 x 1 lattice (also an autoregressive model of the chain), and the 4 x 4 open TFIM at h = 3
(exact diagonalisation).  A wrong sign or scale anywhere in the sampler, E_loc
or the gradient would stop the energy short of the ground state.
"""

import numpy as np
import pytest
import torch

import psr_inputs as I
from oracle import hamiltonian as OH

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_13807_amd as P  # noqa: N813
    P.lib()
    return P


@pytest.mark.parametrize("geom,lx,ly,hfield,steps,delta0", [
    (1, 12, 1, 1.0, 1500, None),     # 2D snake model on a 12 x 1 lattice
    (0, 12, 1, 1.0, 1500, None),     # the chain model (one minGRU layer, head on h)
    (1, 4, 4, 3.0, 1500, 500.0),     # 4 x 4, with the appendix's learning-rate decay
])
def test_vmc_reaches_exact_ground_energy(P, geom, lx, ly, hfield, steps, delta0):
    from paper_2605_13807_amd.vmc import lr_decay, vmc

    if ly == 1:
        exact = lx * OH.tfim_obc_exact_energy_per_site(lx)
    else:
        exact = OH.ground_energy(OH.Hamiltonian("tfim", lx, ly, J=1.0, h=hfield))
    print(f"VMC TFIM {lx}x{ly} h={hfield}: exact ground energy {exact:.6f}", flush=True)
    m = P.Model(geom, lx, ly, 1 if geom == 0 else 2, 32, P.FP32)
    th = torch.from_numpy(I.params(P.param_count(m), 32, 1200 + lx)).cuda()
    h = P.Hamiltonian(P.TFIM, lx, ly, J=1.0, h=hfield)
    # constant learning rate, or the appendix's decay eta0 / (1 + t / delta0)
    lr = 1e-2 if delta0 is None else lr_decay(1e-2, delta0)
    hist = vmc(m, h, th, steps=steps, batch=1024, lr=lr, seed=3, log_every=250)
    e0 = hist[0][0]
    e = np.mean([x for x, _ in hist[-100:]])
    var = np.mean([v for _, v in hist[-100:]])
    rel = abs(e - exact) / abs(exact)
    print(f"  first step {e0:.6f}; mean of the last 100 steps {e:.6f} (rel err {rel:.2e}), variance {var:.3e}")
    assert rel <= 1e-3
    # variational: the mean energy does not fall below the ground energy (beyond noise)
    assert e >= exact - 5e-4 * abs(exact)
    assert var < hist[0][1]


def test_vmc_table_one_small_chains(P):
    """Table I's small open TFIM chains at h = 1: energy per site against the exact formula.

    The paper's rows use its 1D LRU ansatz; here the 2-layer d = 32 minGRU snake
    model on an N x 1 lattice, 1500 steps of 1024 samples with the appendix's
    learning-rate decay.  Prints e(N), the exact value, the relative error and
    the time per training step.
    """
    import time

    from paper_2605_13807_amd.vmc import lr_decay, vmc

    print("   N   e_vmc(N)      e_exact(N)    rel err    ms/step", flush=True)
    for n in (6, 8, 10, 16):
        exact = OH.tfim_obc_exact_energy_per_site(n)
        m = P.Model(P.SNAKE_2D, n, 1, 2, 32, P.FP32)
        th = torch.from_numpy(I.params(P.param_count(m), 32, 1300 + n)).cuda()
        h = P.Hamiltonian(P.TFIM, n, 1, J=1.0, h=1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = vmc(m, h, th, steps=1500, batch=1024, lr=lr_decay(1e-2, 500.0), seed=5)
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / 1500
        e = np.mean([x for x, _ in hist[-100:]]) / n
        rel = abs(e - exact) / abs(exact)
        print(f"  {n:3d}  {e:.7f}  {exact:.7f}  {rel:.2e}  {ms:.2f}", flush=True)
        assert rel <= 1e-3
        assert e >= exact - 5e-4 * abs(exact)


def test_vmc_lru_table_one_small_chains(P):
    """Table I's own ansatz, the 1D LRU (3 layers, d = d_h = 64, GLU residual), trained on
    the small open TFIM chains at h = 1 with the library's LRU sampler, E_loc and backward;
    energy per site against the exact formula of Table I's caption.  Prints e(N), the
    exact value, the relative error and the time per training step."""
    import time

    from paper_2605_13807_amd.vmc import lr_decay, vmc

    print("\n  LRU (3 layers, d = d_h = 64), 1024 samples, 1500 steps", flush=True)
    print("   N   e_vmc(N)      e_exact(N)    rel err    ms/step", flush=True)
    for n in (6, 10, 16):
        exact = OH.tfim_obc_exact_energy_per_site(n)
        m = P.LruModel(n, 3, 64, 64)
        th = torch.from_numpy(I.params(P.lru_param_count(m), 64, 900 + n)).cuda()
        h = P.Hamiltonian(P.TFIM, n, 1, J=1.0, h=1.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = vmc(m, h, th, steps=1500, batch=1024, lr=lr_decay(3e-3, 500.0), seed=7)
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / 1500
        e = float(np.mean([x[0] for x in hist[-100:]])) / n
        rel = abs(e - exact) / abs(exact)
        print(f"  {n:3d}  {e:.7f}  {exact:.7f}  {rel:.2e}  {ms:.2f}", flush=True)
        assert rel <= 1e-3
        assert e >= exact - 5e-4 * abs(exact)
