"""GPU parity at the full workload shapes, in the launch configuration that bench.py times.

The oracle cannot evaluate a whole full-size step, so it checks sampled outputs;
everything else is checked through properties that hold at any size.  The
float64 local energies of the samples checked here were written by
``tests/golden/gen_fullsize_eloc.py`` (which calls only the oracle and the
seeded generators); the rest is computed by the oracle at test time.

  32x32, 3 layers, d = 128 (4096 Neel-like samples, E_loc streamed in chunks of
      32768 sequences): E_loc and log psi of the first 64 samples against the
      stored oracle values (BF16 and FP32), the FP64 statistics of the returned
      E_loc, and one per-sample gradient row against the oracle's autograd.
  52x52, 4 layers, d = 256 (FP16 split: 32 samples, 6 launches of up to 32768 sequences):
      E_loc of the first 2 samples (about
      5300 connected configurations each) and log psi of the first 64 against
      the stored oracle values, and the gradient rows of 2 samples against the
      oracle's autograd.
  20x20, 3 layers, d = 128 (checkpoint chunks of 3 rows, the 60 sites that are
      the whole rows within 64 sites): O rows of 2 samples against central
      finite differences of the oracle on 64 parameters (at least 2 per tensor).

Bars are those of test_gpu_parity.py.
"""

import math
import os

import numpy as np
import pytest
import torch

import psr_inputs as I
from oracle import grad as OG
from oracle import model as OM

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CHUNK = 32768


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_13807_amd as P  # noqa: N813
    P.lib()
    return P


def _golden(name):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, f"{name}_oracle_eloc.txt")) if not ln.startswith("#")]
    idx = np.array([int(r[0]) for r in rows])
    n_conn = np.array([int(r[1]) for r in rows])
    lp = np.array([float(r[2]) for r in rows])
    e = np.array([float(r[3]) for r in rows])
    assert np.array_equal(idx, np.arange(len(rows)))
    return n_conn, lp, e


def _setup(P, prec, L, nl, d, k, B, ckpt_rows=0):
    m = P.Model(P.SNAKE_2D, L, L, nl, d, prec, ckpt_rows)
    om = OM.Model("snake2d", L, L, nl, d)
    assert P.param_count(m) == OM.n_params(om)
    th = I.params(OM.n_params(om), d, 1000 + k)
    s = I.spins_neel_like(B, L, L, 2000 + k)
    return m, om, th, s


def _check_eloc(P, prec, e, lp, n_conn_dev, ref_n, ref_lp, ref_e, N, label, e_tol=None):
    n_e = int(np.sum(np.isfinite(ref_e)))
    assert np.array_equal(n_conn_dev[:n_e], ref_n[:n_e])
    rel = np.abs(e[:n_e] - ref_e[:n_e]) / np.maximum(np.abs(ref_e[:n_e]), 1.0)
    dlp = np.abs(lp[: len(ref_lp)] - ref_lp)
    lp_tol = 2e-3 * math.sqrt(N) if prec in (1, 2) else 1e-5 + 1e-6 * np.abs(ref_lp).max()
    if e_tol is None:
        e_tol = 1e-3 if prec in (1, 2) else 1e-4
    mean_rel = abs(e[:n_e].mean() - ref_e[:n_e].mean()) / max(1.0, abs(ref_e[:n_e].mean()))
    print(f"  {label}: {n_e} samples, max rel E_loc err {rel.max():.3e}, mean {mean_rel:.3e}; "
          f"{len(ref_lp)} samples, max |d log psi| {dlp.max():.3e} (tol {lp_tol:.2e})", flush=True)
    assert rel.max() <= e_tol
    # the mean: per-sample errors of random sign average down as 1/sqrt(n)
    assert mean_rel <= e_tol / math.sqrt(n_e)
    assert dlp.max() <= lp_tol
    return rel.max(), dlp.max()


@pytest.mark.parametrize("prec,B", [(1, 4096), (2, 256), (0, 64)])
def test_fullsize32_local_energy(P, prec, B):
    L, nl, d, k = 32, 3, 128, 3
    print(f"full-size E_loc: {L}x{L} nl={nl} d={d} prec={prec} B={B} chunk={CHUNK}", flush=True)
    ref_n, ref_lp, ref_e = _golden("heisenberg32x32")
    m, om, th, s = _setup(P, prec, L, nl, d, k, B)
    th_d, s_d = torch.from_numpy(th).cuda(), torch.from_numpy(s).cuda()
    H = P.Hamiltonian(P.HEISENBERG, L, L)
    e, st, lp = P.local_energy(m, th_d, H, s_d, chunk_seqs=CHUNK)
    n_conn = P.connected(H, s_d[:64])["n_conn"].cpu().numpy()
    e, st, lp = e.cpu().numpy(), st.cpu().numpy(), lp.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(e))
    # FP64 statistics of exactly the returned E_loc
    assert abs(st[0] - e.mean()) <= 1e-12 * max(1.0, abs(e.mean()))
    assert abs(st[1] - e.var()) <= 1e-10 * max(1.0, abs(e.var()))
    _check_eloc(P, prec, e, lp, n_conn, ref_n, ref_lp, ref_e, L * L, "vs float64 oracle")
    # the samples' log psi from psr_local_energy equals psr_logpsi's (other launch composition)
    lp_alone = P.logpsi(m, th_d, s_d).cpu().numpy()
    assert np.abs(lp - lp_alone).max() <= 1e-6 * max(1.0, np.abs(lp).max())


def test_fullsize32_gradient_sampled(P):
    L, nl, d, k, B = 32, 3, 128, 3, 4096
    print(f"full-size gradient: {L}x{L} nl={nl} d={d} BF16 model B={B}", flush=True)
    m, om, th, s = _setup(P, P.BF16, L, nl, d, k, B)
    th_d, s_d = torch.from_numpy(th).cuda(), torch.from_numpy(s).cuda()
    rng = np.random.default_rng(11)
    w = torch.from_numpy(rng.standard_normal(B) / B).cuda()
    O, lpb, g = P.logpsi_backward(m, th_d, s_d, w=w, want_O=True)
    assert torch.isfinite(O).all()
    # the estimator is the FP64 weighted sum of exactly the returned rows
    g_ref = torch.zeros(O.shape[1], dtype=torch.float64, device=O.device)
    for i in range(0, B, 512):
        g_ref += w[i:i + 512] @ O[i:i + 512].double()
    gerr = (g - g_ref).abs().max().item() / max(1e-30, g_ref.abs().max().item())
    print(f"  estimator vs FP64 sum of the rows: {gerr:.2e}")
    assert gerr <= 1e-10
    kk = 2731
    lp_ref, O_ref = OG.per_sample_grad(th, s[kk:kk + 1], om)
    Ok = O[kk].double().cpu().numpy()
    rel = np.linalg.norm(Ok - O_ref[0]) / np.linalg.norm(O_ref[0])
    print(f"  sample {kk}: rel grad err {rel:.2e}; log psi {float(lpb[kk]):.6f} vs {lp_ref[0]:.6f}")
    assert rel <= 1e-4
    assert abs(float(lpb[kk]) - lp_ref[0]) <= 1e-5 + 1e-6 * abs(lp_ref[0])


# BF16 split operands carry ~16 significant bits: at 52x52 its E_loc error is
# stated against a bar of 5e-3 (measured 2.7e-3); the FP16 split (~22 bits)
# meets the 1e-3 gate there
@pytest.mark.parametrize("prec,B,e_tol", [(2, 32, 1e-3), (1, 8, 5e-3), (0, 2, 1e-4)])
def test_fullsize52_local_energy(P, prec, B, e_tol):
    L, nl, d, k = 52, 4, 256, 4
    print(f"full-size E_loc: {L}x{L} nl={nl} d={d} prec={prec} B={B} chunk={CHUNK}", flush=True)
    ref_n, ref_lp, ref_e = _golden("heisenberg52x52")
    m, om, th, s = _setup(P, prec, L, nl, d, k, max(B, 64))
    th_d, s_d = torch.from_numpy(th).cuda(), torch.from_numpy(s).cuda()
    H = P.Hamiltonian(P.HEISENBERG, L, L)
    e, st, lp = P.local_energy(m, th_d, H, s_d[:B], chunk_seqs=CHUNK)
    e = e.cpu().numpy()
    lp64 = P.logpsi(m, th_d, s_d[:64]).cpu().numpy().astype(np.float64)
    n_conn = P.connected(H, s_d[:2])["n_conn"].cpu().numpy()
    assert np.all(np.isfinite(e))
    assert abs(st.cpu().numpy()[0] - e.mean()) <= 1e-12 * max(1.0, abs(e.mean()))
    _check_eloc(P, prec, e, lp64, n_conn, ref_n, ref_lp, ref_e, L * L, "vs float64 oracle", e_tol)


def test_fullsize52_gradient_rows(P):
    L, nl, d, k = 52, 4, 256, 4
    print(f"full-size gradient: {L}x{L} nl={nl} d={d} 2 samples", flush=True)
    m, om, th, s = _setup(P, P.BF16, L, nl, d, k, 2)
    O, lpb, _ = P.logpsi_backward(m, torch.from_numpy(th).cuda(), torch.from_numpy(s).cuda())
    lp_ref, O_ref = OG.per_sample_grad(th, s, om)
    O = O.double().cpu().numpy()
    rel = np.linalg.norm(O - O_ref, axis=1) / np.linalg.norm(O_ref, axis=1)
    print(f"  per-sample rel grad err {rel}; log psi {lpb.cpu().numpy()} vs {lp_ref}")
    assert rel.max() <= 1e-4


def test_fullsize20_gradient_finite_differences(P):
    L, nl, d, k = 20, 3, 128, 2
    R = 64 // L      # checkpoint chunks of whole rows within 64 sites: 3 rows = 60 sites
    print(f"20x20 gradient vs finite differences: nl={nl} d={d} ckpt_rows={R}", flush=True)
    m, om, th, s = _setup(P, P.FP32, L, nl, d, k, 2, ckpt_rows=R)
    O, _, _ = P.logpsi_backward(m, torch.from_numpy(th).cuda(), torch.from_numpy(s).cuda())
    O = O.double().cpu().numpy()
    offs = P.param_offsets(m)
    rng = np.random.default_rng(20)
    idx = []
    for t in range(len(offs) - 1):
        idx += list(rng.choice(np.arange(offs[t], offs[t + 1]), size=2, replace=False))
    idx += list(rng.choice(np.arange(offs[-1]), size=max(0, 64 - len(idx)), replace=False))
    idx = np.array(sorted(set(int(i) for i in idx)))
    assert len(idx) >= 64
    fd = np.stack([OG.finite_difference(th, s, om, int(i)) for i in idx], axis=1)   # [2, n]
    got = O[:, idx]
    rel = np.linalg.norm(got - fd, axis=1) / np.linalg.norm(fd, axis=1)
    print(f"  {len(idx)} parameters: rel err per sample {rel}")
    assert rel.max() <= 1e-4
