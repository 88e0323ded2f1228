"""GPU parity at the full 32x32 workload, in the launch configuration that bench.py times.

The 32x32 open Heisenberg model (3 layers, d = 128) with the benchmark's seeds,
4096 Neel-like samples and E_loc streamed in 32768-sequence chunks.  The oracle
cannot evaluate the whole workload, so it checks sampled outputs one by one;
everything else is checked through properties that hold at any size.
Tolerances are those of test_gpu_parity.py.
"""

import numpy as np
import pytest
import torch

import psr_inputs as I
from oracle import grad as OG
from oracle import hamiltonian as OH
from oracle import model as OM

pytestmark = pytest.mark.gpu

L, NL, D, SEED = 32, 3, 128, 3     # the heisenberg32x32 workload: lattice side, layers, width, seed index
B_FULL, CHUNK = 4096, 32768
SAMPLED = (0, 2731)                # samples checked against the oracle


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_13807_amd as P  # noqa: N813
    P.lib()
    return P


def _setup(P, prec, B):
    m = P.Model(P.SNAKE_2D, L, L, NL, D, prec)
    om = OM.Model("snake2d", L, L, NL, D)
    assert P.param_count(m) == OM.n_params(om)
    th = I.params(OM.n_params(om), D, 1000 + SEED)
    s = I.spins_neel_like(B, L, L, 2000 + SEED)
    return m, om, th, s


def _logpsi64(P, m, th_d, seqs):
    """log psi summed in float64 from the per-site log p the kernel sums itself."""
    _, lps = P.logpsi(m, th_d, seqs, site_logp=True)
    return 0.5 * lps.double().sum(dim=1).cpu().numpy()


def _eloc_from_logpsi(P, m, th_d, H, s_one):
    """E_loc of one sample from the library's own log psi of its connected set (float64 combine)."""
    c = P.connected(H, s_one, configs=True)
    n = int(c["n_conn"][0].item())
    conf = c["conn"][0, :n].contiguous()
    lp0 = _logpsi64(P, m, th_d, s_one)[0]
    lpc = _logpsi64(P, m, th_d, conf)
    mel = c["mel"][0, :n].double().cpu().numpy()
    return float(c["diag"][0].item()) + float(np.sum(mel * np.exp(lpc - lp0))), conf


def test_fullsize_local_energy_bf16(P):
    print(f"full-size E_loc: {L}x{L} nl={NL} d={D} BF16 B={B_FULL} chunk={CHUNK}", flush=True)
    m, om, th, s = _setup(P, P.BF16, B_FULL)
    th_d = torch.from_numpy(th).cuda()
    s_d = torch.from_numpy(s).cuda()
    H = P.Hamiltonian(P.HEISENBERG, L, L)
    e, st, lp = P.local_energy(m, th_d, H, s_d, chunk_seqs=CHUNK)
    e = e.cpu().numpy()
    st = st.cpu().numpy()
    assert np.all(np.isfinite(e))
    # FP64 statistics of exactly the returned E_loc
    assert abs(st[0] - e.mean()) <= 1e-12 * max(1.0, abs(e.mean()))
    assert abs(st[1] - e.var()) <= 1e-10 * max(1.0, abs(e.var()))
    # the samples' log psi: the same kernel in a different launch composition
    lp_alone = P.logpsi(m, th_d, s_d).cpu().numpy()
    lp = lp.cpu().numpy()
    assert np.abs(lp - lp_alone).max() <= 1e-6 * max(1.0, np.abs(lp).max())
    rng = np.random.default_rng(5)
    for k in SAMPLED:
        # E_loc of this sample rebuilt from its connected set, evaluated in a small launch
        e_k, conf = _eloc_from_logpsi(P, m, th_d, H, s_d[k:k + 1])
        print(f"  sample {k}: E_loc {e[k]:.9f} streamed vs {e_k:.9f} rebuilt, {conf.shape[0]} connected")
        assert abs(e[k] - e_k) <= 1e-5 * max(1.0, abs(e_k))
        # log psi of the sample and of 15 sampled connected configurations against the BF16 reading
        pick = torch.from_numpy(rng.choice(conf.shape[0], size=15, replace=False)).to(conf.device)
        seqs = np.concatenate([s[k:k + 1], conf[pick].cpu().numpy()], axis=0)
        got = P.logpsi(m, th_d, torch.from_numpy(seqs).cuda()).double().cpu().numpy()
        reading = OM.logpsi(th, seqs, om, bf16=True)
        exact = OM.logpsi(th, seqs, om)
        err = np.abs(got - reading).max()
        dev_r = np.abs(reading - exact).max()
        print(f"    log psi vs BF16 reading {err:.3e}; reading vs exact {dev_r:.3e}")
        assert err <= 1e-4 + 0.5 * dev_r


def test_fullsize_local_energy_fp32_sampled(P):
    B = 64      # about 1.8k connected each: three full 32768-sequence launches and a partial one
    print(f"full-size E_loc: {L}x{L} nl={NL} d={D} FP32 B={B} chunk={CHUNK}", flush=True)
    m, om, th, s = _setup(P, P.FP32, B)
    th_d = torch.from_numpy(th).cuda()
    H = P.Hamiltonian(P.HEISENBERG, L, L)
    e, st, lp = P.local_energy(m, th_d, H, torch.from_numpy(s).cuda(), chunk_seqs=CHUNK)
    e = e.cpu().numpy()
    k = SAMPLED[0]
    oh = OH.Hamiltonian("heisenberg", L, L, J=1.0)
    ref = OH.local_energy(lambda c: OM.logpsi(th, c, om), oh, s[k:k + 1])[0]
    rel = abs(e[k] - ref) / max(abs(ref), 1.0)
    print(f"  sample {k}: E_loc {e[k]:.9f} vs oracle {ref:.9f} (rel {rel:.2e})")
    assert rel <= 1e-4
    lp_ref = OM.logpsi(th, s[k:k + 1], om)[0]
    assert abs(float(lp[k]) - lp_ref) <= 1e-5 + 1e-6 * abs(lp_ref)


def test_fullsize_gradient_sampled(P):
    print(f"full-size gradient: {L}x{L} nl={NL} d={D} BF16 model B={B_FULL}", flush=True)
    m, om, th, s = _setup(P, P.BF16, B_FULL)
    th_d = torch.from_numpy(th).cuda()
    s_d = torch.from_numpy(s).cuda()
    rng = np.random.default_rng(11)
    w = torch.from_numpy(rng.standard_normal(B_FULL) / B_FULL).cuda()
    O, lpb, g = P.logpsi_backward(m, th_d, s_d, w=w, want_O=True)
    assert torch.isfinite(O).all()
    # the estimator is the FP64 weighted sum of exactly the returned rows
    g_ref = torch.zeros(O.shape[1], dtype=torch.float64, device=O.device)
    for i in range(0, B_FULL, 512):
        g_ref += w[i:i + 512] @ O[i:i + 512].double()
    gerr = (g - g_ref).abs().max().item() / max(1e-30, g_ref.abs().max().item())
    print(f"  estimator vs FP64 sum of the rows: {gerr:.2e}")
    assert gerr <= 1e-10
    k = SAMPLED[1]
    lp_ref, O_ref = OG.per_sample_grad(th, s[k:k + 1], om)
    Ok = O[k].double().cpu().numpy()
    rel = np.linalg.norm(Ok - O_ref[0]) / np.linalg.norm(O_ref[0])
    print(f"  sample {k}: rel grad err {rel:.2e}; log psi {float(lpb[k]):.6f} vs {lp_ref[0]:.6f}")
    assert rel <= 1e-4
    # the backward runs in FP32: its log psi is the FP32 model's
    assert abs(float(lpb[k]) - lp_ref[0]) <= 1e-5 + 1e-6 * abs(lp_ref[0])
