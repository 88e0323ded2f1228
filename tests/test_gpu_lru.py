"""GPU parity of the 1D LRU ansatz (Sec. II.B Eq. (lru), Sec. II.E) through the C ABI.

The library's FP32 log psi and per-site log p against the float64 oracle
(``oracle/lru.py``), element by element, with the tolerances of the 2D forward
tests: |d log psi| <= 1e-5 + 1e-6 max|log psi| and 1e-4 per site.  The cases
cover every path of the kernel: short chains packed many to a group with
unchunked scans, chunked scans with a ragged last chunk, one chain per group,
one-site chains, more groups than workgroups in flight, the paper's Table I
model (3 layers, d = d_h = 64) at N = 6 and N = 256, and the full E_loc batch
of that model at N = 256 on sampled outputs.
"""

import numpy as np
import pytest
import torch

import psr_inputs as I
from oracle import lru as OL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_13807_amd as P  # noqa: N813
    P.lib()
    return P


def _case(P, n, nl, d, dh, B, seed):
    m = P.LruModel(n, nl, d, dh)
    om = OL.LruModel(n, nl, d, dh)
    assert P.lru_param_count(m) == OL.n_params(om)
    th = I.params(OL.n_params(om), d, 3000 + seed)
    s = I.spins_bernoulli(B, n, 4000 + seed)
    return m, om, th, s


def _tol(ref):
    return 1e-5 + 1e-6 * float(np.abs(ref).max())


LRU_CASES = [
    # n, nl, d, dh, B
    (16, 1, 16, 32, 33),       # 16 chains per group, one scan chunk per chain
    (16, 1, 32, 32, 33),       # the same with d = d_h: the output map must wait for every scan store
    (6, 3, 64, 64, 100),       # the Table I model at N = 6; ragged last group
    (100, 2, 32, 16, 7),       # 2 chains per group, 16 chunks of 7 sites (ragged last chunk)
    (256, 3, 64, 64, 5),       # the Table I model at N = 256: one chain per group, 8 chunks
    (257, 2, 32, 32, 3),       # one site past a group's columns
    (1, 2, 16, 16, 9),         # one-site chains: only the head's bias and the zero input
    (1000, 1, 64, 256, 2),     # long chains, 256 complex units: 2 chunks of 500
    (16, 1, 16, 32, 20000),    # 1250 groups over at most 1024 workgroups
]


@pytest.mark.parametrize("n,nl,d,dh,B", LRU_CASES)
def test_lru_logpsi_parity(P, n, nl, d, dh, B):
    print(f"LRU case n={n} nl={nl} d={d} dh={dh} B={B}", flush=True)
    m, om, th, s = _case(P, n, nl, d, dh, B, seed=n + nl + d)
    ref_site = OL.site_logp(th, s, om)
    ref = 0.5 * ref_site.sum(axis=1)
    got, site = P.lru_logpsi(m, torch.from_numpy(th).cuda(), torch.from_numpy(s).cuda(), site_logp=True)
    got = got.cpu().numpy().astype(np.float64)
    site = site.cpu().numpy().astype(np.float64)
    err, serr = np.abs(got - ref).max(), np.abs(site - ref_site).max()
    print(f"  max|dlogpsi| = {err:.3e} (tol {_tol(ref):.3e}); max site err {serr:.3e}; |log psi| ~ {np.abs(ref).max():.1f}")
    assert err <= _tol(ref)
    assert serr <= 1e-4


def test_lru_batch_position_invariance_and_empty(P):
    m, om, th, s = _case(P, 40, 2, 32, 32, 61, seed=1)
    tt, ss = torch.from_numpy(th).cuda(), torch.from_numpy(s).cuda()
    a = P.lru_logpsi(m, tt, ss)
    perm = torch.randperm(61, generator=torch.Generator().manual_seed(0)).cuda()
    c = P.lru_logpsi(m, tt, ss[perm])
    # each chain's arithmetic does not depend on its position in the batch
    assert torch.equal(c, a[perm])
    assert P.lru_logpsi(m, tt, ss[:0]).numel() == 0


def test_lru_normalised_over_all_configurations(P):
    """sum over all 2^N configurations of psi^2 = 1, from the library alone (N = 12)."""
    n = 12
    m, om, th, _ = _case(P, n, 3, 32, 32, 1, seed=2)
    idx = np.arange(2 ** n)
    allc = ((idx[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int8)
    lp = P.lru_logpsi(m, torch.from_numpy(th).cuda(), torch.from_numpy(allc).cuda()).double()
    total = torch.exp(2.0 * lp).sum().item()
    print(f"  sum psi^2 = {total:.9f}")
    assert abs(total - 1.0) <= 1e-4


def test_lru_full_eloc_batch_sampled(P):
    """The Table I model at N = 256 on the E_loc batch of 1024 samples (each with its 256
    single-flip TFIM configurations: 263,168 chains), in the launch that the benchmark
    times; sampled chains against the oracle, the rest through the flip structure."""
    n, nl, d, dh, nsamp = 256, 3, 64, 64, 1024
    m = P.LruModel(n, nl, d, dh)
    om = OL.LruModel(n, nl, d, dh)
    th = I.params(OL.n_params(om), d, 3000 + 7)
    s = torch.from_numpy(I.spins_bernoulli(nsamp, n, 4000 + 7)).cuda()
    H = P.Hamiltonian(P.TFIM, n, 1, J=1.0, h=1.0)
    c = P.connected(H, s, configs=True)
    assert int(c["n_conn"].min().item()) == n
    seqs = torch.cat([s, c["conn"].reshape(-1, n)], dim=0).contiguous()
    print(f"LRU full batch: {seqs.shape[0]} chains of {n} sites", flush=True)
    lp = P.lru_logpsi(m, torch.from_numpy(th).cuda(), seqs)
    assert bool(torch.isfinite(lp).all())
    picks = [0, nsamp - 1, nsamp, nsamp + 255, seqs.shape[0] - 1, 123457]
    sub = seqs[picks].cpu().numpy()
    ref = OL.logpsi(th, sub, om)
    got = lp[picks].double().cpu().numpy()
    err = np.abs(got - ref).max()
    print(f"  sampled chains: max|dlogpsi| = {err:.3e}")
    assert err <= _tol(ref)
    # the same chains evaluated alone, in a small launch: identical values
    alone = P.lru_logpsi(m, torch.from_numpy(th).cuda(), seqs[picks].contiguous())
    assert torch.equal(alone, lp[picks])


ELOC_CASES = [
    # kind, n, nl, d, dh, B
    ("tfim", 10, 2, 16, 16, 20),
    ("heisenberg", 9, 1, 32, 32, 15),
    ("tfim", 64, 3, 64, 64, 6),
    ("tfim", 256, 3, 64, 64, 2),      # the Table I model at N = 256: ratios of log psi ~ 180
]


@pytest.mark.parametrize("kind,n,nl,d,dh,B", ELOC_CASES)
def test_lru_local_energy_parity(P, kind, n, nl, d, dh, B):
    """E_loc against the oracle's E_loc with the LRU oracle's log psi (Sec. III.B), and the
    FP64 statistics of exactly the returned values."""
    from oracle import hamiltonian as OH
    print(f"LRU E_loc case {kind} n={n} nl={nl} d={d} dh={dh} B={B}", flush=True)
    m, om, th, s = _case(P, n, nl, d, dh, B, seed=5 * n + d)
    if kind == "tfim":
        H, oh = P.Hamiltonian(P.TFIM, n, 1, J=1.0, h=1.0), OH.Hamiltonian("tfim", n, 1, J=1.0, h=1.0)
    else:
        H, oh = P.Hamiltonian(P.HEISENBERG, n, 1, J=1.0), OH.Hamiltonian("heisenberg", n, 1, J=1.0)
    th_d = torch.from_numpy(th).cuda()
    e, st, lp = P.lru_local_energy(m, th_d, H, torch.from_numpy(s).cuda())
    e, st = e.cpu().numpy(), st.cpu().numpy()
    ref = OH.local_energy(lambda c: OL.logpsi(th, c, om), oh, s)
    rel = np.abs(e - ref).max() / max(1.0, np.abs(ref).max())
    print(f"  max rel E_loc err {rel:.3e}; mean {st[0]:.6f}")
    assert rel <= 1e-4
    assert abs(st[0] - e.mean()) <= 1e-12 * max(1.0, abs(e.mean()))
    assert abs(st[1] - e.var()) <= 1e-10 * max(1.0, e.var())
    assert torch.equal(lp, P.lru_logpsi(m, th_d, torch.from_numpy(s).cuda()))


# ----------------------------------------------------------------------------
# The LRU's exact sampler and per-sample gradients (Sec. III.B), against the
# float64 oracle (oracle/lru.py sampler, oracle/lru_grad.py autograd).
# ----------------------------------------------------------------------------

from oracle import lru_grad as OLG  # noqa: E402

LRU_SAMPLE_CASES = [
    # n, nl, d, dh, B
    (12, 2, 16, 16, 64),
    (9, 1, 32, 48, 20),       # d != d_h
    (1, 2, 16, 16, 5),        # one site
    (64, 3, 64, 64, 32),      # the Table I model
    (256, 3, 64, 64, 8),
]


@pytest.mark.parametrize("n,nl,d,dh,B", LRU_SAMPLE_CASES)
def test_lru_sampler_decisions(P, n, nl, d, dh, B):
    """Every decision of the GPU sampler against the oracle's conditional on the GPU's own
    prefix (float32 against float64: a disagreement is accepted only where u is within 2e-5
    of p), log psi of the samples to the FP32 bar, and agreement with psr_lru_logpsi."""
    print(f"LRU sampler n={n} nl={nl} d={d} dh={dh} B={B}", flush=True)
    m, om, th, _ = _case(P, n, nl, d, dh, B, seed=7 * n + dh)
    u = I.uniforms(B, n, 300 + n)
    th_d = torch.from_numpy(th).cuda()
    s, lp = P.lru_sample(m, th_d, torch.from_numpy(u).cuda())
    s = s.cpu().numpy()
    p1 = OL.conditionals(th, s, om)
    bad = ((u < p1) != (s == 1)) & (np.abs(u - p1) > 2e-5)
    assert not bad.any(), int(bad.sum())
    ref = OL.logpsi(th, s, om)
    got = lp.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 1e-5 + 1e-6 * np.abs(ref).max()
    again = P.lru_logpsi(m, th_d, torch.from_numpy(s).cuda()).cpu().numpy()
    assert np.abs(again - got).max() <= 1e-5 + 1e-6 * np.abs(ref).max()


def test_lru_sampler_distribution(P):
    """Pearson chi^2 of 40000 GPU draws against the brute-force distribution of an 8-site chain."""
    from scipy.stats import chi2
    import itertools
    m, om, th, _ = _case(P, 8, 2, 16, 16, 1, seed=88)
    th = (1.25 * th).astype(np.float32)   # mass spread over ~200 bins, far from uniform
    cfg = np.array(list(itertools.product([0, 1], repeat=8)), dtype=np.int8)
    p = np.exp(2.0 * OL.logpsi(th, cfg, om))
    u = I.uniforms(40000, 8, 89)
    s, _ = P.lru_sample(m, torch.from_numpy(th).cuda(), torch.from_numpy(u).cuda())
    codes = s.cpu().numpy().astype(np.int64) @ (1 << np.arange(7, -1, -1))
    obs = np.bincount(codes, minlength=256).astype(np.float64)
    exp = p * 40000
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    pv = chi2.sf(((o - e) ** 2 / e).sum(), len(o) - 1)
    print(f"  chi^2 p-value {pv:.3f}")
    assert pv > 1e-3


LRU_GRAD_CASES = [
    # n, nl, d, dh, B
    (10, 2, 16, 16, 6),
    (9, 1, 32, 48, 5),        # d != d_h
    (1, 2, 16, 16, 3),        # one site
    (64, 3, 64, 64, 4),       # the Table I model
    (256, 3, 64, 64, 2),
]


@pytest.mark.parametrize("n,nl,d,dh,B", LRU_GRAD_CASES)
def test_lru_per_sample_gradient(P, n, nl, d, dh, B):
    """O rows against float64 autograd (per sample ||dO|| / ||O|| <= 1e-4), log psi to the
    FP32 bar, and the FP64 estimator equal to the weighted sum of exactly the returned rows."""
    print(f"LRU gradient n={n} nl={nl} d={d} dh={dh} B={B}", flush=True)
    m, om, th, s = _case(P, n, nl, d, dh, B, seed=11 * n + d)
    lp_ref, O_ref = OLG.per_sample_grad(th, s, om)
    th_d, s_d = torch.from_numpy(th).cuda(), torch.from_numpy(s).cuda()
    w = torch.from_numpy(np.linspace(-1.0, 1.0, B)).cuda()
    O, lp, g = P.lru_backward(m, th_d, s_d, w=w)
    O64 = O.double().cpu().numpy()
    rel = np.linalg.norm(O64 - O_ref, axis=1) / np.linalg.norm(O_ref, axis=1)
    print(f"  per-sample rel grad err {rel.max():.3e}")
    assert rel.max() <= 1e-4
    assert np.abs(lp.cpu().numpy() - lp_ref).max() <= 1e-5 + 1e-6 * np.abs(lp_ref).max()
    g_ref = w.cpu().numpy() @ O64
    assert np.abs(g.cpu().numpy() - g_ref).max() <= 1e-9 * max(1.0, np.abs(g_ref).max())
    # g alone (no O rows requested)
    _, _, g2 = P.lru_backward(m, th_d, s_d, w=w, want_O=False)
    assert torch.equal(g, g2)
