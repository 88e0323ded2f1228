"""GPU parity of the exact autoregressive sampler (f1) through the C ABI.

Every decision of the GPU sampler is checked against the oracle's conditional
on the GPU's own prefix (teacher forcing): sigma_t = 1 iff u_t < p(sigma_t = 1 |
sigma_<t).  The kernel takes that decision on its float32 p, the oracle's p is
float64, so a disagreement is accepted only where u_t lies within the float32
error of p (|u_t - p| <= 2e-5).  log psi of each sample: the FP32 bar of
test_gpu_parity.py.  The distribution: Pearson chi^2 of 40000 GPU samples
against the brute-force p of a 3x3 model.  Both geometries (snake and chain).
"""

import numpy as np
import pytest
import torch

import psr_inputs as I
from oracle import model as OM
from oracle import sample as OS

pytestmark = pytest.mark.gpu

TIE = 2e-5


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_13807_amd as P  # noqa: N813
    P.lib()
    return P


SAMPLE_CASES = [
    # geometry (0 chain, 1 snake), lx, ly, nl, d, prec, B, theta scale
    (1, 4, 4, 3, 32, 0, 37, 1.5),      # residual active, ragged workgroup, uneven conditionals
    (1, 5, 3, 2, 64, 0, 50, 1.0),      # odd width
    (1, 1, 6, 2, 32, 1, 20, 1.5),      # one column; BF16 model descriptor (the sampler is FP32)
    (1, 7, 1, 2, 32, 0, 16, 1.5),      # one row
    (1, 10, 10, 2, 64, 0, 40, 1.0),    # the 10x10 workload shape
    (1, 6, 5, 3, 128, 0, 20, 1.5),
    (1, 3, 4, 4, 256, 0, 17, 1.0),
    (1, 32, 32, 3, 128, 1, 32, 1.0),   # the 32x32 workload shape
    (0, 16, 1, 1, 32, 0, 40, 1.5),     # the 16-site chain workload
    (0, 9, 1, 1, 64, 0, 19, 2.0),
]


@pytest.mark.parametrize("geom,lx,ly,nl,d,prec,B,scale", SAMPLE_CASES)
def test_sample_decisions_and_logpsi(P, geom, lx, ly, nl, d, prec, B, scale):
    print(f"sample case geom={geom} {lx}x{ly} nl={nl} d={d} prec={prec} B={B} scale={scale}", flush=True)
    m = P.Model(geom, lx, ly, nl, d, prec)
    om = OM.Model("chain" if geom == 0 else "snake2d", lx, ly, nl, d)
    th = (scale * I.params(OM.n_params(om), d, 300 + lx)).astype(np.float32)
    u = I.uniforms(B, lx * ly, 400 + lx)
    s, lp = P.sample(m, torch.from_numpy(th).cuda(), torch.from_numpy(u).cuda())
    s = s.cpu().numpy()
    lp = lp.cpu().numpy().astype(np.float64)
    assert set(np.unique(s)) <= {0, 1}
    p1 = OS.conditionals(th.astype(np.float64), s, om)
    want = u.astype(np.float64) < p1
    bad = want != (s == 1)
    near = np.abs(u - p1) <= TIE
    print(f"  decisions that differ from the oracle: {int(bad.sum())} (all within {TIE} of p: {bool(near[bad].all())})")
    assert near[bad].all()
    assert bad.sum() <= max(1, bad.size // 10000)
    ref = OM.logpsi(th.astype(np.float64), s, om)
    err = np.abs(lp - ref).max()
    print(f"  max |d log psi| = {err:.3e}")
    assert err <= 1e-5 + 1e-6 * np.abs(ref).max()


def test_sample_distribution_chi2(P):
    from scipy.stats import chi2

    lx, ly, nl, d, B = 3, 3, 2, 32, 40000
    m = P.Model(P.SNAKE_2D, lx, ly, nl, d, 0)
    om = OM.Model("snake2d", lx, ly, nl, d)
    th = (1.5 * I.params(OM.n_params(om), d, 77)).astype(np.float32)
    p = np.exp(2.0 * OM.logpsi(th.astype(np.float64), OM.all_configs(lx * ly), om))
    s, _ = P.sample(m, torch.from_numpy(th).cuda(), torch.from_numpy(I.uniforms(B, lx * ly, 81)).cuda())
    s = s.cpu().numpy().astype(np.int64)
    idx = (s * (1 << np.arange(lx * ly - 1, -1, -1))).sum(axis=1)
    counts = np.bincount(idx, minlength=1 << (lx * ly)).astype(np.float64)
    e = p * B
    big = e >= 5
    obs = np.append(counts[big], counts[~big].sum())
    exp_ = np.append(e[big], e[~big].sum())
    stat = float(((obs - exp_) ** 2 / exp_).sum())
    pv = float(chi2.sf(stat, obs.size - 1))
    print(f"  chi^2 {stat:.1f} on {obs.size - 1} degrees of freedom, p-value {pv:.3g}")
    assert pv > 1e-3


def test_sample_agrees_with_logpsi_and_edges(P):
    m = P.Model(P.SNAKE_2D, 6, 4, 2, 64, 0)
    th = torch.from_numpy(I.params(P.param_count(m), 64, 90)).cuda()
    u = torch.from_numpy(I.uniforms(33, 24, 91)).cuda()
    s, lp = P.sample(m, th, u)
    assert torch.allclose(lp, P.logpsi(m, th, s), atol=2e-5, rtol=0)
    # equal uniforms give equal samples
    s2, lp2 = P.sample(m, th, u)
    assert torch.equal(s, s2) and torch.equal(lp, lp2)
    # u = 0 is below every p: all ones; u = 1 is above every p: all zeros
    ones, _ = P.sample(m, th, torch.zeros_like(u))
    zeros, _ = P.sample(m, th, torch.ones_like(u))
    assert bool((ones == 1).all()) and bool((zeros == 0).all())
    # empty batch; uniforms of the wrong width
    e, le = P.sample(m, th, u[:0])
    assert e.shape == (0, 24) and le.numel() == 0
    with pytest.raises(ValueError):
        P.sample(m, th, torch.zeros(2, 23).cuda())
