"""psr_logpsi_static (no workspace, the library's static device scratch) against
psr_logpsi: two calls in a row, the second with a smaller batch, must give the
same log psi, bit for bit (same kernels on the same inputs)."""

import numpy as np
import pytest
import torch

import psr_inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_13807_amd as P  # noqa: N813
    P.lib()
    return P


@pytest.mark.parametrize("lx,ly,nl,d,prec", [(10, 10, 2, 64, 1), (32, 32, 3, 128, 0), (52, 52, 4, 256, 2)])
def test_logpsi_static_matches_logpsi(P, lx, ly, nl, d, prec):
    m = P.Model(P.SNAKE_2D, lx, ly, nl, d, prec)
    th = torch.from_numpy(I.params(P.param_count(m), d, 1000 + d)).cuda()
    cap = P.lib().psr_static_scratch_bytes()
    per = P.workspace_bytes(m, P.OP_LOGPSI, 1)
    B1 = max(2, min(300, cap // (2 * per)))
    for B in (B1, max(1, B1 // 3)):   # the second call smaller than the first
        print(f"static logpsi {lx}x{ly} nl={nl} d={d} prec={prec} B={B}", flush=True)
        s = torch.from_numpy(I.spins_zero_mag(B, lx * ly, 7 + B)).cuda()
        assert P.workspace_bytes(m, P.OP_LOGPSI, B) <= cap
        ref, ref_site = P.logpsi(m, th, s, site_logp=True)
        got, got_site = P.logpsi_static(m, th, s, site_logp=True)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert torch.equal(got_site, ref_site)
        assert np.all(np.isfinite(got.cpu().numpy()))
