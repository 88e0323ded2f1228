"""Pins of the 1D LRU oracle (Sec. II.B Eq. (lru), Sec. II.E, Table I) against facts outside itself.

* the parameter count of the paper's 3-layer, d = d_h = 64 model (about 75,000, Table I);
* normalisation of the autoregressive distribution over all 2^N configurations;
* causality: the conditional of site t sees sigma_<t only, and does see sigma_{t-1};
* the propagator at a hand-chosen point (lambda = i/2 exactly);
* the recurrence against scipy's IIR filter and against its impulse response
  lambda^n in closed form;
* a hand-derived closed form of a 3-site, d = d_h = 1 model (every term of the
  layer enters it);
* the residual: present from the second layer on, absent on the first.
"""

import itertools
import math

import numpy as np
import pytest
import scipy.signal

import psr_inputs as I
from oracle import lru as OL


def _theta(m, seed, scale=1.0):
    return scale * I.params(OL.n_params(m), m.d, seed).astype(np.float64)


def test_param_count_of_the_table_one_model():
    m = OL.LruModel(n_sites=64, n_layers=3, d=64, dh=64)
    P = OL.n_params(m)
    assert P == 75138
    assert abs(P - 75000) / 75000 < 0.005


@pytest.mark.parametrize("nl,d,dh", [(1, 4, 8), (2, 8, 4), (3, 8, 8)])
def test_normalised_over_all_configurations(nl, d, dh):
    N = 8
    m = OL.LruModel(N, nl, d, dh)
    th = _theta(m, 11 + nl)
    allc = np.array(list(itertools.product([0, 1], repeat=N)), dtype=np.int8)
    p = np.exp(2.0 * OL.logpsi(th, allc, m))
    assert abs(p.sum() - 1.0) <= 1e-12
    assert p.max() / p.min() > 1.5      # a non-trivial distribution


def test_causal_and_uses_the_previous_spin():
    N = 10
    m = OL.LruModel(N, 2, 8, 8)
    th = _theta(m, 5, scale=2.0)
    s = I.spins_bernoulli(6, N, 77)
    base = OL.site_logp(th, s, m)
    for t in range(N - 1):
        s2 = s.copy()
        s2[:, t] ^= 1
        alt = OL.site_logp(th, s2, m)
        np.testing.assert_array_equal(alt[:, :t], base[:, :t])
        assert np.abs(alt[:, t + 1] - base[:, t + 1]).max() > 1e-6


def test_propagator_at_a_hand_chosen_point():
    # e^nu = ln 2 gives |lambda| = 1/2; e^theta = pi/2 gives a quarter turn
    lm = OL.lam(np.array([math.log(math.log(2.0))]), np.array([math.log(math.pi / 2)]))[0]
    assert abs(lm - 0.5j) <= 1e-15


def test_recurrence_is_a_first_order_iir_filter():
    N = 12
    m = OL.LruModel(N, 1, 6, 5)
    th = _theta(m, 8, scale=2.0)
    p = OL.unpack(th, m)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, N, m.d))
    _, h = OL.layer(x, p, 0, return_h=True)
    Bc = p["B0"][:m.dh] + 1j * p["B0"][m.dh:]
    drive = np.exp(p["gamma0"]) * (x @ Bc.T)
    lm = OL.lam(p["nu0"], p["theta0"])
    for u in range(m.dh):
        ref = scipy.signal.lfilter([1.0], [1.0, -lm[u]], drive[:, :, u], axis=1)
        np.testing.assert_allclose(h[:, :, u], ref, rtol=1e-12, atol=1e-14)


def test_impulse_response_in_closed_form():
    N, t0, k = 9, 2, 3
    m = OL.LruModel(N, 1, 5, 4)
    th = _theta(m, 9, scale=2.0)
    p = OL.unpack(th, m)
    x = np.zeros((1, N, m.d))
    x[0, t0, k] = 1.0
    _, h = OL.layer(x, p, 0, return_h=True)
    a, b = np.exp(p["nu0"]), np.exp(p["theta0"])
    col = np.exp(p["gamma0"]) * (p["B0"][:m.dh, k] + 1j * p["B0"][m.dh:, k])
    for t in range(N):
        n = t - t0
        want = np.zeros(m.dh, complex) if n < 0 else np.exp(-n * a) * (np.cos(n * b) + 1j * np.sin(n * b)) * col
        np.testing.assert_allclose(h[0, t], want, rtol=1e-12, atol=1e-15)


def test_hand_derived_three_site_model():
    """d = d_h = 1, one layer, three sites: every conditional written out by hand."""
    m = OL.LruModel(3, 1, 1, 1)
    names = [n for n, _ in OL.tensor_shapes(m)]
    assert names == ["E", "nu0", "theta0", "gamma0", "B0", "D0", "C0", "Wglu0", "bglu0", "W_o", "b_o"]
    rng = np.random.default_rng(21)
    th = rng.uniform(-1.2, 1.2, OL.n_params(m))
    e0, e1, nu, tht, gam, br, bi, D, cr, ci, wa, wg, ba, bg, wo0, wo1, bo0, bo1 = th
    lm = complex(math.exp(-math.exp(nu)) * math.cos(math.exp(tht)), math.exp(-math.exp(nu)) * math.sin(math.exp(tht)))
    emb = (e0, e1)

    def cond(y):
        g = (wa * y + ba) / (1.0 + math.exp(-(wg * y + bg)))
        l0, l1 = wo0 * g + bo0, wo1 * g + bo1
        z = math.log(math.exp(l0) + math.exp(l1))
        return (l0 - z, l1 - z)

    for s in itertools.product([0, 1], repeat=3):
        # site 0: zero input, zero state
        lp = cond(0.0)[s[0]]
        # site 1: h_1 = e^gamma (b x_1),  y_1 = Re(c h_1) + D x_1
        x1 = emb[s[0]]
        h1 = math.exp(gam) * complex(br, bi) * x1
        lp += cond((complex(cr, ci) * h1).real + D * x1)[s[1]]
        # site 2: h_2 = lambda h_1 + e^gamma (b x_2)
        x2 = emb[s[1]]
        h2 = lm * h1 + math.exp(gam) * complex(br, bi) * x2
        lp += cond((complex(cr, ci) * h2).real + D * x2)[s[2]]
        got = OL.logpsi(th, np.array([s], dtype=np.int8), m)[0]
        assert abs(got - 0.5 * lp) <= 1e-13


def test_residual_from_the_second_layer_only():
    N = 7
    s = I.spins_bernoulli(5, N, 31)
    # two layers, the second one's GLU zeroed: x^(2) = x^(1), so log psi is the one-layer model's
    m2, m1 = OL.LruModel(N, 2, 6, 4), OL.LruModel(N, 1, 6, 4)
    th2 = _theta(m2, 40, scale=2.0)
    p2 = OL.unpack(th2, m2)
    p2["Wglu1"][:] = 0.0
    p2["bglu1"][:] = 0.0
    th1 = np.concatenate([p2[n].ravel() for n, _ in OL.tensor_shapes(m1)])
    np.testing.assert_allclose(OL.logpsi(th2, s, m2), OL.logpsi(th1, s, m1), rtol=0, atol=1e-13)
    # one layer with its GLU zeroed: no residual, so the head sees zero and every site has softmax(b_o)
    p1 = OL.unpack(th1, m1)
    p1["Wglu0"][:] = 0.0
    p1["bglu0"][:] = 0.0
    bo = p1["b_o"]
    lse = math.log(math.exp(bo[0]) + math.exp(bo[1]))
    want = 0.5 * (bo[s.astype(int)] - lse).sum(axis=1)
    np.testing.assert_allclose(OL.logpsi(th1, s, m1), want, rtol=0, atol=1e-13)


# ---------------------------------------------------------------------------
# planted mistakes: each plausible error in the oracle's layer is rejected by a pin
# ---------------------------------------------------------------------------

def _faulty_layer(kind):
    def layer(x, p, l, return_h=False):
        dh = p[f"nu{l}"].shape[0]
        Bc = p[f"B{l}"][:dh] + 1j * p[f"B{l}"][dh:]
        Cc = p[f"C{l}"][:, :dh] + 1j * p[f"C{l}"][:, dh:]
        lm = OL.lam(p[f"nu{l}"], p[f"theta{l}"])
        v = np.exp(p[f"gamma{l}"]) * (x @ Bc.T)
        h = np.zeros(v.shape, dtype=np.complex128)
        st = np.zeros(v[:, 0].shape, dtype=np.complex128)
        for t in range(x.shape[1]):
            st = lm * st + v[:, t]
            h[:, t] = st
        y = (h @ Cc.T).real + (0.0 if kind == "no_D" else p[f"D{l}"] * x)
        d = x.shape[2]
        W, b = p[f"Wglu{l}"], p[f"bglu{l}"]
        if kind == "swapped_glu":
            g = (y @ W[d:].T + b[d:]) * OL.sigmoid(y @ W[:d].T + b[:d])
        else:
            g = (y @ W[:d].T + b[:d]) * OL.sigmoid(y @ W[d:].T + b[d:])
        res = (l >= 0) if kind == "residual_everywhere" else (l >= 1)
        xn = g + (x if res else 0.0)
        return (xn, h) if return_h else xn
    return layer


@pytest.mark.parametrize("kind", ["no_D", "swapped_glu", "residual_everywhere"])
def test_planted_layer_mistakes_are_rejected(monkeypatch, kind):
    monkeypatch.setattr(OL, "layer", _faulty_layer(kind))
    caught = 0
    for pin in (test_hand_derived_three_site_model, test_residual_from_the_second_layer_only):
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught >= 1, kind


def test_planted_conjugate_propagator_is_rejected(monkeypatch):
    orig = OL.lam
    monkeypatch.setattr(OL, "lam", lambda nu, th: np.conj(orig(nu, th)))
    with pytest.raises(AssertionError):
        test_propagator_at_a_hand_chosen_point()
    with pytest.raises(AssertionError):
        test_hand_derived_three_site_model()


def test_planted_missing_input_shift_is_rejected(monkeypatch):
    """Feeding E[:, sigma_t] instead of E[:, sigma_{t-1}] makes site t see its own spin:
    the distribution is no longer normalised."""
    orig_site_logp = OL.site_logp

    def site_logp(theta, spins, m):
        p = OL.unpack(theta, m)
        s = np.asarray(spins).astype(np.int64)
        x = p["E"].T[s]
        for l in range(m.n_layers):
            x = OL.layer(x, p, l)
        logits = x @ p["W_o"].T + p["b_o"]
        mx = logits.max(axis=2, keepdims=True)
        lse = mx[..., 0] + np.log(np.exp(logits - mx).sum(axis=2))
        return np.take_along_axis(logits, s[..., None], axis=2)[..., 0] - lse

    monkeypatch.setattr(OL, "site_logp", site_logp)
    with pytest.raises(AssertionError):
        test_normalised_over_all_configurations(2, 8, 4)
    monkeypatch.setattr(OL, "site_logp", orig_site_logp)


# ----------------------------------------------------------------------------
# The LRU's per-sample gradient (the separately written torch forward) and its
# exact sampler: pinned by finite differences of the numpy oracle, by the score
# identity over all configurations, and by the distribution of the draws.
# ----------------------------------------------------------------------------

from oracle import lru_grad as OLG  # noqa: E402


@pytest.mark.parametrize("n,nl,d,dh", [(9, 2, 8, 6), (12, 3, 16, 16)])
def test_lru_gradient_matches_finite_differences(n, nl, d, dh):
    """O rows of the autograd forward equal central differences of lru.logpsi on a
    random set of parameters (at least two per tensor), and its log psi equals the oracle's."""
    m = OL.LruModel(n, nl, d, dh)
    th = I.params(OL.n_params(m), d, 200 + n)
    s = I.spins_bernoulli(3, n, 201 + n)
    lp, O = OLG.per_sample_grad(th, s, m)
    assert np.allclose(lp, OL.logpsi(th, s, m), atol=1e-12)
    rng = I.rng(202)
    idx, off = [], 0
    for _, shp in OL.tensor_shapes(m):
        k = int(np.prod(shp))
        idx += list(rng.choice(np.arange(off, off + k), size=min(2, k), replace=False))
        off += k
    fd = np.stack([OLG.finite_difference(th, s, m, int(i)) for i in idx], axis=1)
    assert np.abs(O[:, idx] - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def test_lru_score_identity():
    """sum_sigma p(sigma) d log psi / d theta = 0 over all 2^8 configurations (the
    gradient of the normalisation; pins every component of the gradient at once)."""
    m = OL.LruModel(8, 2, 6, 4)
    th = 1.5 * I.params(OL.n_params(m), 6, 210)
    cfg = np.array(list(itertools.product([0, 1], repeat=8)), dtype=np.int8)
    lp, O = OLG.per_sample_grad(th, cfg, m)
    p = np.exp(2.0 * lp)
    assert abs(math.fsum(p) - 1.0) < 1e-12
    assert np.abs(p @ O).max() < 1e-10


def _chi2_p(samples, p):
    """Pearson chi^2 p-value of integer-coded samples against probabilities p (bins with expectation >= 5)."""
    from scipy.stats import chi2
    n = samples.shape[1]
    codes = samples.astype(np.int64) @ (1 << np.arange(n - 1, -1, -1))
    obs = np.bincount(codes, minlength=len(p)).astype(np.float64)
    exp = p * samples.shape[0]
    keep = exp >= 5
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    stat = ((o - e) ** 2 / e).sum()
    return chi2.sf(stat, len(o) - 1)


def test_lru_sampler_reproduces_brute_force_distribution():
    """Exact site-by-site draws follow p(sigma) = prod_t p(sigma_t | sigma_<t) (Pearson chi^2 over
    all 2^8 configurations); the same test rejects a planted mistake (the classes swapped)."""
    m = OL.LruModel(8, 2, 8, 6)
    th = 1.5 * I.params(OL.n_params(m), 8, 220)
    cfg = np.array(list(itertools.product([0, 1], repeat=8)), dtype=np.int8)
    p = np.exp(2.0 * OL.logpsi(th, cfg, m))
    u = I.rng(221).random((20000, 8))
    s, lp = OL.sample(th, u, m)
    assert np.allclose(lp, OL.logpsi(th, s, m), atol=1e-12)
    assert _chi2_p(s, p) > 1e-3
    wrong = np.zeros_like(s)
    for t in range(8):
        wrong[:, t] = (u[:, t] < 1.0 - OL.conditionals(th, wrong, m)[:, t]).astype(np.int8)
    assert _chi2_p(wrong, p) < 1e-6


def test_lru_sampler_decision_rule():
    m = OL.LruModel(6, 2, 8, 8)
    th = I.params(OL.n_params(m), 8, 230)
    s0, _ = OL.sample(th, np.zeros((2, 6)), m)
    s1, _ = OL.sample(th, np.ones((2, 6)), m)
    assert (s0 == 1).all() and (s1 == 0).all()
    u = I.rng(231).random((10, 6))
    s, _ = OL.sample(th, u, m)
    assert ((u < OL.conditionals(th, s, m)) == (s == 1)).all()
