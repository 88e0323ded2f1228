"""Pins of the float64 oracle to facts that do not come from the oracle itself.

Each test names what it pins and where the fact comes from: a value the paper
prints, a closed form, an exact invariant of the method, or a textbook /
library result.  They run on the CPU (no ``gpu`` marker).
"""

import math
import os

import numpy as np
import pytest
from scipy.special import expit
from scipy.stats import norm

import psr_inputs as I
from oracle import grad as G
from oracle import hamiltonian as H
from oracle import model as M

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _theta(m, seed):
    return I.params(M.n_params(m), m.d, seed)


# ----------------------------------------------------------------------------
# P1: normalisation of the autoregressive wave function, by brute force.
# sum_sigma |psi|^2 = 1 holds only if every conditional depends on earlier sites
# alone, so it pins the snake order and both predecessor maps (Sec. II.F).
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("geom,lx,ly,nl,d", [
    ("chain", 16, 1, 1, 32),      # the 16-site chain workload, all 2^16 states
    ("snake2d", 4, 4, 3, 8),      # 4x4 snake, three layers (residual active)
    ("snake2d", 3, 4, 2, 6),      # non-square, odd width
    ("snake2d", 5, 2, 3, 5),
    ("snake2d", 1, 6, 2, 4),      # a single column: only vertical predecessors
    ("snake2d", 7, 1, 2, 4),      # a single row: only horizontal predecessors
])
def test_p1_normalisation(geom, lx, ly, nl, d):
    m = M.Model(geom, lx, ly, nl, d)
    th = _theta(m, 11 + lx + 10 * ly)
    lp = M.logpsi(th, M.all_configs(m.n_sites), m)
    assert abs(math.fsum(np.exp(2.0 * lp)) - 1.0) <= 1e-12


def test_p1_causality_and_predecessors():
    """Flipping the spin at snake position t leaves log p at positions <= t
    untouched (bit for bit) and changes the conditionals of the two sites that
    have it as horizontal or vertical predecessor."""
    m = M.Model("snake2d", 4, 3, 3, 6)
    th = _theta(m, 5)
    base = I.spins_bernoulli(1, m.n_sites, 6)
    order = M.snake_order(m.lx, m.ly)
    pos = {site: k for k, site in enumerate(order)}
    lp0, _ = M.forward(th, base, m)
    for k, (i, j) in enumerate(order):
        s = base.copy()
        s[0, j * m.lx + i] ^= 1
        lp1, _ = M.forward(th, s, m)
        for k2, (i2, j2) in enumerate(order):
            a = j2 * m.lx + i2
            if k2 <= k:
                if k2 < k:
                    assert lp1[0, a] == lp0[0, a]
            for pred in (M.h_pred(i2, j2), M.v_pred(i2, j2)):
                if pred == (i, j):
                    assert pos[(i2, j2)] > k
                    assert lp1[0, a] != lp0[0, a]


# ----------------------------------------------------------------------------
# P2: score identity sum_sigma p(sigma) d log psi / d theta = 0 (normalisation
# is constant in theta).  Pins the gradient reference.
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("geom,lx,ly,nl,d", [
    ("chain", 8, 1, 1, 6),
    ("snake2d", 3, 3, 3, 5),
])
def test_p2_score_identity(geom, lx, ly, nl, d):
    m = M.Model(geom, lx, ly, nl, d)
    th = _theta(m, 21)
    cfg = M.all_configs(m.n_sites)
    lp, O = G.per_sample_grad(th, cfg, m)
    p = np.exp(2.0 * lp)
    assert abs(p.sum() - 1.0) < 1e-12
    assert np.abs(p @ O).max() <= 1e-10


# ----------------------------------------------------------------------------
# P3: the scan is a reassociation of the sequential recurrence (Sec. II.A).
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("geom,lx,ly,nl,d", [
    ("chain", 33, 1, 1, 7),
    ("snake2d", 7, 5, 3, 6),
    ("snake2d", 20, 3, 2, 4),
])
def test_p3_seq_equals_blelloch(geom, lx, ly, nl, d):
    m = M.Model(geom, lx, ly, nl, d)
    th = _theta(m, 31)
    s = I.spins_bernoulli(16, m.n_sites, 32)
    a = M.logpsi(th, s, m, "seq")
    b = M.logpsi(th, s, m, "scan")
    assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(a).max())


def test_p3_blelloch_against_cumulative_product():
    """Affine scan pinned to the unrolled sum h_t = sum_k (prod_{k<r<=t} a_r) b_k."""
    g = I.rng(3)
    a = g.uniform(0.1, 1.0, size=(2, 13, 3))
    b = g.standard_normal((2, 13, 3))
    want = np.zeros_like(b)
    for t in range(13):
        for k in range(t + 1):
            want[:, t] += np.prod(a[:, k + 1: t + 1], axis=1) * b[:, k]
    assert np.abs(M.affine_blelloch(a, b) - want).max() < 1e-13
    assert np.abs(M.affine_seq(a, b) - want).max() < 1e-13


# ----------------------------------------------------------------------------
# P4: constant gate.  With W_z = 0 the gate is z = sigma(b_z) at every site and
# the recurrence unrolls to the geometric kernel of Sec. II.E:
#   h_t = sum_{k<=t} z^(t-k) (1 - z) htilde_k.
# ----------------------------------------------------------------------------

def test_p4_constant_gate_chain():
    m = M.Model("chain", 12, 1, 1, 5)
    th = _theta(m, 41).astype(np.float64)
    P = M.unpack(th, m)
    th[:10] = 0.0                                # W_z is the first d*2 entries
    P = M.unpack(th, m)
    s = I.spins_bernoulli(4, 12, 42)
    _, hid = M.forward(th, s, m, keep_hidden=True)
    z = expit(P["bz0"])
    xprev = np.zeros((4, 12, 2))
    xprev[:, 1:] = np.eye(2)[s[:, :-1]]
    htil = xprev @ P["Wh0"].T + P["bh0"]
    want = np.zeros((4, 12, 5))
    for t in range(12):
        for k in range(t + 1):
            want[:, t] += z ** (t - k) * (1 - z) * htil[:, k]
    assert np.abs(hid[0] - want).max() < 1e-13


def test_p4_constant_gate_first_row_2d():
    """Row 0, layer 0 of the snake has no vertical input: same closed form."""
    m = M.Model("snake2d", 6, 2, 1, 4)
    th = _theta(m, 43).astype(np.float64)
    th[:16] = 0.0                                # W_z^(0) is d x 4 = 16 entries
    P = M.unpack(th, m)
    s = I.spins_bernoulli(3, 12, 44)
    _, hid = M.forward(th, s, m, keep_hidden=True)
    z = expit(P["bz0"])
    u = np.zeros((3, 6, 4))
    u[:, 1:, 0:2] = np.eye(2)[s[:, :5]]          # H-pred of (i, 0) is (i-1, 0)
    htil = u @ P["Wh0"][:, :4].T + P["bh0"]
    want = np.zeros((3, 6, 4))
    for t in range(6):
        for k in range(t + 1):
            want[:, t] += z ** (t - k) * (1 - z) * htil[:, k]
    assert np.abs(hid[0][:, :6] - want).max() < 1e-13


# ----------------------------------------------------------------------------
# P5: theta = 0.  Every logit is zero, p = 1/2 per site, log psi = -(N/2) ln 2,
# every ratio psi(sigma')/psi(sigma) is 1 and E_loc is diag + sum of elements.
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["tfim", "heisenberg"])
def test_p5_zero_parameters(kind):
    lx, ly = (10, 1) if kind == "tfim" else (4, 3)
    geom = "chain" if ly == 1 else "snake2d"
    m = M.Model(geom, lx, ly, 1 if geom == "chain" else 2, 4)
    th = np.zeros(M.n_params(m))
    s = I.spins_bernoulli(9, m.n_sites, 51)
    lp = M.logpsi(th, s, m)
    assert np.abs(lp + 0.5 * m.n_sites * math.log(2.0)).max() < 1e-13
    ham = H.Hamiltonian(kind, lx, ly, J=1.3, h=0.7)
    e = H.local_energy(lambda c: M.logpsi(th, c, m), ham, s)
    sp = 2.0 * s - 1.0
    zz = np.zeros(9)
    anti = np.zeros(9)
    for y in range(ly):
        for x in range(lx):
            a = y * lx + x
            for b in ([a + 1] if x + 1 < lx else []) + ([a + lx] if y + 1 < ly else []):
                zz += sp[:, a] * sp[:, b]
                anti += (s[:, a] != s[:, b])
    if kind == "tfim":
        want = -1.3 * zz - 0.7 * m.n_sites
    else:
        want = 1.3 / 4 * zz - 1.3 / 2 * anti
    assert np.abs(e - want).max() < 1e-12


def test_head_only_closed_form():
    """All layer weights zero: x = GELU(0) = 0, logits = b_o at every site."""
    m = M.Model("snake2d", 3, 3, 3, 4)
    th = np.zeros(M.n_params(m))
    th[-2:] = [0.3, -1.1]
    s = I.spins_bernoulli(5, 9, 52)
    lp, _ = M.forward(th, s, m)
    want = np.where(s == 1, -1.1, 0.3) - np.logaddexp(0.3, -1.1)
    assert np.abs(lp - want).max() < 1e-14


def test_gelu_is_x_times_gaussian_cdf():
    x = np.linspace(-8, 8, 401)
    assert np.abs(M.gelu(x) - x * norm.cdf(x)).max() < 1e-15 * 8


def test_one_site_closed_form():
    """1x1 lattice, one layer, d = 1: no predecessors, so h = (1 - sigma(b_z)) b_h,
    x = GELU(C h) and log p = logit[sigma] - logsumexp(logits)."""
    m = M.Model("snake2d", 1, 1, 1, 1)
    th = _theta(m, 53).astype(np.float64)
    P = M.unpack(th, m)
    h = (1 - expit(P["bz0"][0])) * P["bh0"][0]
    x = h * P["C0"][0, 0]
    x = x * norm.cdf(x)
    lg = P["Wo"][:, 0] * x + P["bo"]
    for sv in (0, 1):
        lp, _ = M.forward(th, np.array([[sv]]), m)
        assert abs(lp[0, 0] - (lg[sv] - np.logaddexp(lg[0], lg[1]))) < 1e-15


def test_residual_wiring():
    """With C^(2) = D^(2) = 0 the third layer's output is GELU(h^(1)) (Sec. II.G:
    s^(l) = h^(l-1) for l >= 2), so the head sees GELU of the layer-1 state."""
    m = M.Model("snake2d", 3, 2, 3, 4)
    th = _theta(m, 54).astype(np.float64)
    P = M.unpack(th, m)
    P["C2"][:] = 0.0
    P["D2"][:] = 0.0
    flat = np.concatenate([P[n].reshape(-1) for n, _ in M.tensor_shapes(m)])
    s = I.spins_bernoulli(4, 6, 55)
    lp, hid = M.forward(flat, s, m, keep_hidden=True)
    x = hid[1] * norm.cdf(hid[1])
    lg = x @ P["Wo"].T + P["bo"]
    want = np.take_along_axis(lg, s[..., None].astype(np.int64), 2)[..., 0] - np.logaddexp(lg[..., 0], lg[..., 1])
    assert np.abs(lp - want).max() < 1e-13


# ----------------------------------------------------------------------------
# P6: E_loc from the enumeration equals (H psi)(sigma) / psi(sigma) with H built
# independently from Pauli Kronecker products; <H> >= E_0 (variational bound).
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind,geom,lx,ly,marshall", [
    ("tfim", "chain", 10, 1, True),
    ("heisenberg", "snake2d", 3, 3, True),
    ("heisenberg", "snake2d", 3, 3, False),
    ("heisenberg", "snake2d", 4, 3, True),
    ("tfim", "snake2d", 2, 5, True),
])
def test_p6_eloc_matches_dense_hamiltonian(kind, geom, lx, ly, marshall):
    m = M.Model(geom, lx, ly, 1 if geom == "chain" else 2, 5)
    th = _theta(m, 61)
    ham = H.Hamiltonian(kind, lx, ly, J=1.0, h=0.9, marshall=marshall)
    cfg = M.all_configs(m.n_sites)
    lp = M.logpsi(th, cfg, m)
    e_enum = H.local_energy(lambda c: M.logpsi(th, c, m), ham, cfg)
    e_dense = H.local_energy_dense(lp, ham)
    scale = max(1.0, np.abs(e_dense).max())
    assert np.abs(e_enum - e_dense).max() <= 1e-10 * scale
    energy = math.fsum(np.exp(2 * lp) * e_enum)
    assert energy >= H.ground_energy(ham) - 1e-10


# ----------------------------------------------------------------------------
# P7: Hamiltonian conventions pinned by exact spectra.
# ----------------------------------------------------------------------------

def _golden_tfim():
    rows = []
    with open(os.path.join(GOLDEN, "tfim_obc_exact.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, e = line.split()
                rows.append((n, float(e)))
    return rows


def test_p7_tfim_exact_formula_reproduces_table_one():
    for n, e in _golden_tfim():
        if n == "inf":
            assert abs(-4.0 / math.pi - e) < 5e-8
        else:
            assert abs(H.tfim_obc_exact_energy_per_site(int(n)) - e) < 5e-8


@pytest.mark.parametrize("n", [6, 8, 10, 12])
def test_p7_tfim_exact_diagonalisation(n):
    """Ground energy of the Pauli-built TFIM chain equals N e_exact(N) (Table I)."""
    e0 = H.ground_energy(H.Hamiltonian("tfim", n, 1, J=1.0, h=1.0))
    want = dict(_golden_tfim())[str(n)]
    assert abs(e0 / n - want) < 5e-8


def test_p7_heisenberg_textbook_spectra():
    # two spins 1/2: singlet at -3J/4
    assert abs(H.ground_energy(H.Hamiltonian("heisenberg", 2, 1)) + 0.75) < 1e-12
    # 2x2 open plaquette = 4-site ring: E0 = -2J
    assert abs(H.ground_energy(H.Hamiltonian("heisenberg", 2, 2)) + 2.0) < 1e-12
    # Marshall rotation is a similarity transform: same spectrum, and the
    # rotated matrix is sign-free (off-diagonal elements <= 0)
    for lx, ly in ((2, 2), (3, 2), (3, 3)):
        a = H.sparse_hamiltonian(H.Hamiltonian("heisenberg", lx, ly, marshall=True)).toarray()
        b = H.sparse_hamiltonian(H.Hamiltonian("heisenberg", lx, ly, marshall=False)).toarray()
        assert np.abs(np.linalg.eigvalsh(a) - np.linalg.eigvalsh(b)).max() < 1e-10
        off = a - np.diag(np.diag(a))
        assert off.max() <= 0.0 and off.min() < 0.0
        assert (b - np.diag(np.diag(b))).max() > 0.0


# ----------------------------------------------------------------------------
# P8: the enumeration reproduces H's sparsity pattern and elements exactly.
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind,lx,ly", [("heisenberg", 3, 3), ("heisenberg", 4, 2), ("tfim", 9, 1)])
def test_p8_enumeration_matches_nonzero_pattern(kind, lx, ly):
    ham = H.Hamiltonian(kind, lx, ly, J=1.0, h=0.8)
    n = ham.n_sites
    Hs = H.sparse_hamiltonian(ham).tocsr()
    cfg = H.all_bits(n)
    conn = H.connected(ham, cfg)
    flips = H.apply_flips(cfg, conn)
    weights = 1 << np.arange(n - 1, -1, -1)
    idx_to = flips.astype(np.int64) @ weights
    off = 0
    for k in range(cfg.shape[0]):
        row = Hs.getrow(k)
        got = {}
        for q in range(off, off + conn["n_conn"][k]):
            got[int(idx_to[q])] = conn["mel"][q]
        off += conn["n_conn"][k]
        want = {int(c): v for c, v in zip(row.indices, row.data) if c != k and v != 0}
        assert got == want
        assert conn["diag"][k] == row[0, k]
    if kind == "heisenberg":
        anti = sum((cfg[:, a] != cfg[:, b]) for a, b in H.bonds(lx, ly))
        assert np.array_equal(conn["n_conn"], anti)


# ----------------------------------------------------------------------------
# P9: per-sample gradients (torch float64 autograd, separately written forward)
# against central finite differences of the numpy oracle.
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("geom,lx,ly,nl,d", [("snake2d", 4, 3, 3, 6), ("chain", 9, 1, 1, 5)])
def test_p9_gradient_finite_differences(geom, lx, ly, nl, d):
    m = M.Model(geom, lx, ly, nl, d)
    th = _theta(m, 71)
    s = I.spins_bernoulli(8, m.n_sites, 72)
    lp_t, O = G.per_sample_grad(th, s, m)
    assert np.abs(lp_t - M.logpsi(th, s, m)).max() < 1e-12
    g = I.rng(73)
    idx = []
    off = 0
    for _, shp in M.tensor_shapes(m):           # at least two entries per tensor
        k = int(np.prod(shp))
        idx += list(off + g.choice(k, size=min(2, k), replace=False))
        off += k
    extra = min(64 - len(idx), M.n_params(m)) if len(idx) < 64 else 0
    idx = sorted(set(idx) | set(int(v) for v in g.choice(M.n_params(m), size=extra, replace=False)))
    for p in idx:
        fd = G.finite_difference(th, s, m, int(p))
        assert np.abs(fd - O[:, p]).max() <= 1e-7 * max(1.0, np.abs(O[:, p]).max())


def test_gradient_estimator_against_finite_difference_of_energy():
    """g = (2/B) sum (E_loc - mean) O_s is the derivative of the exact energy
    <psi|H|psi> when the batch is the whole basis weighted by p (Sec. III.B)."""
    m = M.Model("snake2d", 3, 2, 2, 4)
    ham = H.Hamiltonian("heisenberg", 3, 2)
    th = _theta(m, 74).astype(np.float64)
    cfg = M.all_configs(6)
    Hs = H.sparse_hamiltonian(ham)

    def energy(t):
        psi = np.exp(M.logpsi(t, cfg, m))
        return psi @ (Hs @ psi)

    lp, O = G.per_sample_grad(th, cfg, m)
    p = np.exp(2 * lp)
    e = H.local_energy(lambda c: M.logpsi(th, c, m), ham, cfg)
    mean = p @ e
    exact_grad = 2 * (p * (e - mean)) @ O
    for k in (0, 7, 40, M.n_params(m) - 1):
        t1, t2 = th.copy(), th.copy()
        t1[k] += 1e-5
        t2[k] -= 1e-5
        assert abs((energy(t1) - energy(t2)) / 2e-5 - exact_grad[k]) < 1e-8
    # the uniform-batch estimator reduces to the same formula with weights 1/B
    mean_u, var_u = G.energy_stats(e)
    assert abs(mean_u - e.mean()) < 1e-13 and abs(var_u - e.var()) < 1e-12
    gu = G.gradient_estimate(e, O)
    assert np.abs(gu - 2 * ((e - e.mean()) @ O) / e.size).max() < 1e-12


# ----------------------------------------------------------------------------
# P10: tensor shapes reproduce the parameter counts the paper states for its
# 2x2-patch models (16-state alphabet: u^(0) has 2 x 16 entries, 16-way head).
# ----------------------------------------------------------------------------

def test_p10_parameter_counts_match_paper():
    with open(os.path.join(GOLDEN, "param_counts.txt")) as f:
        rows = [list(map(int, l.split())) for l in f if l.strip() and not l.startswith("#")]
    for nl, d, stated in rows:
        shapes = M.snake_tensor_shapes(nl, d, du0=32, n_out=16)
        count = sum(int(np.prod(s)) for _, s in shapes)
        assert abs(count - stated) / stated < 0.025, (nl, d, count)
    # the single-site models used here
    assert M.n_params(M.Model("chain", 16, 1, 1, 32)) == 258
    assert M.n_params(M.Model("snake2d", 10, 10, 2, 64)) == 29826
    assert M.n_params(M.Model("snake2d", 32, 32, 3, 128)) == 199170
    assert M.n_params(M.Model("snake2d", 52, 52, 4, 256)) == 1119746


# ----------------------------------------------------------------------------
# f1: exact autoregressive sampling (Sec. III.B) against the brute-force distribution
# ----------------------------------------------------------------------------

def _chi2_pvalue(samples: np.ndarray, p: np.ndarray) -> float:
    """Pearson chi^2 of sampled configuration counts against p (bins with expected < 5 merged)."""
    from scipy.stats import chi2

    n = samples.shape[1]
    idx = (samples.astype(np.int64) * (1 << np.arange(n - 1, -1, -1))).sum(axis=1)   # all_configs order
    counts = np.bincount(idx, minlength=1 << n).astype(np.float64)
    expected = p * samples.shape[0]
    big = expected >= 5
    obs = np.append(counts[big], counts[~big].sum())
    exp_ = np.append(expected[big], expected[~big].sum())
    keep = exp_ > 0
    stat = float(((obs[keep] - exp_[keep]) ** 2 / exp_[keep]).sum())
    return float(chi2.sf(stat, keep.sum() - 1))


@pytest.mark.parametrize("geom,lx,ly,nl,d", [("snake2d", 3, 3, 2, 32), ("snake2d", 4, 2, 3, 32), ("chain", 8, 1, 1, 32)])
def test_f1_sampler_reproduces_brute_force_distribution(geom, lx, ly, nl, d):
    from oracle import sample as S

    m = M.Model(geom, lx, ly, nl, d)
    th = 1.5 * I.params(M.n_params(m), d, 77)          # far from uniform, mass spread over many bins
    N = lx * ly
    p = np.exp(2.0 * M.logpsi(th, M.all_configs(N), m))
    assert abs(math.fsum(p) - 1.0) < 1e-12
    u = I.rng(78).random((20000, N))
    s, lp = S.sample(th, u, m)
    assert np.allclose(lp, M.logpsi(th, s, m), atol=1e-12)
    pv = _chi2_pvalue(s, p)
    assert pv > 1e-3, pv
    # planted mistake: the two classes swapped (sigma_t = 1 iff u < 1 - p) must be rejected
    wrong = np.zeros_like(s)
    for t in S.visiting_order(m):
        wrong[:, t] = (u[:, t] < 1.0 - S.conditionals(th, wrong, m)[:, t]).astype(np.int8)
    assert _chi2_pvalue(wrong, p) < 1e-6


def test_f1_sampler_decision_rule():
    from oracle import sample as S

    m = M.Model("snake2d", 3, 2, 2, 32)
    th = I.params(M.n_params(m), 32, 79)
    s0, _ = S.sample(th, np.zeros((2, 6)), m)               # u = 0 < p: every spin 1
    s1, _ = S.sample(th, np.ones((2, 6)), m)                # u = 1 >= p: every spin 0
    assert (s0 == 1).all() and (s1 == 0).all()
    # the conditionals of a sample are those its decisions were taken on
    u = I.rng(80).random((16, 6))
    s, _ = S.sample(th, u, m)
    p1 = S.conditionals(th, s, m)
    assert ((u < p1) == (s == 1)).all()


# ----------------------------------------------------------------------------
# f2: 2x2 patch inputs (Sec. II.F) and the c4v symmetrisation of the 2D runs
# (Sec. III.C, Tables II and VI).  The patch encoding and the c4v formula are
# readings (the paper gives neither); these pins fix what any such reading must
# satisfy: a bijective local alphabet, causality on the patch grid,
# normalisation, the group structure, invariance, and E_loc = (H psi)/psi.
# ----------------------------------------------------------------------------

from oracle import symmetry as S  # noqa: E402


def test_patch_states_are_a_bijection_of_the_four_spins():
    """The 16 configurations of a 2x2 lattice map to the 16 states, one each; a
    single up spin at (a, b) of the patch is state 2^(a + 2b)."""
    m = M.Model("snake2d", 2, 2, 1, 4, patch=2)
    cfg = M.all_configs(4)
    st = M.patch_states(cfg, m)[:, 0]
    assert sorted(st.tolist()) == list(range(16))
    for a in range(2):
        for b in range(2):
            one = np.zeros((1, 4), dtype=np.int8)
            one[0, b * 2 + a] = 1
            assert M.patch_states(one, m)[0, 0] == 2 ** (a + 2 * b)
    # patches tile the lattice: patch (I, J) reads only its own four spins
    m2 = M.Model("snake2d", 6, 4, 1, 4, patch=2)
    sp = np.zeros((1, 24), dtype=np.int8)
    sp[0, 3 * 6 + 5] = 1                       # spin (5, 3): patch (2, 1), a = b = 1
    st = M.patch_states(sp, m2)[0]
    assert st.tolist() == [0, 0, 0, 0, 0, 8]


@pytest.mark.parametrize("lx,ly,nl,d", [(4, 4, 3, 8), (4, 2, 2, 6), (2, 6, 3, 5), (6, 2, 2, 4)])
def test_patch_normalisation(lx, ly, nl, d):
    """sum over all 2^N configurations of |psi|^2 = 1 with 16-way conditionals on
    the patch grid (three layers: the residual is active)."""
    m = M.Model("snake2d", lx, ly, nl, d, patch=2)
    th = _theta(m, 300 + lx + ly)
    lp = M.logpsi(th.astype(np.float64) * 1.5, M.all_configs(lx * ly), m)
    assert abs(math.fsum(np.exp(2.0 * lp)) - 1.0) <= 1e-12


def test_patch_causality():
    """Changing a spin of patch t changes log p only at patches t, t+1, ... in the
    zigzag order of the patch grid."""
    m = M.Model("snake2d", 6, 4, 2, 8, patch=2)
    th = _theta(m, 77)
    base = I.spins_bernoulli(1, 24, 78)
    lp0, _ = M.forward(th, base, m)
    order = [j * m.px + i for (i, j) in M.snake_order(m.px, m.py)]
    rank = {p: r for r, p in enumerate(order)}
    for site in range(24):
        x, y = site % 6, site // 6
        patch = (y // 2) * m.px + x // 2
        s = base.copy()
        s[0, site] ^= 1
        lp, _ = M.forward(th, s, m)
        changed = np.nonzero(np.abs(lp[0] - lp0[0]) > 0)[0]
        assert all(rank[p] >= rank[patch] for p in changed)
        assert patch in changed    # the patch's own conditional sees its own state


def test_patch_head_only_and_zero_parameters():
    """With every parameter zero but the head bias, each patch is drawn from
    softmax(b_o) independently; with all zero, log psi = -(N/2) ln 2."""
    m = M.Model("snake2d", 4, 6, 2, 8, patch=2)
    P = M.n_params(m)
    th = np.zeros(P)
    s = I.spins_bernoulli(5, 24, 9)
    assert np.allclose(M.logpsi(th, s, m), -12.0 * math.log(2.0), atol=1e-12)
    bo = I.rng(10).standard_normal(16)
    th[P - 16:] = bo
    logsm = bo - np.log(np.exp(bo).sum())
    want = 0.5 * logsm[M.patch_states(s, m)].sum(axis=1)
    assert np.allclose(M.logpsi(th, s, m), want, atol=1e-12)


def test_patch_parameter_counts():
    """n_params of the patch model equals the tensor-shape count that the paper's
    figures are checked against (about 800,000 and about 7.1 million)."""
    for nl, d, want in ((3, 256, 816656), (6, 512, 7141392)):
        m = M.Model("snake2d", 52, 52, nl, d, patch=2)
        assert M.n_params(m) == want
        shapes = M.snake_tensor_shapes(nl, d, du0=32, n_out=16)
        assert sum(int(np.prod(s)) for _, s in shapes) == want


def test_c4v_is_the_symmetry_group_of_the_square():
    """Eight distinct site permutations, closed under composition, with inverses;
    they preserve the nearest-neighbour bonds of the open lattice."""
    for L in (2, 3, 4, 5):
        perms = S.c4v_perms(L)
        keys = {tuple(p) for p in perms}
        assert len(keys) == 8
        for p in perms:
            assert sorted(p.tolist()) == list(range(L * L))
            for q in perms:
                assert tuple(p[q]) in keys          # closure
            assert tuple(np.argsort(p)) in keys      # inverse
        bonds = {frozenset(b) for b in H.bonds(L, L)}
        for p in perms:
            assert {frozenset((p[a], p[b])) for a, b in H.bonds(L, L)} == bonds


@pytest.mark.parametrize("patch", [1, 2])
def test_c4v_invariance_and_normalisation(patch):
    """psi_c4v(sigma o T_k) = psi_c4v(sigma) for every configuration and k, and
    the symmetrised wave function stays normalised (4x4, all 2^16 states)."""
    m = M.Model("snake2d", 4, 4, 2, 8, patch=patch)
    th = _theta(m, 400 + patch) * 1.5
    cfg = M.all_configs(16)
    fn = lambda c: M.logpsi(th, c, m)   # noqa: E731
    lp = S.logpsi_c4v(fn, cfg, 4)
    assert abs(math.fsum(np.exp(2.0 * lp)) - 1.0) <= 1e-12
    for t in S.transformed(cfg[::97], 4):
        assert np.allclose(S.logpsi_c4v(fn, t, 4), lp[::97], atol=1e-12)
    # the unsymmetrised model is not invariant (so the test above is not vacuous)
    assert np.abs(fn(S.transformed(cfg[::97], 4)[1]) - fn(cfg[::97])).max() > 1e-3


@pytest.mark.parametrize("patch", [1, 2])
def test_c4v_local_energy_matches_sparse_hamiltonian(patch):
    """E_loc of the symmetrised wave function from the connected configurations
    equals (H psi_c4v)(sigma) / psi_c4v(sigma) with H built from Pauli matrices
    (4x4 open Heisenberg, Marshall basis), and its |psi|^2 average is >= E_0."""
    m = M.Model("snake2d", 4, 4, 2, 8, patch=patch)
    th = _theta(m, 500 + patch)
    ham = H.Hamiltonian("heisenberg", 4, 4)
    fn = lambda c: S.logpsi_c4v(lambda t: M.logpsi(th, t, m), c, 4)   # noqa: E731
    cfg = H.all_bits(16)
    lp_all = fn(cfg)
    e_dense = H.local_energy_dense(lp_all, ham)
    pick = I.rng(11).choice(len(cfg), size=40, replace=False)
    e_conn = H.local_energy(fn, ham, cfg[pick])
    assert np.allclose(e_conn, e_dense[pick], rtol=1e-10, atol=1e-10)
    p = np.exp(2.0 * lp_all)
    assert float(p @ e_dense) >= H.ground_energy(ham) - 1e-9
