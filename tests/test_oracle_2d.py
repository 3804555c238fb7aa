"""Pins of the 2-D oracle (CPU only): kernels -log(r)/(2 pi) and K_0(lambda r)
with the Fourier-space PSWF split (Sec. 4.6) and the windowed root kernel
(Sec. 4.7).

  * Bessel K_0, K_1 against scipy.special (library routines);
  * the residual tables against the quadrature that defines them, and the
    split's compact support (R_l(s_l) = 0 to the split precision);
  * the plane-wave weights against closed forms: D_l at the origin equals
    M_{l+1}(0) - M_l(0), which for the log kernel is log(2)/(2 pi) at every
    level; the k -> 0 limits of Dhat_l and That;
  * the truncated-kernel transforms That against direct Hankel quadrature;
  * physical-vs-plane-wave agreement of D_l on the colleague range and of
    W_0 on the root box (the precision the split promises);
  * end to end: O(N^2) direct sums (uniform, clustered, both kernels), closed
    forms for a charged ring probed by zero-charge points (mean-value
    property: constant inside for log, I_0 K_0 addition theorem for K_0),
    scaling and translation invariance, N = 0 and 1, coincident points.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import dmk_inputs


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def setup(oracle_mod):
    pr = oracle_mod.params2_for(1e-6)
    ps = oracle_mod.PSWF(pr.c)
    return pr, ps


KERNELS = [("log", 0, 0.0), ("yukawa10", 1, 10.0), ("yukawa03", 1, 0.3)]


def test_bessel_k(oracle_mod):
    for x in np.concatenate([np.geomspace(1e-6, 2.0, 40), np.linspace(2.0, 60.0, 40)]):
        assert abs(oracle_mod.bessel_k0(x) / special.k0(x) - 1) < 1e-13, x
        assert abs(oracle_mod.bessel_k1(x) / special.k1(x) - 1) < 1e-13, x


def test_params_2d(oracle_mod):
    pr = oracle_mod.params2_for(1e-6)
    assert (pr.nf, pr.p) == (12, 18) and abs(pr.c - 13.74) < 1e-5
    assert abs(pr.hw - 2 * math.pi / (3 + math.sqrt(2))) < 1e-15
    assert pr.nw == math.ceil(pr.c / pr.hw) == 10


@pytest.mark.parametrize("name,kern,lam", KERNELS)
def test_residual_table_matches_quadrature(oracle_mod, setup, name, kern, lam):
    pr, ps = setup
    sp = oracle_mod.Split2(ps, kern, lam, 6)
    rng = np.random.default_rng(3)
    for l in range(6):
        mu = lam * 2.0 ** -l
        for x in rng.uniform(0, 1, 6):
            a = sp.smooth(l, x)
            b = ps.smooth_quad(kern, mu, x)
            assert abs(a - b) < 1e-13 * max(1.0, abs(b)), (l, x)
        # M_l(0) is the r -> 0 limit of the smooth part (log: plus -log(s_l)/2pi)
        m0 = sp.smooth(l, 0.0) + (-math.log(2.0 ** -l) / (2 * math.pi) if kern == 0 else 0.0)
        assert abs(sp.self_[l] - m0) < 1e-12


@pytest.mark.parametrize("name,kern,lam", KERNELS)
def test_residual_compact_support(oracle_mod, setup, name, kern, lam):
    """R_l = K - M_l vanishes from r = s_l on, to the precision of the split:
    the smooth part there equals the kernel itself."""
    pr, ps = setup
    for l in (0, 3):
        s = 2.0 ** -l
        mu = lam * s
        for x in (1.0, 1.1, 1.5):
            k = oracle_mod.kernel2(kern, lam, x * s)
            m = ps.smooth_quad(kern, mu, x)
            if kern == 0:
                m = m - math.log(s) / (2 * math.pi)
            assert abs(k - m) < 1e-7, (l, x, k - m)


def test_log_weights_sum_closed_form(oracle_mod, setup):
    """D_l(0) = M_{l+1}(0) - M_l(0) = log(2)/(2 pi) for the log kernel at every level."""
    pr, ps = setup
    for l in (0, 2, 7):
        v = ps.d2_pw(pr, 0, 0.0, l, np.zeros(2))
        assert abs(v - math.log(2) / (2 * math.pi)) < 1e-7, l


def test_yukawa_weights_sum(oracle_mod, setup):
    pr, ps = setup
    lam = 10.0
    sp = oracle_mod.Split2(ps, 1, lam, 6)
    for l in (0, 3):
        v = ps.d2_pw(pr, 1, lam, l, np.zeros(2))
        assert abs(v - (sp.self_[l + 1] - sp.self_[l])) < 5e-7, l


@pytest.mark.parametrize("name,kern,lam", KERNELS)
def test_dhat_small_k_limit(setup, name, kern, lam):
    pr, ps = setup
    for l in (0, 4):
        k = 1e-4 * 2.0 ** l
        a, b = ps.d2hat(kern, lam, l, 0.0), ps.d2hat(kern, lam, l, k)
        assert abs(a - b) < 1e-6 * abs(a), l


def _that_log_quad(k, A):
    f = lambda r: -math.log(r) / (2 * math.pi) * special.j0(k * r) * 2 * math.pi * r
    return integrate.quad(f, 0, A, limit=400, epsabs=1e-13, epsrel=1e-12)[0]


def _that_yuk_quad(k, A, lam):
    f = lambda r: special.k0(lam * r) * special.j0(k * r) * 2 * math.pi * r
    return integrate.quad(f, 0, A, limit=400, epsabs=1e-13, epsrel=1e-12)[0]


@pytest.mark.parametrize("name,kern,lam", KERNELS)
def test_truncated_kernel_transform(setup, name, kern, lam):
    """That(k) (the transform of K cut at A = 1 + sqrt 2) against Hankel quadrature;
    What_0 = mollifier transform x That."""
    pr, ps = setup
    A = 1 + math.sqrt(2)
    for k in (0.0, 0.3, 1.7, 6.0, 12.5):
        kap = math.hypot(k, lam)
        mol = ps.psi(kap / ps.c) / ps.psi0
        want = (_that_log_quad(k, A) if kern == 0 else _that_yuk_quad(k, A, lam)) * mol
        got = ps.w02hat(kern, lam, k)
        assert abs(got - want) < 1e-10 * max(1.0, abs(want)), k


@pytest.mark.parametrize("name,kern,lam", KERNELS)
def test_plane_wave_split_accuracy(oracle_mod, setup, name, kern, lam):
    """The trapezoidal plane-wave sums reproduce D_l = R_l - R_{l+1} for offsets
    in the colleague range and W_0 = K - R_0 inside the root box."""
    pr, ps = setup
    sp = oracle_mod.Split2(ps, kern, lam, 8)
    rng = np.random.default_rng(5)
    scale = 1.0
    for l in (0, 2, 6):
        s = 2.0 ** -l
        for _ in range(40):
            x = rng.uniform(-2 * s, 2 * s, 2)
            r = math.hypot(*x)
            want = sp.residual(l, r) - sp.residual(l + 1, r)
            assert abs(ps.d2_pw(pr, kern, lam, l, x) - want) < 5e-7 * scale, (l, x)
    for _ in range(60):
        x = rng.uniform(-1, 1, 2)
        r = math.hypot(*x)
        want = oracle_mod.kernel2(kern, lam, r) - sp.residual(0, r)
        assert abs(ps.w02_pw(pr, kern, lam, x) - want) < 1e-6, x


def _dmk2(oracle_mod, pts, q, kern, lam, ns, tol=1e-6):
    pr = oracle_mod.params2_for(tol)
    ps = oracle_mod.PSWF(pr.c)
    tr = oracle_mod.Tree(pts, ns)
    return oracle_mod.dmk_eval(tr, pr, ps, q, kern=kern, lam=lam)["u"], tr


CASES2 = [
    ("uniform", lambda: dmk_inputs.uniform_square(3000, 41), 40),
    ("gaussian", lambda: dmk_inputs.gaussian_2d(3000, 42), 30),
]


@pytest.mark.parametrize("case", CASES2, ids=[c[0] for c in CASES2])
@pytest.mark.parametrize("name,kern,lam", KERNELS)
def test_vs_direct(oracle_mod, case, name, kern, lam):
    _, gen, ns = case
    pts, q = gen()
    u, tr = _dmk2(oracle_mod, pts, q, kern, lam, ns)
    ud = oracle_mod.direct2(kern, lam, pts, q)
    assert rel_l2(u, ud) < 2e-6


def test_direct2_brute_force(oracle_mod):
    rng = np.random.default_rng(9)
    pts = rng.random((60, 2))
    pts[7] = pts[3]  # coincident pair: no interaction
    q = rng.uniform(-1, 1, 60)
    d = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=2)
    mask = d > 0
    for kern, lam in ((0, 0.0), (1, 4.0)):
        K = np.zeros_like(d)
        K[mask] = -np.log(d[mask]) / (2 * np.pi) if kern == 0 else special.k0(lam * d[mask])
        want = K @ q
        got = oracle_mod.direct2(kern, lam, pts, q)
        assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("kern,lam", [(0, 0.0), (1, 6.0)])
def test_ring_closed_form(oracle_mod, kern, lam):
    """Unit total charge spread evenly over a circle of radius a (n points, the
    trapezoidal rule, spectrally exact off the circle) plus zero-charge probes:
    log: -log(a)/(2 pi) inside, -log(r)/(2 pi) outside;
    K_0: I_0(lam r) K_0(lam a) inside, K_0(lam r) I_0(lam a) outside."""
    a, n = 0.3, 3000
    th = 2 * np.pi * np.arange(n) / n
    ring = np.stack([a * np.cos(th), a * np.sin(th)], axis=1) + 0.5
    rng = np.random.default_rng(11)
    rin = rng.uniform(0, 0.5 * a, 40)
    rout = rng.uniform(1.5 * a, 0.45, 40)
    ph = rng.uniform(0, 2 * np.pi, 80)
    rr = np.concatenate([rin, rout])
    probes = np.stack([rr * np.cos(ph), rr * np.sin(ph)], axis=1) + 0.5
    pts = np.concatenate([ring, probes])
    q = np.concatenate([np.full(n, 1.0 / n), np.zeros(80)])
    u, _ = _dmk2(oracle_mod, pts, q, kern, lam, 40)
    if kern == 0:
        want = np.where(rr < a, -np.log(a), -np.log(rr)) / (2 * np.pi)
    else:
        want = np.where(rr < a, special.i0(lam * rr) * special.k0(lam * a),
                        special.k0(lam * rr) * special.i0(lam * a))
    # eps bounds each level's split error relative to the potential scale; the
    # ring's tree is 6-7 levels deep, so the bar is 2 eps as for adaptive 3-D trees
    assert np.max(np.abs(u[n:] - want)) < 2e-6 * np.max(np.abs(want))


@pytest.mark.parametrize("kern,lam", [(0, 0.0), (1, 3.0)])
def test_invariances(oracle_mod, kern, lam):
    pts, q = dmk_inputs.gaussian_2d(1500, 43, sigma=0.05)
    u, _ = _dmk2(oracle_mod, pts, q, kern, lam, 30)
    ut, _ = _dmk2(oracle_mod, pts + np.array([3.0, -7.0]), q, kern, lam, 30)
    assert rel_l2(ut, u) < 1e-9
    al = 4.0
    us, _ = _dmk2(oracle_mod, al * pts, q, kern, lam / al, 30)
    # log(al r) = log r + log al: u changes by -log(al)/(2 pi) times the other charges
    shift = (-math.log(al) / (2 * math.pi)) * (q.sum() - q) if kern == 0 else 0.0
    assert rel_l2(us, u + shift) < 1e-9


def test_degenerate_2d(oracle_mod):
    for kern, lam in ((0, 0.0), (1, 5.0)):
        u, _ = _dmk2(oracle_mod, np.zeros((0, 2)), np.zeros(0), kern, lam, 10)
        assert u.shape == (0,)
        u, _ = _dmk2(oracle_mod, np.array([[0.2, 0.7]]), np.array([1.5]), kern, lam, 10)
        assert abs(u[0]) < 1e-6
        # coincident points carry no interaction with each other
        pts = np.array([[0.1, 0.1], [0.1, 0.1], [0.6, 0.3]])
        q = np.array([1.0, -2.0, 0.5])
        u, _ = _dmk2(oracle_mod, pts, q, kern, lam, 10)
        ud = oracle_mod.direct2(kern, lam, pts, q)
        # the potentials nearly cancel here; the split error scales with sum |q|
        assert np.max(np.abs(u - ud)) < 1e-6 * np.abs(q).sum()
