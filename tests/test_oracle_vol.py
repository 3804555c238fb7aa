"""Pins of the volume-potential oracle (continuous sources, Gaussian split).

Each check compares the oracle with something it does not compute itself:
closed-form potentials (uniform cube, box-restricted Gaussian), scipy's
erf/erfc and radial quadrature of the split kernels, and structural
invariants of the level-restricted tree.  Sizes are small so the CPU suite
stays fast.
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf, erfc

import oracle as O
from vol_exact import cube_potential, gauss_box_potential

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

TOL = 1e-3


@pytest.fixture(scope="module")
def vp():
    return O.vparams_for(TOL, 8)


@pytest.fixture(scope="module")
def gs(vp):
    return O.GSplit(vp)


# ------------------------------------------------------------------ pins of the pins
def test_cube_closed_form_against_quadrature():
    x = np.array([[0.1, -0.2, 0.3], [0.9, 0.1, 0.0]])
    for k in range(2):
        f = lambda z, y, w: 1.0 / np.sqrt((x[k, 0] - w) ** 2 + (x[k, 1] - y) ** 2 + (x[k, 2] - z) ** 2)
        if k == 1:
            ref, _ = integrate.tplquad(f, -0.5, 0.5, -0.5, 0.5, -0.5, 0.5, epsabs=1e-10, epsrel=1e-10)
            assert cube_potential(x[k:k + 1])[0] == pytest.approx(ref / (4 * np.pi), rel=1e-8)
    # centre value of the unit cube: 2.3800772... / (4 pi) (classical constant)
    assert cube_potential(np.zeros((1, 3)))[0] * 4 * np.pi == pytest.approx(2.380077363, rel=1e-8)


def test_gauss_box_formula_against_full_space():
    c = np.array([0.02, -0.01, 0.03])
    sig = 0.03
    x = np.array([[0.1, 0.1, 0.0], [0.02, -0.01, 0.04]])
    r = np.linalg.norm(x - c, axis=1)
    full = (np.pi * sig ** 2) ** 1.5 * erf(r / sig) / (4 * np.pi * r)
    assert np.allclose(gauss_box_potential(x, c, sig), full, rtol=1e-10)


# --------------------------------------------------------------------- split
def test_params(vp):
    assert vp.sigma0 == pytest.approx(1 / np.sqrt(np.log(1e3)))
    assert (vp.p, vp.nf, vp.q) == (18, 12, 8)
    with pytest.raises(ValueError):
        O.vparams_for(1e-4, 8)


def test_split_kernels_against_erf(gs, vp):
    # D_l and R_L against scipy, and the telescoping sum M_0 + D_0 + D_1 + R_2 = 1/r
    for r in [1e-3, 0.05, 0.3, 0.9]:
        s = [vp.sigma0 / 2 ** l for l in range(3)]
        assert gs.d(1, r) == pytest.approx((erf(r / s[2]) - erf(r / s[1])) / r, rel=1e-12, abs=1e-14)
        assert gs.r(2, r) == pytest.approx(erfc(r / s[2]) / r, rel=1e-12)
        tot = gs.m(0, r) + gs.d(0, r) + gs.d(1, r) + gs.r(2, r)
        assert tot == pytest.approx(1 / r, rel=1e-13)


def test_dhat_is_the_radial_fourier_transform(gs, vp):
    # 3-D radial transform F(k) = (4 pi / k) int_0^inf D(r) r sin(kr) dr
    for l in (0, 2):
        for k in (0.5, 7.0, 30.0 * 2 ** l):
            ref, _ = integrate.quad(lambda r: gs.d(l, r) * r * np.sin(k * r), 0, 8.0 / 2 ** l, limit=400,
                                    epsabs=1e-14)
            assert gs.dhat(l, k) == pytest.approx(4 * np.pi / k * ref, rel=1e-7, abs=1e-12)
    # k -> 0: pi (sigma_l^2 - sigma_{l+1}^2)
    s0 = vp.sigma0
    assert gs.dhat(0, 0.0) == pytest.approx(np.pi * (s0 ** 2 - (s0 / 2) ** 2), rel=1e-14)
    assert gs.dhat(0, 1e-6) == pytest.approx(gs.dhat(0, 0.0), rel=1e-9)


def test_w0hat_is_truncated_kernel_times_gaussian(gs, vp):
    A = np.sqrt(3) + 1
    for k in (0.3, 4.0, 11.0):
        trunc, _ = integrate.quad(lambda r: np.sin(k * r), 0, A, limit=200)  # (4 pi/k) int_0^A (1/r) r sin(kr)
        assert gs.w0hat(k) == pytest.approx(4 * np.pi / k * trunc * np.exp(-k * k * vp.sigma0 ** 2 / 4), rel=1e-10)


def test_plane_wave_sums_reproduce_the_kernels(gs, vp):
    rng = np.random.default_rng(3)
    d0 = gs.d(0, 0.0)
    worst = 0.0
    for _ in range(12):
        x = rng.uniform(-2, 2, 3)   # colleague range: |x_i| <= 2 s_l
        worst = max(worst, abs(gs.d_pw(0, x) - gs.d(0, np.linalg.norm(x))))
    assert worst < 3e-4 * d0
    # level 2 at the same relative offsets: the weights scale as 2^l
    x = np.array([0.3, -0.2, 0.1])
    assert gs.d_pw(2, x / 4) == pytest.approx(4 * gs.d_pw(0, x), rel=1e-10)
    m0 = gs.m(0, 0.0)
    for _ in range(12):
        x = rng.uniform(-1, 1, 3)
        if np.linalg.norm(x) > np.sqrt(3):
            continue
        assert abs(gs.w0_pw(x) - gs.m(0, np.linalg.norm(x))) < 1e-5 * m0


def test_sum_of_gaussians_reproduces_erfc(gs, vp):
    sq = np.sqrt(np.log(1 / TOL))
    for lo, hi in [(sq, vp.tau_a), (2 * sq, vp.tau_a / 2 * 2 ** 3)]:
        t, w = gs.sog(lo, hi)
        assert len(t) % vp.tpan_gl == 0 and np.all(w > 0)
        r = np.geomspace(1e-4, 3.0, 300)
        approx = (np.exp(-np.outer(r ** 2, t ** 2)) @ w) + erfc(hi * r) / r
        exact = erfc(lo * r) / r
        # 5 nodes per unit panel in log t: 3e-6 of 1/r, far below tol = 1e-3
        assert np.max(np.abs(approx - exact) * r) < 1e-5


# ---------------------------------------------------------------------- tree
def _gauss(c, sig):
    c = np.asarray(c)
    return lambda x: np.exp(-np.sum((x - c) ** 2, axis=1) / sig ** 2)


def test_tree_invariants(vp):
    f = _gauss([0.1, -0.2, 0.05], 0.04)
    T = O.VTree(vp, f, 1.0, 0, 9)
    lev, ijk = T.level, T.ijk
    # leaves tile the cube
    assert np.sum(8.0 ** -lev.astype(float)) == pytest.approx(1.0, abs=1e-15)
    # Morton order: keys strictly increasing
    def key(l, c):
        k = 0
        for b in range(21):
            for d in range(3):
                k |= ((int(c[d]) << (21 - l)) >> b & 1) << (3 * b + 2 - d)
        return k
    keys = [key(int(l), c) for l, c in zip(lev, ijk)]
    assert all(a < b for a, b in zip(keys, keys[1:]))
    # 2:1 balance over face, edge and corner contacts
    lo = ijk * (2.0 ** -lev[:, None])
    hi = lo + 2.0 ** -lev[:, None]
    for i in range(T.nleaf):
        touch = np.all((lo <= hi[i] + 1e-15) & (hi >= lo[i] - 1e-15), axis=1)
        assert np.max(np.abs(lev[touch] - lev[i])) <= 1
    # resolution: every leaf below the maximum level is resolved (tail <= tol)
    q = vp.q
    xyz = T.nodes().reshape(T.nleaf, q, q, q, 3)
    th = np.pi * (np.arange(q) + 0.5) / q
    Cm = np.cos(np.outer(np.arange(q), th)) * np.where(np.arange(q) == 0, 1.0, 2.0)[:, None] / q
    for b in range(T.nleaf):
        fv = f(xyz[b].reshape(-1, 3)).reshape(q, q, q)
        c = np.einsum("ia,jb,kc,abc->ijk", Cm, Cm, Cm, fv)
        mask = np.zeros((q, q, q), bool)
        mask[q - 2:, :, :] = mask[:, q - 2:, :] = mask[:, :, q - 2:] = True
        if lev[b] < 9:
            # below the maximum level every leaf is resolved (the children of
            # resolved boxes that the balance rule splits are resolved too)
            assert np.sum(np.abs(c[mask])) <= TOL
    # the parent of the deepest leaves was not resolved
    deep = np.argmax(lev)
    pl, pc = lev[deep] - 1, ijk[deep] // 2
    s = 2.0 ** -pl
    cen = -0.5 + (pc + 0.5) * s
    xn = np.cos(th)
    P = np.stack(np.meshgrid(cen[0] + s / 2 * xn, cen[1] + s / 2 * xn, cen[2] + s / 2 * xn, indexing="ij"), -1)
    c = np.einsum("ia,jb,kc,abc->ijk", Cm, Cm, Cm, f(P.reshape(-1, 3)).reshape(q, q, q))
    mask = np.zeros((q, q, q), bool)
    mask[q - 2:, :, :] = mask[:, q - 2:, :] = mask[:, :, q - 2:] = True
    assert np.sum(np.abs(c[mask])) > TOL


def test_tree_levels_and_nodes(vp):
    T = O.VTree(vp, lambda x: np.ones(len(x)), 1.0, 2, 2)
    assert T.nleaf == 64 and np.all(T.level == 2)
    xyz = T.nodes()
    q = vp.q
    th = np.pi * (np.arange(q) + 0.5) / q
    c0 = -0.5 + (T.ijk[0] + 0.5) * 0.25
    assert np.allclose(xyz[:q ** 3].reshape(q, q, q, 3)[:, 0, 0, 0], c0[0] + 0.125 * np.cos(th))
    assert np.allclose(xyz[:q ** 3].reshape(q, q, q, 3)[0, 0, :, 2], c0[2] + 0.125 * np.cos(th))
    # a constant density is resolved on the root
    T0 = O.VTree(vp, lambda x: np.full(len(x), 3.0), 1.0, 0, 8)
    assert T0.nleaf == 1


# --------------------------------------------------------------- volume potential
@pytest.mark.parametrize("level", [0, 1, 2])
def test_uniform_cube(vp, level):
    """Unit density on uniform trees (level 0: the root is the only leaf, far
    field W_0 alone) against the closed form.  Nodes at least 2.5/t_a from
    the boundary of B_0 to 1e-4 of max u.  Nearer the boundary the asymptotic
    part extends the leaf polynomial beyond B_0 (the expansion integrates over
    R^3): there the error stays below that part's size."""
    T = O.VTree(vp, lambda x: np.ones(len(x)), 1e9, level, level)
    assert T.nleaf == 8 ** level
    xyz = T.nodes()
    r = T.eval(np.ones(len(xyz)))
    ex = cube_potential(xyz)
    err = np.abs(r["u"] - ex)
    ta = vp.tau_a * 2 ** level
    inner = (0.5 - np.max(np.abs(xyz), axis=1)) >= 2.5 / ta
    assert inner.sum() >= 8 ** level
    assert np.max(err[inner]) < 1e-4 * np.max(ex)
    assert np.all(err < r["utail"] + 1e-4 * np.max(ex))
    # a dropped asymptotic part shows at the interior nodes
    assert np.max(np.abs(r["u"] - r["utail"] - ex)[inner]) > 1e-3 * np.max(ex)


def test_gaussian_density(vp):
    c, sig = np.array([0.05, -0.03, 0.02]), 0.08
    f = _gauss(c, sig)
    T = O.VTree(vp, f, 1.0, 0, 8)
    xyz = T.nodes()
    r = T.eval(f(xyz))
    idx = np.random.default_rng(0).choice(len(xyz), 120, replace=False)
    ex = gauss_box_potential(xyz[idx], c, sig)
    assert np.linalg.norm(r["u"][idx] - ex) < 1e-4 * np.linalg.norm(ex)


def test_two_gaussians_and_parts(vp):
    """Two Gaussians of different widths and signs: closed form at sampled
    nodes; the three parts add up to u."""
    c1, s1, c2, s2 = np.array([0.1, 0.1, -0.1]), 0.12, np.array([-0.15, 0.0, 0.1]), 0.05
    f1, f2 = _gauss(c1, s1), _gauss(c2, s2)
    T = O.VTree(vp, lambda x: f1(x) - 0.5 * f2(x), 1.0, 0, 6)
    xyz = T.nodes()
    r = T.eval(f1(xyz) - 0.5 * f2(xyz))
    idx = np.random.default_rng(1).choice(len(xyz), 80, replace=False)
    ex = gauss_box_potential(xyz[idx], c1, s1) - 0.5 * gauss_box_potential(xyz[idx], c2, s2)
    assert np.linalg.norm(r["u"][idx] - ex) < 1e-4 * np.linalg.norm(ex)
    assert np.allclose(r["u"], r["ufar"] + r["unear"] + r["utail"], rtol=1e-14, atol=0)


# ------------------------------------------------- tol 1e-6: the PSWF split
TOL6 = 1e-6


@pytest.fixture(scope="module")
def vp6():
    return O.vparams_for(TOL6, 8)


def test_pswf_params(vp6):
    pr = O.params_for(TOL6)
    assert vp6.split == 1 and (vp6.p, vp6.nf) == (pr.p, pr.nf) == (18, 12)
    assert (vp6.nw, vp6.hw, vp6.c) == (pr.nw, pr.hw, pr.c)
    assert vp6.tau_a == pytest.approx(20.0) and (vp6.tpan_gl, vp6.tpan_w, vp6.theta1) == (10, 1.4, 5.0)
    assert vp6.nfit == 20 and vp6.fit_err < 1e-6
    with pytest.raises(ValueError):
        O.vparams_for(1e-4, 8)


@pytest.mark.parametrize("tau", [10.0, 20.0, 40.0])
def test_pswf_residual_as_gaussians(vp6, tau):
    """The near field's Gaussians (fitted ones, the log-t quadrature from
    theta_1 to tau) plus the asymptotic part erfc(tau x)/x reproduce the PSWF
    residual (1 - Phi(x))/x of the point-code oracle, which is zero beyond
    x = 1 (side s_L = 1; tau = t_a s_L for the three level differences)."""
    t, w, _ = O.vfit(vp6)
    tq, wq = O.GSplit(vp6).sog(vp6.theta1, tau)
    assert len(tq) % vp6.tpan_gl == 0
    ps = O.PSWF(vp6.c)
    x = np.concatenate([np.linspace(0.005, 1.0, 400), np.linspace(1.0, 5.4, 200)])
    g = np.exp(-np.outer(x * x, t * t)) @ w + np.exp(-np.outer(x * x, tq * tq)) @ wq + erfc(tau * x) / x
    ref = np.array([ps.r(0, xx) for xx in x])
    assert np.all(ref[x >= 1.0] == 0.0)
    assert np.max(np.abs(g - ref)) < 1.5e-6
    # without the fitted part the sum misses h(x) = (erf(theta_1 x) - Phi(x))/x
    assert np.max(np.abs(g - np.exp(-np.outer(x * x, t * t)) @ w - ref)) > 0.1


@pytest.mark.parametrize("level", [1, 2])
def test_pswf_uniform_cube(vp6, level):
    """Unit density on uniform trees against the closed form: 1e-7 of max u
    at nodes at least 2.5/t_a inside B_0 (measured: 1e-8 and 3e-8)."""
    T = O.VTree(vp6, lambda x: np.ones(len(x)), 1e9, level, level)
    xyz = T.nodes()
    r = T.eval(np.ones(len(xyz)))
    ex = cube_potential(xyz)
    err = np.abs(r["u"] - ex)
    inner = (0.5 - np.max(np.abs(xyz), axis=1)) >= 2.5 / (vp6.tau_a * 2 ** level)
    assert inner.sum() >= 8 ** level
    assert np.max(err[inner]) < 1e-7 * np.max(ex)
    assert np.allclose(r["u"], r["ufar"] + r["unear"] + r["utail"], rtol=1e-14, atol=0)
    # the 1e-3 code is 1e-4-accurate only: the 1e-6 result is not the 1e-3 one
    r3 = O.VTree(O.vparams_for(1e-3, 8), lambda x: np.ones(len(x)), 1e9, level, level).eval(np.ones(len(xyz)))
    assert np.max(np.abs(r3["u"] - ex)[inner]) > 10 * np.max(err[inner])
