"""Pins of the oracle's 3-D Yukawa split e^{-lambda r}/(4 pi r) (Sec. 4.6,
eq. yukawaPSWFkernels; windowed root kernel of Sec. 4.7).  CPU only.

Each check ties the oracle to something fixed independently of its own
formulas:
  * the transform of the truncated kernel (closed form in yuk3.c) against
    adaptive quadrature of its radial integral (scipy);
  * lambda -> 0: the difference-kernel transform reduces to the 1/r one of
    Sec. 3.7 (eq. differencekernelft3, computed by separate code in pswf.c),
    and the mollified kernel to Phi(x)/x, the 1/r split's window built from
    Legendre antiderivatives;
  * compact support (the defining property of the split, Sec. 4.6): the
    mollified kernel M_l equals e^{-lambda r}/r for r >= s_l, so the
    residual vanishes there;
  * the plane-wave (trapezoidal) sums of D_l and of the windowed W_0 equal
    the physical-space kernels M_{l+1} - M_l and M_0 on the ranges they serve;
  * the tables against the quadrature they are fitted to;
  * end to end: the oracle DMK against O(N^2) direct sums with
    exp(-lambda r)/(4 pi r), and its lambda -> 0 limit against the 1/r oracle.
"""
import math

import numpy as np
import pytest

import dmk_inputs


@pytest.fixture(scope="module")
def y6(oracle_mod):
    pr = oracle_mod.params_for(1e-6)
    ps = oracle_mod.PSWF(pr.c)
    return pr, ps, oracle_mod.Yuk3(ps, 6.0, 8)


def test_truncated_kernel_transform(oracle_mod, y6):
    integrate = pytest.importorskip("scipy.integrate")
    pr, ps, _ = y6
    A = 1.0 + math.sqrt(3.0)
    for lam in (1e-3, 0.1, 0.5, 6.0, 30.0):
        y = oracle_mod.Yuk3(ps, lam)
        for k in (0.0, 0.3, 2.0, 7.5, 19.0):  # k = 0 at small lambda A: the series branch
            if k == 0.0:
                ref = 4 * math.pi * integrate.quad(lambda r: r * math.exp(-lam * r), 0, A, epsabs=0, epsrel=1e-13)[0]
            else:
                ref = 4 * math.pi / k * integrate.quad(lambda r: math.exp(-lam * r) * math.sin(k * r), 0, A,
                                                       epsabs=0, epsrel=1e-13, limit=200)[0]
            assert y.that(k) == pytest.approx(ref, rel=1e-11, abs=1e-14), (lam, k)


def test_laplace_limits(oracle_mod, y6):
    pr, ps, _ = y6
    y0 = oracle_mod.Yuk3(ps, 1e-9)
    for l in (0, 3):
        for k in (0.5, 3.0, 11.0, 40.0):
            assert y0.dhat(l, k) == pytest.approx(ps.dhat(l, k), rel=1e-12)
    # the mollified kernel's quadrature (cut where the mollifier argument
    # reaches 2) against Phi(x)/x; the cut costs a few 1e-7 of the scale
    for x in (0.0, 0.1, 0.4, 0.8, 1.0, 1.4):
        ref = ps.psi0 / ps.c0 if x == 0.0 else ps.phi(x) / x
        assert abs(y0.smooth_quad(1e-12, x) - ref) < 5e-7 * ps.psi0 / ps.c0


@pytest.mark.parametrize("lam", [0.5, 6.0, 40.0])
def test_mollified_kernel_is_the_kernel_beyond_the_box(oracle_mod, y6, lam):
    pr, ps, _ = y6
    y = oracle_mod.Yuk3(ps, lam)
    for l in (0, 2, 5):
        s = 2.0 ** -l
        for r in np.linspace(1.0, 2.0, 9) * s:
            m = y.smooth_quad(lam * s, r / s) / s
            assert abs(m - math.exp(-lam * r) / r) * s < 1e-6, (lam, l, r)  # to precision eps


def test_tables_match_quadrature(y6):
    pr, ps, y = y6
    for l in (0, 3, 7):
        s = 2.0 ** -l
        for x in np.linspace(0.0, 1.0, 23):
            assert abs(y.smooth(l, x) - y.smooth_quad(6.0 * s, x)) < 1e-12
        assert y.self_[l] == pytest.approx(y.smooth_quad(6.0 * s, 0.0) / s, rel=1e-13)


def test_plane_wave_sums(y6):
    pr, ps, y = y6
    rng = np.random.default_rng(3)
    for l in (0, 2):
        s = 2.0 ** -l
        err = 0.0
        for _ in range(16):
            x = rng.uniform(-2 * s, 2 * s, 3)
            r = np.linalg.norm(x)
            phys = y.smooth_quad(6.0 * s / 2, r / (s / 2)) / (s / 2) - y.smooth_quad(6.0 * s, r / s) / s
            err = max(err, abs(y.d_pw(pr, l, x) - phys) * s)
        assert err < 1e-6, (l, err)
    err = 0.0
    for _ in range(16):
        x = rng.uniform(-1, 1, 3)
        err = max(err, abs(y.w0_pw(pr, x) - y.smooth_quad(6.0, np.linalg.norm(x))))
    assert err < 1e-6, err


@pytest.mark.parametrize("case,tol,lam,bar", [
    ("uniform_2k", 1e-6, 6.0, 1e-6),
    ("uniform_2k", 1e-3, 6.0, 1e-3),
    ("uniform_2k", 1e-6, 40.0, 1e-6),
    ("clusters_4k", 1e-6, 6.0, 2e-6),
    ("clusters_4k", 1e-5, 12.0, 2e-5),
])
def test_dmk_against_direct_sums(oracle_mod, case, tol, lam, bar):
    if case == "uniform_2k":
        pts, q = dmk_inputs.uniform_cube(2000, 1)
        ns = 50
    else:
        pts, q = dmk_inputs.two_clusters_and_background(4000, 5)
        ns = 20
    pr = oracle_mod.params_for(tol)
    ps = oracle_mod.PSWF(pr.c)
    tr = oracle_mod.Tree(pts, ns)
    u = oracle_mod.dmk_eval(tr, pr, ps, q, kern=oracle_mod.YUK3, lam=lam)["u"]
    ud = oracle_mod.direct_yuk3(lam, pts, q)
    err = float(np.linalg.norm(u - ud) / np.linalg.norm(ud))
    assert err < bar, err


def test_small_lambda(oracle_mod):
    """lambda S = 1e-3, the smallest the oracle accepts: the k -> 0 limits of
    the root window and of the difference kernels stay accurate."""
    pts, q = dmk_inputs.uniform_cube(1500, 2)
    pr = oracle_mod.params_for(1e-6)
    ps = oracle_mod.PSWF(pr.c)
    tr = oracle_mod.Tree(pts, 40)
    lam = 1e-3 / tr.side
    u = oracle_mod.dmk_eval(tr, pr, ps, q, kern=oracle_mod.YUK3, lam=lam)["u"]
    ud = oracle_mod.direct_yuk3(lam, pts, q)
    assert float(np.linalg.norm(u - ud) / np.linalg.norm(ud)) < 1e-6
    with pytest.raises(RuntimeError):
        oracle_mod.dmk_eval(tr, pr, ps, q, kern=oracle_mod.YUK3, lam=0.5e-3 / tr.side)
