"""Pins of the oracle's 3-D 1/r^2 split (PSWF power-function window,
Sec. 4.5, eqs. powerfunctionkernels and powerphil with alpha = 2).  CPU only.

  * C_1 = int_0^1 t psi(t) dt and Phi against scipy quadrature, Phi(1) = 1,
    Phi'(x) = x psi(x)/C_1 by finite differences, the table against the
    defining integral;
  * the splitting identity W_0 + sum_{l<L} D_l + R_L = 1/r^2 on the range
    the windowed root serves (r <= sqrt 3), and compact support of D_l and
    R_L beyond their box size;
  * the radial transform of D_0 against scipy quadrature;
  * plane-wave sums of D_l (colleague range) and W_0 (offsets in the unit
    box) against the physical kernels, within tol of their scale;
  * end to end: the oracle DMK against O(N^2) direct sums of q_j/r_ij^2.
"""
import math

import numpy as np
import pytest

import dmk_inputs


@pytest.fixture(scope="module", params=[1e-3, 1e-6], ids=["tol1e-3", "tol1e-6"])
def p2(request, oracle_mod):
    pr = oracle_mod.params_for(request.param)
    ps = oracle_mod.PSWF(pr.c)
    return request.param, pr, ps, oracle_mod.Pow2(ps)


def test_window_function(p2):
    integrate = pytest.importorskip("scipy.integrate")
    tol, pr, ps, w = p2
    c1 = integrate.quad(lambda t: t * ps.psi(t), 0, 1, epsabs=0, epsrel=1e-13)[0]
    assert w.c1 == pytest.approx(c1, rel=1e-13)
    for x in (0.1, 0.37, 0.8, 0.99):
        ref = integrate.quad(lambda t: t * ps.psi(t), 0, x, epsabs=0, epsrel=1e-13)[0] / c1
        assert w.phi_quad(x) == pytest.approx(ref, rel=1e-12)
        assert abs(w.phi(x) - w.phi_quad(x)) < 1e-13
        h = 1e-5
        deriv = (w.phi(x + h) - w.phi(x - h)) / (2 * h)
        assert deriv == pytest.approx(x * ps.psi(x) / c1, rel=1e-7)
    assert w.phi_quad(1.0 - 1e-12) == pytest.approx(1.0, abs=1e-10)
    assert w.m0(0) == pytest.approx(ps.psi0 / (2 * c1), rel=1e-14)


def test_splitting_identity_and_support(p2):
    tol, pr, ps, w = p2
    rng = np.random.default_rng(0)
    for r in np.concatenate([rng.uniform(1e-3, math.sqrt(3), 30), [0.01, 0.5, 1.0, 1.7]]):
        for L in range(0, 7):
            tot = w.w0(r) + sum(w.d(l, r) for l in range(L)) + w.r(L, r)
            assert tot == pytest.approx(1.0 / r ** 2, rel=1e-12), (r, L)
    for l in (0, 3):
        s = 2.0 ** -l
        assert w.d(l, s * 1.0001) == 0.0 and w.r(l, s * 1.0001) == 0.0
        assert w.d(l, s * 1.7) == 0.0


def test_difference_kernel_transform(p2):
    integrate = pytest.importorskip("scipy.integrate")
    tol, pr, ps, w = p2
    for k in (0.0, 1.3, 6.0, 17.0, 40.0):
        if k == 0.0:
            ref = 4 * math.pi * sum(integrate.quad(lambda r: w.d(0, r) * r * r, a, b, epsabs=0, epsrel=1e-13)[0]
                                    for a, b in ((0, 0.5), (0.5, 1)))
        else:
            ref = 4 * math.pi / k * sum(
                integrate.quad(lambda r: w.d(0, r) * r * math.sin(k * r), a, b, epsabs=0, epsrel=1e-13, limit=200)[0]
                for a, b in ((0, 0.5), (0.5, 1)))
        assert w.dhat(0, k) == pytest.approx(ref, rel=1e-10, abs=1e-12)


def test_plane_wave_sums(p2):
    tol, pr, ps, w = p2
    rng = np.random.default_rng(1)
    for l in (0, 2):
        s = 2.0 ** -l
        err = 0.0
        for _ in range(8):
            x = rng.uniform(-2 * s, 2 * s, 3)
            err = max(err, abs(w.d_pw(pr, l, x) - w.d(l, np.linalg.norm(x))))
        assert err < tol * w.d(l, 0.0), (l, err)
    err = 0.0
    for _ in range(8):
        x = rng.uniform(-1, 1, 3)
        err = max(err, abs(w.w0_pw(pr, x) - w.w0(np.linalg.norm(x))))
    assert err < tol * w.m0(0), err


@pytest.mark.parametrize("case,tol,bar", [
    ("uniform_2k", 1e-6, 1e-6), ("uniform_2k", 1e-3, 1e-3), ("clusters_4k", 1e-6, 2e-6),
    ("clusters_4k", 1e-5, 2e-5),
])
def test_dmk_against_direct_sums(oracle_mod, case, tol, bar):
    if case == "uniform_2k":
        pts, q = dmk_inputs.uniform_cube(2000, 1)
        ns = 50
    else:
        pts, q = dmk_inputs.two_clusters_and_background(4000, 5)
        ns = 20
    pr = oracle_mod.params_for(tol)
    tr = oracle_mod.Tree(pts, ns)
    u = oracle_mod.dmk_eval(tr, pr, oracle_mod.PSWF(pr.c), q, kern=oracle_mod.POW3)["u"]
    ud = oracle_mod.direct_pow2(pts, q)
    assert float(np.linalg.norm(u - ud) / np.linalg.norm(ud)) < bar
