"""Volume potential at tol 1e-6 on the GPU: the PSWF split of Sec. 3.7 for
the far field and, for the near field of Sec. 3.6, the residual
(1 - Phi(r/s_L))/r as a quadrature of Gaussians in t plus Gaussians fitted
by least squares at plan time.

Against the FP64 oracle (its own fit, by another least-squares method):
trees bit-exact, potentials and their far and near parts to 1e-10 relative
l2 in FP64; the mixed path to 1e-5.  Against the closed-form potential of a
box-restricted Gaussian to the trees' resolution.
"""
import sys

import numpy as np
import pytest

import dmk_inputs
from vol_exact import gauss_box_potential

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BAR = 1e-10
TOL = 1e-6

CASES = {
    # name: (sigma, centre, rho_scale, min_level, max_level, closed-form bar)
    "uniform_l2": (0.2, [0.1, -0.05, 0.0], 1e9, 2, 2, 2e-6),
    # one level-1 leaf among level-2 leaves: coarse-neighbour pairs both ways
    "two_level": (0.1, [0.2, 0.15, 0.25], 1.0, 1, 2, 2e-5),
    # adaptive to level 3 (281 leaves on levels 2 and 3): 8e-8 in the oracle
    "adaptive_l3": (0.1, [0.1, -0.05, 0.12], 1.0, 1, 3, 1e-6),
}

_ORACLE = {}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(name, oracle_mod, precision):
    import paper_2308_00292_amd as dmk
    sig, cen, rs, lo, hi, cbar = CASES[name]
    f = lambda x: dmk_inputs.gaussian_mixture(x, np.array([sig]), np.array([cen]), np.array([1.0]))
    vp = oracle_mod.vparams_for(TOL, 8)
    T = oracle_mod.VTree(vp, f, rs, lo, hi)
    _say(f"[vol1e-6 {name}] oracle tree {T.nleaf} leaves; plan")
    plan = dmk.VolPlan(f, tol=TOL, q=8, rho_scale=rs, min_level=lo, max_level=hi, precision=precision)
    torch.cuda.synchronize()
    xyz = T.nodes()
    rho = f(xyz)
    if name not in _ORACLE:
        _say(f"[vol1e-6 {name}] oracle eval")
        _ORACLE[name] = T.eval(rho)
    return T, plan, xyz, rho, _ORACLE[name], (sig, cen, cbar)


@pytest.fixture(scope="module", params=list(CASES))
def case(request, oracle_mod):
    import paper_2308_00292_amd as dmk
    T, plan, xyz, rho, ref, extra = _case(request.param, oracle_mod, dmk.DMK_FP64)
    yield request.param, T, plan, xyz, rho, ref, extra
    plan.close()


def test_tree_and_nodes(case):
    name, T, plan, xyz, *_ = case
    lev, ijk = plan.leaves()
    assert np.array_equal(lev, T.level) and np.array_equal(ijk, T.ijk)
    assert np.allclose(plan.nodes().cpu().numpy(), xyz, rtol=0, atol=1e-15)


def test_potential_and_parts(case):
    name, T, plan, xyz, rho, ref, (sig, cen, cbar) = case
    r = torch.from_numpy(rho).cuda()
    u, far, near = plan.eval(r, parts=True)
    torch.cuda.synchronize()
    u, far, near = u.cpu().numpy(), far.cpu().numpy(), near.cpu().numpy()
    nu = np.linalg.norm(ref["u"])
    _say(f"[vol1e-6 {name}] rel l2 u {np.linalg.norm(u - ref['u']) / nu:.3e} far "
         f"{np.linalg.norm(far - ref['ufar']) / nu:.3e} near "
         f"{np.linalg.norm(near - ref['unear'] - ref['utail']) / nu:.3e}")
    assert np.linalg.norm(far - ref["ufar"]) < BAR * nu
    assert np.linalg.norm(near - ref["unear"] - ref["utail"]) < BAR * nu
    assert np.linalg.norm(u - ref["u"]) < BAR * nu
    # the closed form at sampled nodes (the tree's resolution bounds it)
    idx = np.random.default_rng(0).choice(len(xyz), 200, replace=False)
    ex = gauss_box_potential(xyz[idx], np.array(cen), sig)
    err = np.linalg.norm(u[idx] - ex) / np.linalg.norm(ex)
    _say(f"[vol1e-6 {name}] rel l2 vs closed form {err:.3e}")
    assert err < cbar
    assert np.array_equal(plan.eval(r).cpu().numpy(), plan.eval(r).cpu().numpy())


def test_mixed_precision(oracle_mod):
    """FP32 far-field transforms and near-field factor sums: 1e-5 of the
    FP64 oracle."""
    import paper_2308_00292_amd as dmk
    T, plan, xyz, rho, ref, _ = _case("uniform_l2", oracle_mod, dmk.DMK_MIXED)
    u, far, near = plan.eval(torch.from_numpy(rho).cuda(), parts=True)
    u, near = u.cpu().numpy(), near.cpu().numpy()
    nu = np.linalg.norm(ref["u"])
    _say(f"[vol1e-6 mixed] rel l2 u {np.linalg.norm(u - ref['u']) / nu:.3e} near "
         f"{np.linalg.norm(near - ref['unear'] - ref['utail']) / nu:.3e}")
    assert np.linalg.norm(u - ref["u"]) < 1e-5 * nu
    assert np.linalg.norm(near - ref["unear"] - ref["utail"]) < 1e-5 * nu
    plan.close()
