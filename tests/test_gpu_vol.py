"""Volume potential on the GPU against the FP64 oracle.

Trees (leaf levels and cells) bit-exact; node coordinates equal; potentials
and their far and near parts to 1e-10 relative l2 in FP64.  Cases: a uniform
tree, an adaptive tree with coarse-neighbour pairs, and two Gaussians refined
around caller-given feature points; plus API misuse and determinism.
"""
import sys

import numpy as np
import pytest

import dmk_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BAR = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = {
    # name: (density kwargs, rho_scale, min_level, max_level, features)
    "uniform_l2": (dict(sig=[0.2], cen=[[0.1, -0.05, 0.0]], amp=[1.0]), 1e9, 2, 2, False),
    "adaptive": (dict(sig=[0.05], cen=[[0.1, -0.05, 0.12]], amp=[1.0]), 1.0, 1, 3, False),
    "two_gauss_feat": (dict(sig=[0.12, 0.02], cen=[[-0.1, 0.05, 0.0], [0.13, 0.1, -0.2]], amp=[1.0, -0.7]),
                       10.0, 1, 5, True),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, oracle_mod):
    yield from _case(request.param, oracle_mod, fp64=True)


_ORACLE = {}  # oracle results per case, shared by the FP64 and mixed fixtures


def _case(name, oracle_mod, fp64):
    import paper_2308_00292_amd as dmk
    kw, rs, lo, hi, feat = CASES[name]
    sig, cen, amp = np.array(kw["sig"]), np.array(kw["cen"]), np.array(kw["amp"])
    f = lambda x: dmk_inputs.gaussian_mixture(x, sig, cen, amp)
    features = dmk_inputs.gaussian_features(sig, cen) if feat else None
    vp = oracle_mod.vparams_for(1e-3, 8)
    T = oracle_mod.VTree(vp, f, rs, lo, hi, features=features)
    _say(f"[vol {name}] oracle tree {T.nleaf} leaves; plan")
    plan = dmk.VolPlan(f, tol=1e-3, q=8, rho_scale=rs, min_level=lo, max_level=hi, features=features,
                       precision=dmk.DMK_FP64 if fp64 else dmk.DMK_MIXED)
    torch.cuda.synchronize()
    xyz_o = T.nodes()
    rho = f(xyz_o)
    if name not in _ORACLE:
        _say(f"[vol {name}] oracle eval")
        _ORACLE[name] = T.eval(rho)
    ref = _ORACLE[name]
    yield name, T, plan, xyz_o, rho, ref
    plan.close()


def test_tree_bit_exact(case):
    name, T, plan, *_ = case
    lev, ijk = plan.leaves()
    assert plan.nleaf == T.nleaf
    assert np.array_equal(lev, T.level)
    assert np.array_equal(ijk, T.ijk)


def test_nodes(case):
    name, T, plan, xyz_o, *_ = case
    xyz = plan.nodes().cpu().numpy()
    assert np.allclose(xyz, xyz_o, rtol=0, atol=1e-15)


def test_potential_and_parts(case):
    name, T, plan, xyz_o, rho, ref = case
    r = torch.from_numpy(rho).cuda()
    u, far, near = plan.eval(r, parts=True)
    torch.cuda.synchronize()
    u, far, near = u.cpu().numpy(), far.cpu().numpy(), near.cpu().numpy()
    nu = np.linalg.norm(ref["u"])
    _say(f"[vol {name}] rel l2 u {np.linalg.norm(u - ref['u']) / nu:.3e} far "
         f"{np.linalg.norm(far - ref['ufar']) / nu:.3e} near "
         f"{np.linalg.norm(near - ref['unear'] - ref['utail']) / nu:.3e}")
    assert np.linalg.norm(far - ref["ufar"]) < BAR * nu
    assert np.linalg.norm(near - ref["unear"] - ref["utail"]) < BAR * nu
    assert np.linalg.norm(u - ref["u"]) < BAR * nu
    # u alone, and bit-identical on a second call
    u2 = plan.eval(r).cpu().numpy()
    u3 = plan.eval(r).cpu().numpy()
    assert np.array_equal(u2, u3)
    assert np.allclose(u2, u, rtol=0, atol=1e-15 * np.max(np.abs(u)))


@pytest.fixture(scope="module", params=["adaptive", "two_gauss_feat"])
def case_mixed(request, oracle_mod):
    yield from _case(request.param, oracle_mod, fp64=False)


def test_mixed_precision(case_mixed):
    """Far-field transforms and near-field factor sums in FP32 (the asymptotic
    part and the final sums FP64): 1e-5 of the FP64 oracle, the point code's
    mixed bar, for the potential and for its near part alone."""
    name, T, plan, xyz_o, rho, ref = case_mixed
    lev, ijk = plan.leaves()
    assert np.array_equal(lev, T.level) and np.array_equal(ijk, T.ijk)
    u, far, near = plan.eval(torch.from_numpy(rho).cuda(), parts=True)
    u, far, near = u.cpu().numpy(), far.cpu().numpy(), near.cpu().numpy()
    nu = np.linalg.norm(ref["u"])
    _say(f"[vol mixed {name}] rel l2 u {np.linalg.norm(u - ref['u']) / nu:.3e} far "
         f"{np.linalg.norm(far - ref['ufar']) / nu:.3e} near "
         f"{np.linalg.norm(near - ref['unear'] - ref['utail']) / nu:.3e}")
    assert np.linalg.norm(u - ref["u"]) < 1e-5 * nu
    assert np.linalg.norm(near - ref["unear"] - ref["utail"]) < 1e-5 * nu


def test_api_misuse(oracle_mod):
    import paper_2308_00292_amd as dmk
    f = lambda x: np.ones(len(x))
    with pytest.raises(dmk.DmkError):
        dmk.VolPlan(f, tol=1e-4)
    with pytest.raises(dmk.DmkError):
        dmk.VolPlan(f, q=6)
    with pytest.raises(dmk.DmkError):
        dmk.VolPlan(f, min_level=0)
    with pytest.raises(dmk.DmkError):
        dmk.VolPlan(f, min_level=3, max_level=2)
    with pytest.raises(dmk.DmkError):
        dmk.VolPlan(lambda x: np.full(len(x), np.nan), min_level=1, max_level=3)
    with pytest.raises(dmk.DmkError):
        dmk.VolPlan(f, features=np.array([[0.0, 0.0, 0.0, -1.0]]))
    vp = dmk.VolPlan(f, min_level=1, max_level=1)
    assert vp.nleaf == 8 and vp.n == 8 * 512
    with pytest.raises(TypeError):
        vp.eval(torch.zeros(10, dtype=torch.float64, device="cuda"))
    # a volume plan is not a point plan and vice versa
    q = torch.zeros(vp.n, dtype=torch.float64, device="cuda")
    out = torch.empty_like(q)
    L = dmk.lib()
    import ctypes as C
    rc = L.dmk_eval(vp._h, C.c_void_p(q.data_ptr()), C.c_void_p(out.data_ptr()), None)
    assert rc != 0
    pts = torch.rand(100, 3, dtype=torch.float64, device="cuda")
    pp = dmk.Plan(pts, tol=1e-6)
    rc = L.dmk_vol_eval(pp._h, C.c_void_p(q.data_ptr()), C.c_void_p(out.data_ptr()), None, None, None)
    assert rc != 0
    rc = L.dmk_vol_eval(vp._h, C.c_void_p(q.data_ptr()), None, None, None, None)
    assert rc != 0
    pp.close()
    vp.close()
