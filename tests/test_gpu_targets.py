"""Separate target sets (dmk_plan_targets, 3-D): potentials at ntgt targets
from nsrc sources.  Against the FP64 oracle run on the union of the sets
(sources, then targets with zero charge, which add nothing to any
potential): the tree of the union bit for bit, the potentials at the
targets within 1e-10 (FP64) and 1e-5 (mixed) relative l2, and direct sums
over the sources within tol (2 tol on adaptive sets).  Targets placed
exactly on sources exercise the r = 0 rule; uneven set sizes and empty sets
the edges.  Kernels 1/(4 pi r), exp(-6 r)/(4 pi r) and 1/r^2."""
import sys

import numpy as np
import pytest

import dmk_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(name):
    if name == "clusters_src_uniform_tgt":
        src, q = dmk_inputs.two_clusters_and_background(6000, 901)
        tgt, _ = dmk_inputs.uniform_cube(3000, 902)
        return src, q, tgt, 30
    if name == "uniform_src_sphere_tgt_coincident":
        src, q = dmk_inputs.uniform_cube(4000, 903)
        tgt, _ = dmk_inputs.sphere_and_blobs(5000, 904)
        tgt = np.concatenate([tgt, src[::80]])  # 50 targets exactly on sources
        return src, q, tgt, 40
    if name == "few_sources":
        src, q = dmk_inputs.uniform_cube(200, 905)
        tgt, _ = dmk_inputs.uniform_cube(20000, 906)
        return src, q, tgt, 64
    if name == "few_targets":
        src, q = dmk_inputs.sphere_and_blobs(20000, 907)
        tgt, _ = dmk_inputs.uniform_cube(100, 908)
        return src, q, tgt, 64
    raise KeyError(name)


PARAMS = [("clusters_src_uniform_tgt", "lap", "fp64"), ("clusters_src_uniform_tgt", "lap", "mixed"),
          ("uniform_src_sphere_tgt_coincident", "lap", "fp64"), ("uniform_src_sphere_tgt_coincident", "lap", "mixed"),
          ("few_sources", "lap", "fp64"), ("few_targets", "lap", "mixed"),
          ("clusters_src_uniform_tgt", "yuk", "fp64"), ("clusters_src_uniform_tgt", "pow2", "mixed")]


@pytest.mark.parametrize("name,kn,prec", PARAMS, ids=[f"{a}-{b}-{c}" for a, b, c in PARAMS])
def test_separate_targets(name, kn, prec, oracle_mod):
    import paper_2308_00292_amd as dmk
    src, q, tgt, ns = _case(name)
    tol = 1e-6
    kern, okern, lam = {"lap": (dmk.DMK_LAPLACE, oracle_mod.LAP3, 0.0), "yuk": (dmk.DMK_YUKAWA, oracle_mod.YUK3, 6.0),
                        "pow2": (dmk.DMK_POWER2, oracle_mod.POW3, 0.0)}[kn]
    _say(f"[targets {name} {kn} {prec}] nsrc={len(src)} ntgt={len(tgt)}")
    dev = torch.device("cuda:0")
    plan = dmk.Plan(torch.from_numpy(src).to(dev), tol=tol, leaf_max=ns, kernel=kern, lam=lam,
                    precision=dmk.DMK_FP64 if prec == "fp64" else dmk.DMK_MIXED,
                    targets=torch.from_numpy(np.ascontiguousarray(tgt)).to(dev))
    info = plan.info()
    assert (info["nsrc"], info["ntgt"], info["n"]) == (len(src), len(tgt), len(src) + len(tgt))
    tq = torch.from_numpy(q).to(dev)
    pot = plan.eval(tq).cpu().numpy()
    far, near = plan.eval_parts(tq)
    assert np.array_equal(pot, (far + near).cpu().numpy()) or rel_l2(pot, (far + near).cpu().numpy()) < 1e-15
    g = plan.export_tree()
    plan.close()
    upts, uq, tidx = oracle_mod.union_targets(src, q, tgt)
    tr = oracle_mod.Tree(upts, ns)
    for k in ("perm", "level", "bkey", "parent", "child0", "pstart", "pcount", "colleague", "ncoarse"):
        assert np.array_equal(g[k], getattr(tr, k)), k
    for bit, k in enumerate(("leaf", "fout", "fin", "terminal")):
        assert np.array_equal((g["flags"] >> bit) & 1, getattr(tr, k)), k
    pr = oracle_mod.params_for(tol)
    uo = oracle_mod.dmk_eval(tr, pr, oracle_mod.PSWF(pr.c), uq, kern=okern, lam=lam)["u"][tidx]
    if kn == "lap":
        ud = oracle_mod.direct(upts, uq, tidx)
    elif kn == "yuk":
        ud = oracle_mod.direct_yuk3(lam, upts, uq, tidx)
    else:
        ud = oracle_mod.direct_pow2(upts, uq, tidx)
    e_o, e_d = rel_l2(pot, uo), rel_l2(pot, ud)
    bar_o = 1e-10 if prec == "fp64" else 1e-5
    bar_d = 1e-5 if prec == "mixed" else (tol if name == "few_sources" else 2 * tol)
    _say(f"[targets {name} {kn} {prec}] vs oracle {e_o:.2e} (bar {bar_o:g}); vs direct {e_d:.2e} (bar {bar_d:g})")
    assert e_o < bar_o
    assert e_d < bar_d


def test_separate_targets_edges():
    import paper_2308_00292_amd as dmk
    dev = torch.device("cuda:0")
    src, q = dmk_inputs.uniform_cube(500, 911)
    tgt, _ = dmk_inputs.uniform_cube(300, 912)
    ts, tt, tq = (torch.from_numpy(a).to(dev) for a in (src, tgt, q))
    empty = torch.zeros((0, 3), dtype=torch.float64, device=dev)
    # no sources: zero potentials
    p0 = dmk.Plan(empty, tol=1e-6, targets=tt)
    u = p0.eval(torch.zeros(0, dtype=torch.float64, device=dev)).cpu().numpy()
    p0.close()
    assert u.shape == (300,) and np.all(u == 0.0)
    # no targets: an empty result
    p1 = dmk.Plan(ts, tol=1e-6, targets=empty)
    assert p1.eval(tq).numel() == 0
    p1.close()
    # graph replay equals eager launches
    pe = dmk.Plan(ts, tol=1e-6, leaf_max=20, targets=tt, precision=dmk.DMK_MIXED)
    ref = pe.eval(tq).cpu().numpy()
    pe.close()
    pb = dmk.Plan(ts, tol=1e-6, leaf_max=20, targets=tt, precision=dmk.DMK_MIXED, flags=dmk.DMK_FLAG_BATCHED)
    for _ in range(3):
        assert np.array_equal(pb.eval(tq).cpu().numpy(), ref)
    pb.close()
