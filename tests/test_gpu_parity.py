"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

FP64 mode (both sides use the same Table 1 parameters, so they agree to
rounding, far below the 1e-6 relative l2 the method targets):
  * tree, flags, colleagues, coarse neighbours: bit-exact;
  * residual interaction lists: the same (target leaf, source box) pairs;
  * proxy charges of F_out boxes and local values on the Chebyshev grids of
    the boxes that hold them: max error <= 1e-11 of the box's largest entry;
  * far and near parts and the potential: relative l2 <= 1e-10;
  * against O(N^2) direct summation: relative l2 <= 1e-6 (2e-6 for deep
    adaptive trees, see the oracle's own pins).
Mixed mode (FP32 transforms and pair sums, FP64 offsets and final sums),
same parameters, against the same FP64 oracle: tree and lists bit-exact;
per-box data <= 2e-5 of the box's largest entry; far, near and potential
relative l2 <= 1e-5; against direct summation <= 1e-5.
"""
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


CASES = {
    "cfg1_uniform_2k": lambda: dmk_inputs.make("cfg1_uniform_2k"),
    "two_clusters_6k": lambda: (*dmk_inputs.two_clusters_and_background(6000, 101), 20),
    "sphere_blobs_20k": lambda: (*dmk_inputs.sphere_and_blobs(20000, 102), 40),
    "uniform_30k": lambda: (*dmk_inputs.uniform_cube(30000, 103), 64),
    # leaves of 65..128 points: the kernels' loops over target chunks of 64
    "uniform_50k_ns128": lambda: (*dmk_inputs.uniform_cube(50000, 104), 128),
}


_ORACLE = {}


def _oracle_run(oracle_mod, name):
    if name not in _ORACLE:
        pts, q, ns = CASES[name]()
        pr = oracle_mod.params_for(1e-6)
        ps = oracle_mod.PSWF(pr.c)
        otree = oracle_mod.Tree(pts, ns)
        ores = oracle_mod.dmk_eval(otree, pr, ps, q, keep=True)
        _ORACLE.clear()
        _ORACLE[name] = (pts, q, ns, otree, ores)
    return _ORACLE[name]


PARAMS = [(name, prec) for name in CASES for prec in ("fp64", "mixed")]
BARS = {"fp64": dict(box=1e-11, l2=1e-10), "mixed": dict(box=2e-5, l2=1e-5)}


@pytest.fixture(scope="module", params=PARAMS, ids=[f"{a}-{b}" for a, b in PARAMS])
def case(request, oracle_mod):
    import paper_2308_00292_amd as dmk
    name, prec = request.param
    pts, q, ns, otree, ores = _oracle_run(oracle_mod, name)
    _say(f"[case {name} {prec}] n={len(q)} ns={ns}")
    dev = torch.device("cuda:0")
    tp = torch.from_numpy(pts).to(dev)
    tq = torch.from_numpy(q).to(dev)
    plan = dmk.Plan(tp, tol=1e-6, leaf_max=ns,
                    precision=dmk.DMK_FP64 if prec == "fp64" else dmk.DMK_MIXED)
    pot = plan.eval(tq)
    far, near = plan.eval_parts(tq)
    torch.cuda.synchronize()
    out = dict(name=name, prec=prec, bar=BARS[prec], pts=pts, q=q, ns=ns, otree=otree, ores=ores,
               plan=plan, pot=pot.cpu().numpy(), far=far.cpu().numpy(), near=near.cpu().numpy())
    yield out
    plan.close()


def test_tree_bit_exact(case):
    ot, g = case["otree"], case["plan"].export_tree()
    assert np.array_equal(g["perm"], ot.perm)
    assert np.array_equal(g["level"], ot.level)
    assert np.array_equal(g["bkey"], ot.bkey)
    assert np.array_equal(g["parent"], ot.parent)
    assert np.array_equal(g["child0"], ot.child0)
    assert np.array_equal(g["pstart"], ot.pstart)
    assert np.array_equal(g["pcount"], ot.pcount)
    fl = g["flags"]
    assert np.array_equal(fl & 1, ot.leaf)
    assert np.array_equal((fl >> 1) & 1, ot.fout)
    assert np.array_equal((fl >> 2) & 1, ot.fin)
    assert np.array_equal((fl >> 3) & 1, ot.terminal)
    assert np.array_equal(g["colleague"], ot.colleague)
    assert np.array_equal(g["ncoarse"], ot.ncoarse)
    for b in np.nonzero(ot.ncoarse)[0]:
        k = ot.ncoarse[b]
        assert sorted(g["coarse"][b][:k]) == sorted(ot.coarse[b][:k])
    info = case["plan"].info()
    assert info["side"] == ot.side and np.array_equal(info["center"], ot.center)


def test_near_lists_match_source_centric_definition(case):
    """Gather lists on the GPU == the oracle's source-centric lists (Step 4):
    terminal box T acts on the leaves in its colleagues' subtrees and on its
    coarse-neighbour leaves."""
    ot = case["otree"]
    leaf_box, off, src = case["plan"].export_near_lists()
    got = {int(b): sorted(src[off[i]:off[i + 1]].tolist()) for i, b in enumerate(leaf_box)}
    # descendants (non-empty leaves) of every box
    desc = {}
    for b in np.nonzero((ot.leaf == 1) & (ot.pcount > 0))[0]:
        a = b
        while a >= 0:
            desc.setdefault(int(a), []).append(int(b))
            a = ot.parent[a]
    want = {int(b): [] for b in np.nonzero((ot.leaf == 1) & (ot.pcount > 0))[0]}
    for T in np.nonzero((ot.terminal == 1) & (ot.pcount > 0))[0]:
        tg = set()
        for cb in ot.colleague[T][ot.colleague[T] >= 0]:
            tg.update(desc.get(int(cb), []))
        if ot.leaf[T]:
            for cb in ot.coarse[T][: ot.ncoarse[T]]:
                if ot.pcount[cb] > 0:
                    tg.add(int(cb))
        for B in tg:
            want[B].append(int(T))
    want = {k: sorted(v) for k, v in want.items()}
    assert got == want


def test_proxies_and_locals(case):
    """Proxies of F_out boxes; local values of the boxes that store them (the
    root and the non-empty F_in boxes -- every other box's local polynomial
    is its nearest such ancestor's, by the exactness of Lemma 2.2)."""
    ot, ores, plan, bar = case["otree"], case["ores"], case["plan"], case["bar"]["box"]
    nchk = 0
    for b in np.nonzero(ot.fout)[0][:200]:
        g = plan.box_data(0, b)
        o = ores["proxy"][int(b)]
        assert np.max(np.abs(g - o)) <= bar * np.max(np.abs(o)), b
        nchk += 1
    anchors = np.nonzero((ot.pcount > 0) & ((ot.fin == 1) | (ot.parent < 0)))[0]
    for b in anchors[:400]:
        g = plan.box_data(1, b)
        o = ores["local"][int(b)]
        assert np.max(np.abs(g - o)) <= bar * np.max(np.abs(o)), b
        nchk += 1
    assert nchk > 0


def test_far_near_and_potential(case):
    ot, ores = case["otree"], case["ores"]
    scale = 1.0 / (4 * np.pi * ot.side)
    far_o = np.empty_like(case["far"])
    near_o = np.empty_like(case["near"])
    far_o[ot.perm] = ores["ufar"] * scale
    near_o[ot.perm] = ores["ures"] * scale
    bar = case["bar"]["l2"]
    assert rel_l2(case["far"], far_o) < bar
    assert rel_l2(case["near"], near_o) < bar
    assert rel_l2(case["pot"], ores["u"]) < bar
    assert np.array_equal(case["pot"], case["far"] + case["near"]) or \
        rel_l2(case["pot"], case["far"] + case["near"]) < 1e-15


def test_against_direct_sum(case, oracle_mod):
    pts, q = case["pts"], case["q"]
    n = len(q)
    idx = np.arange(n) if n <= 6000 else np.random.default_rng(0).choice(n, 3000, replace=False)
    ud = oracle_mod.direct(pts, q, idx)
    bar = 1e-6 if case["name"].startswith(("cfg1", "uniform")) else 2e-6
    if case["prec"] == "mixed":
        bar = 1e-5
    assert rel_l2(case["pot"][idx], ud) < bar


def test_deterministic(case):
    import paper_2308_00292_amd  # noqa: F401
    plan = case["plan"]
    tq = torch.from_numpy(case["q"]).to("cuda:0")
    a = plan.eval(tq).cpu().numpy()
    b = plan.eval(tq).cpu().numpy()
    assert np.array_equal(a, b)
    assert np.array_equal(a, case["pot"])


def test_batched_graph_replays_match_eager(case):
    """DMK_FLAG_BATCHED: the eval core is captured into a HIP graph and the
    residual runs on a second stream; every replay (with eager work and
    synchronisations in between) must equal the eager result bit for bit."""
    import paper_2308_00292_amd as dmk
    dev = torch.device("cuda:0")
    tp = torch.from_numpy(case["pts"]).to(dev)
    tq = torch.from_numpy(case["q"]).to(dev)
    prec = dmk.DMK_FP64 if case["prec"] == "fp64" else dmk.DMK_MIXED
    plan = dmk.Plan(tp, tol=1e-6, leaf_max=case["ns"], precision=prec, flags=dmk.DMK_FLAG_BATCHED)
    for rep in range(3):
        u = plan.eval(tq).cpu().numpy()
        assert np.array_equal(u, case["pot"]), rep
        junk = torch.randn(1000, device=dev).sum()  # eager work between replays
        torch.cuda.synchronize()
        del junk
    # new charges through the same graph
    q2 = -2.0 * case["q"]
    u2 = plan.eval(torch.from_numpy(q2).to(dev)).cpu().numpy()
    ref = case["plan"].eval(torch.from_numpy(q2).to(dev)).cpu().numpy()
    assert np.array_equal(u2, ref)
    plan.close()
