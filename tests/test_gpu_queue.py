"""The queue-fed upward and local stages (one launch per stage over every
level, boxes taken from a device work queue in dependency order) against
the same stages launched one level at a time (DMK_FLAG_LEVEL_LAUNCHES; in
2-D, where per-level launches are the default, DMK_FLAG_QUEUE_LAUNCHES
forces the queue).  Each box is computed by the same code in both
schedules, so potentials must agree bit for bit; no queue wait may run out
of its poll bound.  The default (queue) schedule is the one every other GPU
test compares against the oracle.

Cases: deep adaptive 3-D trees (clustered points, 14+ levels), both
precisions, eager and graph replay; a 3-D batch of problems; a volume plan;
and repeated evals (the queues' heads and flags are cleared per eval)."""
import sys

import numpy as np
import pytest

import dmk_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = {
    "clusters_80k": lambda: (*dmk_inputs.two_clusters_and_background(80000, 901), 32),
    "sphere_blobs_60k": lambda: (*dmk_inputs.sphere_and_blobs(60000, 902), 24),
}
PARAMS = [(c, prec, batched) for c in CASES for prec in ("fp64", "mixed") for batched in (False, True)]


@pytest.mark.parametrize("name,prec,batched", PARAMS,
                         ids=[f"{a}-{b}-{'graph' if c else 'eager'}" for a, b, c in PARAMS])
def test_queue_equals_level_launches(name, prec, batched):
    import paper_2308_00292_amd as dmk
    pts, q, ns = CASES[name]()
    dev = torch.device("cuda:0")
    tp, tq = torch.from_numpy(pts).to(dev), torch.from_numpy(q).to(dev)
    precision = dmk.DMK_FP64 if prec == "fp64" else dmk.DMK_MIXED
    base = dmk.DMK_FLAG_BATCHED if batched else 0
    outs = {}
    for sched, fl in (("levels", dmk.DMK_FLAG_LEVEL_LAUNCHES), ("queue", 0)):
        _say(f"[queue {name} {prec} batched={batched}] {sched}")
        plan = dmk.Plan(tp, tol=1e-6, leaf_max=ns, precision=precision, flags=base | fl)
        info = plan.info()
        res = [plan.eval(tq).cpu().numpy() for _ in range(3)]
        torch.cuda.synchronize()
        assert plan.info()["queue_timeouts"] == 0
        plan.close()
        for r in res[1:]:
            assert np.array_equal(r, res[0])
        outs[sched] = res[0]
    assert info["nlevels"] >= 12, info["nlevels"]
    assert np.array_equal(outs["queue"], outs["levels"])


def test_queue_batch3():
    import paper_2308_00292_amd as dmk
    off, pts, q = dmk_inputs.batch_3d(24, 31)
    dev = torch.device("cuda:0")
    tp, tq = torch.from_numpy(pts).to(dev), torch.from_numpy(q).to(dev)
    for precision in (dmk.DMK_FP64, dmk.DMK_MIXED):
        outs = []
        for fl in (dmk.DMK_FLAG_LEVEL_LAUNCHES, 0, dmk.DMK_FLAG_BATCHED):
            _say(f"[queue batch3 prec={precision} flags={fl}]")
            plan = dmk.Plan(tp, tol=1e-6, leaf_max=40, offsets=off, max_depth=18, precision=precision, flags=fl)
            outs.append(plan.eval(tq).cpu().numpy())
            torch.cuda.synchronize()
            assert plan.info()["queue_timeouts"] == 0
            plan.close()
        assert np.array_equal(outs[1], outs[0]) and np.array_equal(outs[2], outs[0])


def test_queue_volume():
    import paper_2308_00292_amd as dmk
    sig, cen, amp = np.array([0.12, 0.02]), np.array([[-0.1, 0.05, 0.0], [0.13, 0.1, -0.2]]), np.array([1.0, -0.7])
    f = lambda x: dmk_inputs.gaussian_mixture(x, sig, cen, amp)
    feats = dmk_inputs.gaussian_features(sig, cen)
    for precision in (dmk.DMK_FP64, dmk.DMK_MIXED):
        outs = []
        for fl in (dmk.DMK_FLAG_LEVEL_LAUNCHES, 0):
            _say(f"[queue volume prec={precision} flags={fl}]")
            vp = dmk.VolPlan(f, tol=1e-3, q=8, rho_scale=10.0, min_level=1, max_level=5, features=feats,
                             precision=precision, flags=fl)
            xyz = vp.nodes().cpu().numpy()
            rho = torch.from_numpy(f(xyz)).to("cuda:0")
            outs.append(vp.eval(rho).cpu().numpy())
            torch.cuda.synchronize()
            assert vp.info()["queue_timeouts"] == 0
            vp.close()
        assert np.array_equal(outs[1], outs[0])


P2_CASES = [("gauss2d_60k", "log"), ("gauss2d_60k", "k0"), ("batch2d", "log")]


@pytest.mark.parametrize("name,kn", P2_CASES, ids=[f"{a}-{b}" for a, b in P2_CASES])
def test_queue_2d(name, kn):
    import paper_2308_00292_amd as dmk
    if name == "batch2d":
        off, pts, q = dmk_inputs.batch_2d(48, 907, nmin=300, nmax=20000)
        extra = dict(offsets=off, max_depth=20)
    else:
        pts, q = dmk_inputs.gaussian_2d(60000, 906)
        extra = {}
    kern = dmk.DMK_LAPLACE if kn == "log" else dmk.DMK_YUKAWA
    dev = torch.device("cuda:0")
    tp, tq = torch.from_numpy(pts).to(dev), torch.from_numpy(q).to(dev)
    for precision in (dmk.DMK_FP64, dmk.DMK_MIXED):
        outs = []
        # 2-D plans launch per level by default: the queue is forced here
        for fl in (0, dmk.DMK_FLAG_QUEUE_LAUNCHES, dmk.DMK_FLAG_QUEUE_LAUNCHES | dmk.DMK_FLAG_BATCHED):
            _say(f"[queue 2-D {name} {kn} prec={precision} flags={fl}]")
            plan = dmk.Plan(tp, tol=1e-6, leaf_max=32, precision=precision, flags=fl, kernel=kern, lam=10.0, **extra)
            res = [plan.eval(tq).cpu().numpy() for _ in range(2)]
            torch.cuda.synchronize()
            assert plan.info()["queue_timeouts"] == 0
            if name != "batch2d":
                assert plan.info()["nlevels"] >= 8
            plan.close()
            assert np.array_equal(res[1], res[0])
            outs.append(res[0])
        assert np.array_equal(outs[1], outs[0]) and np.array_equal(outs[2], outs[0])


def test_schedule_flags_exclusive():
    import paper_2308_00292_amd as dmk
    pts, q = dmk_inputs.uniform_cube(2000, 908)
    with pytest.raises(dmk.DmkError) as e:
        dmk.Plan(torch.from_numpy(pts).to("cuda:0"), tol=1e-6,
                 flags=dmk.DMK_FLAG_LEVEL_LAUNCHES | dmk.DMK_FLAG_QUEUE_LAUNCHES)
    assert e.value.status == -1
