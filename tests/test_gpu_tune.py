"""The autotuner (dmk_tune): the (p, n_f) pair it keeps meets the requested
tolerance on the caller's data, measured against direct sums computed here
by the oracle at the same sample targets; it is the coarsest compiled pair
that does; its leaf capacity is one of the candidates and the fastest of
them in its own timings; a caller's p is respected."""
import sys

import numpy as np
import pytest

import dmk_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PAIRS = [(9, 6), (15, 10), (18, 12)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sample(n):
    ns = min(256, n)
    return np.array([int((k + 0.5) * n / ns) for k in range(ns)], dtype=np.int64)


@pytest.mark.parametrize("tol,prec", [(1e-3, 0), (1e-5, 1), (1e-6, 0)], ids=["1e-3-fp64", "1e-5-mixed", "1e-6-fp64"])
def test_tune_3d(tol, prec, oracle_mod):
    import paper_2308_00292_amd as dmk
    pts, q = dmk_inputs.sphere_and_blobs(30000, 801)
    dev = torch.device("cuda:0")
    tp, tq = torch.from_numpy(pts).to(dev), torch.from_numpy(q).to(dev)
    cand = [32, 64, 96]
    best, ms, err = dmk.tune(tp, tq, cand, tol=tol, precision=prec, reps=2)
    _say(f"[tune 3d tol={tol:g} prec={prec}] best {best} ms {ms} err {err:.2e}")
    assert (best["p"], best["n_f"]) in PAIRS and best["leaf_max"] in cand
    assert ms[best["leaf_max"]] == min(ms.values())
    assert err <= tol
    # the tuned configuration, checked independently against the oracle's direct sums
    pl = dmk.Plan(tp, tol=tol, leaf_max=best["leaf_max"], precision=prec, p=best["p"], n_f=best["n_f"],
                  pswf_c=best["pswf_c"])
    u = pl.eval(tq).cpu().numpy()
    pl.close()
    idx = _sample(len(q))
    ud = oracle_mod.direct(pts, q, idx)
    e = float(np.linalg.norm(u[idx] - ud) / np.linalg.norm(ud))
    assert e == pytest.approx(err, rel=1e-6, abs=1e-12)
    # no coarser pair meets tol at the chosen n_s
    k = PAIRS.index((best["p"], best["n_f"]))
    if k > 0:
        pc, nc = PAIRS[k - 1]
        pl = dmk.Plan(tp, tol=tol, leaf_max=best["leaf_max"], precision=prec, p=pc, n_f=nc, pswf_c=best["pswf_c"])
        u = pl.eval(tq).cpu().numpy()
        pl.close()
        assert float(np.linalg.norm(u[idx] - ud) / np.linalg.norm(ud)) > tol


def test_tune_respects_callers_p_and_2d_kernels(oracle_mod):
    import paper_2308_00292_amd as dmk
    dev = torch.device("cuda:0")
    pts, q = dmk_inputs.uniform_cube(8000, 802)
    best, ms, err = dmk.tune(torch.from_numpy(pts).to(dev), torch.from_numpy(q).to(dev), [40], tol=1e-6, p=15)
    assert best["p"] == 15 and best["n_f"] == 10
    off, p2, q2 = dmk_inputs.batch_2d(6, 9, nmin=500, nmax=4000)
    best, ms, err = dmk.tune(torch.from_numpy(p2).to(dev), torch.from_numpy(q2).to(dev), [30, 60], tol=1e-5,
                             kernel=dmk.DMK_YUKAWA, lam=10.0, offsets=off)
    _say(f"[tune 2d K0] best {best} err {err:.2e}")
    assert err <= 1e-5 and (best["p"], best["n_f"]) in PAIRS
    # the gate's direct sums: K_0 within each problem
    idx = _sample(len(q2))
    b_of = np.searchsorted(off, idx, side="right") - 1
    ud = np.array([oracle_mod.direct2(oracle_mod.YUK2, 10.0, p2[off[b]:off[b + 1]], q2[off[b]:off[b + 1]],
                                      np.array([i - off[b]]))[0] for i, b in zip(idx, b_of)])
    pl = dmk.Plan(torch.from_numpy(p2).to(dev), tol=1e-5, leaf_max=best["leaf_max"], p=best["p"], n_f=best["n_f"],
                  pswf_c=best["pswf_c"], kernel=dmk.DMK_YUKAWA, lam=10.0, offsets=off)
    u = pl.eval(torch.from_numpy(q2).to(dev)).cpu().numpy()
    pl.close()
    e = float(np.linalg.norm(u[idx] - ud) / np.linalg.norm(ud))
    assert e == pytest.approx(err, rel=1e-6, abs=1e-12)
