"""Full-size 2-D batch on the GPU: 512 independent problems of 10^3 .. 2x10^5
points each (1.79x10^7 points in all; U[0,1]^2 or 0.5 + 0.01 N(0, I_2) per
problem), the kernels -log(r)/(2 pi) and K_0(10 r), FP64 and mixed, batched
(graph) mode.  Parity on sampled outputs: for 8 problems, 100 targets each
against direct summation over that problem (2e-6 FP64, 1e-5 mixed); the
potential of every problem finite; timings printed.
"""
import sys
import time

import numpy as np
import pytest

import dmk_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def batch512():
    t0 = time.perf_counter()
    off, pts, q = dmk_inputs.batch_2d(512, 4)
    _say(f"[2d full] generated {len(q)} points in {time.perf_counter() - t0:.1f} s")
    return off, pts, q


@pytest.mark.parametrize("kern,lam", [(0, 0.0), (1, 10.0)], ids=["log", "k0"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_full_batch(batch512, oracle_mod, kern, lam, prec):
    import paper_2308_00292_amd as dmk
    off, pts, q = batch512
    dev = torch.device("cuda:0")
    tp = torch.from_numpy(pts).to(dev)
    tq = torch.from_numpy(q).to(dev)
    torch.cuda.synchronize()
    _say(f"[2d full {kern} {prec}] plan")
    t0 = time.perf_counter()
    plan = dmk.Plan(tp, tol=1e-6, leaf_max=64, offsets=off, kernel=kern, lam=lam, flags=dmk.DMK_FLAG_BATCHED,
                    precision=dmk.DMK_FP64 if prec == "fp64" else dmk.DMK_MIXED)
    torch.cuda.synchronize()
    tplan = time.perf_counter() - t0
    out = torch.empty_like(tq)
    plan.eval(tq, out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(3):
        plan.eval(tq, out)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 3
    info = plan.info()
    _say(f"[2d full {kern} {prec}] plan {tplan:.2f} s, eval {ms:.2f} ms ({len(q) / ms * 1e3:.3g} points/s), "
         f"levels {info['nlevels']} boxes {info['nbox']}")
    u = out.cpu().numpy()
    plan.close()
    assert np.all(np.isfinite(u))
    rng = np.random.default_rng(17)
    bar = 2e-6 if prec == "fp64" else 1e-5
    for b in rng.choice(512, 8, replace=False):
        pb, qb = pts[off[b]:off[b + 1]], q[off[b]:off[b + 1]]
        idx = rng.choice(len(qb), min(100, len(qb)), replace=False)
        ud = oracle_mod.direct2(kern, lam, pb, qb, idx)
        err = np.linalg.norm(u[off[b] + idx] - ud) / np.linalg.norm(ud)
        assert err < bar, (b, err)
