"""Full-size volume potential on the GPU: rho = 8 Gaussians of widths
exp(U[ln 1e-3, ln 1e-1]) centred in [-0.3, 0.3]^3, refined to 3e-8 of the
peak with leaves of side <= 4 s at each centre (about 4e7 Chebyshev nodes),
tol 1e-3, FP64.  Sampled nodes against the closed-form potential of the
box-restricted Gaussians; every value finite; timings printed."""
import sys
import time

import numpy as np
import pytest

import dmk_inputs
from vol_exact import gauss_mixture_potential

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED, RHO_SCALE, MAX_LEVEL = 5, 3e-5, 16


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_full_volume():
    import paper_2308_00292_amd as dmk
    sig, cen, amp = dmk_inputs.vol_gaussians(SEED)
    f = lambda x: dmk_inputs.gaussian_mixture(x, sig, cen, amp)
    feat = dmk_inputs.gaussian_features(sig, cen)
    _say(f"[vol full] widths {np.round(np.sort(sig), 4)}; plan")
    t0 = time.perf_counter()
    plan = dmk.VolPlan(f, tol=1e-3, q=8, rho_scale=RHO_SCALE, min_level=1, max_level=MAX_LEVEL, features=feat)
    torch.cuda.synchronize()
    tplan = time.perf_counter() - t0
    lev, _ = plan.leaves()
    _say(f"[vol full] plan {tplan:.1f} s: {plan.nleaf} leaves, {plan.n} nodes, levels {np.bincount(lev)}")
    xyz = plan.nodes()
    rho = torch.zeros(plan.n, dtype=torch.float64, device="cuda")
    for s, c, a in zip(sig, cen, amp):
        cc = torch.tensor(c, dtype=torch.float64, device="cuda")
        rho += a * torch.exp(-((xyz - cc) ** 2).sum(dim=1) / (s * s))
    out = torch.empty_like(rho)
    plan.eval(rho, out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(3):
        plan.eval(rho, out)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 3
    _say(f"[vol full] eval {ms:.1f} ms = {plan.n / ms * 1e3:.3g} points/s")
    u = out.cpu().numpy()
    assert np.all(np.isfinite(u))
    idx = np.random.default_rng(3).choice(plan.n, 120, replace=False)
    x = xyz.cpu().numpy()[idx]
    ex = gauss_mixture_potential(x, sig, cen, amp)
    err = np.linalg.norm(u[idx] - ex) / np.linalg.norm(ex)
    _say(f"[vol full] sampled rel l2 vs closed form {err:.3e}")
    assert err < 1e-3
    plan.close()
