"""dmk_eval_noalloc (workspace in the library's static device scratch)
against dmk_eval through the C ABI: identical potentials, bit for bit, on
two calls in a row, the second with a smaller point set; plans without
workspace of their own; 2-D and mixed-precision batched plans; the size
limit and the misuse errors."""
import sys

import numpy as np
import pytest

import dmk_inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("dim,precision,flags", [(3, 0, 0), (3, 1, 2), (2, 0, 2), (2, 1, 0)],
                         ids=["3d_fp64", "3d_mixed_batched", "2d_fp64_batched", "2d_mixed"])
def test_noalloc_matches_eval_twice(dim, precision, flags, oracle_mod):
    import paper_2308_00292_amd as dmk
    gen = dmk_inputs.uniform_cube if dim == 3 else dmk_inputs.uniform_square
    results = []
    for n, seed in ((6000, 401), (1500, 402)):  # the second call is smaller
        _say(f"[noalloc] dim {dim} precision {precision} flags {flags} n {n}")
        pts, q = gen(n, seed)
        dp, dq = _dev(pts), _dev(q)
        ref_plan = dmk.Plan(dp, tol=1e-6, leaf_max=40, precision=precision, flags=flags)
        ref = ref_plan.eval(dq).cpu().numpy()
        # a plan with no workspace of its own, evaluated from the static scratch
        pl = dmk.Plan(dp, tol=1e-6, leaf_max=40, precision=precision, flags=flags | dmk.DMK_FLAG_NO_WORKSPACE)
        out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        pl.eval_noalloc(dq, out)
        u = out.cpu().numpy()
        assert np.array_equal(u, ref), f"max diff {np.max(np.abs(u - ref))}"
        # the plan-owning plan through the static scratch as well
        out2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        ref_plan.eval_noalloc(dq, out2)
        assert np.array_equal(out2.cpu().numpy(), ref)
        # and its own workspace is untouched: dmk_eval still gives the same
        assert np.array_equal(ref_plan.eval(dq).cpu().numpy(), ref)
        results.append((pts, q, u))
        with pytest.raises(dmk.DmkError) as e:
            pl.eval(dq)
        assert e.value.status == -6
        pl.close()
        ref_plan.close()
    if dim == 3 and precision == 0:
        pts, q, u = results[1]
        o = oracle_mod.dmk(pts, q, 1e-6, 40)
        assert float(np.linalg.norm(u - o) / np.linalg.norm(o)) < 1e-10


def test_noalloc_size_limit_and_misuse():
    import paper_2308_00292_amd as dmk
    _say("[noalloc] workspace above the static scratch")
    pts, q = dmk_inputs.uniform_cube(200000, 403)
    pl = dmk.Plan(_dev(pts), tol=1e-6, leaf_max=32, flags=dmk.DMK_FLAG_NO_WORKSPACE)
    out = torch.zeros(len(q), dtype=torch.float64, device="cuda:0")
    with pytest.raises(dmk.DmkError) as e:
        pl.eval_noalloc(_dev(q), out)
    assert e.value.status == -1 and b"exceeds" in dmk.lib().dmk_last_error()
    pl.close()
    _say("[noalloc] empty plan and NULL arguments")
    p0 = dmk.Plan(_dev(np.zeros((0, 3))), tol=1e-6, flags=dmk.DMK_FLAG_NO_WORKSPACE)
    e0 = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    p0.eval_noalloc(e0, e0)
    p0.close()
    assert dmk.lib().dmk_eval_noalloc(None, None, None, None) == -1
