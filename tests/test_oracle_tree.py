"""Pins of the oracle's adaptive tree (CPU only), by brute force over boxes.

Definitions (Sec. 3.2 and Step 0 of Sec. 3.5): refinement while a box holds
more than n_s points; level restriction between leaves that share a boundary
point; colleagues; coarse neighbours; flags F_leaf / F_out / F_in.  The
oracle builds the tree by fixing violations one at a time; here every property
is re-derived from box geometry with O(B^2) integer comparisons.
"""
import numpy as np
import pytest

import dmk_inputs


def _coords(tree):
    """integer box coordinates at each box's own level"""
    nb, dim = tree.nbox, tree.dim
    c = np.zeros((nb, dim), dtype=np.int64)
    for b in range(nb):
        key = int(tree.bkey[b])
        l = int(tree.level[b])
        for bit in range(l):
            for d in range(dim):
                c[b, d] |= ((key >> (dim * bit + (dim - 1 - d))) & 1) << bit
    return c


def _extent(tree, coords, L):
    lev = tree.level.astype(np.int64)
    f = (1 << (L - lev))[:, None]
    return coords * f, (coords + 1) * f


def _touch(lo, hi, a, bs):
    """closed boxes of a and each of bs intersect"""
    return np.all((lo[bs] <= hi[a]) & (lo[a] <= hi[bs]), axis=1)


CASES = [
    ("adaptive", lambda: dmk_inputs.two_clusters_and_background(1500, 11), 20),
    ("sphere", lambda: dmk_inputs.sphere_and_blobs(3000, 12), 30),
    ("uniform", lambda: dmk_inputs.uniform_cube(3000, 13), 40),
    ("square2d", lambda: dmk_inputs.uniform_square(3000, 14), 30),
    ("gaussian2d", lambda: dmk_inputs.gaussian_2d(3000, 15, sigma=0.02), 20),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def built(request, oracle_mod):
    _, gen, ns = request.param
    pts, q = gen()
    tree = oracle_mod.Tree(pts, ns)
    coords = _coords(tree)
    L = tree.nlevels - 1
    lo, hi = _extent(tree, coords, L)
    return tree, pts, coords, lo, hi, ns


def test_structure(built):
    tree, pts, coords, lo, hi, ns = built
    assert tree.level_start[0] == 0 and tree.level_start[-1] == tree.nbox
    for l in range(tree.nlevels):
        b0, b1 = tree.level_start[l], tree.level_start[l + 1]
        assert np.all(tree.level[b0:b1] == l)
        assert np.all(np.diff(tree.bkey[b0:b1].astype(np.uint64)) > 0)  # Morton order
    for b in range(tree.nbox):
        if tree.leaf[b]:
            assert tree.child0[b] == -1
        else:
            ch = tree.child0[b] + np.arange(2 ** tree.dim)
            assert np.all(tree.parent[ch] == b)
            assert tree.pcount[ch].sum() == tree.pcount[b]
            assert tree.pstart[ch[0]] == tree.pstart[b]


def test_points_in_boxes(built):
    tree, pts, coords, lo, hi, ns = built
    # the sorted points are the input points, rescaled into [-1/2,1/2]^d
    x = (pts[tree.perm] - tree.center) / tree.side
    assert np.array_equal(x, tree.xs)
    assert np.all(np.abs(tree.xs) < 0.5)
    for b in range(tree.nbox):
        l = tree.level[b]
        s = 2.0 ** -l
        blo = -0.5 + coords[b] * s
        xb = tree.xs[tree.pstart[b]: tree.pstart[b] + tree.pcount[b]]
        assert np.all(xb >= blo - 1e-15) and np.all(xb <= blo + s + 1e-15)


def test_refinement_and_balance(built):
    tree, pts, coords, lo, hi, ns = built
    leaves = np.nonzero(tree.leaf)[0]
    for b in leaves:
        assert tree.pcount[b] <= ns or tree.level[b] == tree.maxdepth
    # level restriction between touching leaves
    for a in leaves:
        t = _touch(lo, hi, a, leaves)
        assert np.all(np.abs(tree.level[leaves[t]] - tree.level[a]) <= 1)
    # minimality: a non-leaf holding <= n_s points is forced by a refined box
    # one level finer that shares a boundary point with it
    nonleaf = np.nonzero(tree.leaf == 0)[0]
    for b in nonleaf:
        if tree.pcount[b] > ns:
            continue
        cand = nonleaf[(tree.level[nonleaf] == tree.level[b] + 1) & (tree.parent[nonleaf] != b)]
        assert np.any(_touch(lo, hi, b, cand)), b


def test_colleagues_and_coarse(built):
    tree, pts, coords, lo, hi, ns = built
    allb = np.arange(tree.nbox)
    for b in range(tree.nbox):
        l = tree.level[b]
        same = allb[tree.level == l]
        t = same[_touch(lo, hi, b, same)]
        got = tree.colleague[b][tree.colleague[b] >= 0]
        assert sorted(got.tolist()) == sorted(t.tolist())
        for j in got:  # offset order (dx, dy[, dz]) lexicographic
            dlt = coords[j] - coords[b]
            k = 0
            for d in range(tree.dim):
                k = 3 * k + int(dlt[d]) + 1
            assert tree.colleague[b][k] == j
        if tree.leaf[b] and l > 0:
            cand = allb[(tree.level == l - 1) & (tree.leaf == 1)]
            t = cand[_touch(lo, hi, b, cand)]
            got = tree.coarse[b][: tree.ncoarse[b]]
            assert sorted(got.tolist()) == sorted(t.tolist())
        else:
            assert tree.ncoarse[b] == 0


def test_flags(built):
    tree, pts, coords, lo, hi, ns = built
    for b in range(tree.nbox):
        assert tree.fout[b] == ((not tree.leaf[b]) and tree.pcount[b] > ns)
        col = tree.colleague[b][tree.colleague[b] >= 0]
        assert tree.fin[b] == int(np.any(tree.fout[col] == 1))
        par = tree.parent[b]
        assert tree.terminal[b] == ((not tree.fout[b]) and (par < 0 or tree.fout[par]))
    # terminal boxes partition the points; tlevel is their level
    owner = np.full(tree.n, -1)
    for b in np.nonzero(tree.terminal)[0]:
        sl = slice(tree.pstart[b], tree.pstart[b] + tree.pcount[b])
        assert np.all(owner[sl] == -1)
        owner[sl] = b
        assert np.all(tree.tlevel[sl] == tree.level[b])
    assert np.all(owner >= 0)


def test_residual_lists_complete(built):
    """Every pair closer than s_{L_s(j)} is covered by the source-centric list
    of j's terminal box (colleague subtrees + coarse-neighbour leaves)."""
    tree, pts, coords, lo, hi, ns = built
    n = tree.n
    owner = np.full(n, -1)
    for b in np.nonzero(tree.terminal)[0]:
        owner[tree.pstart[b]: tree.pstart[b] + tree.pcount[b]] = b
    covered = {}
    for T in np.unique(owner):
        m = np.zeros(n, dtype=bool)
        for cb in tree.colleague[T][tree.colleague[T] >= 0]:
            m[tree.pstart[cb]: tree.pstart[cb] + tree.pcount[cb]] = True
        if tree.leaf[T]:
            for cb in tree.coarse[T][: tree.ncoarse[T]]:
                m[tree.pstart[cb]: tree.pstart[cb] + tree.pcount[cb]] = True
        covered[T] = m
    x = tree.xs
    for j in range(0, n, 3):
        T = owner[j]
        s = 2.0 ** -tree.level[T]
        r = np.linalg.norm(x - x[j], axis=1)
        near = r < s
        assert np.all(covered[T][near]), j


def test_degenerate_inputs(oracle_mod):
    # identical points: the tree stops at the depth cap
    pts = np.tile(np.array([[0.1, 0.2, 0.3]]), (30, 1))
    t = oracle_mod.Tree(pts, 10, 6)
    assert t.side == 1.0 and t.nlevels == 7
    assert t.pcount[t.level_start[6]:].max() == 30
    # empty and single-point inputs
    t0 = oracle_mod.Tree(np.zeros((0, 3)), 10)
    assert t0.nbox == 1 and t0.pcount[0] == 0
    t1 = oracle_mod.Tree(np.array([[0.5, 0.5, 0.5]]), 10)
    assert t1.nbox == 1 and t1.leaf[0] == 1
    # 2-D: identical points stop at the cap as well
    t2 = oracle_mod.Tree(np.tile(np.array([[0.1, 0.2]]), (30, 1)), 10, 5)
    assert t2.nlevels == 6 and t2.pcount[t2.level_start[5]:].max() == 30
