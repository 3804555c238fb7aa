"""Seeded synthetic workloads shared by the tests, the smoke check and the
benchmark.  This module only draws random numbers: it holds none of the
method's arithmetic.

The paper measures only synthetic distributions (uniform points in the unit
box, points on a sphere or circle), so no dataset is involved.  Each recipe
below is a fixed draw order from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import numpy as np


def uniform_cube(n: int, seed: int):
    """Points uniform in [0,1]^3, charges uniform in [-1,1]."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    q = rng.uniform(-1.0, 1.0, n)
    return pts, q


def sphere_and_blobs(n: int, seed: int, frac_sphere: float = 0.7, nblobs: int = 3,
                     sigma: float = 1e-3):
    """Clustered 3-D set: a fraction on the unit sphere (normalised Gaussian
    vectors), the rest split evenly over Gaussian blobs of width sigma whose
    centres are uniform in [-1/2,1/2]^3; shuffled into a random input order;
    charges uniform in [-1,1]."""
    rng = np.random.default_rng(seed)
    ns = int(round(frac_sphere * n))
    g = rng.standard_normal((ns, 3))
    sph = g / np.linalg.norm(g, axis=1)[:, None]
    nb = n - ns
    centres = rng.uniform(-0.5, 0.5, (nblobs, 3))
    counts = np.full(nblobs, nb // nblobs)
    counts[: nb - counts.sum()] += 1
    blobs = np.concatenate([centres[k] + sigma * rng.standard_normal((counts[k], 3))
                            for k in range(nblobs)]) if nb else np.zeros((0, 3))
    pts = np.concatenate([sph, blobs])
    pts = pts[rng.permutation(n)]
    q = rng.uniform(-1.0, 1.0, n)
    return np.ascontiguousarray(pts), q


def two_clusters_and_background(n: int, seed: int):
    """Small adaptive case: two tight clusters plus a uniform background, so
    the tree has coarse neighbours and non-adjacent fine boxes."""
    rng = np.random.default_rng(seed)
    n1 = n // 3
    n2 = n // 3
    n3 = n - n1 - n2
    a = np.array([0.3, 0.3, 0.3]) + 2e-3 * rng.standard_normal((n1, 3))
    b = np.array([0.62, 0.55, 0.71]) + 1e-2 * rng.standard_normal((n2, 3))
    c = rng.random((n3, 3))
    pts = np.concatenate([a, b, c])[rng.permutation(n)]
    q = rng.uniform(-1.0, 1.0, n)
    return np.ascontiguousarray(pts), q


def uniform_square(n: int, seed: int):
    """Points uniform in [0,1]^2, charges uniform in [-1,1]."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    q = rng.uniform(-1.0, 1.0, n)
    return pts, q


def gaussian_2d(n: int, seed: int, sigma: float = 0.01):
    """Points 0.5 + sigma N(0, I_2), charges uniform in [-1,1]."""
    rng = np.random.default_rng(seed)
    pts = 0.5 + sigma * rng.standard_normal((n, 2))
    q = rng.uniform(-1.0, 1.0, n)
    return pts, q


def batch_2d(nprob: int, seed: int, nmin: float = 1e3, nmax: float = 2e5, scale: float = 1.0):
    """Many independent 2-D problems: problem b draws from default_rng(1000 seed + b)
    a size N_b = floor(exp(U[ln nmin, ln nmax]) * scale) (at least 1), then a
    coin for its distribution (uniform in [0,1]^2, or 0.5 + 0.01 N(0, I_2)),
    the points, and charges uniform in [-1,1].  Returns (offsets, pts, q) with
    the problems concatenated."""
    sizes, parts, charges = [], [], []
    for b in range(nprob):
        rng = np.random.default_rng(1000 * seed + b)
        nb = max(1, int(np.floor(np.exp(rng.uniform(np.log(nmin), np.log(nmax))) * scale)))
        if rng.random() < 0.5:
            p = rng.random((nb, 2))
        else:
            p = 0.5 + 0.01 * rng.standard_normal((nb, 2))
        parts.append(p)
        charges.append(rng.uniform(-1.0, 1.0, nb))
        sizes.append(nb)
    off = np.zeros(nprob + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return off, np.ascontiguousarray(np.concatenate(parts)), np.concatenate(charges)


def batch_3d(nprob: int, seed: int, nmin: float = 300, nmax: float = 6000):
    """Many independent 3-D problems: problem b draws from default_rng(1000 seed + b)
    a size N_b = floor(exp(U[ln nmin, ln nmax])) (at least 1), then one of
    three distributions with equal odds (uniform in [0,1]^3; a Gaussian blob
    0.5 + 0.05 N(0, I_3); the unit sphere, normalised Gaussian vectors), the
    points, and charges uniform in [-1,1].  Returns (offsets, pts, q)."""
    sizes, parts, charges = [], [], []
    for b in range(nprob):
        rng = np.random.default_rng(1000 * seed + b)
        nb = max(1, int(np.floor(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))))
        kind = rng.integers(3)
        if kind == 0:
            p = rng.random((nb, 3))
        elif kind == 1:
            p = 0.5 + 0.05 * rng.standard_normal((nb, 3))
        else:
            g = rng.standard_normal((nb, 3))
            p = g / np.linalg.norm(g, axis=1)[:, None]
        parts.append(p)
        charges.append(rng.uniform(-1.0, 1.0, nb))
        sizes.append(nb)
    off = np.zeros(nprob + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return off, np.ascontiguousarray(np.concatenate(parts)), np.concatenate(charges)


# Named workloads: (generator, N, seed, leaf capacity n_s).
CONFIGS = {
    "cfg1_uniform_2k": (uniform_cube, 2_000, 1, 50),
    "cfg2_uniform_1m": (uniform_cube, 1_000_000, 2, 64),
    "cfg3_clustered_10m": (sphere_and_blobs, 10_000_000, 3, 64),
}


def make(name: str, n: int | None = None):
    gen, n0, seed, ns = CONFIGS[name]
    pts, q = gen(n0 if n is None else n, seed)
    return pts, q, ns


# ------------------------------------------------------------ volume densities
def vol_gaussians(seed, n=8, smin=1e-3, smax=1e-1, box=0.3, amp=1.0):
    """n Gaussians exp(-|x - c|^2 / s^2) with s = exp(U[ln smin, ln smax]) and
    centres c ~ U[-box, box]^3, peak value amp each.  Returns (s[n], c[n,3],
    a[n])."""
    rng = np.random.default_rng(seed)
    sig = np.exp(rng.uniform(np.log(smin), np.log(smax), n))
    cen = rng.uniform(-box, box, (n, 3))
    return sig, cen, np.full(n, float(amp))


def gaussian_mixture(x, sig, cen, amp):
    """sum_i a_i exp(-|x - c_i|^2 / s_i^2) at points x[m, 3]."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(len(x))
    for s, c, a in zip(sig, cen, amp):
        out += a * np.exp(-np.sum((x - c) ** 2, axis=1) / (s * s))
    return out


def gaussian_features(sig, cen, factor=4.0):
    """Feature points (x, y, z, h) asking for boxes of side <= factor * s at
    each centre."""
    return np.hstack([np.asarray(cen, dtype=np.float64), factor * np.asarray(sig, dtype=np.float64)[:, None]])
