"""Writes cfg3_oracle_2000.txt: the FP64 oracle's potential, far part and
near part of the 10^7-point clustered workload (dmk_inputs "cfg3_clustered_10m":
seed 3, 70 % on the unit sphere, 30 % in three Gaussian blobs of width 1e-3,
charges U[-1, 1], leaf capacity 64, tol 1e-6) at 2,000 targets drawn with
numpy default_rng(11), the sample the full-size GPU test uses.  Calls only
the oracle (about 7 minutes and 31 GB on 8 host threads).

    python tests/golden/make_cfg3_oracle.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import dmk_inputs  # noqa: E402
import oracle  # noqa: E402

NSAMPLE = 2000


def main():
    pts, q, ns = dmk_inputs.make("cfg3_clustered_10m")
    n = len(q)
    sidx = np.random.default_rng(11).choice(n, NSAMPLE, replace=False)
    tr = oracle.Tree(pts, ns)
    pr = oracle.params_for(1e-6)
    res = oracle.dmk_eval(tr, pr, oracle.PSWF(pr.c), q)
    scale = 1.0 / (4 * np.pi * tr.side)
    far = np.empty(n)
    near = np.empty(n)
    far[tr.perm] = res["ufar"] * scale
    near[tr.perm] = res["ures"] * scale
    with open(os.path.join(HERE, "cfg3_oracle_2000.txt"), "w") as f:
        f.write("# FP64 oracle DMK (tol 1e-6, Table 1 parameters) on the 10^7-point clustered workload,\n")
        f.write("# written by tests/golden/make_cfg3_oracle.py (oracle only); targets from default_rng(11).\n")
        f.write(f"# tree: {tr.nbox} boxes, {tr.nlevels} levels; oracle threads {oracle.num_threads()}\n")
        f.write("# columns: input index, potential, far part, near part\n")
        for i in sidx:
            f.write(f"{int(i)} {res['u'][i]:.17e} {far[i]:.17e} {near[i]:.17e}\n")


if __name__ == "__main__":
    main()
