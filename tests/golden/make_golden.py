"""Write the oracle's reference results for the full-size 3D workload.

Runs the CPU oracle only (no GPU code): H-LU of the 7-point Laplacian on the
32^3 grid (leaf 64, eta 2, eps 1e-6), standard and accumulated.  Stores, per
mode, the rank of every block (pre-order, -1 if not admissible), the oracle's
operation counts, and the values of sampled leaf blocks of the packed L\\R
factors (cluster order).  Takes tens of minutes; the result is committed.

    python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1703_09085_amd import workloads as W  # noqa: E402

DIMS, LEAF, ETA, EPS = (32, 32, 32), 64, 2.0, 1e-6
NSAMPLE = 24




def main():
    x = W.grid_points(DIMS)
    rp, ci, v = W.laplacian_csr(DIMS)
    H0 = oracle.HMatrix.from_csr(x, rp, ci, v, LEAF, ETA)
    c = H0.clusters()
    out = {}
    for mode in ["standard", "accumulated"]:
        G = H0.clone()
        t = time.time()
        st = G.lu(EPS, mode)
        dt = time.time() - t
        b = G.blocks()
        leaves = np.nonzero(b["kind"] > 0)[0]
        rng = np.random.default_rng(7)
        pick = np.sort(rng.choice(leaves, size=NSAMPLE, replace=False))
        # sampled block values: exact entries via unit-vector products with the oracle
        samples = []
        n = G.n
        for i in pick:
            t_, s_ = b["t"][i], b["s"][i]
            r0, nr = int(c["off"][t_]), int(c["size"][t_])
            c0, nc = int(c["off"][s_]), int(c["size"][s_])
            w = np.zeros((nc, nc))
            np.fill_diagonal(w, 1.0)
            vals = G.addeval_block(int(i), w, np.zeros((nr, nc)))
            samples.append(vals.ravel(order="F"))
        out[mode] = dict(seconds=dt, stats=st, rank=b["rank"].astype(np.int16), pick=pick.astype(np.int32),
                         samples=np.concatenate(samples))
        print(mode, f"{dt:.1f}s", st, flush=True)
    np.savez_compressed(os.path.join(HERE, "lap3d_32_lu_eps1e-6.npz"),
                        **{f"{m}_{k}": v for m, d in out.items() for k, v in d.items() if k != "stats"})
    with open(os.path.join(HERE, "lap3d_32_lu_eps1e-6.json"), "w") as f:
        json.dump({m: dict(seconds=d["seconds"], stats=d["stats"]) for m, d in out.items()}, f, indent=1)


if __name__ == "__main__":
    main()
