"""Write the oracle's reference results for the sphere kernel workload.

Runs the CPU oracle only (no GPU code).  4096 points uniform on the unit
sphere (seed 1703), kernel 1/|x - y| with diagonal 1e3, leaf 64, eta 2;
admissible blocks by the truncated SVD at eps 1e-5.  Then Z = 0 and
Z <- blocktrunc(Z + X X) with X the compressed kernel matrix (Sect. 4),
standard and accumulated, at eps 1e-5.  Stores the rank of every block of X
and of both products (pre-order, -1 if not admissible), the oracle's
operation counts, the Frobenius norm of every leaf block of each product, and
each product applied to 16 seeded Gaussian vectors (cluster order).  Takes a
few minutes; the result is committed.

    python tests/golden/make_golden_sphere.py
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

N, SEED, LEAF, ETA, DIAG, EPS = 4096, 1703, 64, 2.0, 1e3, 1e-5
NVEC, VSEED = 16, 11
NAME = "sphere_4096_mul_eps1e-5"


def leaf_norms(H, D):
    b, c = H.blocks(), H.clusters()
    out = np.zeros(len(b["kind"]))
    for i in np.nonzero(b["kind"] > 0)[0]:
        t, s = b["t"][i], b["s"][i]
        r0, nr, c0, nc = c["off"][t], c["size"][t], c["off"][s], c["size"][s]
        out[i] = np.linalg.norm(D[r0:r0 + nr, c0:c0 + nc])
    return out


def main():
    x = W.sphere_points(N, SEED)
    t = time.time()
    X = oracle.HMatrix.from_kernel(x, LEAF, ETA, DIAG, EPS)
    build_s = time.time() - t
    print(f"build {build_s:.1f}s", flush=True)
    V = W.gaussian((N, NVEC), seed=VSEED)
    arrays = {"x_rank": X.blocks()["rank"].astype(np.int16), "v": V}
    meta = {"build_seconds": build_s}
    for mode in ["standard", "accumulated"]:
        Z = X.zeros_like()
        t = time.time()
        st = Z.addmul(1.0, X, X, EPS, mode)
        dt = time.time() - t
        D = Z.to_dense()
        arrays[f"{mode}_rank"] = Z.blocks()["rank"].astype(np.int16)
        arrays[f"{mode}_zv"] = D @ V
        arrays[f"{mode}_leaf_norm"] = leaf_norms(Z, D)
        arrays[f"{mode}_norm"] = np.array([np.linalg.norm(D)])
        meta[mode] = dict(seconds=dt, stats=st)
        print(mode, f"{dt:.1f}s", st, flush=True)
    np.savez_compressed(os.path.join(HERE, NAME + ".npz"), **arrays)
    with open(os.path.join(HERE, NAME + ".json"), "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
