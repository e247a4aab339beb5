"""Writes c5_jump3d_128_boxes1024_eig.txt: the FP64 oracle's per-subdomain
results on the full-scale 3D workload (-div(k grad u) on 128^3, log10 k
uniform in [-3, 3] on 8^3 blocks, 1024 boxes, overlap 2, nev 12).

Only the oracle (oracle.schwarz) and the seeded input generators (workloads)
are called.  For every subdomain i, in the oracle's notation:
  Omega_i (Section 2)          -> n_i, |Omega_Ii| and two checksums of the
                                  ordered index list and of the layer ids
  Definition 1 splitting       -> dim K_i (reading R6)
  eq. 5 / eq. 6 (Section 3.2)  -> nev_i and the selected eigenvalues
The subdomains are spread over the host's cores (one process each, forked
after the matrix is built).

Usage:  python tests/golden/make_c5_golden.py [--procs P]
"""
import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import schwarz as OS  # noqa: E402

NAME = "c5_jump3d_128_boxes1024"
OUT = os.path.join(HERE, NAME + "_eig.txt")
_G = {}


def checksum(v):
    """Order-dependent sums of an integer list (exact in int64 at these
    sizes): sum v_k, sum (k + 1) v_k, sum (k + 1)^2 v_k."""
    v = np.asarray(v, dtype=np.int64)
    k = np.arange(1, len(v) + 1, dtype=np.int64)
    return "%d %d %d" % (v.sum(), (k * v).sum(), (k * k * v).sum())


def one(i):
    As, G, part, ov, nev = _G["As"], _G["G"], _G["part"], _G["ov"], _G["nev"]
    sub = OS.subdomains(As, np.where(part == i, 0, 1), 2, ov, G=G)[0]
    A_ii, _, At = OS.block_splitting(As, sub)
    kd = OS.kernel_dimension(At)
    res = OS.local_eigenproblem(A_ii, At, sub.n_interior, nev, kdim=kd)
    Wi = res["Z"][: sub.n_interior]
    nev_i = np.linalg.matrix_rank(Wi) if Wi.shape[1] else 0
    assert nev_i == Wi.shape[1]
    lam = res["lam_sel"]
    return (i, sub.size, sub.n_interior, checksum(sub.omega), checksum(sub.layer), kd,
            Wi.shape[1], lam.real.copy(), lam.imag.copy())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count())
    args = ap.parse_args()
    A, part, N, o = W.config(NAME)
    As = A.to_scipy()
    _G.update(As=As, G=OS.adjacency(As), part=part, ov=o["overlap"], nev=o["nev"])
    t0 = time.time()
    with mp.get_context("fork").Pool(args.procs) as pool:
        rows = []
        for k, r in enumerate(pool.imap(one, range(N), chunksize=4)):
            rows.append(r)
            if (k + 1) % 64 == 0:
                print(f"{k + 1}/{N} subdomains, {time.time() - t0:.0f} s", flush=True)
    rows.sort(key=lambda r: r[0])
    n0 = sum(r[6] for r in rows)
    with open(OUT, "w") as f:
        f.write(f"# Oracle results on {NAME}: {W.CONFIGS[NAME]['desc']}\n")
        f.write("# written by tests/golden/make_c5_golden.py (oracle.schwarz only)\n")
        f.write("# checksum(v) = sum_k v_k, sum_k (k+1) v_k, sum_k (k+1)^2 v_k (k = 0, 1, ...)\n")
        f.write("# line per subdomain: sub i n_i n_interior checksum(Omega_i) checksum(layers)"
                " dim_K nev_i\n# (three numbers per checksum), then re(lambda_1..nev_i-dim_K) and im(...)\n")
        f.write(f"n {A.n}\nnsub {N}\noverlap {o['overlap']}\nnev {o['nev']}\nn0 {n0}\n")
        for (i, ni, nI, cs_om, cs_lay, kd, nv, lr, li) in rows:
            f.write(f"sub {i} {ni} {nI} {cs_om} {cs_lay} {kd} {nv}\n")
            f.write("re " + " ".join(f"{x:.17g}" for x in lr) + "\n")
            f.write("im " + " ".join(f"{x:.17g}" for x in li) + "\n")
    print(f"wrote {OUT}: n0 {n0}, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
