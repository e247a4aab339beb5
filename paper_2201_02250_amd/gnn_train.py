"""Training and evaluation of the learned warm start on the log-normal
diffusion workload (2D -div(k grad u), 256 x 256, k = exp(2 g) with g a
unit Gaussian field of correlation length 0.05, 8 x 8 blocks, overlap 1,
nev 8).

Data: the fields of numpy generator seeds 0 .. fields + val - 1 (the
workload's own recipe); for every one the exact method itself (FP64 setup on
the GPU) computes the coarse space W_i of every subdomain; the targets are
those blocks and the inputs the subdomain graphs with their node features
(ads_gnn_graph_build).  Training: Adam on the projection loss, one field (64
subdomain graphs) per step, with the library's forward and backward kernels.
Evaluation on held-out fields (seeds from 100000): GMRES(30) iterations to
1e-8 with the exact coarse space, with the learned coarse space
(warm_start = 2) and without a coarse space (RAS), and the eigensolver work
(block steps or sweeps, and time) of the warm-started exact eigensolve
(warm_start = 1) against the cold one, for Krylov-Schur (the default) and
the block subspace iteration.

    python -m paper_2201_02250_amd.gnn_train --fields 2000 --epochs 8 \
        --eval 200 --out paper_2201_02250_amd/gnn/c4_lognormal_nev8.adsgnn

Orchestration only: every arithmetic step runs in the library's kernels.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "c4_lognormal2d_256_blocks64"
NZ = 8  # target columns (nev)


def field_csr(n, indptr, indices, data):
    """A device CSR (ads.DeviceCSR) with the fixed pattern and one field's values."""
    from paper_2201_02250_amd import ads
    A = ads.DeviceCSR.__new__(ads.DeviceCSR)
    A.n, A.nnz = n, int(indices.numel())
    A.indptr, A.indices, A.data = indptr, indices, data
    return A


def log(msg):
    print(msg, flush=True)


def make_data(seeds, pattern, part, N, opts, stream):
    """Per field: node features, edge weights and targets (device tensors);
    the graph structure (the same for every field) from the first one."""
    import torch
    from paper_2201_02250_amd import ads
    from paper_2201_02250_amd import gnn as G
    import workloads as W
    indptr, indices, n, m = pattern
    out, struct = [], None
    for k, s in enumerate(seeds):
        Ah = W.config(WORKLOAD, seed=s)[0]  # same pattern for every seed
        vals = torch.tensor(Ah.data, dtype=torch.float64, device=indptr.device)
        A = field_csr(n, indptr, indices, vals)
        ctx = ads.Context(A, part, N, opts["overlap"], opts["nev"], stream=stream)
        g = G.Graph.from_context(ctx, stream)
        Z = G.targets(ctx, NZ, stream)
        if struct is None:
            struct = (g.node_off, g.row_ptr, g.col, g.mask)
        out.append((g.feat, g.w, Z))
        ctx.close()
        if (k + 1) % 200 == 0:
            torch.cuda.synchronize()
            log(f"[data] {k + 1} fields")
    return struct, out


def graph_of(struct, item):
    from paper_2201_02250_amd import gnn as G
    node_off, row_ptr, col, mask = struct
    feat, w, _ = item
    return G.Graph(node_off, row_ptr, col, w, feat, mask)


def mean_loss(net, struct, data):
    import torch
    tot = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    for item in data:
        g = graph_of(struct, item)
        X = net.forward(g)
        L, _ = net.loss(g, X, item[2])
        tot += L
    return float(tot.item()) / max(len(data), 1)


def train(args):
    import torch
    from paper_2201_02250_amd import ads
    from paper_2201_02250_amd import gnn as G
    import workloads as W
    dev = torch.device("cuda:0")
    A0, part, N, opts = W.config(WORKLOAD)
    m = int(round(np.sqrt(A0.n)))
    indptr = torch.tensor(A0.indptr, dtype=torch.int64, device=dev)
    indices = torch.tensor(A0.indices, dtype=torch.int32, device=dev)
    pattern = (indptr, indices, A0.n, m)
    stream = torch.cuda.current_stream(dev).cuda_stream
    t0 = time.perf_counter()
    seeds = list(range(args.fields + args.val))
    struct, data = make_data(seeds, pattern, part, N, opts, stream)
    train_d, val_d = data[:args.fields], data[args.fields:]
    torch.cuda.synchronize()
    log(f"[data] {len(train_d)} training and {len(val_d)} validation fields in "
        f"{time.perf_counter() - t0:.1f} s")
    shape = G.DEFAULT_SHAPE
    net = G.Net(shape, G.init_params(shape, seed=args.seed), stream)
    rng = np.random.default_rng(args.seed)
    log(f"[train] epoch 0 validation loss {mean_loss(net, struct, val_d):.4f}")
    step = 0
    total_steps = args.epochs * len(train_d)
    for ep in range(args.epochs):
        t1 = time.perf_counter()
        acc = torch.zeros(1, dtype=torch.float64, device=dev)
        for idx in rng.permutation(len(train_d)):
            item = train_d[idx]
            g = graph_of(struct, item)
            X = net.forward(g)
            L, dX = net.loss(g, X, item[2])
            acc += L
            net.grad.zero_()
            net.backward(g, dX)
            # cosine decay of the learning rate
            lr = args.lr * 0.5 * (1.0 + np.cos(np.pi * step / total_steps))
            net.adam(lr)
            step += 1
        tl = float(acc.item()) / len(train_d)
        vl = mean_loss(net, struct, val_d)
        log(f"[train] epoch {ep + 1} train loss {tl:.4f} validation loss {vl:.4f} "
            f"({time.perf_counter() - t1:.1f} s)")
    master = net.master.cpu().numpy()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    G.save_weights(args.out, shape, master)
    log(f"[train] weights written to {args.out}")
    return args.out


def evaluate(weights, fields, first_seed=100000, precision=0):
    """GMRES iterations and eigensolver work on held-out fields (numpy
    generator seeds, disjoint from the training sample)."""
    import torch
    from paper_2201_02250_amd import ads
    import workloads as W
    dev = torch.device("cuda:0")
    log(f"[eval] precision {['fp64', 'fp32', 'bf16'][precision]}")
    rows = []
    for k in range(fields):
        A, part, N, o = W.config(WORKLOAD, seed=first_seed + k)
        Ad = ads.DeviceCSR(A, dev)
        b = torch.tensor(W.rhs(A.n, k), device=dev)
        res = {}
        for label, kw in [("exact", dict()), ("learned", dict(warm_start=2)),
                          ("ras", dict(variant=ads.ADS_VARIANT_RAS)),
                          ("warm", dict(warm_start=1)),
                          ("cold_subspace", dict(eig_solver=ads.ADS_EIG_SUBSPACE)),
                          ("warm_subspace", dict(warm_start=1, eig_solver=ads.ADS_EIG_SUBSPACE))]:
            ctx = ads.Context(Ad, part, N, o["overlap"], o["nev"], gnn_weights_path=weights,
                              precision=precision, **kw)
            x, info = ctx.solve(b, restart=o["restart"], rtol=1e-8)
            res[label] = dict(its=info["its"][0], status=info["status"],
                              sweeps=int(ctx.info["eig_sweeps_max"]),
                              fallbacks=int(ctx.info["eig_fallbacks"]),
                              eig_ms=ctx.info["t_phase_ms"][3], gnn_ms=ctx.info["t_phase_ms"][6])
            ctx.close()
        rows.append(res)
        if k < 5 or (k + 1) % 20 == 0:
            log(f"[eval] field {k}: " + ", ".join(f"{l} its {r['its']}" for l, r in res.items()) +
                f"; Krylov-Schur block steps cold {res['exact']['sweeps']} warm "
                f"{res['warm']['sweeps']}; subspace sweeps cold {res['cold_subspace']['sweeps']} "
                f"warm {res['warm_subspace']['sweeps']}")
    summ = {l: dict(its=float(np.mean([r[l]["its"] for r in rows])),
                    its_max=int(np.max([r[l]["its"] for r in rows])),
                    sweeps=float(np.mean([r[l]["sweeps"] for r in rows])),
                    fallbacks=int(np.sum([r[l]["fallbacks"] for r in rows])),
                    eig_ms=float(np.mean([r[l]["eig_ms"] for r in rows])),
                    gnn_ms=float(np.mean([r[l]["gnn_ms"] for r in rows])))
            for l in rows[0]}
    log("[eval] mean over %d held-out fields: %s" % (fields, json.dumps(summ)))
    return summ


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fields", type=int, default=2000)
    ap.add_argument("--val", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval", type=int, default=20)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2201_02250_amd", "gnn",
                                                  "c4_lognormal_nev8.adsgnn"))
    ap.add_argument("--eval-only", action="store_true")
    args = ap.parse_args()
    w = args.out if args.eval_only else train(args)
    if args.eval > 0:
        for prec in (0, 1):
            evaluate(w, args.eval, precision=prec)


if __name__ == "__main__":
    main()
