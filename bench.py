#!/usr/bin/env python3
"""Benchmark of the two-level Schwarz hot path on one MI355X.

Workload: 2D first-order upwind convection-diffusion on a 512 x 512 grid
(n = 262144), velocity (cos 2 pi y, sin 2 pi x), Peclet 100, 8 x 8 block
partition, overlap 2, nev = 8, right-preconditioned flexible GMRES(50) to a
relative residual of 1e-8, x0 = 0, rhs ~ N(0, 1) (seed 0).

One step = the whole hot path on that input: setup (overlap maps, Definition-1
splitting, local factorizations, local eigenproblems of eq. 5, coarse operator
and its LU) plus the FGMRES solve with the eq. 4 preconditioner.  The matrix
and right-hand side are resident in device memory before the timed region;
the partition (int32 per unknown) is a host array by interface and its upload
is timed.  The production form stores the local factors in FP32 (products
accumulated in FP64; Arnoldi, residuals and the coarse operator in FP64); the
plain FP64 form is timed beside it ("vs plain FP64").

Printed: one JSON line with the metric, the per-step time, the plain-FP64 time
and speedup, the apply kernel's roofline (algorithmic bytes / live hipEvent
duration) and the FP64 CPU oracle timed on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
WORKLOAD = "c2_convdiff2d_512_blocks64"
# measured HBM traffic of the local-solve launches (rocprofv3 FETCH_SIZE and
# WRITE_SIZE, scaled by a plain copy); valid only for the kernel sources it
# was taken with
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_local_solve_hbm_traffic.md")
KERNEL_SOURCES = ["paper_2201_02250_amd/csrc/k_apply.hip", "paper_2201_02250_amd/csrc/k_solve.h"]
COPY_BYTES = 1 << 28  # plain device copy of known size for the counter scaling


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(tile_factor):
    """Bytes per local-solve launch from the committed counter summary, or
    None if it is absent or was taken with other kernel sources or tiles."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(l.split(":", 1) for l in fh.read().splitlines() if l.startswith("- ") and ":" in l)
    except OSError:
        return None
    kv = {k[2:].strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel source hash") != kernel_source_hash():
        return None
    try:
        if abs(float(kv.get("tile factor", "nan")) - tile_factor) > 1e-12:
            return None
    except ValueError:
        return None
    try:
        return int(kv["traffic bytes per local-solve launch"])
    except (KeyError, ValueError):
        return None


def pmc_apply(reps):
    """Counter run: FP32 context on the workload, `reps` applies (direct
    launches), then three plain copies of COPY_BYTES for the scaling."""
    import torch
    import workloads as W
    from paper_2201_02250_amd import ads
    dev = torch.device("cuda:0")
    A, part, N, o = W.config(WORKLOAD)
    Ad = ads.DeviceCSR(A, dev)
    sp = torch.cuda.current_stream(dev).cuda_stream
    ctx = ads.Context(Ad, part, N, o["overlap"], o["nev"], precision=ads.ADS_PREC_FP32, stream=sp,
                      autotune=1)
    ctx.set_graphs(False)
    r = torch.randn(A.n, dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    for _ in range(reps):
        ads.ads_apply(ctx.ctx, r.data_ptr(), z.data_ptr(), 1, sp)
    torch.cuda.synchronize()
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    ctx.close()
    print("pmc_apply: %d applies, 3 copies of %d bytes, kernel source hash %s, tile factor %r"
          % (reps, COPY_BYTES, kernel_source_hash(), ctx.info["tile_factor"]), flush=True)


def apply_bytes(A, part, info, om, off, elem):
    """Algorithmic bytes of one local-solve launch and of one whole apply
    (nrhs = 1); see the design notes for the accounting."""
    import numpy as np
    S = A.to_scipy()
    rl = np.diff(S.indptr)
    nsub = info["nsub"]
    tiles = 0
    lcsr = 0
    gather = 0
    for i in range(nsub):
        ni = int(info["n_i"][i])
        s = int(info["block"][i])
        K = -(-ni // s)
        tiles += (2 * K - 1) * s * s * elem
        omega = np.sort(om[off[i]:off[i + 1]])
        sub = S[omega][:, omega]
        lcsr += sub.nnz * 12 + ni * 8
        gather += ni * (4 + 4 + 8 + 8) + int(rl[omega].sum()) * 12
    n = A.n
    local = tiles + lcsr + gather + n * 8
    n0 = info["n0"]
    nev_tot = int((info["nev_i"] * info["n_interior"]).sum())
    coarse = nev_tot * 8 * 2 + n * (4 + 8) * 2 + n0 * n0 * 8 + n * 8
    return local, local + coarse, tiles


def cpu_baseline():
    """The FP64 oracle, as it stands, on the full workload, one host thread."""
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import schwarz as OS
    A, part, N, o = W.config(WORKLOAD)
    As = A.to_scipy()
    b = W.rhs(A.n, 0)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        P = OS.TwoLevelSchwarz(As, part, N, o["overlap"], o["nev"])
        x, info = OS.gmres(As, b, P.apply, restart=o["restart"], rtol=1e-8, flexible=True)
        t = time.perf_counter() - t0
    return dict(value=round(t * 1e3, 1), unit="ms per setup+solve", cores=1, kind="oracle",
                sample="full workload, one setup+solve (oracle its %d, n0 %d)" % (info["its"], P.n0),
                host_cpus=os.cpu_count())


def profile_workload(name, steps, precision):
    """Profiling driver for the other named workloads (their own right-hand
    side count and Krylov settings): `steps` setup+solve runs, one timing line
    each on stderr, no bench line."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2201_02250_amd import ads

    dev = torch.device("cuda:0")
    A, part, N, o = W.config(name)
    if part is None:
        part = ads.ads_partition_bfs(A, o["seeds"])
    Ad = ads.DeviceCSR(A, dev)
    nrhs = o.get("nrhs", 1)
    B = torch.tensor(np.stack([W.rhs(A.n, s) for s in range(nrhs)], axis=1), device=dev)
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = ads.Context(Ad, part, N, o["overlap"], o["nev"], precision=precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, info = ctx.solve(B, restart=o["restart"], flexible=o["flexible"], rtol=1e-8)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ci = ctx.info
        ctx.close()
        print("[profile] %s step %d: setup %.1f ms solve %.1f ms its max %d status %d n0 %d "
              "tile factor %g phases %s"
              % (name, k, 1e3 * (t1 - t0), 1e3 * (t2 - t1), max(info["its"][:nrhs]), info["status"],
                 ci["n0"], ci["tile_factor"], [round(v, 2) for v in ci["t_phase_ms"][:6]]),
              file=sys.stderr, flush=True)


def config_table(with_oracle):
    """Setup and solve times of every named workload: GPU plain FP64, GPU
    mixed precision (FP32 factors; BF16 too for the 3D jumping-coefficient
    workload), GPU mixed with the learned coarse space (log-normal workload),
    and the FP64 CPU oracle on one host thread (not for the 3D
    jumping-coefficient workload, which it needs minutes for).  One JSON line per (workload, form) on stdout; GPU figures are
    medians of 3 runs after a warm-up run, each creating, solving with and
    releasing its context."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2201_02250_amd import ads
    from workloads.problems import c3b_sizes

    dev = torch.device("cuda:0")
    here = os.path.dirname(os.path.abspath(__file__))
    weights = os.path.join(here, "paper_2201_02250_amd", "gnn", "c4_lognormal_nev8.adsgnn")
    P = {"fp64": ads.ADS_PREC_FP64, "fp32": ads.ADS_PREC_FP32, "bf16": ads.ADS_PREC_BF16}

    def emit(d):
        print(json.dumps(d), flush=True)

    def gpu_rows(name, mk, Bd, restart, flex, forms):
        for form, kw in forms:
            t_set, t_sol, its, rel, n0 = [], [], 0, 0.0, 0
            for rep in range(4):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx = mk(**kw)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, info = ctx.solve(Bd, restart=restart, flexible=flex, rtol=1e-8)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                n0 = ctx.info["n0"]
                ctx.close()
                if rep == 0:
                    continue
                t_set.append(1e3 * (t1 - t0))
                t_sol.append(1e3 * (t2 - t1))
                its = max(info["its"])
                rel = max(info["relres"])
            emit({"workload": name, "form": form, "setup_ms": round(float(np.median(t_set)), 2),
                  "solve_ms": round(float(np.median(t_sol)), 2), "its": int(its),
                  "relres": float(rel), "n0": int(n0)})

    def oracle_row(name, systems, restart, flex):
        from threadpoolctl import threadpool_limits
        from oracle import schwarz as OS  # the oracle, timed as it stands
        t_set = t_sol = 0.0
        its = 0
        with threadpool_limits(1):
            for As, part, N, ov, nev, B in systems:
                t0 = time.perf_counter()
                Pc = OS.TwoLevelSchwarz(As, part, N, ov, nev)
                t1 = time.perf_counter()
                for j in range(B.shape[1]):
                    _, io = OS.gmres(As, B[:, j], Pc.apply, restart=restart, rtol=1e-8,
                                     flexible=flex)
                    its = max(its, io["its"])
                t_set += t1 - t0
                t_sol += time.perf_counter() - t1
        emit({"workload": name, "form": "oracle", "setup_ms": round(1e3 * t_set, 1),
              "solve_ms": round(1e3 * t_sol, 1), "its": int(its), "cores": 1})

    for name in ["c1_laplace2d_64_strips8", "c2_convdiff2d_512_blocks64", "c3a_convdiff3d_64_bfs256",
                 "c3b_convdiff2d_batch32", "c4_lognormal2d_256_blocks64", "c5_jump3d_128_boxes1024"]:
        if name.startswith("c3b"):
            sizes = c3b_sizes()
            As = [W.convdiff2d(m, 0.01) for m in sizes]
            parts = [W.block_partition_2d(m, max(2, round(m / 32))) for m in sizes]
            Ns = [max(2, round(m / 32)) ** 2 for m in sizes]
            b = np.concatenate([W.rhs(A.n, k) for k, A in enumerate(As)])
            Bd = torch.tensor(b, device=dev)
            ov, nev, restart, flex = 2, 10, 30, True

            def mk(**kw):
                return ads.Context(As, parts, Ns, ov, nev, **kw)

            gpu_rows(name, mk, Bd, restart, flex,
                     [("fp64", dict(precision=P["fp64"])), ("fp32", dict(precision=P["fp32"]))])
            if with_oracle:
                offs = np.cumsum([0] + [A.n for A in As])
                oracle_row(name, [(A.to_scipy(), parts[k], Ns[k], ov, nev,
                                   b[offs[k]:offs[k + 1], None]) for k, A in enumerate(As)],
                           restart, flex)
            continue
        A, part, N, o = W.config(name)
        if part is None:
            part = ads.ads_partition_bfs(A, o["seeds"])
        Ad = ads.DeviceCSR(A, dev)
        nrhs = o.get("nrhs", 1)
        B = np.stack([W.rhs(A.n, s) for s in range(nrhs)], axis=1)
        Bd = torch.tensor(B if nrhs > 1 else B[:, 0], device=dev)

        def mk(**kw):
            return ads.Context(Ad, part, N, o["overlap"], o["nev"], **kw)

        forms = [("fp64", dict(precision=P["fp64"])), ("fp32", dict(precision=P["fp32"]))]
        if name.startswith("c5"):
            forms.append(("bf16", dict(precision=P["bf16"])))
        if name.startswith("c4"):
            forms.append(("fp32+learned", dict(precision=P["fp32"], warm_start=2,
                                               gnn_weights_path=weights)))
        gpu_rows(name, mk, Bd, o["restart"], o["flexible"], forms)
        if with_oracle and not name.startswith("c5"):
            oracle_row(name, [(A.to_scipy(), part, N, o["overlap"], o["nev"], B)], o["restart"],
                       o["flexible"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--apply-reps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-apply", action="store_true",
                    help="only run applies and a plain copy (for rocprofv3 --pmc runs)")
    ap.add_argument("--config-table", action="store_true",
                    help="only time every named workload (GPU forms and the oracle); JSON lines")
    ap.add_argument("--no-oracle", action="store_true", help="with --config-table: GPU forms only")
    ap.add_argument("--profile-workload", default=None,
                    help="only run setup+solve of another named workload (profiling driver)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.pmc_apply:
        pmc_apply(args.apply_reps)
        return
    if args.config_table:
        config_table(not args.no_oracle)
        return
    if args.profile_workload:
        from paper_2201_02250_amd import ads
        precs = {"fp64": ads.ADS_PREC_FP64, "fp32": ads.ADS_PREC_FP32, "bf16": ads.ADS_PREC_BF16}
        profile_workload(args.profile_workload, args.steps, precs[args.precision])
        return

    import numpy as np
    import torch
    import workloads as W
    from paper_2201_02250_amd import ads

    dev = torch.device("cuda:0")
    A, part, N, o = W.config(WORKLOAD)
    Ad = ads.DeviceCSR(A, dev)
    b = torch.tensor(W.rhs(A.n, 0), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream
    precs = {"fp64": ads.ADS_PREC_FP64, "fp32": ads.ADS_PREC_FP32, "bf16": ads.ADS_PREC_BF16}
    prec = precs[args.precision]

    def step(p):
        # the production form tunes its tile shapes (the first, warm-up, setup
        # times the candidates; later setups of the same shape hit the cache);
        # the plain FP64 form keeps the bandwidth tiles
        # one whole job: setup, solve and release of the context (its device
        # memory goes back to the library's block cache for the next job)
        ctx = ads.Context(Ad, part, N, o["overlap"], o["nev"], precision=p, stream=sp,
                          autotune=int(p != ads.ADS_PREC_FP64))
        x, info = ctx.solve(b, restart=o["restart"], flexible=True, rtol=1e-8)
        info["ctx_info"] = ctx.info
        ctx.close()
        return x, info

    def timed(p, steps, warmup, label):
        for _ in range(warmup):
            step(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs = [step(p) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        for x, info in runs:
            assert info["status"] == 0, (label, info)
        x, info = runs[-1]
        xh, bh = x.cpu().numpy(), b.cpu().numpy()
        relres = float(np.linalg.norm(bh - A.to_scipy() @ xh) / np.linalg.norm(bh))
        ci = info["ctx_info"]
        meta = dict(its=info["its"][0], relres=relres, setup_ms=info["t_setup_ms"],
                    solve_ms=info["t_solve_ms"], phases=ci["t_phase_ms"][:8],
                    n0=ci["n0"], eig_sweeps_max=ci["eig_sweeps_max"],
                    tile_factor=ci["tile_factor"], tile_tuned=ci["tile_tuned"])
        print("[bench] %s: %.2f ms/step its %d relres %.2e" % (label, dt * 1e3, meta["its"], relres),
              file=sys.stderr, flush=True)
        return dt, meta

    t_prod, m_prod = timed(prec, args.steps, args.warmup, args.precision)
    t_fp64, m_fp64 = timed(ads.ADS_PREC_FP64, args.steps, 1, "fp64")

    # apply: live hipEvent timing of the local-solve kernel and of the whole apply
    ctx = ads.Context(Ad, part, N, o["overlap"], o["nev"], precision=prec, stream=sp, profile=1,
                      autotune=1)
    om, off, nI, lay = ads.ads_export_maps(ctx.ctx)
    r = torch.randn(A.n, dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    for _ in range(args.apply_reps):
        ads.ads_apply(ctx.ctx, r.data_ptr(), z.data_ptr(), 1, sp)
    torch.cuda.synchronize()
    info = ads.ads_get_info(ctx.ctx)
    tile_factor = info["tile_factor"]
    t_local = info["t_kernel_ms"][0] / max(info["n_kernel"][0], 1)
    t_apply = info["t_kernel_ms"][3] / max(info["n_kernel"][3], 1)
    elem = {ads.ADS_PREC_FP64: 8, ads.ADS_PREC_FP32: 4, ads.ADS_PREC_BF16: 2}[prec]
    b_local, b_apply, b_tiles = apply_bytes(A, part, info, om, off, elem)
    ctx.close()
    ach_local = b_local / (t_local * 1e-3) / 1e9
    ach_apply = b_apply / (t_apply * 1e-3) / 1e9

    out = {
        "metric": "setup+GMRES time to 1e-8 rel. residual vs plain FP64; apply HBM GB/s",
        "value": round(t_prod * 1e3, 3),
        "unit": "ms per setup+solve",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_prod * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32-factors/f64", "bf16": "bf16-factors/f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": A.n, "nnz": A.nnz, "subdomains": N,
                   "overlap": o["overlap"], "nev": o["nev"], "krylov": "FGMRES(50)", "rtol": 1e-8,
                   "precision": args.precision},
        "plain_fp64_ms": round(t_fp64 * 1e3, 3),
        "speedup_vs_plain_fp64": round(t_fp64 / t_prod, 3),
        "production": m_prod,
        "plain_fp64": m_fp64,
        "roofline": {"kernel": "k_local_fwd+k_local_bwd", "bound": "hbm",
                     "achieved": round(ach_local, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach_local / HBM_PEAK_GBS, 4), "traffic": measured_traffic(tile_factor),
                     "bytes_per_launch": int(b_local), "avg_launch_us": round(t_local * 1e3, 2),
                     "tile_factor": tile_factor},
        "apply": {"achieved_GBs": round(ach_apply, 1), "frac": round(ach_apply / HBM_PEAK_GBS, 4),
                  "bytes_per_apply": int(b_apply), "avg_us": round(t_apply * 1e3, 2),
                  "factor_tile_bytes": int(b_tiles)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
