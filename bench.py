#!/usr/bin/env python3
"""Benchmark of the two-level Schwarz hot path on one MI355X.

Workload (the largest configuration that fits one GPU): 3D 7-point diffusion
-div(k grad u) on a 128^3 grid (n = 2,097,152), k constant on each of the
16^3 blocks of 8^3 nodes with log10 k uniform in [-3, 3], 1024 boxes of
16 x 16 x 8 unknowns, overlap 2, nev = 12, 16 right-hand sides ~ N(0, 1)
(seeds 0..15), right-preconditioned flexible GMRES(30) to a relative
residual of 1e-8 for every right-hand side, x0 = 0.

One step = the whole hot path on that input: setup (overlap maps,
Definition-1 splitting, local factorizations, local eigenproblems of eq. 5,
coarse operator and its inverse) plus the FGMRES solve of the 16 right-hand
sides with the eq. 4 preconditioner, then the release of the context.  The
matrix and right-hand sides are resident in device memory before the timed
region; the partition (int32 per unknown) is a host array by interface and
its upload is timed.  The production form stores the local factors in FP32
(Arnoldi, residuals and the coarse operator stay FP64); the plain FP64 form
is timed beside it, both with its own eigensolver tolerance (1e-10) and with
the production form's (1e-3), which separates the gain of the precision from
that of the tolerance.

Printed: one JSON line with the metric, the per-step time, the plain-FP64
times and speedups, the roofline of the dominant kernel (the matrix-core
Gauss-Jordan update of the setup's dense inversions: algorithmic flops over
its hipEvent-timed launches inside the timed steps), the local solve's HBM
rate, and the FP64 CPU oracle on a stated sample of the workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
FP64_MFMA_PEAK_TF = 78.6   # MI355X dense FP64 matrix-core peak, TFLOP/s
WORKLOAD = "c5_jump3d_128_boxes1024"
SECONDARY = "c2_convdiff2d_512_blocks64"
METRIC = "setup+GMRES time to 1e-8 rel. residual vs plain FP64; apply HBM GB/s"
# measured HBM traffic of the matrix-core update launches (rocprofv3
# FETCH_SIZE and WRITE_SIZE, scaled by a plain copy); valid only for the
# kernel sources it was taken with
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gj_update_mfma_c5_hbm_traffic.md")
KERNEL_SOURCES = ["paper_2201_02250_amd/csrc/k_gj.h"]
COPY_BYTES = 1 << 28  # plain device copy of known size for the counter scaling
HOST_CORES = 16       # host cores that the oracle baseline may use (the GPU's CPU share)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per matrix-core update launch from the committed counter
    summary, or None if it is absent or was taken with other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    kv = {}
    for l in lines:
        if l.startswith("- ") and ":" in l:
            k, v = l[2:].split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel source hash") != kernel_source_hash():
        return None
    try:
        return int(kv["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def rhs_block(n, nrhs):
    import numpy as np
    import workloads as W
    return np.stack([W.rhs(n, s) for s in range(nrhs)], axis=1)


def pmc_setup():
    """Counter run: one FP32-factor setup of the workload (its matrix-core
    update launches), then three plain copies of COPY_BYTES for the scaling."""
    import torch
    import workloads as W
    from paper_2201_02250_amd import ads
    dev = torch.device("cuda:0")
    A, part, N, o = W.config(WORKLOAD)
    Ad = ads.DeviceCSR(A, dev)
    sp = torch.cuda.current_stream(dev).cuda_stream
    ctx = ads.Context(Ad, part, N, o["overlap"], o["nev"], precision=ads.ADS_PREC_FP32, stream=sp)
    torch.cuda.synchronize()
    ctx.close()
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("pmc_setup: one setup, 3 copies of %d bytes, kernel source hash %s"
          % (COPY_BYTES, kernel_source_hash()), flush=True)


def local_solve_bytes(A, info, om, off, elem, nrhs):
    """Algorithmic bytes of one local solve over every subdomain for nrhs
    right-hand sides: the factor tiles once ((2K - 1) s^2 entries of elem
    bytes per subdomain), the local CSR once, and per right-hand side the
    gathers of r, q and the rows of A for t = r - A q, the padded work
    vector (written and read) and the owner scatter."""
    import numpy as np
    S = A.to_scipy()
    rl = np.diff(S.indptr)
    tiles = lcsr = vec = 0
    for i in range(info["nsub"]):
        ni = int(info["n_i"][i])
        s = int(info["block"][i])
        K = -(-ni // s)
        tiles += (2 * K - 1) * s * s * elem
        omega = om[off[i]:off[i + 1]]
        lcsr += int(rl[omega].sum()) * 12 + ni * 12
        vec += nrhs * (ni * (8 + 8 + 8 + 8) + int(rl[omega].sum()) * 8 + int(info["n_interior"][i]) * 8)
    return tiles + lcsr + vec, tiles


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for l in f:
                if l.startswith("model name"):
                    return l.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_CPU = {}


def _oracle_subdomain(i):
    """The oracle's per-subdomain setup (Omega_i, Definition 1, sparse LU of
    A_ii, eq. 5) and one local solve, wall times measured in the worker."""
    import numpy as np
    import scipy.sparse.linalg as spla
    from oracle import schwarz as OS
    As, G, part, ov, nev = _CPU["As"], _CPU["G"], _CPU["part"], _CPU["ov"], _CPU["nev"]
    t0 = time.perf_counter()
    sub = OS.subdomains(As, np.where(part == i, 0, 1), 2, ov, G=G)[0]
    A_ii, _, At = OS.block_splitting(As, sub)
    lu = spla.splu(A_ii.tocsc())
    OS.local_eigenproblem(A_ii, At, sub.n_interior, nev, kdim=OS.kernel_dimension(At))
    t1 = time.perf_counter()
    lu.solve(np.ones(sub.size))
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def cpu_sample():
    """The FP64 oracle as it stands, on a bounded sample of the workload,
    over all host cores (run before the GPU is initialised, so that the
    process pool can fork): the per-subdomain setup (Omega_i, splitting,
    SuperLU, ARPACK) and one local solve of 32 of the 1024 subdomains in a
    process pool; the dense LU of an order n0 = nev * 1024 coarse matrix
    (LAPACK, all threads) and one solve with it, timed whole."""
    import multiprocessing as mp
    import numpy as np
    import scipy.linalg as sla
    import workloads as W
    from oracle import schwarz as OS
    try:
        from threadpoolctl import threadpool_info
        blas = ",".join(sorted({d.get("internal_api", "?") + ":" + d.get("version", "?")
                                for d in threadpool_info() if d.get("user_api") == "blas"}))
    except Exception:
        blas = "unknown"
    ncpu = min(os.cpu_count() or 1, HOST_CORES)
    A, part, N, o = W.config(WORKLOAD)
    As = A.to_scipy()
    _CPU.update(As=As, G=OS.adjacency(As), part=part, ov=o["overlap"], nev=o["nev"])
    sample = list(range(0, N, N // 32))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(ncpu) as pool:
        res = pool.map(_oracle_subdomain, sample, chunksize=1)
    t_pool = time.perf_counter() - t0
    _CPU.clear()
    n0 = o["nev"] * N
    rng = np.random.default_rng(0)
    E = rng.standard_normal((n0, n0)) + n0 * np.eye(n0)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(ncpu):
        t1 = time.perf_counter()
        lu = sla.lu_factor(E, overwrite_a=True, check_finite=False)
        t_lu = time.perf_counter() - t1
        c = rng.standard_normal(n0)
        t2 = time.perf_counter()
        sla.lu_solve(lu, c, check_finite=False)
        t_cs = time.perf_counter() - t2
    del E, lu
    return dict(N=N, nsample=len(sample), ncpu=ncpu, n0=n0, t_pool=t_pool,
                t_set=sum(r[0] for r in res) * N / len(sample) / ncpu,
                t_sol=sum(r[1] for r in res) * N / len(sample) / ncpu, t_lu=t_lu, t_cs=t_cs,
                blas=blas)


def cpu_baseline(smp, its, nrhs):
    """Setup + solve of the whole workload by the oracle, from the sample:
    the sampled per-subdomain setup scaled to all subdomains and divided by
    the pool size, the coarse LU, and the FGMRES solve as its iterations x
    right-hand sides applies, each the scaled local solves plus a coarse
    solve."""
    total = smp["t_set"] + smp["t_lu"] + its * nrhs * (smp["t_sol"] + smp["t_cs"])
    N, ns, nc = smp["N"], smp["nsample"], smp["ncpu"]
    return dict(value=round(total * 1e3, 1), unit="ms per setup+solve", cores=nc, kind="oracle",
                sample=("setup of %d of %d subdomains (every %dth) in a %d-process pool, scaled "
                        "x%d / %d processes: %.1f s; dense LU of an order-%d coarse matrix: %.1f s; "
                        "solve = %d iterations x %d rhs x (%d local LU solves, scaled the same way, "
                        "+ one coarse LU solve)"
                        % (ns, N, N // ns, nc, N // ns, nc, smp["t_set"], smp["n0"], smp["t_lu"], its,
                           nrhs, N)),
                wall_s=round(smp["t_pool"] + smp["t_lu"] + smp["t_cs"], 1), cpu_model=cpu_model(),
                blas=smp["blas"])


def profile_workload(name, steps, precision):
    """Profiling driver for the named workloads (their own right-hand side
    count and Krylov settings): `steps` setup+solve runs, one timing line
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
    B = torch.tensor(rhs_block(A.n, nrhs), device=dev)
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
    mixed precision (FP32 factors; BF16 where it is accepted), GPU mixed
    with the learned coarse space (log-normal workload), and the FP64 CPU
    oracle on one host thread (not for the 3D jumping-coefficient workload,
    which it needs minutes for).  One JSON line per (workload, form) on
    stdout; GPU figures are medians of 3 runs after a warm-up run, each
    creating, solving with and releasing its context."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2201_02250_amd import ads
    from workloads.problems import c3b_sizes

    dev = torch.device("cuda:0")
    weights = os.path.join(ROOT, "paper_2201_02250_amd", "gnn", "c4_lognormal_nev8.adsgnn")
    P = {"fp64": ads.ADS_PREC_FP64, "fp32": ads.ADS_PREC_FP32, "bf16": ads.ADS_PREC_BF16}

    def emit(d):
        print(json.dumps(d), flush=True)

    def gpu_rows(name, mk, Bd, restart, flex, forms):
        for form, kw in forms:
            t_set, t_sol, its, rel, n0 = [], [], 0, 0.0, 0
            try:
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
            except ads.AdsError as e:
                emit({"workload": name, "form": form, "refused": str(e)})
                continue
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
        B = rhs_block(A.n, nrhs)
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


def secondary_c2(steps):
    """The 2D convection-diffusion workload (512^2, 64 blocks, one
    right-hand side, FGMRES(50)): production and plain FP64 setup+solve."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2201_02250_amd import ads
    dev = torch.device("cuda:0")
    A, part, N, o = W.config(SECONDARY)
    Ad = ads.DeviceCSR(A, dev)
    b = torch.tensor(W.rhs(A.n, 0), dtype=torch.float64, device=dev)
    sp = torch.cuda.current_stream(dev).cuda_stream
    out = {}
    for label, prec in (("fp32", ads.ADS_PREC_FP32), ("fp64", ads.ADS_PREC_FP64)):
        def step():
            ctx = ads.Context(Ad, part, N, o["overlap"], o["nev"], precision=prec, stream=sp,
                              autotune=int(prec != ads.ADS_PREC_FP64))
            _, info = ctx.solve(b, restart=o["restart"], flexible=True, rtol=1e-8)
            ctx.close()
            return info
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [step() for _ in range(steps)]
        torch.cuda.synchronize()
        out[label + "_ms"] = round((time.perf_counter() - t0) / steps * 1e3, 3)
        out[label + "_its"] = infos[-1]["its"][0]
        assert all(i["status"] == 0 for i in infos), infos[-1]
    out["workload"] = SECONDARY
    out["speedup_vs_plain_fp64"] = round(out["fp64_ms"] / out["fp32_ms"], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--apply-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--pmc-setup", action="store_true",
                    help="only run one setup and a plain copy (for rocprofv3 --pmc runs)")
    ap.add_argument("--config-table", action="store_true",
                    help="only time every named workload (GPU forms and the oracle); JSON lines")
    ap.add_argument("--no-oracle", action="store_true", help="with --config-table: GPU forms only")
    ap.add_argument("--profile-workload", default=None,
                    help="only run setup+solve of a named workload (profiling driver)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.pmc_setup:
        pmc_setup()
        return
    if args.config_table:
        config_table(not args.no_oracle)
        return
    if args.profile_workload:
        from paper_2201_02250_amd import ads
        precs = {"fp64": ads.ADS_PREC_FP64, "fp32": ads.ADS_PREC_FP32, "bf16": ads.ADS_PREC_BF16}
        profile_workload(args.profile_workload, args.steps, precs[args.precision])
        return

    smp = None if args.no_cpu_baseline else cpu_sample()  # before the GPU is touched

    import numpy as np
    import torch
    import workloads as W
    from paper_2201_02250_amd import ads

    dev = torch.device("cuda:0")
    A, part, N, o = W.config(WORKLOAD)
    nrhs = o["nrhs"]
    Ad = ads.DeviceCSR(A, dev)
    Bh = rhs_block(A.n, nrhs)
    Bd = torch.tensor(Bh, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream
    precs = {"fp64": ads.ADS_PREC_FP64, "fp32": ads.ADS_PREC_FP32, "bf16": ads.ADS_PREC_BF16}
    prec = precs[args.precision]
    As = A.to_scipy()

    def step(p, eig_tol=0.0, profile=0):
        # one whole job: setup, solve of the 16 right-hand sides and release
        # of the context (its device memory goes back to the library's cache)
        ctx = ads.Context(Ad, part, N, o["overlap"], o["nev"], precision=p, stream=sp,
                          eig_tol=eig_tol, profile=profile)
        x, info = ctx.solve(Bd, restart=o["restart"], flexible=True, rtol=1e-8)
        info["ctx_info"] = ctx.info if not profile else ads.ads_get_info(ctx.ctx)
        ctx.close()
        return x, info

    def timed(p, steps, warmup, label, eig_tol=0.0, profile=0):
        for _ in range(warmup):
            step(p, eig_tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs = [step(p, eig_tol, profile) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        for x, info in runs:
            assert info["status"] == 0, (label, info["statuses"])
        x, info = runs[-1]
        X = x.cpu().numpy()
        relres = float((np.linalg.norm(Bh - As @ X, axis=0) / np.linalg.norm(Bh, axis=0)).max())
        ci = info["ctx_info"]
        meta = dict(its_max=max(info["its"][:nrhs]), relres_max=relres,
                    setup_ms=round(info["t_setup_ms"], 3), solve_ms=round(info["t_solve_ms"], 3),
                    phases=[round(v, 3) for v in ci["t_phase_ms"][:8]], n0=ci["n0"],
                    eig_sweeps_max=ci["eig_sweeps_max"], eig_tol=eig_tol or None)
        print("[bench] %s: %.2f ms/step its %d relres %.2e" % (label, dt * 1e3, meta["its_max"], relres),
              file=sys.stderr, flush=True)
        return dt, meta, runs

    # production form; the matrix-core updates of every timed setup are timed
    # with hipEvents on the stream they run on (profile bit 1: no effect on
    # the launches or graphs)
    t_prod, m_prod, runs = timed(prec, args.steps, args.warmup, args.precision, profile=2)
    mf_ms = sum(r[1]["ctx_info"]["t_mfma_update_ms"] for r in runs)
    mf_n = sum(r[1]["ctx_info"]["n_mfma_update"] for r in runs)
    mf_flops = sum(r[1]["ctx_info"]["mfma_update_flops"] for r in runs)
    del runs
    fp64_steps = max(1, min(args.steps, 2))
    t_fp64, m_fp64, _ = timed(ads.ADS_PREC_FP64, fp64_steps, 1, "fp64")
    t_fp64t, m_fp64t, _ = timed(ads.ADS_PREC_FP64, fp64_steps, 1, "fp64 eig_tol 1e-3", eig_tol=1e-3)

    # the local solve (apply kernel) with 16 right-hand sides, hipEvent-timed
    ctx = ads.Context(Ad, part, N, o["overlap"], o["nev"], precision=prec, stream=sp, profile=1)
    om, off, nI, lay = ads.ads_export_maps(ctx.ctx)
    info = ads.ads_get_info(ctx.ctx)
    om_sorted = [np.sort(om[off[i]:off[i + 1]]) for i in range(N)]
    omc = np.concatenate(om_sorted)
    offc = np.concatenate([[0], np.cumsum([len(v) for v in om_sorted])])
    for _ in range(args.apply_reps):
        ctx.apply(Bd)
    torch.cuda.synchronize()
    info = ads.ads_get_info(ctx.ctx)
    ctx.close()
    t_local = info["t_kernel_ms"][0] / max(info["n_kernel"][0], 1)
    elem = {ads.ADS_PREC_FP64: 8, ads.ADS_PREC_FP32: 4, ads.ADS_PREC_BF16: 2}[prec]
    b_local, b_tiles = local_solve_bytes(A, info, omc, offc, elem, nrhs)
    ach_local = b_local / (t_local * 1e-3) / 1e9

    mf_tf = mf_flops / (mf_ms * 1e-3) / 1e12 if mf_ms > 0 else 0.0
    out = {
        "metric": METRIC,
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
                   "overlap": o["overlap"], "nev": o["nev"], "nrhs": nrhs, "krylov": "FGMRES(30)",
                   "rtol": 1e-8, "precision": args.precision},
        "plain_fp64_ms": round(t_fp64 * 1e3, 3),
        "speedup_vs_plain_fp64": round(t_fp64 / t_prod, 3),
        "plain_fp64_same_eig_tol_ms": round(t_fp64t * 1e3, 3),
        "speedup_from_precision": round(t_fp64t / t_prod, 3),
        "speedup_from_eig_tol": round(t_fp64 / t_fp64t, 3),
        "production": m_prod,
        "plain_fp64": m_fp64,
        "plain_fp64_same_eig_tol": m_fp64t,
        "roofline": {"kernel": "k_gj_update_mfma", "bound": "mfma", "achieved": round(mf_tf, 2),
                     "peak": FP64_MFMA_PEAK_TF, "unit": "TFLOP/s",
                     "frac": round(mf_tf / FP64_MFMA_PEAK_TF, 4), "traffic": measured_traffic(),
                     "flops_per_launch": round(mf_flops / max(mf_n, 1)),
                     "avg_launch_us": round(mf_ms * 1e3 / max(mf_n, 1), 2), "launches": mf_n,
                     "dtype": "f64"},
        "apply": {"kernel": "k_local_solve", "nrhs": nrhs, "achieved_GBs": round(ach_local, 1),
                  "frac": round(ach_local / HBM_PEAK_GBS, 4), "bytes_per_launch": int(b_local),
                  "factor_tile_bytes": int(b_tiles), "avg_us": round(t_local * 1e3, 2)},
    }
    if not args.no_secondary:
        out["secondary"] = secondary_c2(10)
    if smp is not None:
        out["cpu_baseline"] = cpu_baseline(smp, m_prod["its_max"], nrhs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
