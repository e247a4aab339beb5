"""ctypes binding of the ads C interface (include/ads.h).

Argument marshalling only: every computational step runs in the library's HIP
kernels.  The functions keep the C names; `Context` is a small convenience
wrapper used by the tests and the benchmark.  Device buffers are passed as raw
pointers (for example torch tensors' data_ptr()); host arrays as numpy arrays.
Loading fails loudly when the shared library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libads.so")

ADS_ABI_VERSION = 5
ADS_MAX_RESULTS = 64
ADS_OK, ADS_KSP_MAXIT, ADS_KSP_BREAKDOWN = 0, 1, 2
ADS_ERR_ARG, ADS_ERR_HIP, ADS_ERR_OOM, ADS_ERR_SINGULAR = -1, -2, -3, -4
ADS_ERR_EIG_NOCONV, ADS_ERR_NAN, ADS_ERR_UNSUPPORTED = -5, -6, -7
ADS_VARIANT_DEFLATED, ADS_VARIANT_RAS, ADS_VARIANT_ASM, ADS_VARIANT_ADDITIVE, ADS_VARIANT_ADDITIVE_RAS = 0, 1, 2, 3, 4
ADS_PREC_FP64, ADS_PREC_FP32, ADS_PREC_BF16 = 0, 1, 2
ADS_EIG_KRYLOV_SCHUR, ADS_EIG_SUBSPACE = 0, 1

# every symbol declared in include/ads.h
SYMBOLS = ["ads_setup", "ads_setup_batched", "ads_setup_complex", "ads_apply", "ads_apply_noalloc", "ads_solve",
           "ads_get_info",
           "ads_export_maps", "ads_export_splitting", "ads_export_coarse", "ads_partition_bfs",
           "ads_set_graphs", "ads_destroy", "ads_status_string", "ads_last_error",
           "ads_gnn_nparams", "ads_gnn_workspace_floats", "ads_gnn_graph_size",
           "ads_gnn_graph_build", "ads_gnn_targets", "ads_gnn_forward", "ads_gnn_loss",
           "ads_gnn_backward", "ads_gnn_adam", "ads_gnn_round_bf16", "ads_tune_cache_save",
           "ads_tune_cache_load", "ads_tune_cache_clear"]


class ads_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("on_device", C.c_int32)]


class ads_options(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("overlap", C.c_int32), ("nev", C.c_int32),
                ("tau", C.c_double), ("variant", C.c_int32), ("precision", C.c_int32),
                ("warm_start", C.c_int32), ("eig_tol", C.c_double), ("eig_max_sweeps", C.c_int32),
                ("gnn_weights_path", C.c_char_p), ("profile", C.c_int32),
                ("eig_solver", C.c_int32), ("autotune", C.c_int32)]


class ads_gnn_shape(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("width", C.c_int32), ("layers", C.c_int32),
                ("n_out", C.c_int32)]


class ads_gnn_graph(C.Structure):
    _fields_ = [("ngraph", C.c_int32), ("nnode", C.c_int64), ("node_off", C.c_void_p),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("w", C.c_void_p),
                ("feat", C.c_void_p), ("mask", C.c_void_p)]


ADS_GNN_FEATURES = 16


class ads_ksp_options(C.Structure):
    _fields_ = [("restart", C.c_int32), ("flexible", C.c_int32), ("rtol", C.c_double),
                ("maxit", C.c_int32), ("fixed_iters", C.c_int32)]


class ads_ksp_result(C.Structure):
    _fields_ = [("its", C.c_int32 * ADS_MAX_RESULTS), ("relres", C.c_double * ADS_MAX_RESULTS),
                ("status", C.c_int32 * ADS_MAX_RESULTS), ("t_setup_ms", C.c_double),
                ("t_solve_ms", C.c_double)]


class ads_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("omega_total", C.c_int64), ("factor_bytes", C.c_int64),
                ("nsys", C.c_int32), ("nsub", C.c_int32), ("n0", C.c_int32),
                ("eig_sweeps_max", C.c_int32), ("eig_unconverged", C.c_int32),
                ("eig_fallbacks", C.c_int32), ("t_phase_ms", C.c_double * 8),
                ("t_kernel_ms", C.c_double * 4), ("n_kernel", C.c_int64 * 4),
                ("nev_i", C.c_void_p), ("kernel_dim", C.c_void_p), ("n_i", C.c_void_p),
                ("n_interior", C.c_void_p), ("sweeps", C.c_void_p), ("block", C.c_void_p),
                ("eig_resid", C.c_void_p), ("eig_solver", C.c_int32),
                ("tile_factor", C.c_double), ("tile_tuned", C.c_int32),
                ("t_mfma_update_ms", C.c_double), ("n_mfma_update", C.c_int64),
                ("mfma_update_flops", C.c_double), ("local_resid", C.c_double),
                ("is_complex", C.c_int32)]


class DeviceCSR:
    """CSR already resident in device memory (torch tensors on a GPU)."""

    def __init__(self, A, device="cuda:0"):
        import torch
        self.n = A.n
        self.nnz = A.nnz
        self.indptr = torch.tensor(np.asarray(A.indptr, np.int64), device=device)
        self.indices = torch.tensor(np.asarray(A.indices, np.int32), device=device)
        self.data = torch.tensor(np.asarray(A.data, np.float64), device=device)


_lib = None


def lib():
    """Load libads.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # torch ships its own HIP and HSA runtimes under the same sonames as
        # the system's: loading torch first makes the library bind to the
        # runtime that torch's tensors live in (one runtime per process);
        # loaded the other way round, torch finds no GPU
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.ads_setup.argtypes = [C.POINTER(ads_csr), P, I32, C.POINTER(ads_options), P, C.POINTER(P)]
        L.ads_setup_batched.argtypes = [I32, C.POINTER(ads_csr), P, P, C.POINTER(ads_options), P,
                                        C.POINTER(P)]
        L.ads_setup_complex.argtypes = [I32, C.POINTER(ads_csr), P, P, C.POINTER(ads_options), P,
                                        C.POINTER(P)]
        L.ads_apply.argtypes = [P, P, P, I32, P]
        L.ads_apply_noalloc.argtypes = [P, P, P, I32, P]
        L.ads_solve.argtypes = [P, P, P, I32, C.POINTER(ads_ksp_options), C.POINTER(ads_ksp_result), P]
        L.ads_get_info.argtypes = [P, C.POINTER(ads_info)]
        L.ads_export_maps.argtypes = [P, P, P, P, P]
        L.ads_export_splitting.argtypes = [P, P]
        L.ads_export_coarse.argtypes = [P, P, P, P, P]
        L.ads_partition_bfs.argtypes = [C.POINTER(ads_csr), I32, P, P, P]
        L.ads_set_graphs.argtypes = [P, I32]
        L.ads_destroy.argtypes = [P]
        L.ads_status_string.argtypes = [C.c_int]
        L.ads_status_string.restype = C.c_char_p
        L.ads_last_error.argtypes = []
        L.ads_last_error.restype = C.c_char_p
        SH, GR, F = C.POINTER(ads_gnn_shape), C.POINTER(ads_gnn_graph), C.c_float
        L.ads_gnn_nparams.argtypes = [SH]
        L.ads_gnn_workspace_floats.argtypes = [SH, I64]
        L.ads_gnn_graph_size.argtypes = [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I32)]
        L.ads_gnn_graph_build.argtypes = [P, P, P, P, P, P, P, P]
        L.ads_gnn_targets.argtypes = [P, P, I32, P]
        L.ads_gnn_forward.argtypes = [SH, P, GR, P, P, P]
        L.ads_gnn_loss.argtypes = [SH, GR, P, P, I32, P, P, P]
        L.ads_gnn_backward.argtypes = [SH, P, GR, P, P, P, P]
        L.ads_gnn_adam.argtypes = [I64, P, P, P, P, P, I32, F, F, F, F, P]
        L.ads_gnn_round_bf16.argtypes = [I64, P, P, P]
        L.ads_tune_cache_save.argtypes = [C.c_char_p]
        L.ads_tune_cache_load.argtypes = [C.c_char_p]
        L.ads_tune_cache_clear.argtypes = []
        for name in SYMBOLS:
            if name not in ("ads_status_string", "ads_last_error"):
                getattr(L, name).restype = C.c_int
        L.ads_gnn_nparams.restype = I64
        L.ads_gnn_workspace_floats.restype = I64
        _lib = L
    return _lib


class AdsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{ads_status_string(status)}: {msg}")
        self.status = status


def ads_status_string(status: int) -> str:
    return lib().ads_status_string(status).decode()


def ads_last_error() -> str:
    return lib().ads_last_error().decode()


def _check(status):
    if status < 0:
        raise AdsError(status, ads_last_error())
    return status


def _ptr(a):
    return a.ctypes.data if a is not None else None


def make_csr(A):
    """Host CSR (workloads.CSR or scipy.sparse) or a DeviceCSR -> (ads_csr, keep-alive)."""
    if isinstance(A, DeviceCSR):
        return ads_csr(A.n, A.nnz, A.indptr.data_ptr(), A.indices.data_ptr(), A.data.data_ptr(),
                       1), (A,)
    if hasattr(A, "tocsr"):
        A = A.tocsr()
        A.sort_indices()
        n = A.shape[0]
    else:
        n = A.n
    rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.indices, dtype=np.int32)
    if np.iscomplexobj(A.data):  # (re, im) pairs, the layout ads_setup_complex reads
        v = np.ascontiguousarray(A.data, dtype=np.complex128).view(np.float64)
    else:
        v = np.ascontiguousarray(A.data, dtype=np.float64)
    s = ads_csr(n, int(rp[-1]), rp.ctypes.data, ci.ctypes.data, v.ctypes.data, 0)
    return s, (rp, ci, v)


def options(overlap, nev, variant=ADS_VARIANT_DEFLATED, precision=ADS_PREC_FP64, tau=0.0,
            eig_tol=0.0, eig_max_sweeps=0, warm_start=0, gnn_weights_path=None, profile=0,
            eig_solver=0, autotune=0):
    return ads_options(ADS_ABI_VERSION, overlap, nev, tau, variant, precision, warm_start, eig_tol,
                       eig_max_sweeps, gnn_weights_path, profile, eig_solver, autotune)


def ads_setup(A, part, nparts, opts, stream=None):
    return ads_setup_batched([A], [part], [nparts], opts, stream)


def _is_complex(A):
    return not isinstance(A, DeviceCSR) and np.iscomplexobj(A.data)


def ads_setup_batched(As, parts, nparts, opts, stream=None, complex_values=None):
    """ads_setup_batched, or ads_setup_complex when the matrices hold complex
    values (complex_values=None: taken from the first matrix)."""
    nsys = len(As)
    if complex_values is None:
        complex_values = _is_complex(As[0])
    if any(_is_complex(A) != complex_values for A in As):
        raise ValueError("all systems of a context must be real, or all complex")
    arr = (ads_csr * nsys)()
    keep = []
    pp = (C.c_void_p * nsys)()
    parts_c = []
    for k, (A, p) in enumerate(zip(As, parts)):
        s, kk = make_csr(A)
        arr[k] = s
        keep.append(kk)
        pc = np.ascontiguousarray(p, dtype=np.int32)
        parts_c.append(pc)
        pp[k] = pc.ctypes.data
    npc = np.ascontiguousarray(nparts, dtype=np.int32)
    out = C.c_void_p()
    fn = lib().ads_setup_complex if complex_values else lib().ads_setup_batched
    _check(fn(nsys, arr, C.cast(pp, C.c_void_p), npc.ctypes.data, C.byref(opts), stream,
              C.byref(out)))
    return out


def ads_setup_complex(As, parts, nparts, opts, stream=None):
    return ads_setup_batched(As, parts, nparts, opts, stream, complex_values=True)


def ads_apply(ctx, r_ptr, z_ptr, nrhs, stream=None):
    return _check(lib().ads_apply(ctx, r_ptr, z_ptr, nrhs, stream))


def ads_apply_noalloc(ctx, r_ptr, z_ptr, nrhs, stream=None):
    return _check(lib().ads_apply_noalloc(ctx, r_ptr, z_ptr, nrhs, stream))


def ads_solve(ctx, b_ptr, x_ptr, nrhs, kopts, stream=None):
    res = ads_ksp_result()
    st = _check(lib().ads_solve(ctx, b_ptr, x_ptr, nrhs, C.byref(kopts), C.byref(res), stream))
    return st, res


def ads_get_info(ctx):
    info = ads_info()
    _check(lib().ads_get_info(ctx, C.byref(info)))
    nsub = info.nsub
    arrays = {k: np.zeros(nsub, np.int32) for k in ("nev_i", "kernel_dim", "n_i", "n_interior",
                                                     "sweeps", "block")}
    arrays["eig_resid"] = np.zeros(nsub, np.float64)
    for k, a in arrays.items():
        setattr(info, k, a.ctypes.data)
    _check(lib().ads_get_info(ctx, C.byref(info)))
    out = {f[0]: getattr(info, f[0]) for f in ads_info._fields_ if f[0] not in arrays}
    out["t_phase_ms"] = list(info.t_phase_ms)
    out["t_kernel_ms"] = list(info.t_kernel_ms)
    out["n_kernel"] = list(info.n_kernel)
    out.update(arrays)
    return out


def ads_export_maps(ctx):
    info = ads_get_info(ctx)
    tot, nsub = info["omega_total"], info["nsub"]
    om = np.zeros(tot, np.int32)
    off = np.zeros(nsub + 1, np.int64)
    nI = np.zeros(nsub, np.int32)
    lay = np.zeros(tot, np.int32)
    _check(lib().ads_export_maps(ctx, om.ctypes.data, off.ctypes.data, nI.ctypes.data, lay.ctypes.data))
    return om, off, nI, lay


def ads_export_splitting(ctx):
    info = ads_get_info(ctx)
    s = np.zeros(info["omega_total"], np.float64)
    _check(lib().ads_export_splitting(ctx, s.ctypes.data))
    return s


def ads_export_coarse(ctx):
    info = ads_get_info(ctx)
    nsub = info["nsub"]
    woff = np.zeros(nsub + 1, np.int64)
    _check(lib().ads_export_coarse(ctx, None, woff.ctypes.data, None, None))
    W = np.zeros(max(int(woff[-1]), 1), np.float64)
    lr = np.zeros(max(info["n0"], 1))
    li = np.zeros(max(info["n0"], 1))
    _check(lib().ads_export_coarse(ctx, W.ctypes.data, woff.ctypes.data, lr.ctypes.data, li.ctypes.data))
    return W, woff, lr[: info["n0"]] + 1j * li[: info["n0"]], info


def ads_partition_bfs(A, seeds, stream=None):
    s, keep = make_csr(A)
    sd = np.ascontiguousarray(seeds, dtype=np.int32)
    out = np.zeros(s.n, np.int32)
    _check(lib().ads_partition_bfs(C.byref(s), len(sd), sd.ctypes.data, out.ctypes.data, stream))
    return out


def ads_set_graphs(ctx, enable):
    _check(lib().ads_set_graphs(ctx, int(enable)))


def ads_destroy(ctx):
    if ctx is not None and ctx.value:
        lib().ads_destroy(ctx)


def ksp_options(restart=30, flexible=False, rtol=1e-8, maxit=1000, fixed_iters=0):
    return ads_ksp_options(restart, int(flexible), rtol, maxit, fixed_iters)


class Context:
    """Owns an ads context; apply/solve take torch CUDA tensors (FP64, or
    complex128 for complex matrices, passed as their interleaved real views)."""

    def __init__(self, As, parts, nparts, overlap, nev, variant=ADS_VARIANT_DEFLATED,
                 precision=ADS_PREC_FP64, tau=0.0, eig_tol=0.0, eig_max_sweeps=0, stream=None,
                 profile=0, eig_solver=0, warm_start=0, gnn_weights_path=None, autotune=0):
        if not isinstance(As, (list, tuple)):
            As, parts, nparts = [As], [parts], [nparts]
        self._path = (gnn_weights_path.encode() if isinstance(gnn_weights_path, str)
                      else gnn_weights_path)  # kept alive for the call
        self.opts = options(overlap, nev, variant, precision, tau, eig_tol, eig_max_sweeps,
                            warm_start=warm_start, gnn_weights_path=self._path, profile=profile,
                            eig_solver=eig_solver, autotune=autotune)
        self.stream = stream
        self.ctx = ads_setup_batched(As, parts, nparts, self.opts, stream)
        self.info = ads_get_info(self.ctx)
        self.is_complex = bool(self.info["is_complex"])
        self.n = self.info["n"] // (2 if self.is_complex else 1)  # unknowns
        self.nsys = self.info["nsys"]

    def _dtype(self):
        import torch
        return torch.complex128 if self.is_complex else torch.float64

    def _ptr(self, t):
        import torch
        return (torch.view_as_real(t) if self.is_complex else t).data_ptr()

    def apply(self, r, z=None):
        import torch
        nrhs = 1 if r.dim() == 1 else r.shape[1]
        assert r.dtype == self._dtype() and r.is_cuda and r.shape[0] == self.n
        rr = r.contiguous() if r.dim() == 1 else r.t().contiguous()  # column-major n x nrhs
        zz = torch.empty_like(rr)
        ads_apply(self.ctx, self._ptr(rr), self._ptr(zz), nrhs, self.stream)
        return zz if r.dim() == 1 else zz.reshape(nrhs, self.n).t()

    def solve(self, b, restart=30, flexible=False, rtol=1e-8, maxit=1000, fixed_iters=0):
        import torch
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        assert b.dtype == self._dtype() and b.is_cuda and b.shape[0] == self.n
        bb = b.contiguous() if b.dim() == 1 else b.t().contiguous()
        xx = torch.empty_like(bb)
        st, res = ads_solve(self.ctx, self._ptr(bb), self._ptr(xx), nrhs,
                            ksp_options(restart, flexible, rtol, maxit, fixed_iters), self.stream)
        q = self.nsys * nrhs
        out = dict(status=st, its=list(res.its[:q]), relres=list(res.relres[:q]),
                   statuses=list(res.status[:q]), t_setup_ms=res.t_setup_ms,
                   t_solve_ms=res.t_solve_ms)
        x = xx if b.dim() == 1 else xx.reshape(nrhs, self.n).t()
        return x, out

    def set_graphs(self, enable):
        ads_set_graphs(self.ctx, enable)

    def close(self):
        ads_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            if getattr(self, "ctx", None) is not None:
                self.close()
        except Exception:
            pass
