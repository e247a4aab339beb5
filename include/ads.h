/*
 * ads.h -- C interface of the MI355X library for the algebraic two-level
 * overlapping Schwarz preconditioner of Al Daas, Jolivet and Rees,
 * "Efficient algebraic two-level Schwarz preconditioner for sparse matrices".
 *
 * The library solves A x = b for a real sparse A (Section 1, problem
 * statement) with right-preconditioned restarted (F)GMRES (Section 4) and the
 * restricted two-level preconditioner with deflated coarse correction (eq. 4,
 * Section 2), whose coarse space comes from local generalized eigenproblems
 * (eq. 5, eq. 6, Section 3.2) on the local block splitting matrices of
 * Definition 1 (Section 3.1).  Every computational step runs in the library's
 * own HIP kernels on one gfx950 GPU.
 *
 * General conventions
 *  - Every function returns an int status: ADS_OK (0) on success, a negative
 *    ADS_ERR_* code on error, or a positive solver outcome (ADS_KSP_*).  No
 *    C++ exception or abort crosses this interface.  ads_last_error() returns
 *    a thread-local message describing the last error of the calling thread.
 *  - Real FP64 values only.  Column indices must be sorted and unique within
 *    each row; an explicitly stored zero counts as an edge of the graph.
 *  - Ownership: the caller keeps ownership of every pointer it passes in.
 *    ads_setup* copies what it needs into context-owned device memory; the
 *    context owns all device memory it allocates and ads_destroy frees it.
 *  - Streams: `hip_stream` is a hipStream_t (NULL = the default stream).  All
 *    device work is enqueued on that stream; calls that return host data
 *    synchronise it.  One context must not be used by two streams at once.
 *  - Sizes: n < 2^31 and nnz < 2^31 per call (int32 indices on the device).
 */
#ifndef ADS_H
#define ADS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ADS_ABI_VERSION 2
#define ADS_MAX_RESULTS 64 /* entries of ads_ksp_result: nsys * nrhs <= 64 */

/* status codes */
enum {
  ADS_OK = 0,
  ADS_KSP_MAXIT = 1,         /* GMRES stopped at maxit before reaching rtol       */
  ADS_KSP_BREAKDOWN = 2,     /* GMRES breakdown without convergence               */
  ADS_ERR_ARG = -1,          /* invalid argument (message names it)               */
  ADS_ERR_HIP = -2,          /* a HIP runtime call failed                         */
  ADS_ERR_OOM = -3,          /* device allocation failed or exceeded the cap      */
  ADS_ERR_SINGULAR = -4,     /* zero pivot in a local factorization (message names
                                the subdomain) or a singular coarse operator      */
  ADS_ERR_EIG_NOCONV = -5,   /* local eigensolver failed and so did its fallback  */
  ADS_ERR_NAN = -6,          /* non-finite value in the input or the iteration    */
  ADS_ERR_UNSUPPORTED = -7   /* valid input outside what this build implements    */
};

/* preconditioner variants (Section 2) */
enum {
  ADS_VARIANT_DEFLATED = 0,  /* eq. 4: R0^T A00^{-1} R0 + M_RAS^{-1}(I - A R0^T A00^{-1} R0) */
  ADS_VARIANT_RAS = 1        /* eq. 3: one-level restricted additive Schwarz (no coarse space) */
};

/* storage precision of the local factors and of the eigensolver operator */
enum {
  ADS_PREC_FP64 = 0,         /* everything FP64                                          */
  ADS_PREC_FP32 = 1,         /* local factors stored FP32, products accumulated in FP64  */
  ADS_PREC_BF16 = 2          /* local factors stored BF16, products accumulated in FP64  */
};

/* eigensolver for the local eigenproblems of eq. 5 (largest |lambda|) */
enum {
  ADS_EIG_KRYLOV_SCHUR = 0,  /* block Krylov-Schur (block width 4, basis up to 32 vectors,
                                restarts on the ordered Schur form); block subspace
                                iteration where a subdomain is too small for the basis */
  ADS_EIG_SUBSPACE = 1       /* block subspace iteration with Rayleigh-Ritz steps       */
};

typedef struct ads_ctx ads_ctx; /* opaque; owns all device memory it allocates */

/* Sparse matrix in CSR form.  on_device = 0: host pointers; 1: device
 * pointers (read during the call only). */
typedef struct {
  int64_t n, nnz;
  const int64_t* row_ptr; /* [n + 1], row_ptr[0] = 0, row_ptr[n] = nnz */
  const int32_t* col;     /* [nnz], sorted and unique within each row     */
  const double* val;      /* [nnz]                                        */
  int32_t on_device;
} ads_csr;

typedef struct {
  int32_t abi_version;    /* must equal ADS_ABI_VERSION                               */
  int32_t overlap;        /* delta >= 0: graph layers added to each part (Section 2)  */
  int32_t nev;            /* >= 0: coarse vectors per subdomain, kernel part included
                             (eq. 6); a cut inside a cluster of equal |lambda| takes
                             the whole cluster, so nev_i may exceed nev              */
  double tau;             /* <= 0: off; > 0: keep only |lambda| > 1/tau (eq. 6)       */
  int32_t variant;        /* ADS_VARIANT_*                                            */
  int32_t precision;      /* ADS_PREC_*                                               */
  int32_t warm_start;     /* 0: none; 1: learned warm start (initial eigensolver block
                             from the graph network; exact eigensolve still decides) */
  double eig_tol;         /* relative residual of the selected invariant subspace
                             (0 -> 1e-10 with FP64 factors; 1e-3 with FP32/BF16
                             factors, where the coarse space only needs the
                             accuracy of the factors it is built from)             */
  int32_t eig_max_sweeps; /* 0 -> 400 (subspace sweeps, or Krylov-Schur block steps)   */
  const char* gnn_weights_path; /* weights file for warm_start = 1 (NULL otherwise)  */
  int32_t profile;        /* 1: time every apply kernel with hipEvents on its stream
                             (reported in ads_info.t_kernel_ms / n_kernel)           */
  int32_t eig_solver;     /* ADS_EIG_*: method for the eq. 5 eigenproblems            */
} ads_options;

typedef struct {
  int32_t restart;        /* m of GMRES(m), 1..64                                     */
  int32_t flexible;       /* 0: right-preconditioned GMRES; 1: flexible GMRES         */
  double rtol;            /* stop when ||b - A x|| <= rtol ||b|| (Arnoldi estimate and
                             recomputed true residual), x0 = 0 (Section 4)           */
  int32_t maxit;          /* total Arnoldi steps cap (0 -> 1000)                      */
  int32_t fixed_iters;    /* > 0: run exactly this many steps, no convergence test    */
} ads_ksp_options;

typedef struct {
  int32_t its[ADS_MAX_RESULTS];    /* Arnoldi steps per (system, rhs) = sys*nrhs + rhs */
  double relres[ADS_MAX_RESULTS];  /* final true ||b - A x|| / ||b||                 */
  int32_t status[ADS_MAX_RESULTS]; /* ADS_OK, ADS_KSP_MAXIT or ADS_KSP_BREAKDOWN     */
  double t_setup_ms, t_solve_ms;   /* t_setup_ms of the context; t_solve_ms of the call */
} ads_ksp_result;

typedef struct {
  int64_t n;              /* total unknowns over all systems                          */
  int64_t omega_total;    /* sum of |Omega_i| (length of ads_export_maps arrays)      */
  int64_t factor_bytes;   /* device bytes of the local factors used by the apply     */
  int32_t nsys, nsub;     /* systems and subdomains                                   */
  int32_t n0;             /* coarse dimension, all systems                            */
  int32_t eig_sweeps_max; /* largest eigensolver sweep count over subdomains          */
  int32_t eig_unconverged;/* subdomains that hit eig_max_sweeps                       */
  int32_t eig_fallbacks;  /* warm starts rejected in favour of the cold start         */
  double t_phase_ms[8];   /* maps, extract, factor, eig, coarse, other, -, -          */
  double t_kernel_ms[4];  /* profile = 1: summed device time of the apply kernels:
                             local solve, coarse restrict, coarse prolong, total apply */
  int64_t n_kernel[4];    /* number of timed launches of each                         */
  /* optional caller-owned host arrays of length nsub (NULL to skip): */
  int32_t* nev_i;         /* coarse vectors per subdomain                             */
  int32_t* kernel_dim;    /* dim ker(splitting) per subdomain (0 or 1)                */
  int32_t* n_i;           /* |Omega_i|                                                */
  int32_t* n_interior;    /* |Omega_Ii|                                               */
  int32_t* sweeps;        /* eigensolver sweeps (Krylov-Schur: block steps) per subdomain */
  int32_t* block;         /* block size of the local factorization                    */
  double* eig_resid;      /* final ||(T X - X H) V||_F / min |lambda| of the selected
                             invariant subspace per subdomain (eigensolver residual)  */
  int32_t eig_solver;     /* ADS_EIG_* that ran                                      */
} ads_info;

/* Setup for one system (Sections 2 and 3): overlapping subdomains from the
 * graph of A + A^T and the partition `part` (host int32[n], values in
 * [0, nparts), every part non-empty), local block splittings (Definition 1),
 * local factorizations, local eigenproblems (eq. 5) and coarse space (eq. 6),
 * coarse operator E = Z^T A Z and its exact inverse (Gauss-Jordan elimination
 * with partial pivoting).
 * *out receives a new context (NULL on error). */
int ads_setup(const ads_csr* A, const int32_t* part, int32_t nparts, const ads_options* opts,
              void* hip_stream, ads_ctx** out);

/* Same for nsys independent systems A[0..nsys) with partitions part[s]
 * (host int32[A[s].n]) of nparts[s] parts, all set up together, one launch per
 * phase.  Vectors of a batched context concatenate the systems in order. */
int ads_setup_batched(int32_t nsys, const ads_csr* A, const int32_t* const* part,
                      const int32_t* nparts, const ads_options* opts, void* hip_stream,
                      ads_ctx** out);

/* z = M^{-1} r (eq. 4, or eq. 3 for ADS_VARIANT_RAS) for nrhs columns.
 * r_dev, z_dev: device FP64, column-major n x nrhs (n = total unknowns), must
 * not overlap.  1 <= nrhs <= 64. */
int ads_apply(ads_ctx* ctx, const double* r_dev, double* z_dev, int32_t nrhs, void* hip_stream);

/* Solve A x = b with right-preconditioned restarted (F)GMRES, x0 = 0
 * (Section 4), independently for every (system, column).  b_dev, x_dev:
 * device FP64 column-major n x nrhs.  nsys * nrhs <= ADS_MAX_RESULTS.
 * Returns ADS_OK if every column converged, else the largest positive
 * outcome; per-column results in *res. */
int ads_solve(ads_ctx* ctx, const double* b_dev, double* x_dev, int32_t nrhs,
              const ads_ksp_options* kopts, ads_ksp_result* res, void* hip_stream);

/* Context information; see ads_info. */
int ads_get_info(const ads_ctx* ctx, ads_info* info);

/* Index maps (host arrays): omega_concat[omega_total] holds each Omega_i as
 * [Omega_Ii ascending, Omega_Gamma_i ascending] in global (concatenated)
 * numbering; omega_off[nsub + 1] its offsets; n_interior[nsub]; layer
 * [omega_total] = 0 for interior nodes, d in 1..delta for overlap nodes.  Any
 * pointer may be NULL. */
int ads_export_maps(const ads_ctx* ctx, int32_t* omega_concat, int64_t* omega_off,
                    int32_t* n_interior, int32_t* layer);

/* Lumped sums of Definition 1 (host): s_out[omega_total], s_i(j) for the
 * overlap rows (in the omega_concat order) and 0 for interior rows. */
int ads_export_splitting(const ads_ctx* ctx, double* s_out);

/* Coarse space (host): W[sum_i nIi * nev_i], per subdomain the nIi x nev_i
 * row-major block of orthonormal columns spanning D_i Z_i restricted to the
 * interior rows (eq. 6); W_off[nsub + 1] offsets into W; lam_re/lam_im
 * [n0]: the selected eigenvalues of eq. 5 per subdomain in selection order
 * (the kernel column, if any, reports lambda = 0 first). */
int ads_export_coarse(const ads_ctx* ctx, double* W, int64_t* W_off, double* lam_re,
                      double* lam_im);

/* Multi-source BFS partition on the graph of A + A^T: vertex v gets the id of
 * the seed that minimises (graph distance, seed id).  seeds: host int32
 * [nparts], distinct vertices; part_out: host int32[n].  Runs on the GPU. */
int ads_partition_bfs(const ads_csr* A, int32_t nparts, const int32_t* seeds, int32_t* part_out,
                      void* hip_stream);

/* hipGraph replay (default on; off while ads_options.profile is set): the
 * kernels of one apply, and of one Arnoldi step in ads_solve, are captured
 * once and replayed while the buffers and nrhs stay the same.  Graphs run on
 * a stream owned by the context, ordered after the work already queued on the
 * caller's stream, which is ordered after them in turn.  enable = 0 launches
 * every kernel directly on the caller's stream (same results, bit for bit). */
int ads_set_graphs(ads_ctx* ctx, int32_t enable);

/* Frees the context and its device memory (NULL is accepted). */
int ads_destroy(ads_ctx* ctx);

const char* ads_status_string(int status);
const char* ads_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ADS_H */
