/*
 * ads.h -- C interface of the MI355X library for the algebraic two-level
 * overlapping Schwarz preconditioner of Al Daas, Jolivet and Rees,
 * "Efficient algebraic two-level Schwarz preconditioner for sparse matrices".
 *
 * The library solves A x = b for a real or complex sparse A (Section 1,
 * problem statement; the Notation paragraph takes A complex) with
 * right-preconditioned restarted (F)GMRES (Section 4) and the
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
 *  - FP64 values: real (ads_setup, ads_setup_batched) or complex as
 *    interleaved (re, im) pairs (ads_setup_complex).  Column indices must be
 *    sorted and unique within each row; an explicitly stored zero counts as
 *    an edge of the graph.
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

#define ADS_ABI_VERSION 5
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

/* preconditioner variants (Section 2).  R0^T A00^{-1} R0 is the coarse
 * correction with the coarse space of eq. 6; M_RAS^{-1} = sum_i R_i^T D_i
 * A_ii^{-1} R_i (eq. 3) and M_ASM^{-1} = sum_i R_i^T A_ii^{-1} R_i (eq. 1).
 * The non-restricted forms sum the overlapping local solutions of every
 * subdomain that contains a row, in ascending subdomain order. */
enum {
  ADS_VARIANT_DEFLATED = 0,     /* eq. 4: R0^T A00^{-1} R0 + M_RAS^{-1}(I - A R0^T A00^{-1} R0) */
  ADS_VARIANT_RAS = 1,          /* eq. 3: one-level restricted additive Schwarz (no coarse space) */
  ADS_VARIANT_ASM = 2,          /* eq. 1: one-level additive Schwarz (no coarse space)          */
  ADS_VARIANT_ADDITIVE = 3,     /* eq. 2: R0^T A00^{-1} R0 + M_ASM^{-1}, the additive two-level
                                   preconditioner of the condition bound of Section 3.2        */
  ADS_VARIANT_ADDITIVE_RAS = 4  /* R0^T A00^{-1} R0 + M_RAS^{-1}: eq. 2 with the restricted
                                   one-level part                                              */
};

/* storage precision of the local factors and of the eigensolver operator */
enum {
  ADS_PREC_FP64 = 0,         /* everything FP64                                          */
  ADS_PREC_FP32 = 1,         /* local factors stored FP32, products accumulated in FP64  */
  ADS_PREC_BF16 = 2          /* local factors stored BF16, products accumulated in FP64;
                                refused (ADS_ERR_UNSUPPORTED) when a local solve with them
                                leaves a relative residual above 0.25 (ads_info.local_resid)
                                on the given matrix, e.g. strongly jumping coefficients */
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
                             the whole cluster, so nev_i may exceed nev.  At most 30;
                             with tau > 0 it is the cap of the tau rule, at most 60
                             (the paper's setting: tau = 0.3, 60): the eigensolver
                             resolves 24 per subdomain, and a subdomain where the
                             rule keeps all 24 while the cap allows more is refused
                             with ADS_ERR_UNSUPPORTED                               */
  double tau;             /* <= 0: off; > 0: keep only |lambda| > 1/tau (eq. 6)       */
  int32_t variant;        /* ADS_VARIANT_*                                            */
  int32_t precision;      /* ADS_PREC_*                                               */
  int32_t warm_start;     /* 0: none; 1: learned warm start: the graph network's block
                             (ads_gnn_*) starts the exact eigensolve of eig_solver,
                             run to eig_tol: Krylov-Schur takes as its start block
                             fixed pseudo-random combinations of all the network's
                             columns (the block is narrower than the network's
                             output); the subspace iteration takes the columns
                             themselves and falls back to the cold exact eigensolve
                             (ads_info.eig_fallbacks) if it misses the tolerance
                             within 150 sweeps, Krylov-Schur if its start block has
                             no full rank; 2: learned coarse space: the
                             network's block, with the kernel part (the constant)
                             in front on floating subdomains, orthonormalised on the
                             interior rows, is the coarse space itself (nev_i =
                             n_out + dim K_i, no eigensolve; falls back to the
                             exact one if a block is rank deficient)                */
  double eig_tol;         /* relative residual of the selected invariant subspace
                             (0 -> 1e-10 with FP64 factors; 1e-3 with FP32/BF16
                             factors, where the coarse space only needs the
                             accuracy of the factors it is built from)             */
  int32_t eig_max_sweeps; /* 0 -> 400 (subspace sweeps, or Krylov-Schur block steps)   */
  const char* gnn_weights_path; /* weights file for warm_start != 0: 8 bytes
                             "ADSGNN01", int32 n_in (= ADS_GNN_FEATURES), width,
                             layers, n_out, int64 nparams, nparams FP32 master
                             parameters (little endian, order of ads_gnn_*)         */
  int32_t profile;        /* bit 0 (1): time every apply kernel with hipEvents on its
                             stream (ads_info.t_kernel_ms / n_kernel; hipGraph replay
                             off); bit 1 (2): time every matrix-core update of the
                             setup's dense inversions (coarse operator, diagonal
                             blocks) and count its algorithmic flops
                             (ads_info.t_mfma_update_ms / n_mfma_update /
                             mfma_update_flops); graphs unaffected                */
  int32_t eig_solver;     /* ADS_EIG_*: method for the eq. 5 eigenproblems; a block
                             Krylov-Schur run whose basis loses rank (a Krylov space
                             exhausted on very small subdomains) is redone with the
                             block subspace iteration (counted in eig_fallbacks,
                             reported in ads_info.eig_solver)                        */
  int32_t autotune;       /* 0: block size of every subdomain's block-tridiagonal
                             form = its local bandwidth; 1: pick the block sizes by
                             timing candidates (ceil(f * bandwidth), f in
                             {1, 1.25, 1.5, 2, 2.5}, within the fast-path limits) on
                             this context's matrices, cached per workload shape for
                             the process (ads_tune_cache_*)                         */
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
  int32_t eig_fallbacks;  /* warm starts rejected in favour of the cold start, or 1
                             when Krylov-Schur fell back to the subspace iteration  */
  double t_phase_ms[8];   /* maps, extract, factor, eig, coarse, other, learned start,
                             tile tuning                                            */
  double t_kernel_ms[4];  /* profile = 1: summed device time of the apply kernels:
                             local solve, coarse restrict, coarse prolong, total apply */
  int64_t n_kernel[4];    /* number of timed launches of each                         */
  /* optional caller-owned host arrays of length nsub (NULL to skip): */
  int32_t* nev_i;         /* coarse vectors per subdomain                             */
  int32_t* kernel_dim;    /* dim ker(splitting) per subdomain (0, or 1 for a connected
                             floating subdomain; complex A: 0 or 2, the real form
                             of span{1})                                           */
  int32_t* n_i;           /* |Omega_i|                                                */
  int32_t* n_interior;    /* |Omega_Ii|                                               */
  int32_t* sweeps;        /* eigensolver sweeps (Krylov-Schur: block steps) per subdomain */
  int32_t* block;         /* block size of the local factorization                    */
  double* eig_resid;      /* final ||(T X - X H) V||_F / min |lambda| of the selected
                             invariant subspace per subdomain (eigensolver residual)  */
  int32_t eig_solver;     /* ADS_EIG_* that ran                                      */
  double tile_factor;     /* block size / bandwidth factor in use (1 without tuning) */
  int32_t tile_tuned;     /* 0: not tuned; 1: timed in this setup; 2: from the cache */
  double t_mfma_update_ms;   /* profile bit 1: summed device time of the matrix-core
                                Gauss-Jordan updates of the setup                    */
  int64_t n_mfma_update;     /* their launches                                        */
  double mfma_update_flops;  /* their algorithmic flops, sum of 2 n (n - kb) kb       */
  double local_resid;        /* largest relative residual ||t - A_ii x|| / ||t|| of one
                                local solve with the stored factors (pseudo-random t):
                                what the factor precision costs each local solve     */
  int32_t is_complex;        /* 1 for a context of ads_setup_complex: n, omega_total,
                                n0, nev_i, n_i, n_interior, block, the exports and
                                the vectors of ads_apply / ads_solve are then those of
                                the real form (2 real rows per complex unknown, 2 real
                                coarse vectors per complex one)                      */
} ads_info;

/* Setup for one system (Sections 2 and 3): overlapping subdomains from the
 * graph of A + A^T and the partition `part` (host int32[n], values in
 * [0, nparts), every part non-empty), local block splittings (Definition 1),
 * local factorizations, local eigenproblems (eq. 5) and coarse space (eq. 6),
 * coarse operator E = Z^T A Z and its exact inverse (Gauss-Jordan elimination
 * with partial pivoting).
 * The kernel of each splitting (Section 3.2) is spanned by the indicators of
 * the connected components of its graph whose rows all sum to zero; a
 * subdomain of several components of which at least one floats (a kernel of
 * piecewise constants) returns ADS_ERR_UNSUPPORTED naming the subdomain.
 * *out receives a new context (NULL on error). */
int ads_setup(const ads_csr* A, const int32_t* part, int32_t nparts, const ads_options* opts,
              void* hip_stream, ads_ctx** out);

/* Same for nsys independent systems A[0..nsys) with partitions part[s]
 * (host int32[A[s].n]) of nparts[s] parts, all set up together, one launch per
 * phase.  Vectors of a batched context concatenate the systems in order. */
int ads_setup_batched(int32_t nsys, const ads_csr* A, const int32_t* const* part,
                      const int32_t* nparts, const ads_options* opts, void* hip_stream,
                      ads_ctx** out);

/* Complex A (the Notation paragraph of the paper takes A in C^{n x n}): the
 * same setup as ads_setup_batched for nsys complex systems.  A[s].val holds
 * 2 * nnz doubles, entry k as (re, im) at [2k], [2k + 1] (C99 double complex
 * / std::complex<double> layout); row_ptr, col, part and nparts as for real
 * systems.  The method is that of the paper for complex A: moduli in the
 * lumped sums of Definition 1, the adjoint R_0^H in the coarse operator
 * E = R_0 A R_0^H, complex eigenvectors of eq. 5 spanning the coarse space,
 * GMRES with complex inner products.  It runs on the real form of A, in
 * which complex unknown j is real rows 2j (re) and 2j + 1 (im) and entry
 * a_jk the 2 x 2 block [[re, -im], [im, re]]: complex vectors are then the
 * interleaved arrays themselves, ads_apply takes and returns them as they
 * are (2n doubles per column), and ads_solve runs complex GMRES on them.
 * Each eigenvalue mu of eq. 5 appears as the pair (mu, conj(mu)) of the real
 * form, whose invariant subspace is the real form of the complex eigenvector;
 * nev counts complex vectors (at most 15, or 30 as the cap of the tau rule)
 * and the selection keeps whole pairs.  A floating subdomain (the splitting
 * has the complex constant as null vector) has the two-dimensional kernel
 * span{1, i 1} in the real form: two leading coarse vectors, the projections
 * with the complex left null vector l and i l.  Refused with
 * ADS_ERR_UNSUPPORTED: warm_start != 0.  2n and 4 nnz must stay below 2^31.
 * ads_info.is_complex = 1. */
int ads_setup_complex(int32_t nsys, const ads_csr* A, const int32_t* const* part,
                      const int32_t* nparts, const ads_options* opts, void* hip_stream,
                      ads_ctx** out);

/* z = M^{-1} r (eq. 4, or eq. 3 for ADS_VARIANT_RAS) for nrhs columns.
 * r_dev, z_dev: device FP64, column-major n x nrhs (n = total unknowns), must
 * not overlap.  1 <= nrhs <= 64. */
int ads_apply(ads_ctx* ctx, const double* r_dev, double* z_dev, int32_t nrhs, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * z = M^{-1} r as ads_apply (same kernels, same results), with no hipMalloc,
 * hipFree, event or graph creation.  The apply's workspace lives in a
 * file-scope device array of the library, 128 MiB on every GPU the library
 * runs on, held until the process ends; a context whose workspace for nrhs
 * columns exceeds it is rejected with ADS_ERR_ARG (ads_last_error gives the
 * sizes).  The kernels are launched directly on hip_stream.  All calls on
 * one GPU share the array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Arguments as for ads_apply; a context with ads_options.profile bit 0 set
 * is rejected. */
int ads_apply_noalloc(ads_ctx* ctx, const double* r_dev, double* z_dev, int32_t nrhs,
                      void* hip_stream);

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

/* ---------------------------------------------------------------------------
 * Learned warm start (not in the paper): a message-passing graph network on
 * the graph of every subdomain matrix A_ii predicts a block whose span
 * approximates the coarse space of eq. 6 (Section 3.2), used to start the
 * eq. 5 eigensolves (ads_options.warm_start).  Definition, per graph:
 *   h_0 = F W_in^T + b_in;  a_l = A_w h_l;
 *   u_l = h_l W_s,l^T + a_l W_n,l^T + b_l;  h_{l+1} = h_l + relu(u_l);
 *   X = h_L W_out^T
 * Parameters: one flat vector, W_in (width x n_in, row-major), b_in, then per
 * layer W_s (width x width), W_n (width x width), b (width), then W_out
 * (n_out x width).  The network reads BF16 parameters (uint16 bit patterns);
 * the trainer keeps an FP32 master copy.  Activations and every accumulation
 * are FP32.  All pointers below are device pointers unless stated; calls are
 * ordered on the given HIP stream.  Errors as everywhere: ADS_ERR_ARG for bad
 * shapes or null pointers.
 * ------------------------------------------------------------------------- */
#define ADS_GNN_FEATURES 16 /* node features written by ads_gnn_graph_build */

typedef struct {
  int32_t n_in;   /* input features per node, 1..64 */
  int32_t width;  /* hidden width, 1..64 */
  int32_t layers; /* message-passing layers, 0..16 */
  int32_t n_out;  /* output columns, 1..16 */
} ads_gnn_shape;

/* A batch of graphs with consecutively numbered nodes (device pointers, owned
 * by the caller).  The graph must be symmetric: (j, k) is an edge with weight
 * w iff (k, j) is one with the same weight; no self loops. */
typedef struct {
  int32_t ngraph;
  int64_t nnode;
  const int64_t* node_off; /* [ngraph + 1] first node of each graph */
  const int64_t* row_ptr;  /* [nnode + 1] edge list of every node */
  const int32_t* col;      /* [nedge] neighbour node */
  const float* w;          /* [nedge] edge weight */
  const float* feat;       /* [nnode][n_in] node features, row-major */
  const uint8_t* mask;     /* [nnode] 1 on the rows that enter the loss */
} ads_gnn_graph;

/* Number of parameters of the shape (-1 on a bad shape). */
int64_t ads_gnn_nparams(const ads_gnn_shape* shape);

/* Floats of workspace needed by ads_gnn_forward / ads_gnn_backward for a
 * batch of nnode nodes (the activations of every layer are kept there by the
 * forward pass for the backward pass). */
int64_t ads_gnn_workspace_floats(const ads_gnn_shape* shape, int64_t nnode);

/* Sizes of the graph batch of a context's subdomains: one graph per
 * subdomain (node = slot of Omega_i in ascending global order, edges = the
 * off-diagonal entries of A_ii), nnode = sum |Omega_i| (host outputs). */
int ads_gnn_graph_size(const ads_ctx* ctx, int64_t* nnode, int64_t* nedge, int32_t* ngraph);

/* Builds that batch into caller buffers of the sizes above: node_off
 * [ngraph + 1], row_ptr [nnode + 1], col/w [nedge] with symmetric weights
 * (|a_jk| + |a_kj|) / (2 sqrt(|a_jj a_kk|)), feat [nnode][ADS_GNN_FEATURES]
 * (relative diagonal, its log, lumped s_j / a_jj of Definition 1, interior
 * flag, off-diagonal row sum / a_jj, position t = j / (n_i - 1) in the local
 * order and q = (j mod s) / s with s the local block size, sin and cos of
 * pi t, 2 pi t, pi q, 2 pi q, and 1), mask [nnode] = interior flag.
 * ADS_ERR_SINGULAR if a row of A_ii has no diagonal entry. */
int ads_gnn_graph_build(const ads_ctx* ctx, int64_t* node_off, int64_t* row_ptr, int32_t* col,
                        float* w, float* feat, uint8_t* mask, void* hip_stream);

/* Training targets from a context's coarse space: Z [nnode][nz], interior
 * row j of subdomain i = row j of W_i (ads_export_coarse) in its first
 * min(nev_i, nz) columns; all other entries 0.  nz in 1..16. */
int ads_gnn_targets(const ads_ctx* ctx, float* Z, int32_t nz, void* hip_stream);

/* X [nnode][n_out] = network(params) on the batch; ws of
 * ads_gnn_workspace_floats floats keeps the activations. */
int ads_gnn_forward(const ads_gnn_shape* shape, const uint16_t* params, const ads_gnn_graph* g,
                    float* ws, float* X, void* hip_stream);

/* Projection loss of X against targets Z [nnode][nz] on the masked rows:
 * loss = mean over graphs of ||Z_g - X_g C_g||_F^2 / ||Z_g||_F^2 with
 * C_g = (X_g^T X_g)^{-1} X_g^T Z_g; dX [nnode][n_out] = dloss/dX (0 on
 * unmasked rows); *loss (device double).  A graph whose X_g^T X_g is not
 * positive definite contributes 1 and no gradient. */
int ads_gnn_loss(const ads_gnn_shape* shape, const ads_gnn_graph* g, const float* X,
                 const float* Z, int32_t nz, float* dX, double* loss, void* hip_stream);

/* grad [nparams] += d(sum(dX * X))/d(params), using the activations left in
 * ws by the last ads_gnn_forward on the same batch (ws is also scratch). */
int ads_gnn_backward(const ads_gnn_shape* shape, const uint16_t* params, const ads_gnn_graph* g,
                     float* ws, const float* dX, float* grad, void* hip_stream);

/* One Adam step (bias-corrected, step >= 1) on the FP32 master copy, which is
 * then rounded to nearest-even BF16 into params. */
int ads_gnn_adam(int64_t nparams, float* master, uint16_t* params, const float* grad, float* m,
                 float* v, int32_t step, float lr, float beta1, float beta2, float eps,
                 void* hip_stream);

/* params = BF16 (round to nearest even) of the FP32 master copy. */
int ads_gnn_round_bf16(int64_t nparams, const float* master, uint16_t* params, void* hip_stream);

/* The tile tuner's process-wide cache (ads_options.autotune): save it to a
 * text file, merge a saved file into it, or empty it.  Entries are keyed by
 * the workload's shape (precision, sizes, per-subdomain sizes and bandwidths);
 * ADS_ERR_ARG on unreadable or malformed files. */
int ads_tune_cache_save(const char* path);
int ads_tune_cache_load(const char* path);
int ads_tune_cache_clear(void);

/* Frees the context and its device memory (NULL is accepted). */
int ads_destroy(ads_ctx* ctx);

const char* ads_status_string(int status);
const char* ads_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ADS_H */
