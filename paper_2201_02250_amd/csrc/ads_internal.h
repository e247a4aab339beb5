// Internal declarations of the ads library: context layout, error handling,
// small device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ads.h"

namespace ads {

// the variants of Section 2 that carry the coarse space of eq. 6, and those
// whose local part keeps only the owner rows (Boolean partition of unity)
inline bool variant_has_coarse(int v) {
  return v == ADS_VARIANT_DEFLATED || v == ADS_VARIANT_ADDITIVE || v == ADS_VARIANT_ADDITIVE_RAS;
}
inline bool variant_restricted(int v) {
  return v == ADS_VARIANT_DEFLATED || v == ADS_VARIANT_RAS || v == ADS_VARIANT_ADDITIVE_RAS;
}

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);
// message returned by ads_last_error() on this thread
void set_last_error(const std::string& msg);

#define ADS_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e__ = (call);                                                           \
    if (e__ != hipSuccess)                                                             \
      ::ads::fail(ADS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e__));     \
  } while (0)

// Launch-configuration check done on the host before every launch: the grid
// and block must be non-empty and within the documented hardware limits.
inline void check_launch(dim3 g, dim3 b, size_t lds, const char* name) {
  if (g.x == 0 || g.y == 0 || g.z == 0 || b.x == 0 || b.x * b.y * b.z > 1024 || lds > 160 * 1024 ||
      g.y > 65535 || g.z > 65535)
    fail(ADS_ERR_ARG, std::string("bad launch configuration for ") + name);
}

#define ADS_LAUNCH(kernel, grid, block, lds, stream, ...)                              \
  do {                                                                                 \
    ::ads::check_launch(grid, block, lds, #kernel);                                    \
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);                 \
    ADS_HIP(hipGetLastError());                                                        \
  } while (0)

// ---------------------------------------------------------------------------
// Device memory
// ---------------------------------------------------------------------------
// Process-wide cache of device blocks, by device and size class: blocks come
// back here instead of to hipFree (which synchronises the whole device and
// costs tens of microseconds per call), and a later request of the same class
// on the same device reuses them.  Cached blocks are returned to the driver
// only when a hipMalloc fails.  Thread safe.
namespace pool {
size_t size_class(size_t bytes);
// a block of cls bytes on the current device (returned in *dev), nullptr if
// out of memory
void* get(size_t cls, int* dev);
// p (from get on device dev) must no longer be in use by any stream
void put(void* p, size_t cls, int dev);
}  // namespace pool

// Device memory owned by one context or call.  Every block is used on
// `stream` only; release() and the destructor wait for that stream before the
// block goes back to the cache.
struct Arena {
  struct Block {
    void* p;
    size_t cls;
    int dev;
  };
  std::vector<Block> blocks;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  Arena() = default;
  explicit Arena(hipStream_t s) : stream(s) {}
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  template <class T>
  T* alloc(size_t count) {
    if (count == 0) count = 1;
    const size_t cls = pool::size_class(count * sizeof(T));
    int dev = 0;
    void* p = pool::get(cls, &dev);
    if (!p) fail(ADS_ERR_OOM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    blocks.push_back({p, cls, dev});
    bytes += cls;
    return static_cast<T*>(p);
  }
  void release(void* p) {
    for (auto& b : blocks)
      if (b.p == p) {
        (void)hipStreamSynchronize(stream);
        pool::put(b.p, b.cls, b.dev);
        bytes -= b.cls;
        b.p = nullptr;
      }
  }
  ~Arena() {
    bool any = false;
    for (const auto& b : blocks) any |= b.p != nullptr;
    if (!any) return;
    (void)hipStreamSynchronize(stream);
    for (const auto& b : blocks)
      if (b.p) pool::put(b.p, b.cls, b.dev);
  }
};

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct Ctx {
  Arena mem;
  hipStream_t stream = nullptr;
  ads_options opt{};
  int nsys = 0;
  int nsub = 0;
  int64_t n = 0;    // total unknowns (of the real form for a complex context)
  int64_t nnz = 0;  // total entries
  // complex A: the matrix is held in its real form (unknown j -> rows 2j, 2j+1,
  // entry a_jk -> the block [[re, -im], [im, re]]); lumping, kernel detection,
  // the eigenvalue selection and GMRES take the pairs into account
  int cplx = 0;
  std::vector<int64_t> sys_row;  // [nsys+1] row offsets of the systems
  std::vector<int32_t> sys_sub;  // [nsys+1] subdomain offsets of the systems
  std::vector<int32_t> sub_sys;  // [nsub] system of each subdomain
  int32_t* sub_sys_d = nullptr;  // device copy

  // concatenated (block-diagonal) matrix, int32 indices
  int32_t* rowptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  int32_t* tptr = nullptr;  // transpose pattern (graph of A^T)
  int32_t* tcol = nullptr;
  int32_t* part = nullptr;  // global subdomain id of each unknown
  int32_t* ipos = nullptr;  // position of each unknown inside its own Omega_Ii
  // per-subdomain window [wlo, whi) of the global index range containing
  // Omega_i; wpos[woff + v - wlo] = position of v in ascending Omega_i, or -1
  int64_t* wlo = nullptr;
  int64_t* whi = nullptr;
  int64_t* woff = nullptr;
  int32_t* wpos = nullptr;

  // maps: omega in ascending global order ("sorted") and in [I, Gamma] order ("export")
  int64_t omega_total = 0;
  std::vector<int32_t> h_ni, h_nI;
  std::vector<int64_t> h_om_off;
  int32_t* ni = nullptr;
  int32_t* nI = nullptr;
  int64_t* om_off = nullptr;     // [nsub+1]
  int32_t* om_sorted = nullptr;  // [omega_total] global ids, ascending per subdomain
  int32_t* om_sub = nullptr;     // [omega_total] subdomain of each slot
  uint8_t* om_int = nullptr;     // [omega_total] 1 if the slot is interior
  int32_t* om_export = nullptr;  // [omega_total] [I asc, Gamma asc]
  int32_t* om_layer = nullptr;   // [omega_total] layer of each export slot
  int32_t* int_list = nullptr;   // alias into om_export: interior ids start at om_off[i]

  // local matrices: CSR of A_ii in the sorted local order
  int64_t lnnz = 0;
  int64_t* lptr_off = nullptr;  // [omega_total+1] row starts into lcol / lval, sorted order
  int32_t* lcol = nullptr;
  double* lval = nullptr;
  double* lsum = nullptr;       // [omega_total] lumped s (0 on interior rows), sorted order
  int32_t* kdim = nullptr;      // [nsub] kernel dimension of the splitting (0/1)
  int32_t* sub_order = nullptr; // [nsub] subdomains by decreasing (2K - 1) s^2 (longest first)
  std::vector<int32_t> h_kdim;

  // block-tridiagonal factors
  std::vector<int32_t> h_bs, h_nb;  // block size and block count per subdomain
  std::vector<int32_t> h_bw;        // local bandwidth (smallest valid block size)
  int32_t* bw_d = nullptr;          // its device copy
  double tile_factor = 1.0;         // block size / bandwidth target chosen by the tuner
  int tile_tuned = 0;               // 0 default tiles, 1 timed now, 2 from the tuning cache
  std::vector<int64_t> h_fac_off;   // per subdomain, in elements, per matrix
  int32_t* bs = nullptr;
  int32_t* nb = nullptr;
  int64_t* fac_off = nullptr;
  int64_t fac_elems = 0;
  int64_t npad_total = 0;           // sum of nb*bs
  std::vector<int64_t> h_pad_off;
  int64_t* pad_off = nullptr;       // [nsub+1] offsets of padded local vectors
  // coupling lists of the block-tridiagonal form, NCPL slots per padded row
  // (column) with -1 / 0.0 in unused slots; indices are local to the block
  int32_t* cpl_col = nullptr;       // A_k,k-1 by row: columns in block k-1
  double* cpl_val = nullptr;
  int32_t* rcpl_col = nullptr;      // A_k,k+1 by row: columns in block k+1
  double* rcpl_val = nullptr;
  int32_t* ucpl_row = nullptr;      // A_k-1,k by column of block k: rows in block k-1
  double* ucpl_val = nullptr;
  int32_t* lcpl_row = nullptr;      // A_k+1,k by column of block k: rows in block k+1
  double* lcpl_val = nullptr;
  bool cpl_ok = false;              // all four lists complete (<= NCPL per row / column)
  bool solve_fast = false;          // every subdomain fits the prefetching tile solve
  bool sym = false;                 // A equals A^T entry for entry (pattern and values)
  double local_resid = 0.0;         // local_solve_accuracy() after the factorization
  void* facA = nullptr;             // factors of A_ii (apply)
  void* facT = nullptr;             // factors of the regularised splitting (eigensolver)
  int prec = ADS_PREC_FP64;
  int64_t factor_bytes = 0;

  // coarse space
  int n0 = 0;
  std::vector<int32_t> h_nev, h_coff, h_sweeps;
  std::vector<double> h_lam_re, h_lam_im, h_eig_res;
  int32_t* nev = nullptr;      // [nsub]
  int32_t* coff = nullptr;     // [nsub+1] coarse column offset (global over systems)
  int64_t* W_off = nullptr;    // [nsub+1]
  std::vector<int64_t> h_W_off;
  double* W = nullptr;
  std::vector<int32_t> h_n0s;  // per system coarse size
  std::vector<int64_t> h_E_off;
  int64_t* E_off = nullptr;    // [nsys+1] element offsets of the dense per-system E^{-1}
  int32_t* sys_coff = nullptr; // [nsys+1] first coarse index of each system
  double* Einv = nullptr;
  int32_t eig_sweeps_max = 0, eig_unconverged = 0, eig_fallbacks = 0;
  bool eig_krylov_schur = false;  // block Krylov-Schur ran (else block subspace iteration)
  bool eig_ks_lost_rank = false;  // Krylov-Schur lost rank: the setup uses subspace iteration
  // learned warm start: the network's block (node rows of Omega_i in sorted
  // order x gnn_cols, FP32), set by learned_start for the eigensolve
  float* gnn_x = nullptr;
  int gnn_cols = 0;
  ads_gnn_shape gnn_shape{};        // the weights file, read while the arguments
  std::vector<float> gnn_master;    // are checked (FP32 master parameters)
  int h_eig_nblk = 0;  // row blocks of the eigensolver sweep kernels
  int h_eig_nqblk = 0;  // wide row blocks of the Krylov-Schur block QR kernels
  std::vector<int32_t> h_eig_km;  // per subdomain Krylov-Schur Rayleigh quotient order

  // workspace for apply / solve
  int32_t* cover_ptr = nullptr;  // [n + 1] non-restricted variants: per global row, the
  int32_t* cover_idx = nullptr;  //   padded local slots (pad_off[i] + local row), ascending i
  double* work = nullptr;   // padded local vectors, npad_total * work_cols
  double* work2 = nullptr;  // backward results of the two-ended solve, same shape
  double* dummy = nullptr;  // per-thread discard slots of the tile solves
  int work_cols = 0;
  int work_n0 = -1;         // coarse dimension the workspace was sized for
  double* cvec = nullptr;   // partial sums of the coarse restriction, n0 * cols * chunks
  double* yvec = nullptr;   // c and y = E^{-1} c of large coarse systems, 2 n0 cols
  double* qvec = nullptr;   // coarse correction, n * cols
  int cvec_cols = 0;

  double t_phase_ms[8] = {0};
  // apply profiling (opt.profile bit 0): event pairs per kernel, resolved lazily
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[4];
  double prof_ms[4] = {0};
  int64_t prof_n[4] = {0};
  // setup profiling (opt.profile bit 1): the matrix-core Gauss-Jordan updates
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_gj_ev;
  double prof_gj_ms = 0.0, prof_gj_flops = 0.0;
  int64_t prof_gj_n = 0;
  // hipGraph replay: the apply, and in ads_solve the Arnoldi step, are
  // captured once and replayed while their arguments and stream are the same
  bool use_graphs = true;
  bool capturing = false;           // inside a capture: launch eagerly
  hipStream_t priv = nullptr;       // the context's own stream (default priority)
  // pinned host staging of the solver's per-step status
  struct Pinned {
    double* p = nullptr;
    size_t n = 0;
    double* get(size_t need) {
      if (n < need) {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
        if (hipHostMalloc((void**)&p, need * sizeof(double), hipHostMallocDefault) != hipSuccess) {
          p = nullptr;
          return nullptr;
        }
        n = need;
      }
      return p;
    }
    ~Pinned() {
      if (p) (void)hipHostFree(p);
    }
  } pin;
  hipEvent_t dep_ev = nullptr;      // orders priv against the caller's stream
  hipGraphExec_t apply_exec = nullptr;
  const double* ag_r = nullptr;
  double* ag_z = nullptr;
  int ag_nrhs = 0;
  hipStream_t ag_st = nullptr;
  hipStream_t own_stream();
  void drop_apply_graph();
  bool graphs_on() const { return use_graphs && !(opt.profile & 1); }

  void prof_resolve();
  ~Ctx();
  double t_setup_ms = 0;
};

}  // namespace ads

// the opaque handle of the C interface
struct ads_ctx {
  ads::Ctx* c;
};

namespace ads {

inline const Ctx* ctx_of(const ads_ctx* h) { return h->c; }
inline Ctx* ctx_of(ads_ctx* h) { return h->c; }

// graph network (learned warm start), implemented in k_gnn.hip
void gnn_forward_impl(const ads_gnn_shape& s, const uint16_t* params, const ads_gnn_graph& g,
                      float* ws, float* X, hipStream_t st);
void gnn_graph_impl(const Ctx& c, int64_t* node_off, int64_t* row_ptr, int32_t* col, float* w,
                    float* feat, uint8_t* mask, hipStream_t st);
int64_t gnn_edges(const Ctx& c);
// reads and checks a weights file (host only; ADS_ERR_ARG on a missing,
// malformed, mis-shaped or truncated file)
void read_gnn_weights(const char* path, ads_gnn_shape* shape, std::vector<float>* master);
// runs the network (parameters read by read_gnn_weights into c.gnn_shape /
// c.gnn_master) on the context's subdomain graphs into c.gnn_x
void learned_start(Ctx& c);

// ---------------------------------------------------------------------------
// launchers (host functions implemented in the kernel translation units)
// ---------------------------------------------------------------------------
void build_maps(Ctx& c, const std::vector<int32_t>& part_host_concat);
void extract_local(Ctx& c);
void set_tiles(Ctx& c, const std::vector<int32_t>& sizes);
void tune_tiles(Ctx& c);
double time_local_solve(Ctx& c, int reps);
void release_factors(Ctx& c);
void factor_local(Ctx& c, bool only_a = false);
void eigensolve(Ctx& c);
void assemble_coarse(Ctx& c);
bool work_fits(const Ctx& c, int cols);
void ensure_work(Ctx& c, int cols);
// row -> local-solution slots of every subdomain containing the row (eq. 1
// and eq. 2 prolongation), built once per context
void build_cover(Ctx& c);
void apply_prec(Ctx& c, const double* r, double* z, int nrhs, hipStream_t s);
// largest relative residual ||t_i - A_ii x_i|| / ||t_i|| of one local solve
// with the stored factors (fixed pseudo-random right-hand side)
double local_solve_accuracy(Ctx& c);
// the same apply with its workspace in the library's scratch array (no
// allocation; calls that overlap on one GPU race)
void apply_noalloc(Ctx& c, const double* r, double* z, int nrhs, hipStream_t s);

// Capture the launches of f on stream s (not the null stream) into an
// executable graph.  The capture is ended on every exit path.
template <class F>
hipGraphExec_t capture_graph(hipStream_t s, F&& f) {
  ADS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  try {
    f();
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hipGraph_t g = nullptr;
  ADS_HIP(hipStreamEndCapture(s, &g));
  hipGraphExec_t e = nullptr;
  const hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  ADS_HIP(err);
  return e;
}

// Runs f on the context's own stream ordered after the work already queued
// on the caller's stream st, and orders st after it.
template <class F>
void on_own_stream(Ctx& c, hipStream_t st, F&& f) {
  hipStream_t ps = c.own_stream();
  ADS_HIP(hipEventRecord(c.dep_ev, st));
  ADS_HIP(hipStreamWaitEvent(ps, c.dep_ev, 0));
  f(ps);
  ADS_HIP(hipEventRecord(c.dep_ev, ps));
  ADS_HIP(hipStreamWaitEvent(st, c.dep_ev, 0));
}
int gmres_solve(Ctx& c, const double* b, double* x, int nrhs, const ads_ksp_options& ko,
                ads_ksp_result* res, hipStream_t s);
void bfs_partition(const int32_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                   const std::vector<int32_t>& seeds, std::vector<int32_t>& part, hipStream_t s);
void transpose_pattern(Arena& mem, const int32_t* rowptr, const int32_t* col, int64_t n,
                       int64_t nnz, int32_t** tptr, int32_t** tcol, hipStream_t s);
void exclusive_scan_i64(const int32_t* in, int64_t* out, int64_t n, Arena& mem, hipStream_t s);
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, Arena& mem, hipStream_t s);

// host <-> device helpers
template <class T>
T* upload(Arena& mem, const T* h, size_t count, hipStream_t s) {
  T* d = mem.alloc<T>(count);
  if (count) ADS_HIP(hipMemcpyAsync(d, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}
template <class T>
void download(std::vector<T>& h, const T* d, size_t count, hipStream_t s) {
  h.resize(count);
  if (count) ADS_HIP(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, s));
  ADS_HIP(hipStreamSynchronize(s));
}

}  // namespace ads

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
namespace adsd {

__device__ __forceinline__ int lower_bound_i32(const int32_t* a, int n, int32_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int upper_bound_i64(const int64_t* a, int n, int64_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// index of the segment containing flat position f (offsets ascending, off[0] = 0)
__device__ __forceinline__ int segment_of(const int64_t* off, int nseg, int64_t f) {
  return upper_bound_i64(off, nseg + 1, f) - 1;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// deterministic block sum over blockDim.x threads (multiple of 64, <= 1024);
// `red` is LDS scratch of >= 16 doubles.  All threads receive the result.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Packed tile format of the local factors: element (r, c) of an s x s tile is
// stored at ((c / V) * s + r) * V + (c % V) with V = 16 bytes / element size,
// columns padded with zeros to a multiple of V.  A thread that owns row r and
// a run of columns then fetches V entries with one 16-byte load, and lanes
// with consecutive rows read consecutive 16-byte words (fully coalesced).
// subdomain of block b of a per-subdomain launch: the blocks take the
// subdomains in decreasing order of their chain cost (order, set at setup),
// so that the dispatcher, which starts blocks in index order as compute
// units free up, schedules the longest chains first
__device__ __forceinline__ int sub_of(const int32_t* order, int b) { return order ? order[b] : b; }

template <class FT>
struct TileV {
  static constexpr int V = 16 / (int)sizeof(FT);
};
__host__ __device__ inline int tile_cols(int s, int V) { return V * ((s + V - 1) / V); }
__host__ __device__ inline int64_t tile_size(int s, int V) { return (int64_t)s * tile_cols(s, V); }
__host__ __device__ inline int64_t tile_at(int r, int c, int s, int V) {
  return ((int64_t)(c / V) * s + r) * V + (c % V);
}

// storage conversions of factor entries
__device__ __forceinline__ double ld_fac(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ double ld_fac(const float* p, int64_t i) { return (double)p[i]; }
__device__ __forceinline__ double ld_fac(const __hip_bfloat16* p, int64_t i) {
  return (double)__bfloat162float(p[i]);
}
__device__ __forceinline__ void st_fac(double* p, int64_t i, double v) { p[i] = v; }
__device__ __forceinline__ void st_fac(float* p, int64_t i, double v) { p[i] = (float)v; }
__device__ __forceinline__ void st_fac(__hip_bfloat16* p, int64_t i, double v) {
  p[i] = __float2bfloat16((float)v);
}

// 64-bit mix (splitmix64 finaliser) -> uniform double in [-1, 1)
__device__ __forceinline__ double hash_unit(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x = x ^ (x >> 31);
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

}  // namespace adsd
