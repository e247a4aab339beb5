// C interface of the ads library (declared in include/ads.h): argument
// validation, setup orchestration, exports.  No exception crosses the
// interface; errors become status codes plus a thread-local message.
#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <cmath>
#include <cstring>

#include "ads_internal.h"

namespace ads {

namespace pool {
namespace {
std::mutex g_mu;
std::map<std::pair<int, size_t>, std::vector<void*>> g_free;
}  // namespace

size_t size_class(size_t bytes) {
  // 256 B granularity up to 64 KiB, then an eighth of the power of two below
  // (at most 12.5 % rounding)
  if (bytes <= 65536) return (bytes + 255) & ~size_t(255);
  size_t p2 = 1;
  while (p2 * 2 <= bytes) p2 *= 2;
  const size_t step = p2 / 8;
  return (bytes + step - 1) / step * step;
}

void* get(size_t cls, int* devp) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  *devp = dev;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_free.find({dev, cls});
    if (it != g_free.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, cls) == hipSuccess) return p;
  (void)hipGetLastError();
  // out of memory: hand every cached block of this device back and retry
  {
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipDeviceSynchronize();
    for (auto& kv : g_free)
      if (kv.first.first == dev) {
        for (void* q : kv.second) (void)hipFree(q);
        kv.second.clear();
      }
  }
  if (hipMalloc(&p, cls) == hipSuccess) return p;
  (void)hipGetLastError();
  return nullptr;
}

void put(void* p, size_t cls, int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_free[{dev, cls}].push_back(p);
}
}  // namespace pool

static thread_local std::string g_last_error;

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

static int handle(const Error& e) {
  g_last_error = e.msg;
  return e.code;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

struct Timer {
  hipStream_t s;
  std::chrono::steady_clock::time_point t;
  explicit Timer(hipStream_t st) : s(st) {
    ADS_HIP(hipStreamSynchronize(s));
    t = std::chrono::steady_clock::now();
  }
  double lap() {
    ADS_HIP(hipStreamSynchronize(s));
    auto now = std::chrono::steady_clock::now();
    double ms = std::chrono::duration<double, std::milli>(now - t).count();
    t = now;
    return ms;
  }
};

static void check_csr_host(const ads_csr& A, int sys) {
  const std::string w = "system " + std::to_string(sys) + ": ";
  if (A.n <= 0 || A.n >= (int64_t(1) << 31)) fail(ADS_ERR_ARG, w + "n out of range");
  if (A.nnz < 0 || A.nnz >= (int64_t(1) << 31)) fail(ADS_ERR_ARG, w + "nnz out of range");
  if (!A.row_ptr || !A.col || !A.val) fail(ADS_ERR_ARG, w + "null CSR array");
  if (A.row_ptr[0] != 0 || A.row_ptr[A.n] != A.nnz) fail(ADS_ERR_ARG, w + "row_ptr bounds");
  for (int64_t r = 0; r < A.n; ++r) {
    if (A.row_ptr[r + 1] < A.row_ptr[r]) fail(ADS_ERR_ARG, w + "row_ptr not monotone");
    for (int64_t k = A.row_ptr[r]; k < A.row_ptr[r + 1]; ++k) {
      if (A.col[k] < 0 || A.col[k] >= A.n) fail(ADS_ERR_ARG, w + "column index out of range");
      if (k > A.row_ptr[r] && A.col[k] <= A.col[k - 1])
        fail(ADS_ERR_ARG, w + "columns not sorted/unique in row " + std::to_string(r));
      if (!std::isfinite(A.val[k])) fail(ADS_ERR_NAN, w + "non-finite matrix entry");
    }
  }
}

// brings one system's CSR to the host (device input is copied back once)
struct HostCSR {
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
  ads_csr view{};
};

static void to_host(const ads_csr& A, HostCSR& h, hipStream_t s) {
  if (!A.on_device) {
    h.view = A;
    return;
  }
  if (A.n <= 0 || A.nnz < 0) fail(ADS_ERR_ARG, "bad CSR sizes");
  h.rp.resize(A.n + 1);
  h.ci.resize(A.nnz);
  h.v.resize(A.nnz);
  ADS_HIP(hipMemcpyAsync(h.rp.data(), A.row_ptr, (A.n + 1) * 8, hipMemcpyDeviceToHost, s));
  if (A.nnz) {
    ADS_HIP(hipMemcpyAsync(h.ci.data(), A.col, A.nnz * 4, hipMemcpyDeviceToHost, s));
    ADS_HIP(hipMemcpyAsync(h.v.data(), A.val, A.nnz * 8, hipMemcpyDeviceToHost, s));
  }
  ADS_HIP(hipStreamSynchronize(s));
  h.view = A;
  h.view.row_ptr = h.rp.data();
  h.view.col = h.ci.data();
  h.view.val = h.v.data();
  h.view.on_device = 0;
}

// copy one system's CSR into the concatenated arrays (row offset r0, entry
// offset k0), shifting column indices; flags: 1 bad row pointers, 2 column
// out of range, 4 columns not strictly increasing, 8 non-finite value
__global__ void k_import_csr(const int64_t* rp, const int32_t* ci, const double* v, int64_t n,
                             int64_t nnz, int64_t r0, int64_t k0, int32_t* rowptr, int32_t* col,
                             double* val, int32_t* bad) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > n) return;
  const int64_t base = rp[0];
  if (r == n) {
    if (base != 0 || rp[n] != nnz) atomicOr(bad, 1);
    rowptr[r0 + n] = (int32_t)(k0 + nnz);
    return;
  }
  const int64_t a = rp[r], b = rp[r + 1];
  rowptr[r0 + r] = (int32_t)(k0 + a);
  if (b < a || a < 0 || b > nnz) {
    atomicOr(bad, 1);
    return;
  }
  int prev = -1;
  for (int64_t k = a; k < b; ++k) {
    const int c = ci[k];
    if (c < 0 || c >= n) atomicOr(bad, 2);
    if (c <= prev) atomicOr(bad, 4);
    prev = c;
    if (!isfinite(v[k])) atomicOr(bad, 8);
    col[k0 + k] = (int32_t)(c + r0);
    val[k0 + k] = v[k];
  }
}

// *asym = 1 unless every stored a_rc has a stored a_cr of the same value
// (columns sorted within rows: binary search in row c)
__global__ void k_check_symmetric(const int32_t* rowptr, const int32_t* col, const double* val,
                                  int64_t n, int32_t* asym) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) {
    const int c = col[k];
    int lo = rowptr[c], hi = rowptr[c + 1];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (col[mid] < r) lo = mid + 1; else hi = mid;
    }
    if (lo >= rowptr[c + 1] || col[lo] != r || val[lo] != val[k]) {
      atomicOr(asym, 1);
      return;
    }
  }
}

// complex CSR (entry k as (re, im) at v[2k], v[2k + 1]) into the real form:
// unknown r -> rows 2r (re) and 2r + 1 (im) at row offset r0, entry (c, z) ->
// columns 2c, 2c + 1 holding (re, -im) in row 2r and (im, re) in row 2r + 1,
// so that a complex vector stored interleaved is multiplied as it is; flags
// as k_import_csr
__global__ void k_import_csr_complex(const int64_t* rp, const int32_t* ci, const double* v,
                                     int64_t n, int64_t nnz, int64_t r0, int64_t k0,
                                     int32_t* rowptr, int32_t* col, double* val, int32_t* bad) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > n) return;
  if (r == n) {
    if (rp[0] != 0 || rp[n] != nnz) atomicOr(bad, 1);
    rowptr[r0 + 2 * n] = (int32_t)(k0 + 4 * nnz);
    return;
  }
  const int64_t a = rp[r], b = rp[r + 1];
  if (b < a || a < 0 || b > nnz) {
    atomicOr(bad, 1);
    rowptr[r0 + 2 * r] = rowptr[r0 + 2 * r + 1] = (int32_t)k0;
    return;
  }
  const int64_t L = b - a;
  const int64_t e_re = k0 + 4 * a, e_im = e_re + 2 * L;
  rowptr[r0 + 2 * r] = (int32_t)e_re;
  rowptr[r0 + 2 * r + 1] = (int32_t)e_im;
  int prev = -1;
  for (int64_t k = a; k < b; ++k) {
    const int c = ci[k];
    if (c < 0 || c >= n) atomicOr(bad, 2);
    if (c <= prev) atomicOr(bad, 4);
    prev = c;
    const double re = v[2 * k], im = v[2 * k + 1];
    if (!isfinite(re) || !isfinite(im)) atomicOr(bad, 8);
    const int32_t c0 = (int32_t)(r0 + 2 * (int64_t)c);
    const int64_t t = 2 * (k - a);
    col[e_re + t] = c0;
    col[e_re + t + 1] = c0 + 1;
    val[e_re + t] = re;
    val[e_re + t + 1] = -im;
    col[e_im + t] = c0;
    col[e_im + t + 1] = c0 + 1;
    val[e_im + t] = im;
    val[e_im + t + 1] = re;
  }
}

static void import_csr(Ctx& c, const ads_csr& A, int64_t r0, int64_t k0, int32_t* bad,
                       hipStream_t st) {
  const int64_t* rp = A.row_ptr;
  const int32_t* ci = A.col;
  const double* v = A.val;
  const int64_t vlen = c.cplx ? 2 * A.nnz : A.nnz;
  Arena tmp(st);
  if (!A.on_device) {
    rp = upload(tmp, A.row_ptr, A.n + 1, st);
    ci = upload(tmp, A.col, A.nnz, st);
    v = upload(tmp, A.val, vlen, st);
  }
  if (c.cplx)
    ADS_LAUNCH(k_import_csr_complex, dim3((unsigned)((A.n + 256) / 256)), dim3(256), 0, st, rp, ci,
               v, A.n, A.nnz, r0, k0, c.rowptr, c.col, c.val, bad);
  else
    ADS_LAUNCH(k_import_csr, dim3((unsigned)((A.n + 256) / 256)), dim3(256), 0, st, rp, ci, v, A.n,
               A.nnz, r0, k0, c.rowptr, c.col, c.val, bad);
  ADS_HIP(hipStreamSynchronize(st));
}

// largest local-solve relative residual accepted with BF16 factors
static constexpr double BF16_MAX_LOCAL_RESID = 0.25;

static Ctx* setup_impl(int nsys, const ads_csr* A, const int32_t* const* part, const int32_t* nparts,
                       const ads_options* opts, hipStream_t st, bool cplx) {
  if (nsys <= 0) fail(ADS_ERR_ARG, "nsys must be positive");
  if (!A || !part || !nparts || !opts) fail(ADS_ERR_ARG, "null argument");
  if (opts->abi_version != ADS_ABI_VERSION) fail(ADS_ERR_ARG, "abi_version mismatch");
  if (opts->overlap < 0 || opts->overlap > 16) fail(ADS_ERR_ARG, "overlap must be in [0, 16]");
  // nev is the coarse vectors per subdomain, or with the tau rule of eq. 6
  // their cap (the paper's setting: tau = 0.3, at most 60); a complex vector
  // is two real ones of the real form
  const int nev_max = (opts->tau > 0 ? 60 : 30) / (cplx ? 2 : 1);
  if (opts->nev < 0 || opts->nev > nev_max)
    fail(ADS_ERR_ARG, cplx ? "nev must be in [0, 15] for complex A (in [0, 30] as the cap of the "
                             "tau rule)"
                           : "nev must be in [0, 30] (in [0, 60] as the cap of the tau rule)");
  if (cplx && opts->warm_start != 0)
    fail(ADS_ERR_UNSUPPORTED, "the learned warm start is for real A only");
  if (opts->variant < ADS_VARIANT_DEFLATED || opts->variant > ADS_VARIANT_ADDITIVE_RAS)
    fail(ADS_ERR_ARG, "unknown variant");
  if (opts->precision < ADS_PREC_FP64 || opts->precision > ADS_PREC_BF16)
    fail(ADS_ERR_ARG, "unknown precision");
  if (opts->warm_start < 0 || opts->warm_start > 2) fail(ADS_ERR_ARG, "unknown warm_start");
  if (opts->warm_start != 0 && !opts->gnn_weights_path)
    fail(ADS_ERR_ARG, "warm_start needs gnn_weights_path");
  if (opts->eig_solver != ADS_EIG_KRYLOV_SCHUR && opts->eig_solver != ADS_EIG_SUBSPACE)
    fail(ADS_ERR_ARG, "unknown eig_solver");
  // every system's arguments, before any device call
  const int64_t rf = cplx ? 2 : 1;  // real rows per unknown
  for (int s = 0; s < nsys; ++s) {
    if (A[s].n <= 0 || rf * A[s].n >= (int64_t(1) << 31)) fail(ADS_ERR_ARG, "n out of range");
    if (A[s].nnz < 0 || rf * rf * A[s].nnz >= (int64_t(1) << 31))
      fail(ADS_ERR_ARG, "nnz out of range");
    if (!A[s].row_ptr || !A[s].col || !A[s].val) fail(ADS_ERR_ARG, "null CSR array");
    if (!part[s]) fail(ADS_ERR_ARG, "null partition");
    if (nparts[s] <= 0) fail(ADS_ERR_ARG, "nparts must be positive");
  }
  ads_gnn_shape gshape{};
  std::vector<float> gmaster;
  if (opts->warm_start) read_gnn_weights(opts->gnn_weights_path, &gshape, &gmaster);
  auto c = new Ctx();
  try {
    c->gnn_shape = gshape;
    c->gnn_master = std::move(gmaster);
    c->stream = st;
    c->mem.stream = st;
    c->opt = *opts;
    c->cplx = cplx ? 1 : 0;
    c->opt.nev = (int32_t)(rf * opts->nev);  // real coarse vectors of the real form
    c->prec = opts->precision;
    c->nsys = nsys;
    Timer tm(st);
    auto t_start = std::chrono::steady_clock::now();
    // concatenate the systems (block-diagonal matrix): each CSR (host or
    // device) is imported by a kernel that shifts indices and validates it
    c->sys_row.assign(nsys + 1, 0);
    c->sys_sub.assign(nsys + 1, 0);
    std::vector<int64_t> sys_nnz(nsys + 1, 0);
    for (int s = 0; s < nsys; ++s) {
      c->sys_row[s + 1] = c->sys_row[s] + rf * A[s].n;
      c->sys_sub[s + 1] = c->sys_sub[s] + nparts[s];
      sys_nnz[s + 1] = sys_nnz[s] + rf * rf * A[s].nnz;
    }
    c->n = c->sys_row[nsys];
    c->nnz = sys_nnz[nsys];
    c->nsub = c->sys_sub[nsys];
    if (c->n >= (int64_t(1) << 31) || c->nnz >= (int64_t(1) << 31))
      fail(ADS_ERR_UNSUPPORTED, "total n and nnz must be < 2^31");
    c->rowptr = c->mem.alloc<int32_t>(c->n + 1);
    c->col = c->mem.alloc<int32_t>(c->nnz);
    c->val = c->mem.alloc<double>(c->nnz);
    int32_t* bad = c->mem.alloc<int32_t>(1);
    ADS_HIP(hipMemsetAsync(bad, 0, 4, st));
    std::vector<int32_t> pg(c->n);
    c->sub_sys.resize(c->nsub);
    for (int s = 0; s < nsys; ++s) {
      import_csr(*c, A[s], c->sys_row[s], sys_nnz[s], bad, st);
      for (int64_t r = 0; r < A[s].n; ++r) {
        const int32_t p = part[s][r];
        if (p < 0 || p >= nparts[s])
          fail(ADS_ERR_ARG, "part value out of range in system " + std::to_string(s));
        for (int64_t t = 0; t < rf; ++t) pg[c->sys_row[s] + rf * r + t] = p + c->sys_sub[s];
      }
      for (int q = c->sys_sub[s]; q < c->sys_sub[s + 1]; ++q) c->sub_sys[q] = s;
    }
    {
      int32_t h = 0;
      ADS_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, st));
      ADS_HIP(hipStreamSynchronize(st));
      if (h & 8) fail(ADS_ERR_NAN, "non-finite matrix entry");
      if (h) fail(ADS_ERR_ARG, "invalid CSR (row pointers, column range or column order)");
      ADS_LAUNCH(k_check_symmetric, dim3((unsigned)((c->n + 255) / 256)), dim3(256), 0, st,
                 c->rowptr, c->col, c->val, c->n, bad);
      ADS_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, st));
      ADS_HIP(hipStreamSynchronize(st));
      c->sym = h == 0;
    }
    c->sub_sys_d = upload(c->mem, c->sub_sys.data(), c->nsub, st);
    c->t_phase_ms[5] += tm.lap();
    build_maps(*c, pg);
    c->t_phase_ms[0] = tm.lap();
    extract_local(*c);
    c->t_phase_ms[1] = tm.lap();
    tune_tiles(*c);
    c->t_phase_ms[7] = tm.lap();
    {
      // per-subdomain launches take the longest chains first: decreasing
      // (2K - 1) s^2 (tile entries walked by one factorization or solve)
      std::vector<int32_t> ord(c->nsub);
      std::vector<int64_t> cost(c->nsub);
      for (int i = 0; i < c->nsub; ++i) {
        ord[i] = i;
        cost[i] = (int64_t)(2 * c->h_nb[i] - 1) * c->h_bs[i] * c->h_bs[i];
      }
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cost[x] > cost[y]; });
      c->sub_order = upload(c->mem, ord.data(), c->nsub, st);
    }
    factor_local(*c);
    c->local_resid = local_solve_accuracy(*c);
    // BF16 factors (8-bit significands) on strongly varying coefficients: a
    // local solve that leaves more than a quarter of its right-hand side
    // unresolved made FGMRES stall in every measured case (3D jumping
    // coefficients 64^3: 0.33, 128^3: 4.7), while the cases up to 0.12
    // converged
    if (c->prec == ADS_PREC_BF16 && !(c->local_resid <= BF16_MAX_LOCAL_RESID))
      fail(ADS_ERR_UNSUPPORTED,
           "BF16 local factors leave a local-solve relative residual of " +
               std::to_string(c->local_resid) + " (above " + std::to_string(BF16_MAX_LOCAL_RESID) +
               ") on this matrix; use ADS_PREC_FP32");
    c->t_phase_ms[2] = tm.lap();
    const bool coarse = variant_has_coarse(opts->variant) && opts->nev > 0;
    if (coarse) {
      if (opts->warm_start) {
        learned_start(*c);
        c->t_phase_ms[6] = tm.lap();
      }
      eigensolve(*c);
      c->t_phase_ms[3] = tm.lap();
      if (c->n0 > 0) {
        assemble_coarse(*c);
        c->t_phase_ms[4] = tm.lap();
      }
      if (c->facT) {
        c->mem.release(c->facT);
        c->facT = nullptr;
      }
    } else {
      c->n0 = 0;
      c->h_nev.assign(c->nsub, 0);
    }
    if (!variant_restricted(opts->variant)) build_cover(*c);
    ensure_work(*c, 1);
    ADS_HIP(hipStreamSynchronize(st));
    c->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  } catch (...) {
    (void)hipStreamSynchronize(st);
    delete c;
    throw;
  }
  return c;
}

}  // namespace ads

using namespace ads;


extern "C" {

int ads_setup(const ads_csr* A, const int32_t* part, int32_t nparts, const ads_options* opts,
              void* hip_stream, ads_ctx** out) {
  return ads_setup_batched(1, A, &part, &nparts, opts, hip_stream, out);
}

static int setup_entry(int32_t nsys, const ads_csr* A, const int32_t* const* part,
                       const int32_t* nparts, const ads_options* opts, void* hip_stream,
                       ads_ctx** out, bool cplx) {
  if (!out) {
    g_last_error = "out is NULL";
    return ADS_ERR_ARG;
  }
  *out = nullptr;
  try {
    Ctx* c = setup_impl(nsys, A, part, nparts, opts, (hipStream_t)hip_stream, cplx);
    *out = new ads_ctx{c};
    return ADS_OK;
  } catch (const Error& e) {
    return handle(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return ADS_ERR_OOM;
  } catch (...) {
    g_last_error = "unknown error";
    return ADS_ERR_HIP;
  }
}

int ads_setup_batched(int32_t nsys, const ads_csr* A, const int32_t* const* part,
                      const int32_t* nparts, const ads_options* opts, void* hip_stream,
                      ads_ctx** out) {
  return setup_entry(nsys, A, part, nparts, opts, hip_stream, out, false);
}

int ads_setup_complex(int32_t nsys, const ads_csr* A, const int32_t* const* part,
                      const int32_t* nparts, const ads_options* opts, void* hip_stream,
                      ads_ctx** out) {
  return setup_entry(nsys, A, part, nparts, opts, hip_stream, out, true);
}

int ads_apply(ads_ctx* ctx, const double* r_dev, double* z_dev, int32_t nrhs, void* hip_stream) {
  try {
    if (!ctx || !r_dev || !z_dev) fail(ADS_ERR_ARG, "null argument");
    if (nrhs < 1 || nrhs > 64) fail(ADS_ERR_ARG, "nrhs must be in [1, 64]");
    if (r_dev == z_dev) fail(ADS_ERR_ARG, "r and z must not alias");
    Ctx& c = *ctx->c;
    const hipStream_t st = (hipStream_t)hip_stream;
    if (c.graphs_on())
      on_own_stream(c, st, [&](hipStream_t ps) { apply_prec(c, r_dev, z_dev, nrhs, ps); });
    else
      apply_prec(c, r_dev, z_dev, nrhs, st);
    return ADS_OK;
  } catch (const Error& e) {
    return handle(e);
  } catch (...) {
    g_last_error = "unknown error";
    return ADS_ERR_HIP;
  }
}

int ads_apply_noalloc(ads_ctx* ctx, const double* r_dev, double* z_dev, int32_t nrhs,
                      void* hip_stream) {
  try {
    if (!ctx || !r_dev || !z_dev) fail(ADS_ERR_ARG, "null argument");
    if (nrhs < 1 || nrhs > 64) fail(ADS_ERR_ARG, "nrhs must be in [1, 64]");
    if (r_dev == z_dev) fail(ADS_ERR_ARG, "r and z must not alias");
    apply_noalloc(*ctx->c, r_dev, z_dev, nrhs, (hipStream_t)hip_stream);
    return ADS_OK;
  } catch (const Error& e) {
    return handle(e);
  } catch (...) {
    g_last_error = "unknown error";
    return ADS_ERR_HIP;
  }
}

int ads_solve(ads_ctx* ctx, const double* b_dev, double* x_dev, int32_t nrhs,
              const ads_ksp_options* kopts, ads_ksp_result* res, void* hip_stream) {
  try {
    if (!ctx || !b_dev || !x_dev || !kopts) fail(ADS_ERR_ARG, "null argument");
    if (nrhs < 1 || ctx->c->nsys * nrhs > ADS_MAX_RESULTS)
      fail(ADS_ERR_ARG, "nsys * nrhs must be in [1, 64]");
    if (kopts->restart < 1 || kopts->restart > 64) fail(ADS_ERR_ARG, "restart must be in [1, 64]");
    if (!(kopts->rtol >= 0.0)) fail(ADS_ERR_ARG, "rtol must be >= 0");
    if (b_dev == x_dev) fail(ADS_ERR_ARG, "b and x must not alias");
    if (res) std::memset(res, 0, sizeof(*res));
    Ctx& c = *ctx->c;
    const hipStream_t st = (hipStream_t)hip_stream;
    if (!c.graphs_on()) return gmres_solve(c, b_dev, x_dev, nrhs, *kopts, res, st);
    int status = ADS_OK;
    on_own_stream(c, st, [&](hipStream_t ps) {
      status = gmres_solve(c, b_dev, x_dev, nrhs, *kopts, res, ps);
    });
    return status;
  } catch (const Error& e) {
    return handle(e);
  } catch (...) {
    g_last_error = "unknown error";
    return ADS_ERR_HIP;
  }
}

int ads_get_info(const ads_ctx* ctx, ads_info* info) {
  try {
    if (!ctx || !info) fail(ADS_ERR_ARG, "null argument");
    const Ctx& c = *ctx->c;
    info->n = c.n;
    info->omega_total = c.omega_total;
    info->factor_bytes = c.factor_bytes;
    info->nsys = c.nsys;
    info->nsub = c.nsub;
    info->n0 = c.n0;
    info->eig_sweeps_max = c.eig_sweeps_max;
    info->eig_unconverged = c.eig_unconverged;
    info->eig_fallbacks = c.eig_fallbacks;
    info->eig_solver = c.eig_krylov_schur ? ADS_EIG_KRYLOV_SCHUR : ADS_EIG_SUBSPACE;
    info->tile_factor = c.tile_factor;
    info->tile_tuned = c.tile_tuned;
    for (int k = 0; k < 8; ++k) info->t_phase_ms[k] = c.t_phase_ms[k];
    ctx->c->prof_resolve();
    for (int k = 0; k < 4; ++k) {
      info->t_kernel_ms[k] = c.prof_ms[k];
      info->n_kernel[k] = c.prof_n[k];
    }
    info->local_resid = c.local_resid;
    info->is_complex = c.cplx;
    info->t_mfma_update_ms = c.prof_gj_ms;
    info->n_mfma_update = c.prof_gj_n;
    info->mfma_update_flops = c.prof_gj_flops;
    for (int i = 0; i < c.nsub; ++i) {
      if (info->nev_i) info->nev_i[i] = c.h_nev.empty() ? 0 : c.h_nev[i];
      if (info->kernel_dim) info->kernel_dim[i] = c.h_kdim[i];
      if (info->n_i) info->n_i[i] = c.h_ni[i];
      if (info->n_interior) info->n_interior[i] = c.h_nI[i];
      if (info->sweeps) info->sweeps[i] = c.h_sweeps.empty() ? 0 : c.h_sweeps[i];
      if (info->block) info->block[i] = c.h_bs[i];
      if (info->eig_resid) info->eig_resid[i] = c.h_eig_res.empty() ? 0.0 : c.h_eig_res[i];
    }
    return ADS_OK;
  } catch (const Error& e) {
    return handle(e);
  }
}

int ads_export_maps(const ads_ctx* ctx, int32_t* omega_concat, int64_t* omega_off,
                    int32_t* n_interior, int32_t* layer) {
  try {
    if (!ctx) fail(ADS_ERR_ARG, "null context");
    const Ctx& c = *ctx->c;
    std::vector<int32_t> tmp;
    if (omega_concat) {
      download(tmp, c.om_export, c.omega_total, c.stream);
      std::memcpy(omega_concat, tmp.data(), tmp.size() * 4);
    }
    if (layer) {
      download(tmp, c.om_layer, c.omega_total, c.stream);
      std::memcpy(layer, tmp.data(), tmp.size() * 4);
    }
    if (omega_off) std::memcpy(omega_off, c.h_om_off.data(), (c.nsub + 1) * 8);
    if (n_interior) std::memcpy(n_interior, c.h_nI.data(), c.nsub * 4);
    return ADS_OK;
  } catch (const Error& e) {
    return handle(e);
  }
}

int ads_export_splitting(const ads_ctx* ctx, double* s_out) {
  try {
    if (!ctx || !s_out) fail(ADS_ERR_ARG, "null argument");
    const Ctx& c = *ctx->c;
    // lsum is in the sorted order; map to the export order [I, Gamma]
    std::vector<double> ls;
    std::vector<int32_t> srt, exp;
    download(ls, c.lsum, c.omega_total, c.stream);
    download(srt, c.om_sorted, c.omega_total, c.stream);
    download(exp, c.om_export, c.omega_total, c.stream);
    for (int i = 0; i < c.nsub; ++i) {
      const int64_t b = c.h_om_off[i], e = c.h_om_off[i + 1];
      for (int64_t k = b; k < e; ++k) {
        // export slot k holds global id exp[k]; find it in the sorted list
        auto it = std::lower_bound(srt.begin() + b, srt.begin() + e, exp[k]);
        s_out[k] = ls[it - srt.begin()];
      }
    }
    return ADS_OK;
  } catch (const Error& e) {
    return handle(e);
  }
}

int ads_export_coarse(const ads_ctx* ctx, double* W, int64_t* W_off, double* lam_re,
                      double* lam_im) {
  try {
    if (!ctx) fail(ADS_ERR_ARG, "null context");
    const Ctx& c = *ctx->c;
    if (W && c.n0 > 0) {
      std::vector<double> hw;
      download(hw, c.W, c.h_W_off[c.nsub], c.stream);
      std::memcpy(W, hw.data(), hw.size() * 8);
    }
    if (W_off) {
      for (int i = 0; i <= c.nsub; ++i) W_off[i] = c.h_W_off.empty() ? 0 : c.h_W_off[i];
    }
    for (size_t k = 0; k < c.h_lam_re.size(); ++k) {
      if (lam_re) lam_re[k] = c.h_lam_re[k];
      if (lam_im) lam_im[k] = c.h_lam_im[k];
    }
    return ADS_OK;
  } catch (const Error& e) {
    return handle(e);
  }
}

int ads_partition_bfs(const ads_csr* A, int32_t nparts, const int32_t* seeds, int32_t* part_out,
                      void* hip_stream) {
  try {
    if (!A || !seeds || !part_out) fail(ADS_ERR_ARG, "null argument");
    hipStream_t st = (hipStream_t)hip_stream;
    HostCSR h;
    to_host(*A, h, st);
    check_csr_host(h.view, 0);
    if (nparts <= 0 || nparts > h.view.n) fail(ADS_ERR_ARG, "nparts out of range");
    std::vector<int32_t> sd(seeds, seeds + nparts);
    {
      std::vector<int32_t> chk = sd;
      std::sort(chk.begin(), chk.end());
      for (int k = 0; k < nparts; ++k) {
        if (chk[k] < 0 || chk[k] >= h.view.n) fail(ADS_ERR_ARG, "seed out of range");
        if (k && chk[k] == chk[k - 1]) fail(ADS_ERR_ARG, "seeds must be distinct");
      }
    }
    Arena mem(st);
    std::vector<int32_t> rp(h.view.n + 1);
    for (int64_t r = 0; r <= h.view.n; ++r) rp[r] = (int32_t)h.view.row_ptr[r];
    int32_t* d_rp = upload(mem, rp.data(), rp.size(), st);
    int32_t* d_ci = upload(mem, h.view.col, h.view.nnz, st);
    std::vector<int32_t> part;
    bfs_partition(d_rp, d_ci, h.view.n, h.view.nnz, sd, part, st);
    std::memcpy(part_out, part.data(), part.size() * 4);
    return ADS_OK;
  } catch (const Error& e) {
    return handle(e);
  }
}

int ads_set_graphs(ads_ctx* ctx, int32_t enable) {
  try {
    if (!ctx) fail(ADS_ERR_ARG, "null argument");
    Ctx& c = *ctx->c;
    if (c.priv) ADS_HIP(hipStreamSynchronize(c.priv));
    c.drop_apply_graph();
    c.use_graphs = enable != 0;
    return ADS_OK;
  } catch (const Error& e) {
    return handle(e);
  } catch (...) {
    g_last_error = "unknown error";
    return ADS_ERR_HIP;
  }
}

int ads_destroy(ads_ctx* ctx) {
  if (!ctx) return ADS_OK;
  delete ctx->c;
  delete ctx;
  return ADS_OK;
}

const char* ads_status_string(int status) {
  switch (status) {
    case ADS_OK: return "ADS_OK";
    case ADS_KSP_MAXIT: return "ADS_KSP_MAXIT";
    case ADS_KSP_BREAKDOWN: return "ADS_KSP_BREAKDOWN";
    case ADS_ERR_ARG: return "ADS_ERR_ARG";
    case ADS_ERR_HIP: return "ADS_ERR_HIP";
    case ADS_ERR_OOM: return "ADS_ERR_OOM";
    case ADS_ERR_SINGULAR: return "ADS_ERR_SINGULAR";
    case ADS_ERR_EIG_NOCONV: return "ADS_ERR_EIG_NOCONV";
    case ADS_ERR_NAN: return "ADS_ERR_NAN";
    case ADS_ERR_UNSUPPORTED: return "ADS_ERR_UNSUPPORTED";
    default: return "unknown status";
  }
}

const char* ads_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
