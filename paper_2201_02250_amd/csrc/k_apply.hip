// Preconditioner apply, eq. 4 of Section 2 (restricted two-level Schwarz with
// deflated coarse correction), or eq. 3 (RAS) without a coarse space:
//
//   c = R_0 r             k_coarse_restrict   (W_i^T r|Omega_Ii, per subdomain)
//   y = A_00^{-1} c       k_coarse_prolong    (rows of the explicit inverse of E,
//   q = R_0^T y                                then W_i y_i on Omega_Ii)
//   t = r - A q           k_local_solve       (gathered on Omega_i from the CSR)
//   x_i = A_ii^{-1} t|Omega_i                  (block-tridiagonal tiles)
//   z = q + sum_i R_i^T D_i x_i               (Boolean D: owner rows only)
//
// Three launches per apply.  With the Boolean partition of unity every global
// row is written by exactly one subdomain, so no atomics are needed.
#include "ads_internal.h"
#include "k_solve.h"

namespace ads {

static constexpr int APPLY_T = 256;
static constexpr int MAXNEV = 32;

__global__ void __launch_bounds__(APPLY_T)
k_coarse_restrict(const double* __restrict__ r, int64_t n, const int32_t* __restrict__ int_list,
                  const int64_t* __restrict__ om_off, const int32_t* __restrict__ nI,
                  const double* __restrict__ W, const int64_t* __restrict__ W_off,
                  const int32_t* __restrict__ nev, const int32_t* __restrict__ coff,
                  double* __restrict__ c, int n0) {
  __shared__ double red[16];
  const int i = blockIdx.x, j = blockIdx.y;
  const int m = nev[i];
  if (m == 0) return;
  const int nint = nI[i];
  const int32_t* rows = int_list + om_off[i];
  const double* Wi = W + W_off[i];
  const double* rj = r + (int64_t)j * n;
  double acc[MAXNEV];
#pragma unroll
  for (int a = 0; a < MAXNEV; ++a) acc[a] = 0.0;
  for (int k = threadIdx.x; k < nint; k += blockDim.x) {
    const double rv = rj[rows[k]];
    const double* w = Wi + (int64_t)k * m;
#pragma unroll
    for (int a = 0; a < MAXNEV; ++a)
      if (a < m) acc[a] += w[a] * rv;
  }
#pragma unroll
  for (int a = 0; a < MAXNEV; ++a) {
    if (a < m) {
      double v = adsd::block_sum(acc[a], red);
      if (threadIdx.x == 0) c[(int64_t)j * n0 + coff[i] + a] = v;
    }
  }
}

__global__ void __launch_bounds__(APPLY_T)
k_coarse_prolong(const double* __restrict__ c, int n0, const double* __restrict__ Einv,
                 const int64_t* __restrict__ E_off, const int32_t* __restrict__ sys_coff,
                 const int32_t* __restrict__ sub_sys, const int32_t* __restrict__ int_list,
                 const int64_t* __restrict__ om_off, const int32_t* __restrict__ nI,
                 const double* __restrict__ W, const int64_t* __restrict__ W_off,
                 const int32_t* __restrict__ nev, const int32_t* __restrict__ coff,
                 double* __restrict__ q, int64_t n) {
  __shared__ double red[16];
  __shared__ double y[MAXNEV];
  const int i = blockIdx.x, j = blockIdx.y;
  const int m = nev[i];
  const int nint = nI[i];
  const int32_t* rows = int_list + om_off[i];
  double* qj = q + (int64_t)j * n;
  if (m == 0) {
    for (int k = threadIdx.x; k < nint; k += blockDim.x) qj[rows[k]] = 0.0;
    return;
  }
  const int sy = sub_sys[i];
  const int c0 = sys_coff[sy], ns = sys_coff[sy + 1] - c0;
  const double* cj = c + (int64_t)j * n0 + c0;
  const double* E = Einv + E_off[sy];
  const int row0 = coff[i] - c0;
  for (int a = 0; a < m; ++a) {
    const double* er = E + (int64_t)(row0 + a) * ns;
    double acc = 0.0;
    for (int b = threadIdx.x; b < ns; b += blockDim.x) acc += er[b] * cj[b];
    acc = adsd::block_sum(acc, red);
    if (threadIdx.x == 0) y[a] = acc;
  }
  __syncthreads();
  const double* Wi = W + W_off[i];
  for (int k = threadIdx.x; k < nint; k += blockDim.x) {
    const double* w = Wi + (int64_t)k * m;
    double v = 0.0;
    for (int a = 0; a < m; ++a) v += w[a] * y[a];
    qj[rows[k]] = v;
  }
}

template <class FT, int P>
__global__ void __launch_bounds__(APPLY_T)
k_local_solve(const FT* __restrict__ fac, const int64_t* __restrict__ fac_off,
              const int32_t* __restrict__ bsz, const int32_t* __restrict__ nblk,
              const int32_t* __restrict__ ni, const int64_t* __restrict__ om_off,
              const int32_t* __restrict__ om_sorted, const uint8_t* __restrict__ om_int,
              const int64_t* __restrict__ lrow, const int32_t* __restrict__ lcol,
              const double* __restrict__ lval, const int32_t* __restrict__ rowptr,
              const int32_t* __restrict__ col, const double* __restrict__ val,
              const double* __restrict__ r, const double* __restrict__ q, double* __restrict__ z,
              int64_t n, int nrhs, double* __restrict__ work, const int64_t* __restrict__ pad_off,
              int64_t ldw) {
  extern __shared__ double lds[];
  const int i = blockIdx.x;
  const int j0 = blockIdx.y * P;
  const int pc = min(P, nrhs - j0);
  const int s = bsz[i], K = nblk[i], ns = ni[i];
  const int64_t base = om_off[i];
  const int32_t* om = om_sorted + base;
  double* X = work + pad_off[i] + (int64_t)j0 * ldw;
  const int npad = K * s;
  // gather t = r - A q on Omega_i (zero on the padding)
  for (int e = threadIdx.x; e < npad * pc; e += blockDim.x) {
    const int lr = e % npad, jj = e / npad;
    double v = 0.0;
    if (lr < ns) {
      const int g = om[lr];
      const int64_t off = (int64_t)(j0 + jj) * n;
      v = r[off + g];
      if (q) {
        double aq = 0.0;
        for (int k = rowptr[g]; k < rowptr[g + 1]; ++k) aq += val[k] * q[off + col[k]];
        v -= aq;
      }
    }
    X[lr + (int64_t)jj * ldw] = v;
  }
  __syncthreads();
  adsd::block_solve<FT, P>(fac + fac_off[i], s, K, ns, lrow + base, lcol, lval, X, ldw, pc, lds);
  // z = q + R_i^T D_i x_i (interior rows only)
  for (int e = threadIdx.x; e < ns * pc; e += blockDim.x) {
    const int lr = e % ns, jj = e / ns;
    if (!om_int[base + lr]) continue;
    const int g = om[lr];
    const int64_t off = (int64_t)(j0 + jj) * n;
    double v = X[lr + (int64_t)jj * ldw];
    if (q) v += q[off + g];
    z[off + g] = v;
  }
}

void ensure_work(Ctx& c, int cols) {
  if (c.work_cols >= cols) return;
  if (c.work) c.mem.release(c.work);
  if (c.cvec) c.mem.release(c.cvec);
  if (c.qvec) c.mem.release(c.qvec);
  c.work = c.mem.alloc<double>((size_t)c.npad_total * cols);
  c.cvec = c.mem.alloc<double>((size_t)std::max(c.n0, 1) * cols);
  c.qvec = c.mem.alloc<double>((size_t)c.n * cols);
  c.work_cols = cols;
}

template <class FT, int P>
static void launch_local(Ctx& c, const double* r, const double* q, double* z, int nrhs,
                         hipStream_t s) {
  size_t lds = (size_t)adsd::solve_lds_doubles<P>(c.h_bs, APPLY_T) * sizeof(double);
  dim3 grid(c.nsub, (nrhs + P - 1) / P);
  ADS_LAUNCH((k_local_solve<FT, P>), grid, dim3(APPLY_T), lds, s, (const FT*)c.facA, c.fac_off,
             c.bs, c.nb, c.ni, c.om_off, c.om_sorted, c.om_int, c.lptr_off, c.lcol, c.lval,
             c.rowptr, c.col, c.val, r, q, z, c.n, nrhs, c.work, c.pad_off, c.npad_total);
}

template <class FT>
static void local_dispatch(Ctx& c, const double* r, const double* q, double* z, int nrhs,
                           hipStream_t s) {
  if (nrhs == 1)
    launch_local<FT, 1>(c, r, q, z, nrhs, s);
  else if (nrhs <= 4)
    launch_local<FT, 4>(c, r, q, z, nrhs, s);
  else
    launch_local<FT, 8>(c, r, q, z, nrhs, s);
}

void apply_prec(Ctx& c, const double* r, double* z, int nrhs, hipStream_t s) {
  ensure_work(c, nrhs);
  const double* q = nullptr;
  if (c.n0 > 0) {
    ADS_LAUNCH(k_coarse_restrict, dim3(c.nsub, nrhs), dim3(APPLY_T), 0, s, r, c.n, c.int_list,
               c.om_off, c.nI, c.W, c.W_off, c.nev, c.coff, c.cvec, c.n0);
    ADS_LAUNCH(k_coarse_prolong, dim3(c.nsub, nrhs), dim3(APPLY_T), 0, s, c.cvec, c.n0, c.Einv,
               c.E_off, c.sys_coff, c.sub_sys_d, c.int_list, c.om_off, c.nI, c.W, c.W_off, c.nev,
               c.coff, c.qvec, c.n);
    q = c.qvec;
  }
  switch (c.prec) {
    case ADS_PREC_FP64: local_dispatch<double>(c, r, q, z, nrhs, s); break;
    case ADS_PREC_FP32: local_dispatch<float>(c, r, q, z, nrhs, s); break;
    default: local_dispatch<__hip_bfloat16>(c, r, q, z, nrhs, s); break;
  }
}

}  // namespace ads
