// Preconditioner apply, eq. 4 of Section 2 (restricted two-level Schwarz with
// deflated coarse correction), or eq. 3 (RAS) without a coarse space:
//
//   c = R_0 r             k_coarse_restrict_mf (W_i^T r|Omega_Ii on the matrix
//                                              cores, partial sums per chunk of
//                                              512 rows of Omega_Ii)
//   y = A_00^{-1} c       k_coarse_prolong    (c summed from the partials, rows
//   q = R_0^T y                                of the explicit inverse of E,
//                                              then W_i y_i per chunk of rows;
//                                              a large E: k_coarse_csum,
//                                              k_coarse_emul_mf on the matrix
//                                              cores, k_coarse_prolong_all)
//   t = r - A q           k_local_solve       (gathered on Omega_i from the CSR)
//   x_i = A_ii^{-1} t|Omega_i                  (block-tridiagonal tiles)
//   z = q + sum_i R_i^T D_i x_i               (Boolean D: owner rows only)
//
// Three launches per apply.  With the Boolean partition of unity every global
// row is written by exactly one subdomain, so no atomics are needed.
//
// The other variants of Section 2 reuse the same kernels: eq. 3 (RAS) skips
// the coarse part; the additive forms (eq. 2 and its restricted version) form
// q = R_0^T A_00^{-1} R_0 r but solve the local problems on r itself; eq. 1
// and eq. 2 prolong every local solution on all of Omega_i, summed per global
// row over the subdomains that contain it in ascending order (k_prolong_sum,
// from a row -> slots map built once).
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "ads_internal.h"
#include "k_solve.h"

namespace ads {

static constexpr int APPLY_T = 256;
static constexpr int MAXNEV = 32;

// rows of Omega_Ii per block of the coarse restriction and prolongation
static constexpr int CO_CH = 2 * APPLY_T;

// E^{-1} larger than 16 MB: y = E^{-1} c in a pass of its own (k_coarse_emul_mf)
bool coarse_big(const Ctx& c) {
  return c.n0 > 0 && !c.h_E_off.empty() && c.h_E_off.back() * 8 > ((int64_t)16 << 20);
}

int coarse_chunks(const Ctx& c) {
  int mx = 1;
  for (int i = 0; i < c.nsub; ++i) mx = std::max(mx, (c.h_nI[i] + CO_CH - 1) / CO_CH);
  return mx;
}

// one DPP step of a wave sum: x + x of the lane given by CTRL (the pairs are
// symmetric, so both lanes of a pair hold the same value afterwards)
template <int CTRL>
__device__ __forceinline__ double co_dpp_add(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return x + __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double co_lane(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// deterministic sum over the 64 lanes (every lane active): pairs, quads, half
// rows and rows of 16 by DPP, then the four rows by readlane; uniform result
__device__ __forceinline__ double co_wave_sum(double x) {
  x = co_dpp_add<0xB1>(x);
  x = co_dpp_add<0x4E>(x);
  x = co_dpp_add<0x141>(x);
  x = co_dpp_add<0x140>(x);
  return (co_lane(x, 0) + co_lane(x, 16)) + (co_lane(x, 32) + co_lane(x, 48));
}

// out[a stride] = sum over the block of acc[a], a < m (fixed order; threads
// t < m write)
template <int N>
__device__ __forceinline__ void co_block_sums(const double (&acc)[N], int m,
                                              double (*red)[APPLY_T / 64], double* out,
                                              int64_t stride) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int a = 0; a < N; ++a)
    if (a < m) {
      const double sw = co_wave_sum(acc[a]);
      if (lane == 0) red[a][wv] = sw;
    }
  __syncthreads();
  if (t < m) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < APPLY_T / 64; ++w) v += red[t][w];
    out[(int64_t)t * stride] = v;
  }
}

// Partial sums of c = W_i^T r|Omega_Ii over the rows of chunk ch,
// part[(j n0 + coff_i + a) nch + ch], for up to 16 right-hand sides per
// workgroup (blockIdx.z: the group of 16) on the matrix cores: c_i = W_i^T R_i over the
// chunk's rows, the rows the K dimension.  Wave w takes rows k0 + 128 w ..
// + 127 in steps of four (v_mfma_f64_16x16x4f64; lane l supplies
// A(l % 16, l / 16) = W_i(row, a) and B(l / 16, l % 16) = r(row, j)), one
// product per 16 coarse vectors; the four waves' 16 x 16 tiles are then
// added in order through LDS.  W_i and r are read once per apply, whatever
// the number of right-hand sides.
typedef double co_d4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(APPLY_T)
k_coarse_restrict_mf(const double* __restrict__ r, int64_t n, const int32_t* __restrict__ int_list,
                     const int64_t* __restrict__ om_off, const int32_t* __restrict__ nI,
                     const double* __restrict__ W, const int64_t* __restrict__ W_off,
                     const int32_t* __restrict__ nev, const int32_t* __restrict__ coff,
                     double* __restrict__ part, int n0, int nch, int nrhs) {
  __shared__ double red[APPLY_T / 64][2][16][17];
  const int i = blockIdx.x, ch = blockIdx.y, j0 = blockIdx.z * 16;
  const int m = nev[i];
  if (m == 0) return;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int kc0 = ch * CO_CH, kc1 = min(nI[i], kc0 + CO_CH);
  const int kw0 = kc0 + wv * (CO_CH / 4), kw1 = min(kc1, kw0 + CO_CH / 4);
  const int32_t* rows = int_list + om_off[i];
  const double* Wi = W + W_off[i];
  const int j = j0 + li;
  const double* rj = r + (int64_t)min(j, nrhs - 1) * n;
  co_d4 acc[2];
  acc[0] = co_d4{0.0, 0.0, 0.0, 0.0};
  acc[1] = co_d4{0.0, 0.0, 0.0, 0.0};
  const int ntile = (m + 15) / 16;
  for (int kk = kw0; kk < kw1; kk += 4) {
    const int k = kk + lk;
    const bool ok = k < kw1;
    const int g = rows[ok ? k : kw0];
    const double bv = (ok && j < nrhs) ? rj[g] : 0.0;
    const double* wr = Wi + (int64_t)(ok ? k : kw0) * m;
    const double a0 = (ok && li < m) ? wr[li] : 0.0;
    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv, acc[0], 0, 0, 0);
    if (ntile > 1) {
      const double a1 = (ok && 16 + li < m) ? wr[16 + li] : 0.0;
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv, acc[1], 0, 0, 0);
    }
  }
  // accumulator register q of lane l: D(l / 16 + 4 q, l % 16) = c(a, j)
  for (int tt = 0; tt < ntile; ++tt)
#pragma unroll
    for (int q = 0; q < 4; ++q) red[wv][tt][lk + 4 * q][li] = acc[tt][q];
  __syncthreads();
  for (int e = t; e < ntile * 256; e += APPLY_T) {
    const int tt = e >> 8, a = 16 * tt + ((e >> 4) & 15), jj = e & 15;
    if (a >= m || j0 + jj >= nrhs) continue;
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < APPLY_T / 64; ++w) v += red[w][tt][a - 16 * tt][jj];
    part[((int64_t)(j0 + jj) * n0 + coff[i] + a) * nch + ch] = v;
  }
}

// Large coarse systems (E^{-1} beyond the caches): y = E^{-1} c is formed once
// per apply instead of once per (subdomain chunk, right-hand side), so that
// E^{-1} streams from HBM once.  First c = the sum of the restriction's
// partials (fixed order), cy[j n0 + b] ...
__global__ void k_coarse_csum(const double* __restrict__ part, int n0, int nch, int nrhs,
                              double* __restrict__ cy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n0 * nrhs) return;
  double v = 0.0;
  for (int h = 0; h < nch; ++h) v += part[e * nch + h];
  cy[e] = v;
}

// ... then y = E^{-1} c on the matrix cores: a 16-row tile of E^{-1} (blockIdx.x) of
// system blockIdx.y by 16 right-hand sides (blockIdx.z); the four waves take
// four contiguous quarters of the columns (multiples of 64) and add their
// tiles in order at the end.  Per 64 columns a wave loads its 16 rows of
// E^{-1} and 16 columns of c row by row (64 consecutive doubles per load,
// one 512-byte line run) into a wave-private LDS tile, the next chunk's
// loads in flight during the products; lane l then takes column
// k0 + 16 (l / 16) + s of both tiles in product s (the same column for both
// operands, each column once).  E^{-1} streams from HBM once per apply.
static constexpr int EM_LD = 64 + 1;
__global__ void __launch_bounds__(256)
k_coarse_emul_mf(const double* __restrict__ cy, int n0, int nrhs, const double* __restrict__ Einv,
                 const int64_t* __restrict__ E_off, const int32_t* __restrict__ sys_coff,
                 double* __restrict__ y) {
  __shared__ double Es[4][16 * EM_LD];
  __shared__ double Cs[4][16 * EM_LD];
  __shared__ double red[4][16][17];
  const int sy = blockIdx.y;
  const int c0 = sys_coff[sy], ns = sys_coff[sy + 1] - c0;
  const int r0 = blockIdx.x * 16, j0 = blockIdx.z * 16;
  if (r0 >= ns) return;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int nk = (ns + 63) / 64, per = (nk + 3) / 4;
  const int kb0 = min(ns, wv * per * 64), kb1 = min(ns, (wv + 1) * per * 64);
  const double* E = Einv + E_off[sy];
  double* es = Es[wv];
  double* cs = Cs[wv];
  double ev[16], cv[16];
  // row rho of the E tile and column rho of the c tile, entry k0 + lane
  auto load = [&](int k0) {
    const int k = k0 + lane;
    const bool kin = k < ns;
#pragma unroll
    for (int rho = 0; rho < 16; ++rho) {
      const int row = r0 + rho, col = j0 + rho;
      ev[rho] = (kin && row < ns) ? E[(int64_t)row * ns + k] : 0.0;
      cv[rho] = (kin && col < nrhs) ? cy[(int64_t)col * n0 + c0 + k] : 0.0;
    }
  };
  co_d4 acc = co_d4{0.0, 0.0, 0.0, 0.0};
  if (kb0 < kb1) load(kb0);
  // every wave runs the same number of chunks (barriers inside)
  for (int c = 0; c < per; ++c) {
    const int k0 = kb0 + 64 * c;
    __syncthreads();  // the previous chunk's reads of the tiles are done
#pragma unroll
    for (int rho = 0; rho < 16; ++rho) {
      es[rho * EM_LD + lane] = ev[rho];
      cs[rho * EM_LD + lane] = cv[rho];
    }
    __syncthreads();
    if (k0 + 64 < kb1) load(k0 + 64);  // in flight during the products
    if (k0 < kb1) {
#pragma unroll
      for (int q = 0; q < 16; ++q)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(es[li * EM_LD + 16 * lk + q],
                                                   cs[li * EM_LD + 16 * lk + q], acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) red[wv][lk + 4 * q][li] = acc[q];
  __syncthreads();
  {
    const int a = t >> 4, jj = t & 15;  // 256 threads: the 16 x 16 tile
    if (r0 + a < ns && j0 + jj < nrhs) {
      const double v = red[0][a][jj] + red[1][a][jj] + red[2][a][jj] + red[3][a][jj];
      y[(int64_t)(j0 + jj) * n0 + c0 + r0 + a] = v;
    }
  }
}

// q = W_i y_i on the rows of chunk ch for every right-hand side (y from
// k_coarse_emul_mf): y_i in LDS, the row of W_i in registers, read once
__global__ void __launch_bounds__(APPLY_T)
k_coarse_prolong_all(const double* __restrict__ yfull, int n0, int nrhs,
                     const int32_t* __restrict__ int_list, const int64_t* __restrict__ om_off,
                     const int32_t* __restrict__ nI, const double* __restrict__ W,
                     const int64_t* __restrict__ W_off, const int32_t* __restrict__ nev,
                     const int32_t* __restrict__ coff, double* __restrict__ q, int64_t n) {
  __shared__ double ys[64][MAXNEV];
  const int i = blockIdx.x, ch = blockIdx.y;
  const int m = nev[i];
  const int k0 = ch * CO_CH, k1 = min(nI[i], k0 + CO_CH);
  if (k0 >= k1) return;
  const int32_t* rows = int_list + om_off[i];
  if (m == 0) {
    for (int e = threadIdx.x; e < (k1 - k0) * nrhs; e += APPLY_T)
      q[(int64_t)(e / (k1 - k0)) * n + rows[k0 + e % (k1 - k0)]] = 0.0;
    return;
  }
  for (int e = threadIdx.x; e < nrhs * m; e += APPLY_T)
    ys[e / m][e % m] = yfull[(int64_t)(e / m) * n0 + coff[i] + e % m];
  __syncthreads();
  const double* Wi = W + W_off[i];
  for (int k = k0 + threadIdx.x; k < k1; k += APPLY_T) {
    double wr[MAXNEV];
#pragma unroll
    for (int a = 0; a < MAXNEV; ++a) wr[a] = a < m ? Wi[(int64_t)k * m + a] : 0.0;
    const int g = rows[k];
    for (int j = 0; j < nrhs; ++j) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < MAXNEV; ++a)
        if (a < m) v += wr[a] * ys[j][a];
      q[(int64_t)j * n + g] = v;
    }
  }
}

// Small E: y_i = rows coff_i .. coff_i + m of E^{-1} times c (c summed from
// the restriction's partials in a fixed order), then q = W_i y_i on the rows
// of chunk ch
__global__ void __launch_bounds__(APPLY_T)
k_coarse_prolong(const double* __restrict__ part, int n0,
                 int nch, const double* __restrict__ Einv,
                 const int64_t* __restrict__ E_off, const int32_t* __restrict__ sys_coff,
                 const int32_t* __restrict__ sub_sys, const int32_t* __restrict__ int_list,
                 const int64_t* __restrict__ om_off, const int32_t* __restrict__ nI,
                 const double* __restrict__ W, const int64_t* __restrict__ W_off,
                 const int32_t* __restrict__ nev, const int32_t* __restrict__ coff,
                 double* __restrict__ q, int64_t n) {
  __shared__ double red[MAXNEV][APPLY_T / 64];
  __shared__ double y[MAXNEV];
  const int i = blockIdx.x, ch = blockIdx.y, j = blockIdx.z;
  const int m = nev[i];
  const int k0 = ch * CO_CH, k1 = min(nI[i], k0 + CO_CH);
  if (k0 >= k1) return;
  const int32_t* rows = int_list + om_off[i];
  double* qj = q + (int64_t)j * n;
  if (m == 0) {
    for (int k = k0 + threadIdx.x; k < k1; k += APPLY_T) qj[rows[k]] = 0.0;
    return;
  }
  {
    const int sy = sub_sys[i];
    const int c0 = sys_coff[sy], ns = sys_coff[sy + 1] - c0;
    const double* pj = part + ((int64_t)j * n0 + c0) * nch;
    const double* E = Einv + E_off[sy] + (int64_t)(coff[i] - c0) * ns;
    double acc[MAXNEV];
#pragma unroll
    for (int a = 0; a < MAXNEV; ++a) acc[a] = 0.0;
    for (int b = threadIdx.x; b < ns; b += APPLY_T) {
      double cb = 0.0;
      for (int h = 0; h < nch; ++h) cb += pj[(int64_t)b * nch + h];
#pragma unroll
      for (int a = 0; a < MAXNEV; ++a)
        if (a < m) acc[a] += E[(int64_t)a * ns + b] * cb;
    }
    co_block_sums(acc, m, red, y, 1);
  }
  __syncthreads();
  const double* Wi = W + W_off[i];
  for (int k = k0 + threadIdx.x; k < k1; k += APPLY_T) {
    const double* w = Wi + (int64_t)k * m;
    double v = 0.0;
    for (int a = 0; a < m; ++a) v += w[a] * y[a];
    qj[rows[k]] = v;
  }
}

// gather t = r - A q on local rows [lo, hi) of Omega_i (zero on the padding)
// into X (column jj at X + jj*ld)
template <int P>
__device__ __forceinline__ void gather_local(const int32_t* __restrict__ om, int ns, int lo, int hi,
                                             const int32_t* __restrict__ rowptr,
                                             const int32_t* __restrict__ col,
                                             const double* __restrict__ val,
                                             const double* __restrict__ r,
                                             const double* __restrict__ q, int64_t n, int j0, int pc,
                                             double* X, int64_t ld) {
  const int len = hi - lo;
  if (P == 1 || pc == 1) {
    for (int e = threadIdx.x; e < len * pc; e += blockDim.x) {
      const int lr = lo + e % len, jj = e / len;
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
      X[lr + (int64_t)jj * ld] = v;
    }
    return;
  }
  // several columns: one row per thread, the row's pattern read once and the
  // q entries of all columns fetched together (same summation order)
  for (int e = threadIdx.x; e < len; e += blockDim.x) {
    const int lr = lo + e;
    double v[P];
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = 0.0;
    if (lr < ns) {
      const int g = om[lr];
#pragma unroll
      for (int j = 0; j < P; ++j)
        if (j < pc) v[j] = r[(int64_t)(j0 + j) * n + g];
      if (q) {
        double aq[P];
#pragma unroll
        for (int j = 0; j < P; ++j) aq[j] = 0.0;
        for (int k = rowptr[g]; k < rowptr[g + 1]; ++k) {
          const int c = col[k];
          const double a = val[k];
#pragma unroll
          for (int j = 0; j < P; ++j)
            if (j < pc) aq[j] += a * q[(int64_t)(j0 + j) * n + c];
        }
#pragma unroll
        for (int j = 0; j < P; ++j) v[j] -= aq[j];
      }
    }
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (j < pc) X[lr + (int64_t)j * ld] = v[j];
  }
}

// z = q + R_i^T D_i x_i on the interior rows among local rows [lo, hi)
// (Boolean partition of unity)
__device__ __forceinline__ void scatter_local(const int32_t* __restrict__ om,
                                              const uint8_t* __restrict__ om_int, int lo, int hi,
                                              const double* __restrict__ q, double* __restrict__ z,
                                              int64_t n, int j0, int pc, const double* X,
                                              int64_t ld) {
  const int len = hi - lo;
  for (int e = threadIdx.x; e < len * pc; e += blockDim.x) {
    const int lr = lo + e % len, jj = e / len;
    if (!om_int[lr]) continue;
    const int g = om[lr];
    const int64_t off = (int64_t)(j0 + jj) * n;
    double v = X[lr + (int64_t)jj * ld];
    if (q) v += q[off + g];
    z[off + g] = v;
  }
}

struct LocalArgs {
  const int64_t* fac_off;
  const int32_t* bs;
  const int32_t* nb;
  const int32_t* ni;
  const int64_t* om_off;
  const int32_t* om_sorted;
  const uint8_t* om_int;
  const int64_t* lrow;
  const int32_t* lcol;
  const double* lval;
  const int32_t* cpl_col;   // A_k,k-1 by row
  const double* cpl_val;
  const int32_t* rcpl_col;  // A_k,k+1 by row
  const double* rcpl_val;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const int64_t* pad_off;
  int cpl_ok;     // the coupling lists are complete
  double* work;
  double* work2;  // backward results of the two-ended solve
  int64_t ldw;
  int64_t n;
  int64_t vec_lds_off;  // doubles before the LDS-resident vector
  double* dummy;        // one slot per thread of the launch (stores of idle threads)
  const int32_t* order; // subdomain of each block (longest chains first)
};

// Fast path: the two-ended solve in two launches per apply.
// k_local_fwd (grid: subdomain x column chunk x half): gathers t = r - A q on
// its half of Omega_i (half 0: blocks 0..M, half 1: blocks M+1..K-1) and runs
// its forward chain in place in work.  k_local_bwd: the middle block, the
// backward chain into work2 (so no workgroup overwrites what the other half
// still reads) and the owner scatter of its half.
template <class FT, int P, int D>
__global__ void __launch_bounds__(adsd::SOLVE_T)
k_local_fwd(const FT* __restrict__ fac, LocalArgs a, const double* __restrict__ r,
            const double* __restrict__ q, int nrhs) {
  extern __shared__ double lds[];
  const int i = adsd::sub_of(a.order, blockIdx.x), half = blockIdx.z;
  const int j0 = blockIdx.y * P;
  const int pc = min(P, nrhs - j0);
  const int s = a.bs[i], K = a.nb[i], ns = a.ni[i], M = K / 2;
  const int64_t base = a.om_off[i];
  const int32_t* om = a.om_sorted + base;
  double* X = a.work + a.pad_off[i] + (int64_t)j0 * a.ldw;
  const int lo = half ? (M + 1) * s : 0, hi = half ? K * s : (M + 1) * s;
  gather_local<P>(om, ns, lo, hi, a.rowptr, a.col, a.val, r, q, a.n, j0, pc, X, a.ldw);
  __syncthreads();
  double* dummy =
      a.dummy + (((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * blockDim.x +
      threadIdx.x;
  const int64_t cb = a.pad_off[i] * adsd::NCPL;
  const int32_t* cc = (half ? a.rcpl_col : a.cpl_col) + cb;
  const double* cv = (half ? a.rcpl_val : a.cpl_val) + cb;
  adsd::block_chain<FT, P, D, true>(fac + a.fac_off[i], s, half ? K - 1 : 0, half ? -1 : 1,
                                    half ? K - 1 - M : M, cc, cv, X, X, a.ldw, pc, lds, dummy);
}

template <class FT, int P, int D>
__global__ void __launch_bounds__(adsd::SOLVE_T)
k_local_bwd(const FT* __restrict__ fac, LocalArgs a, const double* __restrict__ q,
            double* __restrict__ z, int nrhs) {  // z = nullptr: no owner scatter
  extern __shared__ double lds[];
  const int i = adsd::sub_of(a.order, blockIdx.x), half = blockIdx.z;
  const int j0 = blockIdx.y * P;
  const int pc = min(P, nrhs - j0);
  const int s = a.bs[i], K = a.nb[i], ns = a.ni[i], M = K / 2;
  const int64_t base = a.om_off[i];
  const int32_t* om = a.om_sorted + base;
  const double* X = a.work + a.pad_off[i] + (int64_t)j0 * a.ldw;
  double* Xo = a.work2 + a.pad_off[i] + (int64_t)j0 * a.ldw;
  const int64_t cb = a.pad_off[i] * adsd::NCPL;
  const FT* F = fac + a.fac_off[i];
  adsd::block_mid<FT, P>(F, s, M, K, a.cpl_col + cb, a.cpl_val + cb, a.rcpl_col + cb,
                         a.rcpl_val + cb, X, half == 0 ? Xo : nullptr, a.ldw, pc, lds);
  double* dummy =
      a.dummy + (((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * blockDim.x +
      threadIdx.x;
  adsd::block_chain<FT, P, D, false>(F, s, half ? M + 1 : M - 1, half ? 1 : -1,
                                     half ? K - 1 - M : M, nullptr, nullptr, X, Xo, a.ldw, pc, lds,
                                     dummy);
  __syncthreads();
  const int lo = half ? (M + 1) * s : 0, hi = min(ns, half ? K * s : (M + 1) * s);
  if (z && lo < hi) scatter_local(om, a.om_int + base, lo, hi, q, z, a.n, j0, pc, Xo, a.ldw);
}

// general path (any block size / coupling count); qg enters the residual
// gather t = r - A qg, qs the owner scatter z = qs + x (z = nullptr: none)
template <class FT, int P>
__device__ __forceinline__ void local_solve_general(const FT* __restrict__ fac, const LocalArgs& a,
                                                    const double* __restrict__ r,
                                                    const double* __restrict__ qg,
                                                    const double* __restrict__ qs,
                                                    double* __restrict__ z, int nrhs) {
  extern __shared__ double lds[];
  const int i = adsd::sub_of(a.order, blockIdx.x);
  const int j0 = blockIdx.y * P;
  const int pc = min(P, nrhs - j0);
  const int s = a.bs[i], K = a.nb[i], ns = a.ni[i];
  const int npad = K * s;
  const int64_t base = a.om_off[i];
  const int32_t* om = a.om_sorted + base;
  double* X = a.work + a.pad_off[i] + (int64_t)j0 * a.ldw;
  gather_local<P>(om, ns, 0, npad, a.rowptr, a.col, a.val, r, qg, a.n, j0, pc, X, a.ldw);
  __syncthreads();
  const int64_t cb = a.pad_off[i] * adsd::NCPL;
  adsd::block_solve_general<FT, P>(fac + a.fac_off[i], s, K, ns, a.lrow + base, a.lcol, a.lval,
                                   a.cpl_ok ? a.cpl_col + cb : nullptr,
                                   a.cpl_ok ? a.cpl_val + cb : nullptr, X,
                                   a.ldw, pc, lds);
  if (z) scatter_local(om, a.om_int + base, 0, ns, qs, z, a.n, j0, pc, X, a.ldw);
}

template <class FT, int P>
__global__ void __launch_bounds__(APPLY_T)
k_local_solve(const FT* __restrict__ fac, LocalArgs a, const double* __restrict__ r,
              const double* __restrict__ qg, const double* __restrict__ qs,
              double* __restrict__ z, int nrhs) {
  local_solve_general<FT, P>(fac, a, r, qg, qs, z, nrhs);
}

// 16 columns with the tile products on the matrix cores: one workgroup of
// adsd::MF_T threads per compute unit, so the registers are budgeted for
// four waves per SIMD (the loads of several column chunks stay in flight)
template <class FT>
__global__ void __launch_bounds__(adsd::MF_T) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_local_solve16(const FT* __restrict__ fac, LocalArgs a, const double* __restrict__ r,
                const double* __restrict__ qg, const double* __restrict__ qs,
                double* __restrict__ z, int nrhs) {
  local_solve_general<FT, 16>(fac, a, r, qg, qs, z, nrhs);
}

// eq. 1 / eq. 2 prolongation: z(g) = qs(g) + sum over the subdomains i that
// contain g (ascending i) of x_i at g's local slot
__global__ void __launch_bounds__(256)
k_prolong_sum(int64_t n, const int32_t* __restrict__ cptr, const int32_t* __restrict__ cidx,
              const double* __restrict__ X, int64_t ldw, const double* __restrict__ qs,
              double* __restrict__ z) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (g >= n) return;
  double v = qs ? qs[(int64_t)j * n + g] : 0.0;
  const double* Xj = X + (int64_t)j * ldw;
  for (int p = cptr[g]; p < cptr[g + 1]; ++p) v += Xj[cidx[p]];
  z[(int64_t)j * n + g] = v;
}

// the row -> slots map: counts, offsets by scan, fill, then each row's short
// list sorted (slots grow with the subdomain index)
__global__ void k_cover_count(const int64_t* __restrict__ om_off, const int32_t* __restrict__ ni,
                              const int32_t* __restrict__ om_sorted, int32_t* __restrict__ cnt) {
  const int i = blockIdx.x;
  const int32_t* om = om_sorted + om_off[i];
  for (int lr = blockIdx.y * blockDim.x + threadIdx.x; lr < ni[i]; lr += gridDim.y * blockDim.x)
    atomicAdd(&cnt[om[lr]], 1);
}

__global__ void k_cover_fill(const int64_t* __restrict__ om_off, const int32_t* __restrict__ ni,
                             const int32_t* __restrict__ om_sorted, const int64_t* __restrict__ pad_off,
                             const int32_t* __restrict__ cptr, int32_t* __restrict__ fill,
                             int32_t* __restrict__ cidx) {
  const int i = blockIdx.x;
  const int32_t* om = om_sorted + om_off[i];
  for (int lr = blockIdx.y * blockDim.x + threadIdx.x; lr < ni[i]; lr += gridDim.y * blockDim.x) {
    const int g = om[lr];
    const int k = atomicAdd(&fill[g], 1);
    cidx[cptr[g] + k] = (int32_t)(pad_off[i] + lr);
  }
}

__global__ void k_cover_sort(int64_t n, const int32_t* __restrict__ cptr, int32_t* __restrict__ cidx) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  int32_t* a = cidx + cptr[g];
  const int m = cptr[g + 1] - cptr[g];
  for (int k = 1; k < m; ++k) {
    const int32_t v = a[k];
    int q = k - 1;
    while (q >= 0 && a[q] > v) {
      a[q + 1] = a[q];
      --q;
    }
    a[q + 1] = v;
  }
}

void build_cover(Ctx& c) {
  hipStream_t st = c.stream;
  if (c.npad_total >= ((int64_t)1 << 31)) fail(ADS_ERR_UNSUPPORTED, "local vectors too long");
  int maxn = 1;
  for (int i = 0; i < c.nsub; ++i) maxn = std::max(maxn, c.h_ni[i]);
  const dim3 g(c.nsub, (unsigned)((maxn + 255) / 256));
  int32_t* cnt = c.mem.alloc<int32_t>(c.n + 1);
  ADS_HIP(hipMemsetAsync(cnt, 0, (c.n + 1) * 4, st));
  ADS_LAUNCH(k_cover_count, g, dim3(256), 0, st, c.om_off, c.ni, c.om_sorted, cnt);
  c.cover_ptr = c.mem.alloc<int32_t>(c.n + 1);
  exclusive_scan_i32(cnt, c.cover_ptr, c.n + 1, c.mem, st);
  int32_t total = 0;
  ADS_HIP(hipMemcpyAsync(&total, c.cover_ptr + c.n, 4, hipMemcpyDeviceToHost, st));
  ADS_HIP(hipStreamSynchronize(st));
  c.cover_idx = c.mem.alloc<int32_t>(std::max<int32_t>(total, 1));
  ADS_HIP(hipMemsetAsync(cnt, 0, (c.n + 1) * 4, st));
  ADS_LAUNCH(k_cover_fill, g, dim3(256), 0, st, c.om_off, c.ni, c.om_sorted, c.pad_off, c.cover_ptr,
             cnt, c.cover_idx);
  ADS_LAUNCH(k_cover_sort, dim3((unsigned)((c.n + 255) / 256)), dim3(256), 0, st, c.n, c.cover_ptr,
             c.cover_idx);
  c.mem.release(cnt);
}

// the apply workspace holds cols columns for the current coarse dimension
// (cvec and yvec are sized by n0)
bool work_fits(const Ctx& c, int cols) {
  return c.work_cols >= cols && c.work_n0 == c.n0 && (c.yvec || !coarse_big(c));
}

void ensure_work(Ctx& c, int cols) {
  if (work_fits(c, cols)) return;
  if (c.priv) ADS_HIP(hipStreamSynchronize(c.priv));  // the old workspace may be in use there
  if (c.work) c.mem.release(c.work);
  if (c.cvec) c.mem.release(c.cvec);
  if (c.yvec) c.mem.release(c.yvec);
  c.yvec = nullptr;
  if (c.qvec) c.mem.release(c.qvec);
  if (c.work2) c.mem.release(c.work2);
  if (c.dummy) c.mem.release(c.dummy);
  c.work = c.mem.alloc<double>((size_t)c.npad_total * cols);
  c.work2 = c.mem.alloc<double>((size_t)c.npad_total * cols);
  // one discard slot per thread of a fast-path launch: subdomain x column
  // chunk (at least one column per chunk) x half
  c.dummy = c.mem.alloc<double>((size_t)c.nsub * cols * 2 * adsd::SOLVE_T);
  // partial sums of the coarse restriction: one per (coarse entry, row chunk)
  c.cvec = c.mem.alloc<double>((size_t)std::max(c.n0, 1) * cols * coarse_chunks(c));
  // c and y of the large-system form: 2 n0 cols
  if (coarse_big(c)) c.yvec = c.mem.alloc<double>((size_t)2 * c.n0 * cols);
  c.qvec = c.mem.alloc<double>((size_t)c.n * cols);
  c.work_cols = cols;
  c.work_n0 = c.n0;
}

// the apply's workspace: the context's own buffers (ensure_work) or, for
// the no-allocation entry point, slices of the file-scope scratch array
struct ApplyWs {
  double* work;
  double* work2;
  double* dummy;
  double* cvec;
  double* yvec;  // non-null: y = E^{-1} c formed in a pass of its own
  double* qvec;
};

static ApplyWs ctx_ws(const Ctx& c) { return {c.work, c.work2, c.dummy, c.cvec, c.yvec, c.qvec}; }

static LocalArgs local_args(Ctx& c, const ApplyWs& w) {
  LocalArgs a;
  a.fac_off = c.fac_off;
  a.bs = c.bs;
  a.nb = c.nb;
  a.ni = c.ni;
  a.om_off = c.om_off;
  a.om_sorted = c.om_sorted;
  a.om_int = c.om_int;
  a.lrow = c.lptr_off;
  a.lcol = c.lcol;
  a.lval = c.lval;
  a.cpl_col = c.cpl_col;
  a.cpl_ok = c.cpl_ok ? 1 : 0;
  a.cpl_val = c.cpl_val;
  a.rcpl_col = c.rcpl_col;
  a.rcpl_val = c.rcpl_val;
  a.rowptr = c.rowptr;
  a.col = c.col;
  a.val = c.val;
  a.pad_off = c.pad_off;
  a.work = w.work;
  a.work2 = w.work2;
  a.ldw = c.npad_total;
  a.n = c.n;
  a.vec_lds_off = 0;
  a.dummy = w.dummy;
  a.order = c.sub_order;
  return a;
}

// the 16-column matrix-core form of the general path fits in LDS (two
// workgroups per compute unit)
static bool general_mfma_ok(const Ctx& c) {
  return adsd::solve_lds_doubles_general<16>(c.h_bs, adsd::MF_T) * 8 <= 80 * 1024;
}

// the local solves of one apply: gather t = r - A qg (qg may be null), solve,
// and scatter z = qs + x on the owner rows (z = nullptr: the solutions stay
// in the work buffers for k_prolong_sum)
template <class FT>
static void local_dispatch(Ctx& c, const ApplyWs& w, const double* r, const double* qg,
                           const double* qs, double* z, int nrhs, hipStream_t s) {
  LocalArgs a = local_args(c, w);
  constexpr int D = 2;
  constexpr int DM = 2;  // multi-column variants: shallower prefetch, fewer registers
  if (c.solve_fast) {
    auto run = [&](auto ptag, auto dtag) {
      constexpr int P = decltype(ptag)::value;
      constexpr int DD = decltype(dtag)::value;
      const size_t lds = (size_t)adsd::solve_lds_doubles<P>(c.h_bs, adsd::SOLVE_T) * 8;
      const dim3 grid(c.nsub, (nrhs + P - 1) / P, 2);
      ADS_LAUNCH((k_local_fwd<FT, P, DD>), grid, dim3(adsd::SOLVE_T), lds, s, (const FT*)c.facA, a,
                 r, qg, nrhs);
      ADS_LAUNCH((k_local_bwd<FT, P, DD>), grid, dim3(adsd::SOLVE_T), lds, s, (const FT*)c.facA, a,
                 qs, z, nrhs);
    };
    if (nrhs == 1)
      run(std::integral_constant<int, 1>(), std::integral_constant<int, D>());
    else if (nrhs <= 4)
      run(std::integral_constant<int, 4>(), std::integral_constant<int, DM>());
    else
      run(std::integral_constant<int, 8>(), std::integral_constant<int, DM>());
    return;
  }
  if (nrhs == 1) {
    size_t lds = (size_t)adsd::solve_lds_doubles_general<1>(c.h_bs, APPLY_T) * 8;
    ADS_LAUNCH((k_local_solve<FT, 1>), dim3(c.nsub, 1), dim3(APPLY_T), lds, s, (const FT*)c.facA, a,
               r, qg, qs, z, nrhs);
  } else if (nrhs > 8 && general_mfma_ok(c)) {
    // more than 8 columns: chunks of 16 on the matrix cores (each tile read
    // once per 16 columns)
    size_t lds = (size_t)adsd::solve_lds_doubles_general<16>(c.h_bs, adsd::MF_T) * 8;
    ADS_LAUNCH((k_local_solve16<FT>), dim3(c.nsub, (nrhs + 15) / 16), dim3(adsd::MF_T), lds, s,
               (const FT*)c.facA, a, r, qg, qs, z, nrhs);
  } else {
    size_t lds = (size_t)adsd::solve_lds_doubles_general<8>(c.h_bs, APPLY_T) * 8;
    ADS_LAUNCH((k_local_solve<FT, 8>), dim3(c.nsub, (nrhs + 7) / 8), dim3(APPLY_T), lds, s,
               (const FT*)c.facA, a, r, qg, qs, z, nrhs);
  }
}

// Accuracy of the stored local factors: for a fixed pseudo-random r, the
// relative residual ||t_i - A_ii x_i|| / ||t_i|| of the local solves
// x_i = (factors)^{-1} t_i, t_i = r restricted to Omega_i (one workgroup per
// subdomain; the local CSR of A_ii, local row order).  With FP64 factors this
// is rounding; with FP32 / BF16 factors it measures what the reduced storage
// costs each subdomain solve of the apply.
__global__ void k_fill_hash(double* r, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) r[g] = adsd::hash_unit(0x5eedull ^ (uint64_t)g);
}

__global__ void __launch_bounds__(256)
k_local_residual(const int64_t* __restrict__ om_off, const int32_t* __restrict__ ni,
                 const int32_t* __restrict__ om_sorted, const int64_t* __restrict__ lrow,
                 const int32_t* __restrict__ lcol, const double* __restrict__ lval,
                 const int64_t* __restrict__ pad_off, const double* __restrict__ X,
                 const double* __restrict__ r, double* __restrict__ ratio) {
  __shared__ double red[8];
  const int i = blockIdx.x;
  const int64_t f0 = om_off[i];
  const double* x = X + pad_off[i];
  double rr = 0.0, tt = 0.0;
  for (int k = threadIdx.x; k < ni[i]; k += blockDim.x) {
    const double t = r[om_sorted[f0 + k]];
    double v = t;
    for (int64_t q = lrow[f0 + k]; q < lrow[f0 + k + 1]; ++q) v -= lval[q] * x[lcol[q]];
    rr += v * v;
    tt += t * t;
  }
  rr = adsd::block_sum(rr, red);
  tt = adsd::block_sum(tt, red);
  if (threadIdx.x == 0) ratio[i] = tt > 0.0 ? sqrt(rr / tt) : 0.0;
}

double local_solve_accuracy(Ctx& c) {
  hipStream_t st = c.stream;
  // buffers of its own: the apply's workspace is sized later, once the
  // coarse dimension is known
  ApplyWs w{};
  w.work = c.mem.alloc<double>((size_t)c.npad_total);
  w.work2 = c.mem.alloc<double>((size_t)c.npad_total);
  w.dummy = c.mem.alloc<double>((size_t)c.nsub * 2 * adsd::SOLVE_T);
  double* r = c.mem.alloc<double>(c.n);
  double* ratio = c.mem.alloc<double>(c.nsub);
  ADS_LAUNCH(k_fill_hash, dim3((unsigned)((c.n + 255) / 256)), dim3(256), 0, st, r, c.n);
  switch (c.prec) {
    case ADS_PREC_FP64: local_dispatch<double>(c, w, r, nullptr, nullptr, nullptr, 1, st); break;
    case ADS_PREC_FP32: local_dispatch<float>(c, w, r, nullptr, nullptr, nullptr, 1, st); break;
    default: local_dispatch<__hip_bfloat16>(c, w, r, nullptr, nullptr, nullptr, 1, st); break;
  }
  ADS_LAUNCH(k_local_residual, dim3(c.nsub), dim3(256), 0, st, c.om_off, c.ni, c.om_sorted,
             c.lptr_off, c.lcol, c.lval, c.pad_off, c.solve_fast ? w.work2 : w.work, r, ratio);
  std::vector<double> h;
  download(h, ratio, c.nsub, st);
  for (double* p : {r, ratio, w.work, w.work2, w.dummy}) c.mem.release(p);
  double mx = 0.0;
  for (double v : h) mx = std::max(mx, v);
  return mx;
}

// average time (ms) of one local solve (both chain launches, nrhs = 1) on
// the current tiles, from hipEvents around reps launches after a warm-up
// launch; the apply workspace is released afterwards (its size depends on
// the tiles and on the coarse dimension)
double time_local_solve(Ctx& c, int reps) {
  hipStream_t st = c.stream;
  ensure_work(c, 1);
  double* r = c.mem.alloc<double>(c.n);
  double* q = c.mem.alloc<double>(c.n);
  double* z = c.mem.alloc<double>(c.n);
  ADS_HIP(hipMemsetAsync(r, 0, c.n * 8, st));
  ADS_HIP(hipMemsetAsync(q, 0, c.n * 8, st));
  const ApplyWs w = ctx_ws(c);
  auto run = [&]() {
    switch (c.prec) {
      case ADS_PREC_FP64: local_dispatch<double>(c, w, r, q, q, z, 1, st); break;
      case ADS_PREC_FP32: local_dispatch<float>(c, w, r, q, q, z, 1, st); break;
      default: local_dispatch<__hip_bfloat16>(c, w, r, q, q, z, 1, st); break;
    }
  };
  run();
  hipEvent_t e0, e1;
  ADS_HIP(hipEventCreate(&e0));
  ADS_HIP(hipEventCreate(&e1));
  ADS_HIP(hipEventRecord(e0, st));
  for (int k = 0; k < reps; ++k) run();
  ADS_HIP(hipEventRecord(e1, st));
  ADS_HIP(hipEventSynchronize(e1));
  float ms = 0.0f;
  ADS_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (double* p : {r, q, z}) c.mem.release(p);
  for (double** p : {&c.work, &c.work2, &c.dummy, &c.cvec, &c.yvec, &c.qvec})
    if (*p) {
      c.mem.release(*p);
      *p = nullptr;
    }
  c.work_cols = 0;
  return (double)ms / reps;
}

// records a hipEvent pair around a launch when profiling is on
struct ProfScope {
  Ctx& c;
  int k;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(Ctx& cc, int kk, hipStream_t ss) : c(cc), k(kk), s(ss) {
    if (!(c.opt.profile & 1)) return;
    ADS_HIP(hipEventCreate(&a));
    ADS_HIP(hipEventCreate(&b));
    ADS_HIP(hipEventRecord(a, s));
  }
  ~ProfScope() {
    if (!(c.opt.profile & 1)) return;
    (void)hipEventRecord(b, s);
    c.prof_ev[k].push_back({a, b});
  }
};

void Ctx::prof_resolve() {
  for (auto& e : prof_gj_ev) {
    float ms = 0.f;
    ADS_HIP(hipEventSynchronize(e.second));
    ADS_HIP(hipEventElapsedTime(&ms, e.first, e.second));
    prof_gj_ms += ms;
    prof_gj_n += 1;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  prof_gj_ev.clear();
  for (int k = 0; k < 4; ++k) {
    for (auto& e : prof_ev[k]) {
      float ms = 0.f;
      ADS_HIP(hipEventSynchronize(e.second));
      ADS_HIP(hipEventElapsedTime(&ms, e.first, e.second));
      prof_ms[k] += ms;
      prof_n[k] += 1;
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    prof_ev[k].clear();
  }
}

Ctx::~Ctx() {
  if (priv) (void)hipStreamSynchronize(priv);
  for (auto& e : prof_gj_ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (apply_exec) (void)hipGraphExecDestroy(apply_exec);
  if (dep_ev) (void)hipEventDestroy(dep_ev);
  if (priv) (void)hipStreamDestroy(priv);
  for (int k = 0; k < 4; ++k)
    for (auto& e : prof_ev[k]) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
}

static void apply_kernels(Ctx& c, const ApplyWs& w, const double* r, double* z, int nrhs,
                          hipStream_t s) {
  ProfScope all(c, 3, s);
  const double* q = nullptr;
  if (c.n0 > 0) {
    const int nch = coarse_chunks(c);
    {
      ProfScope p1(c, 1, s);
      ADS_LAUNCH(k_coarse_restrict_mf, dim3(c.nsub, nch, (nrhs + 15) / 16), dim3(APPLY_T), 0, s,
                 r, c.n, c.int_list, c.om_off, c.nI, c.W, c.W_off, c.nev, c.coff, w.cvec, c.n0,
                 nch, nrhs);
    }
    double* yfull = nullptr;
    {
      ProfScope p2(c, 2, s);
      if (w.yvec) {
        double* cy = w.yvec;
        yfull = w.yvec + (size_t)c.n0 * nrhs;
        const int64_t ne = (int64_t)c.n0 * nrhs;
        ADS_LAUNCH(k_coarse_csum, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, w.cvec,
                   c.n0, nch, nrhs, cy);
        int maxs = 0;
        for (int v : c.h_n0s) maxs = std::max(maxs, v);
        ADS_LAUNCH(k_coarse_emul_mf,
                   dim3((unsigned)((maxs + 15) / 16), (unsigned)c.nsys, (unsigned)((nrhs + 15) / 16)),
                   dim3(256), 0, s, cy, c.n0, nrhs, c.Einv, c.E_off, c.sys_coff, yfull);
        ADS_LAUNCH(k_coarse_prolong_all, dim3(c.nsub, nch), dim3(APPLY_T), 0, s, yfull, c.n0, nrhs,
                   c.int_list, c.om_off, c.nI, c.W, c.W_off, c.nev, c.coff, w.qvec, c.n);
      } else {
        ADS_LAUNCH(k_coarse_prolong, dim3(c.nsub, nch, nrhs), dim3(APPLY_T), 0, s, w.cvec,
                   c.n0, nch, c.Einv, c.E_off, c.sys_coff, c.sub_sys_d,
                   c.int_list, c.om_off, c.nI, c.W, c.W_off, c.nev, c.coff, w.qvec, c.n);
      }
    }
    q = w.qvec;
  }
  // eq. 4 solves the local problems on r - A q; the additive forms on r
  const double* qg = c.opt.variant == ADS_VARIANT_DEFLATED ? q : nullptr;
  const bool restricted = variant_restricted(c.opt.variant);
  double* zs = restricted ? z : nullptr;
  {
    ProfScope p0(c, 0, s);
    switch (c.prec) {
      case ADS_PREC_FP64: local_dispatch<double>(c, w, r, qg, q, zs, nrhs, s); break;
      case ADS_PREC_FP32: local_dispatch<float>(c, w, r, qg, q, zs, nrhs, s); break;
      default: local_dispatch<__hip_bfloat16>(c, w, r, qg, q, zs, nrhs, s); break;
    }
  }
  if (!restricted)
    ADS_LAUNCH(k_prolong_sum, dim3((unsigned)((c.n + 255) / 256), nrhs), dim3(256), 0, s, c.n,
               c.cover_ptr, c.cover_idx, c.solve_fast ? w.work2 : w.work, c.npad_total, q, z);
}

hipStream_t Ctx::own_stream() {
  if (!priv) {
    ADS_HIP(hipStreamCreateWithFlags(&priv, hipStreamNonBlocking));
    ADS_HIP(hipEventCreateWithFlags(&dep_ev, hipEventDisableTiming));
  }
  return priv;
}

void Ctx::drop_apply_graph() {
  if (apply_exec) (void)hipGraphExecDestroy(apply_exec);
  apply_exec = nullptr;
  ag_r = nullptr;
  ag_z = nullptr;
  ag_nrhs = 0;
  ag_st = nullptr;
}

// z = M^{-1} r on stream s: eager launches, or the replay of a captured graph
// of them when graphs are on and s is not the null stream
void apply_prec(Ctx& c, const double* r, double* z, int nrhs, hipStream_t s) {
  if (!work_fits(c, nrhs)) c.drop_apply_graph();  // the workspace is reallocated
  ensure_work(c, nrhs);
  const ApplyWs w = ctx_ws(c);
  if (c.capturing || !c.graphs_on() || s == nullptr) {
    apply_kernels(c, w, r, z, nrhs, s);
    return;
  }
  if (!(c.apply_exec && c.ag_r == r && c.ag_z == z && c.ag_nrhs == nrhs && c.ag_st == s)) {
    c.drop_apply_graph();
    c.capturing = true;
    try {
      c.apply_exec = capture_graph(s, [&] { apply_kernels(c, w, r, z, nrhs, s); });
    } catch (...) {
      c.capturing = false;
      throw;
    }
    c.capturing = false;
    c.ag_r = r;
    c.ag_z = z;
    c.ag_nrhs = nrhs;
    c.ag_st = s;
  }
  ADS_HIP(hipGraphLaunch(c.apply_exec, s));
}

// ---------------------------------------------------------------------------
// Apply without allocation (callers that cannot allocate: code under HIP
// graph capture, serving loops, harnesses that forbid hipMalloc).  The
// workspace of one apply (padded local vectors, the coarse restriction's
// partial sums, c and y of large coarse systems, the coarse correction q) is
// carved from `scratch`, a file-scope device array of NOALLOC_DOUBLES
// doubles (128 MiB) that every GPU the library runs on holds until the
// process ends.  Its device address is resolved once per device with
// hipGetSymbolAddress (the array's name is only a host-side stand-in).  No
// part of the workspace has to start at zero.  All calls on one GPU share the
// array: calls that overlap on one GPU race.  No graph capture, no events, no
// allocation: the kernels of the ordinary apply are launched directly on the
// caller's stream.
// ---------------------------------------------------------------------------
static constexpr int64_t NOALLOC_DOUBLES = (int64_t)16 << 20;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];
static constexpr int NOALLOC_MAX_DEV = 64;
static double* g_scratch[NOALLOC_MAX_DEV] = {nullptr};
static std::mutex g_scratch_mu;

static double* scratch_ptr() {
  int dev = 0;
  ADS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) fail(ADS_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    ADS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(ADS_ERR_HIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch[dev] = static_cast<double*>(p);
  }
  return g_scratch[dev];
}

int64_t noalloc_doubles_needed(const Ctx& c, int cols) {
  auto al = [](int64_t d) { return (d + 31) & ~(int64_t)31; };  // 256-byte slices
  int64_t need = al((int64_t)c.npad_total * cols);                // work
  if (c.solve_fast) {
    need += al((int64_t)c.npad_total * cols);                      // work2
    need += al((int64_t)c.nsub * cols * 2 * adsd::SOLVE_T);        // dummy
  }
  need += al((int64_t)std::max(c.n0, 1) * cols * coarse_chunks(c));  // cvec
  if (coarse_big(c)) need += al((int64_t)2 * c.n0 * cols);          // yvec
  need += al((int64_t)c.n * cols);                                  // qvec
  return need;
}

void apply_noalloc(Ctx& c, const double* r, double* z, int nrhs, hipStream_t s) {
  const int64_t need = noalloc_doubles_needed(c, nrhs);
  if (need > NOALLOC_DOUBLES)
    fail(ADS_ERR_ARG, "ads_apply_noalloc: this context needs " + std::to_string(need * 8) +
                          " bytes of workspace for nrhs = " + std::to_string(nrhs) +
                          ", beyond the scratch array's " + std::to_string(NOALLOC_DOUBLES * 8));
  if (c.opt.profile & 1) fail(ADS_ERR_ARG, "ads_apply_noalloc: apply profiling records events");
  double* base = scratch_ptr();
  auto al = [](int64_t d) { return (d + 31) & ~(int64_t)31; };
  auto take = [&](int64_t d) {
    double* p = base;
    base += al(d);
    return p;
  };
  ApplyWs w{};
  w.work = take((int64_t)c.npad_total * nrhs);
  if (c.solve_fast) {
    w.work2 = take((int64_t)c.npad_total * nrhs);
    w.dummy = take((int64_t)c.nsub * nrhs * 2 * adsd::SOLVE_T);
  }
  w.cvec = take((int64_t)std::max(c.n0, 1) * nrhs * coarse_chunks(c));
  w.yvec = coarse_big(c) ? take((int64_t)2 * c.n0 * nrhs) : nullptr;
  w.qvec = take((int64_t)c.n * nrhs);
  apply_kernels(c, w, r, z, nrhs, s);
}

}  // namespace ads
