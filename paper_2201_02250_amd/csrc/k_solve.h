// Block-tridiagonal solve with the stored tiles G_k = D_k^{-1}, P_k = G_k A_k,k+1
// (see k_factor.hip), for P right-hand sides at once, executed by one
// workgroup.  Used by the preconditioner apply (local solves of eq. 3/eq. 4)
// and by the eigensolver (the operator of eq. 5).
//
// X (padded local vectors, column j at X + j*ldx) is overwritten in place:
// forward  y_k = f_k - A_k,k-1 h_{k-1},  h_k = G_k y_k   (h_k stored in X)
// backward x_{K-1} = h_{K-1},  x_k = h_k - P_k x_{k+1}.
// The sparse couplings A_k,k-1 come from the local CSR of A_ii (identical for
// the splitting: Definition 1 only changes the diagonal).
//
// Thread mapping of a dense tile product out = M v (M s x s column-major):
// thread t handles row r = t mod s and column chunk g = t / s; with G chunks,
// partial sums meet in LDS.  Consecutive threads read consecutive rows of a
// tile column (coalesced), the vector entry is an LDS broadcast.
#pragma once
#include "ads_internal.h"

namespace adsd {

// LDS doubles needed by block_solve<P> with blockDim T, maximised over every
// block size in `sizes` (a smaller block can use more column chunks).
template <int P>
inline int64_t solve_lds_doubles(const std::vector<int32_t>& sizes, int T);

template <int P>
struct SolveLds {
  // doubles needed: ybuf (s*P) + hbuf (s*P) + partial (G*s*P)
  static __host__ __device__ int64_t doubles(int s, int T) {
    int G = (2 * s <= T) ? (T / s) : 1;
    return (int64_t)s * P * (2 + (G > 1 ? G : 0));
  }
};

template <int P>
inline int64_t solve_lds_doubles(const std::vector<int32_t>& sizes, int T) {
  int64_t m = 0;
  for (int s : sizes) m = m > SolveLds<P>::doubles(s, T) ? m : SolveLds<P>::doubles(s, T);
  return m;
}

// out[r + j*s] (LDS) = sum_c M[r + c*s] vin[c + j*s]  (+ combine)
// mode 0: out = M v; mode 1: out = base - M v where base[r + j*s] given (global, ld)
template <class FT, int P>
__device__ __forceinline__ void tile_product(const FT* __restrict__ M, int s, const double* vin,
                                             double* part, double* out, int mode,
                                             const double* base, int64_t ldb, int pc) {
  const int t = threadIdx.x, T = blockDim.x;
  const int G = (2 * s <= T) ? (T / s) : 1;
  if (G > 1) {
    const int chunk = (s + G - 1) / G;
    const int r = t % s, g = t / s;
    if (g < G) {
      double acc[P];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] = 0.0;
      const int c0 = g * chunk, c1 = min(s, c0 + chunk);
      for (int cidx = c0; cidx < c1; ++cidx) {
        const double m = ld_fac(M, (int64_t)cidx * s + r);
#pragma unroll
        for (int j = 0; j < P; ++j) acc[j] += m * vin[cidx + j * s];
      }
#pragma unroll
      for (int j = 0; j < P; ++j) part[((int64_t)g * s + r) * P + j] = acc[j];
    }
    __syncthreads();
    for (int e = t; e < s * pc; e += T) {
      const int rr = e % s, j = e / s;
      double v = 0.0;
      for (int gg = 0; gg < G; ++gg) v += part[((int64_t)gg * s + rr) * P + j];
      out[rr + j * s] = mode ? base[rr + j * ldb] - v : v;
    }
  } else {
    for (int r = t; r < s; r += T) {
      double acc[P];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] = 0.0;
      for (int cidx = 0; cidx < s; ++cidx) {
        const double m = ld_fac(M, (int64_t)cidx * s + r);
#pragma unroll
        for (int j = 0; j < P; ++j) acc[j] += m * vin[cidx + j * s];
      }
      for (int j = 0; j < pc; ++j) out[r + j * s] = mode ? base[r + j * ldb] - acc[j] : acc[j];
    }
  }
}

// In-place solve on X (padded length K*s per column, pc <= P columns).
// lrow/lcol/lval: local CSR rows of this subdomain (lrow points at row 0).
template <class FT, int P>
__device__ void block_solve(const FT* __restrict__ fac, int s, int K, int n,
                            const int64_t* __restrict__ lrow, const int32_t* __restrict__ lcol,
                            const double* __restrict__ lval, double* X, int64_t ldx, int pc,
                            double* lds) {
  const int t = threadIdx.x, T = blockDim.x;
  const int64_t ss = (int64_t)s * s;
  double* ybuf = lds;
  double* hbuf = ybuf + (int64_t)s * P;
  double* part = hbuf + (int64_t)s * P;
  // forward sweep
  for (int k = 0; k < K; ++k) {
    const int r0 = k * s;
    __syncthreads();
    for (int e = t; e < s * pc; e += T) {
      const int rr = e % s, j = e / s;
      const int r = r0 + rr;
      double y = X[r + j * ldx];
      if (k > 0 && r < n) {
        for (int64_t q = lrow[r]; q < lrow[r + 1]; ++q) {
          const int cc = lcol[q] - (r0 - s);
          if (cc >= 0 && cc < s) y -= lval[q] * hbuf[cc + j * s];
        }
      }
      ybuf[rr + j * s] = y;
    }
    __syncthreads();
    tile_product<FT, P>(fac + (int64_t)k * 2 * ss, s, ybuf, part, hbuf, 0, nullptr, 0, pc);
    __syncthreads();
    for (int e = t; e < s * pc; e += T) {
      const int rr = e % s, j = e / s;
      X[r0 + rr + j * ldx] = hbuf[rr + j * s];
    }
  }
  // backward sweep: hbuf holds x_{K-1}
  for (int k = K - 2; k >= 0; --k) {
    const int r0 = k * s;
    __syncthreads();
    for (int e = t; e < s * pc; e += T) ybuf[e] = hbuf[e];  // x_{k+1}
    __syncthreads();
    tile_product<FT, P>(fac + (int64_t)k * 2 * ss + ss, s, ybuf, part, hbuf, 1, X + r0, ldx, pc);
    __syncthreads();
    for (int e = t; e < s * pc; e += T) {
      const int rr = e % s, j = e / s;
      X[r0 + rr + j * ldx] = hbuf[rr + j * s];
    }
  }
  __syncthreads();
}

}  // namespace adsd
