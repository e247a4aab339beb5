// Exact subdomain factorizations (Section 4: exact LU of the local matrices).
//
// In the ascending-global local order a grid-like A_ii has a narrow band of
// half-width b.  Cut into blocks of s = b rows it is block tridiagonal, and
// the block LU (no pivoting: the local matrices and splittings here are
// M-matrices) is
//     D_0 = A_00,  D_k = A_kk - A_k,k-1 D_{k-1}^{-1} A_k-1,k.
// The library stores, per block, G_k = D_k^{-1} and P_k = G_k A_k,k+1 as dense
// s x s column-major tiles.  A solve is then a chain of dense s x s products
// (forward: h_k = G_k (f_k - A_k,k-1 h_{k-1}); backward: x_k = h_k - P_k x_{k+1}),
// i.e. n/s sequential steps instead of n, each a wide matrix-vector (or, with
// several right-hand sides, matrix-matrix) product.  Factor bytes equal those
// of a band LU (2 s n entries).
//
// The splitting of Definition 1 is factored the same way.  On a floating
// subdomain (K_i = span{1}) it is singular; its last diagonal entry is doubled
// first.  For f in range(splitting) the solution u of the regularised system
// satisfies u_n = 0 and hence solves the singular system exactly (the left
// null vector has a nonzero last entry), which is all the eigensolver needs.
//
// One workgroup per subdomain; the block D_k and the previous P tile live in
// LDS when 2 s^2 doubles fit, otherwise in a per-workgroup global scratch.
// Inversion is Gauss-Jordan without pivoting in FP64; tiles are stored in the
// precision of the context.
#include <algorithm>

#include "ads_internal.h"
#include "k_solve.h"

namespace ads {

static constexpr int FAC_T = 256;

// store the row-major s x s matrix M (LDS or scratch) as a packed tile
template <class FT>
__device__ __forceinline__ void store_tile(FT* dst, const double* M, int s, int V) {
  const int64_t TS = adsd::tile_size(s, V);
  for (int64_t e = threadIdx.x; e < TS; e += blockDim.x) {
    const int v = (int)(e % V);
    const int64_t rest = e / V;
    const int r = (int)(rest % s), c = (int)(rest / s) * V + v;
    adsd::st_fac(dst, e, c < s ? M[(int64_t)r * s + c] : 0.0);
  }
}

template <class FT, bool USE_LDS>
__global__ void __launch_bounds__(FAC_T)
k_block_factor(const int64_t* lrow, const int32_t* lcol, const double* lval, const double* lsum,
               const uint8_t* om_int, const int64_t* om_off, const int32_t* ni,
               const int32_t* bsz, const int32_t* nblk, const int64_t* fac_off,
               const int32_t* kdim, int splitting, FT* fac, double* gscr, int64_t gscr_stride,
               int32_t* bad_pivot) {
  extern __shared__ double lds[];
  const int i = blockIdx.x;
  const int s = bsz[i], K = nblk[i], n = ni[i];
  const int t = threadIdx.x, T = blockDim.x;
  double* D = USE_LDS ? lds : gscr + (int64_t)i * gscr_stride;
  double* Pp = D + (int64_t)s * s;
  double* colp = Pp + (int64_t)s * s;
  const int64_t rbase = om_off[i];
  const bool regularise = splitting && kdim[i];
  FT* F = fac + fac_off[i];
  const int64_t ss = (int64_t)s * s;
  constexpr int V = adsd::TileV<FT>::V;
  const int64_t TS = adsd::tile_size(s, V);

  for (int k = 0; k < K; ++k) {
    const int r0 = k * s;
    // D = A_kk (rows of block k, columns of block k), splitting diagonal
    for (int64_t e = t; e < ss; e += T) D[e] = 0.0;
    __syncthreads();
    for (int rr = t; rr < s; rr += T) {
      const int r = r0 + rr;
      if (r >= n) {
        D[(int64_t)rr * s + rr] = 1.0;
        continue;
      }
      const int64_t f = rbase + r;
      for (int64_t q = lrow[f]; q < lrow[f + 1]; ++q) {
        const int cc = lcol[q] - r0;
        if (cc < 0 || cc >= s) continue;
        double a = lval[q];
        if (cc == rr && splitting) {
          if (!om_int[f]) a -= lsum[f];
          if (regularise && r == n - 1) a *= 2.0;
        }
        D[(int64_t)rr * s + cc] = a;
      }
    }
    __syncthreads();
    // D -= A_k,k-1 P_{k-1}: each thread owns columns j
    if (k > 0) {
      for (int rr = 0; rr < s; ++rr) {
        const int r = r0 + rr;
        if (r >= n) break;
        const int64_t f = rbase + r;
        for (int64_t q = lrow[f]; q < lrow[f + 1]; ++q) {
          const int cc = lcol[q] - (r0 - s);
          if (cc < 0 || cc >= s) continue;
          const double a = lval[q];
          for (int j = t; j < s; j += T) D[(int64_t)rr * s + j] -= a * Pp[(int64_t)cc * s + j];
        }
      }
    }
    // Gauss-Jordan inversion in place, no pivoting
    for (int p = 0; p < s; ++p) {
      __syncthreads();
      double piv = D[(int64_t)p * s + p];
      if (!(fabs(piv) > 0.0) || !isfinite(piv)) {
        if (t == 0) atomicMax(bad_pivot, i + 1);
        piv = 1.0;
      }
      for (int rr = t; rr < s; rr += T) colp[rr] = D[(int64_t)rr * s + p];
      __syncthreads();
      const double inv = 1.0 / piv;
      for (int j = t; j < s; j += T) D[(int64_t)p * s + j] = (j == p) ? inv : D[(int64_t)p * s + j] * inv;
      __syncthreads();
      for (int64_t e = t; e < ss; e += T) {
        const int rr = (int)(e / s), j = (int)(e - (int64_t)rr * s);
        if (rr == p) continue;
        const double fct = colp[rr];
        const double dpj = D[(int64_t)p * s + j];
        D[e] = (j == p ? 0.0 : D[e]) - fct * dpj;
      }
    }
    __syncthreads();
    // store G_k in the packed tile format
    FT* G = F + (int64_t)k * 2 * TS;
    store_tile(G, D, s, V);
    if (k + 1 < K) {
      // P_k = G_k A_k,k+1: thread owns rows rho
      for (int64_t e = t; e < ss; e += T) Pp[e] = 0.0;
      __syncthreads();
      for (int rr = 0; rr < s; ++rr) {
        const int r = r0 + rr;
        if (r >= n) break;
        const int64_t f = rbase + r;
        for (int64_t q = lrow[f]; q < lrow[f + 1]; ++q) {
          const int cc = lcol[q] - (r0 + s);
          if (cc < 0 || cc >= s) continue;
          const double a = lval[q];
          for (int rho = t; rho < s; rho += T) Pp[(int64_t)rho * s + cc] += D[(int64_t)rho * s + rr] * a;
        }
      }
      __syncthreads();
      store_tile(G + TS, Pp, s, V);
    }
    __syncthreads();
  }
}

// Same factorization, register-resident: 1024 threads; thread t owns column
// j = t % s of D_k for the rows g, g + G, g + 2G, ... (g = t / s, G = 1024 / s,
// at most FMR rows).  The Schur update and P_k use the fixed-width coupling
// lists (A_k,k-1 by row, A_k,k+1 by column).  Gauss-Jordan takes one barrier
// per pivot: the owners of the next pivot row and column publish them into
// the other half of a double buffer while they update.  blockIdx.y selects
// the matrix (0: A_ii, 1: splitting), so both are factored in one launch.
static constexpr int FMR = 9;

__host__ __device__ inline bool factor_fast_ok(int s) {
  if (s < 1 || s > 1024) return false;
  const int G = 1024 / s;
  return (s + G - 1) / G <= FMR;
}

template <class FT, bool USE_LDS>
__global__ void __launch_bounds__(1024)
k_block_factor_fast(const int64_t* lrow, const int32_t* lcol, const double* lval,
                    const double* lsum, const uint8_t* om_int, const int64_t* om_off,
                    const int32_t* ni, const int32_t* bsz, const int32_t* nblk,
                    const int64_t* fac_off, const int32_t* kdim, const int64_t* pad_off,
                    const int32_t* ccol, const double* cval, const int32_t* urow,
                    const double* uval, FT* facA, FT* facT, double* gscr, int64_t gscr_stride,
                    int32_t* bad_pivot) {
  extern __shared__ double lds[];
  const int i = blockIdx.x;
  const int splitting = blockIdx.y;
  FT* fac = splitting ? facT : facA;
  const int s = bsz[i], K = nblk[i], n = ni[i];
  const int t = threadIdx.x, T = blockDim.x;
  // a pointer known to be LDS at compile time keeps ds_* instructions
  double* D = USE_LDS ? lds : gscr + ((int64_t)splitting * gridDim.x + i) * gscr_stride;
  double* Pp = D + (int64_t)s * s;
  double* rowb = Pp + (int64_t)s * s;  // [2][s]
  double* colb = rowb + 2 * s;         // [2][s]
  const int64_t rbase = om_off[i];
  const int64_t pbase = pad_off[i];
  const bool regularise = splitting && kdim[i];
  FT* F = fac + fac_off[i];
  const int ss = s * s;
  constexpr int V = adsd::TileV<FT>::V;
  const int64_t TS = adsd::tile_size(s, V);
  const int G = T / s;
  const int j = t % s, g = t / s;
  const int nr = g < G ? (s - g + G - 1) / G : 0;
  double v[FMR];
  for (int k = 0; k < K; ++k) {
    const int r0 = k * s;
    __syncthreads();
    for (int e = t; e < ss; e += T) D[e] = 0.0;
    __syncthreads();
    for (int rr = t; rr < s; rr += T) {
      const int r = r0 + rr;
      if (r >= n) {
        D[rr * s + rr] = 1.0;
        continue;
      }
      const int64_t f = rbase + r;
      for (int64_t q = lrow[f]; q < lrow[f + 1]; ++q) {
        const int cc = lcol[q] - r0;
        if (cc < 0 || cc >= s) continue;
        double a = lval[q];
        if (cc == rr && splitting) {
          if (!om_int[f]) a -= lsum[f];
          if (regularise && r == n - 1) a *= 2.0;
        }
        D[rr * s + cc] = a;
      }
    }
    __syncthreads();
    if (k > 0) {  // D -= A_k,k-1 P_{k-1}, on the owned elements
      for (int m = 0; m < nr; ++m) {
        const int rr = g + m * G;
        const int64_t cb = (pbase + r0 + rr) * adsd::NCPL;
        double x = D[rr * s + j];
#pragma unroll
        for (int q = 0; q < adsd::NCPL; ++q) {
          const int cc = ccol[cb + q];
          if (cc >= 0) x -= cval[cb + q] * Pp[cc * s + j];
        }
        D[rr * s + j] = x;
      }
    }
    // own elements into registers; publish pivot row/column 0
#pragma unroll
    for (int m = 0; m < FMR; ++m) {
      if (m < nr) {
        const int rr = g + m * G;
        const double x = D[rr * s + j];
        v[m] = x;
        if (rr == 0) rowb[j] = x;
        if (j == 0) colb[rr] = x;
      }
    }
    __syncthreads();
    // Gauss-Jordan inversion, no pivoting, one barrier per pivot
    for (int p = 0; p < s; ++p) {
      const double* rw = rowb + (p & 1) * s;
      const double* cl = colb + (p & 1) * s;
      double* rwn = rowb + ((p + 1) & 1) * s;
      double* cln = colb + ((p + 1) & 1) * s;
      double piv = rw[p];
      if (!(fabs(piv) > 0.0) || !isfinite(piv)) {
        if (t == 0) atomicMax(bad_pivot, i + 1);
        piv = 1.0;
      }
      const double inv = 1.0 / piv;
      const double rj = rw[j] * inv;
#pragma unroll
      for (int m = 0; m < FMR; ++m) {
        if (m < nr) {
          const int rr = g + m * G;
          double x;
          if (rr == p)
            x = (j == p) ? inv : rj;
          else if (j == p)
            x = -cl[rr] * inv;
          else
            x = v[m] - cl[rr] * rj;
          v[m] = x;
          if (rr == p + 1) rwn[j] = x;
          if (j == p + 1) cln[rr] = x;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < FMR; ++m)
      if (m < nr) D[(g + m * G) * s + j] = v[m];
    __syncthreads();
    FT* Gt = F + (int64_t)k * 2 * TS;
    store_tile(Gt, D, s, V);
    if (k + 1 < K) {  // P_k = G_k A_k,k+1 (by columns of block k+1)
      for (int e = t; e < ss; e += T) {
        const int cp = e / s, rho = e - cp * s;
        const int64_t ub = (pbase + r0 + s + cp) * adsd::NCPL;
        double x = 0.0;
#pragma unroll
        for (int q = 0; q < adsd::NCPL; ++q) {
          const int rr = urow[ub + q];
          if (rr >= 0) x += D[rho * s + rr] * uval[ub + q];
        }
        Pp[rho * s + cp] = x;
      }
      __syncthreads();
      store_tile(Gt + TS, Pp, s, V);
    }
  }
}

template <class FT>
static void factor_fast(Ctx& c, bool both) {
  hipStream_t st = c.stream;
  const int nsub = c.nsub;
  FT* fa = c.mem.alloc<FT>(c.fac_elems);
  FT* ft = both ? c.mem.alloc<FT>(c.fac_elems) : nullptr;
  c.facA = fa;
  c.facT = ft;
  int smax = *std::max_element(c.h_bs.begin(), c.h_bs.end());
  size_t need = ((size_t)2 * smax * smax + 4 * smax) * sizeof(double);
  int use_lds = need <= 150 * 1024;
  int64_t stride = (int64_t)2 * smax * smax + 4 * smax;
  double* gscr = use_lds ? nullptr : c.mem.alloc<double>((size_t)stride * nsub * 2);
  int32_t* bad = c.mem.alloc<int32_t>(1);
  ADS_HIP(hipMemsetAsync(bad, 0, 4, st));
  if (use_lds)
    ADS_LAUNCH((k_block_factor_fast<FT, true>), dim3(nsub, both ? 2 : 1), dim3(1024), need, st,
               c.lptr_off, c.lcol, c.lval, c.lsum, c.om_int, c.om_off, c.ni, c.bs, c.nb, c.fac_off,
               c.kdim, c.pad_off, c.cpl_col, c.cpl_val, c.ucpl_row, c.ucpl_val, fa, ft, gscr, stride,
               bad);
  else
    ADS_LAUNCH((k_block_factor_fast<FT, false>), dim3(nsub, both ? 2 : 1), dim3(1024), 0, st,
               c.lptr_off, c.lcol, c.lval, c.lsum, c.om_int, c.om_off, c.ni, c.bs, c.nb, c.fac_off,
               c.kdim, c.pad_off, c.cpl_col, c.cpl_val, c.ucpl_row, c.ucpl_val, fa, ft, gscr, stride,
               bad);
  std::vector<int32_t> hb;
  download(hb, bad, 1, st);
  if (gscr) c.mem.release(gscr);
  if (hb[0])
    fail(ADS_ERR_SINGULAR, "zero pivot in the local matrix or splitting of subdomain " +
                               std::to_string(hb[0] - 1));
}

template <class FT>
static void factor_one(Ctx& c, int splitting, void** out) {
  hipStream_t s = c.stream;
  const int nsub = c.nsub;
  FT* fac = c.mem.alloc<FT>(c.fac_elems);
  *out = fac;
  int smax = *std::max_element(c.h_bs.begin(), c.h_bs.end());
  size_t need = ((size_t)2 * smax * smax + smax) * sizeof(double);
  int use_lds = need <= 120 * 1024;
  double* gscr = nullptr;
  int64_t stride = (int64_t)2 * smax * smax + smax;
  if (!use_lds) gscr = c.mem.alloc<double>((size_t)stride * nsub);
  int32_t* bad = c.mem.alloc<int32_t>(1);
  ADS_HIP(hipMemsetAsync(bad, 0, 4, s));
  if (use_lds)
    ADS_LAUNCH((k_block_factor<FT, true>), dim3(nsub), dim3(FAC_T), need, s, c.lptr_off, c.lcol,
               c.lval, c.lsum, c.om_int, c.om_off, c.ni, c.bs, c.nb, c.fac_off, c.kdim, splitting,
               fac, gscr, stride, bad);
  else
    ADS_LAUNCH((k_block_factor<FT, false>), dim3(nsub), dim3(FAC_T), 0, s, c.lptr_off, c.lcol,
               c.lval, c.lsum, c.om_int, c.om_off, c.ni, c.bs, c.nb, c.fac_off, c.kdim, splitting,
               fac, gscr, stride, bad);
  std::vector<int32_t> hb;
  download(hb, bad, 1, s);
  if (gscr) c.mem.release(gscr);
  if (hb[0])
    fail(ADS_ERR_SINGULAR, std::string("zero pivot in the ") + (splitting ? "splitting" : "local matrix") +
                               " of subdomain " + std::to_string(hb[0] - 1));
}

void factor_local(Ctx& c) {
  const int nsub = c.nsub;
  c.h_fac_off.assign(nsub + 1, 0);
  const int V = c.prec == ADS_PREC_FP64 ? 2 : (c.prec == ADS_PREC_FP32 ? 4 : 8);
  for (int i = 0; i < nsub; ++i)
    c.h_fac_off[i + 1] = c.h_fac_off[i] + (int64_t)2 * c.h_nb[i] * adsd::tile_size(c.h_bs[i], V);
  c.fac_elems = c.h_fac_off[nsub];
  c.fac_off = upload(c.mem, c.h_fac_off.data(), nsub + 1, c.stream);
  const bool need_split = c.opt.variant == ADS_VARIANT_DEFLATED && c.opt.nev > 0;
  size_t esz = c.prec == ADS_PREC_FP64 ? 8 : (c.prec == ADS_PREC_FP32 ? 4 : 2);
  c.factor_bytes = (int64_t)(c.fac_elems * esz);
  bool fast = c.cpl_ok;
  for (int i = 0; i < nsub; ++i) fast = fast && factor_fast_ok(c.h_bs[i]);
  if (fast) {
    switch (c.prec) {
      case ADS_PREC_FP64: factor_fast<double>(c, need_split); break;
      case ADS_PREC_FP32: factor_fast<float>(c, need_split); break;
      default: factor_fast<__hip_bfloat16>(c, need_split); break;
    }
    return;
  }
  switch (c.prec) {
    case ADS_PREC_FP64:
      factor_one<double>(c, 0, &c.facA);
      if (need_split) factor_one<double>(c, 1, &c.facT);
      break;
    case ADS_PREC_FP32:
      factor_one<float>(c, 0, &c.facA);
      if (need_split) factor_one<float>(c, 1, &c.facT);
      break;
    default:
      factor_one<__hip_bfloat16>(c, 0, &c.facA);
      if (need_split) factor_one<__hip_bfloat16>(c, 1, &c.facT);
      break;
  }
}

}  // namespace ads
