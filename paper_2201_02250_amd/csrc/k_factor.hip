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

namespace ads {

static constexpr int FAC_T = 256;

template <class FT>
__global__ void __launch_bounds__(FAC_T)
k_block_factor(const int64_t* lrow, const int32_t* lcol, const double* lval, const double* lsum,
               const uint8_t* om_int, const int64_t* om_off, const int32_t* ni,
               const int32_t* bsz, const int32_t* nblk, const int64_t* fac_off,
               const int32_t* kdim, int splitting, FT* fac, double* gscr, int64_t gscr_stride,
               int use_lds, int32_t* bad_pivot) {
  extern __shared__ double lds[];
  const int i = blockIdx.x;
  const int s = bsz[i], K = nblk[i], n = ni[i];
  const int t = threadIdx.x, T = blockDim.x;
  double* D = use_lds ? lds : gscr + (int64_t)i * gscr_stride;
  double* Pp = D + (int64_t)s * s;
  double* colp = Pp + (int64_t)s * s;
  const int64_t rbase = om_off[i];
  const bool regularise = splitting && kdim[i];
  FT* F = fac + fac_off[i];
  const int64_t ss = (int64_t)s * s;

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
    // store G_k column-major: element (r, c) at r + c*s
    FT* G = F + (int64_t)k * 2 * ss;
    for (int64_t e = t; e < ss; e += T) {
      const int cc = (int)(e / s), rr = (int)(e - (int64_t)cc * s);
      adsd::st_fac(G, e, D[(int64_t)rr * s + cc]);
    }
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
      FT* P = G + ss;
      for (int64_t e = t; e < ss; e += T) {
        const int cc = (int)(e / s), rr = (int)(e - (int64_t)cc * s);
        adsd::st_fac(P, e, Pp[(int64_t)rr * s + cc]);
      }
    }
    __syncthreads();
  }
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
  ADS_LAUNCH((k_block_factor<FT>), dim3(nsub), dim3(FAC_T), use_lds ? need : 0, s, c.lptr_off,
             c.lcol, c.lval, c.lsum, c.om_int, c.om_off, c.ni, c.bs, c.nb, c.fac_off, c.kdim,
             splitting, fac, gscr, stride, use_lds, bad);
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
  for (int i = 0; i < nsub; ++i)
    c.h_fac_off[i + 1] = c.h_fac_off[i] + (int64_t)2 * c.h_nb[i] * c.h_bs[i] * c.h_bs[i];
  c.fac_elems = c.h_fac_off[nsub];
  c.fac_off = upload(c.mem, c.h_fac_off.data(), nsub + 1, c.stream);
  const bool need_split = c.opt.variant == ADS_VARIANT_DEFLATED && c.opt.nev > 0;
  size_t esz = c.prec == ADS_PREC_FP64 ? 8 : (c.prec == ADS_PREC_FP32 ? 4 : 2);
  c.factor_bytes = (int64_t)(c.fac_elems * esz);
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
