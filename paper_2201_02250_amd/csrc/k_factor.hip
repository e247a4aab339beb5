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
// For complex A (kernel dimension 2 in the real form) both real diagonal
// entries of the last unknown are doubled: the real form of adding the real
// part of its complex diagonal entry there, a complex rank-one change of the
// same kind (any nonzero one gives the same solutions in range(splitting)).
//
// One workgroup per subdomain; the block D_k and the previous P tile live in
// LDS when 2 s^2 doubles fit, otherwise in a per-workgroup global scratch.
// Inversion is Gauss-Jordan without pivoting in FP64; tiles are stored in the
// precision of the context.
#include <algorithm>
#include <type_traits>

#include "ads_internal.h"
#include "k_gj.h"
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
          if (regularise && r >= n - kdim[i]) a *= 2.0;
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

// ---------------------------------------------------------------------------
// Fast path: two-ended block factorization, register-resident Gauss-Jordan.
//
// With M = K / 2 the chain is split in two (a "twisted" factorization):
//   top    (k = 0 .. M-1):    D_k = A_kk - A_k,k-1 P_{k-1},  G_k = D_k^{-1},
//                              P_k = G_k A_k,k+1
//   bottom (k = K-1 .. M+1):  E_k = A_kk - A_k,k+1 Q_{k+1}, G_k = E_k^{-1},
//                              Q_k = G_k A_k,k-1
//   middle:                   C = A_MM - A_M,M-1 P_{M-1} - A_M,M+1 Q_{M+1},
//                              G_M = C^{-1}
// Per block the tiles are (G_k, P_k) above the middle, (G_k, Q_k) below it,
// (G_M, unused) at it.  A solve is then two independent chains of about K/2
// dependent steps each (forward from both ends, the middle block, backward
// towards both ends) instead of one chain of 2K - 1 steps; the two halves of
// the factorization run in parallel as well.
//
// Thread t owns column j = t % s of D_k for the rows g, g + G, g + 2G, ...
// (g = t / s, G = 1024 / s, at most FMR rows).  Schur updates and the next
// tile use the fixed-width coupling lists.  Gauss-Jordan takes one barrier
// per pivot: the owners of the next pivot row and column publish them into
// the other half of a double buffer while they update.
// ---------------------------------------------------------------------------
struct FacArgs {
  const int64_t* lrow;
  const int32_t* lcol;
  const double* lval;
  const double* lsum;
  const uint8_t* om_int;
  const int64_t* om_off;
  const int32_t* ni;
  const int32_t* bs;
  const int32_t* nb;
  const int64_t* fac_off;
  const int32_t* kdim;
  const int64_t* pad_off;
  const int32_t* cpl_col;   // A_k,k-1 by row
  const double* cpl_val;
  const int32_t* rcpl_col;  // A_k,k+1 by row
  const double* rcpl_val;
  const int32_t* ucpl_row;  // A_k-1,k by column
  const double* ucpl_val;
  const int32_t* lcpl_row;  // A_k+1,k by column
  const double* lcpl_val;
  double* gscr;             // per (subdomain, matrix) work when LDS is too small
  int64_t gscr_stride;
  double* mid;              // per (subdomain, matrix, half): the FP64 tile next to the middle
  int64_t mid_stride;
  int32_t* bad_pivot;
  const int32_t* order;  // subdomain of each block (longest chains first)
};

// Per-workgroup state of the register-resident block factorization.
template <class FT, int FMR>
struct BlockFac {
  const FacArgs& a;
  int i, splitting, s, K, n, t, G, j, g, nr;
  int64_t rbase, pbase, TS;
  double *D, *Pp, *rowb, *colb;
  double v[FMR];
  __device__ BlockFac(const FacArgs& a_, int i_, int sp, double* base) : a(a_), i(i_), splitting(sp) {
    s = a.bs[i];
    K = a.nb[i];
    n = a.ni[i];
    t = threadIdx.x;
    G = blockDim.x / s;
    j = t % s;
    g = t / s;
    nr = g < G ? (s - g + G - 1) / G : 0;
    rbase = a.om_off[i];
    pbase = a.pad_off[i];
    TS = adsd::tile_size(s, adsd::TileV<FT>::V);
    D = base;
    Pp = D + (int64_t)s * s;
    rowb = Pp + (int64_t)s * s;  // [2][s]
    colb = rowb + 2 * s;         // [2][s]
  }

  // D = A_kk (the splitting diagonal on Definition-1 rows, the regularised
  // last entry on floating subdomains, identity on padding rows)
  __device__ void assemble(int k) {
    const int r0 = k * s, ss = s * s;
    const bool regularise = splitting && a.kdim[i];
    __syncthreads();
    for (int e = t; e < ss; e += blockDim.x) D[e] = 0.0;
    __syncthreads();
    for (int rr = t; rr < s; rr += blockDim.x) {
      const int r = r0 + rr;
      if (r >= n) {
        D[rr * s + rr] = 1.0;
        continue;
      }
      const int64_t f = rbase + r;
      for (int64_t q = a.lrow[f]; q < a.lrow[f + 1]; ++q) {
        const int cc = a.lcol[q] - r0;
        if (cc < 0 || cc >= s) continue;
        double x = a.lval[q];
        if (cc == rr && splitting) {
          if (!a.om_int[f]) x -= a.lsum[f];
          if (regularise && r >= n - a.kdim[i]) x *= 2.0;
        }
        D[rr * s + cc] = x;
      }
    }
    __syncthreads();
  }

  // D -= C Pp with C the row coupling list (ccol, cval) of block k
  __device__ void schur(int k, const int32_t* ccol, const double* cval) {
    const int r0 = k * s;
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
    __syncthreads();
  }

  // D <- D^{-1} (Gauss-Jordan without pivoting, registers, one barrier per pivot)
  __device__ void invert() {
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
    int gn = 0, mn = 0;  // owner of row p + 1: group gn, slot mn
    for (int p = 0; p < s; ++p) {
      const double* rw = rowb + (p & 1) * s;
      const double* cl = colb + (p & 1) * s;
      double* rwn = rowb + ((p + 1) & 1) * s;
      double* cln = colb + ((p + 1) & 1) * s;
      // all LDS reads of the step first, then the arithmetic
      double piv = rw[p];
      const double rwj = rw[j];
      double cvs[FMR];
#pragma unroll
      for (int m = 0; m < FMR; ++m) cvs[m] = cl[m < nr ? g + m * G : 0];
      if (!(fabs(piv) > 0.0) || !isfinite(piv)) {
        if (t == 0) atomicMax(a.bad_pivot, i + 1);
        piv = 1.0;
      }
      // 1 / pivot: hardware reciprocal refined by two Newton steps
      double inv = __builtin_amdgcn_rcp(piv);
      inv = inv * (2.0 - piv * inv);
      inv = inv * (2.0 - piv * inv);
      const double rj = rwj * inv;
      const bool jc = j == p;
      // v - c_r * (row p / pivot) everywhere; row p takes the scaled row (the
      // pivot itself 1 / pivot); column p is fixed up below
      const double rowv = jc ? inv : rj;
#pragma unroll
      for (int m = 0; m < FMR; ++m) {
        const double x = v[m] - cvs[m] * rj;
        v[m] = (g + m * G == p) ? rowv : x;
      }
      if (jc) {
#pragma unroll
        for (int m = 0; m < FMR; ++m)
          if (g + m * G != p) v[m] = -cvs[m] * inv;
      }
      const int pn = p + 1;
      if (++gn == G) {
        gn = 0;
        ++mn;
      }
      if (pn < s) {
        if (g == gn) {
          double xr = v[0];
#pragma unroll
          for (int m = 1; m < FMR; ++m) xr = (m == mn) ? v[m] : xr;
          rwn[j] = xr;
        }
        if (j == pn)
#pragma unroll
          for (int m = 0; m < FMR; ++m)
            if (m < nr) cln[g + m * G] = v[m];
      }
      __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < FMR; ++m)
      if (m < nr) D[(g + m * G) * s + j] = v[m];
    __syncthreads();
  }

  // Pp[rho][c'] = sum_m D[rho][row_m] val_m over the column list of block kc
  // (D holds G_k; the list entries are rows of block k)
  __device__ void next_tile(int kc, const int32_t* crow, const double* cval) {
    const int ss = s * s;
    for (int e = t; e < ss; e += blockDim.x) {
      const int cp = e / s, rho = e - cp * s;
      const int64_t ub = (pbase + (int64_t)kc * s + cp) * adsd::NCPL;
      double x = 0.0;
#pragma unroll
      for (int q = 0; q < adsd::NCPL; ++q) {
        const int rr = crow[ub + q];
        if (rr >= 0) x += D[rho * s + rr] * cval[ub + q];
      }
      Pp[rho * s + cp] = x;
    }
    __syncthreads();
  }
};

template <class FT, bool USE_LDS, int FMR>
__global__ void __launch_bounds__(1024) k_factor_chain(FacArgs a, FT* facA, FT* facT) {
  extern __shared__ double lds[];
  const int i = adsd::sub_of(a.order, blockIdx.x), splitting = blockIdx.y, half = blockIdx.z;
  double* base = USE_LDS ? lds
                         : a.gscr + (((int64_t)splitting * gridDim.x + i) * 2 + half) * a.gscr_stride;
  BlockFac<FT, FMR> B(a, i, splitting, base);
  const int s = B.s, K = B.K, M = K / 2;
  const int k0 = half ? K - 1 : 0, dk = half ? -1 : 1, nsteps = half ? K - 1 - M : M;
  const int32_t* schur_col = half ? a.rcpl_col : a.cpl_col;
  const double* schur_val = half ? a.rcpl_val : a.cpl_val;
  const int32_t* nxt_row = half ? a.lcpl_row : a.ucpl_row;
  const double* nxt_val = half ? a.lcpl_val : a.ucpl_val;
  FT* F = (splitting ? facT : facA) + a.fac_off[i];
  constexpr int V = adsd::TileV<FT>::V;
  for (int q = 0; q < nsteps; ++q) {
    const int k = k0 + q * dk;
    B.assemble(k);
    if (q > 0) B.schur(k, schur_col, schur_val);
    B.invert();
    FT* Gt = F + (int64_t)k * 2 * B.TS;
    store_tile(Gt, B.D, s, V);
    B.next_tile(k + dk, nxt_row, nxt_val);
    store_tile(Gt + B.TS, B.Pp, s, V);
  }
  if (nsteps > 0) {  // the tile next to the middle block, in FP64
    double* mid = a.mid + (((int64_t)splitting * gridDim.x + i) * 2 + half) * a.mid_stride;
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) mid[e] = B.Pp[e];
  }
}

template <class FT, bool USE_LDS, int FMR>
__global__ void __launch_bounds__(1024) k_factor_mid(FacArgs a, FT* facA, FT* facT) {
  extern __shared__ double lds[];
  const int i = adsd::sub_of(a.order, blockIdx.x), splitting = blockIdx.y;
  double* base = USE_LDS ? lds : a.gscr + ((int64_t)splitting * gridDim.x + i) * 2 * a.gscr_stride;
  BlockFac<FT, FMR> B(a, i, splitting, base);
  const int s = B.s, K = B.K, M = K / 2;
  B.assemble(M);
  for (int half = 0; half < 2; ++half) {
    if (half == 0 ? M == 0 : M + 1 > K - 1) continue;
    const double* mid = a.mid + (((int64_t)splitting * gridDim.x + i) * 2 + half) * a.mid_stride;
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) B.Pp[e] = mid[e];
    __syncthreads();
    B.schur(M, half ? a.rcpl_col : a.cpl_col, half ? a.rcpl_val : a.cpl_val);
  }
  B.invert();
  FT* F = (splitting ? facT : facA) + a.fac_off[i];
  FT* Gt = F + (int64_t)M * 2 * B.TS;
  store_tile(Gt, B.D, s, adsd::TileV<FT>::V);
  for (int64_t e = threadIdx.x; e < B.TS; e += blockDim.x) adsd::st_fac(Gt + B.TS, e, 0.0);
}

template <class FT>
static void factor_fast(Ctx& c, bool both) {
  hipStream_t st = c.stream;
  const int nsub = c.nsub;
  FT* fa = c.mem.alloc<FT>(c.fac_elems);
  FT* ft = both ? c.mem.alloc<FT>(c.fac_elems) : nullptr;
  c.facA = fa;
  c.facT = ft;
  const int nmat = both ? 2 : 1;
  int smax = *std::max_element(c.h_bs.begin(), c.h_bs.end());
  size_t need = ((size_t)2 * smax * smax + 4 * smax) * sizeof(double);
  const bool use_lds = need <= 150 * 1024;
  FacArgs a{};
  a.order = c.sub_order;
  a.lrow = c.lptr_off;
  a.lcol = c.lcol;
  a.lval = c.lval;
  a.lsum = c.lsum;
  a.om_int = c.om_int;
  a.om_off = c.om_off;
  a.ni = c.ni;
  a.bs = c.bs;
  a.nb = c.nb;
  a.fac_off = c.fac_off;
  a.kdim = c.kdim;
  a.pad_off = c.pad_off;
  a.cpl_col = c.cpl_col;
  a.cpl_val = c.cpl_val;
  a.rcpl_col = c.rcpl_col;
  a.rcpl_val = c.rcpl_val;
  a.ucpl_row = c.ucpl_row;
  a.ucpl_val = c.ucpl_val;
  a.lcpl_row = c.lcpl_row;
  a.lcpl_val = c.lcpl_val;
  a.gscr_stride = (int64_t)2 * smax * smax + 4 * smax;
  a.gscr = use_lds ? nullptr : c.mem.alloc<double>((size_t)a.gscr_stride * nsub * nmat * 2);
  a.mid_stride = (int64_t)smax * smax;
  a.mid = c.mem.alloc<double>((size_t)a.mid_stride * nsub * nmat * 2);
  a.bad_pivot = c.mem.alloc<int32_t>(1);
  ADS_HIP(hipMemsetAsync(a.bad_pivot, 0, 4, st));
  int rmax = 1;
  for (int b : c.h_bs) rmax = std::max(rmax, adsd::factor_rows(b));
  auto launch = [&](auto lds_tag, auto fmr_tag) {
    constexpr bool L = decltype(lds_tag)::value;
    constexpr int R = decltype(fmr_tag)::value;
    ADS_LAUNCH((k_factor_chain<FT, L, R>), dim3(nsub, nmat, 2), dim3(1024), L ? need : 0, st, a, fa,
               ft);
    ADS_LAUNCH((k_factor_mid<FT, L, R>), dim3(nsub, nmat), dim3(1024), L ? need : 0, st, a, fa, ft);
  };
  auto by_rows = [&](auto lds_tag) {
    if (rmax <= 2) launch(lds_tag, std::integral_constant<int, 2>());
    else if (rmax <= 3) launch(lds_tag, std::integral_constant<int, 3>());
    else if (rmax <= 5) launch(lds_tag, std::integral_constant<int, 5>());
    else if (rmax <= 7) launch(lds_tag, std::integral_constant<int, 7>());
    else launch(lds_tag, std::integral_constant<int, 9>());
  };
  if (use_lds)
    by_rows(std::true_type());
  else
    by_rows(std::false_type());
  std::vector<int32_t> hb;
  download(hb, a.bad_pivot, 1, st);
  if (a.gscr) c.mem.release(a.gscr);
  c.mem.release(a.mid);
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

// ---------------------------------------------------------------------------
// Batched general factorization (block sizes beyond the register-resident
// fast path, coupling lists complete): block step k of every subdomain at
// once, in three passes over the whole GPU instead of one workgroup per
// subdomain:
//   build : D_k = A_kk - A_k,k-1 P_{k-1} in FP64, row-major (the Schur update
//           through the coupling list of A_k,k-1 by row, P_{k-1} kept in FP64);
//   invert: G_k = D_k^{-1} by the batched Gauss-Jordan elimination with
//           partial pivoting (one row per thread up to s = 1024);
//   store : the packed tiles G_k and P_k = G_k A_k,k+1 (the coupling list of
//           A_k,k+1 by column, rows ascending), and P_k in FP64 for step k + 1.
// Subdomains with fewer than k + 1 blocks invert an identity at step k.
// ---------------------------------------------------------------------------
struct BfArgs {
  const int64_t* lrow;
  const int32_t* lcol;
  const double* lval;
  const double* lsum;
  const uint8_t* om_int;
  const int64_t* om_off;
  const int32_t* ni;
  const int32_t* bs;
  const int32_t* nb;
  const int64_t* fac_off;
  const int32_t* kdim;
  const int64_t* pad_off;
  const int32_t* cpl_col;   // A_k,k-1 by row
  const double* cpl_val;
  const int32_t* ucpl_row;  // A_k-1,k by column
  const double* ucpl_val;
  const int64_t* d_off;     // per subdomain: start of its s_i x s_i FP64 work matrices
};

static constexpr int BF_U = 4;  // independent elements per thread and pass (loads in flight)

// D_k rows rr0 .. rr0 + rb - 1 of every subdomain (grid: subdomain x row
// groups; rb * (largest s) doubles of LDS).  Each wave takes rows rr0 + w,
// rr0 + w + (waves), ...: first its lanes scatter the row's entries of A_kk
// (the splitting's diagonal changes included; the columns of a row are
// unique) into LDS, then every element takes its entry and subtracts the
// Schur terms of the row's A_k,k-1 couplings (uniform per row), BF_U
// elements per lane at a time so that their loads of P_{k-1} are in flight
// together.
__global__ void __launch_bounds__(256)
k_bf_build(BfArgs a, int k, int splitting, double* D, const double* Pp, int rb) {
  extern __shared__ double Ls[];
  const int i = blockIdx.x;
  const int s = a.bs[i], K = a.nb[i], n = a.ni[i];
  const int rr0 = blockIdx.y * rb;
  if (rr0 >= s) return;
  const int nr = min(rb, s - rr0), tot = nr * s;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double* Di = D + a.d_off[i] + (int64_t)rr0 * s;
  const double* Pi = Pp + a.d_off[i];
  const int r0 = k * s;
  const bool regularise = splitting && a.kdim[i];
  for (int e = threadIdx.x; e < tot; e += blockDim.x) Ls[e] = 0.0;
  __syncthreads();
  for (int rr = w; rr < nr; rr += nw) {
    const int row = rr0 + rr, r = r0 + row;
    double* L = Ls + rr * s;
    if (k >= K || r >= n) {  // identity rows: past the last block, or padding
      if (lane == 0) L[row] = 1.0;
      continue;
    }
    const int64_t f = a.om_off[i] + r;
    for (int64_t q = a.lrow[f] + lane; q < a.lrow[f + 1]; q += 64) {
      const int j = a.lcol[q] - r0;
      if (j < 0 || j >= s) continue;
      double x = a.lval[q];
      if (j == row && splitting) {
        if (!a.om_int[f]) x -= a.lsum[f];
        if (regularise && r >= n - a.kdim[i]) x *= 2.0;
      }
      L[j] = x;
    }
  }
  __syncthreads();
  for (int rr = w; rr < nr; rr += nw) {
    const int r = r0 + rr0 + rr;
    int cc[adsd::NCPL];
    double cv[adsd::NCPL];
    const bool schur = k > 0 && k < K && r < n;
    const int64_t fp = (a.pad_off[i] + (schur ? r : 0)) * adsd::NCPL;  // coupling slots of this row
#pragma unroll
    for (int m = 0; m < adsd::NCPL; ++m) {
      cc[m] = schur ? a.cpl_col[fp + m] : -1;
      cv[m] = schur ? a.cpl_val[fp + m] : 0.0;
    }
    const double* L = Ls + rr * s;
    double* Dr = Di + (int64_t)rr * s;
    for (int j0 = lane; j0 < s; j0 += 64 * BF_U) {
      double v[BF_U];
#pragma unroll
      for (int u = 0; u < BF_U; ++u) {
        const int j = min(j0 + 64 * u, s - 1);
        double x = L[j];
#pragma unroll
        for (int m = 0; m < adsd::NCPL; ++m)
          if (cc[m] >= 0) x -= cv[m] * Pi[(int64_t)cc[m] * s + j];
        v[u] = x;
      }
#pragma unroll
      for (int u = 0; u < BF_U; ++u)
        if (j0 + 64 * u < s) Dr[j0 + 64 * u] = v[u];
    }
  }
}

// G_k = D_k^{-1} (row-major, from the batched inversion) and P_k = G_k
// A_k,k+1 into the packed tiles, and P_k (FP64, row-major) for the next block
// step.  One workgroup per (subdomain, rb rows): the rows of G_k are read
// into LDS with coalesced loads, P_k's rows are formed there from the column
// coupling list (at most NCPL entries per column of A_k,k+1), and both tiles
// are written in their packed order, where the rb rows of one 16-byte column
// group are contiguous.
template <class FT>
__global__ void __launch_bounds__(256)
k_bf_store(BfArgs a, int k, const double* Ginv, double* Pp, FT* fac, int rb) {
  extern __shared__ double sh[];
  const int i = blockIdx.x;
  const int s = a.bs[i], K = a.nb[i];
  const int r0 = blockIdx.y * rb;
  if (k >= K || r0 >= s) return;
  const int nr = min(rb, s - r0);
  constexpr int V = adsd::TileV<FT>::V;
  const int64_t TS = adsd::tile_size(s, V);
  const int nq = (s + V - 1) / V;
  double* Gs = sh;
  double* Ps = sh + (int64_t)rb * s;
  const double* G = Ginv + a.d_off[i] + (int64_t)r0 * s;
  const int tot = nr * s;
  for (int e0 = threadIdx.x; e0 < tot; e0 += BF_U * blockDim.x) {  // BF_U loads in flight
    double v[BF_U];
#pragma unroll
    for (int u = 0; u < BF_U; ++u) v[u] = G[min(e0 + u * (int)blockDim.x, tot - 1)];
#pragma unroll
    for (int u = 0; u < BF_U; ++u)
      if (e0 + u * (int)blockDim.x < tot) Gs[e0 + u * blockDim.x] = v[u];
  }
  __syncthreads();
  const bool more = k + 1 < K;
  if (more) {
    // one column of A_k,k+1 per thread: its coupling list once, then its
    // entries of the nr rows of P_k
    const int64_t cbase = a.pad_off[i] + (int64_t)(k + 1) * s;  // padded columns of block k + 1
    double* P = Pp + a.d_off[i] + (int64_t)r0 * s;
    for (int cidx = threadIdx.x; cidx < s; cidx += blockDim.x) {
      const int64_t fc = (cbase + cidx) * adsd::NCPL;
      int rw[adsd::NCPL];
      double uv[adsd::NCPL];
#pragma unroll
      for (int m = 0; m < adsd::NCPL; ++m) {
        rw[m] = a.ucpl_row[fc + m];
        uv[m] = a.ucpl_val[fc + m];
      }
      for (int rr = 0; rr < nr; ++rr) {
        double pv = 0.0;
#pragma unroll
        for (int m = 0; m < adsd::NCPL; ++m)
          if (rw[m] >= 0) pv += Gs[rr * s + rw[m]] * uv[m];
        Ps[rr * s + cidx] = pv;
        P[(int64_t)rr * s + cidx] = pv;
      }
    }
    __syncthreads();
  }
  FT* Gt = fac + a.fac_off[i] + (int64_t)k * 2 * TS;
  const int run = nr * V;  // contiguous entries per column group
  for (int e = threadIdx.x; e < nq * run; e += blockDim.x) {
    const int q = e / run, rem = e % run, rr = rem / V, v = rem % V;
    const int cidx = q * V + v;
    const int64_t dst = ((int64_t)q * s + r0 + rr) * V + v;
    const bool in = cidx < s;
    adsd::st_fac(Gt, dst, in ? Gs[rr * s + cidx] : 0.0);
    if (more) adsd::st_fac(Gt + TS, dst, in ? Ps[rr * s + cidx] : 0.0);
  }
}

template <class FT>
static void factor_batched(Ctx& c, int splitting, void** out) {
  hipStream_t st = c.stream;
  const int nsub = c.nsub;
  FT* fac = c.mem.alloc<FT>(c.fac_elems);
  *out = fac;
  constexpr int V = adsd::TileV<FT>::V;
  std::vector<int64_t> hd(nsub + 1, 0);
  int smax = 0, kmax = 0;
  for (int i = 0; i < nsub; ++i) {
    const int b = c.h_bs[i];
    hd[i + 1] = hd[i] + (int64_t)b * b;
    smax = std::max(smax, b);
    kmax = std::max(kmax, (int)c.h_nb[i]);
  }
  int64_t* d_off = upload(c.mem, hd.data(), nsub + 1, st);
  double* D = c.mem.alloc<double>(hd[nsub]);
  double* F = c.mem.alloc<double>(hd[nsub]);
  double* Pp = c.mem.alloc<double>(hd[nsub]);
  BfArgs a{c.lptr_off, c.lcol, c.lval, c.lsum, c.om_int, c.om_off, c.ni, c.bs, c.nb, c.fac_off,
           c.kdim, c.pad_off, c.cpl_col, c.cpl_val, c.ucpl_row, c.ucpl_val, d_off};
  // rows of D_k per workgroup of the build pass (their A_kk entries in LDS)
  const int rbb = std::max(1, std::min(8, 4096 / std::max(smax, 1)));
  const dim3 gb(nsub, (unsigned)((smax + rbb - 1) / rbb));
  const size_t bd_lds = (size_t)rbb * smax * 8;
  // rows of G_k per workgroup of the store pass: G and P rows in LDS
  const int rb = std::max(1, std::min(8, 10240 / std::max(smax, 1)));
  const dim3 gs(nsub, (unsigned)((smax + rb - 1) / rb));
  const size_t st_lds = (size_t)2 * rb * smax * 8;
  // block step k inverts the D_k of the subdomains that still have a block
  // k (a batch of the active ones, at offsets into the same buffers, with
  // their own largest order), so subdomains of few large blocks are not
  // inverted again while others with many small blocks continue
  std::vector<std::vector<int32_t>> act(kmax);
  std::vector<int64_t> h_eoff;
  std::vector<int32_t> h_soff;
  std::vector<size_t> at_e(kmax), at_s(kmax);
  for (int k = 0; k < kmax; ++k) {
    for (int i = 0; i < nsub; ++i)
      if (k < c.h_nb[i]) act[k].push_back(i);
    at_e[k] = h_eoff.size();
    at_s[k] = h_soff.size();
    int32_t so = 0;
    h_soff.push_back(0);
    for (int i : act[k]) {
      h_eoff.push_back(hd[i]);
      so += c.h_bs[i];
      h_soff.push_back(so);
    }
  }
  int64_t* eoff = upload(c.mem, h_eoff.data(), std::max<size_t>(h_eoff.size(), 1), st);
  int32_t* soff = upload(c.mem, h_soff.data(), h_soff.size(), st);
  int32_t* bads = c.mem.alloc<int32_t>(kmax);  // per step: active index + 1 of a zero pivot
  ADS_HIP(hipMemsetAsync(bads, 0, (size_t)kmax * 4, st));
  std::vector<int32_t> orders;
  for (int k = 0; k < kmax; ++k) {
    const int na = (int)act[k].size();
    int smx = 0;
    int64_t tot = 0;
    orders.assign(na, 0);
    for (int j = 0; j < na; ++j) {
      const int b = c.h_bs[act[k][j]];
      smx = std::max(smx, b);
      tot += (int64_t)b * b;
      orders[j] = b;
    }
    const int64_t* ek = eoff + at_e[k];
    const int32_t* sk = soff + at_s[k];
    const int64_t nrow = h_soff[at_s[k] + na];
    ADS_LAUNCH(k_bf_build, gb, dim3(256), bd_lds, st, a, k, splitting, D, Pp, rbb);
    // symmetric A: the D_k are symmetric positive definite (Schur complements
    // of the SPD local matrices), inverted without interchanges; a pivot that
    // is not positive sends this block step back to partial pivoting
    double* inv =
        gj_invert_batched(c, st, na, smx, nrow, tot, D, F, ek, sk, bads + k, c.sym, orders.data());
    if (!inv) {
      ADS_LAUNCH(k_bf_build, gb, dim3(256), bd_lds, st, a, k, splitting, D, Pp, rbb);
      inv = gj_invert_batched(c, st, na, smx, nrow, tot, D, F, ek, sk, bads + k, false,
                              orders.data());
    }
    ADS_LAUNCH((k_bf_store<FT>), gs, dim3(256), st_lds, st, a, k, inv, Pp, fac, rb);
  }
  std::vector<int32_t> hb;
  download(hb, bads, kmax, st);
  for (void* q : {(void*)D, (void*)F, (void*)Pp, (void*)d_off, (void*)eoff, (void*)soff,
                  (void*)bads})
    c.mem.release(q);
  for (int k = 0; k < kmax; ++k)
    if (hb[k])
      fail(ADS_ERR_SINGULAR, std::string("zero pivot in the ") + (splitting ? "splitting" : "local matrix") +
                                 " of subdomain " + std::to_string(act[k][hb[k] - 1]));
}

void release_factors(Ctx& c) {
  for (void** p : {&c.facA, &c.facT, (void**)&c.fac_off})
    if (*p) {
      c.mem.release(*p);
      *p = nullptr;
    }
}

void factor_local(Ctx& c, bool only_a) {
  const int nsub = c.nsub;
  c.h_fac_off.assign(nsub + 1, 0);
  const int V = c.prec == ADS_PREC_FP64 ? 2 : (c.prec == ADS_PREC_FP32 ? 4 : 8);
  for (int i = 0; i < nsub; ++i)
    c.h_fac_off[i + 1] = c.h_fac_off[i] + (int64_t)2 * c.h_nb[i] * adsd::tile_size(c.h_bs[i], V);
  c.fac_elems = c.h_fac_off[nsub];
  c.fac_off = upload(c.mem, c.h_fac_off.data(), nsub + 1, c.stream);
  const bool need_split = !only_a && variant_has_coarse(c.opt.variant) && c.opt.nev > 0;
  size_t esz = c.prec == ADS_PREC_FP64 ? 8 : (c.prec == ADS_PREC_FP32 ? 4 : 2);
  c.factor_bytes = (int64_t)(c.fac_elems * esz);
  if (c.solve_fast) {  // two-ended layout, read by the fast solves
    switch (c.prec) {
      case ADS_PREC_FP64: factor_fast<double>(c, need_split); break;
      case ADS_PREC_FP32: factor_fast<float>(c, need_split); break;
      default: factor_fast<__hip_bfloat16>(c, need_split); break;
    }
    return;
  }
  if (c.cpl_ok) {  // block sizes beyond the fast path: batched block steps
    switch (c.prec) {
      case ADS_PREC_FP64:
        factor_batched<double>(c, 0, &c.facA);
        if (need_split) factor_batched<double>(c, 1, &c.facT);
        break;
      case ADS_PREC_FP32:
        factor_batched<float>(c, 0, &c.facA);
        if (need_split) factor_batched<float>(c, 1, &c.facT);
        break;
      default:
        factor_batched<__hip_bfloat16>(c, 0, &c.facA);
        if (need_split) factor_batched<__hip_bfloat16>(c, 1, &c.facT);
        break;
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
