// Batched dense inversion by blocked Gauss-Jordan elimination with partial
// pivoting, shared by the coarse operator (E_s of each system) and the
// factorization of the local matrices (the diagonal blocks D_k of every
// subdomain at once).
#pragma once
#include <algorithm>
#include <string>

#include "ads_internal.h"

namespace ads {
namespace {  // one copy of the kernels per translation unit

// ---------------------------------------------------------------------------
// Explicit inverse of each dense E_s by blocked Gauss-Jordan elimination with
// partial pivoting (row interchanges, the usual column un-permutation at the
// end).  Column blocks of width nb are processed in turn:
//   panel kernel : one workgroup per system runs the unblocked in-place
//                  Gauss-Jordan steps on the n x nb column panel held in LDS,
//                  records the pivots, writes the panel result S (the panel
//                  columns of the accumulated transform) and the composed row
//                  source map src of the block's interchanges;
//   update kernel: every other column receives the same transform as a rank-nb
//                  product, out(i, j) = in(src i, j) + sum_l (S(i,l) - [i = k0+l]) in(src(k0+l), j),
//                  written to the other buffer of a ping-pong pair (no in-place
//                  races between tiles); the panel columns receive S.
// Every reduction has a fixed order, so the result is deterministic.
// ---------------------------------------------------------------------------
static constexpr int GJ_T = 1024;
static constexpr int GJ_UT = 256;
static constexpr int GJ_TILE = 32;
static constexpr size_t GJ_LDS_MAX = 150 * 1024;

// largest power-of-two panel width <= 32 whose panel fits the LDS budget
static int gj_panel_width(int64_t n) {
  int nb = 32;
  while (nb > 1 && (size_t)n * (nb * 8 + 8 + 4) + 4096 > GJ_LDS_MAX) nb >>= 1;
  return ((size_t)n * (nb * 8 + 8 + 4) + 4096 > GJ_LDS_MAX) ? 0 : nb;
}

// (value, index) max with ties to the smaller index; NaN never wins
__device__ __forceinline__ void gj_better(double& bv, int& bi, double v, int i) {
  if (v > bv || (v == bv && i < bi)) {
    bv = v;
    bi = i;
  }
}

// HBM = false: the panel, the saved pivot column and the row sources live in
// LDS (n (8 nb + 12) bytes); HBM = true (systems too large for LDS): the panel
// is worked on in place in its output S, the row sources in src_all and the
// pivot column in fcol_all (n0 doubles), all through the cache hierarchy.
template <bool HBM>
__global__ void __launch_bounds__(GJ_T)
k_gj_panel(const double* Ain, const int64_t* E_off, const int32_t* sys_coff, int k0, int nb,
           double* Sbuf, int32_t* src_all, int32_t* tot_all, double* fcol_all, int32_t* singular) {
  extern __shared__ double gj_lds[];
  __shared__ double rowk[32], rowkold[32];
  __shared__ double pval[GJ_T / 64];
  __shared__ int pidx[GJ_T / 64];
  __shared__ int swp[32];
  const int sy = blockIdx.x;
  const int base = sys_coff[sy];
  const int n = sys_coff[sy + 1] - base;
  if (k0 >= n) return;
  const int kb = min(nb, n - k0);
  const int t = threadIdx.x, T = blockDim.x, lane = t & 63, wv = t >> 6;
  // n x nb panel, row-major; saved pivot column; row sources
  double* P = HBM ? Sbuf + (int64_t)nb * base : gj_lds;
  double* fcol = HBM ? fcol_all + base : P + (size_t)n * nb;
  int* src = HBM ? src_all + base : reinterpret_cast<int*>(fcol + n);
  const double* A = Ain + E_off[sy];
  const int lnb = __ffs(nb) - 1;  // nb is a power of two
  const int ne = n * nb;
  for (int e = t; e < ne; e += T) {
    const int i = e >> lnb, l = e & (nb - 1);
    P[e] = l < kb ? A[(int64_t)i * n + k0 + l] : 0.0;
  }
  for (int i = t; i < n; i += T) src[i] = i;
  __syncthreads();
  // pivot candidates of the first panel column
  double bv = -1.0;
  int bi = n;
  for (int i = k0 + t; i < n; i += T) gj_better(bv, bi, fabs(P[(int64_t)i * nb]), i);
  for (int l = 0; l < kb; ++l) {
    // block-wide argmax of the candidates (wave shuffles, then the partials)
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      gj_better(bv, bi, ov, oi);
    }
    if (lane == 0) {
      pval[wv] = bv;
      pidx[wv] = bi;
    }
    __syncthreads();
    bv = -1.0;
    bi = n;
    for (int w = 0; w < T / 64; ++w) gj_better(bv, bi, pval[w], pidx[w]);
    const int k = k0 + l;
    int p = bi;
    if (!(bv > 0.0) || p >= n) {
      if (t == 0) atomicMax(singular, sy + 1);
      p = k;
    }
    if (t == 0) swp[l] = p;
    // save the pivot column (rows k and p interchanged) and both rows
    for (int i = t; i < n; i += T) {
      const int si = i == k ? p : (i == p ? k : i);
      fcol[i] = P[(int64_t)si * nb + l];
    }
    if (t < nb) {
      rowk[t] = P[(int64_t)p * nb + t];
      rowkold[t] = P[(int64_t)k * nb + t];
    }
    __syncthreads();
    const double v = fcol[k];
    const double d = (v != 0.0) ? 1.0 / v : 1.0;
    bv = -1.0;
    bi = n;
    for (int e = t; e < ne; e += T) {
      const int i = e >> lnb, j = e & (nb - 1);
      const double old = i == k ? rowk[j] : (i == p ? rowkold[j] : P[e]);
      double nw;
      if (i == k)
        nw = j == l ? d : old * d;
      else
        nw = j == l ? -fcol[i] * d : old - fcol[i] * (rowk[j] * d);
      P[e] = nw;
      if (j == l + 1 && i > k) gj_better(bv, bi, fabs(nw), i);
    }
  }
  __syncthreads();
  if (t == 0)
    for (int l = 0; l < kb; ++l) {
      const int k = k0 + l, p = swp[l];
      const int tmp = src[k];
      src[k] = src[p];
      src[p] = tmp;
    }
  __syncthreads();
  if (!HBM) {
    double* S = Sbuf + (int64_t)nb * base;
    for (int e = t; e < ne; e += T) S[e] = P[e];
    int32_t* so = src_all + base;
    for (int i = t; i < n; i += T) so[i] = src[i];
  }
  // cumulative row map: tot(x) <- tot(src(x)), through the pivot column's
  // storage (free by now)
  int32_t* tot = tot_all + base;
  int* tmp = reinterpret_cast<int*>(fcol);
  for (int i = t; i < n; i += T) tmp[i] = k0 == 0 ? src[i] : tot[src[i]];
  __syncthreads();
  for (int i = t; i < n; i += T) tot[i] = tmp[i];
}

// one DPP step of a wave maximum: x = max(x, x of the lane given by CTRL)
template <int CTRL>
__device__ __forceinline__ double gj_dpp_max(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return fmax(x, __longlong_as_double(((long long)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double gj_lane(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// maximum over the 64 lanes (every lane active): pairs, quads, half rows and
// rows of 16 by DPP (quad_perm 1032, quad_perm 2301, row_half_mirror,
// row_mirror), then the four rows by readlane
__device__ __forceinline__ double gj_wave_max(double x) {
  x = gj_dpp_max<0xB1>(x);
  x = gj_dpp_max<0x4E>(x);
  x = gj_dpp_max<0x141>(x);
  x = gj_dpp_max<0x140>(x);
  return fmax(fmax(gj_lane(x, 0), gj_lane(x, 16)), fmax(gj_lane(x, 32), gj_lane(x, 48)));
}

// Register-resident panel for systems of order <= GJ_T (panel width 32):
// thread i owns row i of the n x 32 column panel (rows in the logical order
// that the previous panels left) and tracks the logical position of that
// row; rows never move.  One barrier per pivot step: every wave publishes its
// best pivot candidate (largest |entry| in the pivot column among the rows
// not yet used, ties to the smaller row) together with that row's values in
// a double-buffered LDS slot, and every thread then takes the first slot of
// largest magnitude.  The result S is written in logical row order.
__global__ void __launch_bounds__(GJ_T)
k_gj_panel_row(const double* Ain, const int64_t* E_off, const int32_t* sys_coff, int k0,
               double* Sbuf, int32_t* src_all, int32_t* tot_all, int32_t* singular) {
  constexpr int NB = 32;
  __shared__ double slot_r[2][GJ_T / 64][NB + 1];  // row values, then the key
  __shared__ int slot_q[2][GJ_T / 64][2];          // physical row, logical position
  const int sy = blockIdx.x;
  const int base = sys_coff[sy];
  const int n = sys_coff[sy + 1] - base;
  if (k0 >= n) return;
  const int kb = min(NB, n - k0);
  const int i = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(i >> 6);  // wave-uniform
  const int nw = (int)(blockDim.x + 63) >> 6;
  const bool live = i < n;
  const double* A = Ain + E_off[sy] + (int64_t)(live ? i : 0) * n + k0;
  double v[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const double a = A[min(j, kb - 1)];  // in bounds for every lane
    v[j] = (live && j < kb) ? a : 0.0;
  }
  int pos = i;
  bool sing = false;
  for (int l = 0; l < kb; ++l) {
    const int k = k0 + l, b = l & 1;
    double f = v[0];  // this row's entry in the pivot column
#pragma unroll
    for (int j = 1; j < NB; ++j) f = j == l ? v[j] : f;
    double cand = (live && pos >= k) ? fabs(f) : -1.0;
    if (!(cand >= 0.0)) cand = -1.0;  // NaN never wins
    const double m = gj_wave_max(cand);
    const bool top = cand == m;
    const unsigned long long hit = __ballot(top);
    // the lowest lane holding the maximum: no lane of the ballot below it
    const unsigned below = __builtin_amdgcn_mbcnt_hi((unsigned)(hit >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((unsigned)hit, 0u));
    if (top && below == 0) {
#pragma unroll
      for (int j = 0; j < NB; ++j) slot_r[b][wv][j] = v[j];
      slot_r[b][wv][NB] = m;
      slot_q[b][wv][0] = i;
      slot_q[b][wv][1] = pos;
    }
    __syncthreads();
    int w = 0;
    double best = slot_r[b][0][NB];
    for (int u = 1; u < nw; ++u) {
      const double kv = slot_r[b][u][NB];
      if (kv > best) {
        best = kv;
        w = u;
      }
    }
    w = __builtin_amdgcn_readfirstlane(w);
    const double* r = slot_r[b][w];
    const int q = slot_q[b][w][0], pq = slot_q[b][w][1];
    sing |= !(best > 0.0);
    const double piv = r[l];
    const double inv = piv != 0.0 ? 1.0 / piv : 1.0;
    const bool me = i == q;
    const double fi = me ? 0.0 : f * inv;  // row i minus fi times the pivot row
    const double sc = me ? inv : 1.0;
    const double vl = me ? inv : -fi;       // the new pivot-column entry
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const double x = (v[j] - fi * r[j]) * sc;
      v[j] = j == l ? vl : x;
    }
    pos = me ? k : (pos == k ? pq : pos);
  }
  if (i == 0 && sing) atomicMax(singular, sy + 1);
  int32_t* tot = tot_all + base;
  int tv = 0;
  if (live) {
    double* S = Sbuf + (int64_t)NB * base + (int64_t)pos * NB;
#pragma unroll
    for (int j = 0; j < NB; ++j) S[j] = v[j];
    src_all[base + pos] = i;
    tv = k0 == 0 ? i : tot[i];
  }
  __syncthreads();  // every read of the old cumulative map precedes the writes
  if (live) tot[pos] = tv;
}

// out = transform of in for the column block [k0, k0 + kb) (see above);
// systems whose order is <= k0 are copied unchanged
__global__ void __launch_bounds__(GJ_UT)
k_gj_update(const double* Ain, double* Aout, const int64_t* E_off, const int32_t* sys_coff, int k0,
            int nb, const double* Sbuf, const int32_t* src_all) {
  __shared__ double Ssh[GJ_TILE][33];
  __shared__ double Rsh[32][GJ_TILE];
  __shared__ int srow[GJ_TILE];
  const int sy = blockIdx.z;
  const int n = sys_coff[sy + 1] - sys_coff[sy];
  const int i0 = blockIdx.y * GJ_TILE, j0 = blockIdx.x * GJ_TILE;
  if (i0 >= n || j0 >= n) return;
  const double* A = Ain + E_off[sy];
  double* B = Aout + E_off[sy];
  const int t = threadIdx.x, tr = t / 16, tc = t % 16;
  if (k0 >= n) {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const int i = i0 + tr + 16 * a, j = j0 + tc + 16 * b;
        if (i < n && j < n) B[(int64_t)i * n + j] = A[(int64_t)i * n + j];
      }
    return;
  }
  const int kb = min(nb, n - k0);
  const double* S = Sbuf + (int64_t)nb * sys_coff[sy];
  const int32_t* src = src_all + sys_coff[sy];
  for (int e = t; e < GJ_TILE * 32; e += GJ_UT) {
    const int r = e / 32, l = e % 32;
    const int i = i0 + r;
    double v = 0.0;
    if (i < n && l < kb) v = S[(int64_t)i * nb + l] - (i == k0 + l ? 1.0 : 0.0);
    Ssh[r][l] = v;
    const int rl = e / GJ_TILE, cc = e % GJ_TILE;
    const int j = j0 + cc;
    Rsh[rl][cc] = (rl < kb && j < n) ? A[(int64_t)src[k0 + rl] * n + j] : 0.0;
  }
  if (t < GJ_TILE) srow[t] = (i0 + t < n) ? src[i0 + t] : 0;
  __syncthreads();
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int r = tr + 16 * a, cc = tc + 16 * b;
      const int i = i0 + r, j = j0 + cc;
      if (i >= n || j >= n) continue;
      double v;
      if (j >= k0 && j < k0 + kb) {
        v = S[(int64_t)i * nb + (j - k0)];
      } else {
        v = A[(int64_t)srow[r] * n + j];
        for (int l = 0; l < kb; ++l) v += Ssh[r][l] * Rsh[l][cc];
      }
      B[(int64_t)i * n + j] = v;
    }
}

// Einv(:, j) = W(:, c_j) with c the inverse of the cumulative row map of
// the interchanges (c(tot(x)) = x)
__global__ void k_gj_unpermute(const double* Win, double* Out, const int64_t* E_off,
                               const int32_t* sys_coff, const int32_t* tot_all, int rows_per_block) {
  extern __shared__ int cmap[];
  const int sy = blockIdx.y;
  const int n = sys_coff[sy + 1] - sys_coff[sy];
  const int r0 = blockIdx.x * rows_per_block;
  if (r0 >= n) return;
  const int32_t* tot = tot_all + sys_coff[sy];
  for (int x = threadIdx.x; x < n; x += blockDim.x) cmap[tot[x]] = x;
  __syncthreads();
  const double* W = Win + E_off[sy];
  double* X = Out + E_off[sy];
  const int r1 = min(n, r0 + rows_per_block);
  for (int64_t e = threadIdx.x; e < (int64_t)(r1 - r0) * n; e += blockDim.x) {
    const int i = r0 + (int)(e / n), j = (int)(e % n);
    X[(int64_t)i * n + j] = W[(int64_t)i * n + cmap[j]];
  }
}

// Inverts the nsys row-major matrices of A in place of a ping-pong pair: system
// sy has order sys_coff[sy + 1] - sys_coff[sy] (device arrays) and starts at
// E_off[sy]; B has the size of A.  Returns A or B, whichever holds the
// inverses (the other is free).  A singular system sets *flag to sy + 1 (the
// largest such index); nrow = sys_coff[nsys] (host).
double* gj_invert_batched(Ctx& c, hipStream_t st, int nsys, int64_t maxs, int64_t nrow,
                                 double* A, double* B, const int64_t* E_off,
                                 const int32_t* sys_coff, int32_t* flag) {
  if (maxs <= 0) return A;
  // register-resident panels (width 32, one row per thread) up to order GJ_T,
  // else LDS panels, else (orders above about 7400) panels in HBM
  const bool reg = maxs <= GJ_T;
  const int nbl = reg ? 32 : gj_panel_width(maxs);
  const bool hbm = nbl == 0;
  const int nb = hbm ? 32 : nbl;
  const int64_t n0t = std::max<int64_t>(nrow, 1);
  int32_t* tot = c.mem.alloc<int32_t>(n0t);
  int32_t* src = c.mem.alloc<int32_t>(n0t);
  double* S = c.mem.alloc<double>(n0t * nb);
  double* fcol = hbm ? c.mem.alloc<double>(n0t) : nullptr;
  double* bufs[2] = {A, B};
  const size_t plds = hbm ? 0 : (size_t)maxs * (nb * 8 + 8 + 4);
  const unsigned tiles = (unsigned)((maxs + GJ_TILE - 1) / GJ_TILE);
  const unsigned rows = (unsigned)((maxs + 63) / 64 * 64);  // one thread per row
  int cur = 0;
  for (int64_t k0 = 0; k0 < maxs; k0 += nb) {
    if (hbm)
      ADS_LAUNCH(k_gj_panel<true>, dim3(nsys), dim3(GJ_T), 0, st, bufs[cur], E_off, sys_coff,
                 (int)k0, nb, S, src, tot, fcol, flag);
    else if (!reg)
      ADS_LAUNCH(k_gj_panel<false>, dim3(nsys), dim3(GJ_T), plds, st, bufs[cur], E_off, sys_coff,
                 (int)k0, nb, S, src, tot, fcol, flag);
    else
      ADS_LAUNCH(k_gj_panel_row, dim3(nsys), dim3(rows), 0, st, bufs[cur], E_off, sys_coff,
                 (int)k0, S, src, tot, flag);
    ADS_LAUNCH(k_gj_update, dim3(tiles, tiles, nsys), dim3(GJ_UT), 0, st, bufs[cur], bufs[1 - cur],
               E_off, sys_coff, (int)k0, nb, S, src);
    cur = 1 - cur;
  }
  const int rpb = 16;
  ADS_LAUNCH(k_gj_unpermute, dim3((unsigned)((maxs + rpb - 1) / rpb), nsys), dim3(256),
             (size_t)maxs * 4, st, bufs[cur], bufs[1 - cur], E_off, sys_coff, tot, rpb);
  c.mem.release(S);
  if (fcol) c.mem.release(fcol);
  c.mem.release(src);
  c.mem.release(tot);
  return bufs[1 - cur];
}

}  // namespace
}  // namespace ads
