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
//   panel        : the unblocked Gauss-Jordan steps on the n x nb column
//                  panel (one workgroup per system with one row per thread up
//                  to GJ_T rows, two to four rows per thread up to 4 GJ_T,
//                  else one launch per pivot over chunks of rows), recording
//                  the pivots; the result S is the panel
//                  columns of the accumulated transform, src the composed row
//                  source map of the block's interchanges;
//   update kernel: every other column receives the same transform as a rank-nb
//                  product, out(i, j) = in(src i, j) + sum_l (S(i,l) - [i = k0+l]) in(src(k0+l), j),
//                  written to the other buffer of a ping-pong pair (no in-place
//                  races between tiles); the panel columns receive S.
// Every reduction has a fixed order, so the result is deterministic.
// ---------------------------------------------------------------------------
static constexpr int GJ_T = 1024;
static constexpr int GJ_UT = 256;
static constexpr int GJ_TILE = 32;
static constexpr int GJ_CH = 256;  // rows per workgroup of the chunked panel

// (value, index) max with ties to the smaller index; NaN never wins
__device__ __forceinline__ void gj_better(double& bv, int& bi, double v, int i) {
  if (v > bv || (v == bv && i < bi)) {
    bv = v;
    bi = i;
  }
}

// Panels of systems above GJ_T rows: one launch per pivot step over chunks
// of GJ_CH rows (grid: chunks x systems).  The panel alternates between two
// buffers (step l reads P[l & 1] and writes P[(l + 1) & 1], rows in the
// logical order of the block: the pivot row and row k trade places), so no
// workgroup reads a row that another one writes.  Every workgroup reduces
// the previous step's per-chunk (|entry|, row) maxima in the same order, and
// so takes the same pivot, then publishes the maxima of its own rows for the
// next column.  Steps past a system's last column copy its panel, so that
// every system's panel ends in the same buffer.

// block-wide (value, index) maximum, ties to the smaller index; the result
// is valid in thread 0
__device__ __forceinline__ void gj_block_best(double& bv, int& bi, double* sv, int* si) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(bv, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    gj_better(bv, bi, ov, oi);
  }
  const int t = threadIdx.x;
  if ((t & 63) == 0) {
    sv[t >> 6] = bv;
    si[t >> 6] = bi;
  }
  __syncthreads();
  if (t == 0)
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) gj_better(bv, bi, sv[w], si[w]);
}

// panel columns [k0, k0 + nb) of the input into P0; maxima of column k0
__global__ void __launch_bounds__(GJ_CH)
k_gjc_init(const double* Ain, const int64_t* E_off, const int32_t* sys_coff, int k0, int nb,
           double* P0, double* part_v, int* part_i, int nchm, int nsys) {
  __shared__ double sv[GJ_CH / 64];
  __shared__ int si[GJ_CH / 64];
  const int sy = blockIdx.y, ch = blockIdx.x;
  const int base = sys_coff[sy], n = sys_coff[sy + 1] - base;
  if (k0 >= n || ch * GJ_CH >= n) return;
  const int kb = min(nb, n - k0);
  const int i = ch * GJ_CH + threadIdx.x;
  double bv = -1.0;
  int bi = n;
  if (i < n) {
    const double* a = Ain + E_off[sy] + (int64_t)i * n + k0;
    double* p = P0 + ((int64_t)base + i) * nb;
    for (int l = 0; l < nb; ++l) p[l] = l < kb ? a[l] : 0.0;
    if (i >= k0) gj_better(bv, bi, fabs(a[0]), i);
  }
  gj_block_best(bv, bi, sv, si);
  if (threadIdx.x == 0) {
    part_v[(int64_t)sy * nchm + ch] = bv;
    part_i[(int64_t)sy * nchm + ch] = bi;
  }
}

// pivot step l (column k0 + l) of every system's panel
__global__ void __launch_bounds__(GJ_CH)
k_gjc_step(const int32_t* sys_coff, int k0, int nb, int l, double* P0, double* P1,
           double* part_v, int* part_i, int nchm, int nsys, int32_t* swp, int32_t* singular) {
  constexpr int NB = 32;
  __shared__ double rowk[NB], rowkold[NB];
  __shared__ double sv[GJ_CH / 64];
  __shared__ int si[GJ_CH / 64];
  __shared__ int sp;
  const int sy = blockIdx.y, ch = blockIdx.x, t = threadIdx.x;
  const int base = sys_coff[sy], n = sys_coff[sy + 1] - base;
  if (k0 >= n || ch * GJ_CH >= n) return;
  const int kb = min(nb, n - k0);
  const int nch = (n + GJ_CH - 1) / GJ_CH;
  const double* Pin = (l & 1) ? P1 : P0;
  double* Pout = (l & 1) ? P0 : P1;
  const int i = ch * GJ_CH + t;
  if (l >= kb) {  // past this system's last column: carry the panel over
    if (i < n)
      for (int j = 0; j < nb; ++j) Pout[((int64_t)base + i) * nb + j] = Pin[((int64_t)base + i) * nb + j];
    return;
  }
  const int k = k0 + l;
  const int64_t pin = (int64_t)(l & 1) * nsys * nchm, pout = (int64_t)((l + 1) & 1) * nsys * nchm;
  if (t < 64) {  // the pivot: maximum of the previous step's chunk maxima
    double bv = -1.0;
    int bi = n;
    for (int c = t; c < nch; c += 64)
      gj_better(bv, bi, part_v[pin + (int64_t)sy * nchm + c], part_i[pin + (int64_t)sy * nchm + c]);
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      gj_better(bv, bi, ov, oi);
    }
    if (t == 0) {
      int p = bi;
      if (!(bv > 0.0) || p >= n) {
        if (ch == 0) atomicMax(singular, sy + 1);
        p = k;
      }
      sp = p;
      if (ch == 0) swp[sy * NB + l] = p;
    }
  }
  __syncthreads();
  const int p = sp;
  if (t < nb) {
    rowk[t] = Pin[((int64_t)base + p) * nb + t];
    rowkold[t] = Pin[((int64_t)base + k) * nb + t];
  }
  __syncthreads();
  double bv = -1.0;
  int bi = n;
  if (i < n) {
    const double* src = Pin + ((int64_t)base + i) * nb;
    double v[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const double x = i == k ? rowk[j] : (i == p ? rowkold[j] : src[min(j, nb - 1)]);
      v[j] = j < nb ? x : 0.0;
    }
    double f = v[0];  // this row's entry in the pivot column
#pragma unroll
    for (int j = 1; j < NB; ++j) f = j == l ? v[j] : f;
    const double piv = rowk[l];
    const double d = piv != 0.0 ? 1.0 / piv : 1.0;
    double* dst = Pout + ((int64_t)base + i) * nb;
    double nxt = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double w;
      if (i == k)
        w = j == l ? d : v[j] * d;
      else
        w = j == l ? -f * d : v[j] - f * (rowk[j] * d);
      if (j < nb) dst[j] = w;
      nxt = j == l + 1 ? w : nxt;
    }
    if (i > k && l + 1 < kb) gj_better(bv, bi, fabs(nxt), i);
  }
  if (l + 1 < kb) {
    gj_block_best(bv, bi, sv, si);
    if (t == 0) {
      part_v[pout + (int64_t)sy * nchm + ch] = bv;
      part_i[pout + (int64_t)sy * nchm + ch] = bi;
    }
  }
}

// the block's composed row sources and the cumulative row map
// tot(x) <- tot(src(x)) (tmp: n0 ints of scratch)
__global__ void __launch_bounds__(GJ_T)
k_gjc_fini(const int32_t* sys_coff, int k0, int nb, const int32_t* swp, int32_t* src_all,
           int32_t* tot_all, int32_t* tmp_all) {
  const int sy = blockIdx.x, t = threadIdx.x, T = blockDim.x;
  const int base = sys_coff[sy], n = sys_coff[sy + 1] - base;
  if (k0 >= n) return;
  const int kb = min(nb, n - k0);
  int32_t* src = src_all + base;
  int32_t* tot = tot_all + base;
  int32_t* tmp = tmp_all + base;
  for (int x = t; x < n; x += T) src[x] = x;
  __syncthreads();
  if (t == 0)
    for (int l = 0; l < kb; ++l) {
      const int k = k0 + l, p = swp[sy * 32 + l];
      const int a = src[k];
      src[k] = src[p];
      src[p] = a;
    }
  __syncthreads();
  for (int x = t; x < n; x += T) tmp[x] = k0 == 0 ? src[x] : tot[src[x]];
  __syncthreads();
  for (int x = t; x < n; x += T) tot[x] = tmp[x];
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
template <int NB>
__global__ void __launch_bounds__(GJ_T)
k_gj_panel_row(const double* Ain, const int64_t* E_off, const int32_t* sys_coff, int k0,
               double* Sbuf, int32_t* src_all, int32_t* tot_all, int32_t* singular) {
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

// Register-resident panel for systems of order <= R * GJ_T: as
// k_gj_panel_row, with R consecutive rows per thread (thread t owns rows
// t R .. t R + R - 1, so lane order is row order and a tie still goes to the
// smallest row).  The thread's best candidate is its first row of largest
// magnitude; the published row is picked from the thread's rows by selects
// (no dynamic register indexing).
template <int NB, int R>
__global__ void __launch_bounds__(GJ_T)
k_gj_panel_rows(const double* Ain, const int64_t* E_off, const int32_t* sys_coff, int k0,
                double* Sbuf, int32_t* src_all, int32_t* tot_all, int32_t* singular) {
  __shared__ double slot_r[2][GJ_T / 64][NB + 1];  // row values, then the key
  __shared__ int slot_q[2][GJ_T / 64][2];          // physical row, logical position
  const int sy = blockIdx.x;
  const int base = sys_coff[sy];
  const int n = sys_coff[sy + 1] - base;
  if (k0 >= n) return;
  const int kb = min(NB, n - k0);
  const int t = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
  const int nw = (int)(blockDim.x + 63) >> 6;
  double v[R][NB];
  int pos[R];
  bool live[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = t * R + q;
    live[q] = i < n;
    pos[q] = i;
    const double* A = Ain + E_off[sy] + (int64_t)(live[q] ? i : 0) * n + k0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const double a = A[min(j, kb - 1)];  // in bounds for every lane
      v[q][j] = (live[q] && j < kb) ? a : 0.0;
    }
  }
  bool sing = false;
  for (int l = 0; l < kb; ++l) {
    const int k = k0 + l, b = l & 1;
    double f[R];  // each row's entry in the pivot column
    double cb = -1.0;
    int qb = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double x = v[q][0];
#pragma unroll
      for (int j = 1; j < NB; ++j) x = j == l ? v[q][j] : x;
      f[q] = x;
      double cand = (live[q] && pos[q] >= k) ? fabs(x) : -1.0;
      if (!(cand >= 0.0)) cand = -1.0;  // NaN never wins
      if (cand > cb) {
        cb = cand;
        qb = q;
      }
    }
    const double m = gj_wave_max(cb);
    const bool top = cb == m;
    const unsigned long long hit = __ballot(top);
    const unsigned below = __builtin_amdgcn_mbcnt_hi((unsigned)(hit >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((unsigned)hit, 0u));
    if (top && below == 0) {
      int pb = pos[0];
#pragma unroll
      for (int q = 1; q < R; ++q) pb = q == qb ? pos[q] : pb;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        double x = v[0][j];
#pragma unroll
        for (int q = 1; q < R; ++q) x = q == qb ? v[q][j] : x;
        slot_r[b][wv][j] = x;
      }
      slot_r[b][wv][NB] = m;
      slot_q[b][wv][0] = t * R + qb;
      slot_q[b][wv][1] = pb;
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
    const int prow = slot_q[b][w][0], pq = slot_q[b][w][1];
    sing |= !(best > 0.0);
    const double piv = r[l];
    const double inv = piv != 0.0 ? 1.0 / piv : 1.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const bool me = t * R + q == prow;
      const double fi = me ? 0.0 : f[q] * inv;  // row minus fi times the pivot row
      const double sc = me ? inv : 1.0;
      const double vl = me ? inv : -fi;         // the new pivot-column entry
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const double x = (v[q][j] - fi * r[j]) * sc;
        v[q][j] = j == l ? vl : x;
      }
      pos[q] = me ? k : (pos[q] == k ? pq : pos[q]);
    }
  }
  if (t == 0 && sing) atomicMax(singular, sy + 1);
  int32_t* tot = tot_all + base;
  int tv[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    tv[q] = 0;
    if (live[q]) {
      const int i = t * R + q;
      double* S = Sbuf + (int64_t)NB * base + (int64_t)pos[q] * NB;
#pragma unroll
      for (int j = 0; j < NB; ++j) S[j] = v[q][j];
      src_all[base + pos[q]] = i;
      tv[q] = k0 == 0 ? i : tot[i];
    }
  }
  __syncthreads();  // every read of the old cumulative map precedes the writes
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (live[q]) tot[pos[q]] = tv[q];
}

// out = transform of in for the column block [k0, k0 + kb) (see above), on
// TL x TL output tiles; each thread accumulates (TL/16)^2 outputs in
// registers, so every LDS read feeds TL/16 products.  Systems whose order is
// <= k0 are copied unchanged.  The sum over l runs in the same order for
// every tile shape.
template <int TL>
__global__ void __launch_bounds__(GJ_UT)
k_gj_update(const double* Ain, double* Aout, const int64_t* E_off, const int32_t* sys_coff, int k0,
            int nb, const double* Sbuf, const int32_t* src_all) {
  constexpr int R = TL / 16;
  __shared__ double Ssh[TL][33];
  __shared__ double Rsh[32][TL];
  __shared__ int srow[TL];
  const int sy = blockIdx.z;
  const int n = sys_coff[sy + 1] - sys_coff[sy];
  const int i0 = blockIdx.y * TL, j0 = blockIdx.x * TL;
  if (i0 >= n || j0 >= n) return;
  const double* A = Ain + E_off[sy];
  double* B = Aout + E_off[sy];
  const int t = threadIdx.x, tr = t / 16, tc = t % 16;
  if (k0 >= n) {
    for (int a = 0; a < R; ++a)
      for (int b = 0; b < R; ++b) {
        const int i = i0 + tr + 16 * a, j = j0 + tc + 16 * b;
        if (i < n && j < n) B[(int64_t)i * n + j] = A[(int64_t)i * n + j];
      }
    return;
  }
  const int kb = min(nb, n - k0);
  const double* S = Sbuf + (int64_t)nb * sys_coff[sy];
  const int32_t* src = src_all + sys_coff[sy];
  for (int e = t; e < TL * 32; e += GJ_UT) {
    const int r = e / 32, l = e % 32;
    const int i = i0 + r;
    double v = 0.0;
    if (i < n && l < kb) v = S[(int64_t)i * nb + l] - (i == k0 + l ? 1.0 : 0.0);
    Ssh[r][l] = v;
    const int rl = e / TL, cc = e % TL;
    const int j = j0 + cc;
    Rsh[rl][cc] = (rl < kb && j < n) ? A[(int64_t)src[k0 + rl] * n + j] : 0.0;
  }
  if (t < TL) srow[t] = (i0 + t < n) ? src[i0 + t] : 0;
  __syncthreads();
  double acc[R][R];
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int b = 0; b < R; ++b) {
      const int i = i0 + tr + 16 * a, j = j0 + tc + 16 * b;
      acc[a][b] = (i < n && j < n) ? A[(int64_t)srow[tr + 16 * a] * n + j] : 0.0;
    }
  for (int l = 0; l < kb; ++l) {
    double sa[R], rb[R];
#pragma unroll
    for (int a = 0; a < R; ++a) sa[a] = Ssh[tr + 16 * a][l];
#pragma unroll
    for (int b = 0; b < R; ++b) rb[b] = Rsh[l][tc + 16 * b];
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < R; ++b) acc[a][b] += sa[a] * rb[b];
  }
#pragma unroll
  for (int a = 0; a < R; ++a)
#pragma unroll
    for (int b = 0; b < R; ++b) {
      const int i = i0 + tr + 16 * a, j = j0 + tc + 16 * b;
      if (i >= n || j >= n) continue;
      B[(int64_t)i * n + j] = (j >= k0 && j < k0 + kb) ? S[(int64_t)i * nb + (j - k0)] : acc[a][b];
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
// largest such index); nrow = sys_coff[nsys] and total = the sum of the
// orders squared (host).
double* gj_invert_batched(Ctx& c, hipStream_t st, int nsys, int64_t maxs, int64_t nrow,
                          int64_t total, double* A, double* B, const int64_t* E_off,
                          const int32_t* sys_coff, int32_t* flag) {
  const bool small_batch = total * 8 <= ((int64_t)32 << 20);  // all matrices within 32 MB
  if (maxs <= 0) return A;
  // register-resident panels (one row per thread) up to order GJ_T, else
  // panels stepped over chunks of rows.  Width 32; register panels of
  // batches small enough for the caches take width 8 (a quarter of the
  // instructions per dependent pivot step, four times the update passes).
  const bool reg = maxs <= GJ_T;
  // orders up to 4 GJ_T: register panels of width 8 with 2-4 rows per thread
  const int R = reg ? 1 : (int)((maxs + GJ_T - 1) / GJ_T);
  const bool multi = !reg && R <= 4;
  const int nb = ((reg && small_batch) || multi) ? 8 : 32;
  const int64_t n0t = std::max<int64_t>(nrow, 1);
  int32_t* tot = c.mem.alloc<int32_t>(n0t);
  int32_t* src = c.mem.alloc<int32_t>(n0t);
  double* S = c.mem.alloc<double>(n0t * nb);
  double* S1 = nullptr;
  double* part_v = nullptr;
  int32_t* part_i = nullptr;
  int32_t* swp = nullptr;
  int32_t* tmp = nullptr;
  const int nchm = (int)((maxs + GJ_CH - 1) / GJ_CH);
  if (!reg && !multi) {
    S1 = c.mem.alloc<double>(n0t * nb);
    part_v = c.mem.alloc<double>((size_t)2 * nsys * nchm);
    part_i = c.mem.alloc<int32_t>((size_t)2 * nsys * nchm);
    swp = c.mem.alloc<int32_t>((size_t)nsys * nb);
    tmp = c.mem.alloc<int32_t>(n0t);
  }
  double* bufs[2] = {A, B};
  // 64 x 64 output tiles when they still give the GPU a few thousand
  // workgroups, else 32 x 32
  const unsigned t64 = (unsigned)((maxs + 63) / 64);
  const bool wide = (int64_t)t64 * t64 * nsys >= 2048;
  const unsigned tiles = wide ? t64 : (unsigned)((maxs + GJ_TILE - 1) / GJ_TILE);
  const unsigned rows = (unsigned)((maxs + 63) / 64 * 64);  // one thread per row
  int cur = 0;
  for (int64_t k0 = 0; k0 < maxs; k0 += nb) {
    double* Sk = S;
    if (multi) {
      const unsigned mrows = (unsigned)(((maxs + R - 1) / R + 63) / 64 * 64);
      if (R == 2)
        ADS_LAUNCH((k_gj_panel_rows<8, 2>), dim3(nsys), dim3(mrows), 0, st, bufs[cur], E_off,
                   sys_coff, (int)k0, S, src, tot, flag);
      else if (R == 3)
        ADS_LAUNCH((k_gj_panel_rows<8, 3>), dim3(nsys), dim3(mrows), 0, st, bufs[cur], E_off,
                   sys_coff, (int)k0, S, src, tot, flag);
      else
        ADS_LAUNCH((k_gj_panel_rows<8, 4>), dim3(nsys), dim3(mrows), 0, st, bufs[cur], E_off,
                   sys_coff, (int)k0, S, src, tot, flag);
    } else if (reg) {
      if (nb == 8)
        ADS_LAUNCH(k_gj_panel_row<8>, dim3(nsys), dim3(rows), 0, st, bufs[cur], E_off, sys_coff,
                   (int)k0, S, src, tot, flag);
      else
        ADS_LAUNCH(k_gj_panel_row<32>, dim3(nsys), dim3(rows), 0, st, bufs[cur], E_off, sys_coff,
                   (int)k0, S, src, tot, flag);
    } else {
      const dim3 g((unsigned)nchm, (unsigned)nsys);
      ADS_LAUNCH(k_gjc_init, g, dim3(GJ_CH), 0, st, bufs[cur], E_off, sys_coff, (int)k0, nb, S,
                 part_v, part_i, nchm, nsys);
      const int L = (int)std::min<int64_t>(nb, maxs - k0);
      for (int l = 0; l < L; ++l)
        ADS_LAUNCH(k_gjc_step, g, dim3(GJ_CH), 0, st, sys_coff, (int)k0, nb, l, S, S1, part_v,
                   part_i, nchm, nsys, swp, flag);
      Sk = (L & 1) ? S1 : S;
      ADS_LAUNCH(k_gjc_fini, dim3(nsys), dim3(GJ_T), 0, st, sys_coff, (int)k0, nb, swp, src, tot,
                 tmp);
    }
    if (wide)
      ADS_LAUNCH(k_gj_update<64>, dim3(tiles, tiles, nsys), dim3(GJ_UT), 0, st, bufs[cur],
                 bufs[1 - cur], E_off, sys_coff, (int)k0, nb, Sk, src);
    else
      ADS_LAUNCH(k_gj_update<GJ_TILE>, dim3(tiles, tiles, nsys), dim3(GJ_UT), 0, st, bufs[cur],
                 bufs[1 - cur], E_off, sys_coff, (int)k0, nb, Sk, src);
    cur = 1 - cur;
  }
  const int rpb = 16;
  ADS_LAUNCH(k_gj_unpermute, dim3((unsigned)((maxs + rpb - 1) / rpb), nsys), dim3(256),
             (size_t)maxs * 4, st, bufs[cur], bufs[1 - cur], E_off, sys_coff, tot, rpb);
  for (void* q : {(void*)S, (void*)S1, (void*)part_v, (void*)part_i, (void*)swp, (void*)tmp})
    if (q) c.mem.release(q);
  c.mem.release(src);
  c.mem.release(tot);
  return bufs[1 - cur];
}

}  // namespace
}  // namespace ads
