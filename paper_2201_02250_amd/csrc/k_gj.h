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
//                  to GJ_T rows, two to four rows per thread up to 4 GJ_T),
//                  or, for larger systems, the panel's pivot rows chosen by
//                  tournament pivoting and its transform formed in parallel
//                  (see k_tslu); the result S is the panel
//                  columns of the accumulated transform, src the composed row
//                  source map of the block's interchanges;
//   update kernel: every other column receives the same transform as a rank-nb
//                  product, out(i, j) = in(src i, j) + sum_l (S(i,l) - [i = k0+l]) in(src(k0+l), j),
//                  written to the other buffer of a ping-pong pair (no in-place
//                  races between tiles); the panel columns receive S.  Large
//                  batches run it on the matrix cores (k_gj_update_mfma).
// Every reduction has a fixed order, so the result is deterministic.
// ---------------------------------------------------------------------------
static constexpr int GJ_T = 1024;
static constexpr int GJ_UT = 256;
static constexpr int GJ_TILE = 32;

// x if keep, else 0, as arithmetic on a value that was loaded from an
// always-valid (clamped) address: the load stays unconditional, so the
// compiler issues all the loads of a tile back to back instead of one
// branch (and one wait) per masked load
__device__ __forceinline__ double gj_keep(double x, bool keep) { return x * (keep ? 1.0 : 0.0); }

// a per-lane (vector register) copy of a workgroup-uniform loop index: the
// column selects "j == l" of the unrolled row updates then compile to lane
// selects instead of one uniform branch per column, and the pivot row's LDS
// reads are no longer split by those branches (one wait each)
__device__ __forceinline__ int gj_lane_copy(int x) {
  int y;
  asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "s"(x));
  return y;
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
      const int k = k0 + l, p = swp[sy * nb + l];
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

// Register-resident panel for systems of order <= T threads (panel width NB:
// 8 or 32 with 1024 threads, 64 with 512 threads so that the 64 entries of a
// row stay in registers): thread i owns row i of the n x NB column panel (rows in the logical order
// that the previous panels left) and tracks the logical position of that
// row; rows never move.  One barrier per pivot step: every wave publishes its
// best pivot candidate (largest |entry| in the pivot column among the rows
// not yet used, ties to the smaller row) together with that row's values in
// a double-buffered LDS slot, and every thread then takes the first slot of
// largest magnitude.  The result S is written in logical row order.
template <int NB, int T = GJ_T>
__global__ void __launch_bounds__(T)
k_gj_panel_row(const double* Ain, const int64_t* E_off, const int32_t* sys_coff, int k0,
               double* Sbuf, int32_t* src_all, int32_t* tot_all, int32_t* singular) {
  __shared__ double slot_r[2][T / 64][NB + 1];  // row values, then the key
  __shared__ int slot_q[2][T / 64][2];          // physical row, logical position
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
  for (int j = 0; j < NB; ++j) v[j] = gj_keep(A[min(j, kb - 1)], live && j < kb);
  int pos = i;
  bool sing = false;
  for (int l = 0; l < kb; ++l) {
    const int k = k0 + l, b = l & 1;
    const int lv = gj_lane_copy(l);
    double f = v[0];  // this row's entry in the pivot column
#pragma unroll
    for (int j = 1; j < NB; ++j) f = j == lv ? v[j] : f;
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
      v[j] = j == lv ? vl : x;
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
    for (int j = 0; j < NB; ++j) v[q][j] = gj_keep(A[min(j, kb - 1)], live[q] && j < kb);
  }
  bool sing = false;
  for (int l = 0; l < kb; ++l) {
    const int k = k0 + l, b = l & 1;
    const int lv = gj_lane_copy(l);
    double f[R];  // each row's entry in the pivot column
    double cb = -1.0;
    int qb = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double x = v[q][0];
#pragma unroll
      for (int j = 1; j < NB; ++j) x = j == lv ? v[q][j] : x;
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
        v[q][j] = j == lv ? vl : x;
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

// ---------------------------------------------------------------------------
// Matrix-core form of the update (large batches and large systems): the
// same transform as k_gj_update on 64 x 64 output tiles, computed with
// v_mfma_f64_16x16x4f64.  The workgroup stages S' = S - [i = k0 + l] (its 64
// rows) and the source rows R = in(src(k0 + l), :) of its 64 columns in LDS,
// GM_K panel columns at a time; wave w owns the 32 x 32 quarter (w / 2, w % 2)
// as 2 x 2 blocks of 16 x 16, whose accumulators start from in(src(i), j).
// Operand layouts of the instruction (16 x 4 by 4 x 16): lane l holds
// A(l % 16, l / 16) and B(l / 16, l % 16); accumulator register r of lane l
// holds D(l / 16 + 4 r, l % 16).  The sum over l runs in steps of four in a
// fixed order, so the result is deterministic.
// ---------------------------------------------------------------------------
typedef double gj_d4 __attribute__((ext_vector_type(4)));
static constexpr int GM_T = 256;
static constexpr int GM_K = 32;     // panel columns staged per pass
static constexpr int GM_KMAX = 128; // widest panel
static constexpr int GM_SLD = GM_K + 1;
static constexpr int GM_RLD = 64 + 4;

static constexpr int GM_GROUP = 16;  // tile rows per column-major sweep
static constexpr int GM_O32_MAX = 23170;  // largest order whose n^2 doubles stay below 2^32 bytes

// base[idx], with a 32-bit unsigned byte offset when O32 (0 <= idx and 8 idx
// < 2^32)
template <bool O32>
__device__ __forceinline__ double gj_ld(const double* base, int64_t idx) {
  if constexpr (O32)
    return *(const double*)((const char*)base + (size_t)(8u * (unsigned)idx));
  else
    return base[idx];
}

// Tile of workgroup h in a one-dimensional grid of T x T tiles per system
// times nsys.  Workgroups are dispatched to the eight XCDs (each with its
// own L2) in turn, h to XCD h % 8; the logical order L gives every XCD one
// contiguous range, so a system's tiles (which share the panel S and the
// source rows R) are read through one L2.  Within a system, L runs over
// groups of GM_GROUP tile rows, column-major inside a group: the tiles that
// run together share their R block and the group's S rows stay cached.
// Both maps are bijections, so the order only affects the caches.
__device__ inline void gj_tile_of(int h, int T, int nsys, int& sy, int& ti, int& tj) {
  const int N = T * T * nsys;
  const int q = N >> 3, r = N & 7, x = h & 7, s = h >> 3;
  const int L = x * q + min(x, r) + s;
  const int TT = T * T;
  sy = L / TT;
  const int p = L - sy * TT;
  const int G = min(T, GM_GROUP);
  const int g = p / (G * T), ib = g * G, Gg = min(G, T - ib);
  const int qq = p - g * G * T;
  tj = qq / Gg;
  ti = ib + (qq - tj * Gg);
}

// The lower triangle of T x T tiles (ti >= tj) in the order of gj_tile_of:
// T (T + 1) / 2 tiles per system; within a group of GM_GROUP tile rows the
// full columns left of the group first, then the group's own triangle, both
// column-major.
__device__ inline void gj_tile_of_lower(int h, int T, int nsys, int& sy, int& ti, int& tj) {
  const int NT = T * (T + 1) / 2;
  const int N = NT * nsys;
  const int q = N >> 3, r = N & 7, x = h & 7, s = h >> 3;
  const int L = x * q + min(x, r) + s;
  sy = L / NT;
  int p = L - sy * NT;
  const int G = min(T, GM_GROUP);
  int ib = 0, Gg = min(G, T);
  for (;;) {  // the group holding p
    const int cnt = ib * Gg + Gg * (Gg + 1) / 2;
    if (p < cnt || ib + Gg >= T) break;
    p -= cnt;
    ib += G;
    Gg = min(G, T - ib);
  }
  if (p < ib * Gg) {
    tj = p / Gg;
    ti = ib + p % Gg;
    return;
  }
  p -= ib * Gg;
  int c = 0;
  while (p >= Gg - c) {
    p -= Gg - c;
    ++c;
  }
  tj = ib + c;
  ti = tj + p;
}

// The band of the next block (sym = 1): the lower tiles in tile rows or
// tile columns bl .. bl + bq - 1, bl + bq <= T, enumerated compactly (the
// rows first, then the columns below them), nb_tiles per system.
__host__ __device__ inline int gj_band_tiles(int T, int bl, int bq) {
  int cnt = 0;
  for (int r = 0; r < bq && bl + r < T; ++r) cnt += bl + r + 1;
  return cnt + bq * max(0, T - bl - bq);
}
__device__ inline void gj_band_tile_of(int h, int T, int bl, int bq, int& ti, int& tj) {
  for (int r = 0; r < bq && bl + r < T; ++r) {
    if (h < bl + r + 1) {
      ti = bl + r;
      tj = h;
      return;
    }
    h -= bl + r + 1;
  }
  const int below = max(1, T - bl - bq);
  tj = bl + h / below;
  ti = bl + bq + h % below;
}

// 64 x 64 tile (i0, j0) of the update, K = kb <= GM_KMAX columns of the
// panel taken in passes of GM_K through LDS: the loads of the next pass are
// issued before the matrix-core products of the current one, so they run
// while it computes.  Grid: T * T * nsys workgroups (gj_tile_of).  At most
// 128 registers per lane, so that four workgroups share a compute unit.
//
// sym = 1 (symmetric systems without interchanges): Gauss-Jordan keeps the
// symmetry of the matrix up to the sign of its cross blocks: with p the
// pivots done and u the others the matrix is [[X, Y], [-Y^T, Z]], X and Z
// symmetric.  The grid covers the lower triangle of tiles only (T (T + 1) / 2
// per system, gj_tile_of_lower), so the upper triangle of the output is
// stale except where the next block reads it: its pivot rows right of it
// (the update's source rows) and its columns above it (its panel and the
// second panel's update).  The tiles below the diagonal in the next block's
// tile rows or columns (mir_lo, mir_lo + nb / 64) are therefore also
// written transposed into their mirrors, negated when exactly one of the
// two index ranges is done after this block (tiles are 64-aligned and the
// blocks 128-aligned: one sign per tile); the transpose goes through LDS so
// that both stores are row-contiguous.  k_gj_mirror completes the upper
// triangle once at the end.  Half the products and about two thirds of the
// traffic of the full update.
//
// part (sym = 1): 0 every lower tile; 1 only the band of the next block (the
// tiles the next block's panel kernels read, which can then start while
// part 2 runs), 2 every lower tile outside that band.
//
// O32 (every system of order <= GM_O32_MAX): the loads address their
// system's matrix and panel with 32-bit byte offsets from a uniform base
// (one register per address instead of two), which fits the kernel in 128
// registers, four waves per SIMD.
template <bool O32>
__global__ void __launch_bounds__(GM_T, O32 ? 4 : 1)
k_gj_update_mfma(const double* Ain, double* Aout, const int64_t* E_off, const int32_t* sys_coff,
                 int k0, int nb, const double* Sbuf, const int32_t* src_all, int T, int nsys,
                 int sym, int mir_lo, int part) {
  __shared__ double lds[64 * GM_SLD + GM_K * GM_RLD];  // S' | R, then the transposed tile
  double* Ssh = lds;
  double* Rsh = lds + 64 * GM_SLD;
  __shared__ int srow[64];
  __shared__ int rsrc[GM_KMAX];
  int sy, ti, tj;
  const int nbt = nb / 64;
  if (sym && part == 1) {
    const int nbd = gj_band_tiles(T, mir_lo, nbt);
    sy = (int)blockIdx.x / nbd;
    gj_band_tile_of((int)blockIdx.x - sy * nbd, T, mir_lo, nbt, ti, tj);
  } else if (sym) {
    gj_tile_of_lower((int)blockIdx.x, T, nsys, sy, ti, tj);
  } else {
    gj_tile_of((int)blockIdx.x, T, nsys, sy, ti, tj);
  }
  const bool band = mir_lo >= 0 && ((unsigned)(ti - mir_lo) < (unsigned)nbt ||
                                    (unsigned)(tj - mir_lo) < (unsigned)nbt);
  if (part == 2 && band) return;
  const int n = sys_coff[sy + 1] - sys_coff[sy];
  const int i0 = ti * 64, j0 = tj * 64;
  if (i0 >= n || j0 >= n) return;
  const double* A = Ain + E_off[sy];
  double* B = Aout + E_off[sy];
  const int t = threadIdx.x;
  const bool mirror = sym && ti > tj && band;
  if (k0 >= n) {  // a finished system of the batch: its lower tiles as they are
    for (int e = t; e < 64 * 64; e += GM_T) {
      const int i = i0 + e / 64, j = j0 + e % 64;
      if (i < n && j < n) B[(int64_t)i * n + j] = A[(int64_t)i * n + j];
    }
    return;
  }
  const int kb = min(nb, n - k0);
  const double* S = Sbuf + (int64_t)nb * sys_coff[sy];
  if (src_all) {
    const int32_t* src = src_all + sys_coff[sy];
    if (t < GM_KMAX) rsrc[t] = t < kb ? src[k0 + t] : 0;
    if (t < 64) srow[t] = (i0 + t < n) ? src[i0 + t] : 0;
    __syncthreads();
  }
  // src_all = nullptr: the row maps are the identity (no loads, no barrier)
  const bool ident = src_all == nullptr;
  const int w = t >> 6, lane = t & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  // a pass: S' rows i0 .. i0 + 63 by panel columns kc .. kc + GM_K - 1
  // (element e = t + GM_T q: row e / GM_K, column e % GM_K) and the source
  // rows of those columns by the tile's 64 columns (row e / 64, column e % 64)
  // the values are loaded raw from clamped addresses and masked only when
  // they go to LDS, so no arithmetic on them sits between the prefetch of
  // the next pass and the products of the current one (which would make the
  // wave wait for the loads before its products)
  constexpr int NQ = 64 * GM_K / GM_T;
  double sv[NQ], rv[NQ];
  auto load_pass = [&](int kc) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = t + GM_T * q;
      const int sr = e / GM_K, sc = e % GM_K, rr = e / 64, rc = e % 64;
      const int i = i0 + sr, j = j0 + rc;
      sv[q] = gj_ld<O32>(S, (int64_t)min(i, n - 1) * nb + min(kc + sc, kb - 1));
      const int kr = min(kc + rr, kb - 1);
      rv[q] = gj_ld<O32>(A, (int64_t)(ident ? k0 + kr : rsrc[kr]) * n + min(j, n - 1));
    }
  };
  load_pass(0);
  gj_d4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ri = wr + bi * 16 + lk + 4 * r;
        const int i = i0 + ri, j = j0 + wc + bj * 16 + li;
        acc[bi][bj][r] =
            gj_keep(A[(int64_t)(ident ? min(i, n - 1) : srow[ri]) * n + min(j, n - 1)], i < n && j < n);
      }
  for (int kc = 0; kc < kb; kc += GM_K) {
    if (kc > 0) __syncthreads();  // the previous pass's LDS reads are done
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = t + GM_T * q;
      const int sr = e / GM_K, sc = e % GM_K, rr = e / 64, rc = e % 64;
      const bool incol = kc + sc < kb;
      Ssh[sr * GM_SLD + sc] = gj_keep(sv[q], i0 + sr < n && incol) -
                              ((incol && i0 + sr == k0 + kc + sc) ? 1.0 : 0.0);
      Rsh[rr * GM_RLD + rc] = gj_keep(rv[q], kc + rr < kb && j0 + rc < n);
    }
    __syncthreads();
    if (kc + GM_K < kb) load_pass(kc + GM_K);  // in flight during the products below
    __builtin_amdgcn_sched_barrier(0);
    const int kp = min(GM_K, (kb - kc + 3) & ~3);
    for (int kk = 0; kk < kp; kk += 4) {
      const double a0 = Ssh[(wr + li) * GM_SLD + kk + lk];
      const double a1 = Ssh[(wr + 16 + li) * GM_SLD + kk + lk];
      const double b0 = Rsh[(kk + lk) * GM_RLD + wc + li];
      const double b1 = Rsh[(kk + lk) * GM_RLD + wc + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  // the panel columns receive S: only the tiles that hold them (a uniform
  // test) load it, so the other tiles store without waiting on loads
  // (no load between the stores: every store would otherwise wait for the
  // one before it)
  const bool touch = j0 < k0 + kb && j0 + 64 > k0;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr + bi * 16 + lk + 4 * r, j = j0 + wc + bj * 16 + li;
        if (i < n && j < n && !(j >= k0 && j < k0 + kb)) B[(int64_t)i * n + j] = acc[bi][bj][r];
      }
  if (touch)
    for (int e = t; e < 64 * 64; e += GM_T) {
      const int i = i0 + e / 64, j = j0 + e % 64;
      if (i < n && j < n && j >= k0 && j < k0 + kb) B[(int64_t)i * n + j] = S[(int64_t)i * nb + (j - k0)];
    }
  if (!mirror) return;
  // the mirror tile: Tl(ii, jj) = the value just stored at (i0 + ii, j0 + jj),
  // written to (j0 + jj, i0 + ii), negated across the done / not-done border
  constexpr int TLD = 65;
  double* Tl = lds;
  __syncthreads();  // every wave is done with S' and R
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = wr + bi * 16 + lk + 4 * r, jj = wc + bj * 16 + li;
        Tl[ii * TLD + jj] = acc[bi][bj][r];
      }
  __syncthreads();
  if (touch)
    for (int e = t; e < 64 * 64; e += GM_T) {
      const int ii = e / 64, jj = e % 64, i = i0 + ii, j = j0 + jj;
      if (i < n && j < n && j >= k0 && j < k0 + kb) Tl[ii * TLD + jj] = S[(int64_t)i * nb + (j - k0)];
    }
  if (touch) __syncthreads();
  const int done = k0 + kb;
  const double sg = ((i0 < done) != (j0 < done)) ? -1.0 : 1.0;
  for (int e = t; e < 64 * 64; e += GM_T) {
    const int jj = e / 64, ii = e % 64, i = i0 + ii, j = j0 + jj;
    if (i < n && j < n) B[(int64_t)j * n + i] = sg * Tl[ii * TLD + jj];
  }
}

// The upper triangle of the symmetric result from its lower triangle (all
// pivots done: no signs), one tile below the diagonal per workgroup
// (gj_tile_of_lower order, diagonal tiles skipped), transposed through LDS.
__global__ void __launch_bounds__(GM_T)
k_gj_mirror(double* A_all, const int64_t* E_off, const int32_t* sys_coff, int T, int nsys) {
  __shared__ double Tl[64 * 65];
  int sy, ti, tj;
  gj_tile_of_lower((int)blockIdx.x, T, nsys, sy, ti, tj);
  const int n = sys_coff[sy + 1] - sys_coff[sy];
  const int i0 = ti * 64, j0 = tj * 64;
  if (ti == tj || i0 >= n || j0 >= n) return;
  double* A = A_all + E_off[sy];
  double v[64 * 64 / GM_T];  // every load in flight before the first store
#pragma unroll
  for (int q = 0; q < 64 * 64 / GM_T; ++q) {
    const int e = threadIdx.x + GM_T * q, ii = e / 64, jj = e % 64;
    v[q] = A[(int64_t)min(i0 + ii, n - 1) * n + min(j0 + jj, n - 1)];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < 64 * 64 / GM_T; ++q) {
    const int e = threadIdx.x + GM_T * q, ii = e / 64, jj = e % 64;
    Tl[ii * 65 + jj] = gj_keep(v[q], i0 + ii < n && j0 + jj < n);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += GM_T) {
    const int jj = e / 64, ii = e % 64;
    if (i0 + ii < n && j0 + jj < n) A[(int64_t)(j0 + jj) * n + i0 + ii] = Tl[ii * 65 + jj];
  }
}

// ---------------------------------------------------------------------------
// Panels of large systems (order above 4 GJ_T): the kb pivot rows of the
// panel are chosen by tournament pivoting (communication-avoiding LU of the
// tall n x kb panel: Grigori, Demmel and Xiang, 2011) instead of one launch
// per pivot, then the panel's transform is formed in parallel:
//   k_tslu          partial-pivoting LU on groups of up to TS_T candidate
//                   rows (one row per thread, the panel entries in registers)
//                   keeps each group's kb pivot rows; level 0 takes the rows
//                   not yet used as pivots in chunks of TS_T, later levels
//                   merge TS_G groups' winners, until one group is left;
//   k_gj_block_inv  the kb x kb block of the winners (in pick order) is
//                   inverted by Gauss-Jordan without further interchanges
//                   (the pick order is a partial-pivoting order for it, so
//                   every multiplier is at most 1 in magnitude), and
//   k_gj_pick_swaps turns the picks into the sequential interchanges of
//                   the block (row k0 + l with the l-th pick's current row);
//   k_gj_panel_form the panel columns of the block transform: the inverse on
//                   the pivot rows, -a_i P^{-1} on every other row.
// The update and the row maps are the ones of the other panel forms.
// ---------------------------------------------------------------------------
static constexpr int TS_T = 256;
static constexpr int TS_NB = 64;
static constexpr int TS_G = TS_T / TS_NB;  // groups merged per workgroup

// groups of system sy's candidates at tournament level lev (0: leaves)
__device__ __host__ inline int ts_groups(int n, int k0, int lev) {
  int g = (n - k0 + TS_T - 1) / TS_T;
  for (int v = 0; v < lev; ++v) g = (g + TS_G - 1) / TS_G;
  return g;
}

__global__ void __launch_bounds__(TS_T)
k_tslu(const double* Ain, const int64_t* E_off, const int32_t* sys_coff, int k0, int lev,
       const int32_t* cin, int32_t* cout, int gstride) {
  __shared__ double slot_r[2][TS_T / 64][TS_NB + 1];
  __shared__ int slot_q[2][TS_T / 64];
  const int sy = blockIdx.y, g = blockIdx.x, t = threadIdx.x;
  const int n = sys_coff[sy + 1] - sys_coff[sy];
  if (k0 >= n) return;
  const int ng = ts_groups(n, k0, lev);
  if (g >= ng) return;
  const int kb = min(TS_NB, n - k0);
  int32_t* out = cout + ((int64_t)sy * gstride + g) * TS_NB;
  int id = -1;
  if (lev == 0) {
    const int i = k0 + g * TS_T + t;
    id = i < n ? i : -1;
  } else {
    const int ngin = ts_groups(n, k0, lev - 1);
    if (ngin == 1) {  // already one group: carry it over
      if (t < TS_NB) out[t] = cin[(int64_t)sy * gstride * TS_NB + t];
      return;
    }
    const int gi = g * TS_G + t / TS_NB;
    if (gi < ngin) id = cin[((int64_t)sy * gstride + gi) * TS_NB + t % TS_NB];
  }
  const double* row = Ain + E_off[sy] + (int64_t)(id >= 0 ? id : 0) * n + k0;
  double v[TS_NB];
#pragma unroll
  for (int j = 0; j < TS_NB; ++j) v[j] = gj_keep(row[min(j, kb - 1)], id >= 0 && j < kb);
  bool alive = id >= 0;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  int picked = 0;
  bool done = false;  // uniform: no nonzero candidate left
#pragma unroll
  for (int l = 0; l < TS_NB; ++l) {
    if (l >= kb || done) continue;  // uniform; the loop stays fully unrolled
    const int b = l & 1;
    double cand = alive ? fabs(v[l]) : -1.0;
    if (!(cand >= 0.0)) cand = -1.0;  // NaN never wins
    const double m = gj_wave_max(cand);
    const bool top = cand == m;
    const unsigned long long hit = __ballot(top);
    const unsigned below = __builtin_amdgcn_mbcnt_hi((unsigned)(hit >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((unsigned)hit, 0u));
    if (top && below == 0) {
#pragma unroll
      for (int j = l; j < TS_NB; ++j) slot_r[b][wv][j] = v[j];
      slot_r[b][wv][TS_NB] = m;
      slot_q[b][wv] = t;
    }
    __syncthreads();
    int w = 0;
    double best = slot_r[b][0][TS_NB];
#pragma unroll
    for (int u = 1; u < TS_T / 64; ++u) {
      const double kv = slot_r[b][u][TS_NB];
      if (kv > best) {
        best = kv;
        w = u;
      }
    }
    w = __builtin_amdgcn_readfirstlane(w);
    if (!(best > 0.0)) {  // no nonzero candidate left in this column
      done = true;
      continue;
    }
    const double* r = slot_r[b][w];
    const int q = slot_q[b][w];
    if (t == q) {
      out[l] = id;
      alive = false;
    }
    picked = l + 1;
    const double f = v[l] / r[l];
#pragma unroll
    for (int j = l + 1; j < TS_NB; ++j) v[j] -= f * r[j];
  }
  for (int l = picked + t; l < TS_NB; l += TS_T) out[l] = -1;
}

// A column panel of the systems' matrices: system sy's rows start at
// base + E_off[sy] with row stride n (its order), or, with E_off = nullptr,
// at base + ld sys_coff[sy] with row stride ld (an n x ld side buffer); the
// panel's first column is c0.
struct GjPanel {
  const double* base;
  const int64_t* E_off;
  int ld;
  int c0;
  __device__ const double* rows(int sy, const int32_t* sys_coff) const {
    return base + (E_off ? E_off[sy] : (int64_t)ld * sys_coff[sy]);
  }
  __device__ int stride(int n) const { return E_off ? n : ld; }
};

// Inverse of the kb x kb pivot block P(l, j) = in(row_l, c0 + j), kb =
// min(NBK, n - kp), by Gauss-Jordan elimination without interchanges: row_l
// = picks[l] (the tournament's pick order, in which every multiplier is at
// most 1 in magnitude) or, with picks = nullptr, row kp + l (symmetric
// positive definite systems, whose pivots stay positive without
// interchanges).  256 threads; thread t owns the entries (br + 16 ii, bc +
// 16 jj), br = t / 16, bc = t % 16, ii, jj < NBK / 16, in registers, so the
// register holding row or column m is the same in every thread (m / 16) and
// only the owners (br or bc = m % 16) differ.  Per step the pivot row and
// column go through a double-buffered LDS slot (one barrier per step); every
// entry takes the rank-one update, then the owners of column m and of row m
// overwrite theirs with -a(i, m) / p and a(m, j) / p (1 / p at the pivot).
// Rows and columns past kb are the identity.  A pivot that is not finite,
// zero, or (spd = 1) not positive sets *bad to sy + 1.  Pinv[sy] is NBK x
// NBK, row-major.
template <int NBK>
__global__ void __launch_bounds__(256)
k_gj_block_inv(GjPanel in, const int32_t* sys_coff, int kp, const int32_t* picks, int pstride,
               int spd, double* Pinv, int32_t* bad) {
  constexpr int Q = NBK / 16;
  __shared__ double prow[2][NBK], pcol[2][NBK];
  const int sy = blockIdx.x, t = threadIdx.x;
  const int n = sys_coff[sy + 1] - sys_coff[sy];
  if (kp >= n) return;
  const int kb = min(NBK, n - kp);
  const int br = t >> 4, bc = t & 15;
  const double* A = in.rows(sy, sys_coff);
  const int ld = in.stride(n), c0 = in.c0;
  double a[Q][Q];
#pragma unroll
  for (int ii = 0; ii < Q; ++ii) {
    const int l = br + 16 * ii;
    int row = -1;
    if (l < kb) row = picks ? picks[(int64_t)sy * pstride + l] : kp + l;
#pragma unroll
    for (int jj = 0; jj < Q; ++jj) {
      const int j = bc + 16 * jj;
      const bool inb = l < kb && j < kb;
      const double x = gj_keep(A[(int64_t)max(row, 0) * ld + c0 + min(j, kb - 1)], inb && row >= 0);
      a[ii][jj] = inb ? x : (l == j ? 1.0 : 0.0);
    }
  }
  bool sing = false;
  for (int m = 0; m < kb; ++m) {
    const int b = m & 1, mq = m >> 4, mr = m & 15;  // register index mq is uniform
    if (br == mr) {
#pragma unroll
      for (int ii = 0; ii < Q; ++ii)
        if (ii == mq)
#pragma unroll
          for (int jj = 0; jj < Q; ++jj) prow[b][bc + 16 * jj] = a[ii][jj];
    }
    if (bc == mr) {
#pragma unroll
      for (int jj = 0; jj < Q; ++jj)
        if (jj == mq)
#pragma unroll
          for (int ii = 0; ii < Q; ++ii) pcol[b][br + 16 * ii] = a[ii][jj];
    }
    __syncthreads();
    // every read of the step issued before the first use
    const double piv = prow[b][m];
    double pr[Q], pc[Q];
#pragma unroll
    for (int jj = 0; jj < Q; ++jj) pr[jj] = prow[b][bc + 16 * jj];
#pragma unroll
    for (int ii = 0; ii < Q; ++ii) pc[ii] = pcol[b][br + 16 * ii];
    sing |= !(fabs(piv) < INFINITY) || (spd ? !(piv > 0.0) : !(piv != 0.0));
    const double inv = piv != 0.0 ? 1.0 / piv : 1.0;
    double f[Q];
#pragma unroll
    for (int ii = 0; ii < Q; ++ii) {
      f[ii] = pc[ii] * inv;
#pragma unroll
      for (int jj = 0; jj < Q; ++jj) a[ii][jj] = a[ii][jj] - f[ii] * pr[jj];
    }
    if (bc == mr) {  // column m: -a(i, m) / p
#pragma unroll
      for (int jj = 0; jj < Q; ++jj)
        if (jj == mq)
#pragma unroll
          for (int ii = 0; ii < Q; ++ii) a[ii][jj] = -f[ii];
    }
    if (br == mr) {  // row m: a(m, j) / p, and 1 / p at the pivot
#pragma unroll
      for (int ii = 0; ii < Q; ++ii)
        if (ii == mq)
#pragma unroll
          for (int jj = 0; jj < Q; ++jj) a[ii][jj] = (bc == mr && jj == mq) ? inv : pr[jj] * inv;
    }
  }
  double* out = Pinv + (int64_t)sy * NBK * NBK;
#pragma unroll
  for (int ii = 0; ii < Q; ++ii)
#pragma unroll
    for (int jj = 0; jj < Q; ++jj) out[(br + 16 * ii) * NBK + bc + 16 * jj] = a[ii][jj];
  if (t == 0 && sing) atomicMax(bad, sy + 1);
}

// the tournament's picks as sequential interchanges: swp[sy nb + l] = the
// row that trades places with row k0 + l (the l-th pick, moved by the
// earlier trades of the block); one thread per system
__global__ void k_gj_pick_swaps(const int32_t* sys_coff, int k0, const int32_t* picks, int pstride,
                                int32_t* swp, int32_t* singular) {
  const int sy = blockIdx.x;
  if (threadIdx.x != 0 || sys_coff[sy + 1] - sys_coff[sy] <= k0) return;
  const int kb = min(TS_NB, sys_coff[sy + 1] - sys_coff[sy] - k0);
  const int32_t* P = picks + (int64_t)sy * pstride;
  bool sing = false;
  for (int a = 0; a < kb; ++a) {
    sing |= P[a] < 0;
    int cur = P[a] >= 0 ? P[a] : k0 + a;
    for (int b = 0; b < a; ++b) {
      const int pb = swp[sy * TS_NB + b];
      if (cur == k0 + b)
        cur = pb;
      else if (cur == pb)
        cur = k0 + b;
    }
    swp[sy * TS_NB + a] = cur;
  }
  if (sing) atomicMax(singular, sy + 1);
}

// S(i, :) of the block transform in the block's row order (src from the row
// maps, src_all = nullptr: the identity): P^{-1} on the pivot rows kp .. kp +
// kb, -in(src(i), panel) P^{-1} on the others, as a matrix-core product: 64
// rows (one 16-row slab per wave) by 64 columns of S per workgroup
// (blockIdx.z picks the column half when NBK = 128); the slab of P^{-1}
// sits in LDS.  S(i, j) is stored at Sbuf[ldS (sys_coff[sy] + i) + sc0 + j].
template <int NBK>
__global__ void __launch_bounds__(256)
k_gj_panel_form(GjPanel in, const int32_t* sys_coff, int kp, const double* Pinv,
                const int32_t* src_all, double* Sbuf, int ldS, int sc0) {
  constexpr int LD = 64 + 4;
  __shared__ double Ps[NBK * LD];
  const int sy = blockIdx.y, t = threadIdx.x;
  const int base = sys_coff[sy], n = sys_coff[sy + 1] - base;
  const int i0 = blockIdx.x * 64, c0 = blockIdx.z * 64;
  if (kp >= n || i0 >= n) return;
  const int kb = min(NBK, n - kp);
  const double* Pi = Pinv + (int64_t)sy * NBK * NBK;
#pragma unroll
  for (int q = 0; q < NBK / 4; ++q) {  // all loads of the slab in flight together
    const int e = t + 256 * q;
    Ps[(e >> 6) * LD + (e & 63)] = Pi[(e >> 6) * NBK + c0 + (e & 63)];
  }
  const int w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int ia = i0 + 16 * w + li;  // this lane's row of the A operand
  const int ra = ia < n ? (src_all ? src_all[base + ia] : ia) : 0;
  const double* arow = in.rows(sy, sys_coff) + (int64_t)ra * in.stride(n) + in.c0;
  double av[NBK / 4];
#pragma unroll
  for (int q = 0; q < NBK / 4; ++q) {
    const int l = 4 * q + lk;
    av[q] = gj_keep(arow[min(l, kb - 1)], ia < n && l < kb);
  }
  __syncthreads();
  gj_d4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = gj_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < NBK / 4; ++q) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], Ps[(4 * q + lk) * LD + 16 * c + li],
                                                    acc[c], 0, 0, 0);
  }
  double* S = Sbuf + (int64_t)ldS * base + sc0;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 16 * w + lk + 4 * r, j = c0 + 16 * c + li;
      if (i >= n) continue;
      double v;
      if (j >= kb)
        v = 0.0;
      else if (i >= kp && i < kp + kb)
        v = Ps[(i - kp) * LD + 16 * c + li];
      else
        v = -acc[c][r];
      S[(int64_t)i * ldS + j] = v;
    }
}

// Blocks of 128 columns without interchanges (symmetric positive definite
// systems, large batches): the block's transform is built from two panels of
// 64 so that one rank-128 update replaces two rank-64 ones (half the passes
// over the matrices).  With W the first panel's S and P2 the rows k0 + 64 ..
// k0 + 64 + kb2 - 1:
//   k_gj_narrow   the block's last 64 columns after the first panel's steps,
//                 C(i, c) = in(i, k0 + 64 + c) + sum_l (W(i, l) - [i = k0 + l]) in(k0 + l, k0 + 64 + c),
//                 whose panel (pivot rows P2) gives the second S2;
//   k_gj_combine  the block's first 64 columns, the product of the two
//                 transforms on W: S(i, l) = [i not in P2] W(i, l) + sum_m S2(i, m) W(k0 + 64 + m, l).
// The two transforms applied in turn equal I + (S - [i = k0 + l]) in(k0 + l, :)
// over the 128 rows of the block, which the update applies.

// C (row stride 64 per system, zero in the columns past the matrix); one 64
// x 64 tile of rows per workgroup, grid (tile rows, nsys); W has row stride 64
__global__ void __launch_bounds__(256)
k_gj_narrow(const double* Ain, const int64_t* E_off, const int32_t* sys_coff, int k0,
            const double* Wbuf, double* Cbuf) {
  // the 64 panel columns in two passes of 32 through LDS (34 KB: the
  // kernel fits beside the update's workgroups when they run together)
  __shared__ double Ssh[64 * 33];
  __shared__ double Rsh[32 * GM_RLD];
  const int sy = blockIdx.y, t = threadIdx.x;
  const int base = sys_coff[sy], n = sys_coff[sy + 1] - base;
  const int i0 = blockIdx.x * 64;
  if (n - k0 <= 64 || i0 >= n) return;  // no second panel
  const int m = min(64, n - k0 - 64);   // columns of C inside the matrix
  const int jc = k0 + 64;
  const double* A = Ain + E_off[sy];
  const double* W = Wbuf + (int64_t)64 * base;
  double* Cm = Cbuf + (int64_t)64 * base;
  const int w = t >> 6, lane = t & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  gj_d4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr + bi * 16 + lk + 4 * r, c = wc + bj * 16 + li;
        acc[bi][bj][r] = gj_keep(A[(int64_t)min(i, n - 1) * n + jc + min(c, m - 1)], i < n && c < m);
      }
  for (int h = 0; h < 2; ++h) {
    if (h) __syncthreads();  // the first pass's reads are done
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = t + 256 * q;
      const int sr = e >> 5, sc = e & 31;  // S' tile: 64 rows x 32 panel columns
      const int i = i0 + sr, l = 32 * h + sc;
      Ssh[sr * 33 + sc] =
          gj_keep(W[(int64_t)min(i, n - 1) * 64 + l], i < n) - (i == k0 + l ? 1.0 : 0.0);
      const int rr = e >> 6, rc = e & 63;  // source rows: 32 panel rows x 64 columns
      Rsh[rr * GM_RLD + rc] = gj_keep(A[(int64_t)(k0 + 32 * h + rr) * n + jc + min(rc, m - 1)], rc < m);
    }
    __syncthreads();
    for (int kk = 0; kk < 32; kk += 4) {
      const double a0 = Ssh[(wr + li) * 33 + kk + lk];
      const double a1 = Ssh[(wr + 16 + li) * 33 + kk + lk];
      const double b0 = Rsh[(kk + lk) * GM_RLD + wc + li];
      const double b1 = Rsh[(kk + lk) * GM_RLD + wc + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr + bi * 16 + lk + 4 * r, c = wc + bj * 16 + li;
        if (i < n) Cm[(int64_t)i * 64 + c] = c < m ? acc[bi][bj][r] : 0.0;
      }
}

// S(:, 0 .. 63) of the 128-column block (row stride 128), S(:, 64 ..) = S2
// already in place; one 64-row slab per workgroup, grid (tile rows, nsys)
__global__ void __launch_bounds__(256)
k_gj_combine(const int32_t* sys_coff, int k0, const double* Wbuf, double* Sbuf) {
  constexpr int LD = 64 + 4;
  __shared__ double Xs[64 * LD];
  const int sy = blockIdx.y, t = threadIdx.x;
  const int base = sys_coff[sy], n = sys_coff[sy + 1] - base;
  const int i0 = blockIdx.x * 64;
  if (k0 >= n || i0 >= n) return;
  const double* W = Wbuf + (int64_t)64 * base;
  double* S = Sbuf + (int64_t)128 * base;
  const int kb2 = min(64, n - k0 - 64);
  if (kb2 <= 0) {  // no second panel: the block's transform is the first one's
    for (int e = t; e < 64 * 64; e += 256) {
      const int i = i0 + (e >> 6), l = e & 63;
      if (i < n) S[(int64_t)i * 128 + l] = W[(int64_t)i * 64 + l];
    }
    return;
  }
  // every load first (raw, from clamped addresses), the masks afterwards, so
  // that all of them are in flight together
  const int w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int ia = i0 + 16 * w + li;  // this lane's row of the S2 operand
  const double* s2 = S + (int64_t)min(ia, n - 1) * 128 + 64;
  double xl[16], av[16], wv[4][4];
#pragma unroll
  for (int q = 0; q < 16; ++q) {  // X = W(P2, :), zero past the matrix
    const int e = t + 256 * q;
    xl[q] = W[(int64_t)min(k0 + 64 + (e >> 6), n - 1) * 64 + (e & 63)];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) av[q] = s2[4 * q + lk];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      wv[c][r] = W[(int64_t)min(i0 + 16 * w + lk + 4 * r, n - 1) * 64 + 16 * c + li];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + 256 * q;
    const int mm = e >> 6, l = e & 63;
    Xs[mm * LD + l] = gj_keep(xl[q], mm < kb2);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) av[q] = gj_keep(av[q], ia < n);
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 16 * w + lk + 4 * r;
      const bool p2 = i >= k0 + 64 && i < k0 + 64 + kb2;
      wv[c][r] = gj_keep(wv[c][r], i < n && !p2);
    }
  __syncthreads();
  gj_d4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = gj_d4{wv[c][0], wv[c][1], wv[c][2], wv[c][3]};
#pragma unroll
  for (int q = 0; q < 16; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], Xs[(4 * q + lk) * LD + 16 * c + li], acc[c],
                                                    0, 0, 0);
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + 16 * w + lk + 4 * r;
      if (i < n) S[(int64_t)i * 128 + 16 * c + li] = acc[c][r];
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


// Algorithmic flops of one part of the symmetric update of an order-n system
// (2 kb per entry of the lower 64 x 64 tiles outside the panel columns
// [k0, k0 + kb)): part 0 every lower tile, 1 the band of tiles bl .. bl + bq
// - 1 in rows or columns, 2 the others.
static double gj_sym_update_flops(int64_t n, int64_t k0, int64_t kb, int part, int bl, int bq) {
  const int64_t T = (n + 63) / 64;
  double ent = 0.0;
  for (int64_t ti = 0; ti < T; ++ti) {
    const int64_t rows = std::min<int64_t>(64, n - 64 * ti);
    for (int64_t tj = 0; tj <= ti; ++tj) {
      const bool band = bl >= 0 && ((ti >= bl && ti < bl + bq) || (tj >= bl && tj < bl + bq));
      if ((part == 1 && !band) || (part == 2 && band)) continue;
      const int64_t c0 = 64 * tj, c1 = std::min<int64_t>(n, c0 + 64);
      const int64_t pc = std::max<int64_t>(0, std::min(c1, k0 + kb) - std::max(c0, k0));
      ent += (double)rows * (double)(c1 - c0 - pc);
    }
  }
  return 2.0 * ent * (double)kb;
}

// Inverts the nsys row-major matrices of A in place of a ping-pong pair: system
// sy has order sys_coff[sy + 1] - sys_coff[sy] (device arrays) and starts at
// E_off[sy]; B has the size of A.  Returns A or B, whichever holds the
// inverses (the other is free).  A singular system sets *flag to sy + 1 (the
// largest such index); nrow = sys_coff[nsys] and total = the sum of the
// orders squared (host).
//
// spd = true (the matrices are symmetric up to rounding and expected to be
// positive definite): large systems and large batches (when their update
// runs on the matrix cores) are inverted without interchanges, in blocks of
// 128 columns, each from two panels of 64 (k_gj_narrow, k_gj_combine): the
// 64 x 64 pivot block inverted by Gauss-Jordan (k_gj_block_inv), the
// panel's transform formed on the matrix cores (k_gj_panel_form); no pivot
// search, no row maps, no final un-permutation.  If a pivot is not positive,
// nothing usable is returned (nullptr, after a synchronisation) and the
// caller repeats the inversion with partial pivoting on a fresh copy.
//
// h_orders (host, nsys entries, may be null): the orders of the systems whose
// inversion the method needs (0 for padding systems); with opt.profile bit 1
// every matrix-core update is timed with hipEvents on st and its algorithmic
// flops, 2 n (n - kb) kb per system, are added to the context's counters.
double* gj_invert_batched(Ctx& c, hipStream_t st, int nsys, int64_t maxs, int64_t nrow,
                          int64_t total, double* A, double* B, const int64_t* E_off,
                          const int32_t* sys_coff, int32_t* flag, bool spd = false,
                          const int32_t* h_orders = nullptr) {
  const bool small_batch = total * 8 <= ((int64_t)32 << 20);  // all matrices within 32 MB
  if (maxs <= 0) return A;
  // register-resident panels (one row per thread) up to order GJ_T; orders
  // up to 4 GJ_T: register panels of width 8 with 2-4 rows per thread; above:
  // tournament-pivoted panels of width 64.  Register panels of batches small
  // enough for the caches take width 8 (a quarter of the instructions per
  // dependent pivot step, more update passes).
  const bool reg = maxs <= GJ_T;
  const int R = reg ? 1 : (int)((maxs + GJ_T - 1) / GJ_T);
  const bool multi = !reg && R <= 4;
  // 64 x 64 matrix-core output tiles when they still give the GPU a few
  // thousand workgroups, else 32 x 32 vector tiles (panels of at most 32)
  const unsigned t64 = (unsigned)((maxs + 63) / 64);
  const bool wide = (int64_t)t64 * t64 * nsys >= 2048;
  // without interchanges (matrix-core updates only): blocks of 128 columns
  // from two panels of 64, rank-128 updates
  const bool direct = spd && wide && (maxs > 4 * GJ_T || (reg && !small_batch));
  const bool tslu = !reg && !multi && !direct;
  constexpr int DNB = 64;   // panel width without interchanges
  const int nb = direct ? 2 * DNB : (tslu ? TS_NB : (((reg && small_batch) || multi) ? 8 : 32));
  const int64_t n0t = std::max<int64_t>(nrow, 1);
  int32_t* tot = c.mem.alloc<int32_t>(n0t);
  int32_t* src = c.mem.alloc<int32_t>(n0t);
  double* S = c.mem.alloc<double>(n0t * nb);
  double* Pinv = nullptr;
  double* W1 = nullptr;  // first panel's S and the block's last 64 columns (128-column blocks)
  double* Cn = nullptr;
  int32_t* cand[2] = {nullptr, nullptr};
  int32_t* swp = nullptr;
  int32_t* tmp = nullptr;
  int32_t* dflag = nullptr;
  const int gstride = (int)((maxs + TS_T - 1) / TS_T);
  if (tslu) Pinv = c.mem.alloc<double>((size_t)nsys * nb * nb);
  if (tslu) {
    for (auto& q : cand) q = c.mem.alloc<int32_t>((size_t)nsys * gstride * TS_NB);
    swp = c.mem.alloc<int32_t>((size_t)nsys * nb);
    tmp = c.mem.alloc<int32_t>(n0t);
  }
  if (direct) {  // no interchanges: no row maps, no pivot search
    Pinv = c.mem.alloc<double>((size_t)nsys * DNB * DNB);
    dflag = c.mem.alloc<int32_t>(1);
    ADS_HIP(hipMemsetAsync(dflag, 0, 4, st));
    W1 = c.mem.alloc<double>(n0t * DNB);
    Cn = c.mem.alloc<double>(n0t * DNB);
  }
  double* bufs[2] = {A, B};
  const unsigned tiles = wide ? t64 : (unsigned)((maxs + GJ_TILE - 1) / GJ_TILE);
  const unsigned rows = (unsigned)((maxs + 63) / 64 * 64);  // one thread per row
  if (wide && (int64_t)tiles * tiles * nsys > INT32_MAX)
    fail(ADS_ERR_UNSUPPORTED, "dense inversion batch too large for one launch");
  int cur = 0;
  if (direct) {
    // Lookahead: the update of block b runs in two launches, first the band
    // of tiles that block b + 1's panel kernels read, then the rest; block
    // b + 1's panel kernels run on a second stream during the rest (their
    // panel, pivot-block and transform buffers alternate between two slots,
    // so they never touch what the running update reads).  The stream of the
    // call waits for them before the next update.
    // (only where the panel kernels leave most of the GPU to the update: a
    // few large systems such as the coarse operator; batches of many small
    // systems keep one stream, their panel kernels filling the GPU anyway)
    const dim3 slabs((unsigned)((maxs + 63) / 64), (unsigned)nsys);
    const bool lookahead = (int64_t)slabs.x * nsys <= 2048;
    double* Sb[2] = {S, lookahead ? c.mem.alloc<double>(n0t * nb) : S};
    double* Pb[2] = {Pinv, lookahead ? c.mem.alloc<double>((size_t)nsys * DNB * DNB) : Pinv};
    double* Wb[2] = {W1, lookahead ? c.mem.alloc<double>(n0t * DNB) : W1};
    double* Cb[2] = {Cn, lookahead ? c.mem.alloc<double>(n0t * DNB) : Cn};
    hipStream_t aux = nullptr;
    hipEvent_t ev_band = nullptr, ev_chain = nullptr;
    struct LaGuard {
      hipStream_t& s;
      hipEvent_t& a;
      hipEvent_t& b;
      ~LaGuard() {
        if (s) {
          (void)hipStreamSynchronize(s);
          (void)hipStreamDestroy(s);
        }
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
      }
    } la_guard{aux, ev_band, ev_chain};
    if (lookahead) {
      ADS_HIP(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
      ADS_HIP(hipEventCreateWithFlags(&ev_band, hipEventDisableTiming));
      ADS_HIP(hipEventCreateWithFlags(&ev_chain, hipEventDisableTiming));
    }
    // P^{-1} of each pivot block without interchanges, then S = P^{-1} on
    // the pivot rows and -in(i, panel) P^{-1} on the others on the matrix
    // cores (the row maps are the identity); the 128-column block from two
    // panels of 64
    auto chain = [&](int64_t k0, int sl, const double* src, hipStream_t s2) {
      const GjPanel p1{src, E_off, 0, (int)k0};
      ADS_LAUNCH(k_gj_block_inv<DNB>, dim3(nsys), dim3(256), 0, s2, p1, sys_coff, (int)k0,
                 (const int32_t*)nullptr, 0, 1, Pb[sl], dflag);
      ADS_LAUNCH(k_gj_panel_form<DNB>, slabs, dim3(256), 0, s2, p1, sys_coff, (int)k0, Pb[sl],
                 (const int32_t*)nullptr, Wb[sl], DNB, 0);
      ADS_LAUNCH(k_gj_narrow, slabs, dim3(256), 0, s2, src, E_off, sys_coff, (int)k0, Wb[sl],
                 Cb[sl]);
      const GjPanel p2{Cb[sl], nullptr, DNB, 0};
      ADS_LAUNCH(k_gj_block_inv<DNB>, dim3(nsys), dim3(256), 0, s2, p2, sys_coff, (int)k0 + DNB,
                 (const int32_t*)nullptr, 0, 1, Pb[sl], dflag);
      ADS_LAUNCH(k_gj_panel_form<DNB>, slabs, dim3(256), 0, s2, p2, sys_coff, (int)k0 + DNB,
                 Pb[sl], (const int32_t*)nullptr, Sb[sl], nb, DNB);
      ADS_LAUNCH(k_gj_combine, slabs, dim3(256), 0, s2, sys_coff, (int)k0, Wb[sl], Sb[sl]);
    };
    const bool prof = (c.opt.profile & 2) && h_orders;
    auto update = [&](int64_t k0, int sl, int part, int mir_lo) {
      unsigned grid = tiles * (tiles + 1) / 2 * (unsigned)nsys;
      if (part == 1) grid = (unsigned)gj_band_tiles((int)tiles, mir_lo, nb / 64) * (unsigned)nsys;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (prof) {
        ADS_HIP(hipEventCreate(&e0));
        ADS_HIP(hipEventCreate(&e1));
        ADS_HIP(hipEventRecord(e0, st));
      }
      if (maxs <= GM_O32_MAX)
        ADS_LAUNCH(k_gj_update_mfma<true>, dim3(grid), dim3(GM_T), 0, st, bufs[cur], bufs[1 - cur],
                   E_off, sys_coff, (int)k0, nb, Sb[sl], (const int32_t*)nullptr, (int)tiles, nsys,
                   1, mir_lo, part);
      else
        ADS_LAUNCH(k_gj_update_mfma<false>, dim3(grid), dim3(GM_T), 0, st, bufs[cur], bufs[1 - cur],
                   E_off, sys_coff, (int)k0, nb, Sb[sl], (const int32_t*)nullptr, (int)tiles, nsys,
                   1, mir_lo, part);
      if (prof) {
        ADS_HIP(hipEventRecord(e1, st));
        c.prof_gj_ev.push_back({e0, e1});
        for (int q = 0; q < nsys; ++q) {
          const int64_t ns = h_orders[q];
          if (ns <= k0) continue;
          c.prof_gj_flops += gj_sym_update_flops(ns, k0, std::min<int64_t>(nb, ns - k0), part,
                                                 mir_lo, nb / 64);
        }
      }
    };
    chain(0, 0, bufs[0], st);
    int b = 0;
    for (int64_t k0 = 0; k0 < maxs; k0 += nb, ++b) {
      const int sl = lookahead ? (b & 1) : 0;
      const bool next = k0 + nb < maxs;
      const int mir_lo = next ? (int)((k0 + nb) / 64) : -1;  // the next block's tiles
      if (next && lookahead) {
        update(k0, sl, 1, mir_lo);
        ADS_HIP(hipEventRecord(ev_band, st));
        ADS_HIP(hipStreamWaitEvent(aux, ev_band, 0));
        chain(k0 + nb, 1 - sl, bufs[1 - cur], aux);
        ADS_HIP(hipEventRecord(ev_chain, aux));
        update(k0, sl, 2, mir_lo);
        ADS_HIP(hipStreamWaitEvent(st, ev_chain, 0));
      } else {
        update(k0, sl, 0, mir_lo);
        if (next) chain(k0 + nb, 0, bufs[1 - cur], st);
      }
      cur = 1 - cur;
    }
    if (lookahead)
      for (void* q : {(void*)Sb[1], (void*)Pb[1], (void*)Wb[1], (void*)Cb[1]}) c.mem.release(q);
  }
  for (int64_t k0 = 0; k0 < maxs && !direct; k0 += nb) {
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
      // tournament: leaves, then merges until one group per system is left
      int lev = 0, io = 0;
      ADS_LAUNCH(k_tslu, dim3((unsigned)ts_groups((int)maxs, (int)k0, 0), (unsigned)nsys),
                 dim3(TS_T), 0, st, bufs[cur], E_off, sys_coff, (int)k0, 0, (const int32_t*)nullptr,
                 cand[0], gstride);
      while (ts_groups((int)maxs, (int)k0, lev) > 1) {
        ++lev;
        ADS_LAUNCH(k_tslu, dim3((unsigned)ts_groups((int)maxs, (int)k0, lev), (unsigned)nsys),
                   dim3(TS_T), 0, st, bufs[cur], E_off, sys_coff, (int)k0, lev,
                   (const int32_t*)cand[io], cand[1 - io], gstride);
        io = 1 - io;
      }
      const int pstride = gstride * TS_NB;
      ADS_LAUNCH(k_gj_block_inv<TS_NB>, dim3(nsys), dim3(256), 0, st,
                 (GjPanel{bufs[cur], E_off, 0, (int)k0}), sys_coff, (int)k0,
                 (const int32_t*)cand[io], pstride, 0, Pinv, flag);
      ADS_LAUNCH(k_gj_pick_swaps, dim3(nsys), dim3(64), 0, st, sys_coff, (int)k0,
                 (const int32_t*)cand[io], pstride, swp, flag);
      ADS_LAUNCH(k_gjc_fini, dim3(nsys), dim3(GJ_T), 0, st, sys_coff, (int)k0, nb, swp, src, tot,
                 tmp);
      ADS_LAUNCH(k_gj_panel_form<TS_NB>, dim3((unsigned)((maxs + 63) / 64), (unsigned)nsys, 1),
                 dim3(256), 0, st, (GjPanel{bufs[cur], E_off, 0, (int)k0}), sys_coff, (int)k0,
                 Pinv, (const int32_t*)src, S, nb, 0);
    }
    if (wide) {
      const bool prof = (c.opt.profile & 2) && h_orders;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (prof) {
        ADS_HIP(hipEventCreate(&e0));
        ADS_HIP(hipEventCreate(&e1));
        ADS_HIP(hipEventRecord(e0, st));
      }
      if (maxs <= GM_O32_MAX)
        ADS_LAUNCH(k_gj_update_mfma<true>, dim3(tiles * tiles * (unsigned)nsys), dim3(GM_T), 0, st,
                   bufs[cur], bufs[1 - cur], E_off, sys_coff, (int)k0, nb, S,
                   (const int32_t*)src, (int)tiles, nsys, 0, -1, 0);
      else
        ADS_LAUNCH(k_gj_update_mfma<false>, dim3(tiles * tiles * (unsigned)nsys), dim3(GM_T), 0, st,
                   bufs[cur], bufs[1 - cur], E_off, sys_coff, (int)k0, nb, S,
                   (const int32_t*)src, (int)tiles, nsys, 0, -1, 0);
      if (prof) {
        ADS_HIP(hipEventRecord(e1, st));
        c.prof_gj_ev.push_back({e0, e1});
        for (int q = 0; q < nsys; ++q) {
          const int64_t ns = h_orders[q];
          if (ns <= k0) continue;
          const int64_t kbq = std::min<int64_t>(nb, ns - k0);
          c.prof_gj_flops += 2.0 * (double)ns * (double)(ns - kbq) * (double)kbq;
        }
      }
    } else
      ADS_LAUNCH(k_gj_update<GJ_TILE>, dim3(tiles, tiles, nsys), dim3(GJ_UT), 0, st, bufs[cur],
                 bufs[1 - cur], E_off, sys_coff, (int)k0, nb, S, src);
    cur = 1 - cur;
  }
  double* result = nullptr;
  if (direct) {
    result = bufs[cur];  // identity row maps: nothing to un-permute
    ADS_LAUNCH(k_gj_mirror, dim3(tiles * (tiles + 1) / 2 * (unsigned)nsys), dim3(GM_T), 0, st,
               result, E_off, sys_coff, (int)tiles, nsys);
    int32_t h = 0;
    ADS_HIP(hipMemcpyAsync(&h, dflag, 4, hipMemcpyDeviceToHost, st));
    ADS_HIP(hipStreamSynchronize(st));
    if (h) result = nullptr;
  } else {
    const int rpb = 16;
    ADS_LAUNCH(k_gj_unpermute, dim3((unsigned)((maxs + rpb - 1) / rpb), nsys), dim3(256),
               (size_t)maxs * 4, st, bufs[cur], bufs[1 - cur], E_off, sys_coff, tot, rpb);
    result = bufs[1 - cur];
  }
  for (void* q : {(void*)S, (void*)Pinv, (void*)cand[0], (void*)cand[1], (void*)swp, (void*)tmp,
                  (void*)dflag, (void*)W1, (void*)Cn})
    if (q) c.mem.release(q);
  c.mem.release(src);
  c.mem.release(tot);
  return result;
}

}  // namespace
}  // namespace ads
