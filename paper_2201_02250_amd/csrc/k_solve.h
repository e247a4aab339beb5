// Block-tridiagonal solve with the stored tiles G_k = D_k^{-1}, P_k = G_k A_k,k+1
// (see k_factor.hip), for up to P right-hand sides, executed by one workgroup.
// Used by the preconditioner apply (local solves of eq. 3 / eq. 4) and by the
// eigensolver (the operator of eq. 5).
//
// X (padded local vectors, column j at X + j*ldx) is overwritten in place:
//   forward   y_k = f_k - A_k,k-1 h_{k-1},   h_k = G_k y_k   (h_k stored in X)
//   backward  x_{K-1} = h_{K-1},   x_k = h_k - P_k x_{k+1}.
// The couplings A_k,k-1 (Definition 1 changes only the diagonal, so A_ii and the
// splitting share them) are stored per local row in a fixed-width list of at
// most NCPL (column in the previous block, value) pairs.
//
// Latency hiding: the 2K-1 tiles form one sequence.  Thread t owns row
// r = t mod s and column chunk g = t / s of every tile; it loads exactly the
// tile entries it multiplies into registers D tiles ahead, so no step waits on
// a global load; the couplings and the forward inputs f_k are prefetched the
// same way.  With LDSX the whole local vector lives in LDS (apply, one column);
// otherwise the backward sweep reads h_k at the start of its step.
#pragma once
#include "ads_internal.h"

namespace adsd {

constexpr int NCPL = 4;     // couplings per row kept by the fast path
constexpr int SOLVE_T = 1024;
constexpr int SOLVE_CH = 8; // max tile columns per thread in the fast path

// columns of a tile handled by one thread of the fast path: the even split of
// s columns over T / s groups, rounded up to whole 16-byte vectors
__host__ __device__ inline int solve_chunk(int s, int T, int V) {
  const int G = T / s;
  const int chunk = (s + G - 1) / G;
  return V * ((chunk + V - 1) / V);
}

// rows per thread of the register-resident factorization for block size s
static constexpr int FMR_MAX = 9;
__host__ __device__ inline int factor_rows(int s) {
  const int G = 1024 / s;
  return (s + G - 1) / G;
}
__host__ __device__ inline bool factor_fast_ok(int s) {
  return s >= 1 && s <= 1024 && factor_rows(s) <= FMR_MAX;
}

// fast path applies when every block size s satisfies this (and the couplings fit)
__host__ __device__ inline bool solve_fast_ok(int s, int T = SOLVE_T, int P = 1, int V = 8) {
  if (s < 1 || s > T || (P == 1 ? 4 : 1) * s * P > T) return false;
  return solve_chunk(s, T, V) <= SOLVE_CH;
}

// LDS doubles of the fast path (ybuf, hbuf, partial sums), excluding an
// LDS-resident vector
template <int P>
inline int64_t solve_lds_doubles(const std::vector<int32_t>& sizes, int T) {
  int64_t m = 0;
  for (int s : sizes) {
    const int G = T / s;
    const int64_t d = (int64_t)s * P * (2 + G);
    m = m > d ? m : d;
  }
  return m;
}

template <class FT>
__device__ __forceinline__ float to_f(FT v);
template <>
__device__ __forceinline__ float to_f<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f<__hip_bfloat16>(__hip_bfloat16 v) { return __bfloat162float(v); }

template <class FT>
struct TileReg {
  using T = float;  // FP32 / BF16 tiles are held as float
};
template <>
struct TileReg<double> {
  using T = double;
};
// one 16-byte load of V consecutive tile entries, widened to the register type
template <class FT>
__device__ __forceinline__ void tile_load_vec(const FT* p, typename TileReg<FT>::T* out);
template <>
__device__ __forceinline__ void tile_load_vec<double>(const double* p, double* out) {
  const double2 v = *reinterpret_cast<const double2*>(p);
  out[0] = v.x;
  out[1] = v.y;
}
template <>
__device__ __forceinline__ void tile_load_vec<float>(const float* p, float* out) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  out[0] = v.x;
  out[1] = v.y;
  out[2] = v.z;
  out[3] = v.w;
}
template <>
__device__ __forceinline__ void tile_load_vec<__hip_bfloat16>(const __hip_bfloat16* p, float* out) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    out[2 * i] = __uint_as_float(w[i] << 16);            // low half (element 2i)
    out[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);  // high half (element 2i+1)
  }
}

// One chain of the two-ended block solve (fast path).  Steps q = 0 ..
// nsteps-1 visit blocks k = k0 + q dk:
//   FWD:  h_k = T0_k (Xin_k - C_k h_prev)   (C: row coupling list of block k
//                                            towards block k - dk)
//   !FWD: x_k = Xin_k - T1_k x_prev          (x_prev in hbuf on entry)
// and write the result to Xout (FWD may run in place).  T0_k / T1_k are the
// two tiles of block k (see the factorization).  ccol/cval: couplings of this
// subdomain's padded rows, NCPL per row.  The LDS work vectors are row-major
// [row * P + column] so that the column index is an immediate offset of the
// LDS instruction.  dummy: a private scratch slot of this thread: threads
// that own no vector entry store there, so every store is unconditional.
// Requires LPE * s * pc <= blockDim.x (LPE lanes per entry in phase C).
template <class FT, int P, int D, bool FWD>
__device__ __forceinline__ void block_chain(const FT* __restrict__ fac, int s, int k0, int dk, int nsteps,
                            const int32_t* __restrict__ ccol, const double* __restrict__ cval,
                            const double* Xin, double* Xout, int64_t ldx, int pc, double* lds,
                            double* dummy) {
  using RT = typename TileReg<FT>::T;
  constexpr int V = TileV<FT>::V;         // elements per 16-byte vector
  constexpr int NV = SOLVE_CH / V;        // vectors per thread per tile
  const int t = threadIdx.x, T = blockDim.x;
  const int chV = solve_chunk(s, T, V);   // columns per thread (multiple of V)
  const int G = (s + chV - 1) / chV;      // column groups in use
  const int nq = (s + V - 1) / V;         // vectors per tile row
  const int r = t % s, g = t / s;
  const int c0 = g * chV;
  const int clen = (g < G) ? max(0, min(chV, s - c0)) : 0;
  const int64_t ss = tile_size(s, V);     // tile stride
  const bool pa = t < s * pc;  // phase-A owner of (prr, pj)
  const int prr = t % s, pj = t / s;
  double* ybuf = lds;
  double* hbuf = ybuf + (int64_t)s * P;
  double* part = hbuf + (int64_t)s * P;
  if (nsteps <= 0) return;
  if (FWD) {  // no predecessor: the couplings of the first block are empty
    for (int e = t; e < s * P; e += T) hbuf[e] = 0.0;
    __syncthreads();
  }

  static_assert(D % 2 == 0, "the tile ring depth must be even");
  RT treg[D][SOLVE_CH];
  int creg_c[2][NCPL];  // couplings and forward inputs: a 2-deep ring of their own
  double creg_v[2][NCPL];
  double xreg[2];
  const int pjc = min(pj, pc - 1);  // clamped column for the unconditional prefetch

  // All prefetch loads are unconditional with clamped, in-bounds addresses:
  // branch-free issue keeps the compiler's wait counts exact, so a step only
  // waits for its own tile, not for the tiles prefetched behind it.
  auto blk = [&](int q) { return k0 + min(q, nsteps - 1) * dk; };
  auto issue_tile = [&](int q, int d) {
    const FT* M = fac + (int64_t)blk(q) * 2 * ss + (FWD ? 0 : ss);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int qi = min(c0 / V + v, nq - 1);
      tile_load_vec<FT>(M + ((int64_t)qi * s + r) * V, &treg[d][v * V]);
    }
  };
  auto issue_aux = [&](int q, int e) {
    if (!FWD || !pa) return;  // only the forward phase-A owners need couplings and inputs
    const int row = blk(q) * s + prr;
    xreg[e] = Xin[row + pjc * ldx];
#pragma unroll
    for (int m = 0; m < NCPL; ++m) {
      creg_c[e][m] = ccol[(int64_t)row * NCPL + m];
      creg_v[e][m] = cval[(int64_t)row * NCPL + m];
    }
  };

  // one step with its tile in slot d; phase-C mapping: LPE consecutive lanes
  // per output entry (e = t / LPE), each summing a strided share of the G
  // partials, combined by shuffles
  constexpr int LPE = (P == 1) ? 4 : 1;
  const int ce = t / LPE, cq = t % LPE;
  const bool cown = ce < s * pc;
  const int crr = ce % s, cj = min(ce / s, pc - 1);
  auto step = [&](int q, int d) {
    const int e = d & 1;  // aux slot (q and d have the same parity: q0 is a multiple of D)
    const int r0 = blk(q) * s;
    // backward: Xin_k for phase C, read by its owner (unconditional)
    double hk = FWD ? 0.0 : Xin[r0 + crr + (int64_t)cj * ldx];
    // phase A: the vector the tile multiplies (branch-free coupling reads)
    if (pa) {
      if (FWD) {
        double y = xreg[e];
#pragma unroll
        for (int m = 0; m < NCPL; ++m) {
          const int cc = creg_c[e][m];
          const double w = cc >= 0 ? creg_v[e][m] : 0.0;
          y -= w * hbuf[max(cc, 0) * P + pj];
        }
        ybuf[prr * P + pj] = y;
      } else {
        ybuf[prr * P + pj] = hbuf[prr * P + pj];  // x_prev
      }
    }
    __syncthreads();
    // phase B: partial products with the tile in registers (groups without
    // columns write zeros so the reduction reads defined values)
    if (g < G) {
      double acc[P];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] = 0.0;
#pragma unroll
      for (int c = 0; c < SOLVE_CH; ++c) {
        const double m = (c < clen) ? (double)treg[d][c] : 0.0;
        const int cc = min(c0 + c, s - 1);
#pragma unroll
        for (int j = 0; j < P; ++j) acc[j] += m * ybuf[cc * P + j];
      }
#pragma unroll
      for (int j = 0; j < P; ++j) part[((int64_t)g * s + r) * P + j] = acc[j];
    }
    issue_tile(q + D, d);
    issue_aux(q + 2, e);
    __syncthreads();
    // phase C: reduce, store
    constexpr int UNR = 8;  // unrolled share; the tail loop covers larger G
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int gg = cq + LPE * u;
      if (gg < G) v += part[((int64_t)gg * s + crr) * P + cj];
    }
    for (int gg = cq + LPE * UNR; gg < G; gg += LPE)  // small block sizes
      v += part[((int64_t)gg * s + crr) * P + cj];
    if (LPE >= 2) v += __shfl_xor(v, 1, 64);
    if (LPE >= 4) v += __shfl_xor(v, 2, 64);
    if (!FWD) v = hk - v;
    const bool wr = cown && cq == 0;
    if (wr) hbuf[crr * P + cj] = v;
    double* dst = wr ? Xout + (r0 + crr + (int64_t)cj * ldx) : dummy;
    *dst = v;
    __syncthreads();
  };

#pragma unroll
  for (int d = 0; d < D; ++d) issue_tile(d, d);
  issue_aux(0, 0);
  issue_aux(1, 1);
  // main part: whole groups of D steps, no per-step guard (exact wait counts)
  const int NTmain = nsteps - nsteps % D;
  for (int q0 = 0; q0 < NTmain; q0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) step(q0 + d, d);
  }
  // tail
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (NTmain + d < nsteps) step(NTmain + d, d);
}

// The middle block of the two-ended solve: x_M = T0_M (Xin_M - L h_{M-1} -
// U g_{M+1}) with L, U the row couplings of block M towards blocks M - 1 and
// M + 1 (lcol/lval, ucol/uval), all read from Xin.  The result goes to hbuf
// (the x_prev of both backward chains) and, if Xout is given, to Xout.
template <class FT, int P>
__device__ __forceinline__ void block_mid(const FT* __restrict__ fac, int s, int M, int K,
                          const int32_t* __restrict__ lcol, const double* __restrict__ lval,
                          const int32_t* __restrict__ ucol, const double* __restrict__ uval,
                          const double* Xin, double* Xout, int64_t ldx, int pc, double* lds) {
  constexpr int V = TileV<FT>::V;
  const int t = threadIdx.x, T = blockDim.x;
  double* ybuf = lds;
  double* hbuf = ybuf + (int64_t)s * P;
  double* part = hbuf + (int64_t)s * P;
  const int r0 = M * s;
  for (int e = t; e < s * pc; e += T) {
    const int rr = e % s, j = e / s;
    const int64_t row = r0 + rr;
    double y = Xin[row + j * ldx];
#pragma unroll
    for (int m = 0; m < NCPL; ++m) {
      const int cl = lcol[row * NCPL + m], cu = ucol[row * NCPL + m];
      if (cl >= 0) y -= lval[row * NCPL + m] * Xin[r0 - s + cl + j * ldx];
      if (cu >= 0) y -= uval[row * NCPL + m] * Xin[r0 + s + cu + j * ldx];
    }
    ybuf[rr * P + j] = y;
  }
  __syncthreads();
  const FT* Mt = fac + (int64_t)M * 2 * tile_size(s, V);
  const int G = T / s, chunk = (s + G - 1) / G;
  const int r = t % s, g = t / s;
  if (g < G) {
    double acc[P];
#pragma unroll
    for (int j = 0; j < P; ++j) acc[j] = 0.0;
    const int c1 = min(s, (g + 1) * chunk);
    for (int c = g * chunk; c < c1; ++c) {
      const double m = ld_fac(Mt, tile_at(r, c, s, V));
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] += m * ybuf[c * P + j];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) part[((int64_t)g * s + r) * P + j] = acc[j];
  }
  __syncthreads();
  for (int e = t; e < s * pc; e += T) {
    const int rr = e % s, j = e / s;
    double v = 0.0;
    for (int gg = 0; gg < G; ++gg) v += part[((int64_t)gg * s + rr) * P + j];
    hbuf[rr * P + j] = v;
    if (Xout) Xout[r0 + rr + j * ldx] = v;
  }
  __syncthreads();
}

}  // namespace adsd

namespace adsd {

// General path (any block size, any number of couplings): the tile entries
// are read directly (no prefetch) and the couplings come from the local CSR.
// acc[j] += sum over the 16-byte column groups [qa, qb) of row r of a tile
// (mr = the row's first vector) times vin[c + j s], columns ascending; U
// loads are issued before any is consumed (addresses clamped in bounds)
template <class FT, int P, int U>
__device__ __forceinline__ void tile_row_dot(const FT* __restrict__ mr, int s, int qa, int qb,
                                             const double* vin, double (&acc)[P]) {
  constexpr int V = TileV<FT>::V;
  using RT = typename TileReg<FT>::T;
  for (int q0 = qa; q0 < qb; q0 += U) {
    RT m[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) tile_load_vec<FT>(mr + (int64_t)min(q0 + u, qb - 1) * s * V, m[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c0 = (q0 + u) * V;
      if (q0 + u < qb) {
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (c0 + v < s)
#pragma unroll
            for (int j = 0; j < P; ++j) acc[j] += (double)m[u][v] * vin[c0 + v + j * s];
      }
    }
  }
}

// out = M vin (mode 0) or base - M vin (mode 1) for one s x s tile and pc
// columns of vin (s x P, column-major in LDS).  G = T / s threads share a
// row when 2 s <= T (column chunks of whole 16-byte groups, partial sums
// in part, summed in chunk order), else each thread owns rows.  WIDE: 8
// loads in flight per thread, else 2 (at most 64 registers in 1024-thread
// kernels).
template <class FT, int P, bool WIDE = true>
__device__ __forceinline__ void tile_product_general(const FT* __restrict__ M, int s,
                                                     const double* vin, double* part, double* out,
                                                     int mode, const double* base, int64_t ldb,
                                                     int pc) {
  constexpr int V = TileV<FT>::V;
  constexpr int U = WIDE ? 8 : 2;
  const int t = threadIdx.x, T = blockDim.x;
  const int nq = (s + V - 1) / V;
  const int G = (2 * s <= T) ? (T / s) : 1;
  if (G > 1) {
    const int qch = (nq + G - 1) / G;
    const int r = t % s, g = t / s;
    if (g < G) {
      double acc[P];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[j] = 0.0;
      const int qa = g * qch, qb = min(nq, qa + qch);
      if (qa < qb) tile_row_dot<FT, P, U>(M + (int64_t)r * V, s, qa, qb, vin, acc);
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
      tile_row_dot<FT, P, U>(M + (int64_t)r * V, s, 0, nq, vin, acc);
      for (int j = 0; j < pc; ++j) out[r + j * s] = mode ? base[r + j * ldb] - acc[j] : acc[j];
    }
  }
}

// ---------------------------------------------------------------------------
// Matrix-core tile product for 16 right-hand sides (general path): out = M
// vin on v_mfma_f64_16x16x4f64, the tile entries widened to FP64 as they
// arrive.  Wave w of the workgroup owns 16-row blocks of the output, MF_RB of
// them per pass over the tile's columns.  Per 16 tile columns, lane (i, kk)
// (i = lane % 16, kk = lane / 16) loads the four entries c0 + 4 kk .. c0 + 4
// kk + 3 of its row 16 rb + i (one 16-byte load for FP32 tiles), and step t
// of the four products pairs column c0 + 4 kk + t of the tile with row c0 +
// 4 kk + t of vin: the same permutation of the sum on both operands.  The
// loads run MF_D chunks of 16 columns ahead of the products.  vin is
// column-major, 16 columns with stride ls = s + 1 (which also keeps the 16
// columns of a lane group on different LDS banks); its row s and the
// columns past pc must hold zeros, so that its reads need no masks.  out
// has stride ldo and may be base (each entry is read and written by the
// same lane).
// ---------------------------------------------------------------------------
constexpr int MF_RB = 2;    // 16-row blocks per wave and pass
constexpr int MF_T = 1024;  // threads of the workgroups that use it

// four consecutive tile entries c .. c + 3 (c % 4 == 0) of row r, as loaded;
// a column group past the tile's g groups is clamped to the last one (its
// entries then only meet columns >= s, whose vector entries are zero)
template <class FT>
struct TileQuad;
template <>
struct TileQuad<float> {
  float4 v;
  __device__ void load(const float* M, int r, int c, int s, int g) {
    v = *reinterpret_cast<const float4*>(M + ((int64_t)min(c >> 2, g - 1) * s + r) * 4);
  }
  __device__ double at(int t) const { return (double)(t == 0 ? v.x : t == 1 ? v.y : t == 2 ? v.z : v.w); }
};
template <>
struct TileQuad<double> {
  double2 a, b;
  __device__ void load(const double* M, int r, int c, int s, int g) {  // groups c / 2, c / 2 + 1
    a = *reinterpret_cast<const double2*>(M + ((int64_t)min(c >> 1, g - 1) * s + r) * 2);
    b = *reinterpret_cast<const double2*>(M + ((int64_t)min((c >> 1) + 1, g - 1) * s + r) * 2);
  }
  __device__ double at(int t) const { return t == 0 ? a.x : t == 1 ? a.y : t == 2 ? b.x : b.y; }
};
template <>
struct TileQuad<__hip_bfloat16> {
  uint2 v;
  __device__ void load(const __hip_bfloat16* M, int r, int c, int s, int g) {  // half of group c / 8
    v = *reinterpret_cast<const uint2*>(M + ((int64_t)min(c >> 3, g - 1) * s + r) * 8 + (c & 4));
  }
  __device__ double at(int t) const {
    const uint32_t w = t < 2 ? v.x : v.y;
    return (double)__uint_as_float((t & 1) ? (w & 0xFFFF0000u) : (w << 16));
  }
};

template <class FT>
__device__ void tile_product_mfma(const FT* __restrict__ M, int s, const double* vin, int ls,
                                  double* out, int64_t ldo, int mode, const double* base,
                                  int64_t ldb, int pc) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int t = threadIdx.x, W = blockDim.x >> 6, w = t >> 6, lane = t & 63;
  const int li = lane & 15, kk = lane >> 4;
  const int nrb = (s + 15) >> 4;
  const int ng = (s + TileV<FT>::V - 1) / TileV<FT>::V;  // stored column groups
  for (int rb0 = w * MF_RB; rb0 < nrb; rb0 += W * MF_RB) {
    int row[MF_RB];
#pragma unroll
    for (int u = 0; u < MF_RB; ++u) row[u] = min((rb0 + u) * 16 + li, s - 1);
    d4 acc[MF_RB];
#pragma unroll
    for (int u = 0; u < MF_RB; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
    // ring of MF_D chunks in flight: chunk c0 + 16 d sits in buf[d]
    constexpr int MF_D = sizeof(FT) == 8 ? 2 : 3;
    TileQuad<FT> buf[MF_D][MF_RB];
#pragma unroll
    for (int d = 0; d < MF_D; ++d) {
#pragma unroll
      for (int u = 0; u < MF_RB; ++u) buf[d][u].load(M, row[u], 16 * d + 4 * kk, s, ng);
      __builtin_amdgcn_sched_barrier(0);  // slots issued in order
    }
    // branch-free: the chunks are rounded up to whole rings; a chunk past
    // the tile multiplies zeros (row s of vin) and its loads are clamped
    const int nit = ((s + 15) / 16 + MF_D - 1) / MF_D;
    for (int it = 0; it < nit; ++it) {
#pragma unroll
      for (int d = 0; d < MF_D; ++d) {
        const int cc = (it * MF_D + d) * 16;
        double b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)  // vin(c, li); row s and the columns past pc hold zeros
          b[q] = vin[min(cc + 4 * kk + q, s) + li * ls];
#pragma unroll
        for (int u = 0; u < MF_RB; ++u)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(buf[d][u].at(q), b[q], acc[u], 0, 0, 0);
        // refill the slot MF_D chunks ahead, after its products; the
        // scheduling barriers keep the loads here (not next to their use,
        // and the slot's entries are not widened ahead of the products)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < MF_RB; ++u) buf[d][u].load(M, row[u], cc + 16 * MF_D + 4 * kk, s, ng);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // accumulator register r of lane l: row 16 rb + l / 16 + 4 r, column l % 16
#pragma unroll
    for (int u = 0; u < MF_RB; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (rb0 + u) * 16 + kk + 4 * r, j = li;
        if (rr < s && j < pc) out[rr + j * ldo] = mode ? base[rr + j * ldb] - acc[u][r] : acc[u][r];
      }
  }
}

template <int P>
inline int64_t solve_lds_doubles_general(const std::vector<int32_t>& sizes, int T) {
  int64_t m = 0;
  for (int s : sizes) {
    const int G = (2 * s <= T) ? (T / s) : 1;
    const int64_t d = P == 16 ? (int64_t)(s + 1) * P  // matrix-core products: the input block only
                              : (int64_t)s * P * (2 + (G > 1 ? G : 0));
    m = m > d ? m : d;
  }
  return m;
}

// ccol / cval: the subdomain's row coupling list of A_k,k-1 (NCPL slots per
// padded row, CSR order), or null when the lists are incomplete; the Schur
// step then walks the local CSR rows.  P = 16: the tile products run on the
// matrix cores (tile_product_mfma), with only their input block in LDS
// (column stride s + 1).
template <class FT, int P, bool WIDE = true>
__device__ void block_solve_general(const FT* __restrict__ fac, int s, int K, int n,
                                    const int64_t* __restrict__ lrow,
                                    const int32_t* __restrict__ lcol,
                                    const double* __restrict__ lval,
                                    const int32_t* __restrict__ ccol,
                                    const double* __restrict__ cval, double* X, int64_t ldx, int pc,
                                    double* lds) {
  constexpr bool MF = P == 16;
  const int t = threadIdx.x, T = blockDim.x;
  const int64_t ss = tile_size(s, TileV<FT>::V);  // tile stride
  const int ls = MF ? s + 1 : s;                  // column stride of the LDS vectors
  double* ybuf = lds;
  double* hbuf = ybuf + (int64_t)ls * P;
  double* part = hbuf + (int64_t)ls * P;
  if constexpr (MF) {
    // only the product's input block in LDS; h_k and x_k go straight to X
    // (the next step reads them there after the barrier)
    // the vector phases take GQ entries per thread at a time, their loads
    // issued together (each entry is an independent chain of loads)
    constexpr int GQ = 8;
    const int ne = s * pc;
    for (int e = t; e < ls * P; e += T) ybuf[e] = 0.0;  // row s, columns past pc
    for (int k = 0; k < K; ++k) {
      const int r0 = k * s;
      __syncthreads();
      for (int e0 = 0; e0 < ne; e0 += T * GQ) {
        double y[GQ];
#pragma unroll
        for (int q = 0; q < GQ; ++q) {
          const int e = min(e0 + t + T * q, ne - 1);
          const int rr = e % s, j = e / s;
          y[q] = X[r0 + rr + j * ldx];
        }
        if (k > 0) {
#pragma unroll
          for (int q = 0; q < GQ; ++q) {
            const int e = min(e0 + t + T * q, ne - 1);
            const int rr = e % s, j = e / s;
            const int r = r0 + rr;
            const double* hp = X + (r0 - s) + j * ldx;  // h_{k-1}
            if (ccol) {
              const int32_t* cr = ccol + (int64_t)r * NCPL;
              const double* vr = cval + (int64_t)r * NCPL;
#pragma unroll
              for (int m = 0; m < NCPL; ++m) {
                const int cc = cr[m];
                if (cc >= 0) y[q] -= vr[m] * hp[cc];
              }
            } else if (r < n) {
              for (int64_t qq = lrow[r]; qq < lrow[r + 1]; ++qq) {
                const int cc = lcol[qq] - (r0 - s);
                if (cc >= 0 && cc < s) y[q] -= lval[qq] * hp[cc];
              }
            }
          }
        }
#pragma unroll
        for (int q = 0; q < GQ; ++q) {
          const int e = e0 + t + T * q;
          if (e < ne) ybuf[e % s + (e / s) * ls] = y[q];
        }
      }
      __syncthreads();
      tile_product_mfma<FT>(fac + (int64_t)k * 2 * ss, s, ybuf, ls, X + r0, ldx, 0, nullptr, 0, pc);
    }
    for (int k = K - 2; k >= 0; --k) {
      const int r0 = k * s;
      __syncthreads();
      for (int e0 = 0; e0 < ne; e0 += T * GQ) {  // x_{k+1}
        double y[GQ];
#pragma unroll
        for (int q = 0; q < GQ; ++q) {
          const int e = min(e0 + t + T * q, ne - 1);
          y[q] = X[r0 + s + e % s + (e / s) * ldx];
        }
#pragma unroll
        for (int q = 0; q < GQ; ++q) {
          const int e = e0 + t + T * q;
          if (e < ne) ybuf[e % s + (e / s) * ls] = y[q];
        }
      }
      __syncthreads();
      tile_product_mfma<FT>(fac + (int64_t)k * 2 * ss + ss, s, ybuf, ls, X + r0, ldx, 1, X + r0,
                            ldx, pc);
    }
    __syncthreads();
    return;
  }
  auto product = [&](const FT* M, int mode, const double* base) {
    tile_product_general<FT, P, WIDE>(M, s, ybuf, part, hbuf, mode, base, ldx, pc);
  };
  for (int k = 0; k < K; ++k) {
    const int r0 = k * s;
    __syncthreads();
    if (ccol) {
      for (int e = t; e < s * pc; e += T) {
        const int rr = e % s, j = e / s;
        const int r = r0 + rr;
        double y = X[r + j * ldx];
        if (k > 0) {
          const int32_t* cr = ccol + (int64_t)r * NCPL;
          const double* vr = cval + (int64_t)r * NCPL;
#pragma unroll
          for (int m = 0; m < NCPL; ++m) {
            const int cc = cr[m];
            if (cc >= 0) y -= vr[m] * hbuf[cc + j * ls];
          }
        }
        ybuf[rr + j * ls] = y;
      }
    } else {
      for (int e = t; e < s * pc; e += T) {
        const int rr = e % s, j = e / s;
        const int r = r0 + rr;
        double y = X[r + j * ldx];
        if (k > 0 && r < n) {
          for (int64_t q = lrow[r]; q < lrow[r + 1]; ++q) {
            const int cc = lcol[q] - (r0 - s);
            if (cc >= 0 && cc < s) y -= lval[q] * hbuf[cc + j * ls];
          }
        }
        ybuf[rr + j * ls] = y;
      }
    }
    __syncthreads();
    product(fac + (int64_t)k * 2 * ss, 0, nullptr);
    __syncthreads();
    for (int e = t; e < s * pc; e += T) {
      const int rr = e % s, j = e / s;
      X[r0 + rr + j * ldx] = hbuf[rr + j * ls];
    }
  }
  for (int k = K - 2; k >= 0; --k) {
    const int r0 = k * s;
    __syncthreads();
    for (int e = t; e < s * pc; e += T) {
      const int rr = e % s, j = e / s;
      ybuf[rr + j * ls] = hbuf[rr + j * ls];
    }
    __syncthreads();
    product(fac + (int64_t)k * 2 * ss + ss, 1, X + r0);
    __syncthreads();
    for (int e = t; e < s * pc; e += T) {
      const int rr = e % s, j = e / s;
      X[r0 + rr + j * ldx] = hbuf[rr + j * ls];
    }
  }
  __syncthreads();
}

}  // namespace adsd
