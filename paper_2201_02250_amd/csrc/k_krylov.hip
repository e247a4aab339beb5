// Right-preconditioned restarted GMRES(m) and flexible GMRES(m), x0 = 0,
// relative tolerance on ||b - A x|| / ||b|| (Section 4), run independently
// for every (system, right-hand side) instance of a context.
//
// Vectors are n x nrhs column-major over the concatenated systems; instance
// q = sys * nrhs + j owns rows [row0(sys), row1(sys)) of column j.  Every
// instance keeps its own cycle position j_q, Hessenberg column, Givens
// rotations and residual estimate, so restarts happen per instance exactly as
// for a single solve.  Orthogonalisation is classical Gram-Schmidt applied
// twice (CGS2); every inner product is reduced in a fixed order (partials per
// row chunk, then a sequential sum), so results are reproducible.
// A cycle ends when the Arnoldi estimate reaches rtol, at m steps, at maxit,
// or on breakdown; the true residual is then recomputed in FP64 and decides
// convergence or restart.
//
// Complex A (a context of ads_setup_complex) is held in its real form and its
// vectors interleaved: (re, im) of unknown t at rows (2t, 2t + 1).  GMRES is
// then the complex method on those arrays: <v, w> = v^H w has real part
// sum v_r w_r and imaginary part sum (J v)_r w_r with J = multiplication by i
// ((J v)_{2t} = -v_{2t+1}, (J v)_{2t+1} = v_{2t}), h v = re(h) v + im(h) J v,
// and the Hessenberg matrix, the rotations [[conj c, conj s], [-s, c]] and
// the least-squares solve are complex.  Segments start at even rows and have
// even length, so the partner row r ^ 1 is always in the same segment.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "ads_internal.h"

namespace ads {

static constexpr int KR_T = 256;
static constexpr int CH_ROWS = 4 * KR_T;  // rows per reduction chunk (4 per thread)

struct KInst {
  const int64_t* row0;   // [Q] first row of the instance's segment
  const int64_t* rows;   // [Q] segment length
  const int32_t* colj;   // [Q] column index
  int Q;
  int64_t n;
  int nch;               // chunks over the longest segment
};

// y = b - A x (mode 1) or y = A x (mode 0) for the columns [j0, j0 + CH)
// (j0 = CH blockIdx.y) of every row: one thread per row reads the row's
// entries once for all CH columns, and the lanes of a wavefront take
// consecutive rows, so that every column's loads of x and stores of y are
// coalesced; each row is summed in CSR order
template <int CH>
__global__ void __launch_bounds__(256)
k_spmv(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
       const double* __restrict__ val, const double* __restrict__ x, const double* __restrict__ b,
       double* __restrict__ y, int64_t n, int nrhs, int mode) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int j0 = blockIdx.y * CH;
  const int nc = min(CH, nrhs - j0);
  double acc[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) acc[j] = 0.0;
  const int k1 = rowptr[r + 1];
  for (int k = rowptr[r]; k < k1; ++k) {
    const double v = val[k];
    const int64_t c = col[k];
#pragma unroll
    for (int j = 0; j < CH; ++j)
      if (j < nc) acc[j] += v * x[(j0 + j) * n + c];
  }
#pragma unroll
  for (int j = 0; j < CH; ++j)
    if (j < nc) {
      const int64_t e = (j0 + j) * n + r;
      y[e] = mode ? b[e] - acc[j] : acc[j];
    }
}

typedef const double __attribute__((address_space(1)))* gcdptr;

// partial inner products <V_i, w> for i <= jq[q] over one row chunk: every
// thread keeps its 4 rows of w in registers and streams V_i; one wavefront
// sum per vector, the 4 wavefront sums added in order.  CPLX: (re, im) of
// each product at [2i], [2i + 1]
template <bool CPLX>
__global__ void __launch_bounds__(KR_T)
k_mdot_partial(const double* const* __restrict__ V, const double* __restrict__ w, KInst I,
               const int32_t* __restrict__ jq, const int32_t* __restrict__ act, double* part,
               int stride) {
  __shared__ double wsum[KR_T / 64][2 * 66];
  const int q = blockIdx.y, ch = blockIdx.x;
  if (!act[q]) return;
  const int J = jq[q];
  const int64_t r0 = I.row0[q], len = I.rows[q];
  const int64_t a = (int64_t)ch * CH_ROWS;
  if (a >= len) return;
  const int64_t off = (int64_t)I.colj[q] * I.n + r0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double wr[4], wj[4];
  int64_t rr[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t r = a + threadIdx.x + k * KR_T;
    const bool ok = r < len;
    rr[k] = ok ? r : a;  // clamped (its w is zeroed)
    const double x = w[off + rr[k]];
    wr[k] = ok ? x : 0.0;
    if (CPLX) {  // the partner row of w, signed so that sum v_r wj_r = im <v, w>
      const double y = w[off + (rr[k] ^ 1)];
      wj[k] = ok ? ((rr[k] & 1) ? -y : y) : 0.0;
    }
  }
#pragma unroll 2
  for (int i = 0; i <= J; ++i) {
    const gcdptr vi = (gcdptr)(V[i] + off);
    double acc = 0.0, acc2 = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double v = vi[rr[k]];
      acc += v * wr[k];
      if (CPLX) acc2 += v * wj[k];
    }
    acc = adsd::wave_sum(acc);
    if (CPLX) acc2 = adsd::wave_sum(acc2);
    if (lane == 0) {
      wsum[wv][CPLX ? 2 * i : i] = acc;
      if (CPLX) wsum[wv][2 * i + 1] = acc2;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < (CPLX ? 2 : 1) * (J + 1); i += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < KR_T / 64; ++k) s += wsum[k][i];
    part[((int64_t)q * I.nch + ch) * stride + i] = s;
  }
}

// h[q][i] = sum over chunks (lanes stride the chunks, then a wavefront sum:
// fixed order); mode 1 accumulates into h.  One wavefront per i; mult = 2
// for the (re, im) entries of complex products.
__global__ void k_mdot_final(const double* part, KInst I, const int32_t* jq, const int32_t* act,
                             double* h, int stride, int accumulate, int mult) {
  const int q = blockIdx.x;
  if (!act[q]) return;
  const int64_t len = I.rows[q];
  const int nch = (int)((len + CH_ROWS - 1) / CH_ROWS);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = wv; i < mult * (jq[q] + 1); i += nw) {
    double s = 0.0;
    for (int ch = lane; ch < nch; ch += 64) s += part[((int64_t)q * I.nch + ch) * stride + i];
    s = adsd::wave_sum(s);
    if (lane == 0) {
      if (accumulate)
        h[(int64_t)q * stride + i] += s;
      else
        h[(int64_t)q * stride + i] = s;
    }
  }
}

// w -= sum_i h_i V_i (h from the last CGS pass; CPLX: complex h_i)
template <bool CPLX>
__global__ void k_cgs_update(const double* const* __restrict__ V, double* __restrict__ w, KInst I,
                             const int32_t* __restrict__ jq, const int32_t* __restrict__ act,
                             const double* __restrict__ h, int stride) {
  const int q = blockIdx.y;
  if (!act[q]) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= I.rows[q]) return;
  const int64_t idx = (int64_t)I.colj[q] * I.n + I.row0[q] + r;
  const int J = jq[q];
  const double* hq = h + (int64_t)q * stride;
  double v = w[idx];
  if (!CPLX) {
    for (int i = 0; i <= J; ++i) v -= hq[i] * V[i][idx];
  } else {
    const int64_t pj = idx ^ 1;                 // partner row
    const double sg = (idx & 1) ? 1.0 : -1.0;   // (J V)_idx = sg * V_pj
    for (int i = 0; i <= J; ++i) v -= hq[2 * i] * V[i][idx] + hq[2 * i + 1] * sg * V[i][pj];
  }
  w[idx] = v;
}

// segment 2-norms squared: partial + final
__global__ void __launch_bounds__(KR_T)
k_norm_partial(const double* __restrict__ w, KInst I, const int32_t* __restrict__ act,
               double* part) {
  __shared__ double red[16];
  const int q = blockIdx.y, ch = blockIdx.x;
  if (!act[q]) return;
  const int64_t len = I.rows[q];
  const int64_t a = (int64_t)ch * CH_ROWS, b = min<int64_t>(len, a + CH_ROWS);
  const int64_t off = (int64_t)I.colj[q] * I.n + I.row0[q];
  double acc = 0.0;
  for (int64_t r = a + threadIdx.x; r < b; r += blockDim.x) acc += w[off + r] * w[off + r];
  acc = adsd::block_sum(acc, red);
  if (threadIdx.x == 0) part[(int64_t)q * I.nch + ch] = acc;
}

// one wavefront per instance: lanes stride the chunks, then a wavefront sum
__global__ void k_norm_final(const double* part, KInst I, const int32_t* act, double* out) {
  const int q = blockIdx.x;
  if (!act[q]) return;
  const int lane = threadIdx.x;
  const int nch = (int)((I.rows[q] + CH_ROWS - 1) / CH_ROWS);
  double s = 0.0;
  for (int ch = lane; ch < nch; ch += 64) s += part[(int64_t)q * I.nch + ch];
  s = adsd::wave_sum(s);
  if (lane == 0) out[q] = sqrt(s);
}

// copy segments: dst(q) = src(q) * scale[q] (scale null -> 1); masked
__global__ void k_seg_scale(const double* __restrict__ src, double* __restrict__ dst, KInst I,
                            const int32_t* __restrict__ mask, const double* __restrict__ scale,
                            int invert) {
  const int q = blockIdx.y;
  if (!mask[q]) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= I.rows[q]) return;
  const int64_t idx = (int64_t)I.colj[q] * I.n + I.row0[q] + r;
  double sc = scale ? (invert ? 1.0 / scale[q] : scale[q]) : 1.0;
  dst[idx] = src[idx] * sc;
}

// gather V_{jq}(q) into a contiguous vector (or Zf_{jq} <- src)
__global__ void k_seg_pick(const double* const* __restrict__ V, double* __restrict__ dst, KInst I,
                           const int32_t* __restrict__ jq, const int32_t* __restrict__ act,
                           int to_basis) {
  const int q = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= I.rows[q]) return;
  const int64_t idx = (int64_t)I.colj[q] * I.n + I.row0[q] + r;
  if (!act[q]) {
    if (!to_basis) dst[idx] = 0.0;
    return;
  }
  if (to_basis)
    ((double* const*)V)[jq[q]][idx] = dst[idx];
  else
    dst[idx] = V[jq[q]][idx];
}

// Arnoldi bookkeeping per instance: Givens rotations and estimate
struct KState {
  double* H;      // [Q][(m+1)*m] column-major: H[i + j*(m+1)]
  double* cs;     // [Q][m]
  double* sn;     // [Q][m]
  double* g;      // [Q][m+1]
  double* h;      // [Q][stride] CGS coefficients of the current step (pass 1)
  double* h2;     // [Q][stride] CGS coefficients, pass 2
  double* hn;     // [Q] norm of the new vector
  double* est;    // [Q] |g_{j+1}|
  int32_t* jq;    // [Q]
  int32_t* brk;   // [Q] breakdown flag
  int m;
  int stride;
  int cplx;       // complex: H, cs, sn, g, h, h2 hold (re, im) pairs
};

__global__ void k_arnoldi_finish(KState S, const int32_t* act, int Q) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q || !act[q]) return;
  const int m = S.m, j = S.jq[q];
  double* H = S.H + (int64_t)q * (m + 1) * m;
  double* cs = S.cs + (int64_t)q * m;
  double* sn = S.sn + (int64_t)q * m;
  double* g = S.g + (int64_t)q * (m + 1);
  const double* h = S.h + (int64_t)q * S.stride;
  const double* h2 = S.h2 + (int64_t)q * S.stride;
  double hc2 = 0.0;
  for (int i = 0; i <= j; ++i) {
    const double hij = h[i] + h2[i];
    H[i + j * (m + 1)] = hij;
    hc2 += hij * hij;
  }
  const double hn = S.hn[q];
  hc2 += hn * hn;
  H[j + 1 + j * (m + 1)] = hn;
  for (int i = 0; i < j; ++i) {
    double a = H[i + j * (m + 1)], b = H[i + 1 + j * (m + 1)];
    H[i + j * (m + 1)] = cs[i] * a + sn[i] * b;
    H[i + 1 + j * (m + 1)] = -sn[i] * a + cs[i] * b;
  }
  const double a = H[j + j * (m + 1)], b = hn;
  const double den = hypot(a, b);
  cs[j] = den > 0 ? a / den : 1.0;
  sn[j] = den > 0 ? b / den : 0.0;
  H[j + j * (m + 1)] = den;
  H[j + 1 + j * (m + 1)] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  S.est[q] = fabs(g[j + 1]);
  S.brk[q] = (hn <= 1e-14 * sqrt(hc2)) ? 1 : 0;
}

// complex Arnoldi bookkeeping (S.cplx): the same steps in complex arithmetic,
// every array entry a (re, im) pair
__global__ void k_arnoldi_finish_c(KState S, const int32_t* act, int Q) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q || !act[q]) return;
  const int m = S.m, j = S.jq[q];
  double* H = S.H + (int64_t)q * 2 * (m + 1) * m;  // entry (i, c) at 2 (i + c (m + 1))
  double* cs = S.cs + (int64_t)q * 2 * m;
  double* sn = S.sn + (int64_t)q * 2 * m;
  double* g = S.g + (int64_t)q * 2 * (m + 1);
  const double* h = S.h + (int64_t)q * S.stride;
  const double* h2 = S.h2 + (int64_t)q * S.stride;
  const int64_t cj = (int64_t)j * (m + 1);
  double hc2 = 0.0;
  for (int i = 0; i <= j; ++i) {
    const double re = h[2 * i] + h2[2 * i], im = h[2 * i + 1] + h2[2 * i + 1];
    H[2 * (i + cj)] = re;
    H[2 * (i + cj) + 1] = im;
    hc2 += re * re + im * im;
  }
  const double hn = S.hn[q];
  hc2 += hn * hn;
  for (int i = 0; i < j; ++i) {
    const double ar = H[2 * (i + cj)], ai = H[2 * (i + cj) + 1];
    const double br = H[2 * (i + 1 + cj)], bi = H[2 * (i + 1 + cj) + 1];
    const double cr = cs[2 * i], ci = cs[2 * i + 1], sr = sn[2 * i], si = sn[2 * i + 1];
    // conj(c) a + conj(s) b ;  -s a + c b
    H[2 * (i + cj)] = cr * ar + ci * ai + sr * br + si * bi;
    H[2 * (i + cj) + 1] = cr * ai - ci * ar + sr * bi - si * br;
    H[2 * (i + 1 + cj)] = -(sr * ar - si * ai) + (cr * br - ci * bi);
    H[2 * (i + 1 + cj) + 1] = -(sr * ai + si * ar) + (cr * bi + ci * br);
  }
  const double ar = H[2 * (j + cj)], ai = H[2 * (j + cj) + 1];
  const double den = hypot(hypot(ar, ai), hn);
  const double cr = den > 0 ? ar / den : 1.0, ci = den > 0 ? ai / den : 0.0;
  const double sr = den > 0 ? hn / den : 0.0;  // s = h_{j+1,j} / rho is real
  cs[2 * j] = cr;
  cs[2 * j + 1] = ci;
  sn[2 * j] = sr;
  sn[2 * j + 1] = 0.0;
  H[2 * (j + cj)] = den;
  H[2 * (j + cj) + 1] = 0.0;
  H[2 * (j + 1 + cj)] = 0.0;
  H[2 * (j + 1 + cj) + 1] = 0.0;
  const double gr = g[2 * j], gi = g[2 * j + 1];
  g[2 * (j + 1)] = -sr * gr;
  g[2 * (j + 1) + 1] = -sr * gi;
  g[2 * j] = cr * gr + ci * gi;  // conj(c) g_j
  g[2 * j + 1] = cr * gi - ci * gr;
  S.est[q] = hypot(g[2 * (j + 1)], g[2 * (j + 1) + 1]);
  S.brk[q] = (hn <= 1e-14 * sqrt(hc2)) ? 1 : 0;
}

// complex y = H^{-1} g (size j+1), pairs in S.h
__global__ void k_cycle_solve_c(KState S, const int32_t* endm, const int32_t* jend, int Q) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q || !endm[q]) return;
  const int m = S.m, k = jend[q];
  const double* H = S.H + (int64_t)q * 2 * (m + 1) * m;
  const double* g = S.g + (int64_t)q * 2 * (m + 1);
  double* y = S.h + (int64_t)q * S.stride;
  for (int r = k - 1; r >= 0; --r) {
    double vr = g[2 * r], vi = g[2 * r + 1];
    for (int c = r + 1; c < k; ++c) {
      const int64_t e = 2 * (r + (int64_t)c * (m + 1));
      vr -= H[e] * y[2 * c] - H[e + 1] * y[2 * c + 1];
      vi -= H[e] * y[2 * c + 1] + H[e + 1] * y[2 * c];
    }
    const int64_t d = 2 * (r + (int64_t)r * (m + 1));
    const double dr = H[d], di = H[d + 1], dd = dr * dr + di * di;
    y[2 * r] = (vr * dr + vi * di) / dd;
    y[2 * r + 1] = (vi * dr - vr * di) / dd;
  }
}

// y = H^{-1} g (size j+1), stored in S.h for the update
__global__ void k_cycle_solve(KState S, const int32_t* endm, const int32_t* jend, int Q) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q || !endm[q]) return;
  const int m = S.m, k = jend[q];
  const double* H = S.H + (int64_t)q * (m + 1) * m;
  const double* g = S.g + (int64_t)q * (m + 1);
  double* y = S.h + (int64_t)q * S.stride;
  for (int r = k - 1; r >= 0; --r) {
    double v = g[r];
    for (int c = r + 1; c < k; ++c) v -= H[r + c * (m + 1)] * y[c];
    y[r] = v / H[r + r * (m + 1)];
  }
}

// x(q) += sum_{i<jend} y_i B_i(q)  (B = Zf for flexible, V otherwise into u;
// CPLX: complex y_i)
template <bool CPLX>
__global__ void k_combine(const double* const* __restrict__ B, double* __restrict__ out, KInst I,
                          const int32_t* __restrict__ endm, const int32_t* __restrict__ jend,
                          const double* __restrict__ y, int stride, int accumulate) {
  const int q = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= I.rows[q]) return;
  const int64_t idx = (int64_t)I.colj[q] * I.n + I.row0[q] + r;
  if (!endm[q]) {
    if (!accumulate) out[idx] = 0.0;
    return;
  }
  const double* yq = y + (int64_t)q * stride;
  double v = accumulate ? out[idx] : 0.0;
  if (!CPLX) {
    for (int i = 0; i < jend[q]; ++i) v += yq[i] * B[i][idx];
  } else {
    const int64_t pj = idx ^ 1;
    const double sg = (idx & 1) ? 1.0 : -1.0;
    for (int i = 0; i < jend[q]; ++i) v += yq[2 * i] * B[i][idx] + yq[2 * i + 1] * sg * B[i][pj];
  }
  out[idx] = v;
}

// V_{jq}(q) = w(q) / hn[q] for masked instances
__global__ void k_next_basis(double* const* __restrict__ V, const double* __restrict__ w, KInst I,
                             const int32_t* __restrict__ jq, const int32_t* __restrict__ mask,
                             const double* __restrict__ hn) {
  const int q = blockIdx.y;
  if (!mask[q]) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= I.rows[q]) return;
  const int64_t idx = (int64_t)I.colj[q] * I.n + I.row0[q] + r;
  V[jq[q]][idx] = w[idx] / hn[q];
}

__global__ void k_add_masked(double* __restrict__ x, const double* __restrict__ u, KInst I,
                             const int32_t* __restrict__ mask) {
  const int q = blockIdx.y;
  if (!mask[q]) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= I.rows[q]) return;
  const int64_t idx = (int64_t)I.colj[q] * I.n + I.row0[q] + r;
  x[idx] += u[idx];
}

// start of a cycle for masked instances: g = [beta, 0..], jq = 0
__global__ void k_cycle_start(KState S, const int32_t* mask, const double* beta, int Q) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q || !mask[q]) return;
  const int gw = S.cplx ? 2 : 1;
  double* g = S.g + (int64_t)q * gw * (S.m + 1);
  for (int i = 0; i < gw * (S.m + 1); ++i) g[i] = 0.0;
  g[0] = beta[q];
  S.jq[q] = 0;
}

__global__ void k_advance(KState S, const int32_t* mask, int Q) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q || !mask[q]) return;
  S.jq[q] += 1;
}

int gmres_solve(Ctx& c, const double* b, double* x, int nrhs, const ads_ksp_options& ko,
                ads_ksp_result* res, hipStream_t st) {
  const int m = ko.restart;
  const int Q = c.nsys * nrhs;
  const int64_t n = c.n;
  const int maxit = ko.maxit > 0 ? ko.maxit : 1000;
  const bool flex = ko.flexible != 0;
  const int fixed = ko.fixed_iters;
  auto t0 = std::chrono::steady_clock::now();
  Arena mem(st);
  // graphs only on the context's own stream (nothing else is queued there);
  // the apply workspace exists before any capture
  const bool use_graph = c.graphs_on() && st == c.priv;
  if (!work_fits(c, nrhs)) c.drop_apply_graph();
  ensure_work(c, nrhs);
  // two captured forms of one Arnoldi step: alone, and preceded by the
  // previous step's basis update (k_advance, k_next_basis) when no instance
  // ended its cycle there
  hipGraphExec_t step_exec = nullptr, step_exec2 = nullptr;
  struct ExecGuard {
    hipGraphExec_t& e;
    ~ExecGuard() {
      if (e) (void)hipGraphExecDestroy(e);
    }
  } exec_guard{step_exec}, exec_guard2{step_exec2};
  // instance table
  std::vector<int64_t> hrow0(Q), hrows(Q);
  std::vector<int32_t> hcol(Q);
  int64_t maxlen = 1;
  for (int s = 0; s < c.nsys; ++s)
    for (int j = 0; j < nrhs; ++j) {
      int q = s * nrhs + j;
      hrow0[q] = c.sys_row[s];
      hrows[q] = c.sys_row[s + 1] - c.sys_row[s];
      hcol[q] = j;
      maxlen = std::max(maxlen, hrows[q]);
    }
  KInst I;
  I.row0 = upload(mem, hrow0.data(), Q, st);
  I.rows = upload(mem, hrows.data(), Q, st);
  I.colj = upload(mem, hcol.data(), Q, st);
  I.Q = Q;
  I.n = n;
  I.nch = (int)((maxlen + CH_ROWS - 1) / CH_ROWS);
  const bool cx = c.cplx != 0;
  const int cw = cx ? 2 : 1;  // doubles per scalar of the Hessenberg bookkeeping
  const int stride = cw * (m + 2);
  const size_t vsz = (size_t)n * nrhs;
  std::vector<double*> hV(m + 1), hZ(flex ? m : 0);
  for (int i = 0; i <= m; ++i) hV[i] = mem.alloc<double>(vsz);
  for (int i = 0; i < (int)hZ.size(); ++i) hZ[i] = mem.alloc<double>(vsz);
  double** dV = upload(mem, hV.data(), m + 1, st);
  double** dZ = flex ? upload(mem, hZ.data(), m, st) : nullptr;
  double* w = mem.alloc<double>(vsz);
  double* z = mem.alloc<double>(vsz);
  double* u = mem.alloc<double>(vsz);
  KState S;
  S.m = m;
  S.stride = stride;
  S.cplx = cx ? 1 : 0;
  S.H = mem.alloc<double>((size_t)Q * cw * (m + 1) * m);
  S.cs = mem.alloc<double>((size_t)Q * cw * m);
  S.sn = mem.alloc<double>((size_t)Q * cw * m);
  S.g = mem.alloc<double>((size_t)Q * cw * (m + 1));
  S.h = mem.alloc<double>((size_t)Q * stride);
  S.h2 = mem.alloc<double>((size_t)Q * stride);
  // per-iteration status read by the host in one copy: est | hn | brk (int32)
  double* stat = mem.alloc<double>((size_t)3 * Q);
  S.est = stat;
  S.hn = stat + Q;
  S.brk = reinterpret_cast<int32_t*>(stat + 2 * Q);
  S.jq = mem.alloc<int32_t>(Q);
  double* part = mem.alloc<double>((size_t)Q * I.nch * stride);
  double* bnorm_d = mem.alloc<double>(Q);
  double* beta_d = mem.alloc<double>(Q);
  int32_t* act_d = mem.alloc<int32_t>(Q);
  int32_t* cont_d = mem.alloc<int32_t>(Q);  // instances continuing their cycle
  // two status slots (est | hn | brk each): a speculative step copies into
  // the other slot while the host reads this one
  double* stat_pin = c.pin.get((size_t)6 * Q);
  if (!stat_pin) fail(ADS_ERR_OOM, "pinned host memory for the solver status");
  hipEvent_t stat_ev[2] = {nullptr, nullptr};
  struct EventGuard {
    hipEvent_t* e;
    ~EventGuard() {
      for (int k = 0; k < 2; ++k)
        if (e[k]) (void)hipEventDestroy(e[k]);
    }
  } ev_guard{stat_ev};
  for (int k = 0; k < 2; ++k) ADS_HIP(hipEventCreateWithFlags(&stat_ev[k], hipEventDisableTiming));
  int32_t* endm_d = mem.alloc<int32_t>(Q);
  int32_t* jend_d = mem.alloc<int32_t>(Q);
  int32_t* all_d = mem.alloc<int32_t>(Q);
  std::vector<int32_t> ones(Q, 1);
  ADS_HIP(hipMemcpyAsync(all_d, ones.data(), Q * 4, hipMemcpyHostToDevice, st));
  ADS_HIP(hipMemsetAsync(S.jq, 0, Q * 4, st));
  const dim3 gseg((unsigned)((maxlen + 255) / 256), Q);
  // y = b - A x (mode 1) or A x (mode 0) over all nrhs columns, in chunks of
  // 1, 4 or 16 columns per thread
  auto spmv = [&](const double* xv, const double* bv, double* yv, int mode) {
    const unsigned gr = (unsigned)((n + 255) / 256);
    if (nrhs == 1)
      ADS_LAUNCH(k_spmv<1>, dim3(gr, 1), dim3(256), 0, st, c.rowptr, c.col, c.val, xv, bv, yv, n,
                 nrhs, mode);
    else if (nrhs <= 4)
      ADS_LAUNCH(k_spmv<4>, dim3(gr, 1), dim3(256), 0, st, c.rowptr, c.col, c.val, xv, bv, yv, n,
                 nrhs, mode);
    else
      ADS_LAUNCH(k_spmv<16>, dim3(gr, (unsigned)((nrhs + 15) / 16)), dim3(256), 0, st, c.rowptr,
                 c.col, c.val, xv, bv, yv, n, nrhs, mode);
  };
  auto norms = [&](const double* v, const int32_t* mask, double* out) {
    ADS_LAUNCH(k_norm_partial, dim3(I.nch, Q), dim3(KR_T), 0, st, v, I, mask, part);
    ADS_LAUNCH(k_norm_final, dim3(Q), dim3(64), 0, st, part, I, mask, out);
  };
  // x = 0, r = b
  ADS_HIP(hipMemsetAsync(x, 0, vsz * 8, st));
  norms(b, all_d, bnorm_d);
  std::vector<double> bnorm, beta(Q), est(Q), hn(Q);
  download(bnorm, bnorm_d, Q, st);
  for (int q = 0; q < Q; ++q)
    if (!std::isfinite(bnorm[q]))
      fail(ADS_ERR_NAN, "non-finite right-hand side (system " + std::to_string(q / nrhs) +
                            ", column " + std::to_string(q % nrhs) + ")");
  std::vector<int32_t> state(Q, 0);  // 0 active, 1 done
  std::vector<int32_t> its(Q, 0), status(Q, ADS_OK), jcur(Q, 0);
  std::vector<int32_t> act(Q, 0), endm(Q, 0), jend(Q, 0);
  std::vector<int32_t> act_up;  // contents of act_d as last uploaded
  std::vector<double> relres(Q, 0.0);
  for (int q = 0; q < Q; ++q)
    if (bnorm[q] == 0.0) state[q] = 1;
  // residual r = b - A x into w, start cycles for all active instances
  auto start_cycles = [&](const std::vector<int32_t>& mask_h) {
    ADS_HIP(hipMemcpyAsync(endm_d, mask_h.data(), Q * 4, hipMemcpyHostToDevice, st));
    spmv(x, b, w, 1);
    norms(w, endm_d, beta_d);
    std::vector<double> hb;
    download(hb, beta_d, Q, st);
    std::vector<int32_t> m2 = mask_h;
    for (int q = 0; q < Q; ++q)
      if (mask_h[q]) {
        relres[q] = bnorm[q] > 0 ? hb[q] / bnorm[q] : 0.0;
        if (hb[q] == 0.0 || (!fixed && hb[q] <= ko.rtol * bnorm[q])) {
          state[q] = 1;
          m2[q] = 0;
        }
      }
    ADS_HIP(hipMemcpyAsync(endm_d, m2.data(), Q * 4, hipMemcpyHostToDevice, st));
    ADS_LAUNCH(k_seg_scale, gseg, dim3(256), 0, st, w, hV[0], I, endm_d, beta_d, 1);
    ADS_LAUNCH(k_cycle_start, dim3((Q + 63) / 64), dim3(64), 0, st, S, endm_d, beta_d, Q);
    for (int q = 0; q < Q; ++q)
      if (m2[q]) jcur[q] = 0;
  };
  {
    std::vector<int32_t> mk(Q);
    for (int q = 0; q < Q; ++q) mk[q] = state[q] == 0;
    start_cycles(mk);
  }
  bool pending = false;  // k_advance / k_next_basis of the last step not yet launched
  std::vector<int32_t> cont_up;
  // Speculation (one system, one right-hand side): the next step is queued
  // before the host reads this step's status, so the GPU does not idle
  // during the round trip.  It is not queued when this step must end the
  // cycle (restart length, iteration limit) or when the trend of the
  // residual estimates predicts convergence at this step.  If this step
  // ends the cycle anyway, the extra step has only written column j + 1 of
  // V, Z and H, the rotations and g below row j + 1 and w, none of which the
  // end of the cycle reads (it solves with the first jend columns, from the
  // host's jend, and recomputes w); the next cycle starts from k_cycle_start.
  const bool spec_on = Q == 1;
  int slot = 0;
  bool inflight = false;  // this step was queued speculatively (status in slot)
  double est1 = -1.0, est2 = -1.0;  // the last two processed estimates
  auto basis_update = [&]() {
    ADS_LAUNCH(k_advance, dim3((Q + 63) / 64), dim3(64), 0, st, S, cont_d, Q);
    ADS_LAUNCH(k_next_basis, gseg, dim3(256), 0, st, dV, w, I, S.jq, cont_d, S.hn);
  };
  for (;;) {
    bool any = false;
    for (int q = 0; q < Q; ++q) {
      act[q] = state[q] == 0;
      any |= act[q] != 0;
    }
    if (!any) break;
    if (act != act_up) {
      ADS_HIP(hipMemcpyAsync(act_d, act.data(), Q * 4, hipMemcpyHostToDevice, st));
      act_up = act;
    }
    // one Arnoldi step: z = M v_j, w = A z, CGS2 against V, h_{j+1,j}, Givens;
    // replayed from a captured graph after the first step when graphs are on
    auto arnoldi_step = [&]() {
      // z = M v_j ; w = A z
      ADS_LAUNCH(k_seg_pick, gseg, dim3(256), 0, st, (const double* const*)dV, u, I, S.jq, act_d, 0);
      apply_prec(c, u, z, nrhs, st);
      if (flex)
        ADS_LAUNCH(k_seg_pick, gseg, dim3(256), 0, st, (const double* const*)dZ, z, I, S.jq, act_d, 1);
      spmv(z, nullptr, w, 0);
      // CGS2: h1 = V^H w, w -= V h1, h2 = V^H w, w -= V h2, h = h1 + h2
      for (int pass = 0; pass < 2; ++pass) {
        double* hp = pass ? S.h2 : S.h;
        if (cx)
          ADS_LAUNCH(k_mdot_partial<true>, dim3(I.nch, Q), dim3(KR_T), 0, st,
                     (const double* const*)dV, w, I, S.jq, act_d, part, stride);
        else
          ADS_LAUNCH(k_mdot_partial<false>, dim3(I.nch, Q), dim3(KR_T), 0, st,
                     (const double* const*)dV, w, I, S.jq, act_d, part, stride);
        ADS_LAUNCH(k_mdot_final, dim3(Q), dim3(512), 0, st, part, I, S.jq, act_d, hp, stride, 0,
                   cw);
        if (cx)
          ADS_LAUNCH(k_cgs_update<true>, gseg, dim3(256), 0, st, (const double* const*)dV, w, I,
                     S.jq, act_d, hp, stride);
        else
          ADS_LAUNCH(k_cgs_update<false>, gseg, dim3(256), 0, st, (const double* const*)dV, w, I,
                     S.jq, act_d, hp, stride);
      }
      norms(w, act_d, S.hn);
      if (cx)
        ADS_LAUNCH(k_arnoldi_finish_c, dim3((Q + 63) / 64), dim3(64), 0, st, S, act_d, Q);
      else
        ADS_LAUNCH(k_arnoldi_finish, dim3((Q + 63) / 64), dim3(64), 0, st, S, act_d, Q);
    };
    auto update_and_step = [&]() {
      basis_update();
      arnoldi_step();
    };
    auto launch_step = [&](bool with_update) {
      if (use_graph) {
        hipGraphExec_t& ex = with_update ? step_exec2 : step_exec;
        if (!ex) {
          c.capturing = true;
          try {
            ex = with_update ? capture_graph(st, update_and_step) : capture_graph(st, arnoldi_step);
          } catch (...) {
            c.capturing = false;
            throw;
          }
          c.capturing = false;
        }
        ADS_HIP(hipGraphLaunch(ex, st));
      } else if (with_update) {
        update_and_step();
      } else {
        arnoldi_step();
      }
    };
    // status of a step (est | hn | brk) through pinned memory
    auto queue_status = [&](int k) {
      ADS_HIP(hipMemcpyAsync(stat_pin + (size_t)3 * Q * k, stat, (size_t)3 * Q * sizeof(double),
                             hipMemcpyDeviceToHost, st));
      ADS_HIP(hipEventRecord(stat_ev[k], st));
    };
    if (!inflight) {
      launch_step(pending);
      queue_status(slot);
    }
    inflight = false;
    pending = false;
    bool spec = false;
    if (spec_on && act[0]) {
      const bool last = jcur[0] + 1 >= m || its[0] + 1 >= (fixed ? fixed : maxit);
      bool near = false;
      if (!fixed && est1 >= 0.0 && est2 > 0.0)
        near = est1 * (est1 / est2) <= 3.0 * ko.rtol * bnorm[0];
      spec = !last && !near;
    }
    if (spec) {
      if (cont_up.size() != 1 || cont_up[0] != 1) {
        cont_up.assign(1, 1);
        ADS_HIP(hipMemcpyAsync(cont_d, cont_up.data(), 4, hipMemcpyHostToDevice, st));
      }
      launch_step(true);
      queue_status(1 - slot);
    }
    ADS_HIP(hipEventSynchronize(stat_ev[slot]));
    const double* stat_h = stat_pin + (size_t)3 * Q * slot;
    std::vector<int32_t> brk(Q);
    for (int q = 0; q < Q; ++q) {
      est[q] = stat_h[q];
      hn[q] = stat_h[Q + q];
    }
    std::memcpy(brk.data(), stat_h + 2 * Q, (size_t)Q * 4);
    if (spec_on && act[0]) {
      est2 = est1;
      est1 = est[0];
    }
    bool anyend = false;
    for (int q = 0; q < Q; ++q) {
      endm[q] = 0;
      if (!act[q]) continue;
      its[q] += 1;
      jend[q] = jcur[q] + 1;
      bool end = false;
      if (fixed) {
        end = its[q] >= fixed || jend[q] == m || brk[q];
      } else {
        end = est[q] <= ko.rtol * bnorm[q] || jend[q] == m || its[q] >= maxit || brk[q];
      }
      if (end) {
        endm[q] = 1;
        anyend = true;
      } else {
        jcur[q] += 1;
      }
    }
    // next basis vector for continuing instances: launched now when a cycle
    // ends (the end-of-cycle residual reuses w), else at the head of the
    // next step's graph
    if (!anyend && spec) {  // the next step is already queued, with its basis update
      inflight = true;
      slot = 1 - slot;
      continue;
    }
    std::vector<int32_t> cont(Q, 0);
    for (int q = 0; q < Q; ++q) cont[q] = act[q] && !endm[q];
    if (cont != cont_up) {
      ADS_HIP(hipMemcpyAsync(cont_d, cont.data(), Q * 4, hipMemcpyHostToDevice, st));
      cont_up = cont;
    }
    if (anyend)
      basis_update();
    else
      pending = true;
    if (!anyend) continue;
    // end of cycle: x += Z y  (flexible)  or  x += M (V y)
    ADS_HIP(hipMemcpyAsync(endm_d, endm.data(), Q * 4, hipMemcpyHostToDevice, st));
    ADS_HIP(hipMemcpyAsync(jend_d, jend.data(), Q * 4, hipMemcpyHostToDevice, st));
    if (cx)
      ADS_LAUNCH(k_cycle_solve_c, dim3((Q + 63) / 64), dim3(64), 0, st, S, endm_d, jend_d, Q);
    else
      ADS_LAUNCH(k_cycle_solve, dim3((Q + 63) / 64), dim3(64), 0, st, S, endm_d, jend_d, Q);
    auto combine = [&](const double* const* B, double* out, int accumulate) {
      if (cx)
        ADS_LAUNCH(k_combine<true>, gseg, dim3(256), 0, st, B, out, I, endm_d, jend_d, S.h, stride,
                   accumulate);
      else
        ADS_LAUNCH(k_combine<false>, gseg, dim3(256), 0, st, B, out, I, endm_d, jend_d, S.h, stride,
                   accumulate);
    };
    if (flex) {
      combine((const double* const*)dZ, x, 1);
    } else {
      combine((const double* const*)dV, u, 0);
      apply_prec(c, u, z, nrhs, st);
      ADS_LAUNCH(k_add_masked, gseg, dim3(256), 0, st, x, z, I, endm_d);
    }
    // true residual and restart decision
    std::vector<int32_t> restart(Q, 0);
    {
      spmv(x, b, w, 1);
      norms(w, endm_d, beta_d);
      std::vector<double> tr;
      download(tr, beta_d, Q, st);
      for (int q = 0; q < Q; ++q) {
        if (!endm[q]) continue;
        if (!std::isfinite(tr[q]))
          fail(ADS_ERR_NAN, "non-finite residual in the iteration (column " + std::to_string(q) + ")");
        relres[q] = tr[q] / bnorm[q];
        if (fixed) {
          if (its[q] >= fixed || brk[q]) state[q] = 1;
          else restart[q] = 1;
          continue;
        }
        if (tr[q] <= ko.rtol * bnorm[q]) {
          state[q] = 1;
          status[q] = ADS_OK;
        } else if (its[q] >= maxit) {
          state[q] = 1;
          status[q] = ADS_KSP_MAXIT;
        } else if (brk[q]) {
          state[q] = 1;
          status[q] = ADS_KSP_BREAKDOWN;
        } else {
          restart[q] = 1;
        }
      }
    }
    bool anyr = false;
    for (int v : restart) anyr |= v != 0;
    if (anyr) start_cycles(restart);
  }
  ADS_HIP(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  int worst = ADS_OK;
  for (int q = 0; q < Q; ++q) {
    if (res && q < ADS_MAX_RESULTS) {
      res->its[q] = its[q];
      res->relres[q] = relres[q];
      res->status[q] = status[q];
    }
    worst = std::max(worst, status[q]);
  }
  if (res) {
    res->t_setup_ms = c.t_setup_ms;
    res->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  }
  return worst;
}

}  // namespace ads
