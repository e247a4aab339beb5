// Learned warm start for the local eigenproblems of eq. 5: a message-passing
// graph network on the graph of each subdomain matrix A_ii predicts a block
// whose span approximates the coarse space of eq. 6 (Section 3.2).  Not part
// of the paper's method; the exact eigensolve stays the reference and the
// fallback.
//
//   h_0 = F W_in^T + b_in
//   a_l = A_w h_l,  u_l = h_l W_s,l^T + a_l W_n,l^T + b_l,  h_{l+1} = h_l + relu(u_l)
//   X = h_L W_out^T
//
// Weights are BF16 (an FP32 master copy is kept by the trainer), activations
// and every accumulation FP32.  Nodes of a batch of graphs are numbered
// consecutively; the graph must be symmetric (w_jk = w_kj), which lets the
// backward pass use the aggregation as its own transpose.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "ads_internal.h"

namespace ads {

namespace {

constexpr int GW = 64;   // largest width
constexpr int GO = 16;   // largest output count
constexpr int DT = 256;  // threads of the dense and reduction kernels
constexpr int DR = 32;   // rows per dense block
constexpr int RB = 256;  // rows per weight-gradient block
constexpr int RC = 64;   // rows staged at a time by the weight-gradient kernel

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}

struct Off {  // offsets of the parameter blocks in the flat vector
  int64_t w_in, b_in, w_out, total;
  int64_t ws(int l) const { return b_in + w + (int64_t)l * (2 * w * w + w); }
  int64_t wn(int l) const { return ws(l) + (int64_t)w * w; }
  int64_t b(int l) const { return ws(l) + 2 * (int64_t)w * w; }
  int64_t w;
};

Off offsets(const ads_gnn_shape& s) {
  Off o;
  o.w = s.width;
  o.w_in = 0;
  o.b_in = (int64_t)s.width * s.n_in;
  o.w_out = o.b_in + s.width + (int64_t)s.layers * (2 * (int64_t)s.width * s.width + s.width);
  o.total = o.w_out + (int64_t)s.n_out * s.width;
  return o;
}

void check_shape(const ads_gnn_shape* s) {
  if (!s) fail(ADS_ERR_ARG, "null shape");
  if (s->n_in < 1 || s->n_in > GW || s->width < 1 || s->width > GW || s->layers < 0 ||
      s->layers > 16 || s->n_out < 1 || s->n_out > GO)
    fail(ADS_ERR_ARG, "network shape out of range (n_in, width <= 64, n_out <= 16, layers <= 16)");
}

void check_graph(const ads_gnn_graph* g, int n_in) {
  if (!g || g->ngraph < 1 || g->nnode < 1 || !g->node_off || !g->row_ptr || !g->col || !g->w ||
      !g->feat || !g->mask)
    fail(ADS_ERR_ARG, "incomplete graph batch");
  if (g->nnode > (int64_t)1 << 30) fail(ADS_ERR_ARG, "graph batch too large");
  (void)n_in;
}

// Y = X1 W1^T (+ X2 W2^T) (+ b), W(o, i) = W[o * so + i * si] in BF16.
// mode 0: Y = result; 1: U = result, Y = X1 + relu(result) (a residual
// layer, I1 = O); 2: Y += result.  One block: DR rows x O (<= 64) outputs;
// the weights are staged transposed in LDS (lanes read consecutive outputs),
// the rows of X1 | X2 staged beside them.
__global__ void __launch_bounds__(DT) k_gnn_dense(int n, const float* X1, int ld1, int I1,
                                                  const uint16_t* W1, int so1, int si1,
                                                  const float* X2, int ld2, int I2,
                                                  const uint16_t* W2, int so2, int si2,
                                                  const uint16_t* bias, int O, int mode, float* Y,
                                                  int ldy, float* U) {
  __shared__ float Wt[2 * GW][GW];
  __shared__ float Xs[DR][2 * GW + 1];
  const int t = threadIdx.x;
  const int I = I1 + I2;
  for (int e = t; e < I * GW; e += DT) {
    const int i = e / GW, o = e % GW;
    float v = 0.0f;
    if (o < O) v = i < I1 ? bf2f(W1[(int64_t)o * so1 + (int64_t)i * si1])
                          : bf2f(W2[(int64_t)o * so2 + (int64_t)(i - I1) * si2]);
    Wt[i][o] = v;
  }
  const int64_t r0 = (int64_t)blockIdx.x * DR;
  for (int e = t; e < DR * I; e += DT) {
    const int r = e / I, i = e % I;
    const int64_t row = r0 + r;
    float v = 0.0f;
    if (row < n) v = i < I1 ? X1[row * ld1 + i] : X2[row * ld2 + (i - I1)];
    Xs[r][i] = v;
  }
  __syncthreads();
  const int o = t % GW, rq = t / GW;  // 4 row groups
  constexpr int NR = DR / (DT / GW);
  float acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0.0f;
  for (int i = 0; i < I; ++i) {
    const float wv = Wt[i][o];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] += Xs[rq + k * (DT / GW)][i] * wv;
  }
  if (o >= O) return;
  const float bv = bias ? bf2f(bias[o]) : 0.0f;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int r = rq + k * (DT / GW);
    const int64_t row = r0 + r;
    if (row >= n) continue;
    const float u = acc[k] + bv;
    if (mode == 0) {
      Y[row * ldy + o] = u;
    } else if (mode == 1) {
      U[row * ldy + o] = u;
      Y[row * ldy + o] = Xs[r][o] + fmaxf(u, 0.0f);
    } else {
      Y[row * ldy + o] += u;
    }
  }
}

// A[j][c] (+)= sum over the edges (j, k) of w_jk H[k][c]; one wave per node,
// one lane per channel, edges in their stored order
__global__ void __launch_bounds__(256) k_gnn_agg(int64_t n, const int64_t* row_ptr,
                                                 const int32_t* col, const float* w,
                                                 const float* H, int width, float* A, int acc) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int c = threadIdx.x & 63;
  if (j >= n || c >= width) return;
  float s = 0.0f;
  for (int64_t e = row_ptr[j]; e < row_ptr[j + 1]; ++e) s += w[e] * H[(int64_t)col[e] * width + c];
  if (acc)
    A[j * width + c] += s;
  else
    A[j * width + c] = s;
}

// D = G * (U > 0)
__global__ void k_gnn_relu_mask(int64_t cnt, const float* G, const float* U, float* D) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) D[e] = U[e] > 0.0f ? G[e] : 0.0f;
}

// partial sums over the rows of one block of RB rows: P^T Q (O x I, row-major)
// and, if bias, the column sums of P (O); rows staged RC at a time
__global__ void __launch_bounds__(DT) k_gnn_wgrad(int64_t n, const float* P, int ldp, int O,
                                                  const float* Q, int ldq, int I, int bias,
                                                  float* part, int64_t pstride) {
  __shared__ float Ps[RC][GW + 1];
  __shared__ float Qs[RC][GW + 1];
  const int t = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * RB;
  constexpr int NE = GW * GW / DT;
  float acc[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) acc[k] = 0.0f;
  float bsum = 0.0f;
  for (int c0 = 0; c0 < RB; c0 += RC) {
    __syncthreads();
    for (int e = t; e < RC * GW; e += DT) {
      const int r = e / GW, q = e % GW;
      const int64_t row = b0 + c0 + r;
      Ps[r][q] = (row < n && q < O) ? P[row * ldp + q] : 0.0f;
      Qs[r][q] = (row < n && q < I) ? Q[row * ldq + q] : 0.0f;
    }
    __syncthreads();
    // thread t owns the entries (o, i) = (t / GW + k DT / GW, t % GW)
    const int i = t % GW, o0 = t / GW;
#pragma unroll 2
    for (int r = 0; r < RC; ++r) {
      const float q = Qs[r][i];
#pragma unroll
      for (int k = 0; k < NE; ++k) acc[k] += Ps[r][o0 + k * (DT / GW)] * q;
    }
    if (bias && t < GW)
      for (int r = 0; r < RC; ++r) bsum += Ps[r][t];
  }
  float* out = part + (int64_t)blockIdx.x * pstride;
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = t + k * DT, o = e / GW, i = e % GW;
    if (o < O && i < I) out[o * I + i] = acc[k];
  }
  if (bias && t < O) out[O * I + t] = bsum;
}

// grad[gw + e] += sum over blocks of part[blk][e] (e < O I), then the bias
// part into grad[gb + o]; blocks summed in order (deterministic)
__global__ void k_gnn_reduce(const float* part, int64_t pstride, int nblk, int OI, int O,
                             float* grad, int64_t gw, int64_t gb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int cnt = OI + (gb >= 0 ? O : 0);
  if (e >= cnt) return;
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * pstride + e];
  if (e < OI)
    grad[gw + e] += s;
  else
    grad[gb + (e - OI)] += s;
}

// projection loss per graph (one block per graph): C = (X^T X)^{-1} X^T Z over
// the masked rows, loss_g = ||Z - X C||^2 / ||Z||^2, dX = -2 (Z - X C) C^T /
// (G ||Z||^2) on masked rows, 0 elsewhere
__global__ void __launch_bounds__(256) k_gnn_loss(int ngraph, const int64_t* node_off,
                                                  const uint8_t* mask, const float* X, int k,
                                                  const float* Z, int nz, float* dX,
                                                  double* gloss) {
  __shared__ double Gm[GO * GO];
  __shared__ double Ym[GO * GO];
  __shared__ double Cm[GO * GO];
  __shared__ double red[256];
  __shared__ int okf;
  const int g = blockIdx.x, t = threadIdx.x;
  const int64_t r0 = node_off[g], r1 = node_off[g + 1];
  // X^T X (k x k), X^T Z (k x nz) and ||Z||^2: one entry per thread pair
  const int nG = k * k, nY = k * nz;
  for (int e = t; e < nG + nY; e += 256) {
    double s = 0.0;
    if (e < nG) {
      const int a = e / k, b = e % k;
      for (int64_t r = r0; r < r1; ++r)
        if (mask[r]) s += (double)X[r * k + a] * X[r * k + b];
      Gm[e] = s;
    } else {
      const int q = e - nG, a = q / nz, b = q % nz;
      for (int64_t r = r0; r < r1; ++r)
        if (mask[r]) s += (double)X[r * k + a] * Z[r * nz + b];
      Ym[q] = s;
    }
  }
  double zz = 0.0;
  for (int64_t r = r0 + t; r < r1; r += 256)
    if (mask[r])
      for (int b = 0; b < nz; ++b) zz += (double)Z[r * nz + b] * Z[r * nz + b];
  red[t] = zz;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double zsum = red[0];
  __syncthreads();
  if (t == 0) {
    // Cholesky G = R^T R (upper R in Gm), then C = R^{-1} R^{-T} Y
    int ok = 1;
    for (int c = 0; c < k; ++c) {
      double d = Gm[c * k + c];
      for (int q = 0; q < c; ++q) d -= Gm[q * k + c] * Gm[q * k + c];
      if (!(d > 0.0)) {
        ok = 0;
        d = 1e-300;
      }
      const double rc = sqrt(d);
      Gm[c * k + c] = rc;
      for (int j = c + 1; j < k; ++j) {
        double v = Gm[c * k + j];
        for (int q = 0; q < c; ++q) v -= Gm[q * k + c] * Gm[q * k + j];
        Gm[c * k + j] = v / rc;
      }
    }
    for (int b = 0; b < nz; ++b) {
      for (int a = 0; a < k; ++a) {  // forward: R^T y = Y
        double v = Ym[a * nz + b];
        for (int q = 0; q < a; ++q) v -= Gm[q * k + a] * Cm[q * nz + b];
        Cm[a * nz + b] = v / Gm[a * k + a];
      }
      for (int a = k - 1; a >= 0; --a) {  // backward: R c = y
        double v = Cm[a * nz + b];
        for (int q = a + 1; q < k; ++q) v -= Gm[a * k + q] * Cm[q * nz + b];
        Cm[a * nz + b] = v / Gm[a * k + a];
      }
    }
    okf = ok && zsum > 0.0;
  }
  __syncthreads();
  const double scale = okf ? -2.0 / ((double)ngraph * zsum) : 0.0;
  double ls = 0.0;
  for (int64_t r = r0 + t; r < r1; r += 256) {
    if (!mask[r]) {
      for (int a = 0; a < k; ++a) dX[r * k + a] = 0.0f;
      continue;
    }
    double res[GO];
    for (int b = 0; b < nz; ++b) {
      double v = Z[r * nz + b];
      for (int a = 0; a < k; ++a) v -= (double)X[r * k + a] * Cm[a * nz + b];
      res[b] = v;
      ls += v * v;
    }
    for (int a = 0; a < k; ++a) {
      double v = 0.0;
      for (int b = 0; b < nz; ++b) v += res[b] * Cm[a * nz + b];
      dX[r * k + a] = (float)(scale * v);
    }
  }
  red[t] = ls;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) gloss[g] = okf ? red[0] / zsum : 1.0;
}

__global__ void k_gnn_loss_sum(int ngraph, const double* gloss, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int g = 0; g < ngraph; ++g) s += gloss[g];
  *out = s / ngraph;
}

__global__ void k_gnn_adam(int64_t np, float* master, uint16_t* wbf, const float* grad, float* m,
                           float* v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np) return;
  const float g = grad[e];
  const float mm = b1 * m[e] + (1.0f - b1) * g;
  const float vv = b2 * v[e] + (1.0f - b2) * g * g;
  m[e] = mm;
  v[e] = vv;
  const float p = master[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  master[e] = p;
  wbf[e] = f2bf(p);
}

__global__ void k_gnn_round(int64_t np, const float* master, uint16_t* wbf) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < np) wbf[e] = f2bf(master[e]);
}

// ---------------------------------------------------------------------------
// graph and features of the subdomain matrices of a context
// ---------------------------------------------------------------------------
// mean |a_jj| per subdomain (one block each) and a check that every local row
// holds its diagonal
__global__ void k_gnn_diag_mean(const int64_t* om_off, const int64_t* lrow, const int32_t* lcol,
                                const double* lval, double* dmean, int32_t* err) {
  __shared__ double red[256];
  const int i = blockIdx.x, t = threadIdx.x;
  const int64_t b = om_off[i], n = om_off[i + 1] - b;
  double s = 0.0;
  for (int64_t r = t; r < n; r += 256) {
    int found = 0;
    for (int64_t q = lrow[b + r]; q < lrow[b + r + 1]; ++q)
      if (lcol[q] == r) {
        s += fabs(lval[q]);
        found = 1;
      }
    if (!found) atomicOr(err, 1);
  }
  red[t] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) dmean[i] = n ? red[0] / n : 1.0;
}

__device__ __forceinline__ double local_entry(const int64_t* lrow, const int32_t* lcol,
                                              const double* lval, int64_t row, int c) {
  int64_t lo = lrow[row], hi = lrow[row + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (lcol[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < lrow[row + 1] && lcol[lo] == c) ? lval[lo] : 0.0;
}

// one thread per node (slot g of subdomain i, local row r): the edges of the
// off-diagonal entries of row r, symmetric weights
// (|a_rk| + |a_kr|) / (2 sqrt(|a_rr a_kk|)), and the ADS_GNN_FEATURES features
__global__ void k_gnn_graph(int64_t T, const int32_t* om_sub, const int64_t* om_off,
                            const uint8_t* om_int, const int64_t* lrow, const int32_t* lcol,
                            const double* lval, const double* lsum, const int32_t* bs,
                            const double* dmean, int64_t* row_ptr, int32_t* col, float* w,
                            float* feat, uint8_t* mask) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g > T) return;
  if (g == T) {
    row_ptr[T] = lrow[T] - T;
    return;
  }
  const int i = om_sub[g];
  const int64_t b = om_off[i];
  const int r = (int)(g - b), n = (int)(om_off[i + 1] - b);
  const double ajj = fabs(local_entry(lrow, lcol, lval, g, r));
  int64_t e = lrow[g] - g;  // one diagonal entry per earlier row
  const int64_t e_end = lrow[g + 1] - (g + 1);
  row_ptr[g] = e;
  double offs = 0.0;
  for (int64_t q = lrow[g]; q < lrow[g + 1]; ++q) {
    const int k = lcol[q];
    if (k == r || e >= e_end) continue;  // (a row without diagonal is reported)
    const double akk = fabs(local_entry(lrow, lcol, lval, b + k, k));
    const double akr = local_entry(lrow, lcol, lval, b + k, r);
    const double den = 2.0 * sqrt(ajj * akk);
    col[e] = (int32_t)(b + k);
    w[e] = den > 0.0 ? (float)((fabs(lval[q]) + fabs(akr)) / den) : 0.0f;
    offs += fabs(lval[q]);
    ++e;
  }
  const double dm = dmean[i] > 0.0 ? dmean[i] : 1.0;
  const double tt = n > 1 ? (double)r / (n - 1) : 0.0;
  const int s = bs[i] > 0 ? bs[i] : 1;
  const double qq = (double)(r % s) / s;
  const double pi = 3.14159265358979323846;
  float f[ADS_GNN_FEATURES];
  f[0] = (float)(ajj / dm);
  f[1] = (float)log(fmax(ajj / dm, 1e-30));
  f[2] = ajj > 0.0 ? (float)(lsum[g] / ajj) : 0.0f;
  f[3] = om_int[g] ? 1.0f : 0.0f;
  f[4] = ajj > 0.0 ? (float)(offs / ajj) : 0.0f;
  f[5] = (float)tt;
  f[6] = (float)qq;
  f[7] = (float)sin(pi * tt);
  f[8] = (float)cos(pi * tt);
  f[9] = (float)sin(2.0 * pi * tt);
  f[10] = (float)cos(2.0 * pi * tt);
  f[11] = (float)sin(pi * qq);
  f[12] = (float)cos(pi * qq);
  f[13] = (float)sin(2.0 * pi * qq);
  f[14] = (float)cos(2.0 * pi * qq);
  f[15] = 1.0f;
  for (int c = 0; c < ADS_GNN_FEATURES; ++c) feat[g * ADS_GNN_FEATURES + c] = f[c];
  mask[g] = om_int[g];
}

// coarse basis rows to node rows (one block per subdomain): interior row of
// local rank q gets W_i[q, 0:min(nev_i, nz)], every other entry is zero
__global__ void k_gnn_targets(const int64_t* om_off, const uint8_t* om_int, const int32_t* nev,
                              const int64_t* W_off, const double* W, int nz, float* Z) {
  __shared__ int wtot[16];
  const int i = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t b = om_off[i];
  const int n = (int)(om_off[i + 1] - b);
  const int m = nev ? nev[i] : 0;
  int run = 0;
  for (int base = 0; base < n; base += blockDim.x) {
    const int r = base + t;
    const int f = r < n ? (int)om_int[b + r] : 0;
    int incl = f;
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    __syncthreads();
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    int off = 0, tot = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      if (q < wv) off += wtot[q];
      tot += wtot[q];
    }
    if (r < n) {
      const int q = run + off + incl - 1;
      for (int c = 0; c < nz; ++c)
        Z[(b + r) * nz + c] = (f && c < m) ? (float)W[W_off[i] + (int64_t)q * m + c] : 0.0f;
    }
    run += tot;
  }
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
void dense(hipStream_t st, int64_t n, const float* X1, int ld1, int I1, const uint16_t* W1, int so1,
           int si1, const float* X2, int ld2, int I2, const uint16_t* W2, int so2, int si2,
           const uint16_t* bias, int O, int mode, float* Y, int ldy, float* U) {
  const unsigned nb = (unsigned)((n + DR - 1) / DR);
  ADS_LAUNCH(k_gnn_dense, dim3(nb), dim3(DT), 0, st, (int)n, X1, ld1, I1, W1, so1, si1, X2, ld2, I2,
             W2, so2, si2, bias, O, mode, Y, ldy, U);
}

void agg(hipStream_t st, const ads_gnn_graph& g, const float* H, int width, float* A, int acc) {
  ADS_LAUNCH(k_gnn_agg, dim3((unsigned)((g.nnode + 3) / 4)), dim3(256), 0, st, g.nnode, g.row_ptr,
             g.col, g.w, H, width, A, acc);
}

// grad[gw..] += P^T Q, grad[gb..] += column sums of P (gb < 0: none)
void wgrad(hipStream_t st, int64_t n, const float* P, int ldp, int O, const float* Q, int ldq, int I,
           float* part, float* grad, int64_t gw, int64_t gb) {
  const int nblk = (int)((n + RB - 1) / RB);
  const int64_t ps = (int64_t)GW * GW + GW;
  ADS_LAUNCH(k_gnn_wgrad, dim3((unsigned)nblk), dim3(DT), 0, st, n, P, ldp, O, Q, ldq, I,
             gb >= 0 ? 1 : 0, part, ps);
  const int cnt = O * I + (gb >= 0 ? O : 0);
  ADS_LAUNCH(k_gnn_reduce, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, part, ps, nblk,
             O * I, O, grad, gw, gb);
}

struct WsLayout {
  int64_t nw;
  float* H(float* ws, int l) const { return ws + (int64_t)l * nw; }
  float* A(float* ws, int l) const { return ws + (int64_t)(L + 1 + l) * nw; }
  float* U(float* ws, int l) const { return ws + (int64_t)(2 * L + 1 + l) * nw; }
  float* dh(float* ws) const { return ws + (int64_t)(3 * L + 1) * nw; }
  float* du(float* ws) const { return ws + (int64_t)(3 * L + 2) * nw; }
  float* tmp(float* ws) const { return ws + (int64_t)(3 * L + 3) * nw; }
  float* part(float* ws) const { return ws + (int64_t)(3 * L + 4) * nw; }
  int L;
};

WsLayout layout(const ads_gnn_shape& s, int64_t nnode) {
  WsLayout w;
  w.L = s.layers;
  w.nw = nnode * s.width;
  return w;
}

}  // namespace

// ---- network on a context's subdomains (used by the setup) ----
void gnn_forward_impl(const ads_gnn_shape& s, const uint16_t* p, const ads_gnn_graph& g, float* ws,
                      float* X, hipStream_t st) {
  const Off o = offsets(s);
  const WsLayout wl = layout(s, g.nnode);
  const int w = s.width;
  dense(st, g.nnode, g.feat, s.n_in, s.n_in, p + o.w_in, s.n_in, 1, nullptr, 0, 0, nullptr, 0, 0,
        p + o.b_in, w, 0, wl.H(ws, 0), w, nullptr);
  for (int l = 0; l < s.layers; ++l) {
    agg(st, g, wl.H(ws, l), w, wl.A(ws, l), 0);
    dense(st, g.nnode, wl.H(ws, l), w, w, p + o.ws(l), w, 1, wl.A(ws, l), w, w, p + o.wn(l), w, 1,
          p + o.b(l), w, 1, wl.H(ws, l + 1), w, wl.U(ws, l));
  }
  dense(st, g.nnode, wl.H(ws, s.layers), w, w, p + o.w_out, w, 1, nullptr, 0, 0, nullptr, 0, 0,
        nullptr, s.n_out, 0, X, s.n_out, nullptr);
}

void gnn_graph_impl(const Ctx& c, int64_t* node_off, int64_t* row_ptr, int32_t* col, float* w,
                    float* feat, uint8_t* mask, hipStream_t st) {
  Arena mem(st);
  double* dmean = mem.alloc<double>(c.nsub);
  int32_t* err = mem.alloc<int32_t>(1);
  ADS_HIP(hipMemsetAsync(err, 0, 4, st));
  ADS_LAUNCH(k_gnn_diag_mean, dim3(c.nsub), dim3(256), 0, st, c.om_off, c.lptr_off, c.lcol, c.lval,
             dmean, err);
  const int64_t T = c.omega_total;
  ADS_LAUNCH(k_gnn_graph, dim3((unsigned)((T + 256) / 256)), dim3(256), 0, st, T, c.om_sub,
             c.om_off, c.om_int, c.lptr_off, c.lcol, c.lval, c.lsum, c.bw_d, dmean, row_ptr, col, w,
             feat, mask);
  ADS_HIP(hipMemcpyAsync(node_off, c.om_off, (c.nsub + 1) * 8, hipMemcpyDeviceToDevice, st));
  std::vector<int32_t> he;
  download(he, err, 1, st);
  if (he[0]) fail(ADS_ERR_SINGULAR, "a subdomain matrix row has no diagonal entry");
}

int64_t gnn_edges(const Ctx& c) { return c.lnnz - c.omega_total; }

void read_gnn_weights(const char* path, ads_gnn_shape* shape, std::vector<float>* master) {
  if (!path) fail(ADS_ERR_ARG, "warm_start needs gnn_weights_path");
  FILE* f = std::fopen(path, "rb");
  if (!f) fail(ADS_ERR_ARG, std::string("cannot open the weights file ") + path);
  char magic[8] = {0};
  int32_t sh[4] = {0, 0, 0, 0};
  int64_t np = 0;
  const bool head = std::fread(magic, 1, 8, f) == 8 && std::fread(sh, 4, 4, f) == 4 &&
                    std::fread(&np, 8, 1, f) == 1;
  if (!head || std::string(magic, 8) != "ADSGNN01") {
    std::fclose(f);
    fail(ADS_ERR_ARG, "not a weights file (magic ADSGNN01)");
  }
  const ads_gnn_shape s{sh[0], sh[1], sh[2], sh[3]};
  try {
    check_shape(&s);
  } catch (...) {
    std::fclose(f);
    throw;
  }
  if (s.n_in != ADS_GNN_FEATURES || np != offsets(s).total) {
    std::fclose(f);
    fail(ADS_ERR_ARG, "weights file: shape does not match the node features");
  }
  master->assign(np, 0.0f);
  const bool body = std::fread(master->data(), 4, np, f) == (size_t)np;
  std::fclose(f);
  if (!body) fail(ADS_ERR_ARG, "weights file truncated");
  *shape = s;
}

void learned_start(Ctx& c) {
  hipStream_t st = c.stream;
  const ads_gnn_shape s = c.gnn_shape;
  const std::vector<float>& master = c.gnn_master;
  const int64_t np = (int64_t)master.size();
  Arena mem(st);
  float* dm = upload(mem, master.data(), np, st);
  uint16_t* pb = mem.alloc<uint16_t>(np);
  ADS_LAUNCH(k_gnn_round, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np, dm, pb);
  const int64_t nn = c.omega_total, ne = std::max<int64_t>(gnn_edges(c), 1);
  int64_t* node_off = mem.alloc<int64_t>(c.nsub + 1);
  int64_t* row_ptr = mem.alloc<int64_t>(nn + 1);
  int32_t* col = mem.alloc<int32_t>(ne);
  float* w = mem.alloc<float>(ne);
  float* feat = mem.alloc<float>(nn * ADS_GNN_FEATURES);
  uint8_t* mask = mem.alloc<uint8_t>(nn);
  gnn_graph_impl(c, node_off, row_ptr, col, w, feat, mask, st);
  ads_gnn_graph g{c.nsub, nn, node_off, row_ptr, col, w, feat, mask};
  const int64_t nblk = (nn + RB - 1) / RB;
  float* ws = mem.alloc<float>((int64_t)(3 * s.layers + 4) * nn * s.width + nblk * ((int64_t)GW * GW + GW));
  float* X = c.mem.alloc<float>(nn * s.n_out);
  gnn_forward_impl(s, pb, g, ws, X, st);
  ADS_HIP(hipStreamSynchronize(st));
  c.gnn_x = X;
  c.gnn_cols = s.n_out;
  c.gnn_master.clear();
  c.gnn_master.shrink_to_fit();
}

}  // namespace ads

using namespace ads;

namespace {
int gnn_handle(const Error& e) {
  ads::set_last_error(e.msg);
  return e.code;
}
}  // namespace

extern "C" {

int64_t ads_gnn_nparams(const ads_gnn_shape* s) {
  try {
    check_shape(s);
    return offsets(*s).total;
  } catch (const Error& e) {
    gnn_handle(e);
    return -1;
  }
}

int64_t ads_gnn_workspace_floats(const ads_gnn_shape* s, int64_t nnode) {
  try {
    check_shape(s);
    if (nnode < 1) fail(ADS_ERR_ARG, "nnode must be positive");
    const int64_t nblk = (nnode + RB - 1) / RB;
    return (int64_t)(3 * s->layers + 4) * nnode * s->width + nblk * ((int64_t)GW * GW + GW);
  } catch (const Error& e) {
    gnn_handle(e);
    return -1;
  }
}

int ads_gnn_graph_size(const ads_ctx* ctx, int64_t* nnode, int64_t* nedge, int32_t* ngraph) {
  try {
    if (!ctx || !nnode || !nedge || !ngraph) fail(ADS_ERR_ARG, "null argument");
    const Ctx& c = *ctx_of(ctx);
    *nnode = c.omega_total;
    *nedge = gnn_edges(c);
    *ngraph = c.nsub;
    return ADS_OK;
  } catch (const Error& e) {
    return gnn_handle(e);
  }
}

int ads_gnn_graph_build(const ads_ctx* ctx, int64_t* node_off, int64_t* row_ptr, int32_t* col,
                        float* w, float* feat, uint8_t* mask, void* stream) {
  try {
    if (!ctx || !node_off || !row_ptr || !col || !w || !feat || !mask) fail(ADS_ERR_ARG, "null argument");
    const Ctx& c = *ctx_of(ctx);
    gnn_graph_impl(c, node_off, row_ptr, col, w, feat, mask, (hipStream_t)stream);
    return ADS_OK;
  } catch (const Error& e) {
    return gnn_handle(e);
  }
}

int ads_gnn_targets(const ads_ctx* ctx, float* Z, int32_t nz, void* stream) {
  try {
    if (!ctx || !Z) fail(ADS_ERR_ARG, "null argument");
    if (nz < 1 || nz > GO) fail(ADS_ERR_ARG, "nz must be in [1, 16]");
    const Ctx& c = *ctx_of(ctx);
    if (c.n0 <= 0 || !c.W) fail(ADS_ERR_ARG, "the context has no coarse space");
    hipStream_t st = (hipStream_t)stream;
    ADS_LAUNCH(k_gnn_targets, dim3(c.nsub), dim3(256), 0, st, c.om_off, c.om_int, c.nev, c.W_off,
               c.W, nz, Z);
    return ADS_OK;
  } catch (const Error& e) {
    return gnn_handle(e);
  }
}

int ads_gnn_forward(const ads_gnn_shape* s, const uint16_t* params, const ads_gnn_graph* g,
                    float* ws, float* X, void* stream) {
  try {
    check_shape(s);
    check_graph(g, s->n_in);
    if (!params || !ws || !X) fail(ADS_ERR_ARG, "null argument");
    gnn_forward_impl(*s, params, *g, ws, X, (hipStream_t)stream);
    return ADS_OK;
  } catch (const Error& e) {
    return gnn_handle(e);
  }
}

int ads_gnn_loss(const ads_gnn_shape* s, const ads_gnn_graph* g, const float* X, const float* Z,
                 int32_t nz, float* dX, double* loss, void* stream) {
  try {
    check_shape(s);
    check_graph(g, s->n_in);
    if (!X || !Z || !dX || !loss) fail(ADS_ERR_ARG, "null argument");
    if (nz < 1 || nz > GO) fail(ADS_ERR_ARG, "nz must be in [1, 16]");
    hipStream_t st = (hipStream_t)stream;
    Arena mem(st);
    double* gl = mem.alloc<double>(g->ngraph);
    ADS_LAUNCH(k_gnn_loss, dim3((unsigned)g->ngraph), dim3(256), 0, st, g->ngraph, g->node_off,
               g->mask, X, s->n_out, Z, nz, dX, gl);
    ADS_LAUNCH(k_gnn_loss_sum, dim3(1), dim3(64), 0, st, g->ngraph, gl, loss);
    return ADS_OK;
  } catch (const Error& e) {
    return gnn_handle(e);
  }
}

int ads_gnn_backward(const ads_gnn_shape* s, const uint16_t* p, const ads_gnn_graph* g,
                     float* ws, const float* dX, float* grad, void* stream) {
  try {
    check_shape(s);
    check_graph(g, s->n_in);
    if (!p || !ws || !dX || !grad) fail(ADS_ERR_ARG, "null argument");
    hipStream_t st = (hipStream_t)stream;
    const Off o = offsets(*s);
    const WsLayout wl = layout(*s, g->nnode);
    const int w = s->width, L = s->layers, k = s->n_out;
    const int64_t n = g->nnode;
    float* dh = wl.dh(ws);
    float* du = wl.du(ws);
    float* tmp = wl.tmp(ws);
    float* part = wl.part(ws);
    // output layer: dh = dX W_out, grad W_out += dX^T h_L
    dense(st, n, dX, k, k, p + o.w_out, 1, w, nullptr, 0, 0, nullptr, 0, 0, nullptr, w, 0, dh, w,
          nullptr);
    wgrad(st, n, dX, k, k, wl.H(ws, L), w, w, part, grad, o.w_out, -1);
    for (int l = L - 1; l >= 0; --l) {
      const int64_t cnt = n * w;
      ADS_LAUNCH(k_gnn_relu_mask, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, cnt, dh,
                 wl.U(ws, l), du);
      wgrad(st, n, du, w, w, wl.H(ws, l), w, w, part, grad, o.ws(l), o.b(l));
      wgrad(st, n, du, w, w, wl.A(ws, l), w, w, part, grad, o.wn(l), -1);
      // tmp = du W_n; dh += du W_s + A_w tmp
      dense(st, n, du, w, w, p + o.wn(l), 1, w, nullptr, 0, 0, nullptr, 0, 0, nullptr, w, 0, tmp, w,
            nullptr);
      dense(st, n, du, w, w, p + o.ws(l), 1, w, nullptr, 0, 0, nullptr, 0, 0, nullptr, w, 2, dh, w,
            nullptr);
      agg(st, *g, tmp, w, dh, 1);
    }
    wgrad(st, n, dh, w, w, g->feat, s->n_in, s->n_in, part, grad, o.w_in, o.b_in);
    return ADS_OK;
  } catch (const Error& e) {
    return gnn_handle(e);
  }
}

int ads_gnn_adam(int64_t np, float* master, uint16_t* params, const float* grad, float* m, float* v,
                 int32_t step, float lr, float beta1, float beta2, float eps, void* stream) {
  try {
    if (np < 1 || !master || !params || !grad || !m || !v || step < 1)
      fail(ADS_ERR_ARG, "bad Adam arguments");
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    ADS_LAUNCH(k_gnn_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, (hipStream_t)stream, np,
               master, params, grad, m, v, lr, beta1, beta2, eps, c1, c2);
    return ADS_OK;
  } catch (const Error& e) {
    return gnn_handle(e);
  }
}

int ads_gnn_round_bf16(int64_t np, const float* master, uint16_t* params, void* stream) {
  try {
    if (np < 1 || !master || !params) fail(ADS_ERR_ARG, "null argument");
    ADS_LAUNCH(k_gnn_round, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
               np, master, params);
    return ADS_OK;
  } catch (const Error& e) {
    return gnn_handle(e);
  }
}

}  // extern "C"
