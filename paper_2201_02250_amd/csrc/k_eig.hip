// Local generalized eigenproblems, eq. 5 of Section 3.2, and the coarse space
// of eq. 6.
//
// Per subdomain (Boolean D: B = D A_ii D = A_ii restricted to interior rows and
// columns; Pi = orthogonal projector onto range(splitting)):
//   non-floating (K = {0}):     T x = Atilde^{-1} B x
//   floating (K = span{1}):     T x = P_perp Atilde_reg^{-1} Pi B Pi x,
//     P_perp = projector onto 1^perp, Atilde_reg = splitting with doubled last
//     diagonal entry, Pi = I - l l^T with l the unit left null vector.
// The nonzero eigenpairs of T are the eigenpairs of eq. 5 on K^perp.
//
// Two methods, all subdomains batched in the same launches:
//  * block Krylov-Schur (default; block width 4): expansion steps through the
//    two-ended operator kernels k_eig_op_fwd / k_eig_op_bwd (or k_eig_op on
//    the general path), block Gram-Schmidt twice with a QR of the block after
//    each pass (k_ks_dots, k_ks_upd, k_ks_qr), restarts from the ordered Schur
//    form of the Rayleigh quotient (k_ks_rr, k_ks_restart);
//  * block subspace iteration (k_eig_op, k_eig_gram, k_eig_orth) with
//    Rayleigh-Ritz steps on a predicted schedule (k_eig_rr, k_eig_resid,
//    k_eig_decide).
// Both use small_eig_select: the Schur form of a real matrix of order <= 32
// in LDS by one wave (Householder Hessenberg reduction, Francis double-shift
// QR, complex triangularisation of the 2 x 2 blocks), eigenvalues ordered by
// |lambda|, the cut of eq. 6 with the cluster rule, Givens reordering so that
// the selected (and the kept) eigenvalues lead, real orthonormal bases of the
// selected (and kept) invariant subspaces.
//   k_eig_finish  W_i = orth([1 | (X V) restricted to Omega_Ii])
// Converged subdomains skip further work.
#include <algorithm>
#include <cmath>

#include "ads_internal.h"
#include "k_solve.h"

namespace ads {

static constexpr int EIG_T = 1024;
static constexpr int PMAX = 32;
static constexpr int EIG_PC = 4;  // columns per workgroup of the operator kernel
// block Krylov-Schur: block width EIG_PC, at most PMAX + EIG_PC basis vectors
static constexpr int KS_W = PMAX + EIG_PC;
static constexpr int KS_PK = KS_W * EIG_PC;  // partial V^T W per row block
static constexpr int KS_BS = KS_W * PMAX;    // Bk per subdomain
static constexpr int VSEL = KS_W * KS_W;     // Vsel per subdomain

static constexpr double CLUSTER_RTOL = 1e-6;
// sweep budget of a warm-started subspace iteration before the cold fallback
static constexpr int WARM_SWEEPS = 150;

#define WAVE_SYNC()                                        \
  do {                                                     \
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); \
    __builtin_amdgcn_wave_barrier();                       \
  } while (0)

struct cd {
  double x, y;
};
__device__ __forceinline__ cd cmk(double a, double b) { return cd{a, b}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd cconj(cd a) { return cd{a.x, -a.y}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return cd{a.x * s, a.y * s}; }
__device__ __forceinline__ double cabs2(cd a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double cabs(cd a) { return hypot(a.x, a.y); }
__device__ __forceinline__ double cnorm1(cd a) { return fabs(a.x) + fabs(a.y); }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
  double d = cabs2(b);
  return cd{(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
__device__ __forceinline__ cd csqrt(cd a) {
  double r = cabs(a);
  if (r == 0.0) return cd{0.0, 0.0};
  double sx = sqrt(0.5 * (r + fabs(a.x)));
  double sy = 0.5 * a.y / sx;
  if (a.x >= 0) return cd{sx, sy};
  return cd{fabs(sy), a.y >= 0 ? sx : -sx};
}

// Givens rotation G = [c s; -conj(s) c] (c real) with G [x; y] = [r; 0]
__device__ __forceinline__ void cgivens(cd x, cd y, double& c, cd& s) {
  double ax = cabs(x), ay = cabs(y);
  if (ay == 0.0) {
    c = 1.0;
    s = cd{0, 0};
    return;
  }
  if (ax == 0.0) {
    c = 0.0;
    s = cscale(cconj(y), 1.0 / ay);
    return;
  }
  double r = hypot(ax, ay);
  c = ax / r;
  s = cscale(cmul(cscale(x, 1.0 / ax), cconj(y)), 1.0 / r);
}

struct SmallEigLds {
  cd A[PMAX * (PMAX + 1)];  // complex Schur form, row-major, leading dimension p | 1
  cd Q[PMAX * (PMAX + 1)];  // Schur vectors, same layout
  cd v[PMAX];
  double Pm[PMAX * (PMAX + 1)];
  double V[PMAX * (PMAX + 1)];  // real basis, column-major p x m (leading dimension p)
  double mag[PMAX];
  double rv[PMAX];
  int rank[PMAX];
  int selected[PMAX];
  double red[64];
};

// Complex Schur form of the real p x p matrix H (row-major) by wave 0 only.
// Returns the number of selected eigenvalues m (leading after reordering),
// their eigenvalues in |lambda| order in lam_out[0..m), and V (p x m real
// orthonormal basis of the selected invariant subspace).  ok = 0 on failure.
__device__ int small_eig_select(int p, const double* H, int count, double tau, SmallEigLds& L,
                                double* lam_re, double* lam_im, int* ok_out, double* cut_gap,
                                int count2 = 0, int* m2_out = nullptr, double* V2 = nullptr,
                                int pair = 0) {
  const int lane = threadIdx.x;  // wave 0 only
  // leading dimension of the work matrices: odd, so that a column access by
  // the lanes of a wave spreads over the LDS banks
  const int ld = p | 1;
  cd* A = L.A;
  cd* Q = L.Q;
  // real arithmetic first: T (in L.Pm) and Z (in L.V), both row-major
  double* T = L.Pm;
  double* Z = L.V;
  const double eps = 2.220446049250313e-16;
  double anorm = 0.0;
  for (int e = lane; e < p * p; e += 64) {
    const int r = e / p, c = e % p;
    T[r * ld + c] = H[e];
    Z[r * ld + c] = (r == c) ? 1.0 : 0.0;
    anorm = fmax(anorm, fabs(H[e]));
  }
  for (int o = 32; o > 0; o >>= 1) anorm = fmax(anorm, __shfl_xor(anorm, o, 64));
  if (!(anorm > 0.0)) anorm = 1.0;
  WAVE_SYNC();
  // Householder reduction to upper Hessenberg form, T <- P T P, Z <- Z P
  for (int k = 0; k + 2 < p; ++k) {
    const int len = p - k - 1;
    const double x = (lane < len) ? T[(k + 1 + lane) * ld + k] : 0.0;
    const double nx = sqrt(adsd::wave_sum(x * x));
    if (nx == 0.0) continue;
    const double x0 = T[(k + 1) * ld + k];
    const double beta = x0 > 0.0 ? -nx : nx;
    const double vl = (lane == 0) ? x - beta : x;
    const double vn2 = adsd::wave_sum(vl * vl);
    if (vn2 == 0.0) continue;
    const double tau = 2.0 / vn2;
    if (lane < len) L.rv[lane] = vl;
    WAVE_SYNC();
    if (lane < p && lane >= k) {  // rows k+1.., column lane
      const int j = lane;
      double w = 0.0;
      for (int l = 0; l < len; ++l) w += L.rv[l] * T[(k + 1 + l) * ld + j];
      w *= tau;
      for (int l = 0; l < len; ++l) T[(k + 1 + l) * ld + j] -= L.rv[l] * w;
    }
    WAVE_SYNC();
    {  // columns k+1..: rows of T (lanes 0..31) and of Z (lanes 32..63)
      double* M = lane < 32 ? T : Z;
      const int i = lane & 31;
      if (i < p) {
        double w = 0.0;
        for (int l = 0; l < len; ++l) w += M[i * ld + k + 1 + l] * L.rv[l];
        w *= tau;
        for (int l = 0; l < len; ++l) M[i * ld + k + 1 + l] -= w * L.rv[l];
      }
    }
    WAVE_SYNC();
    if (lane < len) T[(k + 1 + lane) * ld + k] = (lane == 0) ? beta : 0.0;
    WAVE_SYNC();
  }
  // Francis double-shift QR to real Schur form (1x1 and 2x2 diagonal
  // blocks), T <- Z^T H Z
  int hi = p - 1, its = 0, total = 0, ok = 1, l = 0;
  while (hi >= 1) {
    // window start l: the last negligible subdiagonal entry at or above hi
    // (normwise test: only the largest |lambda| matter); one lane per row
    const double subl = (lane >= 1 && lane <= hi) ? fabs(T[lane * ld + lane - 1]) : 0.0;
    {
      const bool neg = lane >= 1 && lane <= hi &&
                       subl <= eps * fmax(fabs(T[(lane - 1) * ld + lane - 1]) + fabs(T[lane * ld + lane]), anorm);
      const unsigned long long bm = __ballot(neg);
      l = bm ? 63 - __clzll(bm) : 0;
    }
    WAVE_SYNC();
    if (l > 0 && lane == 0) T[l * ld + l - 1] = 0.0;
    WAVE_SYNC();
    if (l < hi - 1 && its >= 20) {
      // stagnation on a tight cluster: split the window at its smallest
      // subdiagonal entry if that is at the rounding level of the matrix
      double bv = (lane > l && lane <= hi) ? subl : 1e300;
      int kb = lane;
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int ok2 = __shfl_xor(kb, o, 64);
        if (ov < bv || (ov == bv && ok2 < kb)) {
          bv = ov;
          kb = ok2;
        }
      }
      if (bv <= 1e3 * eps * anorm) {
        WAVE_SYNC();
        if (lane == 0) T[kb * ld + kb - 1] = 0.0;
        WAVE_SYNC();
        its = 0;
        continue;
      }
    }
    if (l >= hi - 1) {  // a 1x1 or 2x2 block has split off
      hi = l - 1;
      its = 0;
      continue;
    }
    if (++total > 60 * p) {
      ok = 0;
      break;
    }
    ++its;
    // the two shifts r1, r2: the eigenvalues of the trailing 2 x 2 block if
    // complex, else twice the one nearer to its last diagonal entry;
    // exceptional shifts every tenth iteration
    double r1r, r1i, r2r, r2i;
    if (its % 10 == 0) {
      const double w = fabs(T[hi * ld + hi - 1]) + fabs(T[(hi - 1) * ld + hi - 2]);
      r1r = r2r = 0.75 * w + T[hi * ld + hi];
      r1i = 0.6614378277661477 * w;  // sqrt(0.4375) w
      r2i = -r1i;
    } else {
      const double a = T[(hi - 1) * ld + hi - 1], b = T[(hi - 1) * ld + hi];
      const double c = T[hi * ld + hi - 1], d = T[hi * ld + hi];
      const double pp = 0.5 * (a - d), q = pp * pp + b * c;
      if (q >= 0.0) {
        const double e1 = d + pp + copysign(sqrt(q), pp);
        const double e2 = e1 != 0.0 ? (a * d - b * c) / e1 : d + pp - copysign(sqrt(q), pp);
        r1r = r2r = fabs(e1 - d) <= fabs(e2 - d) ? e1 : e2;
        r1i = r2i = 0.0;
      } else {
        r1r = r2r = d + pp;
        r1i = sqrt(-q);
        r2i = -r1i;
      }
    }
    // first column of (T - s1)(T - s2) at the start row mm: the lowest row
    // (>= l) where the bulge it creates is negligible against h(mm, mm-1), so
    // two consecutive small subdiagonal entries do not stall the iteration
    // (one lane per candidate row, the highest acceptable one is taken)
    int mm;
    double x, y, z;
    {
      const int c = lane;  // candidate start row
      const bool cand = c >= l && c <= hi - 2;
      double cx = 0.0, cy = 0.0, cz = 0.0;
      bool good = false;
      if (cand) {
        const double h00 = T[c * ld + c], h01 = T[c * ld + c + 1], h10 = T[(c + 1) * ld + c];
        const double h11 = T[(c + 1) * ld + c + 1], h21 = T[(c + 2) * ld + c + 1];
        // (h00 - r1)(h00 - r2) in factored form (no cancellation of h00^2
        // against the shift terms), scaled
        double s0 = fabs(h00 - r2r) + fabs(r2i) + fabs(h10);
        if (s0 == 0.0) s0 = 1.0;
        const double h10s = h10 / s0;
        cx = h10s * h01 + (h00 - r1r) * ((h00 - r2r) / s0) - r1i * (r2i / s0);
        cy = h10s * (h00 + h11 - r1r - r2r);
        cz = h10s * h21;
        const double sc = fabs(cx) + fabs(cy) + fabs(cz);
        if (sc > 0.0) {
          cx /= sc;
          cy /= sc;
          cz /= sc;
        }
        if (c == l) {
          good = true;
        } else {
          const double e1 = fabs(T[c * ld + c - 1]) * (fabs(cy) + fabs(cz));
          const double e2 = fabs(cx) * (fabs(T[(c - 1) * ld + c - 1]) + fabs(h00) + fabs(h11));
          good = e1 <= eps * e2;
        }
      }
      const unsigned long long bm = __ballot(good);
      mm = 63 - __clzll(bm);  // lane l is always good
      x = __shfl(cx, mm, 64);
      y = __shfl(cy, mm, 64);
      z = __shfl(cz, mm, 64);
    }
    for (int k = mm; k < hi; ++k) {
      const bool three = k < hi - 1;
      if (k > mm) {
        x = T[k * ld + k - 1];
        y = T[(k + 1) * ld + k - 1];
        z = three ? T[(k + 2) * ld + k - 1] : 0.0;
      }
      const double al = sqrt(x * x + y * y + z * z);
      if (al == 0.0) continue;
      const double beta = x > 0.0 ? -al : al;
      const double v0 = x - beta, v1 = y, v2 = z;
      const double tau = 2.0 / (v0 * v0 + v1 * v1 + v2 * v2);
      WAVE_SYNC();
      const int cmin = k > mm ? k - 1 : k;
      if (lane >= cmin && lane < p) {  // rows k..k+2
        const int j = lane;
        double w = v0 * T[k * ld + j] + v1 * T[(k + 1) * ld + j];
        if (three) w += v2 * T[(k + 2) * ld + j];
        w *= tau;
        T[k * ld + j] -= v0 * w;
        T[(k + 1) * ld + j] -= v1 * w;
        if (three) T[(k + 2) * ld + j] -= v2 * w;
      }
      WAVE_SYNC();
      {  // columns k..k+2: rows of T up to min(k+3, hi) and all rows of Z
        double* M = lane < 32 ? T : Z;
        const int i = lane & 31;
        const int imax = lane < 32 ? min(k + 3, hi) : p - 1;
        if (i <= imax) {
          double w = M[i * ld + k] * v0 + M[i * ld + k + 1] * v1;
          if (three) w += M[i * ld + k + 2] * v2;
          w *= tau;
          M[i * ld + k] -= w * v0;
          M[i * ld + k + 1] -= w * v1;
          if (three) M[i * ld + k + 2] -= w * v2;
        }
      }
      WAVE_SYNC();
      if (lane == 0) {
        if (k > mm) {
          T[k * ld + k - 1] = beta;
          T[(k + 1) * ld + k - 1] = 0.0;
          if (three) T[(k + 2) * ld + k - 1] = 0.0;
        } else if (mm > l) {
          // the reflector's effect on the small h(mm, mm-1); its fill below
          // is negligible by the choice of mm
          T[k * ld + k - 1] *= 1.0 - tau * v0 * v0;
        }
      }
      WAVE_SYNC();
    }
  }
  // complex Schur form: each remaining 2x2 block [a b; c d] is triangularised
  // by the unitary G = [u, (-u2, conj(u1))] with u the unit eigenvector
  // (lambda - d, c) of one of its eigenvalues
  for (int e = lane; e < p * ld; e += 64) {
    A[e] = cd{T[e], 0.0};
    Q[e] = cd{Z[e], 0.0};
  }
  WAVE_SYNC();
  for (int k = 0; k + 1 < p;) {
    const double c = T[(k + 1) * ld + k];
    if (c == 0.0) {
      ++k;
      continue;
    }
    const double a = T[k * ld + k], b = T[k * ld + k + 1], d = T[(k + 1) * ld + k + 1];
    const double pp = 0.5 * (a - d), q = pp * pp + b * c;
    cd x1;
    if (q >= 0.0)
      x1 = cd{pp + copysign(sqrt(q), pp), 0.0};
    else
      x1 = cd{pp, sqrt(-q)};
    const double nrm = sqrt(cabs2(x1) + c * c);
    const cd u1 = cscale(x1, 1.0 / nrm);
    const double u2 = c / nrm;
    WAVE_SYNC();
    if (lane < p && lane >= k) {  // rows k, k+1 <- G^H rows
      const int j = lane;
      const cd r0 = A[k * ld + j], r1 = A[(k + 1) * ld + j];
      A[k * ld + j] = cadd(cmul(cconj(u1), r0), cscale(r1, u2));
      A[(k + 1) * ld + j] = csub(cmul(u1, r1), cscale(r0, u2));
    }
    WAVE_SYNC();
    {  // columns k, k+1 <- columns G: A rows up to k+1 (lanes 0..31), Q (lanes 32..63)
      cd* M = lane < 32 ? A : Q;
      const int i = lane & 31;
      const int imax = lane < 32 ? k + 1 : p - 1;
      if (i <= imax) {
        const cd c0 = M[i * ld + k], c1 = M[i * ld + k + 1];
        M[i * ld + k] = cadd(cmul(c0, u1), cscale(c1, u2));
        M[i * ld + k + 1] = csub(cmul(c1, cconj(u1)), cscale(c0, u2));
      }
    }
    WAVE_SYNC();
    if (lane == 0) A[(k + 1) * ld + k] = cd{0.0, 0.0};
    WAVE_SYNC();
    k += 2;
  }
  *ok_out = ok;
  WAVE_SYNC();
  // ranks by |lambda| descending (ties by index)
  if (lane < p) L.mag[lane] = cabs(A[lane * ld + lane]);
  WAVE_SYNC();
  if (lane < p) {
    int rk = 0;
    double mk = L.mag[lane];
    for (int j = 0; j < p; ++j) {
      double mj = L.mag[j];
      rk += (mj > mk) || (mj == mk && j < lane);
    }
    L.rank[lane] = rk;
  }
  WAVE_SYNC();
  // selection: the count largest, extended by the cluster rule, optional tau.
  // A second, larger cut (count2, cluster rule only) marks the set kept for a
  // restart; the wanted set is a prefix of it in |lambda| order.
  int m = 0, mk = 0;
  double cut = 0.0, next = 0.0, cut2 = 0.0;
  const int ck = count2 > count ? count2 : count;
  if (count > 0)
    for (int j = 0; j < p; ++j)
      if (L.rank[j] == count - 1) cut = L.mag[j];
  if (ck > 0)
    for (int j = 0; j < p; ++j)
      if (L.rank[j] == ck - 1) cut2 = L.mag[j];
  for (int j = 0; j < p; ++j) {
    bool sel = count > 0 && L.mag[j] >= (1.0 - CLUSTER_RTOL) * cut;
    if (tau > 0 && !(L.mag[j] > 1.0 / tau)) sel = false;
    const bool keep = sel || (ck > 0 && L.mag[j] >= (1.0 - CLUSTER_RTOL) * cut2);
    if (lane == 0) L.selected[j] = keep;
    m += sel;
    mk += keep;
    if (count > 0 && !(L.mag[j] >= (1.0 - CLUSTER_RTOL) * cut)) next = fmax(next, L.mag[j]);
  }
  if (pair) {
    // the real form of a complex matrix: every eigenvalue has even
    // multiplicity (mu with conj(mu), a real mu twice), and both sets are
    // prefixes in |lambda| order, so a count left odd by rounding takes the
    // next eigenvalue, the partner
    if ((m & 1) && m < p) ++m;
    if (mk < m) mk = m;
    if ((mk & 1) && mk < p) ++mk;
    if (lane == 0)
      for (int j = 0; j < p; ++j) L.selected[j] = L.rank[j] < mk;
  }
  *cut_gap = (cut > 0) ? (cut - next) / cut : 1.0;
  if (m2_out) *m2_out = mk;
  WAVE_SYNC();
  // reorder: move selected eigenvalues (in rank order) to the leading positions
  for (int tpos = 0; tpos < mk; ++tpos) {
    // find the selected entry with the smallest rank at positions >= tpos
    int idx = -1, best = 1 << 30;
    for (int j = tpos; j < p; ++j)
      if (L.selected[j] && L.rank[j] < best) {
        best = L.rank[j];
        idx = j;
      }
    for (int k = idx - 1; k >= tpos; --k) {
      cd t11 = A[k * ld + k], t22 = A[(k + 1) * ld + k + 1], t12 = A[k * ld + k + 1];
      cd x = t12, y = csub(t22, t11);
      double cg;
      cd sg;
      cgivens(x, y, cg, sg);
      WAVE_SYNC();
      if (lane < p && lane >= k) {
        const int j = lane;
        cd a1 = A[k * ld + j], a2 = A[(k + 1) * ld + j];
        A[k * ld + j] = cadd(cscale(a1, cg), cmul(sg, a2));
        A[(k + 1) * ld + j] = csub(cscale(a2, cg), cmul(cconj(sg), a1));
      }
      WAVE_SYNC();
      if (lane < p) {
        const int i = lane;
        if (i <= k + 1) {
          cd b1 = A[i * ld + k], b2 = A[i * ld + k + 1];
          A[i * ld + k] = cadd(cscale(b1, cg), cmul(cconj(sg), b2));
          A[i * ld + k + 1] = csub(cscale(b2, cg), cmul(sg, b1));
        }
        cd q1 = Q[i * ld + k], q2 = Q[i * ld + k + 1];
        Q[i * ld + k] = cadd(cscale(q1, cg), cmul(cconj(sg), q2));
        Q[i * ld + k + 1] = csub(cscale(q2, cg), cmul(sg, q1));
      }
      WAVE_SYNC();
      if (lane == 0) {
        A[k * ld + k] = t22;
        A[(k + 1) * ld + k + 1] = t11;
        A[(k + 1) * ld + k] = cd{0, 0};
        int r0 = L.rank[k], s0 = L.selected[k];
        L.rank[k] = L.rank[k + 1];
        L.selected[k] = L.selected[k + 1];
        L.rank[k + 1] = r0;
        L.selected[k + 1] = s0;
      }
      WAVE_SYNC();
    }
  }
  if (lane < m) {
    lam_re[lane] = A[lane * ld + lane].x;
    lam_im[lane] = A[lane * ld + lane].y;
  }
  // real bases of span(Q[:, 0:m]) (into L.V) and of span(Q[:, 0:mk]) (into
  // V2): the projector Q_b Q_b^H is real for a conjugation-closed selection;
  // pivoted Gram-Schmidt on its columns, then classical Gram-Schmidt twice of
  // each new column against the earlier ones (numerical safety).  Two lanes
  // per column (j = lane & 31): each takes half of the rows, joined by one
  // butterfly step.
  const int jl = lane & 31, hf = lane >> 5;
  const int ih = (p + 1) >> 1;
  const int i0 = hf ? ih : 0, i1 = hf ? p : ih;
  for (int which = 0; which < (V2 ? 2 : 1); ++which) {
    const int mb = which ? mk : m;
    double* VV = which ? V2 : L.V;
    double* P = L.Pm;
    if (jl < p) {
      for (int i = i0; i < i1; ++i) {
        double acc = 0.0;
        for (int t = 0; t < mb; ++t) acc += cmul(Q[i * ld + t], cconj(Q[jl * ld + t])).x;
        P[i * ld + jl] = acc;  // column jl of the projector
      }
    }
    WAVE_SYNC();
    for (int t = 0; t < mb; ++t) {
      double nrm = 0.0;
      if (jl < p)
        for (int i = i0; i < i1; ++i) nrm += P[i * ld + jl] * P[i * ld + jl];
      nrm += __shfl_xor(nrm, 32, 64);
      // argmax over the columns (ties -> smallest index)
      double bn = (jl < p && hf == 0) ? nrm : -1.0;
      int bj = (jl < p && hf == 0) ? jl : 1 << 30;
      for (int o = 32; o > 0; o >>= 1) {
        double on = __shfl_xor(bn, o, 64);
        int oj = __shfl_xor(bj, o, 64);
        if (on > bn || (on == bn && oj < bj)) {
          bn = on;
          bj = oj;
        }
      }
      double inv = bn > 0 ? 1.0 / sqrt(bn) : 0.0;
      if (lane < p) VV[t * p + lane] = P[lane * ld + bj] * inv;
      WAVE_SYNC();
      for (int pass = 0; pass < 2; ++pass) {
        double d = 0.0;
        if (jl < p)
          for (int i = i0; i < i1; ++i) d += VV[t * p + i] * P[i * ld + jl];
        d += __shfl_xor(d, 32, 64);
        if (jl < p)
          for (int i = i0; i < i1; ++i) P[i * ld + jl] -= d * VV[t * p + i];
        WAVE_SYNC();
      }
      if (t > 0) {
        for (int pass = 0; pass < 2; ++pass) {
          // coefficients against the earlier columns, column u = jl
          double d = 0.0;
          if (jl < t)
            for (int i = i0; i < i1; ++i) d += VV[jl * p + i] * VV[t * p + i];
          d += __shfl_xor(d, 32, 64);
          if (lane < t) L.rv[lane] = d;
          WAVE_SYNC();
          if (lane < p) {
            double v = VV[t * p + lane];
            for (int u = 0; u < t; ++u) v -= L.rv[u] * VV[u * p + lane];
            VV[t * p + lane] = v;
          }
          WAVE_SYNC();
        }
        const double vt = lane < p ? VV[t * p + lane] : 0.0;
        const double nn = sqrt(adsd::wave_sum(vt * vt));
        if (lane < p) VV[t * p + lane] = nn > 0 ? vt / nn : 0.0;
        WAVE_SYNC();
      }
    }
  }
  return m;
}

// ---------------------------------------------------------------------------
// block helpers: Gram matrices over rows, Cholesky QR
// ---------------------------------------------------------------------------
// Row passes over an n x p block stage CR rows at a time in LDS, with
// CR * p <= GBUF: 4096 entries per buffer, GNPT per thread.  The next chunk is
// loaded into registers while the current one is processed.
static constexpr int GBUF = 4096;
static constexpr int GNPT = GBUF / EIG_T;

// Chunk geometry: CR rows (a power of two, CR * p <= GBUF); staged entry
// e = t + k * EIG_T of a chunk is row e & (CR - 1), column e >> lcr.
struct ChunkMap {
  int CR, lcr, LDB;
  __device__ ChunkMap(int p) {
    lcr = 31 - __clz(GBUF / p);
    CR = 1 << lcr;
    LDB = CR + 1;
  }
  __device__ int rr(int e) const { return e & (CR - 1); }
  __device__ int cc(int e) const { return e >> lcr; }
};

// body(r0, rows) runs once per chunk with rows [r0, r0 + rows) of U (and V if
// TWO) staged column-major in bufU (bufV), leading dimension cm.LDB
template <bool TWO, class Body>
__device__ __forceinline__ void chunk_pass(const ChunkMap& cm, const double* U, const double* V,
                                           int64_t ld, int n, int p, double* bufU, double* bufV,
                                           Body&& body) {
  double ru[GNPT], rv[GNPT];
  const int t = threadIdx.x;
  auto load = [&](int r0) {
    const int rows = min(cm.CR, n - r0);
#pragma unroll
    for (int k = 0; k < GNPT; ++k) {
      const int e = t + k * EIG_T, rr = cm.rr(e), cc = cm.cc(e);
      const bool ok = cc < p && rr < rows;
      const int64_t idx = ok ? (int64_t)r0 + rr + cc * ld : 0;  // clamped, branch-free
      const double u = U[idx];
      ru[k] = ok ? u : 0.0;
      if (TWO) {
        const double v = V[idx];
        rv[k] = ok ? v : 0.0;
      }
    }
  };
  if (n > 0) load(0);
  for (int r0 = 0; r0 < n; r0 += cm.CR) {
    const int rows = min(cm.CR, n - r0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GNPT; ++k) {
      const int e = t + k * EIG_T, rr = cm.rr(e), cc = cm.cc(e);
      if (cc < p) {
        bufU[rr + cc * cm.LDB] = ru[k];
        if (TWO) bufV[rr + cc * cm.LDB] = rv[k];
      }
    }
    __syncthreads();
    if (r0 + cm.CR < n) load(r0 + cm.CR);
    body(r0, rows);
  }
  __syncthreads();
}

// thread -> Gram entry map: TPE threads share an entry (partial sums joined
// by shuffles)
struct GramMap {
  int tpe, ent, sub, a, b;
  bool own;
  __device__ GramMap(int p) {
    const int t = threadIdx.x;
    tpe = EIG_T / (p * p);
    tpe = tpe >= 4 ? 4 : (tpe >= 2 ? 2 : 1);
    ent = t / tpe;
    sub = t % tpe;
    own = ent < p * p;
    a = ent / p;
    b = ent % p;
  }
  __device__ double join(double v) const {
    if (tpe >= 2) v += __shfl_xor(v, 1, 64);
    if (tpe >= 4) v += __shfl_xor(v, 2, 64);
    return v;
  }
};

// H[a*p+b] = sum_r U[r,a] V[r,b] and, if G != nullptr, G[a*p+b] = sum_r V[r,a] V[r,b]
// over r < n
__device__ __forceinline__ void gram2(const double* U, const double* V, int64_t ld, int n, int p, double* H,
                      double* G, double* bufU, double* bufV) {
  const GramMap gm(p);
  const ChunkMap cm(p);
  const int LDB = cm.LDB;
  double accH = 0.0, accG = 0.0;
  chunk_pass<true>(cm, U, V, ld, n, p, bufU, bufV, [&](int, int rows) {
    if (gm.own)
#pragma unroll 4
      for (int rr = gm.sub; rr < rows; rr += gm.tpe) {
        const double vb = bufV[rr + gm.b * LDB];
        accH += bufU[rr + gm.a * LDB] * vb;
        if (G) accG += bufV[rr + gm.a * LDB] * vb;
      }
  });
  accH = gm.join(accH);
  accG = gm.join(accG);
  if (gm.own && gm.sub == 0) {
    H[gm.ent] = accH;
    if (G) G[gm.ent] = accG;
  }
  __syncthreads();
}

// G = Y^T Y over rows < n
__device__ __forceinline__ void gram(const double* Y, int64_t ld, int n, int p, double* G, double* bufU) {
  const GramMap gm(p);
  const ChunkMap cm(p);
  const int LDB = cm.LDB;
  double acc = 0.0;
  chunk_pass<false>(cm, Y, nullptr, ld, n, p, bufU, nullptr, [&](int, int rows) {
    if (gm.own)
#pragma unroll 4
      for (int rr = gm.sub; rr < rows; rr += gm.tpe)
        acc += bufU[rr + gm.a * LDB] * bufU[rr + gm.b * LDB];
  });
  acc = gm.join(acc);
  if (gm.own && gm.sub == 0) G[gm.ent] = acc;
  __syncthreads();
}

// Xout = Yin Rinv over rows r < n (zero on rows n..npad-1) with Rinv upper
// triangular (row-major p x p); if G != nullptr also G = Xout^T Xout.  Xout
// may alias Yin (each chunk is staged before it is overwritten).
__device__ __forceinline__ void right_mul_upper(const double* Yin, double* Xout, int64_t ld, int n, int npad, int p,
                                const double* Rinv, double* G, double* bufU, double* bufV) {
  const int t = threadIdx.x;
  const GramMap gm(p);
  const ChunkMap cm(p);
  const int LDB = cm.LDB;
  double acc = 0.0;
  chunk_pass<false>(cm, Yin, nullptr, ld, n, p, bufU, nullptr, [&](int r0, int rows) {
#pragma unroll 1
    for (int e = t; e < GBUF; e += EIG_T) {
      const int rr = cm.rr(e), a = cm.cc(e);
      if (a >= p || rr >= rows) continue;
      double v = 0.0;
#pragma unroll 4
      for (int b = 0; b <= a; ++b) v += bufU[rr + b * LDB] * Rinv[b * p + a];
      Xout[r0 + rr + a * ld] = v;
      if (G) bufV[rr + a * LDB] = v;
    }
    if (G) {
      __syncthreads();
      if (gm.own)
#pragma unroll 4
        for (int rr = gm.sub; rr < rows; rr += gm.tpe)
          acc += bufV[rr + gm.a * LDB] * bufV[rr + gm.b * LDB];
    }
  });
  for (int e = t; e < (npad - n) * p; e += EIG_T) {
    const int rr = e % (npad - n), a = e / (npad - n);
    Xout[n + rr + a * ld] = 0.0;
  }
  if (G) {
    acc = gm.join(acc);
    if (gm.own && gm.sub == 0) G[gm.ent] = acc;
  }
  __syncthreads();
}

// Cholesky factor R (upper, R^T R = G) of the p x p SPD matrix G (row-major,
// read only) and Rinv = R^{-1} (row-major, upper), by wave 0 with lane j
// holding column j in registers; rows are exchanged by shuffles.  Returns 0
// (on every lane) if G is not numerically positive definite.
template <int PM>
__device__ __forceinline__ int chol_inv_wave_t(const double* G, double* Rinv, int p) {
  const int j = threadIdx.x;
  double g[PM];
#pragma unroll
  for (int i = 0; i < PM; ++i) g[i] = (j < p && i < p) ? G[i * p + j] : 0.0;
  int ok = 1;
#pragma unroll
  for (int k = 0; k < PM; ++k) {
    if (k < p) {
      double d = __shfl(g[k], k, 64);
      if (!(d > 0.0)) {
        ok = 0;
        d = 1e-300;
      }
      const double rkk = sqrt(d);
      g[k] = (j == k) ? rkk : (j > k ? g[k] / rkk : g[k]);  // row k of R
#pragma unroll
      for (int i = k + 1; i < PM; ++i) {
        const double rki = __shfl(g[k], i, 64);
        if (j >= i && i < p) g[i] -= rki * g[k];
      }
    }
  }
  // column j of R^{-1} by back substitution; x_i overwrites g[i] once row i
  // of R has been used
#pragma unroll
  for (int i = PM - 1; i >= 0; --i) {
    const double rii = __shfl(g[i], i, 64);
    double sacc = 0.0;
#pragma unroll
    for (int k = i + 1; k < PM; ++k) {
      const double rik = __shfl(g[i], k, 64);
      if (k <= j && k < p) sacc += rik * g[k];
    }
    if (i < p) g[i] = (j == i) ? 1.0 / rii : (j > i ? -sacc / rii : 0.0);
  }
  if (j < p)
#pragma unroll
    for (int i = 0; i < PM; ++i)
      if (i < p) Rinv[i * p + j] = g[i];
  WAVE_SYNC();
  return ok;
}

// Cholesky of the p x p SPD matrix G in place (upper factor R, row-major,
// R[a*p+b] for b >= a).  Wave 0 only.  Returns 0 if not positive definite.
__device__ __forceinline__ int chol_upper(double* G, int p) {
  const int lane = threadIdx.x;
  int ok = 1;
  for (int k = 0; k < p; ++k) {
    double d = G[k * p + k];
    if (!(d > 0.0)) {
      ok = 0;
      d = 1e-300;
    }
    double rkk = sqrt(d);
    WAVE_SYNC();
    if (lane < p && lane > k) G[k * p + lane] /= rkk;
    if (lane == k) G[k * p + k] = rkk;
    WAVE_SYNC();
    if (lane < p && lane > k) {
      const int j = lane;
      for (int i = k + 1; i <= j; ++i) G[i * p + j] -= G[k * p + i] * G[k * p + j];
    }
    WAVE_SYNC();
  }
  return ok;
}

// Rinv = R^{-1} for the upper triangular R (row-major p x p); wave 0, lane j
// solves column j
__device__ __forceinline__ void tri_inverse(const double* R, double* Rinv, int p) {
  const int j = threadIdx.x;
  if (j < p) {
    for (int i = p - 1; i >= 0; --i) {
      double v = (i == j) ? 1.0 : 0.0;
      for (int k = i + 1; k <= j; ++k) v -= R[i * p + k] * Rinv[k * p + j];
      Rinv[i * p + j] = (i <= j) ? v / R[i * p + i] : 0.0;
    }
  }
  WAVE_SYNC();
}

// R^T R = G and Rinv = R^{-1}: registers for p <= 16, else in LDS (G is
// overwritten then).  Wave 0 only.
__device__ __forceinline__ int chol_inv_wave(double* G, double* Rinv, int p) {
  if (p <= 16) return chol_inv_wave_t<16>(G, Rinv, p);
  const int ok = chol_upper(G, p);
  tri_inverse(G, Rinv, p);
  return ok;
}

struct EigShared {
  double G[PMAX * PMAX];
  double Ri[PMAX * PMAX];
  double bufU[GBUF + PMAX];
  double bufV[GBUF + PMAX];
  double red[16];
  int flag[4];
};

// Cholesky QR twice: X <- orth(Y) over rows < n (Y is overwritten); G0, if
// given, already holds Y^T Y.  The first product by R^{-1} also forms the
// Gram matrix of the second pass.
__device__ __forceinline__ int cholqr2_g(double* Y, double* X, int64_t ld, int n, int npad, int p, EigShared& S,
                         const double* G0) {
  if (G0) {
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) S.G[e] = G0[e];
    __syncthreads();
  } else {
    gram(Y, ld, n, p, S.G, S.bufU);
  }
  int ok = 1;
  for (int pass = 0; pass < 2; ++pass) {
    if (threadIdx.x < 64) {
      const int o = chol_inv_wave(S.G, S.Ri, p);
      if (threadIdx.x == 0) S.flag[0] = o;
    }
    __syncthreads();
    ok &= S.flag[0];
    __syncthreads();
    if (pass == 0)
      right_mul_upper(Y, Y, ld, n, npad, p, S.Ri, S.G, S.bufU, S.bufV);
    else
      right_mul_upper(Y, X, ld, n, npad, p, S.Ri, nullptr, S.bufU, S.bufV);
  }
  return ok;
}

__device__ __forceinline__ int cholqr2(double* Y, double* X, int64_t ld, int n, int npad, int p, EigShared& S) {
  return cholqr2_g(Y, X, ld, n, npad, p, S, nullptr);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
struct EigArgs {
  const int64_t* fac_off;
  const int32_t* bs;
  const int32_t* nb;
  const int32_t* ni;
  const int32_t* nI;
  const int64_t* om_off;
  const uint8_t* om_int;
  const int64_t* lrow;
  const int32_t* lcol;
  const double* lval;
  const int32_t* kdim;
  const int64_t* pad_off;
  const int32_t* cpl_col;
  const double* cpl_val;
  int cpl_ok;               // the coupling lists are complete
  const int32_t* rcpl_col;  // A_k,k+1 by row (fast coupling lists)
  const double* rcpl_val;
  const int32_t* ucpl_row;  // A_k-1,k by column
  const double* ucpl_val;
  const int32_t* lcpl_row;  // A_k+1,k by column
  const double* lcpl_val;
  double* dummy;    // per-thread discard slots (subdomain x chunk x thread)
  double* X;        // per subdomain npad x p at p*pad_off
  double* Y;
  double* W;        // per subdomain npad x p: forward results of the two-ended solve
  double* ell;      // per subdomain npad (unit left null vector; floating only)
  double* bell;     // B * ell
  double* btl;      // B^T * ell
  double* gam;      // per subdomain (ell^T B ell, ell^T J B ell)
  double* colsum;   // per (subdomain, column chunk, half, row parity) PC partial column
                    // sums of Y (parity 1 only for complex A)
  int defer;        // 1: the projection onto 1^perp is applied by k_eig_gram
  int32_t* done;    // converged flag
  int32_t* sweeps;
  int32_t* msel;    // selected count
  double* Vsel;     // per subdomain p x p (column-major p x m)
  double* lam;      // per subdomain 2*p (re, im)
  double* rres;     // per subdomain relative residual of the last Rayleigh-Ritz step
  double* rbest;    // best relative residual so far (stagnation test)
  int32_t* stall;   // consecutive Rayleigh-Ritz steps without a gain on rbest
  double* rlast;    // residual of the last Rayleigh-Ritz step
  int32_t* swlast;  // its sweep
  int32_t* next_rr; // sweep of the next Rayleigh-Ritz step
  double* HVs;      // per subdomain H V (p x m)
  const int32_t* blk_sub;   // row block -> subdomain
  const int32_t* blk_r0;    // row block -> first row
  const int32_t* sub_blk0;  // subdomain -> first row block (nsub + 1)
  const int32_t* qblk_sub;  // wide row blocks of k_ks_qr (KS_QRB rows): same maps
  const int32_t* qblk_r0;
  const int32_t* qsub_blk0;
  double* partA;    // per row block p x p partial products (PMAX^2 stride)
  double* partB;
  double* partH;
  double* partR;    // per row block partial squared residual
  int lrb;          // log2 of the row-block height
  // block Krylov-Schur state (block width p)
  int ks;           // 1: the operator kernels map columns jcur .. jcur + p - 1 of V
  int km;           // largest Rayleigh quotient order (the storage of V and Bk)
  const int32_t* kmi;     // per subdomain: its Rayleigh quotient order (<= km)
  const int32_t* kkeepi;  // per subdomain: basis vectors kept by a restart
  double* V;        // per subdomain npad x (km + p) basis, at (km + p) * pad_off
  double* Bk;       // per subdomain (km + p) x km row-major: T V_k = V_{k+p} Bk
  int32_t* jcur;    // per subdomain: first column of the block expanded next
  int32_t* kprev;   // per subdomain: Rayleigh quotient order of the last restart
  double* partK;    // per row block KS_PK partial products V^T W
  double* partK2;
  double* Ures;     // per subdomain kept Schur basis (order x kept, column-major)
  double* Racc;     // per subdomain two accumulated EIG_PC x EIG_PC triangular factors
  const float* x0;  // learned start block (node rows x x0_ld), interior rows used
  int x0_cols;      // start columns taken from it (subspace iteration)
  int x0_ld;        // columns of the network's block
  int x0_mix;       // Krylov-Schur: every start column a fixed combination of all x0_ld
  int32_t* err;
  int p;
  int nev;
  double tau;
  double tol;
  int sym;          // A symmetric: the splitting is too, its left null vector is the constant
  int pair;         // complex A in its real form: eigenvalues come in pairs, local rows
                    // (2t, 2t + 1) are the real and imaginary parts of one unknown
  const int32_t* order;  // subdomain of each block of the operator launches (longest first)
};

// (J v)_r in the real form of a complex vector (J multiplies by i: rows
// (2t, 2t + 1) <- (-v_{2t+1}, v_{2t})); r < n, n even
__device__ __forceinline__ double jrot(const double* v, int r) {
  return (r & 1) ? v[r - 1] : -v[r + 1];
}

// transposed solve with the splitting tiles for the left null vector:
// Atilde_reg^T l = e_er, er the last row (real A) or the real row of the last
// unknown (complex A; l is then the real form of the complex left null
// vector and J l the second one).  One-off per floating subdomain, single
// column.
template <class FT>
__device__ void transposed_solve_last(const FT* fac, int s, int K, int n, int er,
                                      const int64_t* lrow, const int32_t* lcol,
                                      const double* lval, const int32_t* urow,
                                      const double* uval, const int32_t* drow,
                                      const double* dval, double* x, double* tmp) {
  // urow / uval: A_k-1,k by column, drow / dval: A_k+1,k by column (NCPL
  // slots per padded column, rows ascending), or null: one thread then walks
  // the CSR rows (the same order of the sums)
  const int t = threadIdx.x, T = blockDim.x;
  constexpr int V = adsd::TileV<FT>::V;
  constexpr int U = 8;  // tile loads in flight per thread
  constexpr int NC = adsd::NCPL;
  const int64_t TS = adsd::tile_size(s, V);
  const int npad = K * s;
  for (int r = t; r < npad; r += T) x[r] = (r == er) ? 1.0 : 0.0;
  __syncthreads();
  // tmp[r] = sum_cc G(cc, r) v[cc] over cc ascending (G^T v)
  auto gt_product = [&](const FT* G, const double* v) {
    for (int r = t; r < s; r += T) {
      double acc = 0.0;
      for (int c0 = 0; c0 < s; c0 += U) {
        double m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) m[u] = adsd::ld_fac(G, adsd::tile_at(min(c0 + u, s - 1), r, s, V));
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (c0 + u < s) acc += m[u] * v[c0 + u];
      }
      tmp[r] = acc;
    }
  };
  // forward with U^T: w_k = G_k^T (f_k - A_{k-1,k}^T w_{k-1})
  for (int k = 0; k < K; ++k) {
    const int r0 = k * s;
    if (k > 0 && urow) {
      for (int cc = t; cc < s; cc += T) {
        const int64_t f = (int64_t)(r0 + cc) * NC;
        double v = x[r0 + cc];
#pragma unroll
        for (int m = 0; m < NC; ++m) {
          const int rw = urow[f + m];
          if (rw >= 0) v -= uval[f + m] * x[r0 - s + rw];
        }
        x[r0 + cc] = v;
      }
    } else if (k > 0 && t == 0) {
      for (int rr = 0; rr < s; ++rr) {
        const int r = r0 - s + rr;
        if (r >= n) break;
        for (int64_t q = lrow[r]; q < lrow[r + 1]; ++q) {
          const int cidx = lcol[q];
          if (cidx >= r0 && cidx < r0 + s) x[cidx] -= lval[q] * x[r];
        }
      }
    }
    __syncthreads();
    gt_product(fac + (int64_t)k * 2 * TS, x + r0);
    __syncthreads();
    for (int r = t; r < s; r += T) x[r0 + r] = tmp[r];
    __syncthreads();
  }
  // backward with L^T: l_k = w_k - G_k^T (A_{k+1,k}^T l_{k+1})
  for (int k = K - 2; k >= 0; --k) {
    const int r0 = k * s;
    if (drow) {
      for (int cc = t; cc < s; cc += T) {
        const int64_t f = (int64_t)(r0 + cc) * NC;
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < NC; ++m) {
          const int rw = drow[f + m];
          if (rw >= 0) v += dval[f + m] * x[r0 + s + rw];
        }
        tmp[s + cc] = v;
      }
    } else {
      for (int r = t; r < s; r += T) tmp[s + r] = 0.0;
      __syncthreads();
      if (t == 0) {
        for (int rr = 0; rr < s; ++rr) {
          const int r = r0 + s + rr;
          if (r >= n) break;
          for (int64_t q = lrow[r]; q < lrow[r + 1]; ++q) {
            const int cidx = lcol[q];
            if (cidx >= r0 && cidx < r0 + s) tmp[s + cidx - r0] += lval[q] * x[r];
          }
        }
      }
    }
    __syncthreads();
    gt_product(fac + (int64_t)k * 2 * TS, tmp + s);
    __syncthreads();
    for (int r = t; r < s; r += T) x[r0 + r] -= tmp[r];
    __syncthreads();
  }
}

// part[g * s + r] = sum over the g-th column chunk of G_k^T y (1024 threads,
// Gn = T / s groups), then res[r] = sum_g part[g * s + r] in group order
template <class FT>
__device__ __forceinline__ void tile_tmatvec(const FT* G, int s, const double* y, double* part,
                                             double* res, bool subtract) {
  constexpr int V = adsd::TileV<FT>::V;
  const int t = threadIdx.x, T = blockDim.x;
  const int Gn = T / s, chunk = (s + Gn - 1) / Gn;
  if (t < Gn * s) {
    const int r = t % s, g = t / s;
    const int c1 = min(s, (g + 1) * chunk);
    double acc = 0.0;
    for (int cc = g * chunk; cc < c1; ++cc) acc += adsd::ld_fac(G, adsd::tile_at(cc, r, s, V)) * y[cc];
    part[g * s + r] = acc;
  }
  __syncthreads();
  for (int r = t; r < s; r += T) {
    double v = 0.0;
    for (int g = 0; g < Gn; ++g) v += part[g * s + r];
    res[r] = subtract ? res[r] - v : v;
  }
  __syncthreads();
}

// l solves Atilde_reg^T l = e_er with the two-ended splitting tiles: the
// transposed system has the transposed two-ended factorization, so
//   forward top    w_k = G_k^T (f_k - A_k-1,k^T w_{k-1})      k = 0 .. M-1
//   forward bottom v_k = G_k^T (f_k - A_k+1,k^T v_{k+1})      k = K-1 .. M+1
//   middle         l_M = G_M^T (f_M - A_M-1,M^T w - A_M+1,M^T v)
//   backward top   l_k = w_k - G_k^T (A_k+1,k^T l_{k+1})      k = M-1 .. 0
//   backward bottom l_k = v_k - G_k^T (A_k-1,k^T l_{k-1})     k = M+1 .. K-1
// with A_k-1,k^T and A_k+1,k^T applied by column from the coupling lists.
// In three phases (separate launches, so that the two halves run on two
// workgroups): 0 the forward half `half` (with its rows of e_er), 1 the
// middle block, 2 the backward half `half`.  LDS: s (y) + T (partials).
template <class FT>
__device__ void transposed_solve_cpl(const FT* fac, int s, int K, int n, int er, const int32_t* urow,
                                     const double* uval, const int32_t* lrw, const double* lvl,
                                     double* x, double* lds, int phase, int half) {
  const int t = threadIdx.x, T = blockDim.x;
  constexpr int V = adsd::TileV<FT>::V;
  constexpr int NC = adsd::NCPL;
  const int64_t TS = adsd::tile_size(s, V);
  const int npad = K * s, M = K / 2;
  double* ybuf = lds;
  double* part = ybuf + s;
  // y_c = (keep ? x_k[c] : 0) - sum of the by-column lists (up: rows of
  // block k-1, dn: rows of block k+1) applied to x
  auto gather = [&](int k, bool keep, bool up, bool dn) {
    const int r0 = k * s;
    for (int c = t; c < s; c += T) {
      double v = keep ? x[r0 + c] : 0.0;
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        const int64_t e = (int64_t)(r0 + c) * NC + m;
        if (up) {
          const int rr = urow[e];
          if (rr >= 0) v -= uval[e] * x[r0 - s + rr];
        }
        if (dn) {
          const int rr = lrw[e];
          if (rr >= 0) v -= lvl[e] * x[r0 + s + rr];
        }
      }
      ybuf[c] = v;
    }
    __syncthreads();
  };
  if (phase == 0) {
    const int lo = half ? M * s : 0, hi = half ? npad : M * s;
    for (int r = lo + t; r < hi; r += T) x[r] = (r == er) ? 1.0 : 0.0;
    __syncthreads();
    if (!half) {
      for (int k = 0; k < M; ++k) {
        gather(k, true, k > 0, false);
        tile_tmatvec(fac + (int64_t)k * 2 * TS, s, ybuf, part, x + k * s, false);
      }
    } else {
      for (int k = K - 1; k > M; --k) {
        gather(k, true, false, k < K - 1);
        tile_tmatvec(fac + (int64_t)k * 2 * TS, s, ybuf, part, x + k * s, false);
      }
    }
  } else if (phase == 1) {
    gather(M, true, M > 0, M < K - 1);
    tile_tmatvec(fac + (int64_t)M * 2 * TS, s, ybuf, part, x + M * s, false);
  } else if (!half) {
    // backward: x_k -= G_k^T (-y) with y = -(A^T l_neighbour)
    for (int k = M - 1; k >= 0; --k) {
      gather(k, false, false, true);
      for (int c = t; c < s; c += T) ybuf[c] = -ybuf[c];
      __syncthreads();
      tile_tmatvec(fac + (int64_t)k * 2 * TS, s, ybuf, part, x + k * s, true);
    }
  } else {
    for (int k = M + 1; k < K; ++k) {
      gather(k, false, true, false);
      for (int c = t; c < s; c += T) ybuf[c] = -ybuf[c];
      __syncthreads();
      tile_tmatvec(fac + (int64_t)k * 2 * TS, s, ybuf, part, x + k * s, true);
    }
  }
}

// the unnormalised left null vector of the splitting on floating subdomains
// (fast coupling lists), one phase of transposed_solve_cpl per launch
template <class FT>
__global__ void __launch_bounds__(EIG_T) k_eig_ell(const FT* fac, EigArgs a, int phase) {
  extern __shared__ double dyn[];
  const int i = blockIdx.x;
  if (!a.kdim[i]) return;
  const int64_t po = a.pad_off[i] * adsd::NCPL;
  transposed_solve_cpl<FT>(fac + a.fac_off[i], a.bs[i], a.nb[i], a.ni[i], a.ni[i] - a.kdim[i],
                           a.ucpl_row + po,
                           a.ucpl_val + po, a.lcpl_row + po, a.lcpl_val + po,
                           a.ell + a.pad_off[i], dyn, phase, blockIdx.y);
}

// btl = B^T l and gam = l^T B l for a floating subdomain, B = D A_ii D: for
// every interior column c, the rows of A's column (transposed pattern, rows
// ascending) that are interior rows of Omega_i, in that order
// largest padded local size nb * bs over the subdomains
static int64_t npad_max(const Ctx& c) {
  int64_t m = 1;
  for (int i = 0; i < c.nsub; ++i) m = std::max(m, (int64_t)c.h_nb[i] * c.h_bs[i]);
  return m;
}

__global__ void k_eig_btl(EigArgs a, const int32_t* om_sorted, const int32_t* rowptr,
                          const int32_t* col, const double* val, const int32_t* tptr,
                          const int32_t* tcol, const int64_t* wlo, const int64_t* whi,
                          const int64_t* woff, const int32_t* wpos) {
  __shared__ double red[16];
  const int i = blockIdx.x;
  if (!a.kdim[i]) return;
  const int n = a.ni[i], npad = a.nb[i] * a.bs[i];
  const int64_t base = a.om_off[i];
  const int64_t wl = wlo[i], wh = whi[i], wo = woff[i];
  const double* l = a.ell + a.pad_off[i];
  double* bt = a.btl + a.pad_off[i];
  // one column per thread, the columns spread over blockIdx.y
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  if (c < npad) {
    double v = 0.0;
    if (c < n && a.om_int[base + c]) {
      const int gc = om_sorted[base + c];
      for (int q = tptr[gc]; q < tptr[gc + 1]; ++q) {
        const int gr = tcol[q];
        if (gr < wl || gr >= wh) continue;
        const int r = wpos[wo + (gr - wl)];
        if (r < 0 || !a.om_int[base + r]) continue;
        double arc = 0.0;
        for (int k = rowptr[gr]; k < rowptr[gr + 1]; ++k)
          if (col[k] == gc) arc = val[k];
        v += arc * l[r];
      }
    }
    bt[c] = v;
  }
  if (blockIdx.y != 0) return;
  // gam = (l^T B l, l^T J B l): the 2 x 2 matrix [l, J l]^T B [l, J l] of a
  // complex splitting is [[g, h], [-h, g]] (B and B^T commute with J)
  const double* bl = a.bell + a.pad_off[i];
  double g = 0.0, h = 0.0;
  for (int r = threadIdx.x; r < n; r += blockDim.x) g += l[r] * bl[r];
  g = adsd::block_sum(g, red);
  if (a.kdim[i] == 2) {
    for (int r = threadIdx.x; r < n; r += blockDim.x) h += l[r] * jrot(bl, r);
    h = adsd::block_sum(h, red);
  }
  if (threadIdx.x == 0) {
    a.gam[2 * i] = g;
    a.gam[2 * i + 1] = h;
  }
}

template <class FT, bool CPL>
__global__ void __launch_bounds__(EIG_T) k_eig_init(const FT* fac, EigArgs a, double* scratch) {
  __shared__ double red[16];
  const int i = blockIdx.x;
  const int s = a.bs[i], K = a.nb[i], n = a.ni[i], npad = K * s, p = a.p;
  const int64_t ld = npad;
  double* X = a.Y + a.pad_off[i] * p;  // random start block, orthonormalised into X
  const int64_t base = a.om_off[i];
  for (int64_t e = threadIdx.x; e < (int64_t)npad * p; e += blockDim.x) {
    const int r = (int)(e % npad), j = (int)(e / npad);
    double v = 0.0;
    if (r < n) {
      if (a.x0 && a.x0_mix) {
        // learned start for the block Krylov method: the block is narrower
        // than the network's (x0_ld columns spanning an approximation of the
        // wanted space), so each start column is a fixed pseudo-random
        // combination of all of them; one expansion then reaches the rest
        double acc = 0.0;
        if (a.om_int[base + r])
          for (int q = 0; q < a.x0_ld; ++q)
            acc += (double)a.x0[(base + r) * a.x0_ld + q] *
                   adsd::hash_unit((0x5EEDull << 40) ^ ((uint64_t)q << 8) ^ (uint64_t)j);
        v = acc;
      } else if (a.x0 && j < a.x0_cols) {  // interior rows of the network's block
        v = a.om_int[base + r] ? (double)a.x0[(base + r) * a.x0_ld + j] : 0.0;
      }
      else if (a.pair && (j & 1)) {
        // complex A: the odd columns are i times the even ones (J x: rows
        // (2t, 2t + 1) <- (-x_{2t+1}, x_{2t})), so that the start block, and
        // with it the Krylov space, is closed under multiplication by i
        const double h = adsd::hash_unit(((uint64_t)i << 40) ^ ((uint64_t)(j - 1) << 24) ^
                                         (uint64_t)(r ^ 1));
        v = (r & 1) ? h : -h;
      } else
        v = adsd::hash_unit(((uint64_t)i << 40) ^ ((uint64_t)j << 24) ^ (uint64_t)r);
    }
    X[r + j * ld] = v;
  }
  __syncthreads();
  if (a.kdim[i]) {
    const int kd = a.kdim[i];
    double* l = a.ell + a.pad_off[i];
    extern __shared__ double dyn[];
    if (a.sym) {
      // symmetric splitting: its left null vector is its right one, the
      // constant (exact, no solve with the ill-conditioned regularised matrix);
      // complex A: the real form of the complex constant, 1 on the real rows
      for (int r = threadIdx.x; r < npad; r += blockDim.x)
        l[r] = (r < n && (kd == 1 || !(r & 1))) ? 1.0 : 0.0;
      __syncthreads();
    } else if constexpr (!CPL) {  // (with the coupling lists, k_eig_ell has formed l)
      transposed_solve_last<FT>(fac + a.fac_off[i], s, K, n, n - kd, a.lrow + base, a.lcol,
                                a.lval,
                                a.cpl_ok ? a.ucpl_row + a.pad_off[i] * adsd::NCPL : nullptr,
                                a.cpl_ok ? a.ucpl_val + a.pad_off[i] * adsd::NCPL : nullptr,
                                a.cpl_ok ? a.lcpl_row + a.pad_off[i] * adsd::NCPL : nullptr,
                                a.cpl_ok ? a.lcpl_val + a.pad_off[i] * adsd::NCPL : nullptr, l,
                                dyn);
    }
    double nn = 0.0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) nn += l[r] * l[r];
    nn = adsd::block_sum(nn, red);
    const double inv = 1.0 / sqrt(nn);
    for (int r = threadIdx.x; r < npad; r += blockDim.x) l[r] = (r < n) ? l[r] * inv : 0.0;
    __syncthreads();
    // B l
    double* bl = a.bell + a.pad_off[i];
    for (int r = threadIdx.x; r < npad; r += blockDim.x) {
      double v = 0.0;
      if (r < n && a.om_int[base + r])
        for (int64_t q = a.lrow[base + r]; q < a.lrow[base + r + 1]; ++q)
          if (a.om_int[base + a.lcol[q]]) v += a.lval[q] * l[a.lcol[q]];
      bl[r] = v;
    }
    // X <- projection onto K^perp, column j by wave j mod (number of waves):
    // minus the column mean (complex A: the means of the real and of the
    // imaginary rows, K being span{1, J 1} in the real form)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = wv; j < p; j += nw) {
      if (kd == 2) {
        double se = 0.0, so = 0.0;
        for (int r = lane; r < n; r += 64) {
          if (r & 1)
            so += X[r + j * ld];
          else
            se += X[r + j * ld];
        }
        se = adsd::wave_sum(se) / (n / 2);
        so = adsd::wave_sum(so) / (n / 2);
        for (int r = lane; r < n; r += 64) X[r + j * ld] -= (r & 1) ? so : se;
      } else {
        double sm = 0.0;
        for (int r = lane; r < n; r += 64) sm += X[r + j * ld];
        sm = adsd::wave_sum(sm) / n;
        for (int r = lane; r < n; r += 64) X[r + j * ld] -= sm;
      }
    }
  }
}

// per-column block sums of PC partial values (wave shuffles, then the wave
// partials in a fixed order); out[j] for j < pc
template <int PC>
__device__ __forceinline__ void block_sum_cols(double (&v)[PC], double (*red)[16], double* out,
                                               int pc) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < PC; ++j) {
    double x = v[j];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[j][wv] = x;
  }
  __syncthreads();
  if ((int)threadIdx.x < pc) {
    double x = 0.0;
    for (int w = 0; w < nw; ++w) x += red[threadIdx.x][w];
    out[threadIdx.x] = x;
  }
  __syncthreads();
}

// Y = T X for columns [j0, j0 + PC), fast path: the two-ended solve in two
// launches.  k_eig_op_fwd (grid: subdomain x column chunk x half) forms
// F = B Pi X on its half of the rows (half 0: blocks 0..M, half 1: blocks
// M+1..K-1) with alpha = l^T X and beta = l^T B Pi X = btl^T X - alpha gam
// (both from X, so each half needs only its own rows of F), then runs its
// forward chain in place in W.  k_eig_op_bwd: the middle block and the
// backward chain from W into Y, and on floating subdomains the per-half
// column sums of Y; the projection onto 1^perp is applied by k_eig_gram.
// Complex A (kernel dimension 2): Pi = I - l l^T - (J l)(J l)^T, with
// alpha2 = (J l)^T X, beta2 = (J l)^T B Pi X = (J btl)^T X + alpha h -
// alpha2 g and beta = btl^T X - alpha g - alpha2 h ((g, h) = gam), and the
// column sums split into real and imaginary rows.
template <class FT, int PC, int D>
__global__ void __launch_bounds__(1024) k_eig_op_fwd(const FT* fac, EigArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[PC][16];
  __shared__ double alpha[PC], beta[PC], alpha2[PC], beta2[PC];
  const int i = adsd::sub_of(a.order, blockIdx.x), half = blockIdx.z;
  if (a.done[i] || (a.ks && a.jcur[i] + a.p > a.kmi[i])) return;
  const int j0 = blockIdx.y * PC;
  const int p = a.p;
  const int pc = min(PC, p - j0);
  if (pc <= 0) return;
  const int t = threadIdx.x, T = blockDim.x;
  const int s = a.bs[i], K = a.nb[i], n = a.ni[i], npad = K * s, M = K / 2;
  const int64_t ld = npad;
  const int64_t base = a.om_off[i];
  const double* X = a.ks ? a.V + a.pad_off[i] * (a.km + p) + a.jcur[i] * ld
                         : a.X + a.pad_off[i] * p + j0 * ld;
  double* Wv = a.W + a.pad_off[i] * p + j0 * ld;
  const bool floating = a.kdim[i] != 0;
  const double* l = a.ell + a.pad_off[i];
  const double* bl = a.bell + a.pad_off[i];
  const uint8_t* oi = a.om_int + base;
  const int64_t* lrow = a.lrow + base;
  const bool cpair = a.kdim[i] == 2;
  double acc[PC], acc2[PC];
  if (floating) {  // alpha = l^T X, delta = btl^T X over all rows
    const double* bt = a.btl + a.pad_off[i];
#pragma unroll
    for (int j = 0; j < PC; ++j) acc[j] = acc2[j] = 0.0;
    for (int r = t; r < n; r += T) {
      const double lr = l[r], br = bt[r];
#pragma unroll
      for (int j = 0; j < PC; ++j)
        if (j < pc) {
          const double x = X[r + j * ld];
          acc[j] += lr * x;
          acc2[j] += br * x;
        }
    }
    block_sum_cols<PC>(acc, red, alpha, pc);
    block_sum_cols<PC>(acc2, red, beta, pc);
    if (cpair) {  // the same with J l and J btl
#pragma unroll
      for (int j = 0; j < PC; ++j) acc[j] = acc2[j] = 0.0;
      for (int r = t; r < n; r += T) {
        const double lr = jrot(l, r), br = jrot(bt, r);
#pragma unroll
        for (int j = 0; j < PC; ++j)
          if (j < pc) {
            const double x = X[r + j * ld];
            acc[j] += lr * x;
            acc2[j] += br * x;
          }
      }
      block_sum_cols<PC>(acc, red, alpha2, pc);
      block_sum_cols<PC>(acc2, red, beta2, pc);
      if (t < pc) {
        const double g = a.gam[2 * i], h = a.gam[2 * i + 1];
        const double a1 = alpha[t], a2 = alpha2[t];
        beta[t] -= a1 * g + a2 * h;
        beta2[t] += a1 * h - a2 * g;
      }
    } else if (t < pc) {
      beta[t] -= alpha[t] * a.gam[2 * i];
    }
    __syncthreads();
  }
  const int lo = half ? (M + 1) * s : 0, hi = half ? npad : (M + 1) * s;
  for (int r = lo + t; r < hi; r += T) {
    double v[PC];
#pragma unroll
    for (int j = 0; j < PC; ++j) v[j] = 0.0;
    if (r < n && oi[r]) {
      const int64_t q1 = lrow[r + 1];
      for (int64_t q = lrow[r]; q < q1; ++q) {
        const int c = a.lcol[q];
        if (!oi[c]) continue;
        const double av = a.lval[q];
#pragma unroll
        for (int j = 0; j < PC; ++j)
          if (j < pc) v[j] += av * X[c + j * ld];
      }
    }
    if (floating && r < n) {
      const double br = bl[r], lr = l[r];
#pragma unroll
      for (int j = 0; j < PC; ++j) {
        const int jj = j < pc ? j : 0;
        v[j] -= alpha[jj] * br + beta[jj] * lr;
      }
      if (cpair) {
        const double jbr = jrot(bl, r), jlr = jrot(l, r);
#pragma unroll
        for (int j = 0; j < PC; ++j) {
          const int jj = j < pc ? j : 0;
          v[j] -= alpha2[jj] * jbr + beta2[jj] * jlr;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < PC; ++j)
      if (j < pc) Wv[r + j * ld] = v[j];
  }
  __syncthreads();
  double* dummy =
      a.dummy + (((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * blockDim.x +
      threadIdx.x;
  const int64_t cb = a.pad_off[i] * adsd::NCPL;
  const int32_t* cc = (half ? a.rcpl_col : a.cpl_col) + cb;
  const double* cv = (half ? a.rcpl_val : a.cpl_val) + cb;
  adsd::block_chain<FT, PC, D, true>(fac + a.fac_off[i], s, half ? K - 1 : 0, half ? -1 : 1,
                                     half ? K - 1 - M : M, cc, cv, Wv, Wv, ld, pc, lds, dummy);
}

template <class FT, int PC, int D>
__global__ void __launch_bounds__(1024) k_eig_op_bwd(const FT* fac, EigArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[PC][16];
  __shared__ double sums[PC];
  const int i = adsd::sub_of(a.order, blockIdx.x), half = blockIdx.z;
  if (a.done[i] || (a.ks && a.jcur[i] + a.p > a.kmi[i])) return;
  const int j0 = blockIdx.y * PC;
  const int p = a.p;
  const int pc = min(PC, p - j0);
  if (pc <= 0) return;
  const int t = threadIdx.x, T = blockDim.x;
  const int s = a.bs[i], K = a.nb[i], n = a.ni[i], npad = K * s, M = K / 2;
  const int64_t ld = npad;
  const double* Wv = a.W + a.pad_off[i] * p + j0 * ld;
  double* Y = a.Y + a.pad_off[i] * p + j0 * ld;
  const int64_t cb = a.pad_off[i] * adsd::NCPL;
  const FT* F = fac + a.fac_off[i];
  adsd::block_mid<FT, PC>(F, s, M, K, a.cpl_col + cb, a.cpl_val + cb, a.rcpl_col + cb,
                          a.rcpl_val + cb, Wv, half == 0 ? Y : nullptr, ld, pc, lds);
  double* dummy =
      a.dummy + (((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * blockDim.x +
      threadIdx.x;
  adsd::block_chain<FT, PC, D, false>(F, s, half ? M + 1 : M - 1, half ? 1 : -1,
                                      half ? K - 1 - M : M, nullptr, nullptr, Wv, Y, ld, pc, lds,
                                      dummy);
  if (a.kdim[i]) {  // partial column sums of this half's rows (padding rows are zero)
    // slots (subdomain, chunk, half, row parity): all rows in parity 0 for
    // real A, real and imaginary rows apart for complex A
    __syncthreads();
    const int lo = half ? (M + 1) * s : 0, hi = min(n, half ? npad : (M + 1) * s);
    double* cs = a.colsum + (((int64_t)i * gridDim.y + blockIdx.y) * 2 + half) * 2 * PC;
    const int npar = a.kdim[i];
    for (int par = 0; par < npar; ++par) {
      double acc[PC];
#pragma unroll
      for (int j = 0; j < PC; ++j) acc[j] = 0.0;
      for (int r = lo + t; r < hi; r += T) {
        if (npar == 2 && (r & 1) != par) continue;
#pragma unroll
        for (int j = 0; j < PC; ++j)
          if (j < pc) acc[j] += Y[r + j * ld];
      }
      block_sum_cols<PC>(acc, red, sums, pc);
      if (t < pc) cs[par * PC + t] = sums[t];
    }
  }
}

// Y = T X for columns [j0, j0 + PC), general path (one-ended factorization,
// any block size).  T = Pi_1 Atilde^{-1} Pi B Pi on floating subdomains
// (Pi = I - l l^T, Pi_1 the projection onto 1^perp), Atilde^{-1} B otherwise;
// B = D A_ii D.
template <class FT, int PC>
__global__ void __launch_bounds__(1024) k_eig_op(const FT* fac, EigArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[PC][16];
  __shared__ double alpha[PC], beta[PC], alpha2[PC], beta2[PC];
  const int i = adsd::sub_of(a.order, blockIdx.x);
  if (a.done[i] || (a.ks && a.jcur[i] + a.p > a.kmi[i])) return;
  const int j0 = blockIdx.y * PC;
  const int p = a.p;
  const int pc = min(PC, p - j0);
  if (pc <= 0) return;
  const int t = threadIdx.x, T = blockDim.x;
  const int s = a.bs[i], K = a.nb[i], n = a.ni[i], npad = K * s;
  const int64_t ld = npad;
  const int64_t base = a.om_off[i];
  const double* X = a.ks ? a.V + a.pad_off[i] * (a.km + p) + a.jcur[i] * ld
                         : a.X + a.pad_off[i] * p + j0 * ld;
  double* Y = a.Y + a.pad_off[i] * p + j0 * ld;
  const bool floating = a.kdim[i] != 0;
  const double* l = a.ell + a.pad_off[i];
  const double* bl = a.bell + a.pad_off[i];
  const uint8_t* oi = a.om_int + base;
  const int64_t* lrow = a.lrow + base;
  // complex A (kernel dimension 2): Pi = I - l l^T - (J l)(J l)^T, the
  // second term through alpha2 = (J l)^T X, B J l = J B l and beta2
  const bool cpair = a.kdim[i] == 2;
  double acc[PC], acc2[PC];
  if (floating) {  // alpha = l^T X
#pragma unroll
    for (int j = 0; j < PC; ++j) acc[j] = 0.0;
    for (int r = t; r < n; r += T) {
      const double lr = l[r];
#pragma unroll
      for (int j = 0; j < PC; ++j)
        if (j < pc) acc[j] += lr * X[r + j * ld];
    }
    block_sum_cols<PC>(acc, red, alpha, pc);
    if (cpair) {
#pragma unroll
      for (int j = 0; j < PC; ++j) acc[j] = 0.0;
      for (int r = t; r < n; r += T) {
        const double lr = jrot(l, r);
#pragma unroll
        for (int j = 0; j < PC; ++j)
          if (j < pc) acc[j] += lr * X[r + j * ld];
      }
      block_sum_cols<PC>(acc, red, alpha2, pc);
    }
  }
  // F = B (Pi X) = B X - alpha B l, row-parallel over all PC columns;
  // beta = l^T F on the way
#pragma unroll
  for (int j = 0; j < PC; ++j) acc[j] = acc2[j] = 0.0;
  for (int r = t; r < npad; r += T) {
    double v[PC];
#pragma unroll
    for (int j = 0; j < PC; ++j) v[j] = 0.0;
    if (r < n && oi[r]) {
      const int64_t q1 = lrow[r + 1];
      for (int64_t q = lrow[r]; q < q1; ++q) {
        const int c = a.lcol[q];
        if (!oi[c]) continue;
        const double av = a.lval[q];
#pragma unroll
        for (int j = 0; j < PC; ++j)
          if (j < pc) v[j] += av * X[c + j * ld];
      }
      if (floating) {
        const double br = bl[r], lr = l[r];
        if (cpair) {
          const double jbr = jrot(bl, r), jlr = jrot(l, r);
#pragma unroll
          for (int j = 0; j < PC; ++j) {
            const int jj = j < pc ? j : 0;
            v[j] -= alpha[jj] * br + alpha2[jj] * jbr;
            acc[j] += lr * v[j];
            acc2[j] += jlr * v[j];
          }
        } else {
#pragma unroll
          for (int j = 0; j < PC; ++j) {
            v[j] -= alpha[j < pc ? j : 0] * br;
            acc[j] += lr * v[j];
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < PC; ++j)
      if (j < pc) Y[r + j * ld] = v[j];
  }
  if (floating) {  // F <- Pi F
    block_sum_cols<PC>(acc, red, beta, pc);
    if (cpair) block_sum_cols<PC>(acc2, red, beta2, pc);
    for (int r = t; r < n; r += T) {
      const double lr = l[r], jlr = cpair ? jrot(l, r) : 0.0;
#pragma unroll
      for (int j = 0; j < PC; ++j)
        if (j < pc) Y[r + j * ld] -= cpair ? beta[j] * lr + beta2[j] * jlr : beta[j] * lr;
    }
  }
  __syncthreads();
  const int64_t cb = a.pad_off[i] * adsd::NCPL;
  // eight tile loads in flight per thread: the registers then allow one
  // workgroup per compute unit, which streams the tiles faster than two with
  // two loads each (the dependent block chain leaves each workgroup's loads
  // as the only source of parallelism)
  adsd::block_solve_general<FT, PC, true>(fac + a.fac_off[i], s, K, n, a.lrow + base, a.lcol,
                                           a.lval, a.cpl_ok ? a.cpl_col + cb : nullptr,
                                           a.cpl_ok ? a.cpl_val + cb : nullptr, Y,
                                    ld, pc, lds);
  if (floating && !cpair) {  // projection onto 1^perp
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PC; ++j) acc[j] = 0.0;
    for (int r = t; r < n; r += T) {
#pragma unroll
      for (int j = 0; j < PC; ++j)
        if (j < pc) acc[j] += Y[r + j * ld];
    }
    block_sum_cols<PC>(acc, red, alpha, pc);
    for (int r = t; r < n; r += T) {
#pragma unroll
      for (int j = 0; j < PC; ++j)
        if (j < pc) Y[r + j * ld] -= alpha[j] / n;
    }
  } else if (floating) {  // onto K^perp: the means of the real and imaginary rows apart
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PC; ++j) acc[j] = acc2[j] = 0.0;
    for (int r = t; r < n; r += T) {
#pragma unroll
      for (int j = 0; j < PC; ++j)
        if (j < pc) {
          if (r & 1)
            acc2[j] += Y[r + j * ld];
          else
            acc[j] += Y[r + j * ld];
        }
    }
    block_sum_cols<PC>(acc, red, alpha, pc);
    block_sum_cols<PC>(acc2, red, alpha2, pc);
    const int nh = n / 2;
    for (int r = t; r < n; r += T) {
#pragma unroll
      for (int j = 0; j < PC; ++j)
        if (j < pc) Y[r + j * ld] -= ((r & 1) ? alpha2[j] : alpha[j]) / nh;
    }
  }
}

// ---------------------------------------------------------------------------
// Row-block kernels of a sweep: every subdomain's rows are cut into blocks of
// RB rows (RB a power of two, RB * pq <= RBE, pq = p rounded up to 4), one
// workgroup per block, the block staged whole in LDS.  Partial p x p products
// per block are summed by their consumers in block order (deterministic).
//   orthonormalisation (Cholesky QR twice):  k_eig_gram -> k_eig_orth(0) -> k_eig_orth(1)
//   Rayleigh-Ritz sweeps: k_eig_gram(rr) -> k_eig_rr -> k_eig_resid -> k_eig_decide,
//                         then the orthonormalisation of the unconverged ones
// ---------------------------------------------------------------------------
static constexpr int RBE = 8192;
static constexpr int RB_NPT = RBE / EIG_T;

// log2 of the row-block height for a block of width p
__host__ __device__ inline int rb_log2(int p) {
  const int pq = (p + 3) & ~3;
  int l = 0;
  while ((2 << l) * pq <= RBE) ++l;
  return l;
}

// rows [r0, r0 + rows) of the column-major block M (leading dimension ld, p
// columns) into S[r + c * RB] for c < pq, zero outside; loads issued first
__device__ __forceinline__ void stage_rows(const double* M, int64_t ld, int r0, int rows, int p,
                                           int pq, int lrb, double* S) {
  const int t = threadIdx.x, RB = 1 << lrb;
  double v[RB_NPT];
#pragma unroll
  for (int k = 0; k < RB_NPT; ++k) {
    const int e = t + k * EIG_T, r = e & (RB - 1), c = e >> lrb;
    const bool ok = c < p && r < rows;
    const double x = M[ok ? (int64_t)r0 + r + c * ld : 0];
    v[k] = ok ? x : 0.0;
  }
#pragma unroll
  for (int k = 0; k < RB_NPT; ++k) {
    const int e = t + k * EIG_T;
    if ((e >> lrb) < pq) S[e] = v[k];
  }
}

// out[a * p + b] = sum_{r < rows} U[r + a RB] V[r + b RB] for a, b < p.  Wave w
// takes the 4 x 4 tiles w, w + 16, ...; its lanes split the rows; the lane
// sums are joined by a butterfly (same order on every run).
__device__ __forceinline__ void block_gram(const double* U, const double* V, int rows, int p,
                                           int pq, int RB, double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = pq >> 2;
  for (int tile = wv; tile < q * q; tile += EIG_T / 64) {
    const int ta = tile / q, tb = tile % q;
    const double* Ua = U + 4 * ta * RB;
    const double* Vb = V + 4 * tb * RB;
    double acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0;
    for (int r = lane; r < rows; r += 64) {
      double u[4], v[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        u[x] = Ua[r + x * RB];
        v[x] = Vb[r + x * RB];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x * 4 + y] += u[x] * v[y];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[k] += __shfl_xor(acc[k], o, 64);
    if (lane < 16) {
      const int x = lane >> 2, y = lane & 3;
      const int ra = 4 * ta + x, cb = 4 * tb + y;
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k == lane) v = acc[k];
      if (ra < p && cb < p) out[ra * p + cb] = v;
    }
  }
}

// sum of the per-block partial p x p products of a subdomain (blocks
// b0..b1-1): EIG_T / p^2 thread groups take every G-th block, then the group
// sums are added in group order; tmp holds EIG_T doubles of LDS
__device__ __forceinline__ void sum_parts(const double* part, int b0, int b1, int p, double* out,
                                          double* tmp) {
  const int t = threadIdx.x, pp = p * p;
  const int G = EIG_T / pp;
  const int e = t % pp, g = t / pp;
  if (g < G) {
    double sacc = 0.0;
#pragma unroll 4
    for (int bb = b0 + g; bb < b1; bb += G) sacc += part[(int64_t)bb * PMAX * PMAX + e];
    tmp[g * pp + e] = sacc;
  }
  __syncthreads();
  if (t < pp) {
    double sacc = 0.0;
    for (int k = 0; k < G; ++k) sacc += tmp[k * pp + t];
    out[t] = sacc;
  }
  __syncthreads();
}

// sum of the per-block partial vectors of cnt entries (stride ld) of blocks
// b0..b1-1, in a fixed grouping; tmp holds EIG_T doubles of LDS
__device__ __forceinline__ void sum_parts_n(const double* part, int64_t ld, int b0, int b1,
                                            int cnt, double* out, double* tmp) {
  const int t = threadIdx.x;
  const int G = EIG_T / cnt;
  const int e = t % cnt, g = t / cnt;
  if (g < G) {
    double sacc = 0.0;
#pragma unroll 4
    for (int bb = b0 + g; bb < b1; bb += G) sacc += part[(int64_t)bb * ld + e];
    tmp[g * cnt + e] = sacc;
  }
  __syncthreads();
  if (t < cnt) {
    double sacc = 0.0;
    for (int k = 0; k < G; ++k) sacc += tmp[k * cnt + t];
    out[t] = sacc;
  }
  __syncthreads();
}

// out[x * ldo + y] = sum_{r < rows} U[r + x RB] V[r + y RB] for x < nu, y < nv
// (U and V staged with zero columns up to a multiple of 4); 4 x 4 tiles per
// wave as in block_gram
__device__ __forceinline__ void block_gram_rect(const double* U, int nu, const double* V, int nv,
                                                int rows, int RB, double* out, int ldo) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int qa = (nu + 3) >> 2, qb = (nv + 3) >> 2;
  for (int tile = wv; tile < qa * qb; tile += EIG_T / 64) {
    const int ta = tile / qb, tb = tile % qb;
    const double* Ua = U + 4 * ta * RB;
    const double* Vb = V + 4 * tb * RB;
    double acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0;
    for (int r = lane; r < rows; r += 64) {
      double u[4], v[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        u[x] = Ua[r + x * RB];
        v[x] = Vb[r + x * RB];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x * 4 + y] += u[x] * v[y];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[k] += __shfl_xor(acc[k], o, 64);
    if (lane < 16) {
      const int x = lane >> 2, y = lane & 3;
      const int ra = 4 * ta + x, cb = 4 * tb + y;
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k == lane) v = acc[k];
      if (ra < nu && cb < nv) out[ra * ldo + cb] = v;
    }
  }
}

// partial Gram matrices of one row block: Y^T Y (and X^T Y for Rayleigh-Ritz)
__global__ void __launch_bounds__(EIG_T) k_eig_gram(EigArgs a, int rr) {
  extern __shared__ double rbuf[];
  const int b = blockIdx.x, i = a.blk_sub[b];
  if (a.done[i]) return;
  const int p = a.p, pq = (p + 3) & ~3, lrb = a.lrb, RB = 1 << lrb;
  const int r0 = a.blk_r0[b], rows = min(RB, a.ni[i] - r0);
  const int64_t ld = (int64_t)a.nb[i] * a.bs[i];
  double* Ys = rbuf;
  double* Xs = rbuf + RB * pq;
  double* Y = a.Y + a.pad_off[i] * p;
  stage_rows(Y, ld, r0, rows, p, pq, lrb, Ys);
  if (rr) stage_rows(a.X + a.pad_off[i] * p, ld, r0, rows, p, pq, lrb, Xs);
  if (a.defer && a.kdim[i]) {
    // projection onto K^perp left by the two-ended operator: subtract the
    // column means (from the per-half sums) from this block's rows (complex
    // A: the means of the real and of the imaginary rows)
    __shared__ double mu[2][PMAX];
    const int nch = (p + EIG_PC - 1) / EIG_PC, kd = a.kdim[i];
    if ((int)threadIdx.x < kd * p) {
      const int par = threadIdx.x / p, j = threadIdx.x % p, ch = j / EIG_PC, jj = j % EIG_PC;
      const double* cs = a.colsum + (int64_t)i * nch * 4 * EIG_PC;
      mu[par][j] = (cs[((ch * 2 + 0) * 2 + par) * EIG_PC + jj] +
                    cs[((ch * 2 + 1) * 2 + par) * EIG_PC + jj]) /
                   (a.ni[i] / kd);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < RB * p; e += EIG_T) {
      const int r = e & (RB - 1), c = e >> lrb;
      if (r < rows) {
        const double v = Ys[e] - mu[kd == 2 ? ((r0 + r) & 1) : 0][c];
        Ys[e] = v;
        Y[r0 + r + c * ld] = v;
      }
    }
  }
  __syncthreads();
  block_gram(Ys, Ys, rows, p, pq, RB, a.partA + (int64_t)b * PMAX * PMAX);
  if (rr) block_gram(Xs, Ys, rows, p, pq, RB, a.partH + (int64_t)b * PMAX * PMAX);
}

// Cholesky factor R (upper, row-major) of G + shift I and its inverse for a
// block of p <= EIG_PC columns, by one thread; returns 0 on a non-positive
// pivot
__device__ inline int chol_small(const double* G, double shift, double* R, double* Rinv, int p) {
  int ok = 1;
  for (int k = 0; k < p; ++k) {
    double d = G[k * p + k] + shift;
    for (int q = 0; q < k; ++q) d -= R[q * p + k] * R[q * p + k];
    if (!(d > 0.0)) {
      ok = 0;
      d = 1e-300;
    }
    const double rkk = sqrt(d);
    for (int j = 0; j < p; ++j) {
      double v = 0.0;
      if (j == k)
        v = rkk;
      else if (j > k) {
        v = G[k * p + j];
        for (int q = 0; q < k; ++q) v -= R[q * p + k] * R[q * p + j];
        v /= rkk;
      }
      R[k * p + j] = v;
    }
  }
  for (int j = 0; j < p; ++j)
    for (int ii = p - 1; ii >= 0; --ii) {
      double v = 0.0;
      if (ii == j)
        v = 1.0 / R[ii * p + ii];
      else if (ii < j) {
        for (int k = ii + 1; k <= j; ++k) v -= R[ii * p + k] * Rinv[k * p + j];
        v /= R[ii * p + ii];
      }
      Rinv[ii * p + j] = v;
    }
  return ok;
}

__device__ __forceinline__ double ks_shift(const double* G, int p, int n) {
  double tr = 0.0;
  for (int k = 0; k < p; ++k) tr += G[k * p + k];
  return 11.0 * ((double)n * p + p * (p + 1)) * 1.1102230246251565e-16 * tr;
}

// one Cholesky QR pass on a row block (block subspace iteration): R^T R = sum
// of the partial Gram matrices, then Y <- Y R^{-1} with the new block's
// partial Gram (pass 0), or X <- Y R^{-1} (pass 1)
__global__ void __launch_bounds__(EIG_T) k_eig_orth(EigArgs a, int pass) {
  extern __shared__ double rbuf[];
  __shared__ double Gs[PMAX * PMAX];
  __shared__ double Ri[PMAX * PMAX];
  __shared__ int okf;
  const int b = blockIdx.x, i = a.blk_sub[b];
  if (a.done[i]) return;
  const int p = a.p, pq = (p + 3) & ~3, lrb = a.lrb, RB = 1 << lrb;
  const int r0 = a.blk_r0[b], rows = min(RB, a.ni[i] - r0);
  const int64_t ld = (int64_t)a.nb[i] * a.bs[i];
  double* Y = a.Y + a.pad_off[i] * p;
  double* Ys = rbuf;
  double* Ws = rbuf + RB * pq;
  stage_rows(Y, ld, r0, rows, p, pq, lrb, Ys);
  sum_parts(pass == 0 ? a.partA : a.partB, a.sub_blk0[i], a.sub_blk0[i + 1], p, Gs, Ws);
  if (threadIdx.x < 64) {
    const int o = chol_inv_wave(Gs, Ri, p);
    if (threadIdx.x == 0) okf = o;
  }
  __syncthreads();
  if (!okf && threadIdx.x == 0) atomicOr(a.err, 2);
  double* out = pass == 0 ? Y : a.X + a.pad_off[i] * p;
#pragma unroll 1
  for (int k = 0; k < RB_NPT; ++k) {
    const int e = threadIdx.x + k * EIG_T, r = e & (RB - 1), c = e >> lrb;
    if (c >= pq) continue;
    double v = 0.0;
    if (c < p && r < rows) {
      for (int q = 0; q <= c; ++q) v += Ys[r + q * RB] * Ri[q * p + c];
      out[r0 + r + c * ld] = v;
    }
    Ws[e] = v;
  }
  if (pass == 0) {
    __syncthreads();
    block_gram(Ws, Ws, rows, p, pq, RB, a.partB + (int64_t)b * PMAX * PMAX);
  }
}

// Rayleigh-Ritz on H = X^T Y (one workgroup per subdomain): the selected
// invariant subspace V, H V and the eigenvalues
__global__ void __launch_bounds__(EIG_T) k_eig_rr(EigArgs a) {
  __shared__ SmallEigLds se;
  __shared__ double H[PMAX * PMAX];
  __shared__ double tmp[EIG_T];
  __shared__ double lam_re[PMAX], lam_im[PMAX];
  __shared__ int flag[2];
  const int i = blockIdx.x;
  if (a.done[i]) return;
  const int p = a.p;
  const int count = a.nev - a.kdim[i];
  sum_parts(a.partH, a.sub_blk0[i], a.sub_blk0[i + 1], p, H, tmp);
  if (threadIdx.x < 64) {
    int ok = 1;
    double gap = 1.0;
    const int m = small_eig_select(p, H, count, a.tau, se, lam_re, lam_im, &ok, &gap, 0, nullptr,
                                   nullptr, a.pair);
    if (threadIdx.x == 0) {
      flag[0] = m;
      flag[1] = ok;
    }
  }
  __syncthreads();
  const int m = flag[0];
  if (threadIdx.x == 0) {
    if (!flag[1]) atomicOr(a.err, 4);
    // the selected cluster must leave at least one Ritz value outside it,
    // otherwise the cluster may extend beyond the subspace
    if (m + a.kdim[i] >= p) atomicOr(a.err, 16);
    a.msel[i] = m;
  }
  double* Vs = a.Vsel + (int64_t)i * VSEL;
  double* HV = a.HVs + (int64_t)i * PMAX * PMAX;
  for (int e = threadIdx.x; e < p * m; e += blockDim.x) {
    const int r = e % p, c = e / p;
    double v = 0.0;
    for (int k = 0; k < p; ++k) v += H[r * p + k] * se.V[c * p + k];
    HV[e] = v;
    Vs[e] = se.V[e];
  }
  double* lam = a.lam + (int64_t)i * 2 * PMAX;
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    lam[c] = lam_re[c];
    lam[PMAX + c] = lam_im[c];
  }
}

// partial ||Y V - X (H V)||_F^2 of one row block
__global__ void __launch_bounds__(EIG_T) k_eig_resid(EigArgs a) {
  extern __shared__ double rbuf[];
  __shared__ double Vs[PMAX * PMAX], HV[PMAX * PMAX];
  __shared__ double red[16];
  const int b = blockIdx.x, i = a.blk_sub[b];
  if (a.done[i]) return;
  const int p = a.p, pq = (p + 3) & ~3, lrb = a.lrb, RB = 1 << lrb;
  const int r0 = a.blk_r0[b], rows = min(RB, a.ni[i] - r0);
  const int64_t ld = (int64_t)a.nb[i] * a.bs[i];
  const int m = a.msel[i];
  for (int e = threadIdx.x; e < p * m; e += blockDim.x) {
    Vs[e] = a.Vsel[(int64_t)i * VSEL + e];
    HV[e] = a.HVs[(int64_t)i * PMAX * PMAX + e];
  }
  double* Ys = rbuf;
  double* Xs = rbuf + RB * pq;
  stage_rows(a.Y + a.pad_off[i] * p, ld, r0, rows, p, pq, lrb, Ys);
  stage_rows(a.X + a.pad_off[i] * p, ld, r0, rows, p, pq, lrb, Xs);
  __syncthreads();
  double rn = 0.0;
#pragma unroll 1
  for (int k = 0; k < RB_NPT; ++k) {
    const int e = threadIdx.x + k * EIG_T, r = e & (RB - 1), c = e >> lrb;
    if (c >= m || r >= rows) continue;
    double v = 0.0;
    for (int q = 0; q < p; ++q) v += Ys[r + q * RB] * Vs[c * p + q] - Xs[r + q * RB] * HV[c * p + q];
    rn += v * v;
  }
  rn = adsd::block_sum(rn, red);
  if (threadIdx.x == 0) a.partR[b] = rn;
}

// convergence test and schedule, one thread per subdomain.  Converged: the
// relative residual ||Y V - X H V||_F / min |lambda| is below the tolerance,
// or has stagnated within 100x of it (the rounding floor of the operator on
// strongly non-normal subdomains: three Rayleigh-Ritz steps in a row without a
// 5% gain on the best residual).  The next Rayleigh-Ritz sweep is predicted
// from the residual decay since the last one (1 to 8 sweeps ahead).
__global__ void k_eig_decide(EigArgs a, int nsub, int sw, int final_sweep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsub || a.done[i]) return;
  const int m = a.msel[i];
  double rn = 0.0;
  for (int bb = a.sub_blk0[i]; bb < a.sub_blk0[i + 1]; ++bb) rn += a.partR[bb];
  rn = sqrt(rn);
  const double* lam = a.lam + (int64_t)i * 2 * PMAX;
  double lmin = 1e300;
  for (int c = 0; c < m; ++c) lmin = fmin(lmin, hypot(lam[c], lam[PMAX + c]));
  const double rel = m ? rn / lmin : 0.0;
  const double best = a.rbest[i];
  const bool gain = !(best > 0.0) || rel < 0.95 * best;
  const int stall = (m && !gain) ? a.stall[i] + 1 : 0;
  const bool ok_tol = (m == 0) || (rel <= a.tol) || (rel <= 100.0 * a.tol && stall >= 3);
  a.rres[i] = rel;
  if (gain) a.rbest[i] = rel;
  a.stall[i] = stall;
  if (ok_tol || final_sweep) {
    a.done[i] = ok_tol ? 1 : 2;
    a.sweeps[i] = sw + 1;
  }
  int next = 2;
  const double rl = a.rlast[i];
  const int dsw = sw - a.swlast[i];
  if (rl > 0.0 && rel > 0.0 && dsw > 0) {
    const double rate = pow(rel / rl, 1.0 / dsw);
    if (rate < 0.97) {
      const double need = log(a.tol / rel) / log(rate);
      next = need < 1.0 ? 1 : (need > 8.0 ? 8 : (int)ceil(need));
    }
  }
  a.next_rr[i] = sw + next;
  a.rlast[i] = rel;
  a.swlast[i] = sw;
}

// ---------------------------------------------------------------------------
// Block Krylov-Schur.  Per subdomain a block Krylov decomposition
//   T V_k = V_{k+p} Bk,   V_{k+p} = [V_k | V_res] orthonormal, Bk (k+p) x k,
// is expanded block by block (columns jcur .. jcur+p-1 of V through the
// operator, block classical Gram-Schmidt twice against V_{jcur+p}, Cholesky QR
// twice for the new block), then the Rayleigh quotient H = Bk(0:k, 0:k) is
// brought to ordered Schur form (wanted set, then the kept set), convergence
// is judged from the residual block R = Bk(k:k+p, 0:k) on the wanted Schur
// vectors, and otherwise the decomposition is restarted on the kept ones:
//   V <- [V_k U | V_res],  Bk <- [U^T H U ; R U].
// Row-block kernels per expansion step (W = the operator's output block),
// block Gram-Schmidt twice with the QR of the block after each pass:
//   k_ks_dots(0): deferred 1^perp projection of W, partial V^T W
//   k_ks_upd(0): W -= V h1, Bk(:, jcur..) = h1, partial W^T W
//   k_ks_qr(0 .. 2): W = Q1 R_A (shifted Cholesky QR three times)
//   k_ks_dots(1): partial V^T Q1
//   k_ks_upd(1): Q1 -= V h2, Bk(:, jcur..) += h2 R_A, partial Q1^T Q1
//   k_ks_qr(3, 4): Q1 = V_new R_B (Cholesky QR twice), Bk subdiagonal R_B R_A
//   k_ks_advance: jcur += p
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool ks_active(const EigArgs& a, int i) {
  return !a.done[i] && a.jcur[i] + a.p <= a.kmi[i];
}

// partial V^T Y of one row block (pass 0: the operator's output, after the
// deferred projection onto 1^perp; pass 1: the block Q1 of the first pass)
__global__ void __launch_bounds__(EIG_T) k_ks_dots(EigArgs a, int pass) {
  extern __shared__ double rbuf[];
  __shared__ double mu[2][EIG_PC];
  const int b = blockIdx.x, i = a.blk_sub[b];
  if (!ks_active(a, i)) return;
  const int p = a.p, J = a.jcur[i] + p, lrb = a.lrb, RB = 1 << lrb;
  if (J == 0) return;
  const int r0 = a.blk_r0[b], rows = min(RB, a.ni[i] - r0);
  const int64_t ld = (int64_t)a.nb[i] * a.bs[i];
  double* Wg = a.Y + a.pad_off[i] * p;
  const double* Vg = a.V + a.pad_off[i] * (a.km + p);
  double* Ws = rbuf;
  double* Vs = rbuf + RB * EIG_PC;
  stage_rows(Wg, ld, r0, rows, p, EIG_PC, lrb, Ws);
  stage_rows(Vg, ld, r0, rows, J, (J + 3) & ~3, lrb, Vs);
  if (pass == 0 && a.defer && a.kdim[i]) {
    // projection onto K^perp left by the two-ended operator (one column
    // chunk; slots (half, row parity) as k_eig_op_bwd writes them)
    const int kd = a.kdim[i];
    if ((int)threadIdx.x < kd * p) {
      const int par = threadIdx.x / p, j = threadIdx.x % p;
      const double* cs = a.colsum + (int64_t)i * 4 * EIG_PC;
      mu[par][j] = (cs[(0 * 2 + par) * EIG_PC + j] + cs[(1 * 2 + par) * EIG_PC + j]) /
                   (a.ni[i] / kd);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < RB * p; e += EIG_T) {
      const int r = e & (RB - 1), c = e >> lrb;
      if (r < rows) {
        const double v = Ws[e] - mu[kd == 2 ? ((r0 + r) & 1) : 0][c];
        Ws[e] = v;
        Wg[r0 + r + c * ld] = v;
      }
    }
  }
  __syncthreads();
  block_gram_rect(Vs, J, Ws, p, rows, RB, (pass ? a.partK2 : a.partK) + (int64_t)b * KS_PK, p);
}

// Y <- Y - V h with h the summed partial products, and the partial Gram
// matrix of the result.  Coefficients (first block of the subdomain):
// pass 0: Bk(0:J, jcur ..) = h; pass 1: Bk(0:J, jcur ..) += h R_A, where R_A
// is the triangular factor of the first pass's QR.  With no basis yet (the
// start block) only the Gram matrix is formed.
__global__ void __launch_bounds__(EIG_T) k_ks_upd(EigArgs a, int pass) {
  extern __shared__ double rbuf[];
  __shared__ double h[KS_PK];
  __shared__ double tmp[EIG_T];
  const int b = blockIdx.x, i = a.blk_sub[b];
  if (!ks_active(a, i)) return;
  const int p = a.p, jc = a.jcur[i], J = jc + p, lrb = a.lrb, RB = 1 << lrb;
  const int r0 = a.blk_r0[b], rows = min(RB, a.ni[i] - r0);
  const int64_t ld = (int64_t)a.nb[i] * a.bs[i];
  double* Wg = a.Y + a.pad_off[i] * p;
  const double* Vg = a.V + a.pad_off[i] * (a.km + p);
  double* Ws = rbuf;
  double* Vs = rbuf + RB * EIG_PC;
  stage_rows(Wg, ld, r0, rows, p, EIG_PC, lrb, Ws);
  if (J > 0) {
    stage_rows(Vg, ld, r0, rows, J, (J + 3) & ~3, lrb, Vs);
    sum_parts_n(pass ? a.partK2 : a.partK, KS_PK, a.sub_blk0[i], a.sub_blk0[i + 1], J * p, h, tmp);
    if (b == a.sub_blk0[i] && jc >= 0) {
      const double* RA = a.Racc + (int64_t)i * 2 * EIG_PC * EIG_PC;
      for (int e = threadIdx.x; e < J * p; e += EIG_T) {
        const int r = e / p, cc = e % p;
        double* dst = a.Bk + (int64_t)i * KS_BS + (int64_t)r * a.km + jc + cc;
        if (pass == 0) {
          *dst = h[e];
        } else {
          double v = 0.0;
          for (int q = 0; q <= cc; ++q) v += h[r * p + q] * RA[q * p + cc];
          *dst += v;
        }
      }
    }
    for (int e = threadIdx.x; e < RB * EIG_PC; e += EIG_T) {
      const int r = e & (RB - 1), c = e >> lrb;
      if (c < p && r < rows) {
        double v = Ws[e];
        for (int q = 0; q < J; ++q) v -= Vs[r + q * RB] * h[q * p + c];
        Ws[e] = v;
        Wg[r0 + r + c * ld] = v;
      }
    }
  }
  __syncthreads();
  block_gram_rect(Ws, p, Ws, p, rows, RB, a.partA + (int64_t)b * PMAX * PMAX, p);
}

// one Cholesky QR pass of the new block W (p <= EIG_PC columns, in Y) on a
// wide row block (KS_QT threads, KS_QR rows each; W rows held in registers).
// Steps 0..2: shifted Cholesky QR three times of the first Gram-Schmidt
// pass's block (the first Cholesky of G + s I, s = 11 (n p + p (p + 1)) u
// tr(G), as in the shifted CholeskyQR3 of Fukaya, Kannan, Nakatsukasa,
// Yamamoto and Yanagisawa, which stays backward stable when the block is
// numerically rank deficient, e.g. an exhausted Krylov direction); steps 3..4:
// Cholesky QR twice of the second pass's block, the last one into
// V(:, J .. J+p-1).  Steps 0 and 3 read the Gram partials of k_ks_upd (its
// row blocks); the others those of the previous step (these row blocks).  The
// first block of each subdomain accumulates the triangular factors (R_A of
// steps 0..2, R_B of steps 3..4) and finally writes R_B R_A into Bk.
static constexpr int KS_QT = 256;
static constexpr int KS_QR = 4;
static constexpr int KS_QRB = KS_QT * KS_QR;  // rows per block

__global__ void __launch_bounds__(KS_QT) k_ks_qr(EigArgs a, int step) {
  constexpr int PC = EIG_PC;
  __shared__ double Gs[PC * PC];
  __shared__ double Rs[PC * PC];
  __shared__ double Ri[PC * PC];
  __shared__ double tmp[KS_QT];
  __shared__ double wred[KS_QT / 64][10];
  const int b = blockIdx.x, i = a.qblk_sub[b];
  if (!ks_active(a, i)) return;
  const int t = threadIdx.x;
  const int p = a.p, n = a.ni[i];
  const int64_t ld = (int64_t)a.nb[i] * a.bs[i];
  const int jc = a.jcur[i], J = jc + p;
  const int r0 = a.qblk_r0[b];
  double* Y = a.Y + a.pad_off[i] * p;
  double y[KS_QR][PC];
#pragma unroll
  for (int k = 0; k < KS_QR; ++k) {
    const int r = r0 + t + k * KS_QT;
#pragma unroll
    for (int c = 0; c < PC; ++c) y[k][c] = (r < n && c < p) ? Y[r + c * ld] : 0.0;
  }
  const bool from_upd = step == 0 || step == 3;
  const double* gin = from_upd ? a.partA : ((step == 1 || step == 4) ? a.partB : a.partH);
  const int g0 = from_upd ? a.sub_blk0[i] : a.qsub_blk0[i];
  const int g1 = from_upd ? a.sub_blk0[i + 1] : a.qsub_blk0[i + 1];
  {  // Gram matrix: KS_QT / 16 groups of 16 threads over the partials
    const int e = t & 15, g = t >> 4, G = KS_QT / 16;
    double sacc = 0.0;
    for (int bb = g0 + g; bb < g1; bb += G) sacc += gin[(int64_t)bb * PMAX * PMAX + e];
    tmp[t] = sacc;
    __syncthreads();
    if (t < 16) {
      double v = 0.0;
      for (int k = 0; k < G; ++k) v += tmp[k * 16 + t];
      if (t < p * p) Gs[t] = v;
    }
    __syncthreads();
  }
  if (t == 0) {
    const double sh = step == 0 ? ks_shift(Gs, p, n) : 0.0;
    if (!chol_small(Gs, sh, Rs, Ri, p)) atomicOr(a.err, 2);
  }
  __syncthreads();
  if (b == a.qsub_blk0[i] && t < 64) {
    // accumulate R <- R_step R (first step of a chain: R <- R_step)
    double* acc = a.Racc + (int64_t)i * 2 * PC * PC + (step >= 3 ? PC * PC : 0);
    const bool first = step == 0 || step == 3;
    double v = 0.0;
    if (t < p * p) {
      const int r = t / p, cc = t % p;
      if (first)
        v = Rs[t];
      else
        for (int q = r; q <= cc; ++q) v += Rs[r * p + q] * acc[q * p + cc];
    }
    WAVE_SYNC();
    if (t < p * p) acc[t] = v;
    if (step == 4 && jc >= 0 && t < p * p) {
      // subdiagonal block R_B R_A (R_B = v just formed, R_A the other slot)
      __shared__ double RB_[PC * PC];
      RB_[t] = v;
      WAVE_SYNC();
      const double* RA = a.Racc + (int64_t)i * 2 * PC * PC;
      const int r = t / p, cc = t % p;
      double w = 0.0;
      for (int q = r; q <= cc; ++q) w += RB_[r * p + q] * RA[q * p + cc];
      a.Bk[(int64_t)i * KS_BS + (int64_t)(J + r) * a.km + jc + cc] = w;
    }
  }
  double* out = step == 4 ? a.V + a.pad_off[i] * (a.km + p) + (int64_t)J * ld : Y;
  double gl[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) gl[q] = 0.0;
#pragma unroll
  for (int k = 0; k < KS_QR; ++k) {
    const int r = r0 + t + k * KS_QT;
    double z[PC];
#pragma unroll
    for (int c = 0; c < PC; ++c) {
      double v = 0.0;
      if (c < p)
#pragma unroll
        for (int q = 0; q <= c; ++q) v += y[k][q] * Ri[q * p + c];
      z[c] = v;
    }
    if (r < n)
#pragma unroll
      for (int c = 0; c < PC; ++c)
        if (c < p) out[r + c * ld] = z[c];
    int q = 0;
#pragma unroll
    for (int c1 = 0; c1 < PC; ++c1)
#pragma unroll
      for (int c2 = c1; c2 < PC; ++c2) gl[q++] += z[c1] * z[c2];
  }
  if (step == 2 || step == 4) return;
  // partial Gram of this block: wave butterflies, then the waves in order
#pragma unroll
  for (int q = 0; q < 10; ++q)
    for (int o = 32; o > 0; o >>= 1) gl[q] += __shfl_xor(gl[q], o, 64);
  if ((t & 63) == 0)
#pragma unroll
    for (int q = 0; q < 10; ++q) wred[t >> 6][q] = gl[q];
  __syncthreads();
  if (t < PC * PC) {
    const int c1 = t / PC, c2 = t % PC;
    const int lo = min(c1, c2), hi = max(c1, c2);
    const int q = lo * PC - lo * (lo - 1) / 2 + (hi - lo);
    double v = 0.0;
    for (int w = 0; w < KS_QT / 64; ++w) v += wred[w][q];
    if (c1 < p && c2 < p)
      (step == 0 || step == 3 ? a.partB : a.partH)[(int64_t)b * PMAX * PMAX + c1 * p + c2] = v;
  }
}

__global__ void k_ks_advance(EigArgs a, int nsub) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsub || !ks_active(a, i)) return;
  if (a.jcur[i] >= 0) a.sweeps[i] += 1;
  a.jcur[i] += a.p;
}

// Schur form of the Rayleigh quotient, convergence test and restart data (one
// workgroup per subdomain).  Converged: ||R V1||_F / min |lambda| below the
// tolerance (V1 the wanted Schur basis), or stagnated within 100x of it (three
// restarts without a 5% gain on the best residual).
__global__ void __launch_bounds__(EIG_T) k_ks_rr(EigArgs a, int final_cycle) {
  __shared__ SmallEigLds se;
  __shared__ double H[PMAX * PMAX];
  __shared__ double Rb[EIG_PC * PMAX];
  __shared__ double V2[PMAX * PMAX];
  __shared__ double lam_re[PMAX], lam_im[PMAX];
  __shared__ double red[16];
  __shared__ int flag[4];
  const int i = blockIdx.x;
  if (a.done[i]) return;
  const int t = threadIdx.x;
  const int p = a.p, km = a.km, m = a.jcur[i];
  double* B = a.Bk + (int64_t)i * KS_BS;
  for (int e = t; e < m * m; e += EIG_T) H[e] = B[(e / m) * km + e % m];
  for (int e = t; e < p * m; e += EIG_T) Rb[e] = B[(m + e / m) * km + e % m];
  __syncthreads();
  if (t < 64) {
    int ok = 1, mk = 0;
    double gap = 1.0;
    const int m1 = small_eig_select(m, H, a.nev - a.kdim[i], a.tau, se, lam_re, lam_im, &ok, &gap,
                                    a.kkeepi[i] - a.kdim[i], &mk, V2, a.pair);
    if (t == 0) {
      flag[0] = m1;
      flag[1] = ok;
      flag[2] = mk;
    }
  }
  __syncthreads();
  const int m1 = flag[0], mk = flag[2];
  double r2 = 0.0;
  for (int e = t; e < p * m1; e += EIG_T) {
    const int r = e % p, cc = e / p;
    double v = 0.0;
    for (int k = 0; k < m; ++k) v += Rb[r * m + k] * se.V[cc * m + k];
    r2 += v * v;
  }
  r2 = adsd::block_sum(r2, red);
  if (t == 0) {
    if (!flag[1]) atomicOr(a.err, 4);
    double lmin = 1e300;
    for (int cc = 0; cc < m1; ++cc) lmin = fmin(lmin, hypot(lam_re[cc], lam_im[cc]));
    const double rel = m1 ? sqrt(r2) / lmin : 0.0;
    const double best = a.rbest[i];
    const bool gain = !(best > 0.0) || rel < 0.95 * best;
    const int stall = (m1 && !gain) ? a.stall[i] + 1 : 0;
    const bool ok_tol = (m1 == 0) || (rel <= a.tol) || (rel <= 100.0 * a.tol && stall >= 3);
    a.rres[i] = rel;
    if (gain) a.rbest[i] = rel;
    a.stall[i] = stall;
    int fin = 0;
    if (ok_tol || final_cycle) fin = ok_tol ? 1 : 2;
    // the wanted cluster must leave a Ritz value outside it, and a restart
    // must leave room for at least one more block
    if (m1 >= m || (!fin && (mk > a.kmi[i] - p || mk < m1))) {
      atomicOr(a.err, 16);
      fin = 2;
    }
    if (fin) a.done[i] = fin;
    a.msel[i] = m1;
    flag[3] = fin;
  }
  __syncthreads();
  if (flag[3]) {
    // Ritz basis in V coordinates, zero below row m (stride km + p)
    const int ldv = km + p;
    double* Vs = a.Vsel + (int64_t)i * VSEL;
    for (int e = t; e < ldv * m1; e += EIG_T) {
      const int r = e % ldv, cc = e / ldv;
      Vs[e] = r < m ? se.V[cc * m + r] : 0.0;
    }
    double* lam = a.lam + (int64_t)i * 2 * PMAX;
    for (int cc = t; cc < m1; cc += EIG_T) {
      lam[cc] = lam_re[cc];
      lam[PMAX + cc] = lam_im[cc];
    }
    return;
  }
  // restart on the kept Schur basis U = V2 (m x mk): HU in se.Pm
  for (int e = t; e < m * mk; e += EIG_T) {
    const int r = e % m, cc = e / m;
    double v = 0.0;
    for (int k = 0; k < m; ++k) v += H[r * m + k] * V2[cc * m + k];
    se.Pm[e] = v;
    a.Ures[(int64_t)i * PMAX * PMAX + e] = V2[e];
  }
  __syncthreads();
  for (int e = t; e < (km + p) * km; e += EIG_T) {
    const int r = e / km, cc = e % km;
    double v = 0.0;
    if (cc < mk && r < mk)
      for (int k = 0; k < m; ++k) v += V2[r * m + k] * se.Pm[cc * m + k];
    else if (cc < mk && r < mk + p)
      for (int k = 0; k < m; ++k) v += Rb[(r - mk) * m + k] * V2[cc * m + k];
    B[e] = v;
  }
  if (t == 0) {
    a.kprev[i] = m;
    a.jcur[i] = mk;
  }
}

// V <- [V_m U | V(:, m .. m+p-1)] on one row block (restarted subdomains)
__global__ void __launch_bounds__(EIG_T) k_ks_restart(EigArgs a) {
  extern __shared__ double rbuf[];
  __shared__ double U[PMAX * PMAX];
  const int b = blockIdx.x, i = a.blk_sub[b];
  if (a.done[i]) return;
  const int p = a.p, m = a.kprev[i], mk = a.jcur[i], lrb = a.lrb, RB = 1 << lrb;
  const int r0 = a.blk_r0[b], rows = min(RB, a.ni[i] - r0);
  const int64_t ld = (int64_t)a.nb[i] * a.bs[i];
  double* Vg = a.V + a.pad_off[i] * (a.km + p);
  double* Vs = rbuf;
  stage_rows(Vg, ld, r0, rows, m + p, (m + p + 3) & ~3, lrb, Vs);
  for (int e = threadIdx.x; e < m * mk; e += EIG_T) U[e] = a.Ures[(int64_t)i * PMAX * PMAX + e];
  __syncthreads();
  for (int e = threadIdx.x; e < RB * (mk + p); e += EIG_T) {
    const int r = e & (RB - 1), cc = e >> lrb;
    if (r >= rows) continue;
    double v;
    if (cc < mk) {
      v = 0.0;
      for (int k = 0; k < m; ++k) v += Vs[r + k * RB] * U[cc * m + k];
    } else {
      v = Vs[r + (m + cc - mk) * RB];
    }
    Vg[r0 + r + cc * ld] = v;
  }
}

// Eigenvalues of eq. 5 on the selected invariant subspace, from the pencil
// itself: with U = X V_sel the Ritz vectors of the subdomain on all n_i local
// rows, H_B = (Pi U)^T B (Pi U) (Pi symmetric, so this is U^T Pi B Pi U) and
// H_A = U^T Atilde U are formed with sparse products only (A_ii's local CSR,
// the lumped sums of Definition 1, the unit left null vector ell of a
// floating subdomain: Pi u = u - ell (ell^T u)), and the reported eigenvalues
// are those of H_A^{-1} H_B (the Galerkin projection of the pencil onto
// span U; exact when span U is invariant).  The operator's own Rayleigh
// quotient carries the forward error of the solves with the regularised
// splitting, which grows with its conditioning; span U, hence the coarse
// space, is unchanged.  One workgroup per subdomain; U is written to ubuf
// (column stride npad), thread (a, b) accumulates entry (a, b) of both
// matrices over row blocks of RR_B rows staged in LDS.
static constexpr int RR_B = EIG_T / PMAX;
__global__ void __launch_bounds__(EIG_T)
k_eig_rayleigh(EigArgs a, const double* __restrict__ lsum, double* __restrict__ ubuf) {
  __shared__ SmallEigLds se;
  __shared__ double Ub[RR_B][PMAX + 1], Vb[RR_B][PMAX + 1], YA[RR_B][PMAX + 1], YB[RR_B][PMAX + 1];
  __shared__ double G[PMAX][2 * PMAX + 1];
  __shared__ double M[PMAX * PMAX];
  __shared__ double pu[2][PMAX], red[PMAX][EIG_T / 64];
  __shared__ double lam_re[PMAX], lam_im[PMAX];
  __shared__ int flag[2];
  const int i = blockIdx.x, t = threadIdx.x;
  const int m = a.msel[i];
  if (m <= 0) return;
  const int p = a.p, ni = a.ni[i], kd = a.kdim[i];
  const int64_t ld = (int64_t)a.nb[i] * a.bs[i];
  const double* X = a.X + a.pad_off[i] * p;
  const double* Vs = a.Vsel + (int64_t)i * VSEL;
  double* U = ubuf + a.pad_off[i] * p;
  const double* ell = a.ell + a.pad_off[i];
  const int64_t f0 = a.om_off[i];
  const uint8_t* isint = a.om_int + f0;
  // U = X V_sel on every local row
  for (int e = t; e < ni * m; e += EIG_T) {
    const int r = e % ni, c = e / ni;
    double v = 0.0;
    for (int j = 0; j < p; ++j) v += X[r + j * ld] * Vs[c * p + j];
    U[r + c * ld] = v;
  }
  __syncthreads();
  // pu = ell^T U (floating subdomains), and (J ell)^T U for complex A
  if (t < PMAX) pu[0][t] = pu[1][t] = 0.0;
  for (int q = 0; q < kd; ++q) {
    double acc[PMAX];
#pragma unroll
    for (int c = 0; c < PMAX; ++c) acc[c] = 0.0;
    for (int r = t; r < ni; r += EIG_T) {
      const double l = q ? jrot(ell, r) : ell[r];
#pragma unroll
      for (int c = 0; c < PMAX; ++c)
        if (c < m) acc[c] += l * U[r + c * ld];
    }
#pragma unroll
    for (int c = 0; c < PMAX; ++c) {
      double v = acc[c];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if ((t & 63) == 0) red[c][t >> 6] = v;
    }
    __syncthreads();
    if (t < m) {
      double v = 0.0;
      for (int w = 0; w < EIG_T / 64; ++w) v += red[t][w];
      pu[q][t] = v;
    }
    __syncthreads();
  }
  __syncthreads();
  const int aa = t / PMAX, bb = t % PMAX;
  double ha = 0.0, hb = 0.0;
  for (int r0 = 0; r0 < ni; r0 += RR_B) {
    {
      const int rr = t / PMAX, c = t % PMAX, r = r0 + rr;  // one (row, column) per thread
      double u = 0.0, v = 0.0, ya = 0.0, yb = 0.0;
      if (r < ni && c < m) {
        const double pc = kd ? pu[0][c] : 0.0, pc2 = kd == 2 ? pu[1][c] : 0.0;
        u = U[r + c * ld];
        v = u - (kd ? ell[r] * pc : 0.0);
        if (kd == 2) v -= jrot(ell, r) * pc2;
        const bool ri = isint[r];
        for (int64_t q = a.lrow[f0 + r]; q < a.lrow[f0 + r + 1]; ++q) {
          const int cc = a.lcol[q];
          const double av = a.lval[q], uc = U[cc + c * ld];
          ya += av * uc;
          if (ri && isint[cc]) {
            double w = uc - (kd ? ell[cc] * pc : 0.0);
            if (kd == 2) w -= jrot(ell, cc) * pc2;
            yb += av * w;
          }
        }
        if (!ri) ya -= lsum[f0 + r] * u;
      }
      Ub[rr][c] = u;
      Vb[rr][c] = v;
      YA[rr][c] = ya;
      YB[rr][c] = yb;
    }
    __syncthreads();
    if (aa < m && bb < m)
      for (int rr = 0; rr < RR_B; ++rr) {
        ha += Ub[rr][aa] * YA[rr][bb];
        hb += Vb[rr][aa] * YB[rr][bb];
      }
    __syncthreads();
  }
  if (aa < m && bb < m) {
    G[aa][bb] = ha;
    G[aa][m + bb] = hb;
  }
  __syncthreads();
  if (t < 64) {  // wave 0: [H_A | H_B] -> [I | H_A^{-1} H_B], partial pivoting
    const int lane = t;
    int ok = 1;
    for (int k = 0; k < m; ++k) {
      double cand = (lane < m && lane >= k) ? fabs(G[lane][k]) : -1.0;
      if (!(cand >= 0.0)) cand = -1.0;
      double mx = cand;
      for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
      const unsigned long long hit = __ballot(cand == mx);
      const int pr = __ffsll((long long)hit) - 1;
      if (!(mx > 0.0)) ok = 0;
      if (pr != k)
        for (int j = lane; j < 2 * m; j += 64) {
          const double x = G[k][j];
          G[k][j] = G[pr][j];
          G[pr][j] = x;
        }
      WAVE_SYNC();
      const double piv = G[k][k];
      const double inv = piv != 0.0 ? 1.0 / piv : 0.0;
      WAVE_SYNC();
      for (int j = lane; j < 2 * m; j += 64) G[k][j] *= inv;
      WAVE_SYNC();
      for (int r = 0; r < m; ++r) {
        if (r == k) continue;
        const double f = G[r][k];
        WAVE_SYNC();
        for (int j = lane; j < 2 * m; j += 64) G[r][j] -= f * G[k][j];
        WAVE_SYNC();
      }
    }
    for (int e = lane; e < m * m; e += 64) M[e] = G[e / m][m + e % m];
    WAVE_SYNC();
    int ok2 = 1;
    double gap = 1.0;
    const int got = small_eig_select(m, M, m, 0.0, se, lam_re, lam_im, &ok2, &gap);
    if (lane == 0) flag[0] = ok && ok2 && got == m;
  }
  __syncthreads();
  if (flag[0] && t < m) {
    double* lam = a.lam + (int64_t)i * 2 * PMAX;
    lam[t] = lam_re[t];
    lam[PMAX + t] = lam_im[t];
  }
}

// W_i = orth([1_I (floating; complex A: 1_I and J 1_I) | (X V)_I]) stored
// row-major nI x nev_i
// Z = [1 | X V] on the interior rows of every subdomain, column-major nint x
// cols in the Y buffer (leading dimension npad): one thread per interior row
// (its local row from the window map), the row of X in registers, the Ritz
// coefficients V in LDS
static constexpr int EZ_T = 256;
__global__ void __launch_bounds__(EZ_T)
k_eig_z(EigArgs a, const int32_t* __restrict__ int_list, const int64_t* __restrict__ wlo,
        const int64_t* __restrict__ woff, const int32_t* __restrict__ wpos) {
  __shared__ double Vsh[VSEL];
  const int i = blockIdx.x;
  const int nint = a.nI[i];
  const int k = blockIdx.y * EZ_T + threadIdx.x;
  if (blockIdx.y * EZ_T >= nint) return;
  const int p = a.p, m = a.msel[i], kd = a.kdim[i], cols = m + kd;
  if (cols == 0) return;
  const int64_t ld = (int64_t)a.nb[i] * a.bs[i];
  const double* Vs = a.Vsel + (int64_t)i * VSEL;
  for (int e = threadIdx.x; e < m * p; e += EZ_T) Vsh[e] = Vs[e];
  __syncthreads();
  if (k >= nint) return;
  const int g = int_list[a.om_off[i] + k];
  const int r = wpos[woff[i] + (g - wlo[i])];
  const double* X = a.X + a.pad_off[i] * p;
  double xr[KS_W];
#pragma unroll
  for (int j = 0; j < KS_W; ++j) xr[j] = j < p ? X[r + j * ld] : 0.0;
  double* Z = a.Y + a.pad_off[i] * p;
  if (kd == 1) Z[k] = 1.0;
  if (kd == 2) {  // complex A: the real form of 1 and of i 1 (real, imaginary rows)
    Z[k] = (g & 1) ? 0.0 : 1.0;
    Z[k + ld] = (g & 1) ? 1.0 : 0.0;
  }
  for (int c = 0; c < m; ++c) {
    const double* vc = Vsh + c * p;
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < KS_W; ++j)
      if (j < p) v += xr[j] * vc[j];
    Z[k + (c + kd) * ld] = v;
  }
}

__global__ void __launch_bounds__(EIG_T) k_eig_finish(EigArgs a, const int64_t* W_off, double* W) {
  __shared__ EigShared S;
  const int i = blockIdx.x;
  const int p = a.p;
  const int nint = a.nI[i];
  const int64_t ld = (int64_t)a.nb[i] * a.bs[i];
  const int m = a.msel[i];
  const int kd = a.kdim[i];
  const int cols = m + kd;
  if (cols == 0) return;
  // Z (interior rows, column-major nint x cols) in the Y buffer, formed by k_eig_z
  double* Z = a.Y + a.pad_off[i] * p;
  // orthonormalise the nint x cols block (Cholesky QR twice, in place)
  const int okz = cholqr2(Z, Z, ld, nint, nint, cols, S);
  if (!okz && threadIdx.x == 0) atomicOr(a.err, 8);
  double* Wi = W + W_off[i];
  for (int64_t e = threadIdx.x; e < (int64_t)nint * cols; e += blockDim.x) {
    const int r = (int)(e / cols), c = (int)(e % cols);
    Wi[e] = Z[r + c * ld];
  }
}

template <class FT>
static void eig_run(Ctx& c, EigArgs& a, const FT* fac) {
  hipStream_t st = c.stream;
  const int nsub = c.nsub;
  int smax = *std::max_element(c.h_bs.begin(), c.h_bs.end());
  double* scratch = nullptr;
  if (2 * smax > 4096) fail(ADS_ERR_UNSUPPORTED, "block size too large for the eigensolver");
  // the coupling-list transposed solve reads the two-ended tiles of the fast
  // path; the general path's one-ended tiles take the CSR form
  const bool cpl = c.solve_fast && c.cpl_ok && c.ucpl_row != nullptr;
  const size_t init_lds =
      cpl ? (size_t)(2 * smax + EIG_T + (smax * adsd::NCPL + 1) / 2 + smax * adsd::NCPL + 8) * 8
          : (size_t)2 * smax * sizeof(double);
  const int pq = (a.p + 3) & ~3;
  const size_t rb_lds = (size_t)2 * (1 << a.lrb) * pq * sizeof(double);
  const unsigned nblk = (unsigned)c.h_eig_nblk;
  auto orth = [&]() {
    ADS_LAUNCH(k_eig_gram, dim3(nblk), dim3(EIG_T), rb_lds, st, a, 0);
    ADS_LAUNCH(k_eig_orth, dim3(nblk), dim3(EIG_T), rb_lds, st, a, 0);
    ADS_LAUNCH(k_eig_orth, dim3(nblk), dim3(EIG_T), rb_lds, st, a, 1);
  };
  if (cpl && !a.sym) {
    const size_t ell_lds = (size_t)(smax + EIG_T) * sizeof(double);
    ADS_LAUNCH((k_eig_ell<FT>), dim3(nsub, 2), dim3(EIG_T), ell_lds, st, fac, a, 0);
    ADS_LAUNCH((k_eig_ell<FT>), dim3(nsub, 1), dim3(EIG_T), ell_lds, st, fac, a, 1);
    ADS_LAUNCH((k_eig_ell<FT>), dim3(nsub, 2), dim3(EIG_T), ell_lds, st, fac, a, 2);
    ADS_LAUNCH((k_eig_init<FT, true>), dim3(nsub), dim3(EIG_T), init_lds, st, fac, a, scratch);
  } else
    ADS_LAUNCH((k_eig_init<FT, false>), dim3(nsub), dim3(EIG_T), init_lds, st, fac, a, scratch);
  orth();
  constexpr int PC = EIG_PC;
  const bool fast = c.solve_fast;
  size_t op_lds = fast ? (size_t)adsd::solve_lds_doubles<PC>(c.h_bs, adsd::SOLVE_T) * sizeof(double)
                       : (size_t)adsd::solve_lds_doubles_general<PC>(c.h_bs, EIG_T) * sizeof(double);
  const unsigned nch = (unsigned)((a.p + PC - 1) / PC);
  if (fast)
    ADS_LAUNCH(k_eig_btl, dim3(nsub, (unsigned)((npad_max(c) + 255) / 256)), dim3(256), 0, st, a,
               c.om_sorted, c.rowptr, c.col, c.val, c.tptr, c.tcol, c.wlo, c.whi, c.woff, c.wpos);
  int maxsw = c.opt.eig_max_sweeps > 0 ? c.opt.eig_max_sweeps : 400;
  if (a.x0) maxsw = std::min(maxsw, WARM_SWEEPS);  // then the cold fallback
  std::vector<int32_t> hdone(nsub, 0), hnext(nsub, 0), hint;
  int next = 3;  // first Rayleigh-Ritz step after 4 sweeps
  for (int sw = 0; sw < maxsw; ++sw) {
    if (fast) {
      constexpr int D = 2;
      ADS_LAUNCH((k_eig_op_fwd<FT, PC, D>), dim3(nsub, nch, 2), dim3(adsd::SOLVE_T), op_lds, st,
                 fac, a);
      ADS_LAUNCH((k_eig_op_bwd<FT, PC, D>), dim3(nsub, nch, 2), dim3(adsd::SOLVE_T), op_lds, st,
                 fac, a);
    } else {
      ADS_LAUNCH((k_eig_op<FT, PC>), dim3(nsub, nch), dim3(EIG_T), op_lds, st, fac, a);
    }
    const bool last = sw == maxsw - 1;
    if (sw < next && !last) {
      orth();
      continue;
    }
    ADS_LAUNCH(k_eig_gram, dim3(nblk), dim3(EIG_T), rb_lds, st, a, 1);
    ADS_LAUNCH(k_eig_rr, dim3(nsub), dim3(EIG_T), 0, st, a);
    ADS_LAUNCH(k_eig_resid, dim3(nblk), dim3(EIG_T), rb_lds, st, a);
    ADS_LAUNCH(k_eig_decide, dim3((nsub + 63) / 64), dim3(64), 0, st, a, nsub, sw, (int)last);
    // err | done | sweeps | msel | jcur | next_rr in one copy
    download(hint, a.err, 1 + 5 * (size_t)nsub, st);
    for (int i = 0; i < nsub; ++i) {
      hdone[i] = hint[1 + i];
      hnext[i] = hint[1 + 4 * nsub + i];
    }
    // next check when the slowest unconverged subdomain is predicted to
    // converge (the others keep iterating meanwhile)
    bool all = true;
    next = sw + 1;
    for (int i = 0; i < nsub; ++i)
      if (hdone[i] == 0) {
        all = false;
        next = std::max(next, hnext[i]);
      }
    if (all) break;
    ADS_LAUNCH(k_eig_orth, dim3(nblk), dim3(EIG_T), rb_lds, st, a, 0);
    ADS_LAUNCH(k_eig_orth, dim3(nblk), dim3(EIG_T), rb_lds, st, a, 1);
  }
  ADS_HIP(hipStreamSynchronize(st));
}

// Learned coarse space: per subdomain the interior rows of [1 (floating
// subdomains: the kernel part) | the network's block] orthonormalised by
// Cholesky QR twice (one block each)
__global__ void __launch_bounds__(EIG_T) k_learned_coarse(const int64_t* om_off,
                                                          const uint8_t* om_int,
                                                          const int32_t* nI, const int32_t* kdim,
                                                          const float* X, int kx,
                                                          const int64_t* W_off, double* W,
                                                          double* Zbuf, int32_t* err) {
  __shared__ EigShared S;
  __shared__ int wtot[EIG_T / 64];
  const int i = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t b = om_off[i];
  const int n = (int)(om_off[i + 1] - b), nint = nI[i];
  const int kd = kdim[i], k = kx + kd;  // the kernel part (constant) leads, as in eq. 6
  double* Z = Zbuf + W_off[i];  // nint x k, column-major
  int run = 0;
  for (int r0 = 0; r0 < n; r0 += EIG_T) {
    const int r = r0 + t;
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
    for (int q = 0; q < EIG_T / 64; ++q) {
      if (q < wv) off += wtot[q];
      tot += wtot[q];
    }
    if (f) {
      const int q = run + off + incl - 1;
      if (kd) Z[q] = 1.0;
      for (int c = 0; c < kx; ++c) Z[q + (int64_t)(c + kd) * nint] = X[(b + r) * kx + c];
    }
    run += tot;
  }
  __syncthreads();
  const int ok = cholqr2(Z, Z, nint, nint, nint, k, S);
  if (!ok && t == 0) atomicOr(err, 1);
  double* Wi = W + W_off[i];
  for (int64_t e = t; e < (int64_t)nint * k; e += EIG_T) {
    const int r = (int)(e / k), c = (int)(e % k);
    Wi[e] = Z[r + (int64_t)c * nint];
  }
}

// the coarse layout and W from the learned block (c.gnn_x, c.gnn_cols
// columns); false if a subdomain's block is not of full rank
static bool learned_coarse(Ctx& c) {
  hipStream_t st = c.stream;
  const int nsub = c.nsub, k = c.gnn_cols;
  c.h_nev.resize(nsub);
  c.h_coff.assign(nsub + 1, 0);
  c.h_W_off.assign(nsub + 1, 0);
  for (int i = 0; i < nsub; ++i) {
    c.h_nev[i] = k + c.h_kdim[i];
    if (c.h_nI[i] < c.h_nev[i] || c.h_nev[i] > PMAX) return false;
    c.h_coff[i + 1] = c.h_coff[i] + c.h_nev[i];
    c.h_W_off[i + 1] = c.h_W_off[i] + (int64_t)c.h_nI[i] * c.h_nev[i];
  }
  double* W = c.mem.alloc<double>(std::max<int64_t>(c.h_W_off[nsub], 1));
  double* Zb = c.mem.alloc<double>(std::max<int64_t>(c.h_W_off[nsub], 1));
  int64_t* Woff = upload(c.mem, c.h_W_off.data(), nsub + 1, st);
  int32_t* err = c.mem.alloc<int32_t>(1);
  ADS_HIP(hipMemsetAsync(err, 0, 4, st));
  ADS_LAUNCH(k_learned_coarse, dim3(nsub), dim3(EIG_T), 0, st, c.om_off, c.om_int, c.nI, c.kdim,
             c.gnn_x, k, Woff, W, Zb, err);
  std::vector<int32_t> he;
  download(he, err, 1, st);
  c.mem.release(Zb);
  if (he[0]) {
    c.mem.release(W);
    return false;
  }
  c.W = W;
  c.W_off = Woff;
  c.n0 = c.h_coff[nsub];
  c.nev = upload(c.mem, c.h_nev.data(), nsub, st);
  c.coff = upload(c.mem, c.h_coff.data(), nsub + 1, st);
  c.h_lam_re.assign(c.n0, 0.0);  // no eigenvalues: the space is predicted
  c.h_lam_im.assign(c.n0, 0.0);
  c.h_sweeps.assign(nsub, 0);
  c.h_eig_res.assign(nsub, 0.0);
  c.eig_sweeps_max = 0;
  c.eig_unconverged = 0;
  c.eig_krylov_schur = false;
  return true;
}

// block Krylov-Schur driver (block width a.p = EIG_PC)
template <class FT>
static void eig_run_ks(Ctx& c, EigArgs& a, const FT* fac) {
  hipStream_t st = c.stream;
  const int nsub = c.nsub;
  int smax = *std::max_element(c.h_bs.begin(), c.h_bs.end());
  double* scratch = nullptr;
  if (2 * smax > 4096) fail(ADS_ERR_UNSUPPORTED, "block size too large for the eigensolver");
  // the coupling-list transposed solve reads the two-ended tiles of the fast
  // path; the general path's one-ended tiles take the CSR form
  const bool cpl = c.solve_fast && c.cpl_ok && c.ucpl_row != nullptr;
  const size_t init_lds =
      cpl ? (size_t)(2 * smax + EIG_T + (smax * adsd::NCPL + 1) / 2 + smax * adsd::NCPL + 8) * 8
          : (size_t)2 * smax * sizeof(double);
  const int RB = 1 << a.lrb;
  const unsigned nqblk = (unsigned)c.h_eig_nqblk;
  const size_t ks_lds = (size_t)RB * (EIG_PC + KS_W) * sizeof(double);
  const unsigned nblk = (unsigned)c.h_eig_nblk;
  const unsigned g64 = (unsigned)((nsub + 63) / 64);
  constexpr int PC = EIG_PC;
  const bool fast = c.solve_fast;
  const size_t op_lds =
      fast ? (size_t)adsd::solve_lds_doubles<PC>(c.h_bs, adsd::SOLVE_T) * sizeof(double)
           : (size_t)adsd::solve_lds_doubles_general<PC>(c.h_bs, EIG_T) * sizeof(double);
  if (cpl && !a.sym) {
    const size_t ell_lds = (size_t)(smax + EIG_T) * sizeof(double);
    ADS_LAUNCH((k_eig_ell<FT>), dim3(nsub, 2), dim3(EIG_T), ell_lds, st, fac, a, 0);
    ADS_LAUNCH((k_eig_ell<FT>), dim3(nsub, 1), dim3(EIG_T), ell_lds, st, fac, a, 1);
    ADS_LAUNCH((k_eig_ell<FT>), dim3(nsub, 2), dim3(EIG_T), ell_lds, st, fac, a, 2);
    ADS_LAUNCH((k_eig_init<FT, true>), dim3(nsub), dim3(EIG_T), init_lds, st, fac, a, scratch);
  } else
    ADS_LAUNCH((k_eig_init<FT, false>), dim3(nsub), dim3(EIG_T), init_lds, st, fac, a, scratch);
  if (fast)
    ADS_LAUNCH(k_eig_btl, dim3(nsub, (unsigned)((npad_max(c) + 255) / 256)), dim3(256), 0, st, a,
               c.om_sorted, c.rowptr, c.col, c.val, c.tptr, c.tcol, c.wlo, c.whi, c.woff, c.wpos);
  // block classical Gram-Schmidt twice of the operator's output against V,
  // each pass followed by the QR of the block (Barlow-Smoktunowicz BCGS2)
  auto orth_block = [&]() {
    ADS_LAUNCH(k_ks_dots, dim3(nblk), dim3(EIG_T), ks_lds, st, a, 0);
    ADS_LAUNCH(k_ks_upd, dim3(nblk), dim3(EIG_T), ks_lds, st, a, 0);
    for (int q = 0; q < 3; ++q) ADS_LAUNCH(k_ks_qr, dim3(nqblk), dim3(KS_QT), 0, st, a, q);
    ADS_LAUNCH(k_ks_dots, dim3(nblk), dim3(EIG_T), ks_lds, st, a, 1);
    ADS_LAUNCH(k_ks_upd, dim3(nblk), dim3(EIG_T), ks_lds, st, a, 1);
    for (int q = 3; q < 5; ++q) ADS_LAUNCH(k_ks_qr, dim3(nqblk), dim3(KS_QT), 0, st, a, q);
    ADS_LAUNCH(k_ks_advance, dim3(g64), dim3(64), 0, st, a, nsub);
  };
  auto step = [&]() {
    if (fast) {
      constexpr int D = 2;
      ADS_LAUNCH((k_eig_op_fwd<FT, PC, D>), dim3(nsub, 1, 2), dim3(adsd::SOLVE_T), op_lds, st, fac,
                 a);
      ADS_LAUNCH((k_eig_op_bwd<FT, PC, D>), dim3(nsub, 1, 2), dim3(adsd::SOLVE_T), op_lds, st, fac,
                 a);
    } else {
      ADS_LAUNCH((k_eig_op<FT, PC>), dim3(nsub, 1), dim3(EIG_T), op_lds, st, fac, a);
    }
    orth_block();
  };
  orth_block();  // start block into V(:, 0 .. p-1)
  const int maxsteps = c.opt.eig_max_sweeps > 0 ? c.opt.eig_max_sweeps : 400;
  std::vector<int32_t> hdone(nsub, 0), hj(nsub, 0), hint;
  int total = 0;
  for (int cyc = 0;; ++cyc) {
    int nst = 0;
    for (int i = 0; i < nsub; ++i)
      if (!hdone[i] && hj[i] + a.p <= c.h_eig_km[i])
        nst = std::max(nst, (c.h_eig_km[i] - a.p - hj[i]) / a.p + 1);
    for (int k = 0; k < nst; ++k) step();
    total += nst;
    ADS_LAUNCH(k_ks_rr, dim3(nsub), dim3(EIG_T), 0, st, a, (int)(total >= maxsteps));
    // err | done | sweeps | msel | jcur in one copy
    download(hint, a.err, 1 + 4 * (size_t)nsub, st);
    bool all = true;
    for (int i = 0; i < nsub; ++i) {
      hdone[i] = hint[1 + i];
      hj[i] = hint[1 + 3 * nsub + i];
      all &= hdone[i] != 0;
    }
    if (all) break;
    ADS_LAUNCH(k_ks_restart, dim3(nblk), dim3(EIG_T), ks_lds, st, a);
  }
  ADS_HIP(hipStreamSynchronize(st));
}

// eigenpairs the eigensolver resolves per subdomain (kernel part included):
// a Rayleigh quotient of order PMAX with room for two expansion blocks
static constexpr int NEV_SOLVE_MAX = PMAX - 2 * EIG_PC;

void eigensolve(Ctx& c) {
  hipStream_t st = c.stream;
  const int nsub = c.nsub;
  // with the tau rule of eq. 6, opt.nev is a cap (up to 60); the eigensolver
  // resolves at most NEV_SOLVE_MAX of them and the rule keeps those above
  // 1/tau; a subdomain where even the last resolved one is kept would need
  // more, and is refused below instead of being truncated
  const int nev_cap = c.opt.nev;
  const bool tau_cap = c.opt.tau > 0 && nev_cap > NEV_SOLVE_MAX;
  const int nev = tau_cap ? NEV_SOLVE_MAX : nev_cap;
  if (c.gnn_x && c.opt.warm_start == 2) {
    // learned coarse space: the network's block itself, orthonormalised
    if (learned_coarse(c)) return;
    c.eig_fallbacks = nsub;  // a rank-deficient prediction: exact eigensolve
    c.gnn_x = nullptr;
  }
  // learned warm start: the exact eigensolve (Krylov-Schur or block
  // subspace iteration) started from the network's block, with the exact
  // cold eigensolve as the fallback
  const bool warm = c.gnn_x && c.opt.warm_start == 1;
  // block subspace iteration: block of p columns
  int p = std::min(PMAX, std::max(2 * nev, nev + 8));
  p = (p + 3) / 4 * 4;
  p = std::min(p, PMAX);
  int minfree = 1 << 30;
  for (int i = 0; i < nsub; ++i) minfree = std::min(minfree, c.h_ni[i] - c.h_kdim[i] - 1);
  p = std::min(p, minfree);
  // block Krylov-Schur: Rayleigh quotients up to km, restarts keep kkeep
  // (before the cluster rule); the basis must fit in the range of the
  // operator (interior rows) of every subdomain
  // (a larger basis means fewer restarts, each with one dense Schur
  // decomposition per subdomain: on 2D convection-diffusion subdomains with
  // nev 8, order 32 keeping 16 converges in the fewest block steps; with
  // nev 12 on 3D coefficient-jump subdomains, keeping nev + 4 = 16 instead of
  // 2 nev = 24 halves the restarts and their Schur decompositions for a few
  // more block steps, a net saving)
  // per subdomain, so that a small subdomain does not shorten the basis of
  // the others (the storage takes the largest order)
  const int km = std::min(PMAX, std::max(4 * nev, nev + 24));
  std::vector<int32_t> h_km(nsub), h_kkeep(nsub);
  bool ks_fits = true;
  for (int i = 0; i < nsub; ++i) {
    const int ki = std::min(km, std::min(c.h_nI[i], c.h_ni[i] - EIG_PC) - c.h_kdim[i] - 1);
    const int kk = std::min(std::max(nev + 4, ki / 2), ki - 2 * EIG_PC);
    h_km[i] = ki;
    h_kkeep[i] = kk;
    ks_fits = ks_fits && ki >= nev + 2 * EIG_PC && kk >= nev && kk + EIG_PC <= ki;
  }
  const bool ks = !c.eig_ks_lost_rank && c.opt.eig_solver == ADS_EIG_KRYLOV_SCHUR && ks_fits;
  if (!ks && p < nev + 1)
    fail(ADS_ERR_UNSUPPORTED, "nev too large for the smallest subdomain or for the eigensolver");
  c.eig_krylov_schur = ks;
  const int pw = ks ? EIG_PC : p;  // columns per operator application
  const int ncol = ks ? km + EIG_PC : p;  // columns of the basis / output blocks
  EigArgs a{};
  a.fac_off = c.fac_off;
  a.bs = c.bs;
  a.nb = c.nb;
  a.ni = c.ni;
  a.nI = c.nI;
  a.om_off = c.om_off;
  a.om_int = c.om_int;
  a.lrow = c.lptr_off;
  a.lcol = c.lcol;
  a.lval = c.lval;
  a.kdim = c.kdim;
  a.pad_off = c.pad_off;
  a.cpl_col = c.cpl_col;
  a.cpl_val = c.cpl_val;
  a.cpl_ok = c.cpl_ok ? 1 : 0;
  a.rcpl_col = c.rcpl_col;
  a.rcpl_val = c.rcpl_val;
  a.ucpl_row = c.ucpl_row;
  a.ucpl_val = c.ucpl_val;
  a.lcpl_row = c.lcpl_row;
  a.lcpl_val = c.lcpl_val;
  const int nch = (pw + EIG_PC - 1) / EIG_PC;
  a.dummy = c.mem.alloc<double>((size_t)nsub * nch * 2 * 1024);
  if (ks) {
    a.V = c.mem.alloc<double>((size_t)c.npad_total * ncol);
    a.X = a.V;
    ADS_HIP(hipMemsetAsync(a.V, 0, (size_t)c.npad_total * ncol * 8, st));
  } else {
    a.X = c.mem.alloc<double>((size_t)c.npad_total * p);
    ADS_HIP(hipMemsetAsync(a.X, 0, (size_t)c.npad_total * p * 8, st));
  }
  a.Y = c.mem.alloc<double>((size_t)c.npad_total * ncol);
  a.W = c.solve_fast ? c.mem.alloc<double>((size_t)c.npad_total * pw) : nullptr;
  a.ell = c.mem.alloc<double>(c.npad_total);
  a.bell = c.mem.alloc<double>(c.npad_total);
  a.btl = c.mem.alloc<double>(c.npad_total);
  a.gam = c.mem.alloc<double>(2 * (size_t)nsub);
  a.colsum = c.mem.alloc<double>((size_t)nsub * nch * 4 * EIG_PC);
  a.defer = c.solve_fast ? 1 : 0;
  ADS_HIP(hipMemsetAsync(a.colsum, 0, (size_t)nsub * nch * 4 * EIG_PC * 8, st));
  // what the host reads back, in one block (one copy per read):
  // doubles rres | lam, then int32 err | done | sweeps | msel | jcur | next_rr
  const size_t rep_d = (size_t)nsub * (1 + 2 * PMAX), rep_i = 1 + 5 * (size_t)nsub;
  double* rep = c.mem.alloc<double>(rep_d + (rep_i + 1) / 2);
  int32_t* rep_int = reinterpret_cast<int32_t*>(rep + rep_d);
  a.rres = rep;
  a.lam = rep + nsub;
  a.err = rep_int;
  a.done = rep_int + 1;
  a.sweeps = rep_int + 1 + nsub;
  a.msel = rep_int + 1 + 2 * nsub;
  a.jcur = rep_int + 1 + 3 * nsub;
  a.next_rr = rep_int + 1 + 4 * nsub;
  a.Vsel = c.mem.alloc<double>((size_t)nsub * VSEL);
  a.rbest = c.mem.alloc<double>(nsub);
  a.stall = c.mem.alloc<int32_t>(nsub);
  ADS_HIP(hipMemsetAsync(a.rbest, 0, nsub * 8, st));
  a.rlast = c.mem.alloc<double>(nsub);
  a.swlast = c.mem.alloc<int32_t>(nsub);
  ADS_HIP(hipMemsetAsync(a.rlast, 0, nsub * 8, st));
  ADS_HIP(hipMemsetAsync(a.swlast, 0, nsub * 4, st));
  a.HVs = ks ? nullptr : c.mem.alloc<double>((size_t)nsub * PMAX * PMAX);
  // row blocks
  a.lrb = ks ? rb_log2(KS_W + EIG_PC) : rb_log2(p);
  std::vector<int32_t> blk_sub, blk_r0, sub_blk0(nsub + 1, 0);
  for (int i = 0; i < nsub; ++i) {
    sub_blk0[i] = (int32_t)blk_sub.size();
    for (int r0 = 0; r0 < c.h_ni[i]; r0 += 1 << a.lrb) {
      blk_sub.push_back(i);
      blk_r0.push_back(r0);
    }
  }
  sub_blk0[nsub] = (int32_t)blk_sub.size();
  c.h_eig_nblk = (int)blk_sub.size();
  a.blk_sub = upload(c.mem, blk_sub.data(), blk_sub.size(), st);
  a.blk_r0 = upload(c.mem, blk_r0.data(), blk_r0.size(), st);
  a.sub_blk0 = upload(c.mem, sub_blk0.data(), nsub + 1, st);
  if (ks) {  // wide row blocks of the block QR passes
    std::vector<int32_t> qb_sub, qb_r0, qsub0(nsub + 1, 0);
    for (int i = 0; i < nsub; ++i) {
      qsub0[i] = (int32_t)qb_sub.size();
      for (int r0 = 0; r0 < c.h_ni[i]; r0 += KS_QRB) {
        qb_sub.push_back(i);
        qb_r0.push_back(r0);
      }
    }
    qsub0[nsub] = (int32_t)qb_sub.size();
    c.h_eig_nqblk = (int)qb_sub.size();
    a.qblk_sub = upload(c.mem, qb_sub.data(), qb_sub.size(), st);
    a.qblk_r0 = upload(c.mem, qb_r0.data(), qb_r0.size(), st);
    a.qsub_blk0 = upload(c.mem, qsub0.data(), nsub + 1, st);
  }
  a.partA = c.mem.alloc<double>((size_t)c.h_eig_nblk * PMAX * PMAX);
  a.partB = c.mem.alloc<double>((size_t)c.h_eig_nblk * PMAX * PMAX);
  a.partH = c.mem.alloc<double>((size_t)c.h_eig_nblk * PMAX * PMAX);
  a.partR = c.mem.alloc<double>(c.h_eig_nblk);
  if (ks) {
    a.ks = 1;
    a.km = km;
    a.kmi = upload(c.mem, h_km.data(), nsub, st);
    c.h_eig_km = h_km;
    a.kkeepi = upload(c.mem, h_kkeep.data(), nsub, st);
    a.Bk = c.mem.alloc<double>((size_t)nsub * KS_BS);
    ADS_HIP(hipMemsetAsync(a.Bk, 0, (size_t)nsub * KS_BS * 8, st));
    std::vector<int32_t> j0(nsub, -EIG_PC);
    ADS_HIP(hipMemcpyAsync(a.jcur, j0.data(), nsub * 4, hipMemcpyHostToDevice, st));
    a.kprev = c.mem.alloc<int32_t>(nsub);
    a.partK = c.mem.alloc<double>((size_t)c.h_eig_nblk * KS_PK);
    a.partK2 = c.mem.alloc<double>((size_t)c.h_eig_nblk * KS_PK);
    a.Ures = c.mem.alloc<double>((size_t)nsub * PMAX * PMAX);
    a.Racc = c.mem.alloc<double>((size_t)nsub * 2 * EIG_PC * EIG_PC);
  }
  ADS_HIP(hipMemsetAsync(a.stall, 0, nsub * 4, st));
  a.p = pw;
  a.x0 = warm ? c.gnn_x : nullptr;
  a.x0_cols = warm ? std::min(c.gnn_cols, pw) : 0;
  a.x0_ld = c.gnn_cols;
  a.x0_mix = (warm && ks) ? 1 : 0;
  a.nev = nev;
  a.tau = c.opt.tau;
  a.tol = c.opt.eig_tol > 0 ? c.opt.eig_tol : (c.prec == ADS_PREC_FP64 ? 1e-10 : 1e-3);
  a.sym = c.sym ? 1 : 0;
  a.pair = c.cplx;
  a.order = c.sub_order;
  ADS_HIP(hipMemsetAsync(a.done, 0, nsub * 4, st));
  ADS_HIP(hipMemsetAsync(a.sweeps, 0, nsub * 4, st));
  ADS_HIP(hipMemsetAsync(a.msel, 0, nsub * 4, st));
  ADS_HIP(hipMemsetAsync(a.err, 0, 4, st));
  ADS_HIP(hipMemsetAsync(a.ell, 0, c.npad_total * 8, st));
  ADS_HIP(hipMemsetAsync(a.bell, 0, c.npad_total * 8, st));
  if (ks) {
    switch (c.prec) {
      case ADS_PREC_FP64: eig_run_ks<double>(c, a, (const double*)c.facT); break;
      case ADS_PREC_FP32: eig_run_ks<float>(c, a, (const float*)c.facT); break;
      default: eig_run_ks<__hip_bfloat16>(c, a, (const __hip_bfloat16*)c.facT); break;
    }
    // the Ritz bases are in V coordinates
    a.X = a.V;
    a.p = ncol;
  } else {
    switch (c.prec) {
      case ADS_PREC_FP64: eig_run<double>(c, a, (const double*)c.facT); break;
      case ADS_PREC_FP32: eig_run<float>(c, a, (const float*)c.facT); break;
      default: eig_run<__hip_bfloat16>(c, a, (const __hip_bfloat16*)c.facT); break;
    }
  }
  std::vector<int32_t> herr, hm, hsw, hdone;
  download(herr, a.err, 1, st);  // (warm fallback and errors first: small)
  auto release_all = [&]() {
    ADS_HIP(hipStreamSynchronize(st));
    for (void* q : {(void*)a.X, (void*)a.Y, (void*)a.W, (void*)a.partA, (void*)a.partB,
                    (void*)a.partH, (void*)a.partR, (void*)a.HVs, (void*)a.btl, (void*)a.colsum,
                    (void*)a.dummy, (void*)a.Bk, (void*)a.partK, (void*)a.partK2, (void*)a.Ures,
                    (void*)a.Racc})
      if (q) c.mem.release(q);
  };
  if (warm) {
    // subspace iteration: every subdomain must reach the tolerance within
    // the warm budget; Krylov-Schur ends as a cold run does, and a start
    // block without rank (a network that predicts nothing) is an error
    download(hdone, a.done, nsub, st);
    int missed = 0;
    if (!ks)
      for (int i = 0; i < nsub; ++i) missed += hdone[i] != 1;
    if (missed || herr[0]) {  // fallback: the exact eigensolve from a cold start
      release_all();
      c.eig_fallbacks = std::max(missed, 1);
      c.gnn_x = nullptr;
      eigensolve(c);
      return;
    }
  }
  if (ks && (herr[0] & 2)) {
    // a new block numerically inside the basis (the Krylov space of a very
    // small subdomain exhausted): the block subspace iteration instead
    release_all();
    c.eig_ks_lost_rank = true;
    c.eig_fallbacks = std::max(c.eig_fallbacks, 1);
    eigensolve(c);
    return;
  }
  if (herr[0] & 4) fail(ADS_ERR_EIG_NOCONV, "small dense eigensolver did not converge");
  if (herr[0] & 16)
    fail(ADS_ERR_UNSUPPORTED,
         "an eigenvalue cluster at the cut fills the eigensolver subspace (e.g. overlap 0)");
  if (herr[0] & 2) fail(ADS_ERR_EIG_NOCONV, "loss of orthogonality in the eigensolver block");
  // the reported eigenvalues from the pencil on the selected subspaces
  ADS_LAUNCH(k_eig_rayleigh, dim3(nsub), dim3(EIG_T), 0, st, a, c.lsum, a.Y);
  // the whole report block in one copy
  std::vector<double> hrep;
  download(hrep, rep, rep_d + (rep_i + 1) / 2, st);
  const int32_t* hi = reinterpret_cast<const int32_t*>(hrep.data() + rep_d);
  hm.assign(hi + 1 + 2 * nsub, hi + 1 + 3 * nsub);
  c.h_sweeps.assign(hi + 1 + nsub, hi + 1 + 2 * nsub);
  c.h_eig_res.assign(hrep.begin(), hrep.begin() + nsub);
  hdone.assign(hi + 1, hi + 1 + nsub);
  c.eig_sweeps_max = 0;
  c.eig_unconverged = 0;
  for (int i = 0; i < nsub; ++i) {
    c.eig_sweeps_max = std::max(c.eig_sweeps_max, c.h_sweeps[i]);
    c.eig_unconverged += (hdone[i] != 1);
  }
  // coarse layout
  c.h_nev.resize(nsub);
  c.h_coff.assign(nsub + 1, 0);
  c.h_W_off.assign(nsub + 1, 0);
  for (int i = 0; i < nsub; ++i) {
    if (hm[i] + c.h_kdim[i] > (ks ? km : p))
      fail(ADS_ERR_UNSUPPORTED, "eigenvalue cluster at the cut exceeds the subspace size in subdomain " +
                                    std::to_string(i));
    c.h_nev[i] = hm[i] + c.h_kdim[i];
    if (tau_cap && c.h_nev[i] >= nev)
      fail(ADS_ERR_UNSUPPORTED, "the tau rule keeps all " + std::to_string(nev) +
                                    " eigenpairs the eigensolver resolves in subdomain " +
                                    std::to_string(i) + " (cap " + std::to_string(nev_cap) +
                                    "); use a smaller tau or nev <= " + std::to_string(nev));
    if (c.h_nev[i] > 32) fail(ADS_ERR_UNSUPPORTED, "more than 32 coarse vectors in one subdomain");
    c.h_coff[i + 1] = c.h_coff[i] + c.h_nev[i];
    c.h_W_off[i + 1] = c.h_W_off[i] + (int64_t)c.h_nI[i] * c.h_nev[i];
  }
  c.n0 = c.h_coff[nsub];
  const double* hlam = hrep.data() + nsub;
  c.h_lam_re.clear();
  c.h_lam_im.clear();
  for (int i = 0; i < nsub; ++i) {
    for (int q = 0; q < c.h_kdim[i]; ++q) {  // the kernel columns
      c.h_lam_re.push_back(0.0);
      c.h_lam_im.push_back(0.0);
    }
    for (int k = 0; k < hm[i]; ++k) {
      c.h_lam_re.push_back(hlam[(size_t)i * 2 * PMAX + k]);
      c.h_lam_im.push_back(hlam[(size_t)i * 2 * PMAX + PMAX + k]);
    }
  }
  c.nev = upload(c.mem, c.h_nev.data(), nsub, st);
  c.coff = upload(c.mem, c.h_coff.data(), nsub + 1, st);
  c.W_off = upload(c.mem, c.h_W_off.data(), nsub + 1, st);
  c.W = c.mem.alloc<double>(std::max<int64_t>(c.h_W_off[nsub], 1));
  {
    int maxint = 1;
    for (int i = 0; i < nsub; ++i) maxint = std::max(maxint, c.h_nI[i]);
    ADS_LAUNCH(k_eig_z, dim3(nsub, (maxint + EZ_T - 1) / EZ_T), dim3(EZ_T), 0, st, a, c.int_list,
               c.wlo, c.woff, c.wpos);
  }
  ADS_LAUNCH(k_eig_finish, dim3(nsub), dim3(EIG_T), 0, st, a, c.W_off, c.W);
  download(herr, a.err, 1, st);
  if (herr[0] & 8) fail(ADS_ERR_EIG_NOCONV, "coarse basis of a subdomain is rank deficient");
  release_all();

}

}  // namespace ads
