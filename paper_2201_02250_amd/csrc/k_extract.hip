// Local matrices and the local block splitting of Definition 1 (Section 3.1).
//
// One thread per local row of every subdomain (rows in ascending global
// order).  The row of A is walked once in ascending column order: columns
// inside Omega_i become local CSR entries, columns outside Omega_i of an
// overlap row are summed in absolute value into s_i (the lumped term), in the
// same left-to-right order as a sequential loop, so s_i is reproducible bit
// for bit.  The same walk gives the local bandwidth (block size of the
// factorization) and the row sums of the splitting used to detect floating
// subdomains (kernel K_i = span{1}, Section 3.2).
//
// Complex A is held in its real form (unknown j -> rows 2j, 2j + 1; entry z
// -> columns 2c, 2c + 1 holding (re z, -im z) in the even row, (im z, re z)
// in the odd one).  There the walk takes the entries in pairs: s_i sums the
// moduli |z| (Definition 1's absolute values of complex entries), and the
// kernel test uses the complex row sum; both rows of an unknown get the same
// s_i, subtracted from their real diagonal entries (re a_jj - s_j).
#include <algorithm>

#include "ads_internal.h"
#include "k_solve.h"

namespace ads {

static constexpr double KERNEL_ROWSUM_TOL = 1e-13;

// position of global index c in ascending Omega_i, or -1 (window lookup)
__device__ __forceinline__ int local_pos(const int32_t* wpos, int64_t wl, int64_t wh, int64_t wo,
                                         int c) {
  return (c >= wl && c < wh) ? wpos[wo + (c - wl)] : -1;
}

__global__ void k_extract_count(const int32_t* rowptr, const int32_t* col, const double* val,
                                const int32_t* om_sorted, const int32_t* om_sub,
                                const uint8_t* om_int, const int64_t* om_off, const int64_t* wlo,
                                const int64_t* whi, const int64_t* woff, const int32_t* wpos,
                                int64_t total, int32_t* cnt, double* lsum, int32_t* bw,
                                int32_t* nfail, uint8_t* rbad, int pair) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int maxd = 0, bad = 0, i = -1;
  if (f < total) {
    i = om_sub[f];
    const int64_t base = om_off[i];
    const int64_t wl = wlo[i], wh = whi[i], wo = woff[i];
    const int r = (int)(f - base);
    const int g = om_sorted[f];
    const bool overlap_row = !om_int[f];
    int count = 0;
    double s = 0.0, rs = 0.0, ars = 0.0;
    double diag = 0.0;
    if (!pair) {
      for (int k = rowptr[g]; k < rowptr[g + 1]; ++k) {
        const int c = col[k];
        const double a = val[k];
        const int p = local_pos(wpos, wl, wh, wo, c);
        if (p >= 0) {
          ++count;
          maxd = max(maxd, abs(p - r));
          if (c == g)
            diag = a;
          else {
            rs += a;
            ars += fabs(a);
          }
        } else if (overlap_row) {
          s += fabs(a);
        }
      }
      const double dt = diag - s;  // diagonal of the splitting
      rs += dt;
      ars += fabs(dt);
      bad = !(fabs(rs) <= KERNEL_ROWSUM_TOL * ars);
    } else {
      const bool odd = g & 1;
      double rsi = 0.0, dim = 0.0;  // imaginary parts of the row sum and diagonal
      for (int k = rowptr[g]; k < rowptr[g + 1]; k += 2) {
        const int c = col[k];  // even: the pair (c, c + 1) is one complex entry
        const double a0 = val[k], a1 = val[k + 1];
        const double zr = odd ? a1 : a0, zi = odd ? a0 : -a1;
        const double mod = hypot(zr, zi);  // same arguments in both rows of the unknown
        const int p = local_pos(wpos, wl, wh, wo, c);
        if (p >= 0) {
          count += 2;
          maxd = max(maxd, max(abs(p - r), abs(p + 1 - r)));
          if (c == (g & ~1)) {
            diag = zr;
            dim = zi;
          } else {
            rs += zr;
            rsi += zi;
            ars += mod;
          }
        } else if (overlap_row) {
          s += mod;
        }
      }
      const double dt = diag - s;  // real part of the splitting's diagonal
      rs += dt;
      rsi += dim;
      ars += hypot(dt, dim);
      bad = !(hypot(rs, rsi) <= KERNEL_ROWSUM_TOL * ars);
    }
    cnt[f] = count;
    lsum[f] = overlap_row ? s : 0.0;
    rbad[f] = (uint8_t)bad;
  }
  // one atomic per run of equal subdomains in the wavefront
  const int lane = threadIdx.x & 63;
  const int iprev = __shfl_up(i, 1, 64);
  const bool head = lane == 0 || iprev != i;
  for (int o = 1; o < 64; o <<= 1) {
    const int om = __shfl_down(maxd, o, 64), ob = __shfl_down(bad, o, 64);
    const int oi = __shfl_down(i, o, 64);
    if (lane + o < 64 && oi == i) {
      maxd = max(maxd, om);
      bad += ob;
    }
  }
  if (head && i >= 0) {
    atomicMax(&bw[i], maxd);
    if (bad) atomicAdd(&nfail[i], bad);
  }
}

__global__ void k_extract_fill(const int32_t* rowptr, const int32_t* col, const double* val,
                               const int32_t* om_sorted, const int32_t* om_sub,
                               const int64_t* wlo, const int64_t* whi, const int64_t* woff,
                               const int32_t* wpos, int64_t total, const int64_t* lrow,
                               int32_t* lcol, double* lval) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  const int i = om_sub[f];
  const int64_t wl = wlo[i], wh = whi[i], wo = woff[i];
  const int g = om_sorted[f];
  int64_t w = lrow[f];
  for (int k = rowptr[g]; k < rowptr[g + 1]; ++k) {
    const int c = col[k];
    const int p = local_pos(wpos, wl, wh, wo, c);
    if (p >= 0) {
      lcol[w] = p;
      lval[w] = val[k];
      ++w;
    }
  }
}

// Connected components of each splitting's graph (stored local entries and
// their transposes; complex A in its real form: the two rows of an unknown are
// one vertex), one workgroup per subdomain: every row starts with its own
// index as label, and sweeps of min-label propagation along the edges (both
// directions) plus pointer jumping run until a sweep changes nothing, leaving
// each row with the smallest row index of its component.  A component floats
// when none of its rows failed the zero-sum test.  Labels and flags live in
// global memory and are read with device-scope atomic loads (the updates are
// atomics performed in L2).  Out: ncomp[i], nfloat[i].
__device__ __forceinline__ int ld_l2(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(1024) k_components(const int64_t* om_off, const int64_t* lrow,
                                                     const int32_t* lcol, const uint8_t* rbad,
                                                     int32_t* lab, int32_t* cbad, int pair,
                                                     int32_t* ncomp, int32_t* nfloat) {
  __shared__ int cnt[2];
  const int i = blockIdx.x, t = threadIdx.x, T = blockDim.x;
  const int64_t base = om_off[i];
  const int n = (int)(om_off[i + 1] - base);
  int32_t* L = lab + base;
  int32_t* cb = cbad + base;
  for (int r = t; r < n; r += T) {
    atomicExch(&L[r], pair ? (r & ~1) : r);
    atomicExch(&cb[r], 0);
  }
  __syncthreads();
  for (;;) {
    int changed = 0;
    for (int r = t; r < n; r += T) {
      int m = ld_l2(&L[r]);
      const int m0 = m;
      for (int64_t q = lrow[base + r]; q < lrow[base + r + 1]; ++q) m = min(m, ld_l2(&L[lcol[q]]));
      if (pair) m = min(m, ld_l2(&L[r ^ 1]));
      if (m < m0) {
        atomicMin(&L[r], m);
        changed = 1;
      }
      for (int64_t q = lrow[base + r]; q < lrow[base + r + 1]; ++q)
        if (ld_l2(&L[lcol[q]]) > m) {
          atomicMin(&L[lcol[q]], m);
          changed = 1;
        }
    }
    __syncthreads();
    for (int r = t; r < n; r += T) {  // pointer jumping (labels only decrease)
      const int m0 = ld_l2(&L[r]);
      int m = m0;
      for (int x = ld_l2(&L[m]); x < m; x = ld_l2(&L[m])) m = x;
      if (m < m0) atomicMin(&L[r], m);
    }
    if (!__syncthreads_or(changed)) break;
  }
  for (int r = t; r < n; r += T)
    if (rbad[base + r]) atomicExch(&cb[ld_l2(&L[r])], 1);
  if (t < 2) cnt[t] = 0;
  __syncthreads();
  int nc = 0, nf = 0;
  for (int r = t; r < n; r += T)
    if (ld_l2(&L[r]) == r) {
      ++nc;
      nf += !ld_l2(&cb[r]);
    }
  if (nc) atomicAdd(&cnt[0], nc);
  if (nf) atomicAdd(&cnt[1], nf);
  __syncthreads();
  if (t == 0) {
    ncomp[i] = cnt[0];
    nfloat[i] = cnt[1];
  }
}

// K_i (reading of Section 3.2): the indicator of the subdomain when it is one
// connected component whose rows all pass the zero-sum test (complex A: its
// real form span{constant real parts, constant imaginary parts}, dimension 2);
// {0} when no component floats
__global__ void k_kernel_dim(const int32_t* nfloat, int nsub, int32_t* kdim, int pair) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsub) kdim[i] = nfloat[i] ? (pair ? 2 : 1) : 0;
}

// per padded local row of block k: the (column in block k + dk, value)
// couplings of the block-tridiagonal form, at most NCPL of them (dk = -1:
// A_k,k-1 by row; dk = +1: A_k,k+1 by row)
__global__ void k_row_couplings(const int64_t* pad_off, int nsub, const int32_t* bs,
                                const int32_t* ni, const int64_t* om_off, const int64_t* lrow,
                                const int32_t* lcol, const double* lval, int64_t total, int dk,
                                int32_t* ccol, double* cval, int32_t* overflow) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  const int i = adsd::segment_of(pad_off, nsub, f);
  const int r = (int)(f - pad_off[i]);
  const int s = bs[i];
  const int k = r / s;
  int cnt = 0;
  if (r < ni[i]) {
    const int64_t row = om_off[i] + r;
    for (int64_t q = lrow[row]; q < lrow[row + 1]; ++q) {
      const int cc = lcol[q] - (k + dk) * s;
      if (cc < 0 || cc >= s) continue;
      if (cnt < adsd::NCPL) {
        ccol[f * adsd::NCPL + cnt] = cc;
        cval[f * adsd::NCPL + cnt] = lval[q];
      }
      ++cnt;
    }
  }
  if (cnt > adsd::NCPL) atomicOr(overflow, 1);
  for (int m = cnt; m < adsd::NCPL; ++m) {
    ccol[f * adsd::NCPL + m] = -1;
    cval[f * adsd::NCPL + m] = 0.0;
  }
}

// per padded local column c' of block kb: the entries a_{r,c'} of the rows r
// of block kb + dr, at most NCPL, sorted by r afterwards (dr = -1: A_kb-1,kb
// by column; dr = +1: A_kb+1,kb by column)
__global__ void k_col_couplings(const int64_t* pad_off, int nsub, const int32_t* bs,
                                const int32_t* ni, const int64_t* om_off, const int64_t* lrow,
                                const int32_t* lcol, const double* lval, int64_t total, int dr,
                                int32_t* ucnt, int32_t* urow, double* uval) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  const int i = adsd::segment_of(pad_off, nsub, f);
  const int r = (int)(f - pad_off[i]);
  const int s = bs[i];
  const int k = r / s;
  if (r >= ni[i]) return;
  const int64_t row = om_off[i] + r;
  for (int64_t q = lrow[row]; q < lrow[row + 1]; ++q) {
    const int cp = lcol[q];
    if (cp / s != k - dr) continue;
    const int64_t fc = pad_off[i] + cp;  // padded slot of column c'
    const int slot = atomicAdd(&ucnt[fc], 1);
    if (slot < adsd::NCPL) {
      urow[fc * adsd::NCPL + slot] = r - k * s;
      uval[fc * adsd::NCPL + slot] = lval[q];
    }
  }
}

__global__ void k_upper_sort(int64_t total, int32_t* ucnt, int32_t* urow, double* uval,
                             int32_t* overflow) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  int n = ucnt[f];
  if (n > adsd::NCPL) {
    atomicOr(overflow, 1);
    n = adsd::NCPL;
  }
  int32_t* rr = urow + f * adsd::NCPL;
  double* vv = uval + f * adsd::NCPL;
  for (int a = 1; a < n; ++a)  // insertion sort by row
    for (int b = a; b > 0 && rr[b - 1] > rr[b]; --b) {
      int tr = rr[b];
      rr[b] = rr[b - 1];
      rr[b - 1] = tr;
      double tv = vv[b];
      vv[b] = vv[b - 1];
      vv[b - 1] = tv;
    }
  for (int m = n; m < adsd::NCPL; ++m) {
    rr[m] = -1;
    vv[m] = 0.0;
  }
}

void extract_local(Ctx& c) {
  hipStream_t s = c.stream;
  const int64_t T = c.omega_total;
  const int nsub = c.nsub;
  int32_t* cnt = c.mem.alloc<int32_t>(T + 1);
  c.lsum = c.mem.alloc<double>(T);
  // kernel dimension | bandwidth in one block (one copy back)
  int32_t* kb = c.mem.alloc<int32_t>(2 * (size_t)nsub);
  int32_t* bw = kb + nsub;
  int32_t* nfail = c.mem.alloc<int32_t>(3 * (size_t)nsub);  // | ncomp | nfloat
  int32_t* ncomp = nfail + nsub;
  int32_t* nfloat = ncomp + nsub;
  uint8_t* rbad = c.mem.alloc<uint8_t>(T);
  int32_t* lab = c.mem.alloc<int32_t>(2 * T);  // | component has a failing row
  ADS_HIP(hipMemsetAsync(bw, 0, nsub * 4, s));
  ADS_HIP(hipMemsetAsync(nfail, 0, nsub * 4, s));
  ADS_HIP(hipMemsetAsync(cnt + T, 0, 4, s));
  unsigned gb = (unsigned)((T + 255) / 256);
  ADS_LAUNCH(k_extract_count, dim3(gb), dim3(256), 0, s, c.rowptr, c.col, c.val, c.om_sorted,
             c.om_sub, c.om_int, c.om_off, c.wlo, c.whi, c.woff, c.wpos, T, cnt, c.lsum, bw,
             nfail, rbad, c.cplx);
  int64_t* lrow = c.mem.alloc<int64_t>(T + 1);
  exclusive_scan_i64(cnt, lrow, T + 1, c.mem, s);
  std::vector<int64_t> hl;
  download(hl, lrow + T, 1, s);
  c.lnnz = hl[0];
  c.lptr_off = lrow;  // flat row starts, [T + 1]
  c.lcol = c.mem.alloc<int32_t>(c.lnnz);
  c.lval = c.mem.alloc<double>(c.lnnz);
  ADS_LAUNCH(k_extract_fill, dim3(gb), dim3(256), 0, s, c.rowptr, c.col, c.val, c.om_sorted,
             c.om_sub, c.wlo, c.whi, c.woff, c.wpos, T, lrow, c.lcol, c.lval);
  ADS_LAUNCH(k_components, dim3(nsub), dim3(1024), 0, s, c.om_off, lrow, c.lcol, rbad, lab,
             lab + T, c.cplx, ncomp, nfloat);
  c.kdim = kb;
  ADS_LAUNCH(k_kernel_dim, dim3((nsub + 255) / 256), dim3(256), 0, s, nfloat, nsub, c.kdim, c.cplx);
  std::vector<int32_t> hkb, hcf;
  download(hkb, kb, 2 * (size_t)nsub, s);
  download(hcf, ncomp, 2 * (size_t)nsub, s);
  c.mem.release(lab);
  c.mem.release(rbad);
  c.mem.release(nfail);
  for (int i = 0; i < nsub; ++i)
    if (hcf[nsub + i] && hcf[i] > 1)
      fail(ADS_ERR_UNSUPPORTED,
           "subdomain " + std::to_string(i) + ": its splitting has " + std::to_string(hcf[i]) +
               " connected components, " + std::to_string(hcf[nsub + i]) +
               " of them floating; a kernel spanned by piecewise constants is not supported");
  c.h_kdim.assign(hkb.begin(), hkb.begin() + nsub);
  c.h_bw.resize(nsub);
  for (int i = 0; i < nsub; ++i) c.h_bw[i] = std::max(1, hkb[nsub + i]);
  c.bw_d = upload(c.mem, c.h_bw.data(), nsub, s);
  c.mem.release(cnt);
  set_tiles(c, c.h_bw);
}

// Block sizes of the block-tridiagonal form (any size >= the local bandwidth
// is valid): the padded layout, the four coupling lists and the fast-path
// flags.  Replaces a previous layout.
void set_tiles(Ctx& c, const std::vector<int32_t>& sizes) {
  hipStream_t s = c.stream;
  const int nsub = c.nsub;
  for (void* q : {(void*)c.bs, (void*)c.nb, (void*)c.pad_off, (void*)c.cpl_col, (void*)c.cpl_val,
                  (void*)c.rcpl_col, (void*)c.rcpl_val, (void*)c.ucpl_row, (void*)c.ucpl_val,
                  (void*)c.lcpl_row, (void*)c.lcpl_val})
    if (q) c.mem.release(q);
  c.h_bs.resize(nsub);
  c.h_nb.resize(nsub);
  c.h_pad_off.assign(nsub + 1, 0);
  for (int i = 0; i < nsub; ++i) {
    const int b = std::max(sizes[i], c.h_bw[i]);
    c.h_bs[i] = b;
    c.h_nb[i] = (c.h_ni[i] + b - 1) / b;
    c.h_pad_off[i + 1] = c.h_pad_off[i] + (int64_t)c.h_nb[i] * b;
  }
  c.npad_total = c.h_pad_off[nsub];
  c.bs = upload(c.mem, c.h_bs.data(), nsub, s);
  c.nb = upload(c.mem, c.h_nb.data(), nsub, s);
  c.pad_off = upload(c.mem, c.h_pad_off.data(), nsub + 1, s);
  // the four coupling lists of the block-tridiagonal form (tile solves and
  // the two-ended factorization)
  const int64_t NP = c.npad_total;
  const unsigned gp = (unsigned)((NP + 255) / 256);
  int32_t* ovf = c.mem.alloc<int32_t>(1);
  ADS_HIP(hipMemsetAsync(ovf, 0, 4, s));
  auto row_list = [&](int dk, int32_t** cc, double** cv) {
    *cc = c.mem.alloc<int32_t>((size_t)NP * adsd::NCPL);
    *cv = c.mem.alloc<double>((size_t)NP * adsd::NCPL);
    ADS_LAUNCH(k_row_couplings, dim3(gp), dim3(256), 0, s, c.pad_off, nsub, c.bs, c.ni, c.om_off,
               c.lptr_off, c.lcol, c.lval, NP, dk, *cc, *cv, ovf);
  };
  int32_t* ucnt = c.mem.alloc<int32_t>(NP);
  auto col_list = [&](int dr, int32_t** cr, double** cv) {
    *cr = c.mem.alloc<int32_t>((size_t)NP * adsd::NCPL);
    *cv = c.mem.alloc<double>((size_t)NP * adsd::NCPL);
    ADS_HIP(hipMemsetAsync(ucnt, 0, NP * 4, s));
    ADS_LAUNCH(k_col_couplings, dim3(gp), dim3(256), 0, s, c.pad_off, nsub, c.bs, c.ni, c.om_off,
               c.lptr_off, c.lcol, c.lval, NP, dr, ucnt, *cr, *cv);
    ADS_LAUNCH(k_upper_sort, dim3(gp), dim3(256), 0, s, NP, ucnt, *cr, *cv, ovf);
  };
  row_list(-1, &c.cpl_col, &c.cpl_val);    // A_k,k-1 by row
  row_list(+1, &c.rcpl_col, &c.rcpl_val);  // A_k,k+1 by row
  col_list(-1, &c.ucpl_row, &c.ucpl_val);  // A_k-1,k by column
  col_list(+1, &c.lcpl_row, &c.lcpl_val);  // A_k+1,k by column
  std::vector<int32_t> hov;
  download(hov, ovf, 1, s);
  c.mem.release(ucnt);
  c.mem.release(ovf);
  // fast path (two-ended factorization, prefetching tile solves): every list
  // complete and every block size within the solve and factorization limits
  c.cpl_ok = hov[0] == 0;
  c.solve_fast = c.cpl_ok;
  const int V = c.prec == ADS_PREC_FP64 ? 2 : (c.prec == ADS_PREC_FP32 ? 4 : 8);
  for (int b : c.h_bs)
    c.solve_fast = c.solve_fast && adsd::solve_fast_ok(b, adsd::SOLVE_T, 1, V) &&
                   adsd::factor_fast_ok(b);
  ADS_HIP(hipStreamSynchronize(s));
}

}  // namespace ads
