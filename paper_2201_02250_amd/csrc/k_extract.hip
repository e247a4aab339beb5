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
#include <algorithm>

#include "ads_internal.h"

namespace ads {

static constexpr double KERNEL_ROWSUM_TOL = 1e-13;

__global__ void k_extract_count(const int32_t* rowptr, const int32_t* col, const double* val,
                                const int32_t* om_sorted, const int32_t* om_sub,
                                const uint8_t* om_int, const int64_t* om_off, const int32_t* ni,
                                int64_t total, int32_t* cnt, double* lsum, int32_t* bw,
                                int32_t* nfail) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  const int i = om_sub[f];
  const int64_t base = om_off[i];
  const int n = ni[i];
  const int32_t* om = om_sorted + base;
  const int r = (int)(f - base);
  const int g = om[r];
  const bool overlap_row = !om_int[f];
  int count = 0, maxd = 0;
  double s = 0.0, rs = 0.0, ars = 0.0;
  double diag = 0.0;
  for (int k = rowptr[g]; k < rowptr[g + 1]; ++k) {
    const int c = col[k];
    const double a = val[k];
    const int p = adsd::lower_bound_i32(om, n, c);
    if (p < n && om[p] == c) {
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
  cnt[f] = count;
  lsum[f] = overlap_row ? s : 0.0;
  atomicMax(&bw[i], maxd);
  if (!(fabs(rs) <= KERNEL_ROWSUM_TOL * ars)) atomicAdd(&nfail[i], 1);
}

__global__ void k_extract_fill(const int32_t* rowptr, const int32_t* col, const double* val,
                               const int32_t* om_sorted, const int32_t* om_sub,
                               const int64_t* om_off, const int32_t* ni, int64_t total,
                               const int64_t* lrow, int32_t* lcol, double* lval) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  const int i = om_sub[f];
  const int64_t base = om_off[i];
  const int n = ni[i];
  const int32_t* om = om_sorted + base;
  const int g = om[f - base];
  int64_t w = lrow[f];
  for (int k = rowptr[g]; k < rowptr[g + 1]; ++k) {
    const int c = col[k];
    const int p = adsd::lower_bound_i32(om, n, c);
    if (p < n && om[p] == c) {
      lcol[w] = p;
      lval[w] = val[k];
      ++w;
    }
  }
}

__global__ void k_kernel_dim(const int32_t* nfail, int nsub, int32_t* kdim) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsub) kdim[i] = (nfail[i] == 0) ? 1 : 0;
}

void extract_local(Ctx& c) {
  hipStream_t s = c.stream;
  const int64_t T = c.omega_total;
  const int nsub = c.nsub;
  int32_t* cnt = c.mem.alloc<int32_t>(T + 1);
  c.lsum = c.mem.alloc<double>(T);
  int32_t* bw = c.mem.alloc<int32_t>(nsub);
  int32_t* nfail = c.mem.alloc<int32_t>(nsub);
  ADS_HIP(hipMemsetAsync(bw, 0, nsub * 4, s));
  ADS_HIP(hipMemsetAsync(nfail, 0, nsub * 4, s));
  ADS_HIP(hipMemsetAsync(cnt + T, 0, 4, s));
  unsigned gb = (unsigned)((T + 255) / 256);
  ADS_LAUNCH(k_extract_count, dim3(gb), dim3(256), 0, s, c.rowptr, c.col, c.val, c.om_sorted,
             c.om_sub, c.om_int, c.om_off, c.ni, T, cnt, c.lsum, bw, nfail);
  int64_t* lrow = c.mem.alloc<int64_t>(T + 1);
  exclusive_scan_i64(cnt, lrow, T + 1, c.mem, s);
  std::vector<int64_t> hl;
  download(hl, lrow + T, 1, s);
  c.lnnz = hl[0];
  c.lptr_off = lrow;  // flat row starts, [T + 1]
  c.lcol = c.mem.alloc<int32_t>(c.lnnz);
  c.lval = c.mem.alloc<double>(c.lnnz);
  ADS_LAUNCH(k_extract_fill, dim3(gb), dim3(256), 0, s, c.rowptr, c.col, c.val, c.om_sorted,
             c.om_sub, c.om_off, c.ni, T, lrow, c.lcol, c.lval);
  c.kdim = c.mem.alloc<int32_t>(nsub);
  ADS_LAUNCH(k_kernel_dim, dim3((nsub + 255) / 256), dim3(256), 0, s, nfail, nsub, c.kdim);
  download(c.h_kdim, c.kdim, nsub, s);
  std::vector<int32_t> hbw;
  download(hbw, bw, nsub, s);
  c.h_bs.resize(nsub);
  c.h_nb.resize(nsub);
  c.h_pad_off.assign(nsub + 1, 0);
  for (int i = 0; i < nsub; ++i) {
    int b = std::max(1, hbw[i]);
    c.h_bs[i] = b;
    c.h_nb[i] = (c.h_ni[i] + b - 1) / b;
    c.h_pad_off[i + 1] = c.h_pad_off[i] + (int64_t)c.h_nb[i] * b;
  }
  c.npad_total = c.h_pad_off[nsub];
  c.bs = upload(c.mem, c.h_bs.data(), nsub, s);
  c.nb = upload(c.mem, c.h_nb.data(), nsub, s);
  c.pad_off = upload(c.mem, c.h_pad_off.data(), nsub + 1, s);
  c.mem.release(cnt);
  ADS_HIP(hipStreamSynchronize(s));
}

}  // namespace ads
