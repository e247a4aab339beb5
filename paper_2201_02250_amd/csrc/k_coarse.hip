// Coarse operator A_00 = R_0 A R_0^T (Section 2) with R_0^T = [R_1^T D_1 Z_1 ...]
// (Section 3.2), i.e. E = W^T A W where W_i holds the interior rows of Z_i.
//
// E is block sparse: block (j, i) is nonzero only when Omega_Ij couples to
// Omega_Ii, i.e. when i owns a first-layer overlap node of subdomain j.  Per
// system the blocks are assembled into a dense n0_s x n0_s matrix, one
// workgroup per nonzero block, with a fixed reduction order (deterministic).
// Then the exact FP64 inverse of each E_s (Section 4 solves the second-level
// system exactly) by Gauss-Jordan elimination with partial pivoting: the apply
// then needs one matrix-vector product instead of two latency-bound
// triangular sweeps.
#include <algorithm>

#include "ads_internal.h"
#include "k_gj.h"

namespace ads {

static constexpr int NB_MAX = 128;
static constexpr int CO_T = 256;
static constexpr int ROWCH = 128;

// neighbour subdomains (same system) of every subdomain, itself first
__global__ void k_neighbours(const int32_t* om_export, const int32_t* om_layer,
                             const int64_t* om_off, const int32_t* nI, const int32_t* ni,
                             const int32_t* part, const int32_t* sys_sub_first,
                             const int32_t* sys_sub_count, const int32_t* sub_sys,
                             int32_t* nbcnt, int32_t* nblist, int32_t* overflow) {
  extern __shared__ uint32_t bits[];
  const int j = blockIdx.x;
  const int sy = sub_sys[j];
  const int first = sys_sub_first[sy], cnt = sys_sub_count[sy];
  const int words = (cnt + 31) / 32;
  for (int w = threadIdx.x; w < words; w += blockDim.x) bits[w] = 0;
  __syncthreads();
  const int64_t b = om_off[j];
  for (int k = nI[j] + threadIdx.x; k < ni[j]; k += blockDim.x) {
    if (om_layer[b + k] != 1) continue;
    const int o = part[om_export[b + k]] - first;
    atomicOr(&bits[o >> 5], 1u << (o & 31));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    nblist[(int64_t)j * NB_MAX + c++] = j;
    for (int o = 0; o < cnt; ++o)
      if ((bits[o >> 5] >> (o & 31)) & 1u) {
        if (c >= NB_MAX) {
          *overflow = 1;
          break;
        }
        nblist[(int64_t)j * NB_MAX + c++] = first + o;
      }
    nbcnt[j] = c;
  }
}

// E block (j, i) = W_j^T A(Omega_Ij, Omega_Ii) W_i
__global__ void __launch_bounds__(CO_T)
k_coarse_block(const int32_t* nbcnt, const int32_t* nblist, const int32_t* rowptr,
               const int32_t* col, const double* val, const int32_t* part, const int32_t* ipos,
               const int32_t* int_list, const int64_t* om_off, const int32_t* nI,
               const double* W, const int64_t* W_off, const int32_t* nev, const int32_t* coff,
               const int32_t* sub_sys, const int32_t* sys_coff, const int64_t* E_off, double* E) {
  __shared__ double Wch[ROWCH * 32];
  __shared__ double Ych[ROWCH * 32];
  const int j = blockIdx.x, t = blockIdx.y;
  if (t >= nbcnt[j]) return;
  const int i = nblist[(int64_t)j * NB_MAX + t];
  const int mj = nev[j], mi = nev[i];
  if (mj == 0 || mi == 0) return;
  const int sy = sub_sys[j];
  const int c0 = sys_coff[sy], ns = sys_coff[sy + 1] - c0;
  const int nint = nI[j];
  const int32_t* rows = int_list + om_off[j];
  const double* Wj = W + W_off[j];
  const double* Wi = W + W_off[i];
  double acc[4];
  for (int q = 0; q < 4; ++q) acc[q] = 0.0;
  for (int k0 = 0; k0 < nint; k0 += ROWCH) {
    const int nr = min(ROWCH, nint - k0);
    __syncthreads();
    for (int rr = threadIdx.x; rr < ROWCH; rr += blockDim.x) {
      double y[32];
      for (int bq = 0; bq < 32; ++bq) y[bq] = 0.0;
      if (rr < nr) {
        const int g = rows[k0 + rr];
        for (int q = rowptr[g]; q < rowptr[g + 1]; ++q) {
          const int cc = col[q];
          if (part[cc] != i) continue;
          const double a = val[q];
          const double* w = Wi + (int64_t)ipos[cc] * mi;
          for (int bq = 0; bq < 32; ++bq)
            if (bq < mi) y[bq] += a * w[bq];
        }
      }
      for (int bq = 0; bq < 32; ++bq)
        if (bq < mi) Ych[rr * 32 + bq] = y[bq];
      for (int aq = 0; aq < 32; ++aq)
        if (aq < mj) Wch[rr * 32 + aq] = (rr < nr) ? Wj[(int64_t)(k0 + rr) * mj + aq] : 0.0;
    }
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + q * CO_T;
      if (e < mj * mi) {
        const int aq = e / mi, bq = e % mi;
        double sacc = 0.0;
        for (int rr = 0; rr < nr; ++rr) sacc += Wch[rr * 32 + aq] * Ych[rr * 32 + bq];
        acc[q] += sacc;
      }
    }
  }
  double* Es = E + E_off[sy];
  const int r0 = coff[j] - c0, q0 = coff[i] - c0;
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + q * CO_T;
    if (e < mj * mi) {
      const int aq = e / mi, bq = e % mi;
      Es[(int64_t)(r0 + aq) * ns + q0 + bq] = acc[q];
    }
  }
}

void assemble_coarse(Ctx& c) {
  hipStream_t st = c.stream;
  const int nsub = c.nsub, nsys = c.nsys;
  c.h_n0s.assign(nsys, 0);
  std::vector<int32_t> sc(nsys + 1, 0), sfirst(nsys), scount(nsys);
  for (int s = 0; s < nsys; ++s) {
    sfirst[s] = c.sys_sub[s];
    scount[s] = c.sys_sub[s + 1] - c.sys_sub[s];
    sc[s] = c.h_coff[c.sys_sub[s]];
  }
  sc[nsys] = c.h_coff[nsub];
  c.h_E_off.assign(nsys + 1, 0);
  int64_t maxs = 0;
  for (int s = 0; s < nsys; ++s) {
    int64_t ns = sc[s + 1] - sc[s];
    c.h_n0s[s] = (int32_t)ns;
    c.h_E_off[s + 1] = c.h_E_off[s] + ns * ns;
    maxs = std::max(maxs, ns);
  }
  c.sys_coff = upload(c.mem, sc.data(), nsys + 1, st);
  c.E_off = upload(c.mem, c.h_E_off.data(), nsys + 1, st);
  const int64_t etot = std::max<int64_t>(c.h_E_off[nsys], 1);
  double* E = c.mem.alloc<double>(etot);
  ADS_HIP(hipMemsetAsync(E, 0, etot * 8, st));
  int32_t* d_first = upload(c.mem, sfirst.data(), nsys, st);
  int32_t* d_count = upload(c.mem, scount.data(), nsys, st);
  int32_t* nbcnt = c.mem.alloc<int32_t>(nsub);
  int32_t* nblist = c.mem.alloc<int32_t>((size_t)nsub * NB_MAX);
  int32_t* flag = c.mem.alloc<int32_t>(2);
  ADS_HIP(hipMemsetAsync(flag, 0, 8, st));
  int maxcnt = *std::max_element(scount.begin(), scount.end());
  size_t bits_lds = (size_t)((maxcnt + 31) / 32) * 4;
  ADS_LAUNCH(k_neighbours, dim3(nsub), dim3(256), bits_lds, st, c.om_export, c.om_layer, c.om_off,
             c.nI, c.ni, c.part, d_first, d_count, c.sub_sys_d, nbcnt, nblist, flag);
  ADS_LAUNCH(k_coarse_block, dim3(nsub, NB_MAX), dim3(CO_T), 0, st, nbcnt, nblist, c.rowptr, c.col,
             c.val, c.part, c.ipos, c.int_list, c.om_off, c.nI, c.W, c.W_off, c.nev, c.coff,
             c.sub_sys_d, c.sys_coff, c.E_off, E);
  std::vector<int32_t> hf;  // both flags are read once, after the inverse
  double* F = c.mem.alloc<double>(etot);
  // symmetric A: E = W^T A W is symmetric (positive definite when A is):
  // inverted without interchanges, or, if a pivot is not positive, assembled
  // again and inverted with partial pivoting
  double* inv = gj_invert_batched(c, st, nsys, maxs, sc[nsys], c.h_E_off[nsys], E, F, c.E_off,
                                  c.sys_coff, flag + 1, c.sym, c.h_n0s.data());
  if (!inv) {
    ADS_HIP(hipMemsetAsync(E, 0, etot * 8, st));
    ADS_LAUNCH(k_coarse_block, dim3(nsub, NB_MAX), dim3(CO_T), 0, st, nbcnt, nblist, c.rowptr,
               c.col, c.val, c.part, c.ipos, c.int_list, c.om_off, c.nI, c.W, c.W_off, c.nev,
               c.coff, c.sub_sys_d, c.sys_coff, c.E_off, E);
    inv = gj_invert_batched(c, st, nsys, maxs, sc[nsys], c.h_E_off[nsys], E, F, c.E_off,
                            c.sys_coff, flag + 1, false, c.h_n0s.data());
  }
  download(hf, flag, 2, st);
  if (hf[0]) fail(ADS_ERR_UNSUPPORTED, "a subdomain has more than 127 neighbours");
  if (hf[1]) fail(ADS_ERR_SINGULAR, "singular coarse operator in system " + std::to_string(hf[1] - 1));
  c.Einv = inv;
  c.mem.release(inv == E ? F : E);
}

}  // namespace ads
