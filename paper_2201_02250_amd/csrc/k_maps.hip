// Overlapping subdomains and index maps (Section 2 of the paper): graph of
// A + A^T, delta BFS layers grown from every part, sorted index lists.
//
// Layout: every subdomain i owns a byte map over a window [wlo_i, whi_i) of
// global indices that is guaranteed to contain Omega_i (the interior range
// widened by delta times the matrix bandwidth).  Byte value 0 = interior,
// d = overlap layer d, 0xFF = outside.  Layers are filled one level per launch;
// the sorted lists come from an order-preserving compaction of each window,
// so Omega_Ii and Omega_Gamma_i are ascending by construction (bit-exact).
#include <algorithm>
#include <climits>

#include "ads_internal.h"

namespace ads {

// ---------------------------------------------------------------------------
// exclusive scan (int32 counts -> int64 / int32 offsets), three-phase
// ---------------------------------------------------------------------------
static constexpr int SCAN_T = 256, SCAN_ITEMS = 8, SCAN_CHUNK = SCAN_T * SCAN_ITEMS;

template <class In, class Out>
__global__ void k_scan_chunks(const In* in, Out* out, Out* chunk_sum, int64_t n) {
  __shared__ Out wsum[SCAN_T / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
  Out v[SCAN_ITEMS];
  Out tot = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int64_t i = base + k;
    v[k] = (i < n) ? (Out)in[i] : (Out)0;
    tot += v[k];
  }
  // inclusive scan of per-thread totals within the wave
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  Out incl = tot;
  for (int o = 1; o < 64; o <<= 1) {
    Out t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  Out woff = 0;
  for (int i = 0; i < w; ++i) woff += wsum[i];
  Out run = woff + incl - tot;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (threadIdx.x == SCAN_T - 1) chunk_sum[blockIdx.x] = woff + incl;
}

template <class Out>
__global__ void k_scan_add(Out* out, const Out* chunk_off, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += chunk_off[i / SCAN_CHUNK];
}

template <class In, class Out>
static void scan_impl(const In* in, Out* out, int64_t n, Arena& mem, hipStream_t s) {
  if (n <= 0) return;
  int64_t nch = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
  Out* csum = mem.alloc<Out>(nch);
  ADS_LAUNCH((k_scan_chunks<In, Out>), dim3((unsigned)nch), dim3(SCAN_T), 0, s, in, out, csum, n);
  if (nch > 1) {
    Out* coff = mem.alloc<Out>(nch);
    scan_impl<Out, Out>(csum, coff, nch, mem, s);
    ADS_LAUNCH((k_scan_add<Out>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, coff, n);
  }
}

void exclusive_scan_i64(const int32_t* in, int64_t* out, int64_t n, Arena& mem, hipStream_t s) {
  scan_impl<int32_t, int64_t>(in, out, n, mem, s);
}
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, Arena& mem, hipStream_t s) {
  scan_impl<int32_t, int32_t>(in, out, n, mem, s);
}

// ---------------------------------------------------------------------------
// transpose pattern: graph of A^T, rows of each column ascending
// ---------------------------------------------------------------------------
__global__ void k_count_cols(const int32_t* col, int64_t nnz, int32_t* cnt) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&cnt[col[k]], 1);
}

__global__ void k_fill_transpose(const int32_t* rowptr, const int32_t* col, int64_t n,
                                 const int32_t* tptr, int32_t* fill, int32_t* tcol) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) {
    int c = col[k];
    int p = atomicAdd(&fill[c], 1);
    tcol[tptr[c] + p] = (int32_t)r;
  }
}

// rows of every column in ascending order (the fill above is unordered)
__global__ void k_sort_transpose(const int32_t* tptr, int64_t n, int32_t* tcol) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int32_t* v = tcol + tptr[c];
  const int m = tptr[c + 1] - tptr[c];
  for (int a = 1; a < m; ++a)
    for (int b = a; b > 0 && v[b - 1] > v[b]; --b) {
      const int32_t x = v[b];
      v[b] = v[b - 1];
      v[b - 1] = x;
    }
}

void transpose_pattern(Arena& mem, const int32_t* rowptr, const int32_t* col, int64_t n,
                       int64_t nnz, int32_t** tptr, int32_t** tcol, hipStream_t s) {
  int32_t* cnt = mem.alloc<int32_t>(n + 1);
  ADS_HIP(hipMemsetAsync(cnt, 0, (n + 1) * sizeof(int32_t), s));
  if (nnz)
    ADS_LAUNCH(k_count_cols, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, col, nnz, cnt);
  *tptr = mem.alloc<int32_t>(n + 1);
  exclusive_scan_i32(cnt, *tptr, n + 1, mem, s);
  ADS_HIP(hipMemsetAsync(cnt, 0, (n + 1) * sizeof(int32_t), s));
  *tcol = mem.alloc<int32_t>(nnz);
  ADS_LAUNCH(k_fill_transpose, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rowptr, col, n,
             *tptr, cnt, *tcol);
  ADS_LAUNCH(k_sort_transpose, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, *tptr, n, *tcol);
}

// ---------------------------------------------------------------------------
// subdomain windows
// ---------------------------------------------------------------------------
// per-part first index, last index and size: each workgroup reduces its
// slice in LDS (nparts <= PR_MAXP), then one global atomic per touched part
static constexpr int PR_MAXP = 4096;
static constexpr int PR_T = 1024;
static constexpr int PR_PER = 16;  // elements per thread

__global__ void __launch_bounds__(PR_T)
k_part_range(const int32_t* part, int64_t n, int nparts, int32_t* lo, int32_t* hi,
             int32_t* count) {
  __shared__ int32_t slo[PR_MAXP], shi[PR_MAXP], scnt[PR_MAXP];
  for (int p = threadIdx.x; p < nparts; p += PR_T) {
    slo[p] = INT32_MAX;
    shi[p] = -1;
    scnt[p] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * PR_T * PR_PER;
  for (int k = 0; k < PR_PER; ++k) {
    const int64_t v = base + (int64_t)k * PR_T + threadIdx.x;
    if (v >= n) break;
    const int p = part[v];
    atomicMin(&slo[p], (int32_t)v);
    atomicMax(&shi[p], (int32_t)v);
    atomicAdd(&scnt[p], 1);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < nparts; p += PR_T)
    if (scnt[p]) {
      atomicMin(&lo[p], slo[p]);
      atomicMax(&hi[p], shi[p]);
      atomicAdd(&count[p], scnt[p]);
    }
}

// largest |column - row| over the stored entries (one atomic per wavefront)
__global__ void k_bandwidth(const int32_t* rowptr, const int32_t* col, int64_t n, int32_t* bw) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int m = 0;
  if (r < n)
    for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) m = max(m, abs(col[k] - (int)r));
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(bw, m);
}

__global__ void k_mark_interior(const int32_t* part, int64_t n, const int64_t* wlo,
                                const int64_t* woff, uint8_t* map) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int p = part[v];
  map[woff[p] + (v - wlo[p])] = 0;
}

// one BFS level: every node of layer d-1 marks its unvisited neighbours (in
// the graphs of A and A^T) as layer d.  Concurrent writers store the same
// value, and a node already at d is skipped, so the result is race-free.
__global__ void k_bfs_layer(const int32_t* rowptr, const int32_t* col, const int32_t* tptr,
                            const int32_t* tcol, const int64_t* wlo, const int64_t* whi,
                            const int64_t* woff, int nsub, int64_t total, uint8_t* map, int d,
                            int32_t* err) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  if (map[f] != (uint8_t)(d - 1)) return;
  int i = adsd::segment_of(woff, nsub, f);
  int64_t v = wlo[i] + (f - woff[i]);
  const int64_t lo = wlo[i], hi = whi[i], base = woff[i];
  for (int pass = 0; pass < 2; ++pass) {
    const int32_t* ptr = pass ? tptr : rowptr;
    const int32_t* idx = pass ? tcol : col;
    for (int k = ptr[v]; k < ptr[v + 1]; ++k) {
      int64_t u = idx[k];
      if (u == v) continue;
      if (u < lo || u >= hi) {
        atomicOr(err, 1);
        continue;
      }
      uint8_t* m = &map[base + (u - lo)];
      if (*m == 0xFF) *m = (uint8_t)d;
    }
  }
}

// per subdomain: number of interior and overlap nodes in the window
__global__ void k_count_window(const uint8_t* map, const int64_t* woff, int32_t* nI,
                               int32_t* ni) {
  __shared__ double red[16];
  const int i = blockIdx.x;
  int64_t a = woff[i], b = woff[i + 1];
  double ci = 0, ca = 0;
  for (int64_t f = a + threadIdx.x; f < b; f += blockDim.x) {
    uint8_t m = map[f];
    ci += (m == 0);
    ca += (m != 0xFF);
  }
  ci = adsd::block_sum(ci, red);
  ca = adsd::block_sum(ca, red);
  if (threadIdx.x == 0) {
    nI[i] = (int32_t)ci;
    ni[i] = (int32_t)ca;
  }
}

// block-wide exclusive scan of small ints (blockDim.x = 256)
__device__ __forceinline__ int block_excl_scan(int v, int* wtot, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  __syncthreads();
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  int off = 0, tot = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    if (k < w) off += wtot[k];
    tot += wtot[k];
  }
  *total = tot;
  return off + incl - v;
}

// order-preserving compaction of each window into the index lists
__global__ void k_compact_window(const uint8_t* map, const int64_t* wlo, const int64_t* woff,
                                 const int64_t* om_off, const int32_t* nI, int32_t* om_sorted,
                                 int32_t* om_sub, uint8_t* om_int, int32_t* om_export,
                                 int32_t* om_layer, int32_t* ipos, int32_t* wpos) {
  __shared__ int wt[1][16];
  const int i = blockIdx.x;
  const int64_t a = woff[i], b = woff[i + 1];
  const int64_t base = om_off[i];
  const int nIi = nI[i];
  int run_all = 0, run_I = 0, run_G = 0;
  for (int64_t c0 = a; c0 < b; c0 += blockDim.x) {
    int64_t f = c0 + threadIdx.x;
    uint8_t m = (f < b) ? map[f] : (uint8_t)0xFF;
    int is_all = (m != 0xFF), is_I = (m == 0), is_G = is_all && !is_I;
    // interior and overlap flags packed in 16-bit fields (at most 1024 per
    // chunk): one scan; "all" is their sum
    int tp;
    const int pp = block_excl_scan(is_I | (is_G << 16), wt[0], &tp);
    const int pI = pp & 0xFFFF, pG = pp >> 16, pA = pI + pG;
    const int tI = tp & 0xFFFF, tG = tp >> 16, tA = tI + tG;
    if (f < b) wpos[f] = is_all ? run_all + pA : -1;
    if (is_all) {
      int64_t v = wlo[i] + (f - a);
      int64_t s = base + run_all + pA;
      om_sorted[s] = (int32_t)v;
      om_sub[s] = i;
      om_int[s] = (uint8_t)is_I;
      if (is_I) {
        om_export[base + run_I + pI] = (int32_t)v;
        om_layer[base + run_I + pI] = 0;
        ipos[v] = run_I + pI;
      } else {
        om_export[base + nIi + run_G + pG] = (int32_t)v;
        om_layer[base + nIi + run_G + pG] = m;
      }
    }
    run_all += tA;
    run_I += tI;
    run_G += tG;
    __syncthreads();
  }
}

void build_maps(Ctx& c, const std::vector<int32_t>& part_h) {
  hipStream_t s = c.stream;
  const int64_t n = c.n;
  const int nsub = c.nsub;
  const int delta = c.opt.overlap;
  c.part = upload(c.mem, part_h.data(), n, s);
  transpose_pattern(c.mem, c.rowptr, c.col, n, c.nnz, &c.tptr, &c.tcol, s);

  // lo | hi | cnt | bw in one block (one copy back)
  int32_t* rng = c.mem.alloc<int32_t>(3 * (size_t)nsub + 1);
  int32_t* lo = rng;
  int32_t* hi = rng + nsub;
  int32_t* cnt = rng + 2 * nsub;
  int32_t* bw = rng + 3 * nsub;
  {
    std::vector<int32_t> init(nsub, INT_MAX);
    ADS_HIP(hipMemcpyAsync(lo, init.data(), nsub * 4, hipMemcpyHostToDevice, s));
    ADS_HIP(hipMemsetAsync(hi, 0xFF, nsub * 4, s));  // -1
    ADS_HIP(hipMemsetAsync(cnt, 0, nsub * 4, s));
    ADS_HIP(hipMemsetAsync(bw, 0, 4, s));
    if (nsub > PR_MAXP) fail(ADS_ERR_UNSUPPORTED, "more than 4096 subdomains");
    ADS_LAUNCH(k_part_range, dim3((unsigned)((n + PR_T * PR_PER - 1) / (PR_T * PR_PER))),
               dim3(PR_T), 0, s, c.part, n, nsub, lo, hi, cnt);
    ADS_LAUNCH(k_bandwidth, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c.rowptr, c.col, n,
               bw);
  }
  std::vector<int32_t> hrng;
  download(hrng, rng, 3 * (size_t)nsub + 1, s);
  const int32_t* hlo = hrng.data();
  const int32_t* hhi = hlo + nsub;
  const int32_t* hcnt = hlo + 2 * nsub;
  const int32_t* hbw = hlo + 3 * nsub;
  std::vector<int64_t> wlo(nsub), whi(nsub), woff(nsub + 1, 0);
  for (int i = 0; i < nsub; ++i) {
    if (hcnt[i] == 0) fail(ADS_ERR_ARG, "part " + std::to_string(i) + " is empty");
    int sy = c.sub_sys[i];
    int64_t ext = (int64_t)delta * hbw[0];
    wlo[i] = std::max<int64_t>(c.sys_row[sy], (int64_t)hlo[i] - ext);
    whi[i] = std::min<int64_t>(c.sys_row[sy + 1], (int64_t)hhi[i] + ext + 1);
    woff[i + 1] = woff[i] + (whi[i] - wlo[i]);
  }
  const int64_t total = woff[nsub];
  int64_t* d_wlo = upload(c.mem, wlo.data(), nsub, s);
  int64_t* d_whi = upload(c.mem, whi.data(), nsub, s);
  int64_t* d_woff = upload(c.mem, woff.data(), nsub + 1, s);
  uint8_t* map = c.mem.alloc<uint8_t>(total);
  ADS_HIP(hipMemsetAsync(map, 0xFF, total, s));
  ADS_LAUNCH(k_mark_interior, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c.part, n, d_wlo,
             d_woff, map);
  // err | nI | ni in one block (one copy back)
  int32_t* cblk = c.mem.alloc<int32_t>(1 + 2 * (size_t)nsub);
  int32_t* err = cblk;
  ADS_HIP(hipMemsetAsync(err, 0, 4, s));
  for (int d = 1; d <= delta; ++d)
    ADS_LAUNCH(k_bfs_layer, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, c.rowptr, c.col,
               c.tptr, c.tcol, d_wlo, d_whi, d_woff, nsub, total, map, d, err);
  c.nI = cblk + 1;
  c.ni = cblk + 1 + nsub;
  ADS_LAUNCH(k_count_window, dim3(nsub), dim3(256), 0, s, map, d_woff, c.nI, c.ni);
  std::vector<int32_t> hcb;
  download(hcb, cblk, 1 + 2 * (size_t)nsub, s);
  if (hcb[0]) fail(ADS_ERR_ARG, "overlap growth left its window (matrix bandwidth inconsistent)");
  c.h_nI.assign(hcb.begin() + 1, hcb.begin() + 1 + nsub);
  c.h_ni.assign(hcb.begin() + 1 + nsub, hcb.end());
  c.h_om_off.assign(nsub + 1, 0);
  for (int i = 0; i < nsub; ++i) {
    if (c.h_nI[i] != hcnt[i]) fail(ADS_ERR_ARG, "internal: interior count mismatch");
    c.h_om_off[i + 1] = c.h_om_off[i] + c.h_ni[i];
  }
  c.omega_total = c.h_om_off[nsub];
  c.om_off = upload(c.mem, c.h_om_off.data(), nsub + 1, s);
  c.om_sorted = c.mem.alloc<int32_t>(c.omega_total);
  c.om_sub = c.mem.alloc<int32_t>(c.omega_total);
  c.om_int = c.mem.alloc<uint8_t>(c.omega_total);
  c.om_export = c.mem.alloc<int32_t>(c.omega_total);
  c.om_layer = c.mem.alloc<int32_t>(c.omega_total);
  c.ipos = c.mem.alloc<int32_t>(n);
  c.wpos = c.mem.alloc<int32_t>(total);
  c.wlo = d_wlo;
  c.whi = d_whi;
  c.woff = d_woff;
  ADS_LAUNCH(k_compact_window, dim3(nsub), dim3(1024), 0, s, map, d_wlo, d_woff, c.om_off, c.nI,
             c.om_sorted, c.om_sub, c.om_int, c.om_export, c.om_layer, c.ipos, c.wpos);
  c.int_list = c.om_export;
  c.mem.release(map);
  ADS_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// multi-source BFS partition: owner = seed minimising (distance, seed id)
// ---------------------------------------------------------------------------
__global__ void k_bfs_seed(const int32_t* seeds, int nseed, int32_t* dist, int32_t* owner) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nseed) return;
  dist[seeds[t]] = 0;
  atomicMin(&owner[seeds[t]], t);
}

__global__ void k_bfs_level(const int32_t* rowptr, const int32_t* col, const int32_t* tptr,
                            const int32_t* tcol, int64_t n, int L, int32_t* dist, int32_t* owner,
                            int32_t* changed) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || dist[v] != L - 1) return;
  int ov = owner[v];
  for (int pass = 0; pass < 2; ++pass) {
    const int32_t* ptr = pass ? tptr : rowptr;
    const int32_t* idx = pass ? tcol : col;
    for (int k = ptr[v]; k < ptr[v + 1]; ++k) {
      int u = idx[k];
      int du = dist[u];
      if (du == INT_MAX || du == L) {
        dist[u] = L;
        atomicMin(&owner[u], ov);
        *changed = 1;
      }
    }
  }
}

void bfs_partition(const int32_t* rowptr, const int32_t* col, int64_t n, int64_t nnz,
                   const std::vector<int32_t>& seeds, std::vector<int32_t>& part, hipStream_t s) {
  Arena mem(s);
  int32_t *tptr, *tcol;
  transpose_pattern(mem, rowptr, col, n, nnz, &tptr, &tcol, s);
  int32_t* dist = mem.alloc<int32_t>(n);
  int32_t* owner = mem.alloc<int32_t>(n);
  int32_t* changed = mem.alloc<int32_t>(1);
  std::vector<int32_t> big(n, INT_MAX);
  ADS_HIP(hipMemcpyAsync(dist, big.data(), n * 4, hipMemcpyHostToDevice, s));
  ADS_HIP(hipMemcpyAsync(owner, big.data(), n * 4, hipMemcpyHostToDevice, s));
  int32_t* dseeds = upload(mem, seeds.data(), seeds.size(), s);
  ADS_LAUNCH(k_bfs_seed, dim3((unsigned)((seeds.size() + 255) / 256)), dim3(256), 0, s, dseeds,
             (int)seeds.size(), dist, owner);
  for (int L = 1; L <= n; ++L) {
    ADS_HIP(hipMemsetAsync(changed, 0, 4, s));
    ADS_LAUNCH(k_bfs_level, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rowptr, col, tptr,
               tcol, n, L, dist, owner, changed);
    int32_t h = 0;
    ADS_HIP(hipMemcpyAsync(&h, changed, 4, hipMemcpyDeviceToHost, s));
    ADS_HIP(hipStreamSynchronize(s));
    if (!h) break;
  }
  download(part, owner, n, s);
  for (int64_t v = 0; v < n; ++v)
    if (part[v] == INT_MAX) fail(ADS_ERR_ARG, "vertex unreachable from the seeds");
}

}  // namespace ads
