// Device symbolic phase: tile patterns of block products and their work lists.
//
// For a product O = op(A) * B of tile patterns, the kernels below compute
//   * the pattern of O (union over k in A.row(i) of B.row(k)), one workgroup
//     per output row with the row's column window held as a bitmap in LDS;
//   * for every output tile (i, j) the list of (A tile, B tile) pairs with
//     A(i,k) and B(k,j) both stored, in increasing k, which is the fixed
//     summation order of the numeric kernels (bitwise-reproducible results).
// This is the tile-level counterpart of reserving the blocks of a sparse
// product before filling it (Sec. III C, m_reserve_blocks) and of the
// product-pattern bookkeeping of a block-sparse library; restricted outputs
// (the gradient kept on C's pattern, rho on S's pattern, Sec. III B) reuse
// the pair kernels with a given output pattern.
#include "kernels.hpp"

namespace omm {

namespace {

constexpr int SYM_THREADS = 256;

__device__ __forceinline__ int a_tile(const PatView& A, int e) { return A.ti ? A.ti[e] : e; }

__global__ __launch_bounds__(SYM_THREADS) void k_sym_count(int row0, PatView A, PatView B,
                                                         const int2* __restrict__ win,
                                                         int* __restrict__ cnt) {
  __shared__ uint32_t bm[MAXW / 32];
  __shared__ int red[SYM_THREADS];
  const int i = row0 + blockIdx.x;
  const int2 w = win[i];
  const int nw = (w.y - w.x + 31) >> 5;
  for (int t = threadIdx.x; t < nw; t += blockDim.x) bm[t] = 0u;
  __syncthreads();
  for (int e = A.rp[i] + threadIdx.x; e < A.rp[i + 1]; e += blockDim.x) {
    const int k = A.ci[e];
    for (int jj = B.rp[k]; jj < B.rp[k + 1]; ++jj) {
      const int c = B.ci[jj] - w.x;
      if (c >= 0 && c < w.y - w.x) atomicOr(&bm[c >> 5], 1u << (c & 31));
    }
  }
  __syncthreads();
  int s = 0;
  for (int t = threadIdx.x; t < nw; t += blockDim.x) s += __popc(bm[t]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = SYM_THREADS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(SYM_THREADS) void k_sym_fill(int row0, PatView A, PatView B,
                                                        const int2* __restrict__ win,
                                                        const int* __restrict__ orp,
                                                        int* __restrict__ oci, int* __restrict__ orow) {
  __shared__ uint32_t bm[MAXW / 32];
  __shared__ int pre[SYM_THREADS + 1];
  const int i = row0 + blockIdx.x;
  const int2 w = win[i];
  const int nw = (w.y - w.x + 31) >> 5;
  for (int t = threadIdx.x; t < nw; t += blockDim.x) bm[t] = 0u;
  __syncthreads();
  for (int e = A.rp[i] + threadIdx.x; e < A.rp[i + 1]; e += blockDim.x) {
    const int k = A.ci[e];
    for (int jj = B.rp[k]; jj < B.rp[k + 1]; ++jj) {
      const int c = B.ci[jj] - w.x;
      if (c >= 0 && c < w.y - w.x) atomicOr(&bm[c >> 5], 1u << (c & 31));
    }
  }
  __syncthreads();
  // each thread owns a contiguous run of words; exclusive scan of the run counts
  const int per = (nw + SYM_THREADS - 1) / SYM_THREADS;
  const int wb = threadIdx.x * per, we = min(nw, wb + per);
  int s = 0;
  for (int t = wb; t < we; ++t) s += __popc(bm[t]);
  pre[threadIdx.x + 1] = s;
  if (threadIdx.x == 0) pre[0] = 0;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int t = 1; t <= SYM_THREADS; ++t) pre[t] += pre[t - 1];
  __syncthreads();
  int pos = orp[i] + pre[threadIdx.x];
  for (int t = wb; t < we; ++t) {
    uint32_t word = bm[t];
    while (word) {
      const int b = __ffs(word) - 1;
      word &= word - 1;
      oci[pos] = w.x + t * 32 + b;
      orow[pos] = i;
      ++pos;
    }
  }
}

// position of column c in output row i (its sorted columns O.ci[o0 .. o0 + no)), or -1
__device__ __forceinline__ int out_pos(const PatView& O, int o0, int no, int c) {
  int lo = 0, hi = no;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (O.ci[o0 + mid] < c) lo = mid + 1; else hi = mid;
  }
  return (lo < no && O.ci[o0 + lo] == c) ? lo : -1;
}

// Pair lists of the density-matrix products: per output tile of row i, its
// (A, B) tile pairs in increasing k.  Output positions are found by binary
// search in the row, so only the row's output count (at most MAXW, checked on
// the host) bounds the LDS counters, not the width of the column window.
__global__ __launch_bounds__(SYM_THREADS) void k_pair_count(int row0, PatView A, PatView B, PatView O,
                                                          const int2* __restrict__ win,
                                                          int64_t* __restrict__ pcnt) {
  __shared__ int cnt[MAXW];
  const int i = row0 + blockIdx.x;
  const int2 w = win[i];
  const int o0 = O.rp[i], no = O.rp[i + 1] - o0;
  for (int t = threadIdx.x; t < no; t += blockDim.x) cnt[t] = 0;
  __syncthreads();
  for (int e = A.rp[i] + threadIdx.x; e < A.rp[i + 1]; e += blockDim.x) {
    const int k = A.ci[e];
    for (int jj = B.rp[k]; jj < B.rp[k + 1]; ++jj) {
      const int c = B.ci[jj];
      const int p = (c >= w.x && c < w.y) ? out_pos(O, o0, no, c) : -1;
      if (p >= 0) atomicAdd(&cnt[p], 1);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < no; t += blockDim.x) pcnt[o0 + t] = cnt[t];
}

__global__ __launch_bounds__(SYM_THREADS) void k_pair_fill(int row0, PatView A, PatView B, PatView O,
                                                         const int2* __restrict__ win,
                                                         const int64_t* __restrict__ pp,
                                                         int2* __restrict__ pairs) {
  __shared__ int fill[MAXW];
  const int i = row0 + blockIdx.x;
  const int2 w = win[i];
  const int o0 = O.rp[i], no = O.rp[i + 1] - o0;
  for (int t = threadIdx.x; t < no; t += blockDim.x) fill[t] = 0;
  __syncthreads();
  // k in increasing order; within one k every output column is hit at most once
  for (int e = A.rp[i]; e < A.rp[i + 1]; ++e) {
    const int k = A.ci[e];
    const int at = a_tile(A, e);
    for (int jj = B.rp[k] + threadIdx.x; jj < B.rp[k + 1]; jj += blockDim.x) {
      const int c = B.ci[jj];
      const int p = (c >= w.x && c < w.y) ? out_pos(O, o0, no, c) : -1;
      if (p >= 0) {
        const int64_t slot = pp[o0 + p] + fill[p];
        fill[p] += 1;
        pairs[slot] = make_int2(at, B.ti ? B.ti[jj] : jj);
      }
    }
    __syncthreads();
  }
}

// index of tile (rows[e], cols[e]) in pattern P, or -1
__global__ void k_find_tiles(int64_t n, const int* __restrict__ rows, const int* __restrict__ cols,
                             PatView P, int* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int r = rows[e], c = cols[e];
  int lo = P.rp[r], hi = P.rp[r + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (P.ci[mid] < c) lo = mid + 1; else hi = mid;
  }
  out[e] = (lo < P.rp[r + 1] && P.ci[lo] == c) ? lo : -1;
}

// transposed pattern: row g of A^T lists rows b of A (inside the window) holding column g
__global__ __launch_bounds__(SYM_THREADS) void k_transpose(int row0, PatView A, const int2* __restrict__ win,
                                                         const int* __restrict__ trp, int* __restrict__ cnt,
                                                         int* __restrict__ tci, int* __restrict__ tti) {
  __shared__ int flag[SYM_THREADS];
  __shared__ int base;
  const int g = row0 + blockIdx.x;
  const int2 w = win[g];
  if (threadIdx.x == 0) base = trp ? trp[g] : 0;
  __syncthreads();
  int total = 0;
  for (int b0 = w.x; b0 < w.y; b0 += SYM_THREADS) {
    const int b = b0 + threadIdx.x;
    int hit = -1;
    if (b < w.y) {
      int lo = A.rp[b], hi = A.rp[b + 1];
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A.ci[mid] < g) lo = mid + 1; else hi = mid;
      }
      if (lo < A.rp[b + 1] && A.ci[lo] == g) hit = lo;
    }
    flag[threadIdx.x] = hit >= 0 ? 1 : 0;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int t = 1; t < SYM_THREADS; ++t) flag[t] += flag[t - 1];
    __syncthreads();
    if (trp && hit >= 0) {
      const int slot = base + total + flag[threadIdx.x] - 1;
      tci[slot] = b;
      tti[slot] = hit;
    }
    total += flag[SYM_THREADS - 1];
    __syncthreads();
  }
  if (!trp && threadIdx.x == 0) cnt[blockIdx.x] = total;
}

__global__ void k_rows_of(int nrows, const int* __restrict__ rp, int* __restrict__ rows) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  for (int e = rp[r]; e < rp[r + 1]; ++e) rows[e] = r;
}


// ---------------------------------------------------------------- grouped work lists
// Output tiles of one output row are taken NT at a time ("groups").  A group's
// entries are the k of A.row(i), in increasing order, for which at least one
// of the group's NT output columns j has B(k, j) stored; an entry holds the A
// tile index and NT B tile indices (-1 where B(k, j) is absent).  A wave can
// then load the A tile once per k for all NT outputs of its group.
__device__ __forceinline__ int find_in_row(const PatView& B, int k, int j) {
  int lo = B.rp[k], hi = B.rp[k + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (B.ci[mid] < j) lo = mid + 1; else hi = mid;
  }
  return (lo < B.rp[k + 1] && B.ci[lo] == j) ? lo : -1;
}

template <bool FILL>
__global__ __launch_bounds__(SYM_THREADS) void k_group_lists(PatView A, PatView B, PatView O, int NT,
                                                           const int* __restrict__ gbase, int64_t* __restrict__ gcnt,
                                                           int64_t* __restrict__ gpres, const int64_t* __restrict__ gp,
                                                           int* __restrict__ ent, int* __restrict__ go0,
                                                           int* __restrict__ gn) {
  const int i = blockIdx.x;
  const int o0 = O.rp[i], no = O.rp[i + 1] - o0;
  const int ng = (no + NT - 1) / NT;
  for (int gl = threadIdx.x; gl < ng; gl += blockDim.x) {
    const int g = gbase[i] + gl;
    const int ob = o0 + gl * NT;
    const int cnt = min(NT, o0 + no - ob);
    int64_t m = 0, pres = 0;
    const int64_t base = FILL ? gp[g] : 0;
    for (int e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int k = A.ci[e];
      int bidx[8];
      bool any = false;
      for (int u = 0; u < NT; ++u) {
        bidx[u] = u < cnt ? find_in_row(B, k, O.ci[ob + u]) : -1;
        if (bidx[u] >= 0) {
          any = true;
          ++pres;
        }
      }
      if (!any) continue;
      if (FILL) {
        int* row = ent + (base + m) * (1 + NT);
        row[0] = a_tile(A, e);
        for (int u = 0; u < NT; ++u) row[1 + u] = bidx[u] >= 0 ? (B.ti ? B.ti[bidx[u]] : bidx[u]) : -1;
      }
      ++m;
    }
    if (!FILL) {
      gcnt[g] = m;
      gpres[g] = pres;
      go0[g] = ob;
      gn[g] = cnt;
    }
  }
}

// ------------------------------------------------------- row-group work lists
// A row group is P consecutive output rows i0 .. i0+P-1 (of one system); its
// groups are the output columns j stored in any of those rows, one group per
// column.  A group's entries are the k of the union of A.row(i0+u), in
// increasing order, with B(k, j) stored and A(i0+u, k) stored for at least one
// u; an entry holds the B tile index (shared by the P outputs) and P A tile
// indices, -2 - t where A(i0+u, k) is absent (t: the entry's first present A
// tile, so a wave that loads unconditionally reads a tile it loads anyway, not
// one tile that every wave of the launch would read).  For the n x n projections (A = C^T,
// B = the H C pattern) a wave then loads each H D, S D tile once for P output
// rows: those tiles are the operands that other output rows reuse from far
// away in time, so this form halves their loads at P = 2.
// The column j is owned by the first row of the group that stores it; the
// group of column j is numbered by a scan over the owning output tiles in tile
// order, i.e. row by row and by column inside a row.
__global__ void k_rg_owned(int64_t ntiles, const int* __restrict__ orow, PatView O, const int* __restrict__ rfirst,
                           int* __restrict__ own) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  const int i = orow[t], j = O.ci[t];
  int o = 1;
  for (int r = rfirst[i]; r < i; ++r)
    if (find_in_row(O, r, j) >= 0) { o = 0; break; }
  own[t] = o;
}

template <bool FILL>
__global__ void k_rg_lists(int64_t ntiles, int P, const int* __restrict__ orow, PatView O, PatView A, PatView B,
                           const int* __restrict__ rfirst, const int* __restrict__ rend,
                           const int* __restrict__ row_sys, const int* __restrict__ own,
                           const int* __restrict__ gidx, int64_t* __restrict__ gcnt, int64_t* __restrict__ gpres,
                           const int64_t* __restrict__ gp, int* __restrict__ ent, int* __restrict__ gto,
                           int4* __restrict__ meta) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles || !own[t]) return;
  const int g = gidx[t];
  const int i = orow[t], j = O.ci[t];
  const int i0 = rfirst[i], nr = rend[i] - i0;   // nr <= P
  int cur[4], end[4];
  for (int u = 0; u < 4; ++u) {
    cur[u] = u < nr ? A.rp[i0 + u] : 0;
    end[u] = u < nr ? A.rp[i0 + u + 1] : 0;
  }
  int64_t m = 0, pres = 0;
  const int64_t base = FILL ? gp[g] : 0;
  for (;;) {   // P-way merge of the A rows, k increasing
    int k = 0x7fffffff;
    for (int u = 0; u < nr; ++u)
      if (cur[u] < end[u]) k = min(k, A.ci[cur[u]]);
    if (k == 0x7fffffff) break;
    const int bi = find_in_row(B, k, j);
    int at[4] = {-1, -1, -1, -1}, first = -1;
    for (int u = 0; u < nr; ++u)
      if (cur[u] < end[u] && A.ci[cur[u]] == k) {
        at[u] = a_tile(A, cur[u]);
        ++cur[u];
        if (first < 0) first = at[u];
        if (bi >= 0) ++pres;
      }
    if (bi < 0) continue;
    if (FILL) {   // an absent A tile is written -2 - t, t the entry's first present A tile
      int* row = ent + (base + m) * (1 + P);
      row[0] = B.ti ? B.ti[bi] : bi;
      for (int u = 0; u < P; ++u) row[1 + u] = at[u] >= 0 ? at[u] : -2 - first;
    }
    ++m;
  }
  if (!FILL) {
    gcnt[g] = m;
    gpres[g] = pres;
    for (int u = 0; u < P; ++u) gto[(size_t)g * P + u] = u < nr ? find_in_row(O, i0 + u, j) : -1;
    meta[g] = make_int4((int)t, P, row_sys[i], 0);
  }
}

__global__ void k_group_base(int nrows, const int* __restrict__ orp, int NT, int* __restrict__ ng) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int no = orp[i + 1] - orp[i];
  ng[i] = (no + NT - 1) / NT;
}

}  // namespace

void group_counts(hipStream_t st, int nrows, const int* orp, int NT, int* ng) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_group_base, dim3((nrows + 255) / 256), dim3(256), 0, st, nrows, orp, NT, ng);
  OMM_HIP(hipGetLastError());
}

void rg_owned(hipStream_t st, int64_t ntiles, const int* orow, PatView O, const int* rfirst, int* own) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_rg_owned, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, st, ntiles, orow, O, rfirst,
                     own);
  OMM_HIP(hipGetLastError());
}

void rg_lists(hipStream_t st, int64_t ntiles, int P, const int* orow, PatView O, PatView A, PatView B,
              const int* rfirst, const int* rend, const int* row_sys, const int* own, const int* gidx, int64_t* gcnt,
              int64_t* gpres, const int64_t* gp, int* ent, int* gto, int4* meta) {
  if (ntiles <= 0) return;
  const dim3 grid((unsigned)((ntiles + 255) / 256));
  if (!gp)
    hipLaunchKernelGGL(k_rg_lists<false>, grid, dim3(256), 0, st, ntiles, P, orow, O, A, B, rfirst, rend, row_sys,
                       own, gidx, gcnt, gpres, gp, ent, gto, meta);
  else
    hipLaunchKernelGGL(k_rg_lists<true>, grid, dim3(256), 0, st, ntiles, P, orow, O, A, B, rfirst, rend, row_sys,
                       own, gidx, gcnt, gpres, gp, ent, gto, meta);
  OMM_HIP(hipGetLastError());
}

void group_lists(hipStream_t st, int nrows, PatView A, PatView B, PatView O, int NT, const int* gbase,
                 int64_t* gcnt, int64_t* gpres, const int64_t* gp, int* ent, int* go0, int* gn) {
  if (nrows <= 0) return;
  if (!gp)
    hipLaunchKernelGGL(k_group_lists<false>, dim3(nrows), dim3(SYM_THREADS), 0, st, A, B, O, NT, gbase, gcnt, gpres,
                       gp, ent, go0, gn);
  else
    hipLaunchKernelGGL(k_group_lists<true>, dim3(nrows), dim3(SYM_THREADS), 0, st, A, B, O, NT, gbase, gcnt, gpres,
                       gp, ent, go0, gn);
  OMM_HIP(hipGetLastError());
}

namespace {
__global__ void k_entry_steps(int ngroups, int NT, const int64_t* __restrict__ gp, const int4* __restrict__ meta,
                              int* __restrict__ ent, const uint32_t* __restrict__ acm,
                              const uint32_t* __restrict__ brm, unsigned long long* __restrict__ act) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  const int W = 1 + NT;
  unsigned long long kept = 0;
  for (int64_t e = gp[g]; e < gp[g + 1]; ++e) {
    int* row = ent + e * W;
    const uint32_t am = acm[row[0]];
    for (int u = 0; u < NT; ++u) {
      const int bt = row[1 + u];
      if (bt < 0) continue;
      const uint32_t m = am & brm[bt];
      const int steps = ((m & 0xfu) ? 1 : 0) | ((m & 0xf0u) ? 2 : 0) | ((m & 0xf00u) ? 4 : 0) | ((m & 0xf000u) ? 8 : 0);
      row[1 + u] = bt | ((~steps & 15) << 27);
      kept += __popc(steps);
    }
  }
  atomicAdd(act + meta[g].z, kept);
}

__global__ void k_group_meta(int ngroups, const int* __restrict__ go0, const int* __restrict__ gn,
                             const int* __restrict__ orow, const int* __restrict__ row_sys, int4* __restrict__ meta) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  const int o0 = go0[g];
  meta[g] = make_int4(o0, gn[g], row_sys[orow[o0]], 0);
}
}  // namespace

void entry_steps(hipStream_t st, int ngroups, int NT, const int64_t* gp, const int4* meta, int* ent,
                 const uint32_t* acm, const uint32_t* brm, unsigned long long* act) {
  if (ngroups <= 0) return;
  hipLaunchKernelGGL(k_entry_steps, dim3((ngroups + 255) / 256), dim3(256), 0, st, ngroups, NT, gp, meta, ent, acm,
                     brm, act);
  OMM_HIP(hipGetLastError());
}

void group_meta(hipStream_t st, int ngroups, const int* go0, const int* gn, const int* orow, const int* row_sys,
                int4* meta) {
  if (ngroups <= 0) return;
  hipLaunchKernelGGL(k_group_meta, dim3((ngroups + 255) / 256), dim3(256), 0, st, ngroups, go0, gn, orow, row_sys,
                     meta);
  OMM_HIP(hipGetLastError());
}

void sym_count(hipStream_t st, int nrows, int row0, PatView A, PatView B, const int2* win, int* cnt) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_sym_count, dim3(nrows), dim3(SYM_THREADS), 0, st, row0, A, B, win, cnt);
  OMM_HIP(hipGetLastError());
}

void sym_fill(hipStream_t st, int nrows, int row0, PatView A, PatView B, const int2* win,
              const int* orp, int* oci, int* orow) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_sym_fill, dim3(nrows), dim3(SYM_THREADS), 0, st, row0, A, B, win, orp, oci, orow);
  OMM_HIP(hipGetLastError());
}

void pair_count(hipStream_t st, int nrows, int row0, PatView A, PatView B, PatView O, const int2* win,
                int64_t* pcnt) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_pair_count, dim3(nrows), dim3(SYM_THREADS), 0, st, row0, A, B, O, win, pcnt);
  OMM_HIP(hipGetLastError());
}

void pair_fill(hipStream_t st, int nrows, int row0, PatView A, PatView B, PatView O, const int2* win,
               const int64_t* pp, int2* pairs) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_pair_fill, dim3(nrows), dim3(SYM_THREADS), 0, st, row0, A, B, O, win, pp, pairs);
  OMM_HIP(hipGetLastError());
}

void find_tiles(hipStream_t st, int64_t n, const int* rows, const int* cols, PatView P, int* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_find_tiles, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, rows, cols, P, out);
  OMM_HIP(hipGetLastError());
}

void transpose_count(hipStream_t st, int nrows, int row0, PatView A, const int2* win, int* cnt) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_transpose, dim3(nrows), dim3(SYM_THREADS), 0, st, row0, A, win,
                     (const int*)nullptr, cnt, (int*)nullptr, (int*)nullptr);
  OMM_HIP(hipGetLastError());
}

void transpose_fill(hipStream_t st, int nrows, int row0, PatView A, const int2* win, const int* trp,
                    int* tci, int* tti) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_transpose, dim3(nrows), dim3(SYM_THREADS), 0, st, row0, A, win, trp, (int*)nullptr,
                     tci, tti);
  OMM_HIP(hipGetLastError());
}

void rows_of(hipStream_t st, int nrows, const int* rp, int* rows) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_rows_of, dim3((nrows + 255) / 256), dim3(256), 0, st, nrows, rp, rows);
  OMM_HIP(hipGetLastError());
}

// Exclusive prefix sums of integer counts (row pointers, work-list offsets).
// Three passes: each workgroup scans SCAN_ITEMS consecutive values per thread
// (a thread's own running sum, then the workgroup's thread totals by a
// Hillis-Steele scan in LDS) and writes its total; the totals are scanned the
// same way (recursively); a last pass adds each workgroup's offset.  Integer
// sums, so the result is exact whatever the order.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int64_t SCAN_TILE = (int64_t)SCAN_THREADS * SCAN_ITEMS;

template <typename I>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(const I* __restrict__ in, I* __restrict__ out,
                                                           I* __restrict__ totals, int64_t n) {
  __shared__ I sh[SCAN_THREADS];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  I v[SCAN_ITEMS];
  I run = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? in[base + k] : (I)0;
    run += v[k];
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  for (int d = 1; d < SCAN_THREADS; d <<= 1) {   // inclusive scan of the thread totals
    const I add = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : (I)0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  I acc = threadIdx.x > 0 ? sh[threadIdx.x - 1] : (I)0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = acc;
    acc += v[k];
  }
  if (threadIdx.x == SCAN_THREADS - 1 && totals) totals[blockIdx.x] = sh[SCAN_THREADS - 1];
}

template <typename I>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add(I* __restrict__ out, const I* __restrict__ offs,
                                                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
  const I o = offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t e = i + (int64_t)k * SCAN_THREADS;
    if (e < n) out[e] += o;
  }
}

template <typename I>
static void excl_scan_impl(hipStream_t st, const I* in, I* out, int64_t n) {
  if (n <= 0) return;
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_tiles<I>, dim3(1), dim3(SCAN_THREADS), 0, st, in, out, (I*)nullptr, n);
    OMM_HIP(hipGetLastError());
    return;
  }
  void* buf = nullptr;
  OMM_HIP(hipMallocAsync(&buf, 2 * nb * sizeof(I), st));
  I* totals = (I*)buf;
  I* offs = totals + nb;
  hipLaunchKernelGGL(k_scan_tiles<I>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, in, out, totals, n);
  OMM_HIP(hipGetLastError());
  excl_scan_impl<I>(st, totals, offs, nb);
  hipLaunchKernelGGL(k_scan_add<I>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, out, (const I*)offs, n);
  OMM_HIP(hipGetLastError());
  OMM_HIP(hipFreeAsync(buf, st));
}

void excl_scan(hipStream_t st, const int* in, int* out, int64_t n) { excl_scan_impl<int>(st, in, out, n); }
void excl_scan64(hipStream_t st, const int64_t* in, int64_t* out, int64_t n) {
  excl_scan_impl<int64_t>(st, in, out, n);
}

}  // namespace omm
