// Work scheduling shared by the tile-product kernels (direction products,
// n x n projections, gradient): per-system activity, block filtering of
// Sec. V, XCD-aware block numbering, split-K reduction and the software
// pipeline over tile-pair work lists; plus the host-side launch helpers.
#pragma once

#include <type_traits>
#include <utility>

#include "kernels.hpp"
#include "tile_ops.hpp"

namespace omm {

namespace {

template <Prec P> struct PT;
template <> struct PT<P64> { typedef double TI; typedef double TO; };
template <> struct PT<P32> { typedef float TI; typedef float TO; };
template <> struct PT<PBF> { typedef bf16 TI; typedef float TO; };

__device__ __forceinline__ bool on(const SysState* __restrict__ st, int s, int mask) {
  return (st[s].phase & mask) != 0;
}

// Zero every atom block of the accumulator tile whose Frobenius norm^2 < eps2
// (filtering of Sec. V).  Row/column segments give, for each tile row/column,
// the [lo, hi) range of its block inside the tile; rseg == nullptr means the
// whole tile height is one block.  Uniform shuffles, fixed summation order.
template <typename V>
__device__ void filter_tile(V& acc, int lane, const uint8_t* __restrict__ rseg,
                            const uint8_t* __restrict__ cseg, double eps2) {
  const int j = lane & 15, q = lane >> 4;
  const int clo = cseg[j], chi = cseg[16 + j];
  // Common case, decided for the whole wave: every column block is an aligned
  // pair of columns (two wavefunctions per atom) and every row block an aligned
  // pair of rows, or the whole tile height.  Then a block's sum of squares takes
  // three lane exchanges per register instead of a pass over the whole tile.
  bool pairs = clo == (j & ~1) && chi == clo + 2;
  if (rseg) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = Lay<V>::row(q, r), lo = row & ~1;
      pairs = pairs && rseg[row] == lo && rseg[16 + row] == lo + 2;
    }
  }
  if (__ballot(!pairs) == 0) {
    double cp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {   // the column pair (j, j ^ 1) of each register's row
      const double sq = (double)acc[r] * (double)acc[r];
      cp[r] = sq + __shfl_xor(sq, 1, 64);
    }
    double tot[4];
    if (!rseg) {   // the whole tile height: all 16 rows (4 registers x 4 lane quads)
      double t = (cp[0] + cp[1]) + (cp[2] + cp[3]);
      t += __shfl_xor(t, 16, 64);
      t += __shfl_xor(t, 32, 64);
#pragma unroll
      for (int r = 0; r < 4; ++r) tot[r] = t;
    } else if (sizeof(acc[0]) == 8) {   // FP64 layout: row 4r + q, its pair row in lane quad q ^ 1
#pragma unroll
      for (int r = 0; r < 4; ++r) tot[r] = cp[r] + __shfl_xor(cp[r], 16, 64);
    } else {                            // FP32 layout: row 4q + r, its pair row in register r ^ 1
#pragma unroll
      for (int r = 0; r < 4; ++r) tot[r] = cp[r & ~1] + cp[r | 1];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (tot[r] < eps2) acc[r] = 0;
    return;
  }
  double rowpart[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double sq = (double)acc[r] * (double)acc[r];
    double sum = 0.0;
    for (int c = 0; c < 16; ++c) {
      const double v = __shfl(sq, c + 16 * q, 64);
      if (c >= clo && c < chi) sum += v;
    }
    rowpart[r] = sum;
  }
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  for (int qq = 0; qq < 4; ++qq) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const double v = __shfl(rowpart[rr], j + 16 * qq, 64);
      const int rho = Lay<V>::row(qq, rr);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = Lay<V>::row(q, r);
        const bool in = rseg ? (rho >= rseg[row] && rho < rseg[16 + row]) : true;
        if (in) tot[r] += v;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (tot[r] < eps2) acc[r] = 0;
}

// The same on a tile taken and returned by value, always inlined.  A kernel
// with many accumulators where the compiler keeps `filter_tile` a call would
// otherwise pass it the address of one element of its accumulator array, and
// the whole array would live in scratch memory; here only the copy does.
template <typename V>
__device__ __forceinline__ V filtered(V acc, int lane, const uint8_t* __restrict__ rseg,
                                      const uint8_t* __restrict__ cseg, double eps2) {
  filter_tile(acc, lane, rseg, cseg, eps2);
  return acc;
}

// Work distribution of the tile-product kernels.  A workgroup holds NW = max(4, KS)
// waves; KS consecutive waves split the pair list of one output tile into KS
// contiguous chunks and add their accumulators in a fixed tree through LDS, so
// results are bitwise reproducible for a given KS.  Logical block ids are
// renumbered so that runs of `run` consecutive ids (neighbouring output
// tiles, which share operand tiles) run on one XCD while successive runs go to
// successive XCDs: the hardware deals workgroups to the 8 XCDs round-robin, so
// physical block p runs on XCD p % 8 as its (p / 8)-th block there.  Every
// part of the grid (every system of a batch) is thereby spread over all XCDs.
// The t blocks of an incomplete last cycle of 8 runs are cut into 8 contiguous
// ranges, one per XCD (t / 8 blocks, one more for the first t % 8 XCDs), so the
// groups of one output row stay on one XCD there too; the renumbering stays a
// bijection on [0, gridDim.x).
__device__ __forceinline__ int xcd_block(int run) {
  const int nb = gridDim.x, p = blockIdx.x;
  const int full = nb - nb % (8 * run);
  const int x = p & 7, k = p >> 3;
  if (p < full) return ((k / run) * 8 + x) * run + (k % run);
  const int t = nb - full, q = t >> 3, r = t & 7;
  return full + x * q + min(x, r) + ((p - full) >> 3);
}

template <int KS> struct Split {
  static constexpr int NW = KS > 4 ? KS : 4;     // waves per workgroup
  static constexpr int G = NW / KS;              // output tiles per workgroup
  static constexpr int RED = KS > 1 ? NW / 2 : 1;   // LDS slots of the reduction tree
};

template <int KS, int NACC, typename V>
__device__ __forceinline__ void ks_reduce(V (&acc)[NACC], V* buf, int grp, int wk, int lane) {
  if (KS == 1) return;
#pragma unroll
  for (int stride = KS / 2; stride >= 1; stride >>= 1) {
    if (wk >= stride && wk < 2 * stride) {
#pragma unroll
      for (int a = 0; a < NACC; ++a) buf[((grp * (KS / 2) + wk - stride) * NACC + a) * 64 + lane] = acc[a];
    }
    __syncthreads();
    if (wk < stride) {
#pragma unroll
      for (int a = 0; a < NACC; ++a) acc[a] += buf[((grp * (KS / 2) + wk) * NACC + a) * 64 + lane];
    }
    __syncthreads();
  }
}

// Wave index as a scalar: every per-wave quantity derived from it (group,
// chunk bounds, entry indices, loop counters) then lives in scalar registers
// and branches on it are scalar branches.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Stages of operand fragments kept in flight by run_entries for a stage of
// `tiles` fragments of type T (register budget about 96 VGPRs).
template <typename T>
constexpr int pipe_depth(int tiles) {
  return tiles * (int)(sizeof(Frag<T>) / 4) <= 24 ? 4 : (tiles * (int)(sizeof(Frag<T>) / 4) <= 48 ? 3 : 2);
}

// A load issued where it is written: relaxed atomic loads are ordered memory
// operations, which the compiler does not sink past the branches that follow,
// so operands of later work are in flight while a data-dependent test (the
// system's phase) resolves.
template <typename T>
__device__ __forceinline__ T ld_early(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// The entry indices of a wave's chunk [b, e) of a group list (W ints per
// entry), in rounds of PB entries (a multiple of D, at most 64 / W): a round
// sits in one register per lane and the next one is fetched a round ahead.
// Constructing it issues the first two rounds' loads.
template <int W, int D>
struct EntryRounds {
  static constexpr int PB = (64 / W) / D * D;
  static_assert(PB >= D, "pipeline deeper than a round");
  const int* ent;
  const int* base;
  int n, cur, nxt;
  // every lane loads (lanes past the round's end read the list's first word,
  // which always exists), so the loads are not held behind a lane mask
  __device__ __forceinline__ int batch(int r0, int lane) const {
    const int left = n - r0;
    const int cnt = left <= 0 ? 0 : (left >= PB ? PB : left);
    return ld_early(lane < cnt * W ? base + (size_t)r0 * W + lane : ent);
  }
  __device__ __forceinline__ EntryRounds(const int* list, int64_t b, int64_t e, int lane)
      : ent(list), base(list + b * W), n((int)(e - b)) {
    cur = batch(0, lane);
    nxt = batch(PB, lane);
  }
};

// Software pipeline over the entries of an EntryRounds: D stages of operand
// fragments are in flight; load(stage, idx) issues the tile loads of one
// entry and use(stage, idx) runs its MFMAs, in entry order.  Indices are read
// from the round registers with uniform lane reads, so no tile address waits
// on an index load.  A round is unrolled in full and every step issues its
// loads unconditionally (past the end it reloads the last entry), so the
// compiler knows at each use exactly how many younger loads are in flight and
// waits for that stage alone; the look-ahead runs across round boundaries, so
// the pipeline never drains.  ROLL: a round is a loop over groups of D entries
// with only the D stages unrolled, several times less code (multi-system
// launches, which run many kernels and shapes per iteration, are faster with
// it; single systems are faster unrolled).
template <int W, int D, typename St, bool ROLL = false, typename LoadF, typename UseF>
__device__ __forceinline__ void run_entries(EntryRounds<W, D>& er, int lane, LoadF&& load, UseF&& use) {
  constexpr int PB = EntryRounds<W, D>::PB;
  const int n = er.n;
  if (n <= 0) return;
  St stg[D];
  int id[D][W];
#pragma unroll
  for (int s = 0; s < D; ++s) {
    const int q = s < n ? s : n - 1;
#pragma unroll
    for (int w = 0; w < W; ++w) id[s][w] = __builtin_amdgcn_readlane(er.cur, q * W + w);
    load(stg[s], id[s]);
  }
  if constexpr (ROLL) {
    for (int r0 = 0;; r0 += PB) {
#pragma unroll 1
      for (int k0 = 0; k0 < PB; k0 += D) {
#pragma unroll
        for (int j = 0; j < D; ++j) {   // entry k0 + j in stage j (k0 is a multiple of D)
          const int k = k0 + j;
          if (r0 + k >= n) return;
          use(stg[j], id[j]);
          const int q = (r0 + k + D < n ? r0 + k + D : n - 1) - r0;
          if (q < PB) {
#pragma unroll
            for (int w = 0; w < W; ++w) id[j][w] = __builtin_amdgcn_readlane(er.cur, q * W + w);
          } else {
#pragma unroll
            for (int w = 0; w < W; ++w) id[j][w] = __builtin_amdgcn_readlane(er.nxt, (q - PB) * W + w);
          }
          load(stg[j], id[j]);
        }
      }
      er.cur = er.nxt;
      er.nxt = er.batch(r0 + 2 * PB, lane);
    }
  } else {
    for (int r0 = 0;; r0 += PB) {
#pragma unroll
      for (int k = 0; k < PB; ++k) {
        if (r0 + k >= n) return;
        use(stg[k % D], id[k % D]);
        // entry r0 + k + D (clamped to the last one) lives in this round or the next
        const int q = (r0 + k + D < n ? r0 + k + D : n - 1) - r0;
        if (q < PB) {
#pragma unroll
          for (int w = 0; w < W; ++w) id[k % D][w] = __builtin_amdgcn_readlane(er.cur, q * W + w);
        } else {
#pragma unroll
          for (int w = 0; w < W; ++w) id[k % D][w] = __builtin_amdgcn_readlane(er.nxt, (q - PB) * W + w);
        }
        load(stg[k % D], id[k % D]);
      }
      er.cur = er.nxt;
      er.nxt = er.batch(r0 + 2 * PB, lane);
    }
  }
}

// f(integral_constant<int, i>) for i = 0 .. N-1, unrolled in the source: loops
// whose bodies inline large helpers (the block filter) can exceed the size up
// to which the compiler honours an unroll pragma, and a loop left rolled over
// register arrays puts them in scratch memory.
template <typename F, int... I>
__device__ __forceinline__ void unrolled_seq(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void unrolled(F&& f) {
  unrolled_seq(f, std::make_integer_sequence<int, N>{});
}

// group record (first output tile, output tiles, system) via early loads
__device__ __forceinline__ int4 group_meta(const GroupView& P, int g) {
  const int* m = reinterpret_cast<const int*>(P.meta + g);
  return make_int4(ld_early(m), ld_early(m + 1), ld_early(m + 2), 0);
}

// chunk [b, e) of group g's entry list handled by split-wave wk
__device__ __forceinline__ void ks_chunk(const GroupView& P, int g, int wk, int KS, int64_t& b, int64_t& e) {
  const int64_t p0 = ld_early(P.gp + g), n = ld_early(P.gp + g + 1) - p0;
  b = p0 + (n * wk) / KS;
  e = p0 + (n * (wk + 1)) / KS;
}

}  // namespace

#define LAUNCH(kern, grid, block, stream, ...)                                   \
  do {                                                                          \
    hipLaunchKernelGGL(kern, grid, block, 0, stream, __VA_ARGS__);              \
    OMM_HIP(hipGetLastError());                                                 \
  } while (0)

template <int KS> static dim3 grid_for(int n) { return dim3((unsigned)((n + Split<KS>::G - 1) / Split<KS>::G)); }
template <int KS> static dim3 block_for() { return dim3(Split<KS>::NW * 64); }

// (NT, KS) dispatch: NT output tiles per wave in {1, 2, 4}, KS waves per
// output group in {1, 2, 4, 8} up to max_split(step, NT) (eight waves of a
// workgroup get at most 256 registers each, too few for the widest groups);
// shapes beyond the limit are neither compiled nor launched
template <int NT, int MAXKS, typename F>
static void ks_of(int ks, F&& f) {
  if (MAXKS >= 8 && ks >= 8) f(std::integral_constant<int, NT>{}, std::integral_constant<int, (MAXKS >= 8 ? 8 : 1)>{});
  else if (ks >= 4) f(std::integral_constant<int, NT>{}, std::integral_constant<int, 4>{});
  else if (ks >= 2) f(std::integral_constant<int, NT>{}, std::integral_constant<int, 2>{});
  else f(std::integral_constant<int, NT>{}, std::integral_constant<int, 1>{});
}
template <int STEP, typename F>
static void nt_ks(int nt, int ks, F&& f) {
  if (nt == 4) ks_of<4, max_split(STEP, 4)>(ks, f);
  else if (nt == 2) ks_of<2, max_split(STEP, 2)>(ks, f);
  else ks_of<1, max_split(STEP, 1)>(ks, f);
}

}  // namespace omm
