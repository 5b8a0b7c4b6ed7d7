// n x n projections of one CG iteration (Sec. III B of arXiv 2209.05934):
// X = C^T SD, Y = C^T HD, S2 = D^T SD, H2 = D^T HD, or at start-up S0 = C^T SC
// and H0 = C^T HC; MFMA tiles over the tile-pair work lists of the n x n pattern.
#include "tile_sched.hpp"

namespace omm {

namespace {

// ------------------------------------------------------------------ S2: n x n projections
// Groups of NT output tiles in one row g of the n x n pattern: per basis tile b
// the C(b,g) and D(b,g) tiles are loaded once for NT tiles of HD and SD.
// S2 = D^T S D and H2 = D^T H D are symmetric: they are formed and stored for
// tiles on or above the diagonal only, and readers take a tile below it as the
// transpose of its mirror (X and Y are not symmetric and are formed in full).
// Inside a diagonal tile the elements below the diagonal take their mirror
// elements (after the block filter), so the kept product is exactly the
// symmetric matrix of its upper triangle, filtered or not.
template <typename TI, typename TM, typename TO, int NPROD, int KS, int NT, bool ROLL>
__global__ __launch_bounds__(Split<KS>::NW * 64) void k_s2(
    GroupView P, const int* __restrict__ orow, const int* __restrict__ ocol, const SysInfo* __restrict__ info, const SysState* __restrict__ st, int mask, const TI* __restrict__ Cm,
    const TI* __restrict__ Dm, const TM* __restrict__ HDm, const TM* __restrict__ SDm, TO* __restrict__ X,
    TO* __restrict__ Y, TO* __restrict__ S2o, TO* __restrict__ H2o, const uint8_t* __restrict__ wseg) {
  typedef typename Acc<TI>::V V;
  typedef Split<KS> SP;
  constexpr int W = 1 + NT;
  __shared__ V red[SP::RED * NPROD * NT * 64];
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int grp = wave / KS, wk = wave - grp * KS;
  const int g = xcd_block(P.xrun) * SP::G + grp;
  const bool valid = g < P.ngroups;
  constexpr int D = pipe_depth<TI>((NPROD == 4 ? 2 : 1) + 2 * NT);
  int4 m = make_int4(0, 0, 0, 0);
  int64_t b = 0, e = 0;
  if (valid) {
    m = group_meta(P, g);
    ks_chunk(P, g, wk, KS, b, e);
  }
  EntryRounds<W, D> er(P.ent, b, e, lane);
  const int o0 = m.x, cnt = m.y, s = m.z;
  const int phase = ld_early(&st[s].phase);
  const double e2 = ld_early(&info[s].eps2);
  // output tile below the diagonal: no S2, H2 products; at start-up (S0, H0,
  // both symmetric) no products at all, the tile is mirrored from above afterwards
  bool low[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int t = min(o0 + u, o0 + max(cnt, 1) - 1);
    low[u] = valid && ld_early(&orow[t]) > ld_early(&ocol[t]);
  }
  const bool act = valid && (phase & mask) != 0;
  V acc[NPROD * NT];
#pragma unroll
  for (int a = 0; a < NPROD * NT; ++a) acc[a] = vzero<V>();
  bool all_low = true;   // every output tile of the group below the diagonal: no D loads (no loads at start-up)
#pragma unroll
  for (int u = 0; u < NT; ++u) all_low = all_low && (u >= cnt || low[u]);
  struct Stage { Frag<TI> c, d, hd[NT], sd[NT]; };
  auto body = [&](auto skip_d) {
    constexpr bool SKIP = decltype(skip_d)::value;
    run_entries<W, D, Stage, ROLL>(
        er, lane,
        [&](Stage& f, const int (&id)[W]) {
          ld_col(f.c, Cm + (size_t)id[0] * TE, lane);                 // A = C^T
          if constexpr (NPROD == 4 && !SKIP) ld_col(f.d, Dm + (size_t)id[0] * TE, lane);  // A = D^T
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            const size_t bt = (size_t)max(id[1 + u], 0) * TE;
            ld_col(f.hd[u], HDm + bt, lane);
            ld_col(f.sd[u], SDm + bt, lane);
          }
        },
        [&](const Stage& f, const int (&id)[W]) {
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            if (id[1 + u] >= 0 && !(NPROD == 2 && low[u])) {
              mma(acc[u], f.c, f.sd[u]);
              mma(acc[NT + u], f.c, f.hd[u]);
              if constexpr (NPROD == 4 && !SKIP) {
                if (!low[u]) {
                  mma(acc[2 * NT + u], f.d, f.sd[u]);
                  mma(acc[3 * NT + u], f.d, f.hd[u]);
                }
              }
            }
          }
        });
  };
  if (act && !(NPROD == 2 && all_low)) {
    if (NPROD == 4 && all_low) body(std::true_type{});
    else body(std::false_type{});
  }
  ks_reduce<KS, NPROD * NT>(acc, red, grp, wk, lane);
  if (!act || wk != 0) return;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    if (u >= cnt) break;
    if (NPROD == 2 && low[u]) continue;   // start-up: mirrored from above afterwards
    const int t = o0 + u;
    if (e2 > 0.0) {
      const uint8_t* rs = wseg + 32 * (size_t)orow[t];
      const uint8_t* cs = wseg + 32 * (size_t)ocol[t];
#pragma unroll
      for (int a = 0; a < NPROD; ++a) filter_tile(acc[a * NT + u], lane, rs, cs, e2);
    }
    if (NPROD == 4 && orow[t] == ocol[t]) {   // diagonal tile of S2, H2: upper triangle mirrored
#pragma unroll
      for (int a = 2; a < 4; ++a) {
        const V tr = transposed_tile(acc[a * NT + u], lane);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (Lay<V>::row(lane >> 4, r) > (lane & 15)) acc[a * NT + u][r] = tr[r];
      }
    }
    const size_t o = (size_t)t * TE;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = out_off<V, TO>(lane, r);
      X[o + e] = (TO)acc[u][r];
      Y[o + e] = (TO)acc[NT + u][r];
      if (NPROD == 4 && !low[u]) {
        S2o[o + e] = (TO)acc[2 * NT + u][r];
        H2o[o + e] = (TO)acc[3 * NT + u][r];
      }
    }
  }
}

// Row-group form: a wave computes the output tiles (i0+u, j), u < P, of P
// consecutive output rows in one column j.  Per entry (basis tile b) it loads
// the H D(b,j), S D(b,j) tiles once for the P outputs and the C(b,i0+u),
// D(b,i0+u) tiles of each row (-2 - t: row u has no tile at b, its products
// are skipped and the slot loads the entry's tile t instead).  H D and S D tiles are each read by every output row whose C
// column reaches their basis tile, rows far apart in the launch order, so they
// are the loads that miss the cache; here each such load serves P rows.  The
// sums run over the same (b, output) pairs in increasing b as the row-major
// groups, so the result is the same up to the split into KS chunks.
// At P = 2 in FP64 the kernel keeps two stages of operands in flight and asks
// for two waves per SIMD (212 registers, no spills); left to itself the
// compiler takes 276 registers and one wave per SIMD, which hides less latency.
template <typename TI, int P>
constexpr bool rg_two_waves() { return P == 2 && sizeof(TI) == 8; }

template <typename TI, typename TM, typename TO, int NPROD, int KS, int P, bool ROLL>
__global__ __launch_bounds__(Split<KS>::NW * 64) __attribute__((amdgpu_waves_per_eu(rg_two_waves<TI, P>() ? 2 : 1))) void k_s2r(
    GroupView G, const int* __restrict__ orow, const int* __restrict__ ocol, const SysInfo* __restrict__ info, const SysState* __restrict__ st, int mask, const TI* __restrict__ Cm,
    const TI* __restrict__ Dm, const TM* __restrict__ HDm, const TM* __restrict__ SDm, TO* __restrict__ X,
    TO* __restrict__ Y, TO* __restrict__ S2o, TO* __restrict__ H2o, const uint8_t* __restrict__ wseg) {
  typedef typename Acc<TI>::V V;
  typedef Split<KS> SP;
  constexpr int W = 1 + P;
  __shared__ V red[SP::RED * NPROD * P * 64];
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int grp = wave / KS, wk = wave - grp * KS;
  const int g = xcd_block(G.xrun) * SP::G + grp;
  const bool valid = g < G.ngroups;
  constexpr int D = rg_two_waves<TI, P>() ? 2 : pipe_depth<TI>((NPROD == 4 ? 2 : 1) * P + 2);
  int4 m = make_int4(0, 0, 0, 0);
  int64_t b = 0, e = 0;
  if (valid) {
    m = group_meta(G, g);
    ks_chunk(G, g, wk, KS, b, e);
  }
  EntryRounds<W, D> er(G.ent, b, e, lane);
  const int s = m.z;
  const int phase = ld_early(&st[s].phase);
  const double e2 = ld_early(&info[s].eps2);
  int to[P];
  bool low[P];   // output tile absent or below the diagonal: no S2, H2 products (none at start-up)
#pragma unroll
  for (int u = 0; u < P; ++u) {
    to[u] = valid ? ld_early(G.gto + (size_t)g * P + u) : -1;
    const int t = max(to[u], 0);
    low[u] = to[u] < 0 || ld_early(&orow[t]) > ld_early(&ocol[t]);
  }
  const bool act = valid && (phase & mask) != 0;
  V acc[NPROD * P];
#pragma unroll
  for (int a = 0; a < NPROD * P; ++a) acc[a] = vzero<V>();
  bool all_low = true;   // every output tile of the group absent or below the diagonal: no D loads
#pragma unroll
  for (int u = 0; u < P; ++u) all_low = all_low && low[u];
  struct Stage { Frag<TI> c[P], d[P], hd, sd; };
  auto body = [&](auto skip_d) {
    constexpr bool SKIP = decltype(skip_d)::value;
    run_entries<W, D, Stage, ROLL>(
        er, lane,
        [&](Stage& f, const int (&id)[W]) {
          const size_t bt = (size_t)id[0] * TE;
          ld_col(f.hd, HDm + bt, lane);
          ld_col(f.sd, SDm + bt, lane);
#pragma unroll
          for (int u = 0; u < P; ++u) {   // absent: -2 - t, a tile this entry loads anyway
            const int a = id[1 + u];
            const size_t at = (size_t)(a >= 0 ? a : -2 - a) * TE;
            ld_col(f.c[u], Cm + at, lane);                                             // A = C^T
            if constexpr (NPROD == 4 && !SKIP) ld_col(f.d[u], Dm + at, lane);          // A = D^T
          }
        },
        [&](const Stage& f, const int (&id)[W]) {
#pragma unroll
          for (int u = 0; u < P; ++u) {
            if (id[1 + u] >= 0 && !(NPROD == 2 && low[u])) {
              mma(acc[u], f.c[u], f.sd);
              mma(acc[P + u], f.c[u], f.hd);
              if constexpr (NPROD == 4 && !SKIP) {
                if (!low[u]) {
                  mma(acc[2 * P + u], f.d[u], f.sd);
                  mma(acc[3 * P + u], f.d[u], f.hd);
                }
              }
            }
          }
        });
  };
  if (act && !(NPROD == 2 && all_low)) {
    if (NPROD == 4 && all_low) body(std::true_type{});
    else body(std::false_type{});
  }
  ks_reduce<KS, NPROD * P>(acc, red, grp, wk, lane);
  if (!act || wk != 0) return;
  // absent output tiles store nothing; at start-up the tiles below the diagonal
  // are mirrored from above afterwards
  unrolled<P>([&](auto uc) __attribute__((always_inline)) {   // inlined: acc stays in registers
    constexpr int u = decltype(uc)::value;
    const int t = to[u];
    if (t >= 0 && !(NPROD == 2 && low[u])) {
      if (e2 > 0.0) {
        const uint8_t* rs = wseg + 32 * (size_t)orow[t];
        const uint8_t* cs = wseg + 32 * (size_t)ocol[t];
#pragma unroll
        for (int a = 0; a < NPROD; ++a) acc[a * P + u] = filtered(acc[a * P + u], lane, rs, cs, e2);
      }
      if (NPROD == 4 && orow[t] == ocol[t]) {   // diagonal tile of S2, H2: upper triangle mirrored
#pragma unroll
        for (int a = 2; a < 4; ++a) {
          const V tr = transposed_tile(acc[a * P + u], lane);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (Lay<V>::row(lane >> 4, r) > (lane & 15)) acc[a * P + u][r] = tr[r];
        }
      }
      const size_t o = (size_t)t * TE;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = out_off<V, TO>(lane, r);
        X[o + e] = (TO)acc[u][r];
        Y[o + e] = (TO)acc[P + u][r];
        if (NPROD == 4 && !low[u]) {
          S2o[o + e] = (TO)acc[2 * P + u][r];
          H2o[o + e] = (TO)acc[3 * P + u][r];
        }
      }
    }
  });
}

}  // namespace

template <typename TI, typename TM, typename TO, int NP>
static void s2_go(hipStream_t s, const Bufs& b, int mask, const TI* C, const TI* D, const TM* HD, const TM* SD,
                  TO* X, TO* Y, TO* S2, TO* H2) {
  if (b.s2.ngroups <= 0) return;
  if (b.s2.rows) {   // row-group list: 2 output rows per wave, at most 4 waves per group
    auto go = [&](auto pc, auto ksc) {
      constexpr int P_ = decltype(pc)::value, K_ = decltype(ksc)::value;
      if (b.roll)
        LAUNCH((k_s2r<TI, TM, TO, NP, K_, P_, true>), grid_for<K_>(b.s2.ngroups), block_for<K_>(), s, b.s2,
               b.tw_row, b.tw_col, b.info, b.st, mask, C, D, HD, SD, X, Y, S2, H2, b.wseg);
      else
        LAUNCH((k_s2r<TI, TM, TO, NP, K_, P_, false>), grid_for<K_>(b.s2.ngroups), block_for<K_>(), s, b.s2,
               b.tw_row, b.tw_col, b.info, b.st, mask, C, D, HD, SD, X, Y, S2, H2, b.wseg);
    };
    ks_of<2, 4>(b.ks[1], go);
    return;
  }
  nt_ks<1>(b.s2.NT, b.ks[1], [&](auto ntc, auto ksc) {
    constexpr int N_ = decltype(ntc)::value, K_ = decltype(ksc)::value;
    if (b.roll)
      LAUNCH((k_s2<TI, TM, TO, NP, K_, N_, true>), grid_for<K_>(b.s2.ngroups), block_for<K_>(), s, b.s2, b.tw_row,
             b.tw_col, b.info, b.st, mask, C, D, HD, SD, X, Y, S2, H2, b.wseg);
    else
      LAUNCH((k_s2<TI, TM, TO, NP, K_, N_, false>), grid_for<K_>(b.s2.ngroups), block_for<K_>(), s, b.s2, b.tw_row,
             b.tw_col, b.info, b.st, mask, C, D, HD, SD, X, Y, S2, H2, b.wseg);
  });
}

// one precision per object file (OMM_PREC 0: FP64, 1: FP32, 2: BF16)
#if OMM_PREC == 0
void launch_s2_p64(hipStream_t s, const Bufs& b, int mask, bool init) {
  if (init) {   // start-up products S0 = C^T S C, H0 = C^T H C (S C, H C in the S D, H D
                // tiles, untransposed) run on the unmarked list
    Bufs bf = b;
    bf.s2 = b.s2_full;
    s2_go<double, double, double, 2>(s, bf, mask, b.C, b.C, b.HD, b.SD, b.S0, b.H0, b.S2, b.H2);
  }
  else s2_go<double, double, double, 4>(s, b, mask, b.C, b.D, b.HD, b.SD, b.X, b.Y, b.S2, b.H2);
}
#elif OMM_PREC == 1
void launch_s2_p32(hipStream_t s, const Bufs& b, int mask) {
  s2_go<float, float, float, 4>(s, b, mask, (const float*)b.Cl, (const float*)b.Dl, b.HDf, b.SDf, b.Xf, b.Yf,
                                b.S2f, b.H2f);
}
#else
void launch_s2_pbf(hipStream_t s, const Bufs& b, int mask) {
  s2_go<bf16, float, float, 4>(s, b, mask, (const bf16*)b.Cl, (const bf16*)b.Dl, b.HDf, b.SDf, b.Xf, b.Yf, b.S2f,
                               b.H2f);
}
#endif

}  // namespace omm
