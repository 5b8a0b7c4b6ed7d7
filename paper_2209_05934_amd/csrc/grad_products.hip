// Gradient of the OMM functional on C's pattern (Eq. 4 of arXiv 2209.05934):
// G = 8 HC - 4 (HC S0 + SC H0), with the two sums <G, G> and <G, G_old> per
// tile that the Polak-Ribiere step needs.
#include "tile_sched.hpp"

namespace omm {

namespace {

// ------------------------------------------------------------------ gradient on C's pattern
// Groups of NT tiles of C's pattern in one basis row b: per k the HC(b,k) and
// SC(b,k) tiles are loaded once for NT tiles of S_W and H_W.  An entry's S_W/H_W
// tile index carries the MFMA steps (groups of four wavefunctions of tile k)
// where HC(b,k) has no nonzero column or S_W(k,g) no nonzero row: those steps
// are skipped (STEPS: contexts with block-sparse systems; dense ones keep every
// step and run the straight-line form, whose MFMAs are not split by branches).
template <typename TI, int KS, int NT, bool ROLL, bool STEPS>
__global__ __launch_bounds__(Split<KS>::NW * 64) void k_grad(
    GroupView P, const SysState* __restrict__ st, int mask, const TI* __restrict__ HCm,
    const TI* __restrict__ SCm, const TI* __restrict__ S0m, const TI* __restrict__ H0m,
    const double* __restrict__ HC, const int* __restrict__ c_in_hc,
    const uint32_t* __restrict__ cmask, const double* __restrict__ Gold, double* __restrict__ G,
    double* __restrict__ gpart, const TI* __restrict__ zt, int keep_all) {
  typedef typename Acc<TI>::V V;
  typedef Split<KS> SP;
  constexpr int W = 1 + NT;
  __shared__ V red[SP::RED * NT * 64];
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int grp = wave / KS, wk = wave - grp * KS;
  const int g = xcd_block(P.xrun) * SP::G + grp;
  const bool valid = g < P.ngroups;
  constexpr int D = pipe_depth<TI>(2 + 2 * NT);
  int4 m = make_int4(0, 0, 0, 0);
  int64_t b = 0, e = 0;
  if (valid) {
    m = group_meta(P, g);
    ks_chunk(P, g, wk, KS, b, e);
  }
  EntryRounds<W, D> er(P.ent, b, e, lane);
  const int o0 = m.x, cnt = m.y;
  const int phase = ld_early(&st[m.z].phase);
  const bool act = valid && (phase & mask) != 0;
  V acc[NT];
#pragma unroll
  for (int a = 0; a < NT; ++a) acc[a] = vzero<V>();
  if (act) {
    struct Stage { Frag<TI> h, s, w[NT], v[NT]; };
    run_entries<W, D, Stage, ROLL>(
        er, lane,
        [&](Stage& f, const int (&id)[W]) {
          if constexpr (STEPS) {   // parts of tiles whose MFMA steps are all skipped come from the zero tile
            // (keep_all = 15: every part from its own tile)
            int kept[NT], ka = 0;
#pragma unroll
            for (int u = 0; u < NT; ++u) {
              kept[u] = id[1 + u] >= 0 ? ent_steps(id[1 + u]) | keep_all : 0;
              ka |= kept[u];
            }
            ld_col_kept(f.h, HCm + (size_t)id[0] * TE, zt, ka, lane);   // HC, SC tiles are stored transposed
            ld_col_kept(f.s, SCm + (size_t)id[0] * TE, zt, ka, lane);
#pragma unroll
            for (int u = 0; u < NT; ++u) {
              const size_t bt = (size_t)ent_tile(id[1 + u]) * TE;
              ld_col_kept(f.w[u], S0m + bt, zt, kept[u], lane);
              ld_col_kept(f.v[u], H0m + bt, zt, kept[u], lane);
            }
          } else {
            ld_col(f.h, HCm + (size_t)id[0] * TE, lane);   // HC, SC tiles are stored transposed
            ld_col(f.s, SCm + (size_t)id[0] * TE, lane);
#pragma unroll
            for (int u = 0; u < NT; ++u) {
              const size_t bt = (size_t)ent_tile(id[1 + u]) * TE;
              ld_col(f.w[u], S0m + bt, lane);
              ld_col(f.v[u], H0m + bt, lane);
            }
          }
        },
        [&](const Stage& f, const int (&id)[W]) {
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            if (id[1 + u] >= 0) {
              if constexpr (STEPS) {   // only the MFMA steps whose wavefunction pairs couple
                const int act = ent_steps(id[1 + u]);
                mma(acc[u], f.h, f.w[u], act);
                mma(acc[u], f.s, f.v[u], act);
              } else {
                mma(acc[u], f.h, f.w[u]);
                mma(acc[u], f.s, f.v[u]);
              }
            }
          }
        });
  }
  ks_reduce<KS, NT>(acc, red, grp, wk, lane);
  if (!act || wk != 0) return;
  const int j = lane & 15, q = lane >> 4;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    if (u >= cnt) break;
    const int t = o0 + u;
    const uint32_t mk = cmask[t];
    const double* hc = HC + (size_t)c_in_hc[t] * TE;
    double gg = 0.0, go = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = Lay<V>::row(q, r);
      const int e = tpos(row, j);
      const bool in = ((mk >> row) & 1u) && ((mk >> (16 + j)) & 1u);
      const double gv = in ? 8.0 * hc[tpos(j, row)] - 4.0 * (double)acc[u][r] : 0.0;
      G[(size_t)t * TE + e] = gv;
      gg += gv * gv;
      go += gv * Gold[(size_t)t * TE + e];
    }
    gg = wave_sum(gg);
    go = wave_sum(go);
    if (lane == 0) {
      gpart[2 * (size_t)t] = gg;
      gpart[2 * (size_t)t + 1] = go;
    }
  }
}

}  // namespace

template <typename TI>
static void grad_go(hipStream_t s, const Bufs& b, int mask, const TI* HC, const TI* SC, const TI* S0, const TI* H0) {
  if (b.grad.ngroups <= 0) return;
  nt_ks<2>(b.grad.NT, b.ks[2], [&](auto ntc, auto ksc) {
    constexpr int N_ = decltype(ntc)::value, K_ = decltype(ksc)::value;
    auto go = [&](auto rollc, auto stepsc) {
      constexpr bool R_ = decltype(rollc)::value, S_ = decltype(stepsc)::value;
      LAUNCH((k_grad<TI, K_, N_, R_, S_>), grid_for<K_>(b.grad.ngroups), block_for<K_>(), s, b.grad, b.st, mask, HC,
             SC, S0, H0, b.HC, b.c_in_hc, b.cmask, b.Gold, b.G, b.gpart, (const TI*)b.zero, b.grad_zero ? 0 : 15);
    };
    if (b.roll) {
      if (b.grad_steps) go(std::true_type{}, std::true_type{});
      else go(std::true_type{}, std::false_type{});
    } else {
      if (b.grad_steps) go(std::false_type{}, std::true_type{});
      else go(std::false_type{}, std::false_type{});
    }
  });
}

// one precision per object file (OMM_PREC 0: FP64, 1: FP32, 2: BF16)
#if OMM_PREC == 0
void launch_grad_p64(hipStream_t s, const Bufs& b, int mask) { grad_go<double>(s, b, mask, b.HC, b.SC, b.S0, b.H0); }
#elif OMM_PREC == 1
void launch_grad_p32(hipStream_t s, const Bufs& b, int mask) {
  grad_go<float>(s, b, mask, (const float*)b.HCl, (const float*)b.SCl, (const float*)b.S0l, (const float*)b.H0l);
}
#else
void launch_grad_pbf(hipStream_t s, const Bufs& b, int mask) {
  grad_go<bf16>(s, b, mask, (const bf16*)b.HCl, (const bf16*)b.SCl, (const bf16*)b.S0l, (const bf16*)b.H0l);
}
#endif

}  // namespace omm
