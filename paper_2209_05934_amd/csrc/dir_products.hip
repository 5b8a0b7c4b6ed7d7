// Direction products HD = H D and SD = S D of one CG iteration on the
// functional of Eq. 4 (arXiv 2209.05934): they feed the quartic line search
// and the updates.  FP64, FP32 or BF16 MFMA tiles over the tile-pair work
// lists of the HC pattern.
#include "tile_sched.hpp"

namespace omm {

namespace {

// ------------------------------------------------------------------ S1: HD = H D, SD = S D
// One wave-group per group of NT output tiles in one row of the HC pattern:
// per k the H and S tiles are loaded once and multiply NT tiles of D.  H and S
// are symmetric: the work list names tile (k, i) for A(i, k), loaded down its
// columns.
// ONE: the single product Z = P G of kinetic preconditioning (Eq. 7; dense
// systems, whose HC and C patterns coincide): Hm = P, Bm = G, Z written in C's
// tile layout with the per-tile sums <Z, G> and <Z, G_old> in zpart.
template <typename TI, typename TO, int KS, int NT, bool ONE, bool ROLL>
__global__ __launch_bounds__(Split<KS>::NW * 64) void k_s1(
    GroupView P, const int* __restrict__ ocol, const SysInfo* __restrict__ info, const SysState* __restrict__ st, int mask, const TI* __restrict__ Hm,
    const TI* __restrict__ Sm, const TI* __restrict__ Bm, TO* __restrict__ O1, TO* __restrict__ O2,
    const int* __restrict__ hc_to_c, const uint8_t* __restrict__ wseg, const double* __restrict__ Gold,
    double* __restrict__ zpart, int* __restrict__ hcnz) {
  typedef typename Acc<TI>::V V;
  typedef Split<KS> SP;
  constexpr int W = 1 + NT;
  constexpr int NA = ONE ? NT : 2 * NT;
  __shared__ V red[SP::RED * NA * 64];
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int grp = wave / KS, wk = wave - grp * KS;
  const int g = xcd_block(P.xrun) * SP::G + grp;
  const bool valid = g < P.ngroups;
  constexpr int D = pipe_depth<TI>((ONE ? 1 : 2) + NT);
  // group record and work-list prefetch first; the system's phase, S = I flag
  // and filter threshold are read while the indices are in flight
  int4 m = make_int4(0, 0, 0, 0);
  int64_t b = 0, e = 0;
  if (valid) {
    m = group_meta(P, g);
    ks_chunk(P, g, wk, KS, b, e);
  }
  EntryRounds<W, D> er(P.ent, b, e, lane);
  const int o0 = m.x, cnt = m.y, s = m.z;
  const int phase = ld_early(&st[s].phase);
  const int ident_raw = ld_early(&info[s].ident_s);
  const double e2 = ld_early(&info[s].eps2);
  const bool act = valid && (phase & mask) != 0;
  const bool ident = act && ident_raw != 0;
  V acc[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = vzero<V>();
  if (act && ONE) {
    struct Stage { Frag<TI> h, b[NT]; };
    run_entries<W, D, Stage, ROLL>(
        er, lane,
        [&](Stage& f, const int (&id)[W]) {
          ld_col(f.h, Hm + (size_t)id[0] * TE, lane);
#pragma unroll
          for (int u = 0; u < NT; ++u) ld_col(f.b[u], Bm + (size_t)max(id[1 + u], 0) * TE, lane);
        },
        [&](const Stage& f, const int (&id)[W]) {
#pragma unroll
          for (int u = 0; u < NT; ++u)
            if (id[1 + u] >= 0) mma(acc[u], f.h, f.b[u]);
        });
  } else if (act) {
    struct Stage { Frag<TI> h, s, b[NT]; };
    // IDENT (S = I): neither S loads nor S products; S B is B's own tile
    auto body = [&](auto identc) {
      constexpr bool IDENT = decltype(identc)::value;
      run_entries<W, D, Stage, ROLL>(
          er, lane,
          [&](Stage& f, const int (&id)[W]) {
            ld_col(f.h, Hm + (size_t)id[0] * TE, lane);   // tile (k, i) of the symmetric H: A(i, k)
            if constexpr (!IDENT) ld_col(f.s, Sm + (size_t)id[0] * TE, lane);
#pragma unroll
            for (int u = 0; u < NT; ++u) ld_col(f.b[u], Bm + (size_t)max(id[1 + u], 0) * TE, lane);
          },
          [&](const Stage& f, const int (&id)[W]) {
#pragma unroll
            for (int u = 0; u < NT; ++u) {
              if (id[1 + u] >= 0) {
                mma(acc[u], f.h, f.b[u]);
                if constexpr (!IDENT) mma(acc[NT + u], f.s, f.b[u]);
              }
            }
          });
    };
    if (ident) body(std::true_type{});
    else body(std::false_type{});
  }
  ks_reduce<KS, NA>(acc, red, grp, wk, lane);
  if (!act || wk != 0) return;
  if constexpr (ONE) {
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      if (u >= cnt) break;
      const int ct = hc_to_c[o0 + u];
      if (ct < 0) continue;
      const size_t base = (size_t)ct * TE;
      double zg = 0.0, zo = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = out_off<V, double>(lane, r);
        const double z = (double)acc[u][r];
        O1[base + e] = (TO)z;
        zg += z * (double)Bm[base + e];
        zo += z * Gold[base + e];
      }
      zg = wave_sum(zg);
      zo = wave_sum(zo);
      if (lane == 0) {
        zpart[2 * (size_t)ct] = zg;
        zpart[2 * (size_t)ct + 1] = zo;
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      if (u >= cnt) break;
      const int t = o0 + u;
      V a1 = acc[u], a2 = acc[NT + u];
      if (ident) {   // S = I: S B is B's own tile
        typedef typename Acc<TI>::S AS;
        const int ct = hc_to_c[t];
#pragma unroll
        for (int r = 0; r < 4; ++r) a2[r] = ct >= 0 ? cvt<AS, TI>(Bm[(size_t)ct * TE + out_off<V, TI>(lane, r)]) : (AS)0;
      }
      if (e2 > 0.0) {
        const uint8_t* cs = wseg + 32 * (size_t)ocol[t];
        filter_tile(a1, lane, nullptr, cs, e2);
        filter_tile(a2, lane, nullptr, cs, e2);
      }
      if (hcnz) {   // which of the two filtered tiles kept a nonzero element (whole-wave ballots)
        bool n1 = false, n2 = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          n1 = n1 || a1[r] != 0;
          n2 = n2 || a2[r] != 0;
        }
        const int f = (__ballot(n1) != 0 ? 1 : 0) | (__ballot(n2) != 0 ? 2 : 0);
        if (lane == 0) hcnz[t] = f;
      }
      TO* o1 = O1 + (size_t)t * TE;
      TO* o2 = O2 + (size_t)t * TE;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = out_off<V, TO>(lane, r);
        o1[e] = (TO)a1[r];
        o2[e] = (TO)a2[r];
      }
    }
  }
}

}  // namespace

template <typename TI, typename TO, bool ONE = false>
static void s1_go(hipStream_t s, const Bufs& b, int mask, const TI* H, const TI* S, const TI* B, TO* O1, TO* O2,
                  int* hcnz = nullptr) {
  if (b.s1.ngroups <= 0) return;
  nt_ks<0>(b.s1.NT, b.ks[0], [&](auto ntc, auto ksc) {
    constexpr int N_ = decltype(ntc)::value, K_ = decltype(ksc)::value;
    if (b.roll)
      LAUNCH((k_s1<TI, TO, K_, N_, ONE, true>), grid_for<K_>(b.s1.ngroups), block_for<K_>(), s, b.s1, b.thc_col,
             b.info, b.st, mask, H, S, B, O1, O2, b.hc_to_c, b.wseg, b.Gold, b.zpart, hcnz);
    else
      LAUNCH((k_s1<TI, TO, K_, N_, ONE, false>), grid_for<K_>(b.s1.ngroups), block_for<K_>(), s, b.s1, b.thc_col,
             b.info, b.st, mask, H, S, B, O1, O2, b.hc_to_c, b.wseg, b.Gold, b.zpart, hcnz);
  });
}

// one precision per object file (OMM_PREC 0: FP64, 1: FP32, 2: BF16)
#if OMM_PREC == 0
void launch_s1_p64(hipStream_t s, const Bufs& b, int mask, bool init) {
  if (init) s1_go<double, double>(s, b, mask, b.H, b.S, b.C, b.HD, b.SD);   // H C, S C (untransposed tiles)
  else s1_go<double, double>(s, b, mask, b.H, b.S, b.D, b.HD, b.SD, b.hcnz);
}

void launch_precon(hipStream_t s, const Bufs& b, int mask) {
  s1_go<double, double, true>(s, b, mask, b.P, b.P, b.G, b.Z, b.Z);
}
#elif OMM_PREC == 1
void launch_s1_p32(hipStream_t s, const Bufs& b, int mask) {
  s1_go<float, float>(s, b, mask, (const float*)b.Hl, (const float*)b.Sl, (const float*)b.Dl, b.HDf, b.SDf, b.hcnz);
}
#else
void launch_s1_pbf(hipStream_t s, const Bufs& b, int mask) {
  s1_go<bf16, float>(s, b, mask, (const bf16*)b.Hl, (const bf16*)b.Sl, (const bf16*)b.Dl, b.HDf, b.SDf, b.hcnz);
}
#endif

}  // namespace omm
