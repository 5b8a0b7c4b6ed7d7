// Numeric kernels of one conjugate-gradient OMM iteration (arXiv 2209.05934, Sec. II/III B).
//
// With H, S (Kim-shifted, Sec. II), coefficients C, search direction D and the
// maintained products HC = H C, SC = S C, H0 = C^T H C, S0 = C^T S C, one
// iteration is
//   direction products   HD = H D, SD = S D                       (k_s1)
//   n x n projections    X = C^T SD, Y = C^T HD, S2 = D^T SD, H2 = D^T HD  (k_s2)
//   FP64 traces          15 Frobenius/trace sums -> quartic c0..c4 (k_traces)
//   exact line search    first minimum of E~(C + xD) = sum c_k x^k  (k_linesearch)
//   updates              C, HC, SC += x (D, HD, SD);  H0, S0 += x(Y+Y^T, X+X^T) + x^2 (H2, S2)
//   gradient             G = P_C[8 HC - 4 (HC S0 + SC H0)]  (kept on C's pattern)  (k_grad)
//   CG update            beta = max(0, <G, G - G_old>/<G_old, G_old>), D = -G + beta D  (k_beta, k_update_d)
// The expansion E~(C + xD) = 4 Tr H_W(x) - 2 <S_W(x), H_W(x)> with
// H_W(x) = H0 + x(Y + Y^T) + x^2 H2 and S_W(x) = S0 + x(X + X^T) + x^2 S2
// follows from Eq. 3-4.  Tile products run on MFMA (FP64, FP32, or BF16 with
// FP32 accumulation); every reduction feeding the line search is FP64 in a
// fixed order.
#include <type_traits>

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

// Work distribution of the tile-product kernels.  A workgroup holds NW = max(4, KS)
// waves; KS consecutive waves split the pair list of one output tile into KS
// contiguous chunks and add their accumulators in a fixed tree through LDS, so
// results are bitwise reproducible for a given KS.  Logical block ids are
// renumbered so that consecutive ids (neighbouring output tiles, which share
// operand tiles) run on the same XCD: the hardware deals workgroups to the 8
// XCDs round-robin.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int x = b & 7, q = nb >> 3, r = nb & 7;
  return x * q + min(x, r) + (b >> 3);
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

// chunk [b, e) of group g's entry list handled by split-wave wk
__device__ __forceinline__ void ks_chunk(const GroupView& P, int g, int wk, int KS, int64_t& b, int64_t& e) {
  const int64_t p0 = P.gp[g], n = P.gp[g + 1] - p0;
  b = p0 + (n * wk) / KS;
  e = p0 + (n * (wk + 1)) / KS;
}

// ------------------------------------------------------------------ S1: HD = H D, SD = S D
// One wave-group per group of NT output tiles in one row of the HC pattern:
// per k the H and S tiles are loaded once and multiply NT tiles of D.
template <typename TI, typename TO, int KS, int NT>
__global__ __launch_bounds__(Split<KS>::NW * 64) void k_s1(
    GroupView P, const int* __restrict__ orow, const int* __restrict__ ocol, const int* __restrict__ brow_sys,
    const SysInfo* __restrict__ info, const SysState* __restrict__ st, int mask, const TI* __restrict__ Hm,
    const TI* __restrict__ Sm, const TI* __restrict__ Bm, TO* __restrict__ O1, TO* __restrict__ O2,
    const int* __restrict__ hc_to_c, const uint8_t* __restrict__ wseg) {
  typedef typename Acc<TI>::V V;
  typedef Split<KS> SP;
  constexpr int W = 1 + NT;
  __shared__ V red[SP::RED * 2 * NT * 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = wave / KS, wk = wave - grp * KS;
  const int g = xcd_block() * SP::G + grp;
  bool act = g < P.ngroups;
  int s = 0, o0 = 0, cnt = 0;
  if (act) {
    o0 = P.go0[g];
    cnt = P.gn[g];
    s = brow_sys[orow[o0]];
    act = on(st, s, mask);
  }
  const bool ident = act && info[s].ident_s != 0;
  V acc[2 * NT];
#pragma unroll
  for (int a = 0; a < 2 * NT; ++a) acc[a] = vzero<V>();
  if (act) {
    int64_t b, e;
    ks_chunk(P, g, wk, KS, b, e);
    if (b < e) {
      Frag<TI> fh, fs, fb[NT];
      int bi[NT];
      {
        const int* en = P.ent + b * W;
        ld_row(fh, Hm + (size_t)en[0] * TE, lane);
        if (!ident) ld_row(fs, Sm + (size_t)en[0] * TE, lane);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          bi[u] = en[1 + u];
          if (bi[u] >= 0) ld_col(fb[u], Bm + (size_t)bi[u] * TE, lane);
        }
      }
      for (int64_t p = b; p < e; ++p) {
        const int* nx = P.ent + (p + 1 < e ? p + 1 : p) * W;   // prefetch the next entry
        Frag<TI> nh, ns, nb[NT];
        int ni[NT];
        ld_row(nh, Hm + (size_t)nx[0] * TE, lane);
        if (!ident) ld_row(ns, Sm + (size_t)nx[0] * TE, lane);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          ni[u] = nx[1 + u];
          if (ni[u] >= 0) ld_col(nb[u], Bm + (size_t)ni[u] * TE, lane);
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          if (bi[u] >= 0) {
            mma(acc[u], fh, fb[u]);
            if (!ident) mma(acc[NT + u], fs, fb[u]);
          }
        }
        fh = nh;
        fs = ns;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          fb[u] = nb[u];
          bi[u] = ni[u];
        }
      }
    }
  }
  ks_reduce<KS, 2 * NT>(acc, red, grp, wk, lane);
  if (!act || wk != 0) return;
  const double e2 = info[s].eps2;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    if (u >= cnt) break;
    const int t = o0 + u;
    V a1 = acc[u], a2 = acc[NT + u];
    if (ident) {   // S = I: S B is B's own tile
      typedef typename Acc<TI>::S AS;
      const int ct = hc_to_c[t];
#pragma unroll
      for (int r = 0; r < 4; ++r) a2[r] = ct >= 0 ? cvt<AS, TI>(Bm[(size_t)ct * TE + out_off<V>(lane, r)]) : (AS)0;
    }
    if (e2 > 0.0) {
      const uint8_t* cs = wseg + 32 * (size_t)ocol[t];
      filter_tile(a1, lane, nullptr, cs, e2);
      filter_tile(a2, lane, nullptr, cs, e2);
    }
    TO* o1 = O1 + (size_t)t * TE;
    TO* o2 = O2 + (size_t)t * TE;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      o1[out_off<V>(lane, r)] = (TO)a1[r];
      o2[out_off<V>(lane, r)] = (TO)a2[r];
    }
  }
}

// ------------------------------------------------------------------ S2: n x n projections
// Groups of NT output tiles in one row g of the n x n pattern: per basis tile b
// the C(b,g) and D(b,g) tiles are loaded once for NT tiles of HD and SD.
template <typename TI, typename TM, typename TO, int NPROD, int KS, int NT>
__global__ __launch_bounds__(Split<KS>::NW * 64) void k_s2(
    GroupView P, const int* __restrict__ orow, const int* __restrict__ ocol, const int* __restrict__ wrow_sys,
    const SysInfo* __restrict__ info, const SysState* __restrict__ st, int mask, const TI* __restrict__ Cm,
    const TI* __restrict__ Dm, const TM* __restrict__ HDm, const TM* __restrict__ SDm, TO* __restrict__ X,
    TO* __restrict__ Y, TO* __restrict__ S2o, TO* __restrict__ H2o, const uint8_t* __restrict__ wseg) {
  typedef typename Acc<TI>::V V;
  typedef Split<KS> SP;
  constexpr int W = 1 + NT;
  __shared__ V red[SP::RED * NPROD * NT * 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = wave / KS, wk = wave - grp * KS;
  const int g = xcd_block() * SP::G + grp;
  bool act = g < P.ngroups;
  int s = 0, o0 = 0, cnt = 0;
  if (act) {
    o0 = P.go0[g];
    cnt = P.gn[g];
    s = wrow_sys[orow[o0]];
    act = on(st, s, mask);
  }
  V acc[NPROD * NT];
#pragma unroll
  for (int a = 0; a < NPROD * NT; ++a) acc[a] = vzero<V>();
  if (act) {
    int64_t b, e;
    ks_chunk(P, g, wk, KS, b, e);
    if (b < e) {
      Frag<TI> fc, fd, fhd[NT], fsd[NT];
      int bi[NT];
      {
        const int* en = P.ent + b * W;
        ld_col(fc, Cm + (size_t)en[0] * TE, lane);                 // A = C^T
        if (NPROD == 4) ld_col(fd, Dm + (size_t)en[0] * TE, lane);  // A = D^T
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          bi[u] = en[1 + u];
          if (bi[u] >= 0) {
            ld_col(fhd[u], HDm + (size_t)bi[u] * TE, lane);
            ld_col(fsd[u], SDm + (size_t)bi[u] * TE, lane);
          }
        }
      }
      for (int64_t p = b; p < e; ++p) {
        const int* nx = P.ent + (p + 1 < e ? p + 1 : p) * W;
        Frag<TI> nc, nd, nhd[NT], nsd[NT];
        int ni[NT];
        ld_col(nc, Cm + (size_t)nx[0] * TE, lane);
        if (NPROD == 4) ld_col(nd, Dm + (size_t)nx[0] * TE, lane);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          ni[u] = nx[1 + u];
          if (ni[u] >= 0) {
            ld_col(nhd[u], HDm + (size_t)ni[u] * TE, lane);
            ld_col(nsd[u], SDm + (size_t)ni[u] * TE, lane);
          }
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          if (bi[u] >= 0) {
            mma(acc[u], fc, fsd[u]);
            mma(acc[NT + u], fc, fhd[u]);
            if (NPROD == 4) {
              mma(acc[2 * NT + u], fd, fsd[u]);
              mma(acc[3 * NT + u], fd, fhd[u]);
            }
          }
        }
        fc = nc;
        fd = nd;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          fhd[u] = nhd[u];
          fsd[u] = nsd[u];
          bi[u] = ni[u];
        }
      }
    }
  }
  ks_reduce<KS, NPROD * NT>(acc, red, grp, wk, lane);
  if (!act || wk != 0) return;
  const double e2 = info[s].eps2;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    if (u >= cnt) break;
    const int t = o0 + u;
    if (e2 > 0.0) {
      const uint8_t* rs = wseg + 32 * (size_t)orow[t];
      const uint8_t* cs = wseg + 32 * (size_t)ocol[t];
#pragma unroll
      for (int a = 0; a < NPROD; ++a) filter_tile(acc[a * NT + u], lane, rs, cs, e2);
    }
    const size_t o = (size_t)t * TE;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = out_off<V>(lane, r);
      X[o + e] = (TO)acc[u][r];
      Y[o + e] = (TO)acc[NT + u][r];
      if (NPROD == 4) {
        S2o[o + e] = (TO)acc[2 * NT + u][r];
        H2o[o + e] = (TO)acc[3 * NT + u][r];
      }
    }
  }
}

// ------------------------------------------------------------------ line search (scalar, one thread per system)
__device__ __forceinline__ double pval(const double* c, double x) {
  return c[0] + x * (c[1] + x * (c[2] + x * (c[3] + x * c[4])));
}
__device__ __forceinline__ double dp(const double* c, double x) {
  return c[1] + x * (2.0 * c[2] + x * (3.0 * c[3] + x * 4.0 * c[4]));
}
__device__ __forceinline__ double d2p(const double* c, double x) {
  return 2.0 * c[2] + x * (6.0 * c[3] + x * 12.0 * c[4]);
}

// root of p' in (lo, hi] given p'(lo) < 0 <= p'(hi): safeguarded Newton + bisection
__device__ double bracket_root(const double* c, double lo, double hi) {
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 300; ++it) {
    const double f = dp(c, x);
    if (f == 0.0) return x;
    if (f < 0.0) lo = x; else hi = x;
    const double d = d2p(c, x);
    double xn = (d > 0.0) ? x - f / d : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (fabs(xn - x) <= 1e-16 * fabs(x) || hi - lo <= 2e-16 * hi) { x = xn; break; }
    x = xn;
  }
  for (int k = 0; k < 2; ++k) {   // Newton polish
    const double d = d2p(c, x);
    if (!(d > 0.0)) break;
    const double xn = x - dp(c, x) / d;
    if (!(xn > 0.0)) break;
    x = xn;
  }
  return x;
}

// first minimum of p along x > 0 (p'(0) = c1 < 0); false when there is none
__device__ bool line_min(const double* c, double& xs) {
  if (!(c[1] < 0.0)) return false;
  // critical points of p' : roots of p'' = 12 c4 x^2 + 6 c3 x + 2 c2
  const double A = 12.0 * c[4], B = 6.0 * c[3], Cq = 2.0 * c[2];
  double r[2];
  int nr = 0;
  if (A != 0.0) {
    const double disc = B * B - 4.0 * A * Cq;
    if (disc >= 0.0) {
      const double sq = sqrt(disc);
      const double tq = -0.5 * (B + copysign(sq, B));
      if (tq != 0.0) { r[nr++] = tq / A; r[nr++] = Cq / tq; }
      else r[nr++] = 0.0;
    }
  } else if (B != 0.0) {
    r[nr++] = -Cq / B;
  }
  if (nr == 2 && r[1] < r[0]) { const double tmp = r[0]; r[0] = r[1]; r[1] = tmp; }
  double lo = 0.0;
  for (int k = 0; k < nr; ++k) {
    const double b = r[k];
    if (!(b > lo)) continue;
    if (dp(c, b) >= 0.0) {
      const double x = bracket_root(c, lo, b);
      if (d2p(c, x) > 0.0) { xs = x; return true; }
    }
    lo = b;
  }
  // last, unbounded interval: sign of p' at +infinity
  const double lead = c[4] != 0.0 ? c[4] : (c[3] != 0.0 ? c[3] : (c[2] != 0.0 ? c[2] : c[1]));
  if (!(lead > 0.0)) return false;
  double hi = lo > 0.0 ? 2.0 * lo : 1.0;
  int guard = 0;
  while (dp(c, hi) < 0.0) {
    lo = hi;
    hi *= 2.0;
    if (++guard > 2000 || !isfinite(hi)) return false;
  }
  const double x = bracket_root(c, lo, hi);
  if (!(d2p(c, x) > 0.0)) return false;
  xs = x;
  return true;
}

// quartic coefficients from the 15 sums, then the step (one thread)
__device__ void ls_finish(SysState& S, const double* a, int mode, int refine_iters) {
  double c[5];
  c[0] = 4.0 * a[0] - 2.0 * a[3];
  c[1] = 8.0 * a[1] - 4.0 * a[4] - 4.0 * a[5];
  c[2] = 4.0 * a[2] - 2.0 * (a[6] + 2.0 * a[7] + 2.0 * a[8] + a[9]);
  c[3] = -4.0 * a[10] - 4.0 * a[11];
  c[4] = -2.0 * a[12];
  const double ne = 4.0 * a[13] - 2.0 * a[14];
  if (mode == LS_REPORT) { S.ne = ne; return; }
  if (mode == LS_INIT) { S.E = c[0]; S.E_prev = c[0]; S.ne = ne; return; }
  double x = 0.0;
  const bool ok = line_min(c, x);
  if (!ok) {
    if (S.steepest) {
      if (S.phase == PH_LOW) {            // low-precision noise: finish in FP64
        S.phase = PH_INIT;
        S.prec = 0;
        S.refine_left = refine_iters > 0 ? refine_iters : -1;
      } else {
        S.status = OMM_ERR_NO_LINE_MIN;
        S.phase = PH_DONE;
      }
      S.x = 0.0;
      return;
    }
    x = 0.0;
    S.restart = 1;
    S.restarts += 1;
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) S.c[k] = c[k];
  S.x = x;
  S.E_prev = S.E;
  if (ok) S.E = pval(c, x);
  S.ne = ne;
  S.iter += 1;
  if (S.phase == PH_FP64) S.iter_fp64 += 1;
}

// ------------------------------------------------------------------ FP64 traces
// sums: 0 Tr H0, 1 Tr Y, 2 Tr H2, 3 <S0,H0>, 4 <S0,Y>, 5 <X,H0>, 6 <S0,H2>, 7 <X,Y>,
//       8 <X,Y^T>, 9 <S2,H0>, 10 <X,H2>, 11 <S2,Y>, 12 <S2,H2>, 13 Tr S0, 14 <S0,S0>
// Every workgroup reduces a chunk of n x n tiles of one system; the last
// workgroup of a system to finish (integer ticket, release/acquire fences) sums
// the system's chunk partials in chunk order and takes the line-search step.
template <typename TN>
__global__ __launch_bounds__(256) void k_traces(const int4* __restrict__ chunks, const SysInfo* __restrict__ info,
                                              SysState* __restrict__ st, int mask, const int* __restrict__ wrow,
                                              const int* __restrict__ wcol, const int* __restrict__ wtr,
                                              const double* __restrict__ H0, const double* __restrict__ S0,
                                              const TN* __restrict__ X, const TN* __restrict__ Y,
                                              const TN* __restrict__ S2, const TN* __restrict__ H2,
                                              double* __restrict__ part, int* __restrict__ ticket, int mode,
                                              int refine_iters) {
  __shared__ double red[4][NSUM];
  __shared__ int last;
  const int4 ch = chunks[blockIdx.x];
  if (!on(st, ch.z, mask)) return;
  double a[NSUM];
#pragma unroll
  for (int k = 0; k < NSUM; ++k) a[k] = 0.0;
  const int e = threadIdx.x, r = e >> 4, c = e & 15;
  for (int t = ch.x; t < ch.y; ++t) {
    const size_t o = (size_t)t * TE + e;
    const double h0 = H0[o], s0 = S0[o];
    const double x = (double)X[o], y = (double)Y[o], s2 = (double)S2[o], h2 = (double)H2[o];
    const double yt = (double)Y[(size_t)wtr[t] * TE + c * 16 + r];
    if (r == c && wrow[t] == wcol[t]) {
      a[0] += h0; a[1] += y; a[2] += h2; a[13] += s0;
    }
    a[3] += s0 * h0; a[4] += s0 * y; a[5] += x * h0; a[6] += s0 * h2; a[7] += x * y;
    a[8] += x * yt; a[9] += s2 * h0; a[10] += x * h2; a[11] += s2 * y; a[12] += s2 * h2;
    a[14] += s0 * s0;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NSUM; ++k) {
    const double v = wave_sum(a[k]);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < NSUM) {
    const int k = threadIdx.x;
    part[(size_t)blockIdx.x * NSUM + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
  __threadfence();
  __syncthreads();
  const int sy = ch.z;
  if (threadIdx.x == 0) {
    const int total = info[sy].ch1 - info[sy].ch0;
    last = (atomicAdd(&ticket[sy], 1) == total - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
#pragma unroll
  for (int k = 0; k < NSUM; ++k) a[k] = 0.0;
  for (int c2 = info[sy].ch0 + threadIdx.x; c2 < info[sy].ch1; c2 += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NSUM; ++k) a[k] += __builtin_nontemporal_load(&part[(size_t)c2 * NSUM + k]);
  }
#pragma unroll
  for (int k = 0; k < NSUM; ++k) {
    const double v = wave_sum(a[k]);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[NSUM];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) tot[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    ls_finish(st[sy], tot, mode, refine_iters);
    ticket[sy] = 0;
  }
}

// ------------------------------------------------------------------ updates (one launch)
// blocks [0, nc): C tiles; [nc, nc + nhc): HC/SC tiles; the rest: n x n tiles
template <typename TL, typename TM, bool LOW>
__global__ __launch_bounds__(256) void k_update(int nc, int nhc, const int* __restrict__ tc_row,
                                              const int* __restrict__ thc_row, const int* __restrict__ tw_row,
                                              const int* __restrict__ brow_sys, const int* __restrict__ wrow_sys,
                                              const int* __restrict__ wtr, const SysState* __restrict__ st,
                                              int mask, double* __restrict__ C, const double* __restrict__ D,
                                              TL* __restrict__ Cl, double* __restrict__ HC, double* __restrict__ SC,
                                              const TM* __restrict__ HD, const TM* __restrict__ SD,
                                              TL* __restrict__ HCl, TL* __restrict__ SCl, double* __restrict__ H0,
                                              double* __restrict__ S0, const TM* __restrict__ X,
                                              const TM* __restrict__ Y, const TM* __restrict__ S2,
                                              const TM* __restrict__ H2, TL* __restrict__ H0l,
                                              TL* __restrict__ S0l) {
  const int b = blockIdx.x;
  const int e = threadIdx.x;
  if (b < nc) {
    const int s = brow_sys[tc_row[b]];
    if (!on(st, s, mask)) return;
    const double x = st[s].x;
    if (x == 0.0) return;
    const size_t o = (size_t)b * TE + e;
    const double v = C[o] + x * D[o];
    C[o] = v;
    if (LOW) Cl[o] = cvt<TL, double>(v);
  } else if (b < nc + nhc) {
    const int t = b - nc;
    const int s = brow_sys[thc_row[t]];
    if (!on(st, s, mask)) return;
    const double x = st[s].x;
    if (x == 0.0) return;
    const size_t o = (size_t)t * TE + e;
    const double h = HC[o] + x * (double)HD[o];
    const double g = SC[o] + x * (double)SD[o];
    HC[o] = h;
    SC[o] = g;
    if (LOW) {
      HCl[o] = cvt<TL, double>(h);
      SCl[o] = cvt<TL, double>(g);
    }
  } else {
    const int t = b - nc - nhc;
    const int s = wrow_sys[tw_row[t]];
    if (!on(st, s, mask)) return;
    const double x = st[s].x;
    if (x == 0.0) return;
    const int r = e >> 4, c = e & 15;
    const size_t o = (size_t)t * TE + e;
    const size_t ot = (size_t)wtr[t] * TE + c * 16 + r;
    const double h = H0[o] + x * ((double)Y[o] + (double)Y[ot]) + x * x * (double)H2[o];
    const double g = S0[o] + x * ((double)X[o] + (double)X[ot]) + x * x * (double)S2[o];
    H0[o] = h;
    S0[o] = g;
    if (LOW) {
      H0l[o] = cvt<TL, double>(h);
      S0l[o] = cvt<TL, double>(g);
    }
  }
}

// ------------------------------------------------------------------ beta, stop rules (one thread per system)
__device__ void beta_finish(SysState& S, int s, double gg, double go, int init, double* __restrict__ hist,
                            const CGParams& prm) {
  const double gn = sqrt(gg);
  if (init) {
    S.gg = gg;
    S.gnorm = gn;
    S.beta = 0.0;
    S.steepest = 1;
    S.restart = 0;
    S.conv_init = (gn <= prm.tol_grad) ? 1 : 0;
    return;
  }
  const double beta = S.restart ? 0.0 : fmax(0.0, (gg - go) / S.gg);
  const int64_t row = S.iter - 1;
  if (prm.hist_on && row >= 0 && row < prm.hist_max) {
    double* h = hist + ((size_t)s * prm.hist_max + row) * HCOLS;
    h[0] = S.E;
    for (int k = 0; k < 5; ++k) h[1 + k] = S.c[k];
    h[6] = S.x; h[7] = gn; h[8] = beta; h[9] = (double)S.restart; h[10] = (double)S.prec;
  }
  const double rel = (S.E + S.E_prev) != 0.0 ? fabs(2.0 * (S.E - S.E_prev) / (S.E + S.E_prev)) : 0.0;
  if (gn <= prm.tol_grad) {
    S.status = OMM_OK;
    S.phase = PH_DONE;
  } else if (prm.rel_tol > 0.0 && !S.restart && rel < prm.rel_tol) {
    S.status = OMM_OK;
    S.phase = PH_DONE;
  } else if (S.phase == PH_LOW && ((!S.restart && rel < prm.low_switch) || S.iter >= prm.low_max_iter)) {
    S.phase = PH_INIT;          // recompute everything in FP64 from C, then refine
    S.prec = 0;
    S.refine_left = prm.refine_iters > 0 ? prm.refine_iters : -1;
  } else if (S.phase == PH_FP64 && S.refine_left > 0 && --S.refine_left == 0) {
    S.status = OMM_OK;
    S.phase = PH_DONE;
  } else if (S.iter >= prm.max_iter) {
    S.status = OMM_ERR_NOT_CONVERGED;
    S.phase = PH_DONE;
  }
  S.beta = beta;
  S.gg = gg;
  S.gnorm = gn;
  S.steepest = (beta == 0.0) ? 1 : 0;
  S.restart = 0;
}

// <G,G> and <G,G_old> of one system summed in tile order, then beta and the stop rules
__global__ __launch_bounds__(256) void k_beta(const SysInfo* __restrict__ info, SysState* __restrict__ st, int mask,
                                            const double* __restrict__ gpart, int init, double* __restrict__ hist,
                                            CGParams prm) {
  __shared__ double red[2][4];
  const int s = blockIdx.x;
  if (!on(st, s, mask)) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double gg = 0.0, go = 0.0;
  for (int t = info[s].c0 + threadIdx.x; t < info[s].c1; t += blockDim.x) {
    gg += gpart[2 * (size_t)t];
    go += gpart[2 * (size_t)t + 1];
  }
  gg = wave_sum(gg);
  go = wave_sum(go);
  if (lane == 0) {
    red[0][wv] = gg;
    red[1][wv] = go;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  gg = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
  go = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  beta_finish(st[s], s, gg, go, init, hist, prm);
}

// ------------------------------------------------------------------ gradient on C's pattern
// Groups of NT tiles of C's pattern in one basis row b: per k the HC(b,k) and
// SC(b,k) tiles are loaded once for NT tiles of S_W and H_W.
template <typename TI, int KS, int NT>
__global__ __launch_bounds__(Split<KS>::NW * 64) void k_grad(
    GroupView P, const int* __restrict__ tc_row, const int* __restrict__ brow_sys, const SysState* __restrict__ st,
    int mask, const TI* __restrict__ HCm, const TI* __restrict__ SCm, const TI* __restrict__ S0m,
    const TI* __restrict__ H0m, const double* __restrict__ HC, const int* __restrict__ c_in_hc,
    const uint32_t* __restrict__ cmask, const double* __restrict__ Gold, double* __restrict__ G,
    double* __restrict__ gpart) {
  typedef typename Acc<TI>::V V;
  typedef Split<KS> SP;
  constexpr int W = 1 + NT;
  __shared__ V red[SP::RED * NT * 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = wave / KS, wk = wave - grp * KS;
  const int g = xcd_block() * SP::G + grp;
  bool act = g < P.ngroups;
  int o0 = 0, cnt = 0;
  if (act) {
    o0 = P.go0[g];
    cnt = P.gn[g];
    act = on(st, brow_sys[tc_row[o0]], mask);
  }
  V acc[NT];
#pragma unroll
  for (int a = 0; a < NT; ++a) acc[a] = vzero<V>();
  if (act) {
    int64_t b, e;
    ks_chunk(P, g, wk, KS, b, e);
    if (b < e) {
      Frag<TI> fh, fs, fw[NT], fv[NT];
      int bi[NT];
      {
        const int* en = P.ent + b * W;
        ld_row(fh, HCm + (size_t)en[0] * TE, lane);
        ld_row(fs, SCm + (size_t)en[0] * TE, lane);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          bi[u] = en[1 + u];
          if (bi[u] >= 0) {
            ld_col(fw[u], S0m + (size_t)bi[u] * TE, lane);
            ld_col(fv[u], H0m + (size_t)bi[u] * TE, lane);
          }
        }
      }
      for (int64_t p = b; p < e; ++p) {
        const int* nx = P.ent + (p + 1 < e ? p + 1 : p) * W;
        Frag<TI> nh, ns, nw[NT], nv[NT];
        int ni[NT];
        ld_row(nh, HCm + (size_t)nx[0] * TE, lane);
        ld_row(ns, SCm + (size_t)nx[0] * TE, lane);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          ni[u] = nx[1 + u];
          if (ni[u] >= 0) {
            ld_col(nw[u], S0m + (size_t)ni[u] * TE, lane);
            ld_col(nv[u], H0m + (size_t)ni[u] * TE, lane);
          }
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          if (bi[u] >= 0) {
            mma(acc[u], fh, fw[u]);
            mma(acc[u], fs, fv[u]);
          }
        }
        fh = nh;
        fs = ns;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          fw[u] = nw[u];
          fv[u] = nv[u];
          bi[u] = ni[u];
        }
      }
    }
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
      const int e = row * 16 + j;
      const bool in = ((mk >> row) & 1u) && ((mk >> (16 + j)) & 1u);
      const double gv = in ? 8.0 * hc[e] - 4.0 * (double)acc[u][r] : 0.0;
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

template <typename TL, bool LOW>
__global__ __launch_bounds__(256) void k_update_d(const int* __restrict__ tc_row, const int* __restrict__ brow_sys,
                                                const SysState* __restrict__ st, int mask, double* __restrict__ D,
                                                const double* __restrict__ G, double* __restrict__ Gold,
                                                TL* __restrict__ Dl) {
  const int t = blockIdx.x;
  const int s = brow_sys[tc_row[t]];
  if (!on(st, s, mask)) return;
  if (LOW && st[s].prec == 0) return;
  const double beta = st[s].beta;
  const size_t o = (size_t)t * TE + threadIdx.x;
  const double g = G[o];
  const double d = -g + beta * D[o];
  D[o] = d;
  Gold[o] = g;
  if (LOW) Dl[o] = cvt<TL, double>(d);
}

__global__ void k_init_finish(SysState* __restrict__ st, int nsys) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  SysState& S = st[s];
  if (S.phase != PH_INIT) return;
  if (S.conv_init) {
    S.status = OMM_OK;
    S.phase = PH_DONE;
  } else {
    S.phase = S.prec ? PH_LOW : PH_FP64;
  }
}

template <typename TL>
__global__ __launch_bounds__(256) void k_cast(int ntiles, const int* __restrict__ trow,
                                            const int* __restrict__ row_sys, const SysState* __restrict__ st,
                                            int mask, const double* __restrict__ src, TL* __restrict__ dst) {
  const int t = blockIdx.x;
  if (t >= ntiles) return;
  const int s = row_sys[trow[t]];
  if (mask && (!on(st, s, mask) || st[s].prec == 0)) return;
  const size_t o = (size_t)t * TE + threadIdx.x;
  dst[o] = cvt<TL, double>(src[o]);
}

// ------------------------------------------------------------------ density matrix (Eq. 5)
__global__ __launch_bounds__(256) void k_cm(PlanView P, const int* __restrict__ orow,
                                          const int* __restrict__ brow_sys, int sys, const double* __restrict__ C,
                                          const double* __restrict__ S0, const int* __restrict__ tw_row,
                                          const int* __restrict__ tw_col, double* __restrict__ CM) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= P.nout) return;
  if (sys >= 0 && brow_sys[orow[t]] != sys) return;
  d4 acc = vzero<d4>();
  const int j = lane & 15, q = lane >> 4;
  for (int64_t p = P.pp[t]; p < P.pp[t + 1]; ++p) {
    const int2 pr = P.pairs[p];
    Frag<double> fa, fb;
    ld_row(fa, C + (size_t)pr.x * TE, lane);
    ld_col(fb, S0 + (size_t)pr.y * TE, lane);
    const bool dg = tw_row[pr.y] == tw_col[pr.y];
#pragma unroll
    for (int s = 0; s < 4; ++s) fb.v[s] = ((dg && KMap<double>::k(q, s) == j) ? 2.0 : 0.0) - fb.v[s];   // 2I - S_W
    mma(acc, fa, fb);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) CM[(size_t)t * TE + out_off<d4>(lane, r)] = acc[r];
}

__global__ __launch_bounds__(256) void k_rho(PlanView P, const int* __restrict__ orow,
                                           const int* __restrict__ brow_sys, int sys,
                                           const double* __restrict__ CM, const double* __restrict__ C,
                                           double* __restrict__ rho) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= P.nout) return;
  if (sys >= 0 && brow_sys[orow[t]] != sys) return;
  d4 acc = vzero<d4>();
  for (int64_t p = P.pp[t]; p < P.pp[t + 1]; ++p) {
    const int2 pr = P.pairs[p];
    Frag<double> fa, fb;
    ld_row(fa, CM + (size_t)pr.x * TE, lane);
    ld_row(fb, C + (size_t)pr.y * TE, lane);      // B = C^T
    mma(acc, fa, fb);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) rho[(size_t)t * TE + out_off<d4>(lane, r)] = 2.0 * acc[r];
}

// ------------------------------------------------------------------ layout conversion
__device__ __forceinline__ int find_col(const PatView& P, int r, int c) {
  int lo = P.rp[r], hi = P.rp[r + 1];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (P.ci[mid] < c) lo = mid + 1; else hi = mid;
  }
  return (lo < P.rp[r + 1] && P.ci[lo] == c) ? lo : -1;
}

template <bool SCATTER>
__global__ __launch_bounds__(256) void k_blkmap(BlkMap M, const double* __restrict__ src, double* __restrict__ dst) {
  const int k = blockIdx.x;
  if (k >= M.nblk) return;
  const int br = M.brow[k], bc = M.bcol[k];
  const int r0 = M.ro[br], nr = M.ro[br + 1] - r0;
  const int c0 = M.co[bc], nc = M.co[bc + 1] - c0;
  const int64_t vo = M.voff[k];
  for (int e = threadIdx.x; e < nr * nc; e += blockDim.x) {
    const int i = e / nc, jj = e % nc;
    const int r = r0 + i, c = c0 + jj;
    const int tix = find_col(M.P, M.rtile[r], M.ctile[c]);
    if (tix < 0) continue;
    const size_t to = (size_t)tix * TE + M.roff[r] * 16 + M.coff[c];
    if (SCATTER) dst[to] = src[vo + e];
    else dst[vo + e] = src[to];
  }
}

__global__ __launch_bounds__(256) void k_gather_w(int t0, const int* __restrict__ tw_row,
                                                const int* __restrict__ tw_col, const int* __restrict__ welem,
                                                int64_t n, const double* __restrict__ tiles,
                                                double* __restrict__ dense) {
  const int t = t0 + blockIdx.x;
  const int e = threadIdx.x, r = e >> 4, c = e & 15;
  const int gi = welem[tw_row[t] * 16 + r], gj = welem[tw_col[t] * 16 + c];
  if (gi < 0 || gj < 0) return;
  dense[(int64_t)gi * n + gj] = tiles[(size_t)t * TE + e];
}

__global__ void k_axpy(int64_t n, double alpha, const double* __restrict__ X, double* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Y[i] += alpha * X[i];
}

__global__ void k_fill(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_pad_identity(double* S, int t_first, int RT, int64_t m) {
  const int64_t r = m + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (int64_t)RT * 16) return;
  const int I = (int)(r / 16), o = (int)(r % 16);
  S[((size_t)t_first + (size_t)I * RT + I) * TE + o * 16 + o] = 1.0;
}

inline dim3 waves_grid(int n) { return dim3((unsigned)((n + 3) / 4)); }

}  // namespace

// =================================================================== launchers
#define LAUNCH(kern, grid, block, stream, ...)                                   \
  do {                                                                          \
    hipLaunchKernelGGL(kern, grid, block, 0, stream, __VA_ARGS__);              \
    OMM_HIP(hipGetLastError());                                                 \
  } while (0)

template <int KS> static dim3 grid_for(int n) { return dim3((unsigned)((n + Split<KS>::G - 1) / Split<KS>::G)); }
template <int KS> static dim3 block_for() { return dim3(Split<KS>::NW * 64); }

// (NT, KS) dispatch: NT is 1 or the step's group width; KS in {1,2,4,8} (at most 4 when NT > 1)
template <int NTG, typename F>
static void nt_ks(int nt, int ks, F&& f) {
  if (nt == 1) {
    switch (ks) {
      case 8: f(std::integral_constant<int, 1>{}, std::integral_constant<int, 8>{}); break;
      case 4: f(std::integral_constant<int, 1>{}, std::integral_constant<int, 4>{}); break;
      case 2: f(std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{}); break;
      default: f(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{}); break;
    }
  } else {
    switch (ks) {
      case 8:
      case 4: f(std::integral_constant<int, NTG>{}, std::integral_constant<int, 4>{}); break;
      case 2: f(std::integral_constant<int, NTG>{}, std::integral_constant<int, 2>{}); break;
      default: f(std::integral_constant<int, NTG>{}, std::integral_constant<int, 1>{}); break;
    }
  }
}

template <typename TI, typename TO>
static void s1_go(hipStream_t s, const Bufs& b, int mask, const TI* H, const TI* S, const TI* B, TO* O1, TO* O2) {
  nt_ks<NT_S1>(b.s1.NT, b.ks[0], [&](auto ntc, auto ksc) {
    constexpr int N_ = decltype(ntc)::value, K_ = decltype(ksc)::value;
    LAUNCH((k_s1<TI, TO, K_, N_>), grid_for<K_>(b.s1.ngroups), block_for<K_>(), s, b.s1, b.thc_row, b.thc_col,
           b.brow_sys, b.info, b.st, mask, H, S, B, O1, O2, b.hc_to_c, b.wseg);
  });
}

void launch_s1(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init, bool filter) {
  (void)filter;
  if (b.s1.ngroups <= 0) return;
  if (prec == P64) {
    if (init) s1_go<double, double>(s, b, mask, b.H, b.S, b.C, b.HC, b.SC);
    else s1_go<double, double>(s, b, mask, b.H, b.S, b.D, b.HD, b.SD);
  } else if (prec == P32) {
    s1_go<float, float>(s, b, mask, (const float*)b.Hl, (const float*)b.Sl, (const float*)b.Dl, b.HDf, b.SDf);
  } else {
    s1_go<bf16, float>(s, b, mask, (const bf16*)b.Hl, (const bf16*)b.Sl, (const bf16*)b.Dl, b.HDf, b.SDf);
  }
}

template <typename TI, typename TM, typename TO, int NP>
static void s2_go(hipStream_t s, const Bufs& b, int mask, const TI* C, const TI* D, const TM* HD, const TM* SD,
                  TO* X, TO* Y, TO* S2, TO* H2) {
  nt_ks<NT_S2>(b.s2.NT, b.ks[1], [&](auto ntc, auto ksc) {
    constexpr int N_ = decltype(ntc)::value, K_ = decltype(ksc)::value;
    LAUNCH((k_s2<TI, TM, TO, NP, K_, N_>), grid_for<K_>(b.s2.ngroups), block_for<K_>(), s, b.s2, b.tw_row,
           b.tw_col, b.wrow_sys, b.info, b.st, mask, C, D, HD, SD, X, Y, S2, H2, b.wseg);
  });
}

void launch_s2(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init, bool filter) {
  (void)filter;
  if (b.s2.ngroups <= 0) return;
  if (prec == P64) {
    if (init) s2_go<double, double, double, 2>(s, b, mask, b.C, b.C, b.HC, b.SC, b.S0, b.H0, b.S2, b.H2);
    else s2_go<double, double, double, 4>(s, b, mask, b.C, b.D, b.HD, b.SD, b.X, b.Y, b.S2, b.H2);
  } else if (prec == P32) {
    s2_go<float, float, float, 4>(s, b, mask, (const float*)b.Cl, (const float*)b.Dl, b.HDf, b.SDf, b.Xf, b.Yf,
                                  b.S2f, b.H2f);
  } else {
    s2_go<bf16, float, float, 4>(s, b, mask, (const bf16*)b.Cl, (const bf16*)b.Dl, b.HDf, b.SDf, b.Xf, b.Yf,
                                 b.S2f, b.H2f);
  }
}

static void traces_go(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init_inputs, int mode,
                      int refine_iters) {
  if (b.nchunks <= 0) return;
  if (prec == P64) {
    if (init_inputs)
      LAUNCH(k_traces<double>, dim3(b.nchunks), dim3(256), s, b.chunks, b.info, b.st, mask, b.tw_row, b.tw_col,
             b.w_tr, b.H0, b.S0, b.S0, b.H0, b.S0, b.H0, b.tpart, b.ticket, mode, refine_iters);
    else
      LAUNCH(k_traces<double>, dim3(b.nchunks), dim3(256), s, b.chunks, b.info, b.st, mask, b.tw_row, b.tw_col,
             b.w_tr, b.H0, b.S0, b.X, b.Y, b.S2, b.H2, b.tpart, b.ticket, mode, refine_iters);
  } else {
    LAUNCH(k_traces<float>, dim3(b.nchunks), dim3(256), s, b.chunks, b.info, b.st, mask, b.tw_row, b.tw_col,
           b.w_tr, b.H0, b.S0, b.Xf, b.Yf, b.S2f, b.H2f, b.tpart, b.ticket, mode, refine_iters);
  }
}

void launch_traces_ls(hipStream_t s, const Bufs& b, Prec prec, int mask, int mode, const CGParams& prm) {
  traces_go(s, b, prec, mask, mode != LS_STEP, mode, prm.refine_iters);
}

void launch_update(hipStream_t s, const Bufs& b, Prec prec, int mask) {
  const int nb = b.n_tc + b.n_thc + b.n_tw;
  if (nb <= 0) return;
  if (prec == P64)
    LAUNCH((k_update<double, double, false>), dim3(nb), dim3(256), s, b.n_tc, b.n_thc, b.tc_row, b.thc_row,
           b.tw_row, b.brow_sys, b.wrow_sys, b.w_tr, b.st, mask, b.C, b.D, (double*)nullptr, b.HC, b.SC, b.HD,
           b.SD, (double*)nullptr, (double*)nullptr, b.H0, b.S0, b.X, b.Y, b.S2, b.H2, (double*)nullptr,
           (double*)nullptr);
  else if (prec == P32)
    LAUNCH((k_update<float, float, true>), dim3(nb), dim3(256), s, b.n_tc, b.n_thc, b.tc_row, b.thc_row, b.tw_row,
           b.brow_sys, b.wrow_sys, b.w_tr, b.st, mask, b.C, b.D, (float*)b.Cl, b.HC, b.SC, b.HDf, b.SDf,
           (float*)b.HCl, (float*)b.SCl, b.H0, b.S0, b.Xf, b.Yf, b.S2f, b.H2f, (float*)b.H0l, (float*)b.S0l);
  else
    LAUNCH((k_update<bf16, float, true>), dim3(nb), dim3(256), s, b.n_tc, b.n_thc, b.tc_row, b.thc_row, b.tw_row,
           b.brow_sys, b.wrow_sys, b.w_tr, b.st, mask, b.C, b.D, (bf16*)b.Cl, b.HC, b.SC, b.HDf, b.SDf,
           (bf16*)b.HCl, (bf16*)b.SCl, b.H0, b.S0, b.Xf, b.Yf, b.S2f, b.H2f, (bf16*)b.H0l, (bf16*)b.S0l);
}

template <typename TI>
static void grad_go(hipStream_t s, const Bufs& b, int mask, const TI* HC, const TI* SC, const TI* S0, const TI* H0) {
  nt_ks<NT_GRAD>(b.grad.NT, b.ks[2], [&](auto ntc, auto ksc) {
    constexpr int N_ = decltype(ntc)::value, K_ = decltype(ksc)::value;
    LAUNCH((k_grad<TI, K_, N_>), grid_for<K_>(b.grad.ngroups), block_for<K_>(), s, b.grad, b.tc_row, b.brow_sys,
           b.st, mask, HC, SC, S0, H0, b.HC, b.c_in_hc, b.cmask, b.Gold, b.G, b.gpart);
  });
}

void launch_grad(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init) {
  (void)init;
  if (b.grad.ngroups <= 0) return;
  if (prec == P64) grad_go<double>(s, b, mask, b.HC, b.SC, b.S0, b.H0);
  else if (prec == P32)
    grad_go<float>(s, b, mask, (const float*)b.HCl, (const float*)b.SCl, (const float*)b.S0l, (const float*)b.H0l);
  else
    grad_go<bf16>(s, b, mask, (const bf16*)b.HCl, (const bf16*)b.SCl, (const bf16*)b.S0l, (const bf16*)b.H0l);
}

void launch_beta(hipStream_t s, const Bufs& b, int mask, bool init, const CGParams& prm) {
  LAUNCH(k_beta, dim3(b.nsys), dim3(256), s, b.info, b.st, mask, b.gpart, init ? 1 : 0, b.hist, prm);
}

void launch_update_d(hipStream_t s, const Bufs& b, Prec prec, int mask) {
  if (b.n_tc <= 0) return;
  if (prec == P64)
    LAUNCH((k_update_d<double, false>), dim3(b.n_tc), dim3(256), s, b.tc_row, b.brow_sys, b.st, mask, b.D, b.G,
           b.Gold, (double*)nullptr);
  else if (prec == P32)
    LAUNCH((k_update_d<float, true>), dim3(b.n_tc), dim3(256), s, b.tc_row, b.brow_sys, b.st, mask, b.D, b.G,
           b.Gold, (float*)b.Dl);
  else
    LAUNCH((k_update_d<bf16, true>), dim3(b.n_tc), dim3(256), s, b.tc_row, b.brow_sys, b.st, mask, b.D, b.G,
           b.Gold, (bf16*)b.Dl);
}

void launch_init_finish(hipStream_t s, const Bufs& b) {
  LAUNCH(k_init_finish, dim3((b.nsys + 63) / 64), dim3(64), s, b.st, b.nsys);
}

template <typename TL>
static void cast_go(hipStream_t s, int n, const int* trow, const int* rsys, const SysState* st, int mask,
                    const double* src, void* dst) {
  if (n <= 0) return;
  LAUNCH(k_cast<TL>, dim3(n), dim3(256), s, n, trow, rsys, st, mask, src, (TL*)dst);
}

void launch_cast_state(hipStream_t s, const Bufs& b, Prec prec, int mask) {
  if (prec == P64) return;
  if (prec == P32) {
    cast_go<float>(s, b.n_tc, b.tc_row, b.brow_sys, b.st, mask, b.C, b.Cl);
    cast_go<float>(s, b.n_tc, b.tc_row, b.brow_sys, b.st, mask, b.D, b.Dl);
    cast_go<float>(s, b.n_thc, b.thc_row, b.brow_sys, b.st, mask, b.HC, b.HCl);
    cast_go<float>(s, b.n_thc, b.thc_row, b.brow_sys, b.st, mask, b.SC, b.SCl);
    cast_go<float>(s, b.n_tw, b.tw_row, b.wrow_sys, b.st, mask, b.H0, b.H0l);
    cast_go<float>(s, b.n_tw, b.tw_row, b.wrow_sys, b.st, mask, b.S0, b.S0l);
  } else {
    cast_go<bf16>(s, b.n_tc, b.tc_row, b.brow_sys, b.st, mask, b.C, b.Cl);
    cast_go<bf16>(s, b.n_tc, b.tc_row, b.brow_sys, b.st, mask, b.D, b.Dl);
    cast_go<bf16>(s, b.n_thc, b.thc_row, b.brow_sys, b.st, mask, b.HC, b.HCl);
    cast_go<bf16>(s, b.n_thc, b.thc_row, b.brow_sys, b.st, mask, b.SC, b.SCl);
    cast_go<bf16>(s, b.n_tw, b.tw_row, b.wrow_sys, b.st, mask, b.H0, b.H0l);
    cast_go<bf16>(s, b.n_tw, b.tw_row, b.wrow_sys, b.st, mask, b.S0, b.S0l);
  }
}

void launch_cast_hs(hipStream_t s, const Bufs& b, Prec prec) {
  if (prec == P32) {
    cast_go<float>(s, b.n_th, b.th_row, b.brow_sys, b.st, 0, b.H, b.Hl);
    cast_go<float>(s, b.n_th, b.th_row, b.brow_sys, b.st, 0, b.S, b.Sl);
  } else if (prec == PBF) {
    cast_go<bf16>(s, b.n_th, b.th_row, b.brow_sys, b.st, 0, b.H, b.Hl);
    cast_go<bf16>(s, b.n_th, b.th_row, b.brow_sys, b.st, 0, b.S, b.Sl);
  }
}

void launch_cm(hipStream_t s, PlanView p, const int* orow, const int* brow_sys, int sys, const double* C,
               const double* S0, const int* tw_row, const int* tw_col, double* CM) {
  if (p.nout <= 0) return;
  LAUNCH(k_cm, waves_grid(p.nout), dim3(256), s, p, orow, brow_sys, sys, C, S0, tw_row, tw_col, CM);
}

void launch_rho(hipStream_t s, PlanView p, const int* orow, const int* brow_sys, int sys, const double* CM,
                const double* C, double* rho) {
  if (p.nout <= 0) return;
  LAUNCH(k_rho, waves_grid(p.nout), dim3(256), s, p, orow, brow_sys, sys, CM, C, rho);
}

void launch_scatter(hipStream_t s, const BlkMap& m, const double* val, double* tiles) {
  if (m.nblk <= 0) return;
  LAUNCH(k_blkmap<true>, dim3(m.nblk), dim3(256), s, m, val, tiles);
}

void launch_gather(hipStream_t s, const BlkMap& m, const double* tiles, double* val) {
  if (m.nblk <= 0) return;
  LAUNCH(k_blkmap<false>, dim3(m.nblk), dim3(256), s, m, tiles, val);
}

void launch_gather_w(hipStream_t s, int t0, int t1, const int* tw_row, const int* tw_col, const int* welem,
                     int64_t n, const double* tiles, double* dense) {
  if (t1 <= t0) return;
  LAUNCH(k_gather_w, dim3(t1 - t0), dim3(256), s, t0, tw_row, tw_col, welem, n, tiles, dense);
}

void launch_axpy_tiles(hipStream_t s, int64_t ntiles, double alpha, const double* X, double* Y) {
  const int64_t n = ntiles * TE;
  if (n <= 0) return;
  LAUNCH(k_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), s, n, alpha, X, Y);
}

void launch_pad_identity(hipStream_t s, double* S, int t_first, int RT, int64_t m) {
  const int64_t npad = (int64_t)RT * 16 - m;
  if (npad <= 0) return;
  LAUNCH(k_pad_identity, dim3((unsigned)((npad + 63) / 64)), dim3(64), s, S, t_first, RT, m);
}

void launch_fill(hipStream_t s, double* p, int64_t n, double v) {
  if (n <= 0) return;
  LAUNCH(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), s, p, n, v);
}

}  // namespace omm
