// Numeric kernels of one conjugate-gradient OMM iteration (arXiv 2209.05934, Sec. II/III B).
//
// With H, S (Kim-shifted, Sec. II), coefficients C, search direction D and the
// maintained products HC = H C, SC = S C, H0 = C^T H C, S0 = C^T S C, one
// iteration is
//   direction products   HD = H D, SD = S D                       (k_s1)
//   n x n projections    X = C^T SD, Y = C^T HD, S2 = D^T SD, H2 = D^T HD  (k_s2)
//   FP64 traces          15 Frobenius/trace sums -> quartic c0..c4 (k_traces)
//   exact line search    first minimum of E~(C + xD) = sum c_k x^k  (in k_update)
//   updates              C, HC, SC += x (D, HD, SD);  H0, S0 += x(Y+Y^T, X+X^T) + x^2 (H2, S2)
//   gradient             G = P_C[8 HC - 4 (HC S0 + SC H0)]  (kept on C's pattern)  (k_grad)
//   CG update            beta = max(0, <G, G - G_old>/<G_old, G_old>), D = -G + beta D  (k_update_d)
// The expansion E~(C + xD) = 4 Tr H_W(x) - 2 <S_W(x), H_W(x)> with
// H_W(x) = H0 + x(Y + Y^T) + x^2 H2 and S_W(x) = S0 + x(X + X^T) + x^2 S2
// follows from Eq. 3-4.  Tile products run on MFMA (FP64, FP32, or BF16 with
// FP32 accumulation); every reduction feeding the line search is FP64 in a
// fixed order.
#include <algorithm>
#include <cfloat>

#include "tile_sched.hpp"

namespace omm {

namespace {

// ------------------------------------------------------------------ line search (one wave per system)
// Every lane holds the same coefficients and takes the same branches.  A root
// bracket shrinks 64-fold per round: lane l evaluates p' at the l-th of 64
// points and a ballot finds the first point at or past the root, so the step
// costs about ten polynomial evaluations instead of a serial Newton chain of
// FP64 divisions.
__device__ __forceinline__ double pval(const double* c, double x) {
  return c[0] + x * (c[1] + x * (c[2] + x * (c[3] + x * c[4])));
}
__device__ __forceinline__ double dp(const double* c, double x) {
  return c[1] + x * (2.0 * c[2] + x * (3.0 * c[3] + x * 4.0 * c[4]));
}
__device__ __forceinline__ double d2p(const double* c, double x) {
  return 2.0 * c[2] + x * (6.0 * c[3] + x * 12.0 * c[4]);
}
// 1/d: hardware reciprocal refined by one Newton step
__device__ __forceinline__ double rcp64(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// first lane whose predicate holds (64 when none)
__device__ __forceinline__ int first_lane(bool p) {
  const unsigned long long m = __ballot(p);
  return m ? __builtin_ctzll(m) : 64;
}

// root of p' in (lo, hi] given p'(lo) < 0 <= p'(hi), p' increasing there
__device__ double root_wave(const double* c, double lo, double hi, int lane) {
  for (int it = 0; it < 16 && hi - lo > 4.0 * DBL_EPSILON * hi; ++it) {
    const double w = hi - lo;
    const double xl = lane == 63 ? hi : fma(w, (double)(lane + 1) * (1.0 / 64.0), lo);
    int f = first_lane(dp(c, xl) >= 0.0);
    if (f == 64) f = 63;   // p'(hi) >= 0 is kept as an invariant; guard all the same
    const double nhi = readlane_d(xl, f);
    const double nlo = f == 0 ? lo : readlane_d(xl, f - 1);
    lo = nlo;
    hi = nhi;
  }
  double x = 0.5 * (lo + hi);
  const double d = d2p(c, x);
  if (d > 0.0) {   // one Newton step inside the final bracket
    const double xn = x - dp(c, x) * rcp64(d);
    if (xn > lo && xn <= hi) x = xn;
  }
  return x;
}

// first minimum of p along x > 0 (p'(0) = c1 < 0); false when there is none
__device__ bool line_min_wave(const double* c, double& xs, int lane) {
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
      if (tq != 0.0) { r[nr++] = tq * rcp64(A); r[nr++] = Cq * rcp64(tq); }
      else r[nr++] = 0.0;
    }
  } else if (B != 0.0) {
    r[nr++] = -Cq * rcp64(B);
  }
  if (nr == 2 && r[1] < r[0]) { const double tmp = r[0]; r[0] = r[1]; r[1] = tmp; }
  double lo = 0.0;
  for (int k = 0; k < nr; ++k) {
    const double b = r[k];
    if (!(b > lo)) continue;
    if (dp(c, b) >= 0.0) {
      const double x = root_wave(c, lo, b, lane);
      if (d2p(c, x) > 0.0) { xs = x; return true; }
    }
    lo = b;
  }
  // last, unbounded interval: sign of p' at +infinity
  const double lead = c[4] != 0.0 ? c[4] : (c[3] != 0.0 ? c[3] : (c[2] != 0.0 ? c[2] : c[1]));
  if (!(lead > 0.0)) return false;
  // 64 doublings per round from lo (or from 2^-40 when lo = 0), at most 32 rounds
  double base = lo > 0.0 ? lo : 0x1p-40;
  double hi = 0.0;
  for (int round = 0; round < 32; ++round) {
    const double xl = ldexp(base, lane + 1);
    const int f = first_lane(dp(c, xl) >= 0.0);
    if (f < 64) {
      hi = readlane_d(xl, f);
      if (f > 0) lo = readlane_d(xl, f - 1);
      break;
    }
    lo = readlane_d(xl, 63);
    base = lo;
    if (!isfinite(base)) return false;
  }
  if (!(hi > 0.0)) return false;
  const double x = root_wave(c, lo, hi, lane);
  if (!(d2p(c, x) > 0.0)) return false;
  xs = x;
  return true;
}

// quartic coefficients c0..c4 of E~(C + xD) and the electron count from the 15 sums
__device__ __forceinline__ void quartic_of(const double* a, double* c, double& ne) {
  c[0] = 4.0 * a[0] - 2.0 * a[3];
  c[1] = 8.0 * a[1] - 4.0 * a[4] - 4.0 * a[5];
  c[2] = 4.0 * a[2] - 2.0 * (a[6] + 2.0 * a[7] + 2.0 * a[8] + a[9]);
  c[3] = -4.0 * a[10] - 4.0 * a[11];
  c[4] = -2.0 * a[12];
  ne = 4.0 * a[13] - 2.0 * a[14];
}

// records in the state of one system the quartic c, the electron count ne and
// the line-search outcome (ok, x) of mode LS_STEP, or the initial energy
// (LS_INIT) or electron count (LS_REPORT); one thread
__device__ void ls_apply(SysState& S, const double* c, double ne, bool ok, double x, int mode, int refine_iters) {
  if (mode == LS_REPORT) { S.ne = ne; return; }
  if (mode == LS_INIT) { S.E = c[0]; S.E_prev = c[0]; S.ne = ne; return; }
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
    S.restarts += 1;
  }
  S.restart = ok ? 0 : 1;   // set at every step: the next beta (in whichever kernel) reads it unchanged
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
// Every workgroup reduces a chunk of n x n tiles of one system, one tile per
// wave at a time (each lane holds four consecutive storage positions of a tile),
// into one partial per sum; the partials of a system are added in chunk order
// by sum_partials wherever the quartic is needed.  A tile is on the block
// diagonal exactly when its transpose is itself.
template <typename TN>
__global__ __launch_bounds__(256) void k_traces(const int4* __restrict__ chunks, const SysState* __restrict__ st,
                                              int mask, const int* __restrict__ wtr,
                                              const double* __restrict__ H0, const double* __restrict__ S0,
                                              const TN* __restrict__ X, const TN* __restrict__ Y,
                                              const TN* __restrict__ S2, const TN* __restrict__ H2,
                                              double* __restrict__ part, int single, int sym2) {
  __shared__ double red[4][NSUM];
  const int4 ch = chunks[blockIdx.x];
  if (!on(st, single ? 0 : ch.z, mask)) return;   // one system: the phase load need not wait for the chunk
  double a[NSUM];
#pragma unroll
  for (int k = 0; k < NSUM; ++k) a[k] = 0.0;
  const int lane = threadIdx.x & 63, wv = wave_id();
  // FP64 storage positions 4 lane + i: element (row, column), its position in
  // a TN tile and the position of its transpose there
  bool on_diag[4];
  int pn[4], ptn[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int p = 4 * lane + i, r = trow(p), c = tcol(p);
    on_diag[i] = r == c;
    pn[i] = tpos_of<TN>(r, c);
    ptn[i] = tpos_of<TN>(c, r);
  }
#pragma unroll 2
  for (int t = ch.x + wv; t < ch.y; t += 4) {
    const int tt = wtr[t];
    const size_t ob = (size_t)t * TE, o = ob + 4 * lane;
    const size_t tb = (size_t)tt * TE;
    const bool mir = sym2 && tt < t;   // S2, H2 below the diagonal: transpose of the mirror tile
    double h0[4], s0[4], x[4], y[4], s2[4], h2[4], yt[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      h0[i] = H0[o + i];
      s0[i] = S0[o + i];
      x[i] = (double)X[ob + pn[i]];
      y[i] = (double)Y[ob + pn[i]];
      s2[i] = (double)(mir ? S2[tb + ptn[i]] : S2[ob + pn[i]]);
      h2[i] = (double)(mir ? H2[tb + ptn[i]] : H2[ob + pn[i]]);
      yt[i] = (double)Y[tb + ptn[i]];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (tt == t && on_diag[i]) {
        a[0] += h0[i]; a[1] += y[i]; a[2] += h2[i]; a[13] += s0[i];
      }
      a[3] += s0[i] * h0[i]; a[4] += s0[i] * y[i]; a[5] += x[i] * h0[i]; a[6] += s0[i] * h2[i];
      a[7] += x[i] * y[i]; a[8] += x[i] * yt[i]; a[9] += s2[i] * h0[i]; a[10] += x[i] * h2[i];
      a[11] += s2[i] * y[i]; a[12] += s2[i] * h2[i]; a[14] += s0[i] * s0[i];
    }
  }
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
}

// The 15 sums of one system in every lane of the calling wave: lane l adds
// chunks ch0 + l, ch0 + l + 64, ... in order, then a butterfly over the wave.
// Four chunks per lane are loaded before any is added (index clamped, value
// masked), so their loads are in flight together.
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int ch0, int ch1, int lane,
                                             double (&a)[NSUM]) {
#pragma unroll
  for (int k = 0; k < NSUM; ++k) a[k] = 0.0;
  for (int c = ch0 + lane; c < ch1; c += 4 * 64) {
    double v[4][NSUM];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int cc = min(c + 64 * q, ch1 - 1);
#pragma unroll
      for (int k = 0; k < NSUM; ++k) v[q][k] = part[(size_t)cc * NSUM + k];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (c + 64 * q < ch1) {
#pragma unroll
        for (int k = 0; k < NSUM; ++k) a[k] += v[q][k];
      }
  }
#pragma unroll
  for (int k = 0; k < NSUM; ++k) a[k] = wave_sum(a[k]);
}

// line-search step (LS_STEP; systems whose step the update kernel does not
// solve itself), initial energy (LS_INIT) or electron count (LS_REPORT):
// one wave per system
__global__ __launch_bounds__(64) void k_ls_state(const SysInfo* __restrict__ info, SysState* __restrict__ st,
                                                int mask, const double* __restrict__ part, int mode,
                                                int refine_iters) {
  const int s = blockIdx.x;
  const int ch0 = info[s].ch0, ch1 = info[s].ch1;
  if ((mode == LS_STEP && ch1 - ch0 <= FUSED_CHUNKS) || !on(st, s, mask)) return;
  double a[NSUM];
  sum_partials(part, ch0, ch1, threadIdx.x, a);
  double c[5], ne, x = 0.0;
  quartic_of(a, c, ne);
  const bool ok = mode == LS_STEP && line_min_wave(c, x, threadIdx.x);
  if (threadIdx.x == 0) ls_apply(st[s], c, ne, ok, x, mode, refine_iters);
}

// ------------------------------------------------------------------ line search + updates (one launch)
// One wave per tile of the concatenated list [C tiles | HC/SC tiles | n x n
// tiles]; each lane holds four consecutive storage positions of a tile.  For a
// system of at most FUSED_CHUNKS trace chunks every wave adds the chunk
// partials and solves the line search itself (same inputs, same operations:
// the same step in every wave, and its operand loads overlap the search); the
// wave of the system's first C tile records the step in the state.  The state
// changes phase only when the step is zero, so waves that read the phase
// before or after that write do the same (nothing).  Larger systems take the
// step k_ls_state left in the state.
template <typename TL, typename TM, bool LOW>
__global__ __launch_bounds__(256) void k_update(int nc, int nhc, int ntot, const int* __restrict__ upd_sys,
                                              const int* __restrict__ wtr, const SysInfo* __restrict__ info,
                                              SysState* __restrict__ st, int mask, const double* __restrict__ part,
                                              int refine_iters, double* __restrict__ C, const double* __restrict__ D,
                                              TL* __restrict__ Cl, double* __restrict__ HC, double* __restrict__ SC,
                                              const TM* __restrict__ HD, const TM* __restrict__ SD,
                                              TL* __restrict__ HCl, TL* __restrict__ SCl, double* __restrict__ H0,
                                              double* __restrict__ S0, const TM* __restrict__ X,
                                              const TM* __restrict__ Y, const TM* __restrict__ S2,
                                              const TM* __restrict__ H2, TL* __restrict__ H0l,
                                              TL* __restrict__ S0l) {
  const int T = blockIdx.x * 4 + wave_id();
  if (T >= ntot) return;
  const int lane = threadIdx.x & 63;
  const int s = upd_sys ? upd_sys[T] : 0;   // null: a single system
  if (!on(st, s, mask)) return;
  const int ch0 = info[s].ch0, ch1 = info[s].ch1;
  const int kind = T < nc ? 0 : (T < nc + nhc ? 1 : 2);
  const int t = kind == 0 ? T : (kind == 1 ? T - nc : T - nc - nhc);
  const size_t ob = (size_t)t * TE, o = ob + 4 * lane;
  // the element (r, c) at FP64 storage position 4 lane + i: position of its
  // transpose (pt), and of it and its transpose in TM tiles (pm, pmt) and TL
  // tiles (pl, plt)
  int pt[4], pm[4], pmt[4], pl[4], plt[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = trow(4 * lane + i), c = tcol(4 * lane + i);
    pt[i] = tpos(c, r);
    pm[i] = tpos_of<TM>(r, c);
    pmt[i] = tpos_of<TM>(c, r);
    pl[i] = tpos_of<TL>(r, c);
    plt[i] = tpos_of<TL>(c, r);
  }
  // operands first: their loads overlap the line search
  double u[4], v[4], p[4], q[4], w[4], z[4];
  if (kind == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) { u[i] = C[o + i]; p[i] = D[o + i]; }
  } else if (kind == 1) {
    // HC, SC tiles are stored transposed: their position 4 lane + i holds element
    // (c, r), whose H D, S D value sits at pmt (the read and written HC, SC are
    // contiguous per lane, the read-only H D, S D are gathered)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      u[i] = HC[o + i]; v[i] = SC[o + i]; p[i] = (double)HD[ob + pmt[i]]; q[i] = (double)SD[ob + pmt[i]];
    }
  } else {
    // H_W and S_W stay symmetric, and so do their increments: the wave of a tile
    // on or above the diagonal also writes the transposed result into the mirror
    // tile (the sum Y + Y^T commutes bitwise), and waves below the diagonal stop
    const int tt = wtr[t];
    if (tt < t) return;
    const size_t tb = (size_t)tt * TE;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      u[i] = H0[o + i]; v[i] = S0[o + i];
      p[i] = (double)Y[ob + pm[i]] + (double)Y[tb + pmt[i]];
      q[i] = (double)X[ob + pm[i]] + (double)X[tb + pmt[i]];
      w[i] = (double)H2[ob + pm[i]];
      z[i] = (double)S2[ob + pm[i]];
    }
  }
  double x = 0.0;
  if (ch1 - ch0 <= FUSED_CHUNKS) {
    double a[NSUM], cq[5], ne;
    sum_partials(part, ch0, ch1, lane, a);
    quartic_of(a, cq, ne);
    const bool ok = line_min_wave(cq, x, lane);
    if (T == info[s].c0 && lane == 0) ls_apply(st[s], cq, ne, ok, x, LS_STEP, refine_iters);
    if (!ok) return;
  } else {
    x = st[s].x;
  }
  if (x == 0.0) return;
  if (kind == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double nv = u[i] + x * p[i];
      C[o + i] = nv;
      if (LOW) Cl[ob + pl[i]] = cvt<TL, double>(nv);
    }
  } else if (kind == 1) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double h = u[i] + x * p[i], g = v[i] + x * q[i];
      HC[o + i] = h;
      SC[o + i] = g;
      if (LOW) {   // element (c, r) of the transposed low-precision copy
        HCl[ob + pl[i]] = cvt<TL, double>(h);
        SCl[ob + pl[i]] = cvt<TL, double>(g);
      }
    }
  } else {
    const int tt = wtr[t];
    const size_t tb = (size_t)tt * TE;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double h = u[i] + x * p[i] + x * x * w[i];
      const double g = v[i] + x * q[i] + x * x * z[i];
      H0[o + i] = h;
      S0[o + i] = g;
      if (LOW) {
        H0l[ob + pl[i]] = cvt<TL, double>(h);
        S0l[ob + pl[i]] = cvt<TL, double>(g);
      }
      if (tt != t) {   // the same element of the mirror tile's transpose
        H0[tb + pt[i]] = h;
        S0[tb + pt[i]] = g;
        if (LOW) {
          H0l[tb + plt[i]] = cvt<TL, double>(h);
          S0l[tb + plt[i]] = cvt<TL, double>(g);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ beta, stop rules (one thread per system)
// Polak-Ribiere beta = <Z, G - G_old> / <Z_old, G_old> with Z = G, or Z = P G
// under kinetic preconditioning (Eq. 7): the sums a = <Z,G>, bo = <Z,G_old>.
// <Z_old,G_old> is read from the slot of the previous iteration and <Z,G>
// stored in the slot of this one, so that a kernel in which one wave records
// the new value while others still read the old one has no conflict.
__device__ __forceinline__ double gg_prev(const SysState& S) { return S.gg2[(S.iter + 1) & 1]; }
__device__ __forceinline__ void gg_store(SysState& S, double v) { S.gg2[S.iter & 1] = v; }
__device__ __forceinline__ double beta_of(const SysState& S, double a, double bo) {
  return S.restart ? 0.0 : fmax(0.0, (a - bo) / gg_prev(S));
}

// gg = <G,G> for the stop rule
__device__ void beta_finish(SysState& S, int s, double gg, double a, double bo, int init,
                            double* __restrict__ hist, const CGParams& prm) {
  const double gn = sqrt(gg);
  if (init) {
    gg_store(S, a);
    S.gnorm = gn;
    S.beta = 0.0;
    S.steepest = 1;
    S.restart = 0;
    S.conv_init = (gn <= prm.tol_grad) ? 1 : 0;
    return;
  }
  const double beta = beta_of(S, a, bo);
  const int64_t row = S.iter - 1;
  if (prm.hist_on && row >= 0 && row < prm.hist_max) {
    double* h = hist + ((size_t)s * prm.hist_max + row) * HCOLS;
    h[0] = S.E;
    for (int k = 0; k < 5; ++k) h[1 + k] = S.c[k];
    h[6] = S.x; h[7] = gn; h[8] = beta; h[9] = (double)S.restart; h[10] = (double)S.prec;
  }
  const double rel = (S.E + S.E_prev) != 0.0 ? fabs(2.0 * (S.E - S.E_prev) / (S.E + S.E_prev)) : 0.0;
  const bool stop = gn <= prm.tol_grad || (prm.rel_tol > 0.0 && !S.restart && rel < prm.rel_tol);
  if (S.phase == PH_LOW &&
      (stop || (!S.restart && rel < prm.low_switch) || S.iter >= prm.low_max_iter)) {
    S.phase = PH_INIT;          // recompute everything in FP64 from C, then refine: the
    S.prec = 0;                 // stop rule ends a run only in FP64
    S.refine_left = prm.refine_iters > 0 ? prm.refine_iters : -1;
  } else if (stop) {
    S.status = OMM_OK;
    S.phase = PH_DONE;
  } else if (S.phase == PH_FP64 && S.refine_left > 0 && --S.refine_left == 0) {
    // the FP64 refinement iterations are spent without the stop rule holding:
    // the run ends, but it has not converged (soft status, results readable)
    S.status = OMM_ERR_NOT_CONVERGED;
    S.phase = PH_DONE;
  } else if (S.iter >= prm.max_iter) {
    S.status = OMM_ERR_NOT_CONVERGED;
    S.phase = PH_DONE;
  }
  S.beta = beta;
  gg_store(S, a);
  S.gnorm = gn;
  S.steepest = (beta == 0.0) ? 1 : 0;
}

// the three sums over tiles u0 + STRIDE q (q = 0, 1, ...) below u1 of one lane:
// <G,G> and (a, bo) from the preconditioned sums or the plain ones; eight
// tiles' values are loaded before any is added (index clamped, value masked),
// so their loads are in flight together, and are added in tile order
template <int STRIDE>
__device__ __forceinline__ void lane_sums(const double* __restrict__ gpart, const double* __restrict__ zpart,
                                          int u0, int u1, double& gg, double& a, double& bo) {
  const double* ab = zpart ? zpart : gpart;
  for (int u = u0; u < u1; u += 8 * STRIDE) {
    double g[8], x[8], y[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const size_t uu = (size_t)min(u + STRIDE * q, u1 - 1);
      g[q] = gpart[2 * uu];
      x[q] = ab[2 * uu];
      y[q] = ab[2 * uu + 1];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (u + STRIDE * q < u1) {
        gg += g[q];
        a += x[q];
        bo += y[q];
      }
  }
}

// <G,G> and <G,G_old> of one system summed in tile order, then beta and the
// stop rules: the start-up step, and in iterations the systems of more than
// FUSED_CTILES C tiles (k_update_d takes the step of the others itself)
__global__ __launch_bounds__(256) void k_beta(const SysInfo* __restrict__ info, SysState* __restrict__ st, int mask,
                                            const double* __restrict__ gpart, const double* __restrict__ zpart,
                                            int init, double* __restrict__ hist, CGParams prm) {
  __shared__ double red[3][4];
  const int s = blockIdx.x;
  if ((!init && info[s].c1 - info[s].c0 <= FUSED_CTILES) || !on(st, s, mask)) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double gg = 0.0, a = 0.0, bo = 0.0;
  lane_sums<256>(gpart, zpart, info[s].c0 + threadIdx.x, info[s].c1, gg, a, bo);
  gg = wave_sum(gg);
  a = wave_sum(a);
  bo = wave_sum(bo);
  if (lane == 0) {
    red[0][wv] = gg;
    red[1][wv] = a;
    red[2][wv] = bo;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  gg = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
  a = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  bo = ((red[2][0] + red[2][1]) + red[2][2]) + red[2][3];
  beta_finish(st[s], s, gg, a, bo, init, hist, prm);
}

// D = -Z + beta D (Z = G, or P G under kinetic preconditioning) and G_old = G:
// one wave per C tile, four consecutive storage positions per lane.
// For a system of at most FUSED_CTILES C tiles every wave adds the per-tile
// sums in tile order and forms beta itself (the same value in every wave); the
// wave of the system's first C tile also applies the stop rules and records
// the state.  Fields it writes that others read are either double-buffered
// (<Z,G>) or only change when the system leaves this step's phase (then its D
// is no longer used).
template <typename TL, bool LOW>
__global__ __launch_bounds__(256) void k_update_d(int nc, const int* __restrict__ upd_sys,
                                                const SysInfo* __restrict__ info, SysState* __restrict__ st, int mask,
                                                double* __restrict__ D, const double* __restrict__ G,
                                                const double* __restrict__ Z, double* __restrict__ Gold,
                                                TL* __restrict__ Dl, const double* __restrict__ gpart,
                                                const double* __restrict__ zpart, double* __restrict__ hist,
                                                CGParams prm, int init) {
  const int t = blockIdx.x * 4 + wave_id();
  if (t >= nc) return;
  const int lane = threadIdx.x & 63;
  const int s = upd_sys ? upd_sys[t] : 0;   // null: a single system
  if (!on(st, s, mask)) return;
  if (LOW && st[s].prec == 0) return;
  const int ci0 = info[s].c0, ci1 = info[s].c1;
  const size_t o = (size_t)t * TE + 4 * lane;
  const double* Zs = zpart ? Z : G;
  double g[4], z[4], dv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) { g[i] = G[o + i]; z[i] = Zs[o + i]; dv[i] = D[o + i]; }
  double beta;
  if (init) {   // start-up: D = -Z (k_beta has recorded the state)
    beta = 0.0;
  } else if (ci1 - ci0 <= FUSED_CTILES) {
    double gg = 0.0, a = 0.0, bo = 0.0;
    lane_sums<64>(gpart, zpart, ci0 + lane, ci1, gg, a, bo);
    gg = wave_sum(gg);
    a = wave_sum(a);
    bo = wave_sum(bo);
    beta = beta_of(st[s], a, bo);
    if (t == ci0 && lane == 0) beta_finish(st[s], s, gg, a, bo, 0, hist, prm);
  } else {
    beta = st[s].beta;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double d = -z[i] + beta * dv[i];
    D[o + i] = d;
    Gold[o + i] = g[i];
    if (LOW) Dl[(size_t)t * TE + tpos_of<TL>(trow(4 * lane + i), tcol(4 * lane + i))] = cvt<TL, double>(d);
  }
}

// H_W and S_W as formed at start-up are made exactly symmetric from their upper
// triangle (the symmetric products keep the blocks on and above the block
// diagonal): a tile below the diagonal becomes the transpose of its mirror, and
// inside a diagonal tile each element below the diagonal takes its mirror
// element.  Only elements below the diagonal are written, only elements on or
// above it are read.  One wave per n x n tile, four elements per lane.
__global__ __launch_bounds__(256) void k_mirror_w(int ntw, int woff, const int* __restrict__ upd_sys,
                                                const int* __restrict__ tw_row, const int* __restrict__ tw_col,
                                                const int* __restrict__ wtr, const SysState* __restrict__ st,
                                                int mask, double* __restrict__ H0, double* __restrict__ S0) {
  const int t = blockIdx.x * 4 + wave_id();
  if (t >= ntw) return;
  const int s = upd_sys ? upd_sys[woff + t] : 0;
  if (!on(st, s, mask)) return;
  const int rt = tw_row[t], ct = tw_col[t];
  if (rt < ct) return;
  const int lane = threadIdx.x & 63;
  const size_t src = (size_t)(rt == ct ? t : wtr[t]) * TE;
  const size_t dst = (size_t)t * TE;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int p = 4 * lane + i, r = trow(p), c = tcol(p);
    if (rt == ct && r <= c) continue;
    H0[dst + p] = H0[src + tpos(c, r)];
    S0[dst + p] = S0[src + tpos(c, r)];
  }
}

// Start-up: H C and S C were formed into the H D and S D tiles (the
// orientation the n x n projections read down columns); the maintained HC and SC are
// stored with each tile transposed, the layout the gradient products read down
// columns.  One wave per HC tile of a system in the masked phase.
__global__ __launch_bounds__(256) void k_hc_from_hd(int nhc, int hoff, const int* __restrict__ upd_sys,
                                                  const SysState* __restrict__ st, int mask,
                                                  const double* __restrict__ HD, const double* __restrict__ SD,
                                                  double* __restrict__ HC, double* __restrict__ SC) {
  const int t = blockIdx.x * 4 + wave_id();
  if (t >= nhc) return;
  const int s = upd_sys ? upd_sys[hoff + t] : 0;
  if (!on(st, s, mask)) return;
  const int lane = threadIdx.x & 63;
  const size_t base = (size_t)t * TE;
#pragma unroll
  for (int i = 0; i < 4; ++i) {   // storage position e = 64 i + lane
    const int e = 64 * i + lane, tp = tpos(tcol(e), trow(e));
    HC[base + tp] = HD[base + e];
    SC[base + tp] = SD[base + e];
  }
}

// The work-list copy the n x n projections of an iteration run on (filtering
// that skips work, Sec. V): in every entry (a C tile, then W - 1 HC tiles or
// -1) an HC tile whose H D and S D tiles were both filtered to zero by the
// direction products of this iteration becomes -1, so the projections neither
// load it nor multiply by it.  Skipping an all-zero tile leaves every sum as it
// is.  One thread per entry.
// A row-group list holds the HC tile first and the C tiles after it (an absent
// one written -2 - t, t a present C tile of the entry): an entry whose HC tile
// was filtered to zero gets every C tile t written as -2 - t, so the
// projections skip its products and still load only tiles of the entry.
template <int W, bool ROWS = false>
__global__ __launch_bounds__(256) void k_mark_pairs(int64_t nent, const int* __restrict__ ent,
                                                  const int* __restrict__ hcnz, int* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nent; e += (int64_t)gridDim.x * 256) {
    const int* in = ent + e * W;
    int* o = out + e * W;
    o[0] = in[0];
    const bool zero = ROWS && hcnz[in[0]] == 0;
#pragma unroll
    for (int w = 1; w < W; ++w) {
      const int v = in[w];
      o[w] = ROWS ? ((zero && v >= 0) ? -2 - v : v) : ((v >= 0 && hcnz[v] == 0) ? -1 : v);
    }
  }
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
__global__ __launch_bounds__(256) void k_cast(int ntiles, const int* __restrict__ tile_row,
                                            const int* __restrict__ row_sys, const SysState* __restrict__ st,
                                            int mask, const double* __restrict__ src, TL* __restrict__ dst) {
  const int t = blockIdx.x;
  if (t >= ntiles) return;
  const int s = row_sys[tile_row[t]];
  if (mask && (!on(st, s, mask) || st[s].prec == 0)) return;
  const int p = threadIdx.x;   // FP64 storage position, moved to its place in a TL tile
  dst[(size_t)t * TE + tpos_of<TL>(trow(p), tcol(p))] = cvt<TL, double>(src[(size_t)t * TE + p]);
}

// ------------------------------------------------------------------ density matrices (Eq. 5, Eq. 6)
// CM = C M with the n x n matrix M = ch H_W + cs (2I - S_W): rho takes (0, 1), the
// energy density rho_E = 2 C H_W C^T + eta rho (Kim correction, Sec. II) takes (1, eta)
__global__ __launch_bounds__(256) void k_cm(PlanView P, const int* __restrict__ orow,
                                          const int* __restrict__ brow_sys, int sys, const double* __restrict__ Ct,
                                          const double* __restrict__ S0, const double* __restrict__ H0, double ch,
                                          double cs, const int* __restrict__ tw_row,
                                          const int* __restrict__ tw_col, double* __restrict__ CMt) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= P.nout) return;
  if (sys >= 0 && brow_sys[orow[t]] != sys) return;
  d4 acc = vzero<d4>();
  const int j = lane & 15, q = lane >> 4;
  for (int64_t p = P.pp[t]; p < P.pp[t + 1]; ++p) {
    const int2 pr = P.pairs[p];
    Frag<double> fa, fb;
    ld_col(fa, Ct + (size_t)pr.x * TE, lane);      // A = C, from its transposed tile
    ld_col(fb, S0 + (size_t)pr.y * TE, lane);
    const bool dg = tw_row[pr.y] == tw_col[pr.y];
#pragma unroll
    for (int s = 0; s < 4; ++s)   // cs (2I - S_W)
      fb.v[s] = cs * (((dg && KMap<double>::k(q, s) == j) ? 2.0 : 0.0) - fb.v[s]);
    if (ch != 0.0) {
      Frag<double> fh;
      ld_col(fh, H0 + (size_t)pr.y * TE, lane);
#pragma unroll
      for (int s = 0; s < 4; ++s) fb.v[s] += ch * fh.v[s];
    }
    mma(acc, fa, fb);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) CMt[(size_t)t * TE + out_off_t<d4, double>(lane, r)] = acc[r];   // stored transposed
}

__global__ __launch_bounds__(256) void k_rho(PlanView P, const int* __restrict__ orow,
                                           const int* __restrict__ brow_sys, int sys,
                                           const double* __restrict__ CMt, const double* __restrict__ Ct,
                                           double* __restrict__ rho) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= P.nout) return;
  if (sys >= 0 && brow_sys[orow[t]] != sys) return;
  d4 acc = vzero<d4>();
  for (int64_t p = P.pp[t]; p < P.pp[t + 1]; ++p) {
    const int2 pr = P.pairs[p];
    Frag<double> fa, fb;
    ld_col(fa, CMt + (size_t)pr.x * TE, lane);    // A = C M, from its transposed tile
    ld_col(fb, Ct + (size_t)pr.y * TE, lane);     // B = C^T
    mma(acc, fa, fb);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) rho[(size_t)t * TE + out_off<d4, double>(lane, r)] = 2.0 * acc[r];
}

// every tile of src transposed into dst (one wave per tile)
__global__ __launch_bounds__(256) void k_transpose_tiles(int64_t n, const double* __restrict__ src,
                                                       double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= n) return;
  const int lane = threadIdx.x & 63;
  const size_t base = (size_t)t * TE;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = 64 * i + lane;
    dst[base + tpos(tcol(e), trow(e))] = src[base + e];
  }
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
    const size_t to = (size_t)tix * TE + tpos(M.roff[r], M.coff[c]);
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
  dense[(int64_t)gi * n + gj] = tiles[(size_t)t * TE + tpos(r, c)];
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
  S[((size_t)t_first + (size_t)I * RT + I) * TE + tpos(o, o)] = 1.0;
}

inline dim3 waves_grid(int n) { return dim3((unsigned)((n + 3) / 4)); }

}  // namespace

// =================================================================== launchers
void launch_traces(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init_inputs, int mode,
                   const CGParams& prm) {
  if (b.nchunks <= 0) return;
  if (prec == P64) {
    if (init_inputs)   // X = S0, Y = H0, S2 = S0, H2 = H0: the sums then hold Tr H0, <S0,H0>, Tr S0, <S0,S0>
      LAUNCH(k_traces<double>, dim3(b.nchunks), dim3(256), s, b.chunks, b.st, mask, b.w_tr, b.H0, b.S0, b.S0,
             b.H0, b.S0, b.H0, b.tpart, b.nsys == 1 ? 1 : 0, 0);
    else
      LAUNCH(k_traces<double>, dim3(b.nchunks), dim3(256), s, b.chunks, b.st, mask, b.w_tr, b.H0, b.S0, b.X, b.Y,
             b.S2, b.H2, b.tpart, b.nsys == 1 ? 1 : 0, 1);
  } else {
    LAUNCH(k_traces<float>, dim3(b.nchunks), dim3(256), s, b.chunks, b.st, mask, b.w_tr, b.H0, b.S0, b.Xf, b.Yf,
           b.S2f, b.H2f, b.tpart, b.nsys == 1 ? 1 : 0, 1);
  }
  if (mode != LS_STEP || b.multi_chunk)
    LAUNCH(k_ls_state, dim3(b.nsys), dim3(64), s, b.info, b.st, mask, b.tpart, mode, prm.refine_iters);
}

void launch_update(hipStream_t s, const Bufs& b, Prec prec, int mask, const CGParams& prm) {
  const int nt = b.n_tc + b.n_thc + b.n_tw;
  if (nt <= 0) return;
  const dim3 grid((unsigned)((nt + 3) / 4));
  if (prec == P64)
    LAUNCH((k_update<double, double, false>), grid, dim3(256), s, b.n_tc, b.n_thc, nt, b.nsys == 1 ? nullptr : b.upd_sys, b.w_tr, b.info,
           b.st, mask, b.tpart, prm.refine_iters, b.C, b.D, (double*)nullptr, b.HC, b.SC, b.HD, b.SD,
           (double*)nullptr, (double*)nullptr, b.H0, b.S0, b.X, b.Y, b.S2, b.H2, (double*)nullptr,
           (double*)nullptr);
  else if (prec == P32)
    LAUNCH((k_update<float, float, true>), grid, dim3(256), s, b.n_tc, b.n_thc, nt, b.nsys == 1 ? nullptr : b.upd_sys, b.w_tr, b.info,
           b.st, mask, b.tpart, prm.refine_iters, b.C, b.D, (float*)b.Cl, b.HC, b.SC, b.HDf, b.SDf,
           (float*)b.HCl, (float*)b.SCl, b.H0, b.S0, b.Xf, b.Yf, b.S2f, b.H2f, (float*)b.H0l, (float*)b.S0l);
  else
    LAUNCH((k_update<bf16, float, true>), grid, dim3(256), s, b.n_tc, b.n_thc, nt, b.nsys == 1 ? nullptr : b.upd_sys, b.w_tr, b.info,
           b.st, mask, b.tpart, prm.refine_iters, b.C, b.D, (bf16*)b.Cl, b.HC, b.SC, b.HDf, b.SDf,
           (bf16*)b.HCl, (bf16*)b.SCl, b.H0, b.S0, b.Xf, b.Yf, b.S2f, b.H2f, (bf16*)b.H0l, (bf16*)b.S0l);
}

void launch_s1(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init) {
  if (prec == P64) launch_s1_p64(s, b, mask, init);
  else if (prec == P32) launch_s1_p32(s, b, mask);
  else launch_s1_pbf(s, b, mask);
}

void launch_s2(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init) {
  if (prec == P64) launch_s2_p64(s, b, mask, init);
  else if (prec == P32) launch_s2_p32(s, b, mask);
  else launch_s2_pbf(s, b, mask);
}

void launch_grad(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init) {
  (void)init;
  if (prec == P64) launch_grad_p64(s, b, mask);
  else if (prec == P32) launch_grad_p32(s, b, mask);
  else launch_grad_pbf(s, b, mask);
}

void launch_beta(hipStream_t s, const Bufs& b, int mask, bool init, const CGParams& prm) {
  if (!init && !b.multi_c) return;   // every system takes its beta in k_update_d
  LAUNCH(k_beta, dim3(b.nsys), dim3(256), s, b.info, b.st, mask, b.gpart, b.P ? b.zpart : nullptr, init ? 1 : 0,
         b.hist, prm);
}

// kinetic preconditioning runs in FP64 only (the library rejects it with low precision)
void launch_update_d(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init, const CGParams& prm) {
  if (b.n_tc <= 0) return;
  const dim3 grid((unsigned)((b.n_tc + 3) / 4));
  const int in = init ? 1 : 0;
  const int* us = b.nsys == 1 ? nullptr : b.upd_sys;
  const double* zp = b.P ? b.zpart : nullptr;
  if (prec == P64)
    LAUNCH((k_update_d<double, false>), grid, dim3(256), s, b.n_tc, us, b.info, b.st, mask, b.D, b.G, b.Z, b.Gold,
           (double*)nullptr, b.gpart, zp, b.hist, prm, in);
  else if (prec == P32)
    LAUNCH((k_update_d<float, true>), grid, dim3(256), s, b.n_tc, us, b.info, b.st, mask, b.D, b.G,
           (const double*)nullptr, b.Gold, (float*)b.Dl, b.gpart, (const double*)nullptr, b.hist, prm, in);
  else
    LAUNCH((k_update_d<bf16, true>), grid, dim3(256), s, b.n_tc, us, b.info, b.st, mask, b.D, b.G,
           (const double*)nullptr, b.Gold, (bf16*)b.Dl, b.gpart, (const double*)nullptr, b.hist, prm, in);
}

void launch_mirror_w(hipStream_t s, const Bufs& b, int mask) {
  if (b.n_tw <= 0) return;
  LAUNCH(k_mirror_w, waves_grid(b.n_tw), dim3(256), s, b.n_tw, b.n_tc + b.n_thc, b.nsys > 1 ? b.upd_sys : nullptr,
         b.tw_row, b.tw_col, b.w_tr, b.st, mask, b.H0, b.S0);
}

void launch_hc_from_hd(hipStream_t s, const Bufs& b, int mask) {
  if (b.n_thc <= 0) return;
  LAUNCH(k_hc_from_hd, waves_grid(b.n_thc), dim3(256), s, b.n_thc, b.n_tc, b.nsys > 1 ? b.upd_sys : nullptr, b.st,
         mask, b.HD, b.SD, b.HC, b.SC);
}

void launch_mark_pairs(hipStream_t s, const Bufs& b) {
  if (!b.hcnz || b.s2.nent <= 0 || b.s2.ent == b.s2_full.ent) return;
  const unsigned grid = (unsigned)std::min<int64_t>((b.s2.nent + 255) / 256, 8192);
  if (b.s2.rows)   // row-group list (2 rows)
    LAUNCH((k_mark_pairs<3, true>), dim3(grid), dim3(256), s, b.s2.nent, b.s2_full.ent, b.hcnz, (int*)b.s2.ent);
  else if (b.s2.NT == 1)
    LAUNCH(k_mark_pairs<2>, dim3(grid), dim3(256), s, b.s2.nent, b.s2_full.ent, b.hcnz, (int*)b.s2.ent);
  else if (b.s2.NT == 2)
    LAUNCH(k_mark_pairs<3>, dim3(grid), dim3(256), s, b.s2.nent, b.s2_full.ent, b.hcnz, (int*)b.s2.ent);
  else
    LAUNCH(k_mark_pairs<5>, dim3(grid), dim3(256), s, b.s2.nent, b.s2_full.ent, b.hcnz, (int*)b.s2.ent);
}

void launch_init_finish(hipStream_t s, const Bufs& b) {
  LAUNCH(k_init_finish, dim3((b.nsys + 63) / 64), dim3(64), s, b.st, b.nsys);
}

template <typename TL>
static void cast_go(hipStream_t s, int n, const int* tile_row, const int* rsys, const SysState* st, int mask,
                    const double* src, void* dst) {
  if (n <= 0) return;
  LAUNCH(k_cast<TL>, dim3(n), dim3(256), s, n, tile_row, rsys, st, mask, src, (TL*)dst);
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
               int64_t ntc, double* Ct, const double* S0, const double* H0, double ch, double cs, const int* tw_row,
               const int* tw_col, double* CMt) {
  if (ntc > 0) LAUNCH(k_transpose_tiles, dim3((unsigned)((ntc + 3) / 4)), dim3(256), s, ntc, C, Ct);
  if (p.nout <= 0) return;
  LAUNCH(k_cm, waves_grid(p.nout), dim3(256), s, p, orow, brow_sys, sys, Ct, S0, H0, ch, cs, tw_row, tw_col, CMt);
}

void launch_rho(hipStream_t s, PlanView p, const int* orow, const int* brow_sys, int sys, const double* CMt,
                const double* Ct, double* rho) {
  if (p.nout <= 0) return;
  LAUNCH(k_rho, waves_grid(p.nout), dim3(256), s, p, orow, brow_sys, sys, CMt, Ct, rho);
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
