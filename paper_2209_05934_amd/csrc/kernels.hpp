// Host-callable launchers of the device kernels.
#pragma once

#include "omm_internal.hpp"

namespace omm {

// ---------------------------------------------------------------- symbolic (symbolic.hip)
void sym_count(hipStream_t st, int nrows, int row0, PatView A, PatView B, const int2* win, int* cnt);
void sym_fill(hipStream_t st, int nrows, int row0, PatView A, PatView B, const int2* win, const int* orp,
              int* oci, int* orow);
void pair_count(hipStream_t st, int nrows, int row0, PatView A, PatView B, PatView O, const int2* win,
                int64_t* pcnt);
void pair_fill(hipStream_t st, int nrows, int row0, PatView A, PatView B, PatView O, const int2* win,
               const int64_t* pp, int2* pairs);
void find_tiles(hipStream_t st, int64_t n, const int* rows, const int* cols, PatView P, int* out);
void transpose_count(hipStream_t st, int nrows, int row0, PatView A, const int2* win, int* cnt);
void transpose_fill(hipStream_t st, int nrows, int row0, PatView A, const int2* win, const int* trp, int* tci,
                    int* tti);
void rows_of(hipStream_t st, int nrows, const int* rp, int* rows);
// grouped work lists: ng[i] = groups of output row i; then entry counts (gp == nullptr) or entries
void group_counts(hipStream_t st, int nrows, const int* orp, int NT, int* ng);
void group_lists(hipStream_t st, int nrows, PatView A, PatView B, PatView O, int NT, const int* gbase,
                 int64_t* gcnt, int64_t* gpres, const int64_t* gp, int* ent, int* go0, int* gn);
// per-group record (first output tile, output tiles, system of the output row)
void group_meta(hipStream_t st, int ngroups, const int* go0, const int* gn, const int* orow, const int* row_sys,
                int4* meta);
// the skipped MFMA steps of every entry of a gradient work list (bits 27-30 of
// its B tile indices): step s is kept where the A tile's 16-bit column mask
// (acm) and the B tile's 16-bit row mask (brm) share a bit in 4s .. 4s+3; the
// kept steps are added per system to act
void entry_steps(hipStream_t st, int ngroups, int NT, const int64_t* gp, const int4* meta, int* ent,
                 const uint32_t* acm, const uint32_t* brm, unsigned long long* act);
// row-group work lists (groups of P consecutive output rows by one column, P <= 4):
// own[t] = 1 where output tile t is the first of its column inside its row
// group (rfirst[i]: first row of row i's group); then, for the owning tiles
// numbered by gidx, entry counts (gp == nullptr: also gto, P output tiles per
// group or -1, and meta) or entries (B tile, then P A tiles; an absent one is
// -2 - t, t the entry's first present A tile)
void rg_owned(hipStream_t st, int64_t ntiles, const int* orow, PatView O, const int* rfirst, int* own);
void rg_lists(hipStream_t st, int64_t ntiles, int P, const int* orow, PatView O, PatView A, PatView B,
              const int* rfirst, const int* rend, const int* row_sys, const int* own, const int* gidx, int64_t* gcnt,
              int64_t* gpres, const int64_t* gp, int* ent, int* gto, int4* meta);
void excl_scan(hipStream_t st, const int* in, int* out, int64_t n);
void excl_scan64(hipStream_t st, const int64_t* in, int64_t* out, int64_t n);

// ---------------------------------------------------------------- numeric (numeric.hip)
enum Prec { P64 = 0, P32 = 1, PBF = 2 };

// group widths (output tiles per wave sharing one operand tile) of the
// grouped work lists built for every product step
constexpr int NPLAN = 3;
constexpr int PLAN_NT[NPLAN] = {1, 2, 4};
// the n x n projections also have a row-group plan (P = 2 output rows of one
// column per wave sharing the H D, S D tiles), plan NPLAN; its launch shape is
// reported and given as tile_group = -2
constexpr int NRG = 1;
constexpr int PLAN_ROWS[NRG] = {2};
constexpr int nplans(int step) { return step == 1 ? NPLAN + NRG : NPLAN; }
// largest split KS of a product step (0 direction, 1 n x n, 2 gradient) at
// group width NT: with KS = 8 a wave has at most 256 registers, too few for
// four output tiles, or for two of the n x n projections (four products each)
constexpr int max_split(int step, int nt) { return (nt >= 4 || (step == 1 && nt >= 2)) ? 4 : 8; }
inline bool plan_ok(int step, int nt, int ks) { return ks <= max_split(step, nt); }

struct Bufs {   // every device buffer the iteration kernels touch
  // patterns (global tile rows/cols)
  const int *th_row, *th_col, *tc_row, *tc_col, *thc_row, *thc_col, *tw_row, *tw_col;
  const int *brow_sys, *wrow_sys;
  const int *c_in_hc, *hc_to_c, *w_tr;
  const int* upd_sys;            // system of each tile of [C tiles | HC tiles | n x n tiles]
  const uint32_t* cmask;
  const uint8_t* wseg;           // per wavefunction tile: lo[16], hi[16]
  const int4* chunks;            // trace chunks (tile begin, end, system)
  int nchunks;
  int multi_chunk;               // some system spans more than FUSED_CHUNKS trace chunks
  int multi_c;                   // some system has more than FUSED_CTILES C tiles
  int n_th, n_tc, n_thc, n_tw;   // tile counts
  GroupView s1, s2, grad;         // grouped work lists of the three product steps
  // Filtering that skips work (Sec. V): the direction products record per HC
  // tile whether H D or S D kept a nonzero element (hcnz, bit 0 / bit 1), and
  // the n x n projections of an iteration run on a copy of their work list in
  // which a pair whose H D and S D tiles are both zero is marked absent
  // (s2.ent points to that copy, s2_full is the list itself, which the
  // start-up products use); hcnz == nullptr: no marking
  GroupView s2_full;
  int* hcnz;
  // FP64 masters
  double *H, *S, *C, *D, *G, *Gold, *HC, *SC, *HD, *SD, *H0, *S0, *X, *Y, *S2, *H2;
  // low-precision copies (float or bf16 storage, typed at launch) and FP32 product outputs
  void *Hl, *Sl, *Cl, *Dl, *HCl, *SCl, *H0l, *S0l;
  float *HDf, *SDf, *Xf, *Yf, *S2f, *H2f;
  double *tpart, *gpart;         // trace partials (nchunks x NSUM), gradient partials (n_tc x 2)
  // kinetic preconditioning (dense, FP64): P = (S + T/tau)^-1 on H's tiles, Z = P G on C's
  // tiles and its per-tile sums <Z,G>, <Z,G_old>; P == nullptr: no preconditioning
  const double* P;
  double *Z, *zpart;
  SysInfo* info;
  SysState* st;
  double* hist;
  int nsys;
  double eps2;                   // filter threshold squared (block-sparse products)
  int ks[3];                     // waves splitting one output tile: direction, n x n, gradient products
  int roll;                      // product kernels with the rolled work-list loop (multi-system contexts)
  int grad_steps;                // gradient entries carry skipped MFMA steps (a block-sparse system present)
  const double* zero;            // one FP64 tile of zeros: operand halves whose MFMA steps are all skipped
                                 // read it (it stays in each CU's L1)
  int grad_zero;                 // 1: the gradient reads those halves from the zero tile, 0: from their
                                 // own tiles (results are the same; the autotuner times both)
};

// the n x n work-list copy of an iteration: pairs whose H D and S D tiles are both zero marked absent
void launch_mark_pairs(hipStream_t s, const Bufs& b);

// one CG iteration step (all systems whose phase matches `mask`), arithmetic `prec`
void launch_s1(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init);
void launch_s2(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init);
// the same per precision (each precision of a product step is its own object file)
void launch_s1_p64(hipStream_t s, const Bufs& b, int mask, bool init);
void launch_s1_p32(hipStream_t s, const Bufs& b, int mask);
void launch_s1_pbf(hipStream_t s, const Bufs& b, int mask);
void launch_s2_p64(hipStream_t s, const Bufs& b, int mask, bool init);
void launch_s2_p32(hipStream_t s, const Bufs& b, int mask);
void launch_s2_pbf(hipStream_t s, const Bufs& b, int mask);
void launch_grad_p64(hipStream_t s, const Bufs& b, int mask);
void launch_grad_p32(hipStream_t s, const Bufs& b, int mask);
void launch_grad_pbf(hipStream_t s, const Bufs& b, int mask);
// Z = P G with the sums <Z,G>, <Z,G_old> per C tile (kinetic preconditioning, FP64)
void launch_precon(hipStream_t s, const Bufs& b, int mask);
// the 15 trace sums (init_inputs: of H0 and S0 alone) and from them the
// line-search step (mode LS_STEP), the initial energy (LS_INIT) or the electron count (LS_REPORT)
void launch_traces(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init_inputs, int mode,
                   const CGParams& prm);
// C, HC, SC, H_W, S_W with the step (solved in place for systems of at most FUSED_CHUNKS trace chunks)
void launch_update(hipStream_t s, const Bufs& b, Prec prec, int mask, const CGParams& prm);
void launch_grad(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init);
void launch_beta(hipStream_t s, const Bufs& b, int mask, bool init, const CGParams& prm);
// beta (systems of at most FUSED_CTILES C tiles: in place), D = -G + beta D, G_old = G
void launch_update_d(hipStream_t s, const Bufs& b, Prec prec, int mask, bool init, const CGParams& prm);
void launch_init_finish(hipStream_t s, const Bufs& b);
// start-up: HC, SC (tiles stored transposed) from the H C, S C products formed in H D, S D
void launch_hc_from_hd(hipStream_t s, const Bufs& b, int mask);
// H_W, S_W made symmetric from their upper triangle (start-up products)
void launch_mirror_w(hipStream_t s, const Bufs& b, int mask);
void launch_cast_state(hipStream_t s, const Bufs& b, Prec prec, int mask);   // C, HC, SC, H0, S0 copies
void launch_cast_hs(hipStream_t s, const Bufs& b, Prec prec);                // H, S copies

// linesearch modes
enum { LS_STEP = 0, LS_INIT = 1, LS_REPORT = 2 };
// systems with at most this many trace chunks solve the line search inside the update kernel
constexpr int FUSED_CHUNKS = 16;
// systems with at most this many C tiles take the CG beta inside the D update kernel
constexpr int FUSED_CTILES = 1024;

// density matrices: CM = C (ch H0 + cs (2I - S0)) on the CM plan, then 2 CM C^T on
// the H pattern; rho takes (ch, cs) = (0, 1), the energy density (1, eta).  Both
// read their operands down tile columns: launch_cm first transposes the ntc tiles
// of C into the scratch Ct (left there for launch_rho) and writes CM with every
// tile transposed (CMt)
void launch_cm(hipStream_t s, PlanView p, const int* orow, const int* brow_sys, int sys, const double* C,
               int64_t ntc, double* Ct, const double* S0, const double* H0, double ch, double cs, const int* tw_row,
               const int* tw_col, double* CMt);
void launch_rho(hipStream_t s, PlanView p, const int* orow, const int* brow_sys, int sys, const double* CMt,
                const double* Ct, double* rho);

// block <-> tile maps for one input matrix of one system
struct BlkMap {
  int nblk;
  const int* brow;       // block row of each stored block
  const int* bcol;       // block column
  const int64_t* voff;   // value offset
  const int* ro;         // first element row of each block row
  const int* co;         // first element column of each block column
  const int* rtile;      // element row -> global tile row
  const int* roff;       // element row -> row inside the tile
  const int* ctile;      // element column -> global tile column
  const int* coff;       // element column -> column inside the tile
  PatView P;             // tile pattern holding the values
};
void launch_scatter(hipStream_t s, const BlkMap& m, const double* val, double* tiles);
void launch_gather(hipStream_t s, const BlkMap& m, const double* tiles, double* val);
void launch_gather_w(hipStream_t s, int t0, int t1, const int* tw_row, const int* tw_col, const int* welem,
                     int64_t n, const double* tiles, double* dense);
void launch_axpy_tiles(hipStream_t s, int64_t ntiles, double alpha, const double* X, double* Y);
void launch_pad_identity(hipStream_t s, double* S, int t_first, int RT, int64_t m);
void launch_fill(hipStream_t s, double* p, int64_t n, double v);

// ---------------------------------------------------------------- Cholesky (cholesky.hip)
// dense tile grid of one system: tile (I, J) at base + I * ld + J
void chol_factor(hipStream_t s, double* A, int base, int RT, double* Linv, int* status);
void chol_reduce_h(hipStream_t s, const double* L, int lbase, int RT, const double* Linv, double* H, int hbase,
                   double* work);
void chol_apply_lt(hipStream_t s, const double* L, int lbase, int RT, const double* Cin, double* Cout, int cbase,
                   int WT);     // Cout = L^T Cin
void chol_solve_lt(hipStream_t s, const double* L, int lbase, int RT, const double* Linv, const double* Cin,
                   double* Cout, int cbase, int WT);   // Cout = L^-T Cin
void chol_inverse(hipStream_t s, const double* L, int RT, const double* Linv, const double* Id, double* work,
                  double* P);   // P = (L L^T)^-1 on a grid at offset 0
void chol_lower_inverse(hipStream_t s, const double* L, int lbase, int RT, const double* Linv, const double* Id,
                        double* X);   // X = L^-1 (lower triangular) on a grid at offset 0, Id the identity grid

}  // namespace omm
