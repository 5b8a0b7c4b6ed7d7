// Internal declarations shared by the HIP sources of the OMM library.
//
// Storage model.  Every matrix lives on the GPU as a list of 16x16 FP64 tiles
// (plus FP32/BF16 copies for mixed precision) indexed by a tile CSR pattern;
// inside a tile the elements follow the storage order of tpos / tpos4
// (tile_ops.hpp), which matches the MFMA operand reads.  Basis rows: in block-sparse mode every atom block starts a new
// tile row (13 orbitals -> 16 rows, 3 zero rows); in dense modes rows are cut
// contiguously.  Wavefunction columns: block-sparse mode packs consecutive
// wavefunction blocks into 16-wide tiles, dense modes cut contiguously.  A
// batch of independent systems is one block-diagonal problem: each system
// owns a contiguous range of tile rows in every pattern, and all per-system
// scalars (line-search step, beta, flags) live in a SysState array.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "omm.h"

namespace omm {

// the message omm_last_error(NULL) returns (per host thread)
void set_global_error(const std::string& msg);

constexpr int T = 16;          // tile edge
constexpr int TE = T * T;      // tile elements
constexpr int MAXW = 8192;     // largest per-system tile window of the symbolic kernels

// Per-system phase flags (bit masks so a launch can select several).
enum : int { PH_INIT = 1, PH_LOW = 2, PH_FP64 = 4, PH_DONE = 8 };

// Number of partial sums produced per trace chunk (see k_traces).
constexpr int NSUM = 15;

struct SysInfo {          // read-only per-system description (device)
  int rb0, rb1;           // basis tile rows
  int wb0, wb1;           // wavefunction tiles
  int h0, h1;             // tile index range in the H/S pattern
  int c0, c1;             // ... in the C pattern
  int hc0, hc1;           // ... in the HC pattern
  int w0, w1;             // ... in the n x n pattern
  int ch0, ch1;           // trace chunk range
  int mode;               // omm_mode
  int ident_s;            // 1: S is the identity (Cholesky-reduced problem)
  int target_low;         // 1: start in the low-precision phase
  int pad;
  int64_t m, n;
  double eta;
  double eps2;            // product filter threshold squared (0 for dense systems)
};

struct SysState {         // mutable per-system CG state (device)
  double E, E_prev, x, beta, gnorm, ne;
  double gg2[2];          // <G,G> of the last two gradients, slot iter & 1 (see gg_prev / gg_store)
  double c[5];
  int64_t iter, iter_fp64, restarts, refine_left;
  int phase, status, restart, steepest, prec, conv_init, pad0, pad1;
};

struct CGParams {         // shared run parameters (kernel argument)
  double tol_grad, rel_tol, low_switch, filter_eps;
  int64_t max_iter, low_max_iter;
  int refine_iters, hist_max, hist_on, low_prec;
};

// History row layout (matches OMM_HISTORY_COLS).
constexpr int HCOLS = 11;

#define OMM_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) throw omm::DeviceError(std::string(#call) + ": " +       \
                                                 hipGetErrorString(e_));           \
  } while (0)

struct DeviceError { std::string msg; explicit DeviceError(std::string m) : msg(std::move(m)) {} };
struct ArgError { std::string msg; explicit ArgError(std::string m) : msg(std::move(m)) {} };
struct OomError { std::string msg; explicit OomError(std::string m) : msg(std::move(m)) {} };

// Tile CSR pattern on the device.  `ti` (optional) maps a position to the
// tile index of another pattern (used by transposed views).
struct PatView {
  const int* rp;
  const int* ci;
  const int* ti;
};

// Work list of a tile product: output tile t sums op(A[pairs[p].x]) * op(B[pairs[p].y])
// over p in [pp[t], pp[t+1]).
struct PlanView {
  int nout;
  const int64_t* pp;
  const int2* pairs;
};

// Grouped work list: group g covers the output tiles go0[g] .. go0[g]+gn[g]-1 of
// one output row; its entries gp[g] .. gp[g+1]-1 are rows of 1 + NT ints
// (A tile, then NT B tiles or -1), in increasing k.
struct GroupView {
  int ngroups;
  int NT;
  int64_t nent;       // entries of the list (rows of 1 + NT ints)
  int xrun;           // consecutive workgroups of a run on one XCD (block numbering)
  const int* go0;
  const int* gn;
  const int64_t* gp;
  const int* ent;
  const int4* meta;   // per group: first output tile, output tiles, system, 0
  int rows;           // 0, or P of a row-group list: the P output tiles of group g are
  const int* gto;     // gto[g * P + u] (or -1), entries are (B tile, P A tiles; absent: -2 - t)
};

}  // namespace omm
