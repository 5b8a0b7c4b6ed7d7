/*
 * omm.h - C ABI of an MI355X (gfx950) library for the conjugate-gradient
 * orbital minimization method (OMM) of arXiv 2209.05934 (Lebedeva, Garcia,
 * Artacho, Ordejon), cubic-scaling (dense, optionally Cholesky-reduced) and
 * linear-scaling (atom-block sparse, localized wavefunctions, filtering).
 *
 * The library minimizes the Ordejon-Mauri functional (Eq. 4)
 *     E~ = 2 Tr[(2I - S_W) H_W],   H_W = C^T H C,  S_W = C^T S C   (Eq. 3)
 * over the m x n coefficient matrix C by conjugate gradients with an exact
 * quartic line search (Sec. I, Sec. III B), for the Kim-shifted Hamiltonian
 * H - eta S (Sec. II), and returns C, the energy and the density matrix
 * rho = 2 C (2I - S_W) C^T on S's pattern (Eq. 5, Sec. III B).  The paper's
 * solver contract (Sec. III B: H, S and an initial guess in a chosen format
 * in, converged coefficients and rho out) is kept; its MatrixSwitch formats
 * become one atom-block BCSR description, and its DBCSR/ScaLAPACK back ends
 * become HIP kernels on one GPU.
 *
 * Conventions for every entry point:
 *   - Matrices are real (Gamma point, Sec. IV A) and given as omm_matrix:
 *     index arrays always live in host memory; `val` lives in host or device
 *     memory as `memspace` says.  Inputs are borrowed for the call only and
 *     deep-copied into memory the context owns.
 *   - Every call is stream-ordered on omm_options.hip_stream and returns when
 *     its work has completed.  Calls on one context must not overlap; there is
 *     no global state, so different contexts are independent.
 *   - Return value: an omm_status.  On an error the context stays valid (soft
 *     errors OMM_ERR_NOT_CONVERGED / OMM_ERR_ELECTRON_COUNT leave readable
 *     results) and omm_last_error() returns a message.
 */
#ifndef OMM_MI355X_H
#define OMM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OMM_OK = 0,
  OMM_ERR_ARG = 1,            /* shape, pattern or option mismatch */
  OMM_ERR_STATE = 2,          /* call order (e.g. minimize before set_coeffs) */
  OMM_ERR_NOT_SPD = 3,        /* Cholesky factorization of S failed (Sec. II) */
  OMM_ERR_NO_LINE_MIN = 4,    /* quartic has no minimum along steepest descent (Sec. IV C) */
  OMM_ERR_NOT_CONVERGED = 5,  /* soft: max_iter reached, results readable */
  OMM_ERR_ELECTRON_COUNT = 6, /* soft: |2Tr[(2I-S_W)S_W] - 2n| above ne_tol (Sec. II, Kim;
                                 n = n_occupied, see omm_set_occupied) */
  OMM_ERR_DEVICE = 7,         /* HIP runtime error */
  OMM_ERR_OOM = 8             /* device allocation failed */
} omm_status;

/* Solver form (Table 1: OMM.UseSparse, OMM.Cholesky). */
typedef enum {
  OMM_DENSE = 0,           /* cubic scaling, dense C */
  OMM_DENSE_CHOLESKY = 1,  /* cubic scaling on S = U^T U, H~ = U^-T H U^-1 (Sec. II) */
  OMM_BLOCK_SPARSE = 2     /* linear scaling: C restricted to the pattern of C0 (Sec. II, III B) */
} omm_mode;

/* Arithmetic of the block products inside the CG iterations.  Energies,
 * traces, quartic coefficients, line search, C/D/G and the final refinement
 * iterations are always FP64. */
typedef enum { OMM_FP64 = 0, OMM_FP32 = 1, OMM_BF16 = 2 } omm_precision;

typedef enum { OMM_HOST = 0, OMM_DEVICE = 1 } omm_memspace;

/* Atom-block compressed sparse row matrix (the paper's block matrices,
 * Sec. III B: equal or per-atom rectangular blocks, zero blocks not stored).
 *   row_bsz[nbrow], col_bsz[nbcol]   block sizes (host)
 *   row_ptr[nbrow+1]                 stored blocks of block row i are
 *                                    row_ptr[i] .. row_ptr[i+1]-1 (host)
 *   col_idx[nnzb]                    block column of each stored block,
 *                                    strictly increasing within a row (host)
 *   val_off[nnzb]                    offset in `val` of the block's values,
 *                                    stored row-major (host)
 *   val[nval]                        float64 values (host or device)
 * A dense matrix is one with every block stored. */
typedef struct {
  int32_t nbrow, nbcol;
  const int32_t* row_bsz;
  const int32_t* col_bsz;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const int64_t* val_off;
  const double* val;
  int64_t nval;
  int32_t memspace; /* omm_memspace of val */
} omm_matrix;

/* Options (Table 1 keys and build-only knobs).  Fill with omm_default_options. */
typedef struct {
  double eta;               /* Kim shift H -> H - eta S (OMM.Eta, Sec. II); default 0 */
  double tol_grad;          /* stop when ||G||_F <= tol_grad (projected real gradient); 1e-9 */
  double rel_tol;           /* stop when |2(E_n-E_{n-1})/(E_n+E_{n-1})| < rel_tol
                               (OMM.RelTol, Table 1, whose default is 1e-9); <= 0
                               disables; default 0 here: the default stop rule is the
                               gradient norm, which bounds the distance to the minimum
                               where a small energy change does not (set 1e-9 for the
                               paper's rule) */
  int64_t max_iter;         /* CG iteration cap; default 10000 */
  double filter_eps;        /* block-sparse mode: product blocks with Frobenius norm
                               < eps are dropped (Sec. V); default 0 */
  int32_t precision;        /* omm_precision of the CG block products; default FP64 */
  int32_t fp64_refine_iters;/* mixed precision: FP64 iterations after the low-precision
                               phase; <= 0 means FP64 until the stop rule; default 5.
                               A run that spends them without meeting the stop rule
                               ends with OMM_ERR_NOT_CONVERGED (results readable) */
  double lowprec_rel_switch;/* mixed precision: relative energy change that ends the
                               low-precision phase (so does meeting the stop rule, a
                               failed steepest-descent line search, or lowprec_max_iter);
                               <= 0 picks 1e-9 (FP32) / 1e-5 (BF16) */
  int64_t lowprec_max_iter; /* mixed precision: cap on low-precision iterations; default max_iter */
  int32_t graph_iters;      /* CG iterations per captured hipGraph replay; <= 0: eager
                               launches; default 16 */
  int32_t history;          /* keep per-iteration history rows (omm_get_history); default 1 */
  int32_t history_max;      /* rows kept per system; default 20000 */
  double ne_tol;            /* electron-count check tolerance; <= 0 disables; default 0 */
  int32_t autotune;         /* 1: time kernel variants at first minimize and keep the
                               fastest (cached in tune_cache when set); default 0 */
  const char* tune_cache;   /* path of the autotuner cache file, or NULL: one line per
                               product step and work-list size, "key code" with
                               code = 10 * group-width plan (0: 1, 1: 2, 2: 4 tiles;
                               for the n x n projections also 3: 2 rows)
                               + waves per group; a line whose shape this library
                               cannot launch is ignored and tuned again */
  void* hip_stream;         /* hipStream_t to run on; NULL: the library makes its own */
  int32_t tile_group[3];    /* launch shape of the tile products (direction products,
                               n x n projections, gradient): output tiles per wave
                               (1, 2 or 4 of one output row; for the n x n
                               projections also -2: two consecutive output rows
                               of one column, which share each loaded H D, S D
                               tile) and waves per output group (1, 2, 4 or 8,
                               at most 4 with 4 tiles per wave or for the n x n
                               projections at 2 or -2); 0 = chosen by the library (heuristic
                               or autotuner).  A step given either value is not tuned.
                               Any shape gives the same result up to the order of
                               the sums; one shape gives bitwise repeatable results.
                               Default 0 */
  int32_t tile_split[3];
  const char* log_jsonl_path; /* NULL, or a file each omm_minimize appends one JSON line
                               per CG iteration and system to, after the solve (the
                               iteration state lives on the device during it):
                               {"solve", "system", "iter", "energy", "c" (the quartic's
                               c0..c4), "x", "grad_norm", "beta", "restart", "fp64"};
                               turns history on.  The library copies this path and
                               tune_cache; omm_init returns OMM_ERR_ARG when it cannot
                               open the file for appending.  Default NULL */
} omm_options;

/* Per-system results of omm_minimize. */
typedef struct {
  double energy;         /* shifted functional E~ (Eq. 4 with H - eta S) */
  double energy_band;    /* E~ + 2 eta n (Kim correction with spin factor 2, Sec. II;
                            n = n_occupied, see omm_set_occupied) */
  double grad_norm;      /* ||G||_F of the projected real gradient at the result */
  double electron_count; /* 2 Tr[(2I - S_W) S_W] (Listing 1) */
  int64_t iters_total;   /* CG iterations (line searches taken) */
  int64_t iters_fp64;    /* of which in FP64 */
  int64_t cg_restarts;   /* steepest-descent restarts */
  int32_t status;        /* omm_status of this system */
  int32_t precision_end; /* omm_precision of the last iteration */
  double seconds;        /* wall time of the omm_minimize call */
} omm_report;

/* Sizes and work counts of one system (for sizing outputs and for roofline figures). */
typedef struct {
  int64_t m, n;             /* basis size, number of wavefunctions */
  int64_t s_nval;           /* values of S's pattern = length of omm_density_matrix output */
  int64_t c_nval;           /* values of C0's pattern = length of omm_get_coeffs output */
  int64_t tiles_h, tiles_c, tiles_hc, tiles_w;  /* 16x16 tiles of H/S, C, HC, H_W */
  int64_t pairs_s1, pairs_s2, pairs_grad;       /* tile products per CG iteration step */
  double flops_alg_iter;    /* algorithmic flops of one CG iteration: 2*r*k*c summed
                               over the unpadded atom-block products (with kinetic
                               preconditioning: plus the product P G, 2 m^2 n) */
  double flops_exec_iter;   /* flops the tile kernels execute per iteration */
  double bytes_alg_iter;    /* algorithmic HBM bytes of one iteration's products
                               (each unpadded operand and output element moved once,
                               at the context's operand/output precision) */
  /* the same three figures per product step: [0] direction products H D, S D,
   * [1] n x n projections, [2] gradient products */
  double flops_alg_step[3];
  double flops_exec_step[3];
  double bytes_alg_step[3];
  /* launch shape in use per product step: output tiles per wave (group width;
   * -2 for two output rows of one column in the n x n projections) and waves
   * splitting one group's work list (chosen by heuristic or autotuner) */
  int32_t tile_group[3];
  int32_t tile_split[3];
} omm_sizes;

typedef struct omm_ctx omm_ctx;

/* Fills *opt with the defaults listed above. */
void omm_default_options(omm_options* opt);

/* Creates a context for one system (Sec. III B solver input).
 *   H, S  : m x m, identical block structure, square diagonal blocks, both symmetric
 *           (all blocks stored, not one triangle; a block pattern that is not
 *           symmetric is OMM_ERR_ARG).  H is shifted to H - eta S here.
 *   n_occ : number of wavefunction columns n (1 <= n <= m).
 *   mode  : omm_mode.  OMM_DENSE_CHOLESKY factorizes S (OMM_ERR_NOT_SPD if it fails).
 *   opt   : may be NULL for defaults.
 * On success *out owns device copies of H and S; free it with omm_destroy. */
int omm_init(omm_ctx** out, const omm_matrix* H, const omm_matrix* S, int64_t n_occ,
             int32_t mode, const omm_options* opt);

/* Creates one context holding `count` independent systems (snapshots, separate
 * structures) that every later call advances together, each with its
 * own H[i], S[i], n_occ[i], modes[i] and Kim shift etas[i] (etas may be NULL:
 * opt->eta for all); the other options are shared (filter_eps applies to the
 * block-sparse systems only).  System indices 0..count-1 are used by the
 * per-system calls below. */
int omm_init_batch(omm_ctx** out, int32_t count, const omm_matrix* H, const omm_matrix* S,
                   const int64_t* n_occ, const int32_t* modes, const double* etas,
                   const omm_options* opt);

/* Complex Hermitian systems, e.g. the k-points of a periodic structure (Eqs.
 * 3-5 with C^dagger; the paper's runs are at the Gamma point, Sec. IV A): the
 * same arguments as omm_init_batch, with H[i], S[i] complex Hermitian.  Their
 * omm_matrix structures are as for real matrices, but `val` holds 2 nval
 * doubles, the real and imaginary part of each value interleaved, in host
 * memory (memspace OMM_HOST); n_occ[i] counts complex wavefunctions.  Each
 * system is held as its real embedding [[Re Z, -Im Z], [Im Z, Re Z]] (every
 * atom block split into a real-part and an imaginary-part block), on which the
 * real kernels run: the embedded functional is twice the complex one and CG
 * on it takes the steps of complex CG with real inner products, at twice the
 * flops of complex arithmetic.  On such a context: omm_set_coeffs and
 * omm_update_hs take complex matrices (host); omm_density_matrix,
 * omm_energy_density and omm_get_coeffs write complex values (2 nval
 * doubles, host memory only), omm_get_projected complex n x n matrices;
 * reports, history and omm_query describe the complex system (energy,
 * electron count, quartic halved, gradient norm divided by sqrt 2, tol_grad
 * applies to it; omm_query's work counts are those of the embedding).
 * omm_density_matrix_noalloc refuses complex contexts.  Errors as omm_init_batch. */
int omm_init_complex(omm_ctx** out, int32_t count, const omm_matrix* H, const omm_matrix* S,
                     const int64_t* n_occ, const int32_t* modes, const double* etas,
                     const omm_options* opt);

/* Sets the initial guess of system `sys` (Sec. III D: random values inside the
 * localization radius).  C0 is m x n with the same block rows as H; its block
 * pattern is the pattern kept fixed during minimization (Sec. III B) and must
 * include every column block once; in dense modes every block must be stored.
 * Column blocks must be at most 16 wide in OMM_BLOCK_SPARSE mode. */
int omm_set_coeffs(omm_ctx* ctx, int32_t sys, const omm_matrix* C0);

/* New values of H and S for system `sys` on the block structure and value
 * layout (val_off) given at init: the next SCF step (new H) or MD step (new H
 * and S) reuses the context, its symbolic phase, tuned kernels and captured
 * graphs (Sec. III A, Fig. 2: the solver is called again at every SCF step).
 * The Kim shift and, in OMM_DENSE_CHOLESKY mode, the Cholesky reduction are
 * redone; a kinetic preconditioner is removed (it depends on S: set it again).
 * Values host or device, borrowed for the call.  A warm start from the
 * previous solution is omm_set_coeffs with the C of omm_get_coeffs.  Outputs
 * (rho, C, ...) wait for the next omm_minimize (OMM_ERR_STATE before it).
 * Different structure or layout: OMM_ERR_ARG; S not positive definite in
 * Cholesky mode: OMM_ERR_NOT_SPD. */
int omm_update_hs(omm_ctx* ctx, int32_t sys, const omm_matrix* H, const omm_matrix* S);

/* Coefficient reuse across MD steps (Sec. III D; Table 1 OMM.Extrapolate),
 * host memory only, no context: writes into out (to->nval doubles, in the
 * layout of to->val_off) the guess for the pattern `to` of the new geometry.
 * Blocks of `to` missing from `cur` start at zero (atoms that came within the
 * localization radius); blocks of `cur` missing from `to` are dropped.  With
 * prev != NULL (the step before cur) a block present in both takes the linear
 * extrapolation 2 cur - prev; otherwise the value of cur.  cur, prev and to
 * must have the same block rows and columns and block sizes.  Errors:
 * OMM_ERR_ARG, message in omm_last_error(NULL). */
int omm_remap_coeffs(const omm_matrix* cur, const omm_matrix* prev, const omm_matrix* to, double* out);

/* Restart file of C (Sec. III E, the m_write / m_read pair): omm_write_coeffs
 * stores the block structure and values of C (host memory) in a binary file
 * (magic "OMMCOEF1", little-endian: int32 nbrow, nbcol; int64 nnzb, nval;
 * int32 row_bsz[nbrow], col_bsz[nbcol]; int64 row_ptr[nbrow+1]; int32
 * col_idx[nnzb]; then each block's row-major doubles in block order).
 * omm_read_coeffs reads such a file and, as omm_remap_coeffs does, corrects
 * its pattern to `to` (the current geometry's): out receives to->nval
 * doubles.  File or format errors: OMM_ERR_ARG, message in
 * omm_last_error(NULL). */
int omm_write_coeffs(const char* path, const omm_matrix* C);
int omm_read_coeffs(const char* path, const omm_matrix* to, double* out);

/* Kim functional with more wavefunctions than occupied states (Sec. II, step
 * 2: C is m x n' with n' > n): the n_occ given at init is the column count n'
 * of C, and this call declares that only n_occupied of them are occupied
 * (2 n_occupied electrons).  It changes what is reported, not what is
 * minimized: energy_band = E~ + 2 eta n_occupied and the electron-count check
 * against 2 n_occupied.  Default n_occupied = n'.  Requires
 * 1 <= n_occupied <= n'; otherwise OMM_ERR_ARG.  May be called at any time. */
int omm_set_occupied(omm_ctx* ctx, int32_t sys, int64_t n_occupied);

/* Kinetic-energy preconditioning (Sec. II, Eq. 7; Table 1 OMM.Precon and
 * OMM.TPreconScale): computes P = (S + T/tau)^-1 once on the device (Cholesky
 * factorization and explicit inverse) and from the next omm_minimize on
 * multiplies every CG gradient by P: the direction follows -P G and
 * beta = max(0, <P G, G - G_old> / <P G_old, G_old>).  The minimum is the
 * same; only the path to it changes.  T is the kinetic-energy matrix on the
 * block structure of H and S (values host or device, borrowed for the call),
 * tau > 0 its scale.  Dense only, like the paper: the context must hold one
 * OMM_DENSE system and use FP64 products, else OMM_ERR_ARG.  S + T/tau not
 * positive definite: OMM_ERR_NOT_SPD.  T == NULL removes the preconditioner.
 * The library owns P (m x m doubles) until omm_destroy. */
int omm_set_preconditioner(omm_ctx* ctx, const omm_matrix* T, double tau);

/* Runs CG on every system of the context until each one stops (tol_grad,
 * rel_tol, max_iter, or a failed line search).  reports[count] receives the
 * per-system results (may be NULL).  Returns the worst per-system status.
 * Calling it again restarts from the coefficients set by omm_set_coeffs. */
int omm_minimize(omm_ctx* ctx, omm_report* reports);

/* omm_minimize for `count` independently built contexts in one go (the solver
 * contract of Sec. III B, applied to many problems at once: separate
 * structures, SCF snapshots).  Each context keeps its own systems, options,
 * tuned kernels and outputs; their CG iterations are captured together into
 * one hipGraph (the contexts dealt to 4 branch streams, so the kernels of
 * different contexts may run concurrently), one replay runs graph_iters
 * iterations of all of them (the smallest graph_iters of the list), and the
 * host reads the states of all contexts once per replay.  Contexts that
 * finish early idle (their kernels exit at once) until all are done.  The
 * graph is kept by ctxs[0] and reused while the same contexts are passed in
 * the same order and none of them has been re-planned.  The call runs on the
 * stream of ctxs[0] and returns when every context is done; all contexts
 * must live on the current device.  reports receives the reports of
 * ctxs[0]'s systems, then ctxs[1]'s, ... (may be NULL).  Returns the worst
 * status; messages in omm_last_error(ctxs[0]).  Contexts built together with
 * omm_init_batch run faster still (one launch per kernel for all systems). */
int omm_batch_minimize(omm_ctx* const* ctxs, int32_t count, omm_report* reports);

/* rho = 2 C (2I - S_W) C^T (Eq. 5) of system `sys` at the current C, on the
 * block pattern of S and in the value layout (val_off) of the S passed at init:
 * `rho` holds s_nval doubles in host or device memory (omm_memspace `where`). */
int omm_density_matrix(omm_ctx* ctx, int32_t sys, double* rho, int32_t where);

/* omm_density_matrix for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, with the intermediate C (2I - S_W) and
 * rho tiles in a fixed device scratch array of the library (32 MiB per GPU,
 * held until the process ends) instead of context buffers, and no host
 * staging: `rho_dev` is device memory (s_nval doubles, caller-owned) on the
 * context's device, which must be current.  The call allocates and frees
 * nothing.  A context needing more than 16384 scratch tiles (the C M tiles
 * plus the tiles of S's block pattern, 16 x 16 doubles each) gets
 * OMM_ERR_ARG.  All calls on one GPU share its scratch array: calls that
 * overlap in time on one GPU (from several host threads or streams) race and
 * must be serialized by the caller.  Returns when the result is in rho_dev. */
int omm_density_matrix_noalloc(omm_ctx* ctx, int32_t sys, double* rho_dev);

/* Energy density rho_E = 2 C H_W C^T (Eq. 6, the S-derivative term of the
 * forces) with the Kim correction rho_E + eta rho (Sec. II), where H_W =
 * C^T (H - eta S) C and eta is the system's shift; at eta = 0 this is plain
 * 2 C H_W C^T.  Same pattern, layout, memory spaces, call order and errors as
 * omm_density_matrix: `rho_e` holds s_nval doubles owned by the caller. */
int omm_energy_density(omm_ctx* ctx, int32_t sys, double* rho_e, int32_t where);

/* Current C of system `sys` in the layout of its C0 (c_nval doubles).  For
 * OMM_DENSE_CHOLESKY this is the back-transformed C = U^-1 C~. */
int omm_get_coeffs(omm_ctx* ctx, int32_t sys, double* C, int32_t where);

/* Dense n x n row-major H_W and S_W (Eq. 3) of system `sys` at the current C
 * (either pointer may be NULL). */
int omm_get_projected(omm_ctx* ctx, int32_t sys, double* HW, double* SW, int32_t where);

/* Per-iteration history of the last omm_minimize of system `sys` (host memory):
 * rows of OMM_HISTORY_COLS doubles [E~ after the step, c0, c1, c2, c3, c4, x*,
 * ||G||_F after the step, beta, restart flag, precision]; *rows receives the
 * number of rows written (at most max_rows). */
#define OMM_HISTORY_COLS 11
int omm_get_history(omm_ctx* ctx, int32_t sys, double* out, int64_t max_rows, int64_t* rows);

/* Sizes and work counts of system `sys` (sys = -1: sums over the batch). */
int omm_query(const omm_ctx* ctx, int32_t sys, omm_sizes* sizes);

/* Device time of the tile-product kernels of the last omm_minimize, measured
 * with HIP events on the context's stream around every launch of each kernel
 * class (0: direction products H D, S D; 1: n x n projections; 2: gradient
 * products).  ms[3] total milliseconds, launches[3] launch counts.  Timing is
 * recorded only when enabled with omm_set_timing(ctx, 1) before the call. */
int omm_set_timing(omm_ctx* ctx, int32_t enable);
int omm_kernel_times(const omm_ctx* ctx, double* ms, int64_t* launches);

/* Average device time in milliseconds (*avg_ms) of one launch of product step
 * `step` (0: direction products H D, S D; 1: n x n projections; 2: gradient
 * products), over `reps` (1..100000) launches issued back to back on the
 * context's stream between two HIP events, after one untimed launch.  It uses
 * the context's tuned launch shape and its product precision (the low
 * precision of a mixed run) on the operands of the last omm_minimize, which
 * must have run (else OMM_ERR_STATE); it overwrites only intermediate
 * products, so coefficients, energies and density matrices are unchanged.
 * Blocks until the timing is done. */
int omm_time_step(omm_ctx* ctx, int32_t step, int32_t reps, double* avg_ms);

/* Name of a status code. */
const char* omm_status_str(int32_t status);

/* Message of the last error on this context ("" if none); ctx may be NULL for
 * errors of a failed omm_init/omm_init_batch or of the context-free calls
 * (omm_remap_coeffs, omm_write_coeffs, omm_read_coeffs) on the calling thread. */
const char* omm_last_error(const omm_ctx* ctx);

/* Releases every device buffer of the context. */
void omm_destroy(omm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* OMM_MI355X_H */
