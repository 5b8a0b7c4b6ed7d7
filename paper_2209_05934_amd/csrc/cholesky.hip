// FP64 Cholesky reduction of the generalized problem for cubic-scaling OMM
// (arXiv 2209.05934, Sec. II: reducing the generalized eigenvalue problem to
// standard form via the Cholesky factorization; dense matrices only, Sec. III B).
//
//   S = L L^T (L = U^T lower triangular),  H~ = L^-1 H L^-T,  C~ = L^T C,
//   and after minimization C = L^-T C~.
//
// All matrices are dense grids of 16x16 tiles (tile (I, J) at base + I*ld + J,
// elements in the storage order of tpos).
// The factorization is right-looking by tile columns: factor the diagonal
// tile (and invert it) in LDS, scale the panel below it by L_KK^-T on MFMA,
// update the trailing lower triangle with one MFMA tile product per tile.
// Triangular solves run tile row by tile row with one wave per tile column.
#include "kernels.hpp"
#include "tile_ops.hpp"

namespace omm {

namespace {

__device__ __forceinline__ size_t tix(int base, int ld, int I, int J) {
  return ((size_t)base + (size_t)I * ld + J) * TE;
}

__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ A, int base, int RT, int K,
                                                 double* __restrict__ Linv, int* __restrict__ status) {
  __shared__ double a[16][17];
  __shared__ double li[16][17];
  const int tid = threadIdx.x, r = tid >> 4, c = tid & 15;
  double* tile = A + tix(base, RT, K, K);
  a[r][c] = tile[tpos(r, c)];
  __syncthreads();
  for (int k = 0; k < 16; ++k) {
    if (tid == 0) {
      double d = a[k][k];
      if (!(d > 0.0)) {
        *status = 1;
        d = 1.0;
      }
      a[k][k] = sqrt(d);
    }
    __syncthreads();
    if (tid > k && tid < 16) a[tid][k] /= a[k][k];
    __syncthreads();
    if (r > k && c > k && c <= r) a[r][c] -= a[r][k] * a[c][k];
    __syncthreads();
  }
  tile[tpos(r, c)] = (c <= r) ? a[r][c] : 0.0;
  if (tid < 16) {   // column j of L^-1 by forward substitution
    const int j = tid;
    for (int i = 0; i < 16; ++i) {
      if (i < j) {
        li[i][j] = 0.0;
        continue;
      }
      double s = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) s -= a[i][k] * li[k][j];
      li[i][j] = s / a[i][i];
    }
  }
  __syncthreads();
  Linv[(size_t)K * TE + tpos(r, c)] = li[r][c];
}

// L(I,K) = A(I,K) L_KK^-T for I > K
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ A, int base, int RT, int K,
                                                  const double* __restrict__ Linv) {
  const int lane = threadIdx.x & 63;
  const int I = K + 1 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (I >= RT) return;
  double* t = A + tix(base, RT, I, K);
  Frag<double> fa, fb;
  ld_row(fa, t, lane);
  ld_row(fb, Linv + (size_t)K * TE, lane);     // B = Linv^T
  d4 acc = vzero<d4>();
  mma(acc, fa, fb);
#pragma unroll
  for (int r = 0; r < 4; ++r) t[out_off<d4, double>(lane, r)] = acc[r];
}

// A(I,J) -= L(I,K) L(J,K)^T for K < J <= I
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ A, int base, int RT, int K,
                                                   int64_t npair) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= npair) return;
  int64_t i = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > p) --i;
  while ((i + 1) * (i + 2) / 2 <= p) ++i;
  const int64_t j = p - i * (i + 1) / 2;
  const int I = K + 1 + (int)i, J = K + 1 + (int)j;
  Frag<double> fa, fb;
  ld_row(fa, A + tix(base, RT, I, K), lane);
  ld_row(fb, A + tix(base, RT, J, K), lane);   // B = L(J,K)^T
  d4 acc = vzero<d4>();
  mma(acc, fa, fb);
  double* t = A + tix(base, RT, I, J);
#pragma unroll
  for (int r = 0; r < 4; ++r) t[out_off<d4, double>(lane, r)] -= acc[r];
}

// forward substitution, tile row I of X = L^-1 op(B): X(I,J) = Linv_I (op(B)(I,J) - sum_{K<I} L(I,K) X(K,J))
__global__ __launch_bounds__(256) void k_trsm_fwd(const double* __restrict__ L, int lbase, int RT,
                                                const double* __restrict__ Linv, const double* __restrict__ B,
                                                int bbase, int transB, double* __restrict__ X, int xbase,
                                                int ncols, int I) {
  const int lane = threadIdx.x & 63;
  const int J = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (J >= ncols) return;
  d4 acc = vzero<d4>();
  for (int K = 0; K < I; ++K) {
    Frag<double> fa, fb;
    ld_row(fa, L + tix(lbase, RT, I, K), lane);
    ld_col(fb, X + tix(xbase, ncols, K, J), lane);
    mma(acc, fa, fb);
  }
  const int j = lane & 15, q = lane >> 4;
  d4 rhs;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = Lay<d4>::row(q, r);
    const double bv = transB ? B[tix(bbase, ncols, J, I) + tpos(j, row)] : B[tix(bbase, ncols, I, J) + tpos(row, j)];
    rhs[r] = bv - acc[r];
  }
  __shared__ __align__(16) double lt[4][TE];
  Frag<double> fa, fb = acc_as_b_lds(rhs, lt[threadIdx.x >> 6], lane);
  ld_row(fa, Linv + (size_t)I * TE, lane);
  d4 out = vzero<d4>();
  mma(out, fa, fb);
  double* t = X + tix(xbase, ncols, I, J);
#pragma unroll
  for (int r = 0; r < 4; ++r) t[out_off<d4, double>(lane, r)] = out[r];
}

// Cout = L^T Cin on a dense RT x WT grid
__global__ __launch_bounds__(256) void k_apply_lt(const double* __restrict__ L, int lbase, int RT,
                                                const double* __restrict__ Cin, double* __restrict__ Cout,
                                                int cbase, int WT) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= RT * WT) return;
  const int I = p / WT, g = p % WT;
  d4 acc = vzero<d4>();
  for (int K = I; K < RT; ++K) {
    Frag<double> fa, fb;
    ld_col(fa, L + tix(lbase, RT, K, I), lane);    // A = L(K,I)^T
    ld_col(fb, Cin + tix(cbase, WT, K, g), lane);
    mma(acc, fa, fb);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) Cout[tix(cbase, WT, I, g) + out_off<d4, double>(lane, r)] = acc[r];
}

// backward substitution, tile row I of Cout = L^-T Cin
__global__ __launch_bounds__(256) void k_trsm_bwd_t(const double* __restrict__ L, int lbase, int RT,
                                                  const double* __restrict__ Linv, const double* __restrict__ Cin,
                                                  double* __restrict__ Cout, int cbase, int WT, int I) {
  const int lane = threadIdx.x & 63;
  const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (g >= WT) return;
  d4 acc = vzero<d4>();
  for (int K = I + 1; K < RT; ++K) {
    Frag<double> fa, fb;
    ld_col(fa, L + tix(lbase, RT, K, I), lane);    // A = L(K,I)^T
    ld_col(fb, Cout + tix(cbase, WT, K, g), lane);
    mma(acc, fa, fb);
  }
  d4 rhs;
#pragma unroll
  for (int r = 0; r < 4; ++r) rhs[r] = Cin[tix(cbase, WT, I, g) + out_off<d4, double>(lane, r)] - acc[r];
  __shared__ __align__(16) double lt[4][TE];
  Frag<double> fa, fb = acc_as_b_lds(rhs, lt[threadIdx.x >> 6], lane);
  ld_col(fa, Linv + (size_t)I * TE, lane);         // A = Linv_I^T
  d4 out = vzero<d4>();
  mma(out, fa, fb);
#pragma unroll
  for (int r = 0; r < 4; ++r) Cout[tix(cbase, WT, I, g) + out_off<d4, double>(lane, r)] = out[r];
}

}  // namespace

#define CLAUNCH(kern, grid, ...)                                         \
  do {                                                                  \
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, __VA_ARGS__);       \
    OMM_HIP(hipGetLastError());                                         \
  } while (0)

void chol_factor(hipStream_t s, double* A, int base, int RT, double* Linv, int* status) {
  for (int K = 0; K < RT; ++K) {
    CLAUNCH(k_chol_diag, dim3(1), A, base, RT, K, Linv, status);
    const int rest = RT - K - 1;
    if (rest <= 0) break;
    CLAUNCH(k_chol_panel, dim3((rest + 3) / 4), A, base, RT, K, (const double*)Linv);
    const int64_t np = (int64_t)rest * (rest + 1) / 2;
    CLAUNCH(k_chol_update, dim3((unsigned)((np + 3) / 4)), A, base, RT, K, np);
  }
}

void chol_reduce_h(hipStream_t s, const double* L, int lbase, int RT, const double* Linv, double* H, int hbase,
                   double* work) {
  for (int I = 0; I < RT; ++I)   // work = L^-1 H
    CLAUNCH(k_trsm_fwd, dim3((RT + 3) / 4), L, lbase, RT, Linv, (const double*)H, hbase, 0, work, 0, RT, I);
  for (int I = 0; I < RT; ++I)   // H = L^-1 work^T = L^-1 H L^-T
    CLAUNCH(k_trsm_fwd, dim3((RT + 3) / 4), L, lbase, RT, Linv, (const double*)work, 0, 1, H, hbase, RT, I);
}

void chol_apply_lt(hipStream_t s, const double* L, int lbase, int RT, const double* Cin, double* Cout, int cbase,
                   int WT) {
  CLAUNCH(k_apply_lt, dim3((RT * WT + 3) / 4), L, lbase, RT, Cin, Cout, cbase, WT);
}

void chol_solve_lt(hipStream_t s, const double* L, int lbase, int RT, const double* Linv, const double* Cin,
                   double* Cout, int cbase, int WT) {
  for (int I = RT - 1; I >= 0; --I)
    CLAUNCH(k_trsm_bwd_t, dim3((WT + 3) / 4), L, lbase, RT, Linv, Cin, Cout, cbase, WT, I);
}

void chol_lower_inverse(hipStream_t s, const double* L, int lbase, int RT, const double* Linv, const double* Id,
                        double* X) {
  for (int I = 0; I < RT; ++I)
    CLAUNCH(k_trsm_fwd, dim3((RT + 3) / 4), L, lbase, RT, Linv, Id, 0, 0, X, 0, RT, I);
}

// P = (L L^T)^-1 = L^-T (L^-1 I) on a dense RT x RT grid at offset 0: forward
// substitution against the identity grid Id, then backward substitution with
// L^T (the explicit inverse of kinetic preconditioning, Eq. 7)
void chol_inverse(hipStream_t s, const double* L, int RT, const double* Linv, const double* Id, double* work,
                  double* P) {
  chol_lower_inverse(s, L, 0, RT, Linv, Id, work);
  chol_solve_lt(s, L, 0, RT, Linv, work, P, 0, RT);
}

}  // namespace omm
