// Device helpers: 16x16 tile fragments and CDNA MFMA products for gfx950.
//
// One 64-lane wavefront multiplies two 16x16 tiles.  Lane l = i + 16*q
// (i = l & 15, q = l >> 4) supplies, at MFMA step s = 0..3, A[i][k] and
// B[k][j=i] for one tile index k = K(q, s).  The pairing of k with (q, s) is
// free as long as A and B agree (KMap).  Accumulator register r of lane (j, q)
// holds output row
//   v_mfma_f64_16x16x4f64 : 4r + q
//   v_mfma_f32_16x16x4f32 and v_mfma_f32_16x16x16bf16_1k : 4q + r
// (the f64 placement was measured on gfx950 with delta operands).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace omm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16;

__device__ __forceinline__ bf16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16)0x7fc0;   // NaN
  u += 0x7fffu + ((u >> 16) & 1u);                               // round to nearest even
  return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float(((uint32_t)h) << 16); }

// value conversions between storage types
template <typename D, typename S> __device__ __forceinline__ D cvt(S v);
template <> __device__ __forceinline__ double cvt<double, double>(double v) { return v; }
template <> __device__ __forceinline__ float cvt<float, double>(double v) { return (float)v; }
template <> __device__ __forceinline__ float cvt<float, float>(float v) { return v; }
template <> __device__ __forceinline__ double cvt<double, float>(float v) { return (double)v; }
template <> __device__ __forceinline__ bf16 cvt<bf16, double>(double v) { return f2bf((float)v); }
template <> __device__ __forceinline__ bf16 cvt<bf16, float>(float v) { return f2bf(v); }
template <> __device__ __forceinline__ bf16 cvt<bf16, bf16>(bf16 v) { return v; }
template <> __device__ __forceinline__ float cvt<float, bf16>(bf16 v) { return bf2f(v); }
template <> __device__ __forceinline__ double cvt<double, bf16>(bf16 v) { return (double)bf2f(v); }

// accumulator type for an operand type
template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4 V; typedef double S; };
template <> struct Acc<float> { typedef f4 V; typedef float S; };
template <> struct Acc<bf16> { typedef f4 V; typedef float S; };

template <typename T> struct Frag { T v[4]; };
// BF16 values are kept packed as the operand of the BF16 MFMA
template <> struct Frag<bf16> { s4 v; };

// Storage order inside a 16x16 tile.  Element (r, c) has the row-major index
// e = 16 r + c, and e = 64 s + l splits it into a row group s (rows 4s .. 4s+3)
// and a lane l.  Row groups 2h and 2h + 1 are interleaved element by element:
// e sits at position 128 (s >> 1) + 2 l + (s & 1).  The four values a lane
// reads for an operand of a tile product (row group s = MFMA step s, lane l)
// are then two adjacent pairs, one 16-byte load each for FP64, and the
// accumulator registers r = 0, 1 and 2, 3 of an FP64 product land in adjacent
// pairs as well.
__host__ __device__ constexpr int tpos(int r, int c) {
  return ((r >> 3) << 7) | ((r & 3) << 5) | (c << 1) | ((r >> 2) & 1);
}
// row and column of the element at storage position p
__host__ __device__ constexpr int trow(int p) { return ((p >> 7) << 3) | ((p & 1) << 2) | ((p >> 5) & 3); }
__host__ __device__ constexpr int tcol(int p) { return (p >> 1) & 15; }
// Tiles of 4-byte values (FP32 copies and products) keep a lane's four
// operand values together: element 64 s + l at position 4 l + s, one 16-byte
// load per lane.  BF16 tiles keep the FP64 order (two 4-byte loads per lane,
// measured faster than one 8-byte load).
__host__ __device__ constexpr int tpos4(int r, int c) { return ((r & 3) << 6) | (c << 2) | (r >> 2); }
// position of element (r, c) in a tile of storage type S
template <typename S> __host__ __device__ constexpr int tpos_of(int r, int c) {
  return sizeof(S) == 4 ? tpos4(r, c) : tpos(r, c);
}

// tile index k supplied by lane-quad q at step s: the four quads of step s take
// the consecutive k = 4s .. 4s+3 (row group s of the tile, see tpos), so a
// column load reads two whole row groups per instruction (1 KB of an FP64
// tile) and MFMA step s contracts over one aligned group of four k, which a
// work-list entry can mark as all zero (step masks below)
template <typename T> struct KMap { static __device__ __forceinline__ int k(int q, int s) { return 4 * s + q; } };

// output row of accumulator register r in lane-quad q
template <typename V> struct Lay;
template <> struct Lay<d4> { static __device__ __forceinline__ int row(int q, int r) { return 4 * r + q; } };
template <> struct Lay<f4> { static __device__ __forceinline__ int row(int q, int r) { return 4 * q + r; } };

// "row" load: lane (i, q) takes tile[i][K(q, s)]   (A operand, or B^T)
template <typename T, typename S>
__device__ __forceinline__ void ld_row(Frag<T>& f, const S* __restrict__ t, int lane) {
  const int i = lane & 15, q = lane >> 4;
#pragma unroll
  for (int s = 0; s < 4; ++s) f.v[s] = cvt<T, S>(t[tpos_of<S>(i, KMap<T>::k(q, s))]);
}
// "col" load: lane (j, q) takes tile[K(q, s)][j] (B operand, or A^T): element
// 64 s + lane, at 2 lane + (s & 1) + 128 (s >> 1) in an FP64 or BF16 tile (two
// loads) and at 4 lane + s in an FP32 tile (one load)
template <typename T>
__device__ __forceinline__ void ld_col(Frag<T>& f, const double* __restrict__ t, int lane) {
  const double2 a = ((const double2*)t)[lane], b = ((const double2*)t)[64 + lane];
  f.v[0] = cvt<T, double>(a.x);
  f.v[1] = cvt<T, double>(a.y);
  f.v[2] = cvt<T, double>(b.x);
  f.v[3] = cvt<T, double>(b.y);
}
template <typename T>
__device__ __forceinline__ void ld_col(Frag<T>& f, const float* __restrict__ t, int lane) {
  const float4 a = ((const float4*)t)[lane];
  f.v[0] = cvt<T, float>(a.x);
  f.v[1] = cvt<T, float>(a.y);
  f.v[2] = cvt<T, float>(a.z);
  f.v[3] = cvt<T, float>(a.w);
}
__device__ __forceinline__ void ld_col(Frag<bf16>& f, const bf16* __restrict__ t, int lane) {
  const uint32_t* p = (const uint32_t*)t;
  f.v = __builtin_bit_cast(s4, make_uint2(p[lane], p[64 + lane]));
}

// A column load of the MFMA steps whose bit (kept >> s) & 1 is set (kept wave-uniform):
// the part of the tile a load instruction reads (steps 0-1 and 2-3 of an FP64 or BF16
// tile, all four of an FP32 tile) comes from the zero tile z when none of its steps
// is kept.  The instructions stay the same; the skipped MFMA steps never use the values.
template <typename T>
__device__ __forceinline__ void ld_col_kept(Frag<T>& f, const double* __restrict__ t, const double* __restrict__ z,
                                            int kept, int lane) {
  const double2 a = ((const double2*)((kept & 3) ? t : z))[lane];
  const double2 b = ((const double2*)((kept & 12) ? t : z))[64 + lane];
  f.v[0] = cvt<T, double>(a.x);
  f.v[1] = cvt<T, double>(a.y);
  f.v[2] = cvt<T, double>(b.x);
  f.v[3] = cvt<T, double>(b.y);
}
template <typename T>
__device__ __forceinline__ void ld_col_kept(Frag<T>& f, const float* __restrict__ t, const float* __restrict__ z,
                                            int kept, int lane) {
  ld_col(f, kept ? t : z, lane);
}
__device__ __forceinline__ void ld_col_kept(Frag<bf16>& f, const bf16* __restrict__ t, const bf16* __restrict__ z,
                                            int kept, int lane) {
  const uint32_t* p0 = (const uint32_t*)((kept & 3) ? t : z);
  const uint32_t* p1 = (const uint32_t*)((kept & 12) ? t : z);
  f.v = __builtin_bit_cast(s4, make_uint2(p0[lane], p1[64 + lane]));
}

__device__ __forceinline__ void mma(d4& acc, const Frag<double>& a, const Frag<double>& b) {
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[s], b.v[s], acc, 0, 0, 0);
}
__device__ __forceinline__ void mma(f4& acc, const Frag<float>& a, const Frag<float>& b) {
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[s], b.v[s], acc, 0, 0, 0);
}
// the same, only the steps s whose bit (act >> s) & 1 is set (act wave-uniform):
// a step whose four k hold no nonzero product contributes exact zeros
__device__ __forceinline__ void mma(d4& acc, const Frag<double>& a, const Frag<double>& b, int act) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
    if ((act >> s) & 1) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[s], b.v[s], acc, 0, 0, 0);
}
__device__ __forceinline__ void mma(f4& acc, const Frag<float>& a, const Frag<float>& b, int act) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
    if ((act >> s) & 1) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[s], b.v[s], acc, 0, 0, 0);
}
__device__ __forceinline__ void mma(f4& acc, const Frag<bf16>& a, const Frag<bf16>& b) {
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.v, b.v, acc, 0, 0, 0);
}
// one instruction covers all 16 k: the step mask cannot skip part of it
__device__ __forceinline__ void mma(f4& acc, const Frag<bf16>& a, const Frag<bf16>& b, int) { mma(acc, a, b); }

// Work-list entries may carry, in bits 27-30 of a B tile index, the MFMA steps
// whose four k hold no structurally nonzero product (set: skip); -1 is an absent
// tile.  Tile indices stay below 2^27.
constexpr int ENT_TILE_MASK = (1 << 27) - 1;
__device__ __forceinline__ int ent_tile(int id) { return id < 0 ? 0 : (id & ENT_TILE_MASK); }
__device__ __forceinline__ int ent_steps(int id) { return ~(id >> 27) & 15; }

template <typename V> __device__ __forceinline__ V vzero();
template <> __device__ __forceinline__ d4 vzero<d4>() { return d4{0.0, 0.0, 0.0, 0.0}; }
template <> __device__ __forceinline__ f4 vzero<f4>() { return f4{0.f, 0.f, 0.f, 0.f}; }

// accumulator register r of this lane sits at offset out_off<V, S>(lane, r) of
// a tile of storage type S
template <typename V, typename S>
__device__ __forceinline__ int out_off(int lane, int r) { return tpos_of<S>(Lay<V>::row(lane >> 4, r), lane & 15); }
// the same element in a tile stored transposed
template <typename V, typename S>
__device__ __forceinline__ int out_off_t(int lane, int r) { return tpos_of<S>(lane & 15, Lay<V>::row(lane >> 4, r)); }

// The transpose of an accumulator tile, in the same register layout: lane
// (j, q) register r receives element (j, row) with row = Lay<V>::row(q, r),
// which sits in lane row + 16 q' register r' with Lay<V>::row(q', r') = j.
// Shuffles of the whole wave (call with every lane active).
template <typename V>
__device__ __forceinline__ V transposed_tile(const V& a, int lane) {
  const int j = lane & 15, q = lane >> 4;
  constexpr bool F64 = sizeof(a[0]) == 8;
  const int qs = F64 ? (j & 3) : (j >> 2);   // Lay<d4>::row(q, r) = 4r + q, Lay<f4>::row(q, r) = 4q + r
  const int rs = F64 ? (j >> 2) : (j & 3);
  V out;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int src = Lay<V>::row(q, r) + 16 * qs;
    const auto v0 = __shfl(a[0], src, 64), v1 = __shfl(a[1], src, 64);
    const auto v2 = __shfl(a[2], src, 64), v3 = __shfl(a[3], src, 64);
    out[r] = rs == 0 ? v0 : (rs == 1 ? v1 : (rs == 2 ? v2 : v3));
  }
  return out;
}

// an FP64 accumulator tile as the B operand of the next product, through a
// 16x16 LDS tile owned by the calling wave, 16-byte aligned (LDS operations of
// one wave complete in order, so the reads see the writes)
__device__ __forceinline__ Frag<double> acc_as_b_lds(const d4& a, double* t, int lane) {
#pragma unroll
  for (int r = 0; r < 4; ++r) t[out_off<d4, double>(lane, r)] = a[r];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  Frag<double> f;
  ld_col(f, t, lane);
  return f;
}

// a double moved across lanes by a DPP pattern (both 32-bit halves)
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double lane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Deterministic full-wave sum, the same value in every lane (call with the
// whole wave active).  Within each row of 16 lanes: pairs (quad_perm 1,0,3,2),
// quads (quad_perm 2,3,0,1), then the mirrored half-row and row; every step
// adds two equal-shaped partial sums, so all lanes of a row agree.  The four
// row sums are then added in a fixed order from uniform lane reads.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  v += dpp_mov<0x140>(v);
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

}  // namespace omm
