// Device-side helpers shared by the gfx950 kernels: complex storage types,
// bfloat16 rounding, MFMA wrappers and deterministic wave64 reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qst {

template <typename R>
struct alignas(2 * sizeof(R)) Cx {
  R re, im;
};

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// --------------------------------------------------------------------------
// bfloat16 round-to-nearest-even of a float (gfx950's FP32 -> BF16
// conversion instruction in the default rounding mode), as the 16-bit
// pattern and as the float it represents; bf16x8 converts eight floats with
// four packed conversions.  The split x = hi + lo takes hi = bf16(x) and
// lo = bf16(x - hi) (x - hi is exact in FP32).
// --------------------------------------------------------------------------
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf16_value(float x) { return float((__bf16)x); }
__device__ __forceinline__ float bf16_to_float(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }
__device__ __forceinline__ uint32_t bf16x2_bits(float a, float b) {
  const bf2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u16x8 bf16x8(const float (&v)[8]) {
  const u32x4 w = {bf16x2_bits(v[0], v[1]), bf16x2_bits(v[2], v[3]), bf16x2_bits(v[4], v[5]),
                   bf16x2_bits(v[6], v[7])};
  return __builtin_bit_cast(u16x8, w);
}
// hi and lo planes of eight values
__device__ __forceinline__ void bf16x8_split(const float (&v)[8], u16x8& hi, u16x8& lo) {
  hi = bf16x8(v);
  float r[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = v[i] - bf16_to_float(hi[i]);
  lo = bf16x8(r);
}

// --------------------------------------------------------------------------
// MFMA 16x16 tiles.  For the fp64/fp32 K=4 forms lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; for the bf16 K=32 form lane l supplies
// A[l%16][8(l/16)+0..7] and B[8(l/16)+0..7][l%16].  Lane l holds the four
// outputs D[row(l/16, v)][l%16], v = 0..3, with row = 4(l/16) + v for the
// fp32 and bf16 forms and row = l/16 + 4v for the fp64 form.
// --------------------------------------------------------------------------
template <typename R>
struct Mfma;

template <>
struct Mfma<double> {
  typedef d4 acc;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int v) { return q + 4 * v; }
};

template <>
struct Mfma<float> {
  typedef f4 acc;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
};

__device__ __forceinline__ f4 mfma_bf16(u16x8 a, u16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                 __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

__device__ __forceinline__ u16x8 bf16_neg(u16x8 a) { return a ^ (uint16_t)0x8000u; }

// --------------------------------------------------------------------------
// Deterministic reductions (fixed order for a fixed launch shape).
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a 256-thread block; result valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* lds4) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) lds4[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
  return s;
}

// Workgroups of a launch are handed to the 8 XCDs in turn (workgroup b to
// XCD b % 8), and each XCD has its own L2.  xcd_order renumbers them so that
// each XCD runs one contiguous range of logical indices; logical neighbours,
// which share cache lines and operand panels, then share an L2.  It is a
// bijection on [0, grid) for every grid size, so correctness never depends
// on the hardware's actual placement.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t grid) {
  constexpr int64_t kXcds = 8;
  const int64_t per = grid / kXcds, rem = grid % kXcds;
  const int64_t x = b % kXcds, q = b / kXcds;
  return x < rem ? x * (per + 1) + q : rem * (per + 1) + (x - rem) * per + q;
}

// Lower-triangular tile index t -> (R, C) with R >= C, t = R(R+1)/2 + C.
__device__ __forceinline__ void tri_decode(int64_t t, int& R, int& C) {
  int r = int((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
  while (int64_t(r) * (r + 1) / 2 > t) --r;
  while (int64_t(r + 1) * (r + 2) / 2 <= t) ++r;
  R = r;
  C = int(t - int64_t(r) * (r + 1) / 2);
}

// Sum of nb FP64 partials in a fixed order by a 256-thread block (strided
// per thread, then block_sum256); result valid in thread 0.
__device__ __forceinline__ double sum_partials256(const double* part, int nb, double* lds4) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[b];
  return block_sum256(acc, lds4);
}

// Per-outcome arithmetic of the likelihood in the storage precision of p
// and f: ln p_k (the sum over k is accumulated in FP64 on every path) and
// the cotangent g'_k = F - f_k / p_k (F where f_k = 0).  FP64 storage: FP64
// throughout.  FP32 storage: the hardware base-2 logarithm times ln 2 and
// the hardware reciprocal (about one ulp each, the size of the rounding of
// p itself; p is a probability, far from the denormal range the hardware
// flushes, except where it is 0 or negative, which the callers treat
// apart).
__device__ __forceinline__ double ln_prob(double p) { return log(p); }
__device__ __forceinline__ double ln_prob(float p) {
  return double(__builtin_amdgcn_logf(p) * 0.693147180559945309f);
}
__device__ __forceinline__ double cotangent(double F, double f, double p) { return f != 0.0 ? F - f / p : F; }
__device__ __forceinline__ float cotangent(double F, float f, float p) {
  return f != 0.0f ? float(F) - f * __builtin_amdgcn_rcpf(p) : float(F);
}

}  // namespace qst
