// Exact three-part bf16 split of FP32 values and the fragment-blocked
// operand planes of the QST_F32X6 complex products (written by the split
// kernels of k_xgemm.hip and, in the combined likelihood-and-gradient call,
// by the last adjoint POVM stage).
//
// x = h + m + l exactly for every finite FP32 x: h = bf16(x), m = bf16(x - h),
// l = bf16(x - h - m), each rounded to nearest even; x - h and x - h - m are
// exact in FP32, and the three parts carry 3 x 8 significand bits.
//
// Planes of a d x d complex matrix as the row operand of a product (row r,
// k = column): unit (rb, kb, g, s) of 1 KB holds rows 32 rb .. 32 rb + 31,
// k = 16 kb .. 16 kb + 15 of group g (re, im, re + im, re - im) and part s
// (h, m, l); lane u of the unit holds row 32 rb + u % 32, k = 16 kb +
// 8 (u / 32) .. + 7 as one 16-byte vector (the MFMA fragment of that lane).
// Unit (rb, kb, g, s) starts at vector (((rb * d / 16 + kb) * NG + g) * 3 + s) * 64.
#pragma once

#include "qst_device.h"

namespace qst {

constexpr int kX6UnitVecs = 64;  // 16-byte vectors per 1 KB unit

__device__ __forceinline__ uint32_t bf16x2_rne(float a, float b) {
  typedef __bf16 bf2v_t __attribute__((ext_vector_type(2)));
  const bf2v_t v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// x = H + M + L exactly, eight values, bf16 bit patterns packed in pairs.
__device__ __forceinline__ void split3(const float (&x)[8], u16x8& H, u16x8& M, u16x8& L) {
  u32x4 h, m, l;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    h[i] = bf16x2_rne(x[2 * i], x[2 * i + 1]);
    float r0 = x[2 * i] - bf16_lo(h[i]), r1 = x[2 * i + 1] - bf16_hi(h[i]);
    m[i] = bf16x2_rne(r0, r1);
    r0 -= bf16_lo(m[i]);
    r1 -= bf16_hi(m[i]);
    l[i] = bf16x2_rne(r0, r1);
  }
  H = __builtin_bit_cast(u16x8, h);
  M = __builtin_bit_cast(u16x8, m);
  L = __builtin_bit_cast(u16x8, l);
}

// One lane's slot of a unit block: the 8 values (re, im) split into the
// NG groups (re, im, re + im and, with NG = 4, re - im), three parts each.
// out points at the unit block's first unit plus the lane.
template <int NG>
__device__ __forceinline__ void write_unit_block(u16x8* out, const float (&re)[8], const float (&im)[8]) {
  float g2[8];
  split3(re, out[0 * kX6UnitVecs], out[1 * kX6UnitVecs], out[2 * kX6UnitVecs]);
  split3(im, out[3 * kX6UnitVecs], out[4 * kX6UnitVecs], out[5 * kX6UnitVecs]);
#pragma unroll
  for (int e = 0; e < 8; ++e) g2[e] = re[e] + im[e];
  split3(g2, out[6 * kX6UnitVecs], out[7 * kX6UnitVecs], out[8 * kX6UnitVecs]);
  if constexpr (NG == 4) {
#pragma unroll
    for (int e = 0; e < 8; ++e) g2[e] = re[e] - im[e];
    split3(g2, out[9 * kX6UnitVecs], out[10 * kX6UnitVecs], out[11 * kX6UnitVecs]);
  }
}

}  // namespace qst
