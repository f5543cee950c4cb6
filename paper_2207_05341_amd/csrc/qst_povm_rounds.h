// Register-round machinery of the specialised product-POVM passes, shared by
// the pass kernels (k_povm_fast.hip) and the T T^dagger epilogue that applies
// the first pass to each finished output tile (qst_gemm_tiles.h).  See
// k_povm_fast.hip for the round structure.
#pragma once

#include "qst_device.h"
#include "qst_povm_ops.h"

namespace qst {

template <int G>
struct Rounds;
template <>
struct Rounds<3> {
  static constexpr int n = 2;
  static constexpr int bA[2] = {0, 1}, bB[2] = {1, 2};
  static constexpr bool opA[2] = {true, false}, opB[2] = {true, true};
};
template <>
struct Rounds<4> {
  static constexpr int n = 2;
  static constexpr int bA[2] = {0, 2}, bB[2] = {1, 3};
  static constexpr bool opA[2] = {true, true}, opB[2] = {true, true};
};
template <>
struct Rounds<5> {
  static constexpr int n = 3;
  static constexpr int bA[3] = {0, 2, 3}, bB[3] = {1, 3, 4};
  static constexpr bool opA[3] = {true, true, true}, opB[3] = {true, false, true};
};
template <>
struct Rounds<6> {
  static constexpr int n = 3;
  static constexpr int bA[3] = {0, 2, 4}, bB[3] = {1, 3, 5};
  static constexpr bool opA[3] = {true, true, true}, opB[3] = {true, true, true};
};

// Fixed bits of a round: the G-2 bit positions other than (bA, bB), listed
// in increasing order, each contributing an (r, c) pair.  Enumeration index
// u (2(G-2) bits): bit 2i of u is c at the i-th fixed position, bit 2i+1 is
// r there (interleaved, so for the top round u equals the outcome digits of
// the low positions).
template <int G>
__device__ __forceinline__ void fixed_bits(int u, int bA, int bB, int& r, int& c) {
  r = 0;
  c = 0;
  int i = 0;
#pragma unroll
  for (int b = 0; b < G; ++b) {
    if (b == bA || b == bB) continue;
    c |= ((u >> (2 * i)) & 1) << b;
    r |= ((u >> (2 * i + 1)) & 1) << b;
    ++i;
  }
}

// Contract the flagged bits of a 16-value register block x[mA * 4 + mB].
template <typename R, bool ADJ, bool TETRA>
__device__ __forceinline__ void contract16(Cx<R> x[16], bool opA, bool opB, const ModeMatrix& A) {
  if (opA) {
#pragma unroll
    for (int mB = 0; mB < 4; ++mB) {
      Cx<R> v[4] = {x[mB], x[4 + mB], x[8 + mB], x[12 + mB]};
      apply4<R, ADJ, TETRA>(v, A);
      x[mB] = v[0];
      x[4 + mB] = v[1];
      x[8 + mB] = v[2];
      x[12 + mB] = v[3];
    }
  }
  if (opB) {
#pragma unroll
    for (int mA = 0; mA < 4; ++mA) apply4<R, ADJ, TETRA>(x + 4 * mA, A);
  }
}

// (r, c) of value (mA, mB) of a round with fixed part (rf, cf).
__device__ __forceinline__ void rc_of(int rf, int cf, int bA, int bB, int mA, int mB, int& r, int& c) {
  r = rf | ((mA >> 1) << bA) | ((mB >> 1) << bB);
  c = cf | ((mA & 1) << bA) | ((mB & 1) << bB);
}

// Swizzled LDS position of (r, c) in a 2^G x 2^G tile (matrix-side kernel):
// c' = c ^ ((c >> A) & 3) ^ ((r & MR) << B), a bijection in c for every r.
// The constants spread each round's 16-lane groups over distinct banks: in
// round 0 a group varies c's high bits (the 4 x 4 block corners), in later
// rounds the low bits of r and of c.  Chosen by a 32-bank model of the
// three rounds (the model reproduces the measured conflict rates), in LDS
// cycles per ideal: G=6 1.0 (fp32) / 1.33 (fp64), G=5 1.33 / 1.0,
// G=4 2.0 / 2.0, against 2.7..4.0 for a plain c ^ r.
template <int G>
__device__ __forceinline__ int swz(int r, int c) {
  constexpr int A = G == 6 ? 4 : (G == 5 ? 3 : 2);
  constexpr int B = G == 4 ? 1 : 2;
  constexpr int MR = G == 4 ? 7 : 3;
  constexpr int M = (1 << G) - 1;
  return (r << G) | (c ^ ((c >> A) & 3) ^ (((r & MR) << B) & M));
}

// value m = mA*4 + mB of round 0 <-> 4 x 4 block entry (ri, ci)
__device__ __forceinline__ int blk_ri(int m) { return (((m & 3) >> 1) << 1) | ((m >> 2) >> 1); }
__device__ __forceinline__ int blk_ci(int m) { return ((m & 1) << 1) | ((m >> 2) & 1); }

// Forward matrix-side rounds of one 2^G x 2^G tile by its 4^(G-2) threads
// (thread t): x holds the thread's round-0 values (the 4 x 4 block at rows
// 4aq.., columns 4bq.., aq = t >> (G-2), bq = t & (2^(G-2) - 1), value m at
// blk_ri(m), blk_ci(m)); L is the tile's LDS area (4^G values, swizzled);
// out (NULL: compute, exchange, but store nothing) receives the tile's
// outcome-side values X'[kg].  Every thread of the workgroup must call it
// (it contains barriers).
template <typename R, bool TETRA, int G>
__device__ __forceinline__ void mat_fwd_rounds(Cx<R> (&x)[16], Cx<R>* L, int t, const ModeMatrix& A, Cx<R>* out) {
  using RD = Rounds<G>;
  const int bq = t & ((1 << (G - 2)) - 1), aq = t >> (G - 2);
#pragma unroll
  for (int rd = 0; rd < RD::n; ++rd) {
    const int bA = RD::bA[rd], bB = RD::bB[rd];
    int rf, cf;
    if (rd == 0) {
      rf = 4 * aq;
      cf = 4 * bq;
    } else {
      fixed_bits<G>(t, bA, bB, rf, cf);
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        int r, c;
        rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
        x[m] = L[swz<G>(r, c)];
      }
    }
    contract16<R, false, TETRA>(x, RD::opA[rd], RD::opB[rd], A);
    if (rd + 1 < RD::n) {
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        int r, c;
        rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
        L[swz<G>(r, c)] = x[m];
      }
      __syncthreads();
    } else if (out) {
#pragma unroll
      for (int m = 0; m < 16; ++m) out[t + ((m >> 2) << (2 * bA)) + ((m & 3) << (2 * bB))] = x[m];
    }
  }
}

}  // namespace qst
