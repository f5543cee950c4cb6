// Generic product-POVM pass bodies (any group size g and chunk J, runtime),
// as device functions taking a virtual block index: used by the per-pass
// kernels of k_povm.hip and by the batched persistent kernel.  See
// k_povm.hip for the data view and the Hermitian storage rule.
#pragma once

#include "qst_povm_ops.h"

namespace qst {
namespace generic_pass {

// Insert a zero bit at position b of x.
__device__ __forceinline__ int ins0(int x, int b) { return ((x >> b) << (b + 1)) | (x & ((1 << b) - 1)); }

// Bits of r and c interleaved, r above c: k = sum_b (2 r_b + c_b) 4^b.
__device__ __forceinline__ int interleave(int r, int c, int g) {
  int k = 0;
  for (int b = 0; b < g; ++b) k |= (((r >> b) & 1) << (2 * b + 1)) | (((c >> b) & 1) << (2 * b));
  return k;
}
__device__ __forceinline__ void deinterleave(int k, int g, int& r, int& c) {
  r = 0;
  c = 0;
  for (int b = 0; b < g; ++b) {
    r |= ((k >> (2 * b + 1)) & 1) << b;
    c |= ((k >> (2 * b)) & 1) << b;
  }
}

// In-place contraction of the g qubit axes held in LDS.
template <typename R, bool ADJ, bool TETRA>
__device__ __forceinline__ void contract_group(Cx<R>* buf, int g, int J, const ModeMatrix& A) {
  const int groups = (1 << (2 * (g - 1))) * J;
  for (int b = 0; b < g; ++b) {
    for (int h = threadIdx.x; h < groups; h += blockDim.x) {
      const int j = h % J;
      const int rc = h / J;
      const int c0 = ins0(rc & ((1 << (g - 1)) - 1), b);
      const int r0 = ins0(rc >> (g - 1), b);
      int pos[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int r = r0 | ((m >> 1) << b), c = c0 | ((m & 1) << b);
        pos[m] = ((r << g) | c) * J + j;
      }
      Cx<R> x[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) x[m] = buf[pos[m]];
      apply4<R, ADJ, TETRA>(x, A);
#pragma unroll
      for (int m = 0; m < 4; ++m) buf[pos[m]] = x[m];
    }
    __syncthreads();
  }
}

// One workgroup's share (virtual block bid) of a forward pass; buf holds
// 4^g * J complex values of LDS.
template <typename R, bool TETRA, bool MATSIDE, bool PSIDE>
__device__ void fwd_pass_body(const PassArgs& a, const ModeMatrix& A, int64_t bid, Cx<R>* buf) {
  const int g = a.g, J = a.J, U = a.U, n = a.n;
  const int Up = U - g;
  const int64_t kd = int64_t(1) << (2 * (n - U));
  const int64_t nchunks = kd / J;
  const int64_t ch = bid % nchunks;
  int Rhi, Chi;
  tri_decode(bid / nchunks, Rhi, Chi);
  const int64_t kd0 = ch * J;
  const int tile = 1 << (2 * g);
  const int elems = tile * J;
  const int gm = (1 << g) - 1;

  const Cx<R>* in = static_cast<const Cx<R>*>(a.in);
  for (int e = threadIdx.x; e < elems; e += blockDim.x) {
    const int j = e % J;
    const int rc = e / J;
    const int c = rc & gm, r = rc >> g;
    const int64_t Rr = (int64_t(Rhi) << g) | r, Cr = (int64_t(Chi) << g) | c;
    const bool mirror = Rr < Cr;
    const int64_t rr = mirror ? Cr : Rr, cc = mirror ? Rr : Cr;
    Cx<R> v;
    if constexpr (MATSIDE) {
      v = in[rr * a.ld + cc];
    } else {
      v = in[((rr << U) | cc) * kd + kd0 + j];
    }
    if (mirror) v.im = -v.im;
    buf[e] = v;
  }
  __syncthreads();
  contract_group<R, false, TETRA>(buf, g, J, A);

  for (int e = threadIdx.x; e < elems; e += blockDim.x) {
    const int j = e % J;
    const int kg = e / J;
    int r, c;
    deinterleave(kg, g, r, c);
    const Cx<R> v = buf[((r << g) | c) * J + j];
    if constexpr (PSIDE) {
      static_cast<R*>(a.out)[int64_t(kg) * kd + kd0 + j] = v.re;
    } else {
      const int64_t base = ((int64_t(Rhi) << Up) | Chi) * (kd * tile);
      static_cast<Cx<R>*>(a.out)[base + int64_t(kg) * kd + kd0 + j] = v;
    }
  }
}

// One workgroup's share (virtual block bid) of an adjoint pass.
template <typename R, bool TETRA, bool MATSIDE, bool PSIDE>
__device__ void adj_pass_body(const PassArgs& a, const ModeMatrix& A, int64_t bid, Cx<R>* buf) {
  const int g = a.g, J = a.J, U = a.U, n = a.n;
  const int Up = U - g;
  const int64_t kd = int64_t(1) << (2 * (n - U));
  const int64_t nchunks = kd / J;
  const int64_t ch = bid % nchunks;
  int Rhi, Chi;
  tri_decode(bid / nchunks, Rhi, Chi);
  const int64_t kd0 = ch * J;
  const int tile = 1 << (2 * g);
  const int elems = tile * J;
  const int gm = (1 << g) - 1;

  double F = 0.0;
  if constexpr (PSIDE) F = *a.F;
  for (int e = threadIdx.x; e < elems; e += blockDim.x) {
    const int j = e % J;
    const int kg = e / J;
    int r, c;
    deinterleave(kg, g, r, c);
    Cx<R> v;
    if constexpr (PSIDE) {
      // cotangent g'_k = F - f_k / p_k (F where f_k = 0)
      const int64_t k = int64_t(kg) * kd + kd0 + j;
      v = {cotangent(F, static_cast<const R*>(a.f)[k], static_cast<const R*>(a.p)[k]), R(0)};
    } else {
      const int64_t base = ((int64_t(Rhi) << Up) | Chi) * (kd * tile);
      v = static_cast<const Cx<R>*>(a.in)[base + int64_t(kg) * kd + kd0 + j];
    }
    buf[((r << g) | c) * J + j] = v;
  }
  __syncthreads();
  contract_group<R, true, TETRA>(buf, g, J, A);

  Cx<R>* out = static_cast<Cx<R>*>(a.out);
  for (int e = threadIdx.x; e < elems; e += blockDim.x) {
    const int j = e % J;
    const int rc = e / J;
    const int c = rc & gm, r = rc >> g;
    const int64_t Rr = (int64_t(Rhi) << g) | r, Cr = (int64_t(Chi) << g) | c;
    if (Rr < Cr) continue;  // upper triangle: the conjugate of a stored entry
    const Cx<R> v = buf[e];
    if constexpr (MATSIDE) {
      out[Rr * a.ld + Cr] = v;
      if (Rr != Cr) out[Cr * a.ld + Rr] = Cx<R>{v.re, -v.im};
    } else {
      out[((Rr << U) | Cr) * kd + kd0 + j] = v;
    }
  }
}

}  // namespace generic_pass
}  // namespace qst
