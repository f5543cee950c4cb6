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

// In-place contraction of the g qubit axes held in LDS, for nb consecutive
// blocks of 4^g * J values each.
template <typename R, bool ADJ, bool TETRA>
__device__ __forceinline__ void contract_group(Cx<R>* buf, int g, int J, const ModeMatrix& A, int nb = 1) {
  // every extent is a power of two: divisions are shifts
  const int lgJ = __builtin_ctz(unsigned(J));
  const int lgP = 2 * (g - 1) + lgJ;  // groups of four per block
  const int groups = nb << lgP;
  for (int b = 0; b < g; ++b) {
    for (int h0 = threadIdx.x; h0 < groups; h0 += blockDim.x) {
      Cx<R>* blk = buf + ((h0 >> lgP) << (lgP + 2));
      const int h = h0 & ((1 << lgP) - 1);
      const int j = h & (J - 1);
      const int rc = h >> lgJ;
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
      for (int m = 0; m < 4; ++m) x[m] = blk[pos[m]];
      apply4<R, ADJ, TETRA>(x, A);
#pragma unroll
      for (int m = 0; m < 4; ++m) blk[pos[m]] = x[m];
    }
    __syncthreads();
  }
}

// Block bid of a pass: its (Rhi, Chi) tile pair and first outcome chunk.
// Pair indices below 2^22 use a single-precision square root (exact after
// the integer corrections), larger ones the general decode.
// lgC = log2 of the chunks per pair, lgJ = log2 J.
__device__ __forceinline__ void block_coords(int64_t bid, int lgC, int lgJ, int& Rhi, int& Chi, int64_t& kd0) {
  const int64_t pr = bid >> lgC;
  if (pr < (int64_t(1) << 22)) {
    const int q = int(pr);
    int r = int((sqrtf(8.0f * float(q) + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > q) --r;
    while ((r + 1) * (r + 2) / 2 <= q) ++r;
    Rhi = r;
    Chi = q - r * (r + 1) / 2;
  } else {
    tri_decode(pr, Rhi, Chi);
  }
  kd0 = (bid & ((int64_t(1) << lgC) - 1)) << lgJ;
}

// Element loops load kLoadBatch values per thread before storing any, so
// that that many memory round trips overlap (one workgroup alone on a CU
// has nothing else to hide them behind).  The loads are unconditional: an
// index past the end is clamped to the last element and its value dropped
// (a load under a branch is waited for where the branch rejoins).
constexpr int kLoadBatch = 4;

// Coordinates of the blocks an element loop visits, in increasing order.
// UNI (4^g J a multiple of 64, so the 64 lanes of a wave are in the same
// block in every iteration): a per-wave cursor in scalar registers steps
// through the blocks -- chunks of a pair, then the pairs (Rhi, Chi) row by
// row over the lower triangle -- without division or square root.
// Otherwise each element decodes its own block.
template <bool UNI>
struct BlockWalk {
  int64_t b, ch;
  int R, C, lgC, lgJ;
  __device__ __forceinline__ BlockWalk(int64_t bid0, int lgC_, int lgJ_) : b(bid0), ch(0), R(0), C(0), lgC(lgC_), lgJ(lgJ_) {
    if constexpr (UNI) {
      int64_t kd0;
      block_coords(bid0, lgC, lgJ, R, C, kd0);
      ch = kd0 >> lgJ;
    }
  }
  // Block of element e0 (given relative to the call's first block bid0).
  __device__ __forceinline__ void at(int64_t bid0, int blk, int& Rhi, int& Chi, int64_t& kd0) {
    if constexpr (UNI) {
      const int64_t bid = bid0 + __builtin_amdgcn_readfirstlane(blk);
      while (b < bid) {
        ++b;
        if (++ch == (int64_t(1) << lgC)) {
          ch = 0;
          if (C < R) {
            ++C;
          } else {
            ++R;
            C = 0;
          }
        }
      }
      Rhi = R;
      Chi = C;
      kd0 = ch << lgJ;
    } else {
      block_coords(bid0 + blk, lgC, lgJ, Rhi, Chi, kd0);
    }
  }
};

// Forward pass over the blocks bid0 .. bid0 + nb - 1 (see fwd_pass_body).
template <typename R, bool TETRA, bool MATSIDE, bool PSIDE, bool UNI, int LB>
__device__ __forceinline__ void fwd_pass_impl(const PassArgs& a, const ModeMatrix& A, int64_t bid0, Cx<R>* buf, int nb) {
  const int g = a.g, J = a.J, U = a.U, n = a.n;
  const int Up = U - g;
  const int64_t kd = int64_t(1) << (2 * (n - U));
  const int tile = 1 << (2 * g);
  const int elems = tile * J;
  const int gm = (1 << g) - 1;
  // every extent is a power of two: divisions are shifts
  const int lgJ = __builtin_ctz(unsigned(J));
  const int lgE = 2 * g + lgJ;
  const int lgC = 2 * (n - U) - lgJ;  // chunks of J outcome digits per pair

  const Cx<R>* in = static_cast<const Cx<R>*>(a.in);
  const int total = elems * nb;
  BlockWalk<UNI> walk(bid0, lgC, lgJ);
  for (int base = 0; base < total; base += LB * int(blockDim.x)) {
    R vr[LB], vi[LB];  // scalar arrays stay in registers
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int e0 = base + u * int(blockDim.x) + int(threadIdx.x);
      const int ec = e0 < total ? e0 : total - 1;
      const int e = ec & (elems - 1);
      int Rhi, Chi;
      int64_t kd0;
      walk.at(bid0, ec >> lgE, Rhi, Chi, kd0);
      const int j = e & (J - 1);
      const int rc = e >> lgJ;
      const int c = rc & gm, r = rc >> g;
      const int64_t Rr = (int64_t(Rhi) << g) | r, Cr = (int64_t(Chi) << g) | c;
      const bool mirror = Rr < Cr;
      const int64_t rr = mirror ? Cr : Rr, cc = mirror ? Rr : Cr;
      const Cx<R> v = MATSIDE ? in[rr * a.ld + cc] : in[((rr << U) | cc) * kd + kd0 + j];
      vr[u] = v.re;
      vi[u] = mirror ? -v.im : v.im;
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int e0 = base + u * int(blockDim.x) + int(threadIdx.x);
      if (e0 < total) buf[e0] = Cx<R>{vr[u], vi[u]};
    }
  }
  __syncthreads();
  contract_group<R, false, TETRA>(buf, g, J, A, nb);

  BlockWalk<UNI> walk2(bid0, lgC, lgJ);
  for (int e0 = threadIdx.x; e0 < elems * nb; e0 += blockDim.x) {
    const int e = e0 & (elems - 1);
    int Rhi, Chi;
    int64_t kd0;
    walk2.at(bid0, e0 >> lgE, Rhi, Chi, kd0);
    const int j = e & (J - 1);
    const int kg = e >> lgJ;
    int r, c;
    deinterleave(kg, g, r, c);
    const Cx<R> v = buf[(e0 - e) + ((r << g) | c) * J + j];
    if constexpr (PSIDE) {
      static_cast<R*>(a.out)[int64_t(kg) * kd + kd0 + j] = v.re;
    } else {
      const int64_t base = ((int64_t(Rhi) << Up) | Chi) * (kd * tile);
      static_cast<Cx<R>*>(a.out)[base + int64_t(kg) * kd + kd0 + j] = v;
    }
  }
}

// Adjoint pass over the blocks bid0 .. bid0 + nb - 1 (see adj_pass_body).
template <typename R, bool TETRA, bool MATSIDE, bool PSIDE, bool UNI, int LB>
__device__ __forceinline__ void adj_pass_impl(const PassArgs& a, const ModeMatrix& A, int64_t bid0, Cx<R>* buf, int nb) {
  const int g = a.g, J = a.J, U = a.U, n = a.n;
  const int Up = U - g;
  const int64_t kd = int64_t(1) << (2 * (n - U));
  const int tile = 1 << (2 * g);
  const int elems = tile * J;
  const int gm = (1 << g) - 1;
  // every extent is a power of two: divisions are shifts
  const int lgJ = __builtin_ctz(unsigned(J));
  const int lgE = 2 * g + lgJ;
  const int lgC = 2 * (n - U) - lgJ;  // chunks of J outcome digits per pair

  // outcome side in: the cotangent F - f/p of (f, p), or with p == NULL the
  // values of f as given
  double F = 0.0;
  [[maybe_unused]] const bool direct = a.p == nullptr;
  if constexpr (PSIDE) F = direct ? 0.0 : *a.F;
  const int total = elems * nb;
  BlockWalk<UNI> walk(bid0, lgC, lgJ);
  for (int base0 = 0; base0 < total; base0 += LB * int(blockDim.x)) {
    R vr[LB], vi[LB];  // PSIDE: f_k and p_k
    int dst[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int e0 = base0 + u * int(blockDim.x) + int(threadIdx.x);
      const int ec = e0 < total ? e0 : total - 1;
      const int e = ec & (elems - 1);
      int Rhi, Chi;
      int64_t kd0;
      walk.at(bid0, ec >> lgE, Rhi, Chi, kd0);
      const int j = e & (J - 1);
      const int kg = e >> lgJ;
      int r, c;
      deinterleave(kg, g, r, c);
      dst[u] = e0 < total ? (ec - e) + ((r << g) | c) * J + j : -1;
      if constexpr (PSIDE) {
        const int64_t k = int64_t(kg) * kd + kd0 + j;
        vr[u] = static_cast<const R*>(a.f)[k];
        vi[u] = direct ? R(1) : static_cast<const R*>(a.p)[k];
      } else {
        const int64_t base = ((int64_t(Rhi) << Up) | Chi) * (kd * tile);
        const Cx<R> v = static_cast<const Cx<R>*>(a.in)[base + int64_t(kg) * kd + kd0 + j];
        vr[u] = v.re;
        vi[u] = v.im;
      }
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      if (dst[u] < 0) continue;
      // cotangent g'_k = F - f_k / p_k (F where f_k = 0)
      if constexpr (PSIDE) buf[dst[u]] = Cx<R>{direct ? vr[u] : cotangent(F, vr[u], vi[u]), R(0)};
      else buf[dst[u]] = Cx<R>{vr[u], vi[u]};
    }
  }
  __syncthreads();
  contract_group<R, true, TETRA>(buf, g, J, A, nb);

  Cx<R>* out = static_cast<Cx<R>*>(a.out);
  BlockWalk<UNI> walk2(bid0, lgC, lgJ);
  for (int e0 = threadIdx.x; e0 < elems * nb; e0 += blockDim.x) {
    const int e = e0 & (elems - 1);
    int Rhi, Chi;
    int64_t kd0;
    walk2.at(bid0, e0 >> lgE, Rhi, Chi, kd0);
    const int j = e & (J - 1);
    const int rc = e >> lgJ;
    const int c = rc & gm, r = rc >> g;
    const int64_t Rr = (int64_t(Rhi) << g) | r, Cr = (int64_t(Chi) << g) | c;
    if (Rr < Cr) continue;  // upper triangle: the conjugate of a stored entry
    const Cx<R> v = buf[e0];
    if constexpr (MATSIDE) {
      out[Rr * a.ld + Cr] = v;
      if (Rr != Cr) out[Cr * a.ld + Rr] = Cx<R>{v.re, -v.im};
    } else {
      out[((Rr << U) | Cr) * kd + kd0 + j] = v;
    }
  }
}

// One workgroup's share of a forward / adjoint pass: the nb consecutive
// virtual blocks bid0 .. bid0 + nb - 1; buf holds nb * 4^g * J complex
// values of LDS.  The block walk runs on the scalar unit whenever a block
// is a whole number of waves.
// LB: values loaded per thread before any is stored (kLoadBatch, or more
// where the caller's register budget allows).
template <typename R, bool TETRA, bool MATSIDE, bool PSIDE, int LB = kLoadBatch>
__device__ __forceinline__ void fwd_pass_body(const PassArgs& a, const ModeMatrix& A, int64_t bid0, Cx<R>* buf, int nb = 1) {
  if ((((1 << (2 * a.g)) * a.J) & 63) == 0)
    fwd_pass_impl<R, TETRA, MATSIDE, PSIDE, true, LB>(a, A, bid0, buf, nb);
  else
    fwd_pass_impl<R, TETRA, MATSIDE, PSIDE, false, LB>(a, A, bid0, buf, nb);
}
template <typename R, bool TETRA, bool MATSIDE, bool PSIDE, int LB = kLoadBatch>
__device__ __forceinline__ void adj_pass_body(const PassArgs& a, const ModeMatrix& A, int64_t bid0, Cx<R>* buf, int nb = 1) {
  if ((((1 << (2 * a.g)) * a.J) & 63) == 0)
    adj_pass_impl<R, TETRA, MATSIDE, PSIDE, true, LB>(a, A, bid0, buf, nb);
  else
    adj_pass_impl<R, TETRA, MATSIDE, PSIDE, false, LB>(a, A, bid0, buf, nb);
}

}  // namespace generic_pass
}  // namespace qst
