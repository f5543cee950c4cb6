// Per-qubit 4 x 4 mode contractions of the product-POVM map and the pass
// arguments shared by the generic and the specialised pass kernels.
//
// One qubit, forward: y[a] = sum_m W[a][m] x[m] with m = 2 r + c and
// W[a][2r+c] = (M_a)_{c,r}, so that sum_m W[a][m] X_m = Tr(M_a X) (Born rule,
// Sec. 2.1).  Adjoint: x[m] = sum_a V[m][a] g[a], V[m][a] = (M_a)_{r,c}.
//
// For the tetrahedral POVM of Sec. 4.1, M_a = (I + s_a.sigma)/4 with
// s_a = t(+-1, +-1, +-1), t = 1/sqrt(3): Tr(M_a X) = (u0 + s_a . (u1,u2,u3))/4
// with the Pauli coordinates u = (x0+x3, x1+x2, i(x1-x2), x0-x3), and the
// four sign patterns of s_a form a 4 x 4 Hadamard matrix; the fast forms below
// use 12 complex additions and 4 real scalings per 4 values.
#pragma once

#include "qst.h"
#include "qst_device.h"

namespace qst {

struct ModeMatrix {
  double a[32];  // 4 x 4 complex, row-major (re, im)
};

struct PassArgs {
  const void* in;       // forward: rho or intermediate; adjoint: intermediate
  void* out;            // forward: intermediate or p; adjoint: intermediate or G'
  const void* p;        // adjoint, last pass: probabilities
  const void* f;        // adjoint / fused last pass: frequencies
  const double* F;      // adjoint, last pass: F = sum f
  const double* Fpart;  // fused last pass: kReduceBlocks FP64 partial sums of F = sum f
  double* part;         // fused last pass: FP64 partials [4][blocks] (L, F_c terms, bad0, bad1)
  const void* pt;       // fused last pass: target distribution of F_c, or NULL
  void* gplanes;        // adjoint pass 0 of the combined call: G' as split operand planes instead of G'
  int64_t ld;           // row stride of the matrix (rho or G')
  int n, U, g, J;
};

template <typename R>
__device__ __forceinline__ Cx<R> cadd(Cx<R> x, Cx<R> y) { return {x.re + y.re, x.im + y.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> csub(Cx<R> x, Cx<R> y) { return {x.re - y.re, x.im - y.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> cscale(Cx<R> x, R s) { return {x.re * s, x.im * s}; }
template <typename R>
__device__ __forceinline__ Cx<R> cmuli(Cx<R> x) { return {-x.im, x.re}; }  // i * x

template <typename R>
__device__ __forceinline__ void tetra_fwd(Cx<R> x[4]) {
  const R q = R(0.25), t4 = R(0.14433756729740644113);  // 1/4, 1/(4 sqrt 3)
  const Cx<R> a = cscale(cadd(x[0], x[3]), q);
  const Cx<R> b = cscale(cadd(x[1], x[2]), t4);
  const Cx<R> c = cscale(cmuli(csub(x[1], x[2])), t4);
  const Cx<R> e = cscale(csub(x[0], x[3]), t4);
  const Cx<R> P = cadd(b, c), Q = csub(b, c);
  const Cx<R> ape = cadd(a, e), ame = csub(a, e);
  x[0] = cadd(ape, P);  // s_0 = t( 1,  1,  1)
  x[1] = csub(ape, P);  // s_1 = t(-1, -1,  1)
  x[2] = csub(ame, Q);  // s_2 = t(-1,  1, -1)
  x[3] = cadd(ame, Q);  // s_3 = t( 1, -1, -1)
}

template <typename R>
__device__ __forceinline__ void tetra_adj(Cx<R> x[4]) {
  const R q = R(0.25), t4 = R(0.14433756729740644113);
  const Cx<R> s01 = cadd(x[0], x[1]), d01 = csub(x[0], x[1]);
  const Cx<R> s23 = cadd(x[2], x[3]), d23 = csub(x[2], x[3]);
  const Cx<R> v0 = cscale(cadd(s01, s23), q);   // (g0+g1+g2+g3)/4
  const Cx<R> v1 = cscale(csub(d01, d23), t4);  // t(g0-g1-g2+g3)/4: sigma_x weight
  const Cx<R> v2 = cscale(cadd(d01, d23), t4);  // t(g0-g1+g2-g3)/4: sigma_y weight
  const Cx<R> v3 = cscale(csub(s01, s23), t4);  // t(g0+g1-g2-g3)/4: sigma_z weight
  const Cx<R> iv2 = cmuli(v2);
  x[0] = cadd(v0, v3);
  x[1] = csub(v1, iv2);
  x[2] = cadd(v1, iv2);
  x[3] = csub(v0, v3);
}

template <typename R>
__device__ __forceinline__ void generic4(Cx<R> x[4], const ModeMatrix& A) {
  Cx<R> y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    R re = 0, im = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const R ar = R(A.a[2 * (4 * i + j)]), ai = R(A.a[2 * (4 * i + j) + 1]);
      re += ar * x[j].re - ai * x[j].im;
      im += ar * x[j].im + ai * x[j].re;
    }
    y[i] = {re, im};
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] = y[i];
}

template <typename R, bool ADJ, bool TETRA>
__device__ __forceinline__ void apply4(Cx<R> x[4], const ModeMatrix& A) {
  if constexpr (TETRA) {
    if constexpr (ADJ) tetra_adj(x);
    else tetra_fwd(x);
  } else {
    generic4(x, A);
  }
}

// Launches a specialised pass kernel when one covers (g, J, side); returns
// false (launching nothing) otherwise.
bool launch_pass_fast(bool adjoint, qst_prec prec, bool tetra, const PassArgs& a, const ModeMatrix& A,
                      bool matside, bool pside, int64_t blocks, hipStream_t s, hipError_t* err);

// Fused last pass of qst_likelihood (forward + NLL terms + cotangent
// g' = F - f/p + adjoint), in place on a.out; partial sums to a.part.  Returns false (and
// launches nothing) when no specialised form covers (g, J).
bool launch_fused_fast(qst_prec prec, bool tetra, const PassArgs& a, const ModeMatrix& Af,
                       const ModeMatrix& Aa, int64_t blocks, hipStream_t s, hipError_t* err);

}  // namespace qst
