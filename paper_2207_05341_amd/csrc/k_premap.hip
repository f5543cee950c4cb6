// Pre-maps of the paper's state-map modes, applied to the network output T
// before the state map (and, being self-adjoint, to dL/dT' after it):
//
//  * Hermitian part (X + X^dagger) / 2: with it, rho = T' T'^dagger / Tr is
//    Chol_H, the unified map of Sec. 3.2 (Eq. unified_DP; Eq. abs_P at
//    P = 2); the Hermitian part is the paper's remark on non-Hermitian
//    matrices in Sec. 2.2.2.
//  * Lower triangle (row >= column, the rest zero): Chol_Delta, the
//    decomposition of Sec. 2.2.1 (Eq. T_matrix) with a lower-triangular T.
//
// Both are HBM-bound: one read and one write of d^2 complex values.
#include <hip/hip_runtime.h>

#include "qst_device.h"
#include "qst_kernels.h"

namespace qst {

namespace {

constexpr int kPB = 32;  // tile side of the Hermitian part

// Hermitian part over the tile pairs (I, J), I >= J, of B x B tiles
// (B = min(d, 32)); workgroup b owns tiles (I, J) and (J, I) of the lower
// triangle index b.  Both tiles are read into LDS before either is written,
// so Y may equal X.  Y_IJ[r][c] = (X_IJ[r][c] + conj(X_JI[c][r])) / 2 and
// Y_JI = Y_IJ^dagger (computed from the same two tiles).
template <typename R>
__global__ __launch_bounds__(256) void hermitian_part_kernel(const Cx<R>* X, int64_t ldx, int lgB, Cx<R>* Y,
                                                             int64_t ldy) {
  __shared__ Cx<R> a[kPB][kPB + 1], b[kPB][kPB + 1];
  const int B = 1 << lgB;
  int I, J;
  tri_decode(blockIdx.x, I, J);
  const int64_t r0 = int64_t(I) << lgB, c0 = int64_t(J) << lgB;
  const int elems = B * B;
#pragma unroll
  for (int q = 0; q < kPB * kPB / 256; ++q) {
    const int e = int(threadIdx.x) + 256 * q;
    if (e < elems) {
      const int r = e >> lgB, c = e & (B - 1);
      a[r][c] = X[(r0 + r) * ldx + c0 + c];
      b[r][c] = X[(c0 + r) * ldx + r0 + c];
    }
  }
  __syncthreads();
  const R h = R(0.5);
#pragma unroll
  for (int q = 0; q < kPB * kPB / 256; ++q) {
    const int e = int(threadIdx.x) + 256 * q;
    if (e < elems) {
      const int r = e >> lgB, c = e & (B - 1);
      const Cx<R> x = a[r][c], y = b[c][r];
      Y[(r0 + r) * ldy + c0 + c] = Cx<R>{(x.re + y.re) * h, (x.im - y.im) * h};
      if (I != J) {
        const Cx<R> u = b[r][c], v = a[c][r];
        Y[(c0 + r) * ldy + r0 + c] = Cx<R>{(u.re + v.re) * h, (u.im - v.im) * h};
      }
    }
  }
}

// Lower triangle: Y[r][c] = X[r][c] for c <= r, 0 above (the strict upper
// part of X is not read).  One element per thread over d x d.
template <typename R>
__global__ __launch_bounds__(256) void lower_part_kernel(const Cx<R>* X, int64_t ldx, int n, Cx<R>* Y, int64_t ldy) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= (int64_t(1) << (2 * n))) return;
  const int64_t r = e >> n, c = e & ((int64_t(1) << n) - 1);
  Y[r * ldy + c] = c <= r ? X[r * ldx + c] : Cx<R>{R(0), R(0)};
}

template <typename R>
hipError_t launch_premap_t(int mode, const void* X, int64_t ldx, void* Y, int64_t ldy, int n, hipStream_t s) {
  const Cx<R>* x = static_cast<const Cx<R>*>(X);
  Cx<R>* y = static_cast<Cx<R>*>(Y);
  if (mode == QST_PREMAP_HERMITIAN) {
    const int lgB = n < 5 ? n : 5;
    const int64_t m = int64_t(1) << (n - lgB);
    hermitian_part_kernel<R><<<unsigned(m * (m + 1) / 2), 256, 0, s>>>(x, ldx, lgB, y, ldy);
  } else {
    const int64_t D = int64_t(1) << (2 * n);
    lower_part_kernel<R><<<unsigned((D + 255) / 256), 256, 0, s>>>(x, ldx, n, y, ldy);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_premap(qst_prec prec, int mode, const void* X, int64_t ldx, void* Y, int64_t ldy, int n,
                         hipStream_t s) {
  if (prec == QST_F64) return launch_premap_t<double>(mode, X, ldx, Y, ldy, n, s);
  return launch_premap_t<float>(mode, X, ldx, Y, ldy, n, s);
}

}  // namespace qst
