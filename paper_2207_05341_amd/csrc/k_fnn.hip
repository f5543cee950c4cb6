// The mapping network of Sec. 3.1: a 3-layer FNN from the measured
// distribution x (4^N inputs) through H = 2N hidden units with a leaky ReLU
// (negative slope 0.01) to 4^N real outputs y, which fill the Hermitian T
// of Chol_H: y read as a real d x d matrix Y (row major),
//   T_ij = Y_ij + i Y_ji (i > j),  T_ij = Y_ji - i Y_ij (i < j),  T_ii = Y_ii.
// W1 is H x 4^N and W2 is 4^N x H, both row major.  At N = 11 they hold
// 92M values each: every kernel here streams one of them once and is bound
// by HBM bandwidth.
//
// Forward:  fnn_l1_partial -> fnn_hidden (h_pre, h) -> fnn_l2 (y) -> fnn_fill (T)
// Backward: fnn_unfill (dL/dy from dL/dT) -> fnn_l2_back (dW2, db2, partial
//           W2^T dL/dy) -> fnn_dh (dL/dh_pre = db1) -> fnn_l1_back (dW1)
// Sums are in FP64 with fixed orders (bitwise reproducible).
#include <hip/hip_runtime.h>

#include "qst_device.h"
#include "qst_kernels.h"
#include "qst_plan.h"

namespace qst {

namespace {

constexpr double kSlope = 0.01;
constexpr int kH = kFnnMaxHidden;
constexpr int kTB = 32;  // tile side of the fill maps

__device__ __forceinline__ double leaky(double v) { return v > 0.0 ? v : kSlope * v; }

// 16-byte vectors of R (4 floats or 2 doubles).
template <typename R>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float4 type;
  static constexpr int n = 4;
  static __device__ __forceinline__ float at(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
  }
};
template <>
struct Vec16<double> {
  typedef double2 type;
  static constexpr int n = 2;
  static __device__ __forceinline__ double at(const double2& v, int i) { return i == 0 ? v.x : v.y; }
};

// Block b sums W1[h][c] x[c] over its slice of columns, for every hidden
// unit h, in FP64: each thread takes 16-byte column groups (strided by the
// block), loading the group of x and of every W1 row before using any;
// then wave sums, and the four waves in order.
template <typename R>
__global__ __launch_bounds__(256) void fnn_l1_partial_kernel(const R* __restrict__ W1, const R* __restrict__ x,
                                                             int64_t D, int H, double* __restrict__ part) {
  typedef typename Vec16<R>::type V;
  constexpr int VN = Vec16<R>::n;
  __shared__ double wsum[4][kH];
  const int nb = gridDim.x;
  const int64_t G = D / VN;  // column groups
  const int64_t chunk = (G + nb - 1) / nb;
  const int64_t beg = int64_t(blockIdx.x) * chunk;
  const int64_t end = beg + chunk < G ? beg + chunk : G;
  const V* xv = reinterpret_cast<const V*>(x);
  double acc[kH];
#pragma unroll
  for (int h = 0; h < kH; ++h) acc[h] = 0.0;
  for (int64_t gi = beg + threadIdx.x; gi < end; gi += 256) {
    const V xg = xv[gi];
    V wg[kH];
#pragma unroll
    for (int h = 0; h < kH; ++h)
      if (h < H) wg[h] = reinterpret_cast<const V*>(W1 + int64_t(h) * D)[gi];
#pragma unroll
    for (int h = 0; h < kH; ++h) {
      if (h < H) {
#pragma unroll
        for (int i = 0; i < VN; ++i) acc[h] += double(Vec16<R>::at(wg[h], i)) * double(Vec16<R>::at(xg, i));
      }
    }
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int h = 0; h < kH; ++h) {
    const double s = wave_sum(acc[h]);
    if (l == 0) wsum[w][h] = s;
  }
  __syncthreads();
  if (threadIdx.x < H) {
    const int h = threadIdx.x;
    part[int64_t(blockIdx.x) * H + h] = ((wsum[0][h] + wsum[1][h]) + wsum[2][h]) + wsum[3][h];
  }
}

// h_pre = sum of the block partials + b1; h = leaky(h_pre).  Workgroup k
// sums hidden unit k's partials (strided per thread, then block_sum256).
template <typename R>
__global__ __launch_bounds__(256) void fnn_hidden_kernel(const double* __restrict__ part, int nb,
                                                         const R* __restrict__ b1, int H, R* __restrict__ h_pre,
                                                         double* __restrict__ h) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += part[int64_t(b) * H + k];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) {
    const R hp = R(s + double(b1[k]));
    h_pre[k] = hp;
    h[k] = leaky(double(hp));
  }
}

// y_k = sum_h W2[k][h] h_h + b2_k.  A block takes 256 consecutive rows of
// W2 (256 H contiguous values), staged in LDS with coalesced loads; thread t
// then forms output k0 + t from its row.
template <typename R>
__global__ __launch_bounds__(256) void fnn_l2_kernel(const R* __restrict__ W2, const R* __restrict__ b2,
                                                     const double* __restrict__ h, int64_t D, int H, R* __restrict__ y) {
  __shared__ double hs[kH];
  __shared__ __align__(16) R w[256 * kH];
  if (threadIdx.x < H) hs[threadIdx.x] = h[threadIdx.x];
  typedef typename Vec16<R>::type V;
  const int64_t k0 = int64_t(blockIdx.x) * 256;
  const int rows = D - k0 < 256 ? int(D - k0) : 256;
  // rows * H is a whole number of 16-byte vectors (D and H are even and
  // rows is 256 or D, a power of four)
  const int nv = rows * H / Vec16<R>::n;
  const V* src = reinterpret_cast<const V*>(W2 + k0 * H);
  for (int e = threadIdx.x; e < nv; e += 256) reinterpret_cast<V*>(w)[e] = src[e];
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= rows) return;
  double s = double(b2[k0 + t]);
  for (int j = 0; j < H; ++j) s += double(w[t * H + j]) * hs[j];
  y[k0 + t] = R(s);
}

// Tile pair (I, J), I >= J, of the d x d maps, B x B tiles (B = min(d, 32)):
// both tiles of the input are staged in LDS before either output tile is
// written.
// fill: T from Y.
template <typename R>
__global__ __launch_bounds__(256) void fnn_fill_kernel(const R* __restrict__ Y, int lgB, int d, Cx<R>* __restrict__ T,
                                                       int64_t ldT) {
  __shared__ R a[kTB][kTB + 1], b[kTB][kTB + 1];
  const int B = 1 << lgB;
  int I, J;
  tri_decode(blockIdx.x, I, J);
  const int64_t r0 = int64_t(I) << lgB, c0 = int64_t(J) << lgB;
  for (int e = threadIdx.x; e < B * B; e += 256) {
    const int r = e >> lgB, c = e & (B - 1);
    a[r][c] = Y[(r0 + r) * d + c0 + c];
    b[r][c] = Y[(c0 + r) * d + r0 + c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < B * B; e += 256) {
    const int r = e >> lgB, c = e & (B - 1);
    // element (i, j) = (r0 + r, c0 + c): Y_ij = a[r][c], Y_ji = b[c][r]
    const int64_t i = r0 + r, j = c0 + c;
    const R yij = a[r][c], yji = b[c][r];
    T[i * ldT + j] = i > j ? Cx<R>{yij, yji} : (i < j ? Cx<R>{yji, -yij} : Cx<R>{yij, R(0)});
    if (I != J) {  // element (j', i') = (c0 + r, r0 + c): Y = b[r][c], its mirror a[c][r]; row < column there
      T[(c0 + r) * ldT + r0 + c] = Cx<R>{a[c][r], -b[r][c]};
    }
  }
}

// unfill (the adjoint of fill): dL/dy from G = dL/dT,
//   gy_ij = Re G_ij + Re G_ji (i > j),  Im G_ji - Im G_ij (i < j),  Re G_ii.
template <typename R>
__global__ __launch_bounds__(256) void fnn_unfill_kernel(const Cx<R>* __restrict__ G, int64_t ldG, int lgB, int d,
                                                         R* __restrict__ gy) {
  __shared__ Cx<R> a[kTB][kTB + 1], b[kTB][kTB + 1];
  const int B = 1 << lgB;
  int I, J;
  tri_decode(blockIdx.x, I, J);
  const int64_t r0 = int64_t(I) << lgB, c0 = int64_t(J) << lgB;
  for (int e = threadIdx.x; e < B * B; e += 256) {
    const int r = e >> lgB, c = e & (B - 1);
    a[r][c] = G[(r0 + r) * ldG + c0 + c];
    b[r][c] = G[(c0 + r) * ldG + r0 + c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < B * B; e += 256) {
    const int r = e >> lgB, c = e & (B - 1);
    const int64_t i = r0 + r, j = c0 + c;
    const Cx<R> gij = a[r][c], gji = b[c][r];
    gy[i * d + j] = i > j ? gij.re + gji.re : (i < j ? gji.im - gij.im : gij.re);
    if (I != J) {  // (c0 + r, r0 + c), row < column: Im G_(col,row) - Im G_(row,col)
      gy[(c0 + r) * d + r0 + c] = a[c][r].im - b[r][c].im;
    }
  }
}

// dW2[k][h] = gy_k h_h, db2_k = gy_k, and per block the partial sums of
// W2[k][h] gy_k (wave sums, waves in order).  Block b takes the chunks of
// 256 consecutive rows b, b + nb, ...: each chunk of W2 is staged in LDS
// with coalesced loads, thread t reads its row, overwrites it with the row
// of dW2, and the chunk is stored with coalesced stores.
template <typename R>
__global__ __launch_bounds__(256) void fnn_l2_back_kernel(const R* __restrict__ W2, const R* __restrict__ gy,
                                                          const double* __restrict__ h, int64_t D, int H,
                                                          R* __restrict__ dW2, R* __restrict__ db2,
                                                          double* __restrict__ part) {
  __shared__ double hs[kH];
  __shared__ double wsum[4][kH];
  __shared__ __align__(16) R w[256 * kH];
  if (threadIdx.x < H) hs[threadIdx.x] = h[threadIdx.x];
  const int t = threadIdx.x;
  double acc[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) acc[j] = 0.0;
  for (int64_t k0 = int64_t(blockIdx.x) * 256; k0 < D; k0 += int64_t(gridDim.x) * 256) {
    const int rows = D - k0 < 256 ? int(D - k0) : 256;
    const int nv = rows * H / Vec16<R>::n;
    __syncthreads();  // the previous chunk is stored
    for (int e = t; e < nv; e += 256)
      reinterpret_cast<typename Vec16<R>::type*>(w)[e] = reinterpret_cast<const typename Vec16<R>::type*>(W2 + k0 * H)[e];
    __syncthreads();
    if (t < rows) {
      const R g = gy[k0 + t];
      const double gd = double(g);
      db2[k0 + t] = g;
#pragma unroll
      for (int j = 0; j < kH; ++j) {
        if (j < H) {
          acc[j] += double(w[t * H + j]) * gd;
          w[t * H + j] = R(gd * hs[j]);
        }
      }
    }
    __syncthreads();
    for (int e = t; e < nv; e += 256)
      reinterpret_cast<typename Vec16<R>::type*>(dW2 + k0 * H)[e] = reinterpret_cast<const typename Vec16<R>::type*>(w)[e];
  }
  const int wv = t >> 6, l = t & 63;
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    const double sum = wave_sum(acc[j]);
    if (l == 0) wsum[wv][j] = sum;
  }
  __syncthreads();
  if (t < H) part[int64_t(blockIdx.x) * H + t] = ((wsum[0][t] + wsum[1][t]) + wsum[2][t]) + wsum[3][t];
}

// h = leaky(h_pre) (the backward's copy of the hidden activations).
template <typename R>
__global__ __launch_bounds__(64) void fnn_leaky_kernel(const R* __restrict__ h_pre, int H, double* __restrict__ h) {
  const int k = threadIdx.x;
  if (k < H) h[k] = leaky(double(h_pre[k]));
}

// dL/dh_pre = (sum of the partials) * leaky'(h_pre) = db1; workgroup k
// for hidden unit k, as fnn_hidden_kernel.
template <typename R>
__global__ __launch_bounds__(256) void fnn_dh_kernel(const double* __restrict__ part, int nb,
                                                     const R* __restrict__ h_pre, int H, double* __restrict__ dh,
                                                     R* __restrict__ db1) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += part[int64_t(b) * H + k];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) {
    const double v = s * (double(h_pre[k]) > 0.0 ? 1.0 : kSlope);
    dh[k] = v;
    db1[k] = R(v);
  }
}

// dW1[h][c] = dL/dh_pre_h x_c.
template <typename R>
__global__ __launch_bounds__(256) void fnn_l1_back_kernel(const R* __restrict__ x, const double* __restrict__ dh,
                                                          int64_t D, int H, R* __restrict__ dW1) {
  __shared__ double ds[kH];
  if (threadIdx.x < H) ds[threadIdx.x] = dh[threadIdx.x];
  __syncthreads();
  const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (c >= D) return;
  const double xv = double(x[c]);
  for (int j = 0; j < H; ++j) dW1[int64_t(j) * D + c] = R(ds[j] * xv);
}

// One Rprop step per entry (iRprop-): s = sign(g) sign(prev); the step
// grows by eta+ where s > 0, shrinks by eta- where s < 0 (and that entry's
// gradient is dropped), and is clamped; param moves by -sign(g') step.
template <typename R>
__global__ __launch_bounds__(256) void rprop_kernel(R* __restrict__ w, const R* __restrict__ g, R* __restrict__ prev,
                                                    R* __restrict__ step, int64_t count, R eta_minus, R eta_plus,
                                                    R smin, R smax) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += int64_t(gridDim.x) * 256) {
    const R gi = g[i], pi = prev[i];
    const int s = ((gi > R(0)) - (gi < R(0))) * ((pi > R(0)) - (pi < R(0)));
    R st = step[i];
    if (s > 0) st = st * eta_plus;
    else if (s < 0) st = st * eta_minus;
    st = st < smin ? smin : (st > smax ? smax : st);
    const R gg = s < 0 ? R(0) : gi;
    const R sg = R((gg > R(0)) - (gg < R(0)));
    w[i] = w[i] - sg * st;
    prev[i] = gg;
    step[i] = st;
  }
}

template <typename R>
hipError_t run_fnn_forward(int n, const void* W1, const void* b1, const void* W2, const void* b2, const void* x,
                           void* h_pre, void* T, int64_t ldT, void* ws, hipStream_t s) {
  const FnnLayout L = fnn_layout(n, sizeof(R));
  unsigned char* base = static_cast<unsigned char*>(ws);
  double* part = reinterpret_cast<double*>(base + L.part);
  double* h = reinterpret_cast<double*>(base + L.hvec);
  R* y = reinterpret_cast<R*>(base + L.yvec);
  const int H = 2 * n, d = 1 << n;
  const int64_t D = int64_t(1) << (2 * n);
  fnn_l1_partial_kernel<R><<<kFnnBlocks, 256, 0, s>>>(static_cast<const R*>(W1), static_cast<const R*>(x), D, H, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fnn_hidden_kernel<R><<<unsigned(H), 256, 0, s>>>(part, kFnnBlocks, static_cast<const R*>(b1), H,
                                                    static_cast<R*>(h_pre), h);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  fnn_l2_kernel<R><<<unsigned((D + 255) / 256), 256, 0, s>>>(static_cast<const R*>(W2), static_cast<const R*>(b2), h,
                                                             D, H, y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int lgB = n < 5 ? n : 5;
  const int64_t m = int64_t(1) << (n - lgB);
  fnn_fill_kernel<R><<<unsigned(m * (m + 1) / 2), 256, 0, s>>>(y, lgB, d, static_cast<Cx<R>*>(T), ldT);
  return hipGetLastError();
}

template <typename R>
hipError_t run_fnn_backward(int n, const void* W2, const void* x, const void* h_pre, const void* G, int64_t ldG,
                            void* dW1, void* db1, void* dW2, void* db2, void* ws, hipStream_t s) {
  const FnnLayout L = fnn_layout(n, sizeof(R));
  unsigned char* base = static_cast<unsigned char*>(ws);
  double* part = reinterpret_cast<double*>(base + L.part);
  double* h = reinterpret_cast<double*>(base + L.hvec);
  double* dh = reinterpret_cast<double*>(base + L.dhvec);
  R* gy = reinterpret_cast<R*>(base + L.yvec);
  const int H = 2 * n, d = 1 << n;
  const int64_t D = int64_t(1) << (2 * n);
  const R* hp = static_cast<const R*>(h_pre);
  // h = leaky(h_pre) again (H values) for dW2
  fnn_leaky_kernel<R><<<1, 64, 0, s>>>(hp, H, h);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int lgB = n < 5 ? n : 5;
  const int64_t m = int64_t(1) << (n - lgB);
  fnn_unfill_kernel<R><<<unsigned(m * (m + 1) / 2), 256, 0, s>>>(static_cast<const Cx<R>*>(G), ldG, lgB, d, gy);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  fnn_l2_back_kernel<R><<<kFnnBlocks, 256, 0, s>>>(static_cast<const R*>(W2), gy, h, D, H, static_cast<R*>(dW2),
                                                  static_cast<R*>(db2), part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  fnn_dh_kernel<R><<<unsigned(H), 256, 0, s>>>(part, kFnnBlocks, hp, H, dh, static_cast<R*>(db1));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  fnn_l1_back_kernel<R><<<unsigned((D + 255) / 256), 256, 0, s>>>(static_cast<const R*>(x), dh, D, H,
                                                                  static_cast<R*>(dW1));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fnn_forward(qst_prec prec, int n, const void* W1, const void* b1, const void* W2, const void* b2,
                              const void* x, void* h_pre, void* T, int64_t ldT, void* ws, hipStream_t s) {
  if (prec == QST_F64) return run_fnn_forward<double>(n, W1, b1, W2, b2, x, h_pre, T, ldT, ws, s);
  return run_fnn_forward<float>(n, W1, b1, W2, b2, x, h_pre, T, ldT, ws, s);
}

hipError_t launch_rprop(qst_prec prec, int64_t count, void* w, const void* g, void* prev, void* step, double eta_minus,
                        double eta_plus, double smin, double smax, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const int64_t blocks = (count + 255) / 256;
  const unsigned grid = unsigned(blocks < 8192 ? blocks : 8192);
  if (prec == QST_F64)
    rprop_kernel<double><<<grid, 256, 0, s>>>(static_cast<double*>(w), static_cast<const double*>(g),
                                              static_cast<double*>(prev), static_cast<double*>(step), count, eta_minus,
                                              eta_plus, smin, smax);
  else
    rprop_kernel<float><<<grid, 256, 0, s>>>(static_cast<float*>(w), static_cast<const float*>(g),
                                             static_cast<float*>(prev), static_cast<float*>(step), count,
                                             float(eta_minus), float(eta_plus), float(smin), float(smax));
  return hipGetLastError();
}

hipError_t launch_fnn_backward(qst_prec prec, int n, const void* W2, const void* x, const void* h_pre, const void* G,
                               int64_t ldG, void* dW1, void* db1, void* dW2, void* db2, void* ws, hipStream_t s) {
  if (prec == QST_F64) return run_fnn_backward<double>(n, W2, x, h_pre, G, ldG, dW1, db1, dW2, db2, ws, s);
  return run_fnn_backward<float>(n, W2, x, h_pre, G, ldG, dW1, db1, dW2, db2, ws, s);
}

}  // namespace qst
