// Complex products of the likelihood path on the gfx950 matrix cores.
//
//   state map  rho = T T^dagger / tau       (Eq. T_matrix; Eq. unified_DP)
//   gradient   grad = s (2 / tau) G' T      (adjoint of the state map)
//
// Complex products run as real MFMA products on split real/imaginary
// fragments:  (A B^dagger)_re = Ar Br^T + Ai Bi^T, (A B^dagger)_im =
// Ai Br^T - Ar Bi^T;  (A B)_re = Ar Br - Ai Bi, (A B)_im = Ar Bi + Ai Br.
// T T^dagger is Hermitian, so only lower-triangular 64 x 64 output tiles are
// computed and each off-diagonal tile is also written to its mirror
// position as the conjugate transpose.
//
// Tiles: 256 threads (4 wave64), 64 x 64 complex output per workgroup, each
// wave a 32 x 32 quadrant as 2 x 2 MFMA 16 x 16 blocks.  Operand panels are
// staged through LDS with the next panel prefetched into registers while
// the current one is consumed.
#include "qst_device.h"
#include "qst_kernels.h"

namespace qst {

namespace {

constexpr int BM = 64;     // output tile (complex)
constexpr int BK = 16;     // K panel for fp32/fp64 (complex)
constexpr int PADC = 1;    // LDS row padding (complex elements)
constexpr int BKH = 32;    // K panel for bf16 (complex) = one MFMA K step
constexpr int PADH = 8;    // LDS row padding (bf16 elements)

// ---------------------------------------------------------------------------
// fp32 / fp64 MFMA kernel.  HERK: C = A A^dagger (A = B = T), lower tiles.
// HEMM: C = A B (A = G', B = T), all tiles.
// ---------------------------------------------------------------------------
template <typename R, bool HERK>
__global__ __launch_bounds__(256) void gemm_cx_kernel(const Cx<R>* __restrict__ A, int64_t lda,
                                                      const Cx<R>* __restrict__ B, int64_t ldb,
                                                      Cx<R>* __restrict__ C, int64_t ldc, int d,
                                                      const double* __restrict__ tau_dev,
                                                      const double* __restrict__ upstream_dev) {
  typedef typename Mfma<R>::acc acc_t;
  __shared__ Cx<R> As[BK][BM + PADC];
  __shared__ Cx<R> Bs[BK][BM + PADC];

  const int tiles = d / BM;
  int tr, tc;
  if constexpr (HERK) {
    tri_decode(blockIdx.x, tr, tc);
  } else {
    tr = blockIdx.x / tiles;
    tc = blockIdx.x % tiles;
  }
  const int64_t R0 = int64_t(tr) * BM, C0 = int64_t(tc) * BM;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int li = lane & 15, lk = lane >> 4;

  // global -> register mapping
  const int a_row = t >> 2, a_k = (t & 3) * 4;                  // A panel: 64 rows x 16 k
  const int hb_k = t >> 4, hb_n = (t & 15) * 4;                 // HEMM B panel: 16 k x 64 n
  const Cx<R>* Ap = A + (R0 + a_row) * lda + a_k;
  const Cx<R>* Bp = HERK ? (B + (C0 + a_row) * ldb + a_k) : (B + int64_t(hb_k) * ldb + C0 + hb_n);

  Cx<R> ra[4], rb[4];
  auto load_panel = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) ra[i] = Ap[k0 + i];
    if constexpr (HERK) {
#pragma unroll
      for (int i = 0; i < 4; ++i) rb[i] = Bp[k0 + i];
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) rb[i] = Bp[int64_t(k0) * ldb + i];
    }
  };

  acc_t accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = acc_t{0, 0, 0, 0};
      accI[i][j] = acc_t{0, 0, 0, 0};
    }

  load_panel(0);
  for (int k0 = 0; k0 < d; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) As[a_k + i][a_row] = ra[i];
    if constexpr (HERK) {
#pragma unroll
      for (int i = 0; i < 4; ++i) Bs[a_k + i][a_row] = rb[i];
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) Bs[hb_k][hb_n + i] = rb[i];
    }
    __syncthreads();
    if (k0 + BK < d) load_panel(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + lk;
      Cx<R> a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk][wr * 32 + i * 16 + li];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk][wc * 32 + j * 16 + li];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if constexpr (HERK) {
            accR[i][j] = Mfma<R>::step(a[i].re, b[j].re, accR[i][j]);
            accR[i][j] = Mfma<R>::step(a[i].im, b[j].im, accR[i][j]);
            accI[i][j] = Mfma<R>::step(a[i].im, b[j].re, accI[i][j]);
            accI[i][j] = Mfma<R>::step(-a[i].re, b[j].im, accI[i][j]);
          } else {
            accR[i][j] = Mfma<R>::step(a[i].re, b[j].re, accR[i][j]);
            accR[i][j] = Mfma<R>::step(-a[i].im, b[j].im, accR[i][j]);
            accI[i][j] = Mfma<R>::step(a[i].re, b[j].im, accI[i][j]);
            accI[i][j] = Mfma<R>::step(a[i].im, b[j].re, accI[i][j]);
          }
        }
      }
    }
  }

  double scale;
  if constexpr (HERK) {
    scale = 1.0 / *tau_dev;
  } else {
    scale = 2.0 / *tau_dev;
    if (upstream_dev) scale *= *upstream_dev;
  }
  const R sc = R(scale);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = C0 + wc * 32 + j * 16 + li;
      const int64_t rbase = R0 + wr * 32 + i * 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = rbase + Mfma<R>::row(lk, v);
        C[row * ldc + col] = Cx<R>{accR[i][j][v] * sc, accI[i][j][v] * sc};
        if (HERK && tr != tc) C[col * ldc + row] = Cx<R>{accR[i][j][v] * sc, -accI[i][j][v] * sc};
      }
    }
  }
}

// ---------------------------------------------------------------------------
// bf16 MFMA kernel for T T^dagger: T rounded to bf16 (RNE), fp32 accumulate.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void herk_bf16_kernel(const Cx<float>* __restrict__ T, int64_t ldt,
                                                        Cx<float>* __restrict__ C, int64_t ldc, int d,
                                                        const double* __restrict__ tau_dev) {
  __shared__ __align__(16) uint16_t Ar[BM][BKH + PADH], Ai[BM][BKH + PADH];
  __shared__ __align__(16) uint16_t Br[BM][BKH + PADH], Bi[BM][BKH + PADH];
  int tr, tc;
  tri_decode(blockIdx.x, tr, tc);
  const int64_t R0 = int64_t(tr) * BM, C0 = int64_t(tc) * BM;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int li = lane & 15, lq = lane >> 4;
  const int row = t >> 2, kq = (t & 3) * 8;  // 64 rows x 32 k, 8 complex per thread
  const Cx<float>* Ap = T + (R0 + row) * ldt + kq;
  const Cx<float>* Bp = T + (C0 + row) * ldt + kq;

  Cx<float> ra[8], rb[8];
  auto load_panel = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      ra[i] = Ap[k0 + i];
      rb[i] = Bp[k0 + i];
    }
  };
  f4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = f4{0, 0, 0, 0};
      accI[i][j] = f4{0, 0, 0, 0};
    }
  load_panel(0);
  for (int k0 = 0; k0 < d; k0 += BKH) {
    __syncthreads();
    {
      u16x8 xr, xi, yr, yi;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        xr[i] = bf16_bits(ra[i].re);
        xi[i] = bf16_bits(ra[i].im);
        yr[i] = bf16_bits(rb[i].re);
        yi[i] = bf16_bits(rb[i].im);
      }
      *reinterpret_cast<u16x8*>(&Ar[row][kq]) = xr;
      *reinterpret_cast<u16x8*>(&Ai[row][kq]) = xi;
      *reinterpret_cast<u16x8*>(&Br[row][kq]) = yr;
      *reinterpret_cast<u16x8*>(&Bi[row][kq]) = yi;
    }
    __syncthreads();
    if (k0 + BKH < d) load_panel(k0 + BKH);
    u16x8 a_r[2], a_i[2], b_r[2], b_i[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a_r[i] = *reinterpret_cast<const u16x8*>(&Ar[wr * 32 + i * 16 + li][lq * 8]);
      a_i[i] = *reinterpret_cast<const u16x8*>(&Ai[wr * 32 + i * 16 + li][lq * 8]);
      b_r[i] = *reinterpret_cast<const u16x8*>(&Br[wc * 32 + i * 16 + li][lq * 8]);
      b_i[i] = *reinterpret_cast<const u16x8*>(&Bi[wc * 32 + i * 16 + li][lq * 8]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const u16x8 na = bf16_neg(a_r[i]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        accR[i][j] = mfma_bf16(a_r[i], b_r[j], accR[i][j]);
        accR[i][j] = mfma_bf16(a_i[i], b_i[j], accR[i][j]);
        accI[i][j] = mfma_bf16(a_i[i], b_r[j], accI[i][j]);
        accI[i][j] = mfma_bf16(na, b_i[j], accI[i][j]);
      }
    }
  }
  const float sc = float(1.0 / *tau_dev);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = C0 + wc * 32 + j * 16 + li;
      const int64_t row0 = R0 + wr * 32 + i * 16 + lq * 4;
#pragma unroll
      for (int v = 0; v < 4; ++v) C[(row0 + v) * ldc + col] = Cx<float>{accR[i][j][v] * sc, accI[i][j][v] * sc};
      if (tr != tc) {
        Cx<float>* dst = C + col * ldc + row0;
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[v] = Cx<float>{accR[i][j][v] * sc, -accI[i][j][v] * sc};
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split-bf16 MFMA kernel for grad = s (2/tau) G' T: each operand x = hi + lo
// with hi = bf16(x), lo = bf16(x - hi); the product keeps hi*hi + hi*lo +
// lo*hi (the lo*lo term is below fp32 rounding of the sum).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void hemm_bf16x3_kernel(const Cx<float>* __restrict__ G, int64_t ldg,
                                                          const Cx<float>* __restrict__ T, int64_t ldt,
                                                          Cx<float>* __restrict__ C, int64_t ldc, int d,
                                                          const double* __restrict__ tau_dev,
                                                          const double* __restrict__ upstream_dev) {
  // plane order: re_hi, im_hi, re_lo, im_lo
  __shared__ __align__(16) uint16_t As[4][BM][BKH + PADH];
  __shared__ __align__(16) uint16_t Bt[4][BM][BKH + PADH];  // transposed: [n][k]
  const int tiles = d / BM;
  const int tr = blockIdx.x / tiles, tc = blockIdx.x % tiles;
  const int64_t R0 = int64_t(tr) * BM, C0 = int64_t(tc) * BM;
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int li = lane & 15, lq = lane >> 4;
  const int a_row = t >> 2, a_k = (t & 3) * 8;   // A panel: 64 rows x 32 k
  const int b_k = t >> 3, b_n = (t & 7) * 8;     // B panel: 32 k x 64 n
  const Cx<float>* Ap = G + (R0 + a_row) * ldg + a_k;
  const Cx<float>* Bp = T + int64_t(b_k) * ldt + C0 + b_n;

  Cx<float> ra[8], rb[8];
  auto load_panel = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      ra[i] = Ap[k0 + i];
      rb[i] = Bp[int64_t(k0) * ldt + i];
    }
  };
  f4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = f4{0, 0, 0, 0};
      accI[i][j] = f4{0, 0, 0, 0};
    }
  load_panel(0);
  for (int k0 = 0; k0 < d; k0 += BKH) {
    __syncthreads();
    {
      u16x8 h0, h1, l0, l1;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint16_t hr = bf16_bits(ra[i].re), hi = bf16_bits(ra[i].im);
        h0[i] = hr;
        h1[i] = hi;
        l0[i] = bf16_bits(ra[i].re - __uint_as_float(uint32_t(hr) << 16));
        l1[i] = bf16_bits(ra[i].im - __uint_as_float(uint32_t(hi) << 16));
      }
      *reinterpret_cast<u16x8*>(&As[0][a_row][a_k]) = h0;
      *reinterpret_cast<u16x8*>(&As[1][a_row][a_k]) = h1;
      *reinterpret_cast<u16x8*>(&As[2][a_row][a_k]) = l0;
      *reinterpret_cast<u16x8*>(&As[3][a_row][a_k]) = l1;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint16_t hr = bf16_bits(rb[i].re), hi = bf16_bits(rb[i].im);
        Bt[0][b_n + i][b_k] = hr;
        Bt[1][b_n + i][b_k] = hi;
        Bt[2][b_n + i][b_k] = bf16_bits(rb[i].re - __uint_as_float(uint32_t(hr) << 16));
        Bt[3][b_n + i][b_k] = bf16_bits(rb[i].im - __uint_as_float(uint32_t(hi) << 16));
      }
    }
    __syncthreads();
    if (k0 + BKH < d) load_panel(k0 + BKH);
    u16x8 a[2][4], b[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        a[i][pl] = *reinterpret_cast<const u16x8*>(&As[pl][wr * 32 + i * 16 + li][lq * 8]);
        b[i][pl] = *reinterpret_cast<const u16x8*>(&Bt[pl][wc * 32 + i * 16 + li][lq * 8]);
      }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const u16x8 nih = bf16_neg(a[i][1]), nil = bf16_neg(a[i][3]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // (Ah + Al)(Bh + Bl) without Al Bl; complex: re = ar br - ai bi, im = ar bi + ai br
        // hi * hi
        accR[i][j] = mfma_bf16(a[i][0], b[j][0], accR[i][j]);
        accR[i][j] = mfma_bf16(nih, b[j][1], accR[i][j]);
        accI[i][j] = mfma_bf16(a[i][0], b[j][1], accI[i][j]);
        accI[i][j] = mfma_bf16(a[i][1], b[j][0], accI[i][j]);
        // hi * lo
        accR[i][j] = mfma_bf16(a[i][0], b[j][2], accR[i][j]);
        accR[i][j] = mfma_bf16(nih, b[j][3], accR[i][j]);
        accI[i][j] = mfma_bf16(a[i][0], b[j][3], accI[i][j]);
        accI[i][j] = mfma_bf16(a[i][1], b[j][2], accI[i][j]);
        // lo * hi
        accR[i][j] = mfma_bf16(a[i][2], b[j][0], accR[i][j]);
        accR[i][j] = mfma_bf16(nil, b[j][1], accR[i][j]);
        accI[i][j] = mfma_bf16(a[i][2], b[j][1], accI[i][j]);
        accI[i][j] = mfma_bf16(a[i][3], b[j][0], accI[i][j]);
      }
    }
  }
  double scale = 2.0 / *tau_dev;
  if (upstream_dev) scale *= *upstream_dev;
  const float sc = float(scale);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = C0 + wc * 32 + j * 16 + li;
      const int64_t row0 = R0 + wr * 32 + i * 16 + lq * 4;
#pragma unroll
      for (int v = 0; v < 4; ++v) C[(row0 + v) * ldc + col] = Cx<float>{accR[i][j][v] * sc, accI[i][j][v] * sc};
    }
}

// ---------------------------------------------------------------------------
// Small matrices (d < 64): one thread per output entry.
// ---------------------------------------------------------------------------
template <typename R, bool BF16>
__global__ void herk_small_kernel(const Cx<R>* __restrict__ T, int64_t ldt, Cx<R>* __restrict__ C,
                                  int64_t ldc, int d, const double* __restrict__ tau_dev) {
  const int i = blockIdx.x, j = threadIdx.x;
  if (j >= d) return;
  R sr = 0, si = 0;
  for (int k = 0; k < d; ++k) {
    Cx<R> a = T[int64_t(i) * ldt + k], b = T[int64_t(j) * ldt + k];
    if constexpr (BF16) {
      a = {R(bf16_value(float(a.re))), R(bf16_value(float(a.im)))};
      b = {R(bf16_value(float(b.re))), R(bf16_value(float(b.im)))};
    }
    sr += a.re * b.re + a.im * b.im;
    si += a.im * b.re - a.re * b.im;
  }
  const double inv = 1.0 / *tau_dev;
  C[int64_t(i) * ldc + j] = Cx<R>{R(sr * inv), R(si * inv)};
}

template <typename R, bool SPLIT>
__global__ void hemm_small_kernel(const Cx<R>* __restrict__ G, int64_t ldg, const Cx<R>* __restrict__ T,
                                  int64_t ldt, Cx<R>* __restrict__ C, int64_t ldc, int d,
                                  const double* __restrict__ tau_dev, const double* __restrict__ upstream_dev) {
  const int i = blockIdx.x, j = threadIdx.x;
  if (j >= d) return;
  R sr = 0, si = 0;
  for (int k = 0; k < d; ++k) {
    const Cx<R> a = G[int64_t(i) * ldg + k], b = T[int64_t(k) * ldt + j];
    if constexpr (SPLIT) {
      const float ahr = bf16_value(float(a.re)), ahi = bf16_value(float(a.im));
      const float alr = bf16_value(float(a.re) - ahr), ali = bf16_value(float(a.im) - ahi);
      const float bhr = bf16_value(float(b.re)), bhi = bf16_value(float(b.im));
      const float blr = bf16_value(float(b.re) - bhr), bli = bf16_value(float(b.im) - bhi);
      sr += (ahr * bhr - ahi * bhi) + (ahr * blr - ahi * bli) + (alr * bhr - ali * bhi);
      si += (ahr * bhi + ahi * bhr) + (ahr * bli + ahi * blr) + (alr * bhi + ali * bhr);
    } else {
      sr += a.re * b.re - a.im * b.im;
      si += a.re * b.im + a.im * b.re;
    }
  }
  double scale = 2.0 / *tau_dev;
  if (upstream_dev) scale *= *upstream_dev;
  C[int64_t(i) * ldc + j] = Cx<R>{R(sr * scale), R(si * scale)};
}

}  // namespace

hipError_t launch_herk(qst_prec prec, const void* T, int64_t ldt, void* rho, int64_t ldr, int n,
                       const double* tau_dev, hipStream_t s) {
  const int d = 1 << n;
  ProfScope prof(d < BM ? "herk_small" : (prec == QST_F64 ? "herk_f64" : prec == QST_F32 ? "herk_f32" : "herk_bf16"), s);
  if (d < BM) {
    if (prec == QST_F64)
      herk_small_kernel<double, false><<<d, 64, 0, s>>>(static_cast<const Cx<double>*>(T), ldt,
                                                        static_cast<Cx<double>*>(rho), ldr, d, tau_dev);
    else if (prec == QST_F32)
      herk_small_kernel<float, false><<<d, 64, 0, s>>>(static_cast<const Cx<float>*>(T), ldt,
                                                       static_cast<Cx<float>*>(rho), ldr, d, tau_dev);
    else
      herk_small_kernel<float, true><<<d, 64, 0, s>>>(static_cast<const Cx<float>*>(T), ldt,
                                                      static_cast<Cx<float>*>(rho), ldr, d, tau_dev);
    return hipGetLastError();
  }
  const int tiles = d / BM;
  const unsigned blocks = unsigned(tiles * (tiles + 1) / 2);
  if (prec == QST_F64) {
    gemm_cx_kernel<double, true><<<blocks, 256, 0, s>>>(static_cast<const Cx<double>*>(T), ldt,
                                                        static_cast<const Cx<double>*>(T), ldt,
                                                        static_cast<Cx<double>*>(rho), ldr, d, tau_dev, nullptr);
  } else if (prec == QST_F32) {
    gemm_cx_kernel<float, true><<<blocks, 256, 0, s>>>(static_cast<const Cx<float>*>(T), ldt,
                                                       static_cast<const Cx<float>*>(T), ldt,
                                                       static_cast<Cx<float>*>(rho), ldr, d, tau_dev, nullptr);
  } else {
    herk_bf16_kernel<<<blocks, 256, 0, s>>>(static_cast<const Cx<float>*>(T), ldt,
                                            static_cast<Cx<float>*>(rho), ldr, d, tau_dev);
  }
  return hipGetLastError();
}

hipError_t launch_hemm(qst_prec prec, const void* G, int64_t ldg, const void* T, int64_t ldt, void* out,
                       int64_t ldo, int n, const double* tau_dev, const double* upstream_dev,
                       hipStream_t s) {
  const int d = 1 << n;
  ProfScope prof(d < BM ? "hemm_small" : (prec == QST_F64 ? "hemm_f64" : prec == QST_F32 ? "hemm_f32" : "hemm_bf16x3"), s);
  if (d < BM) {
    if (prec == QST_F64)
      hemm_small_kernel<double, false><<<d, 64, 0, s>>>(static_cast<const Cx<double>*>(G), ldg,
                                                        static_cast<const Cx<double>*>(T), ldt,
                                                        static_cast<Cx<double>*>(out), ldo, d, tau_dev,
                                                        upstream_dev);
    else if (prec == QST_F32)
      hemm_small_kernel<float, false><<<d, 64, 0, s>>>(static_cast<const Cx<float>*>(G), ldg,
                                                       static_cast<const Cx<float>*>(T), ldt,
                                                       static_cast<Cx<float>*>(out), ldo, d, tau_dev,
                                                       upstream_dev);
    else
      hemm_small_kernel<float, true><<<d, 64, 0, s>>>(static_cast<const Cx<float>*>(G), ldg,
                                                      static_cast<const Cx<float>*>(T), ldt,
                                                      static_cast<Cx<float>*>(out), ldo, d, tau_dev,
                                                      upstream_dev);
    return hipGetLastError();
  }
  const int tiles = d / BM;
  const unsigned blocks = unsigned(tiles * tiles);
  if (prec == QST_F64) {
    gemm_cx_kernel<double, false><<<blocks, 256, 0, s>>>(static_cast<const Cx<double>*>(G), ldg,
                                                         static_cast<const Cx<double>*>(T), ldt,
                                                         static_cast<Cx<double>*>(out), ldo, d, tau_dev,
                                                         upstream_dev);
  } else if (prec == QST_F32) {
    gemm_cx_kernel<float, false><<<blocks, 256, 0, s>>>(static_cast<const Cx<float>*>(G), ldg,
                                                        static_cast<const Cx<float>*>(T), ldt,
                                                        static_cast<Cx<float>*>(out), ldo, d, tau_dev,
                                                        upstream_dev);
  } else {
    hemm_bf16x3_kernel<<<blocks, 256, 0, s>>>(static_cast<const Cx<float>*>(G), ldg,
                                              static_cast<const Cx<float>*>(T), ldt,
                                              static_cast<Cx<float>*>(out), ldo, d, tau_dev, upstream_dev);
  }
  return hipGetLastError();
}

}  // namespace qst
