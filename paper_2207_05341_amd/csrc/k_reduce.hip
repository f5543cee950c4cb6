// FP64 reductions of the likelihood path, deterministic two-stage form:
//   tau = sum_ij |T_ij|^2                 (denominator of Eq. T_matrix)
//   L = -sum_{f_k != 0} f_k ln p_k, F = sum_k f_k   (Eq. MLE / loss, Sec. 3.1)
// Stage 1: block b of kReduceBlocks owns the contiguous element range
// [b*chunk, (b+1)*chunk) and reduces it in a fixed order (strided per thread,
// then a wave64 shuffle tree and a 4-wave combine).  Stage 2: one block
// reduces the partials in a fixed order.  No floating-point atomics, so the
// results are bitwise reproducible run to run.
#include "qst_device.h"
#include "qst_kernels.h"
#include "qst_plan.h"

namespace qst {

namespace {

// ROUND: 0 = T as given, 1 = bf16(T), 2 = bf16 hi + lo of T (exact in fp32).
// WITH_F: also F = sum f over the same element range (f has 4^N = d^2
// entries, element e of T and f alike), partials[nb + b].
template <typename R, int ROUND, bool WITH_F = false>
__global__ __launch_bounds__(256) void tau_partial_kernel(const Cx<R>* __restrict__ T, int64_t ld,
                                                          int n, double* __restrict__ partials,
                                                          const R* __restrict__ f = nullptr) {
  __shared__ double red[4];
  const int64_t d = int64_t(1) << n;
  const int64_t total = d * d;
  const int64_t chunk = (total + gridDim.x - 1) / gridDim.x;
  const int64_t beg = int64_t(blockIdx.x) * chunk;
  const int64_t end = beg + chunk < total ? beg + chunk : total;
  // Up to 16 strided elements per thread are loaded before any arithmetic
  // (all loads in flight at once); the per-thread summation order is fixed.
  constexpr int U = 16;
  double acc = 0.0, accf = 0.0;
  for (int64_t e0 = beg + threadIdx.x; e0 < end; e0 += U * int64_t(blockDim.x)) {
    Cx<R> v[U];
    R fv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + u * int64_t(blockDim.x);
      v[u] = e < end ? T[(e >> n) * ld + (e & (d - 1))] : Cx<R>{R(0), R(0)};
      if constexpr (WITH_F) fv[u] = e < end ? f[e] : R(0);
    }
    if constexpr (WITH_F) {
#pragma unroll
      for (int u = 0; u < U; ++u) accf += double(fv[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double x = double(v[u].re), y = double(v[u].im);
      if constexpr (ROUND == 1) {
        x = double(bf16_value(float(v[u].re)));
        y = double(bf16_value(float(v[u].im)));
      } else if constexpr (ROUND == 2) {
        const float hr = bf16_value(float(v[u].re)), hi = bf16_value(float(v[u].im));
        x = double(hr + bf16_value(float(v[u].re) - hr));
        y = double(hi + bf16_value(float(v[u].im) - hi));
      }
      acc += x * x + y * y;
    }
  }
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  if constexpr (WITH_F) {
    const double sf = block_sum256(accf, red);
    if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = sf;
  }
}

// BF16 path with planes: the partial sums of tau_partial_kernel<float, 1,
// WITH_F> over the same per-block element ranges, and bf16(T) stored as a
// re plane and an im plane (d x d row-major each: element e = r d + c at
// planes[e] and planes[d^2 + e]), the operands of the bf16 product.  Each
// thread takes 8 consecutive elements of a row at a time (16-byte plane
// stores); needs the block range to be a multiple of 8 (d^2 / kReduceBlocks
// for d >= 256).
template <bool WITH_F>
__global__ __launch_bounds__(256) void tau_planes_kernel(const Cx<float>* __restrict__ T, int64_t ld, int n,
                                                         double* __restrict__ partials,
                                                         const float* __restrict__ f,
                                                         uint16_t* __restrict__ planes) {
  __shared__ double red[4];
  const int64_t d = int64_t(1) << n;
  const int64_t total = d * d;
  const int64_t chunk = (total + gridDim.x - 1) / gridDim.x;
  const int64_t beg = int64_t(blockIdx.x) * chunk;
  const int64_t end = beg + chunk < total ? beg + chunk : total;
  constexpr int U = 2;
  double acc = 0.0, accf = 0.0;
  for (int64_t e0 = beg + 8 * int64_t(threadIdx.x); e0 < end; e0 += 8 * U * int64_t(blockDim.x)) {
    Cx<float> v[U][8];
    float fv[U][8];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + u * 8 * int64_t(blockDim.x);
      const bool in = e < end;
      const Cx<float>* src = T + (e >> n) * ld + (e & (d - 1));
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        v[u][i] = in ? src[i] : Cx<float>{0.f, 0.f};
        if constexpr (WITH_F) fv[u][i] = in ? f[e + i] : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + u * 8 * int64_t(blockDim.x);
      float re[8], im[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        re[i] = v[u][i].re;
        im[i] = v[u][i].im;
      }
      const u16x8 hr = bf16x8(re), hi = bf16x8(im);
      if (e < end) {
        *reinterpret_cast<u16x8*>(planes + e) = hr;
        *reinterpret_cast<u16x8*>(planes + total + e) = hi;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double x = double(bf16_to_float(hr[i])), y = double(bf16_to_float(hi[i]));
        acc += x * x + y * y;
        if constexpr (WITH_F) accf += double(fv[u][i]);
      }
    }
  }
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  if constexpr (WITH_F) {
    const double sf = block_sum256(accf, red);
    if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = sf;
  }
}

// One 256-thread block: out[i] = sum_b partials[i*nb + b] for i < nsum.
__global__ __launch_bounds__(256) void finish_sums_kernel(const double* __restrict__ partials, int nb,
                                                          int nsum, double* __restrict__ out) {
  __shared__ double red[4];
  for (int i = 0; i < nsum; ++i) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partials[int64_t(i) * nb + b];
    const double s = block_sum256(acc, red);
    if (threadIdx.x == 0) out[i] = s;
  }
}

// Stage 1 of the NLL: partials laid out [4][nb]: L, F, bad0, bad1.
template <typename R, bool WITH_P>
__global__ __launch_bounds__(256) void nll_partial_kernel(const R* __restrict__ p,
                                                          const R* __restrict__ f, int64_t D,
                                                          double* __restrict__ partials) {
  __shared__ double red[4];
  const int nb = gridDim.x;
  const int64_t chunk = (D + nb - 1) / nb;
  const int64_t beg = int64_t(blockIdx.x) * chunk;
  const int64_t end = beg + chunk < D ? beg + chunk : D;
  // Up to 16 strided elements per thread loaded before any arithmetic.
  constexpr int U = 16;
  double L = 0.0, F = 0.0, bad0 = 0.0, bad1 = 0.0;
  for (int64_t k0 = beg + threadIdx.x; k0 < end; k0 += U * int64_t(blockDim.x)) {
    R fv[U], pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = k0 + u * int64_t(blockDim.x);
      const bool in = k < end;
      fv[u] = in ? f[k] : R(0);
      if constexpr (WITH_P) pv[u] = in ? p[k] : R(1);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double fk = double(fv[u]);
      F += fk;
      if constexpr (WITH_P) {
        const double pk = double(pv[u]);
        if (fk != 0.0) {
          if (pk > 0.0) {
            L -= fk * ln_prob(pv[u]);
          } else {
            bad0 += 1.0;
          }
        }
        if (pk != pk || fk != fk) bad1 += 1.0;
      }
    }
  }
  double s = block_sum256(L, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  s = block_sum256(F, red);
  if (threadIdx.x == 0) partials[nb + blockIdx.x] = s;
  if constexpr (WITH_P) {
    s = block_sum256(bad0, red);
    if (threadIdx.x == 0) partials[2 * nb + blockIdx.x] = s;
    s = block_sum256(bad1, red);
    if (threadIdx.x == 0) partials[3 * nb + blockIdx.x] = s;
  }
}

// Stage 2 of the NLL: nll[0] = L (+inf if a bad term, NaN if a NaN input),
// nll[1] = F; bad[0], bad[1] counts.
__global__ __launch_bounds__(256) void nll_finish_kernel(const double* __restrict__ partials, int nb,
                                                         double* __restrict__ nll,
                                                         unsigned long long* __restrict__ bad) {
  __shared__ double red[4];
  double sums[4];
  for (int i = 0; i < 4; ++i) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partials[int64_t(i) * nb + b];
    sums[i] = block_sum256(acc, red);
  }
  if (threadIdx.x == 0) {
    double L = sums[0];
    if (sums[1] != sums[1] || sums[3] > 0.0) {
      L = __builtin_nan("");
    } else if (sums[2] > 0.0) {
      L = __builtin_inf();
    }
    nll[0] = L;
    nll[1] = sums[1];
    if (bad) {
      bad[0] = (unsigned long long)sums[2];
      bad[1] = (unsigned long long)sums[3];
    }
  }
}

// Stage 2 of qst_likelihood's NLL: L and the counters from the fused pass's
// partials [4][nb] (slot 1 unused), F from the kReduceBlocks F partials of
// the tau kernel, summed exactly as the fused pass sums them.
__global__ __launch_bounds__(256) void likelihood_finish_kernel(const double* __restrict__ part, int nb,
                                                                const double* __restrict__ Fpart,
                                                                double* __restrict__ nll,
                                                                unsigned long long* __restrict__ bad,
                                                                double* __restrict__ fc) {
  __shared__ double red[4];
  // Each thread sums slots 0, 2, 3 (and the F_c slot 1) of part with stride
  // 256 and the F partials likewise, in increasing index, as before; the
  // loads of all of them are issued U per array before any of the adds
  // (indices past the end are clamped and their values not added), so the
  // arrays' latencies overlap.  Block sums as sum_partials256 / block_sum256.
  constexpr int U = 4;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // slots 0, 2, 3, F, F_c
  const int nmax = nb > kReduceBlocks ? nb : kReduceBlocks;
  for (int b0 = threadIdx.x; b0 < nmax; b0 += 256 * U) {
    double v[5][U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + 256 * u;
      const int bp = b < nb ? b : nb - 1, bf = b < kReduceBlocks ? b : kReduceBlocks - 1;
      v[0][u] = part[bp];
      v[1][u] = part[int64_t(2) * nb + bp];
      v[2][u] = part[int64_t(3) * nb + bp];
      v[3][u] = Fpart[bf];
      v[4][u] = fc ? part[int64_t(nb) + bp] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + 256 * u;
      if (b < nb) {
        acc[0] += v[0][u];
        acc[1] += v[1][u];
        acc[2] += v[2][u];
        acc[4] += v[4][u];
      }
      if (b < kReduceBlocks) acc[3] += v[3][u];
    }
  }
  if (fc) {  // F_c = (sum of the F_c terms)^2 from slot 1
    const double t = block_sum256(acc[4], red);
    if (threadIdx.x == 0) fc[0] = t * t;
  }
  double sums[4];
  sums[0] = block_sum256(acc[0], red);
  sums[1] = block_sum256(acc[3], red);
  sums[2] = block_sum256(acc[1], red);
  sums[3] = block_sum256(acc[2], red);
  if (threadIdx.x == 0) {
    double L = sums[0];
    if (sums[1] != sums[1] || sums[3] > 0.0) {
      L = __builtin_nan("");
    } else if (sums[2] > 0.0) {
      L = __builtin_inf();
    }
    nll[0] = L;
    nll[1] = sums[1];
    if (bad) {
      bad[0] = (unsigned long long)sums[2];
      bad[1] = (unsigned long long)sums[3];
    }
  }
}

}  // namespace

hipError_t launch_tau(qst_prec prec, const void* T, int64_t ld, int n, double* partials,
                      double* tau_dev, hipStream_t s, const void* f, void* planes) {
  const int nb = kReduceBlocks;
  ProfScope prof("tau_reduce", s);
  prec = storage_prec(prec);  // QST_F32X6 reaches here only below kX6Tile, where it runs as QST_F32
  const Cx<double>* T64 = static_cast<const Cx<double>*>(T);
  const Cx<float>* T32 = static_cast<const Cx<float>*>(T);
  const double* f64 = static_cast<const double*>(f);
  const float* f32 = static_cast<const float*>(f);
  if (prec == QST_F64) {
    if (f) tau_partial_kernel<double, 0, true><<<nb, 256, 0, s>>>(T64, ld, n, partials, f64);
    else tau_partial_kernel<double, 0><<<nb, 256, 0, s>>>(T64, ld, n, partials);
  } else if (prec == QST_F32) {
    if (f) tau_partial_kernel<float, 0, true><<<nb, 256, 0, s>>>(T32, ld, n, partials, f32);
    else tau_partial_kernel<float, 0><<<nb, 256, 0, s>>>(T32, ld, n, partials);
  } else if ((int64_t(1) << n) <= kBf16SplitMaxDim) {
    if (f) tau_partial_kernel<float, 2, true><<<nb, 256, 0, s>>>(T32, ld, n, partials, f32);
    else tau_partial_kernel<float, 2><<<nb, 256, 0, s>>>(T32, ld, n, partials);
  } else {
    uint16_t* pl = static_cast<uint16_t*>(planes);
    if (pl && f) tau_planes_kernel<true><<<nb, 256, 0, s>>>(T32, ld, n, partials, f32, pl);
    else if (pl) tau_planes_kernel<false><<<nb, 256, 0, s>>>(T32, ld, n, partials, nullptr, pl);
    else if (f) tau_partial_kernel<float, 1, true><<<nb, 256, 0, s>>>(T32, ld, n, partials, f32);
    else tau_partial_kernel<float, 1><<<nb, 256, 0, s>>>(T32, ld, n, partials);
  }
  if (tau_dev) finish_sums_kernel<<<1, 256, 0, s>>>(partials, nb, 1, tau_dev);
  return hipGetLastError();
}

hipError_t launch_nll(qst_prec prec, const void* p, const void* f, int n, double* partials,
                      double* nll_dev, unsigned long long* bad_dev, hipStream_t s) {
  const int nb = kReduceBlocks;
  ProfScope prof("nll_reduce", s);
  const int64_t D = int64_t(1) << (2 * n);
  if (prec == QST_F64) {
    nll_partial_kernel<double, true><<<nb, 256, 0, s>>>(static_cast<const double*>(p),
                                                        static_cast<const double*>(f), D, partials);
  } else {
    nll_partial_kernel<float, true><<<nb, 256, 0, s>>>(static_cast<const float*>(p),
                                                       static_cast<const float*>(f), D, partials);
  }
  nll_finish_kernel<<<1, 256, 0, s>>>(partials, nb, nll_dev, bad_dev);
  return hipGetLastError();
}

hipError_t launch_nll_partials(qst_prec prec, const void* p, const void* f, int64_t D, double* partials,
                               hipStream_t s) {
  const int nb = kReduceBlocks;
  if (prec == QST_F64)
    nll_partial_kernel<double, true><<<nb, 256, 0, s>>>(static_cast<const double*>(p),
                                                        static_cast<const double*>(f), D, partials);
  else
    nll_partial_kernel<float, true><<<nb, 256, 0, s>>>(static_cast<const float*>(p),
                                                       static_cast<const float*>(f), D, partials);
  return hipGetLastError();
}

hipError_t launch_likelihood_finish(const double* part, int nb, const double* Fpart, double* nll_dev,
                                   unsigned long long* bad_dev, hipStream_t s, double* fc_dev) {
  likelihood_finish_kernel<<<1, 256, 0, s>>>(part, nb, Fpart, nll_dev, bad_dev, fc_dev);
  return hipGetLastError();
}

hipError_t launch_fsum(qst_prec prec, const void* f, int n, double* partials, double* F_dev,
                       hipStream_t s) {
  const int nb = kReduceBlocks;
  const int64_t D = int64_t(1) << (2 * n);
  ProfScope prof("fsum_reduce", s);
  if (prec == QST_F64) {
    nll_partial_kernel<double, false><<<nb, 256, 0, s>>>(nullptr, static_cast<const double*>(f), D, partials);
  } else {
    nll_partial_kernel<float, false><<<nb, 256, 0, s>>>(nullptr, static_cast<const float*>(f), D, partials);
  }
  finish_sums_kernel<<<1, 256, 0, s>>>(partials + nb, nb, 1, F_dev);
  return hipGetLastError();
}

}  // namespace qst
