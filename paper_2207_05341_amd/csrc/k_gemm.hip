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
// Tiles: 256 threads (4 wave64), 64 x 64 complex output per tile, each wave a
// 32 x 32 quadrant as 2 x 2 MFMA 16 x 16 blocks.  Operand panels are staged
// through LDS with the next panel prefetched into registers while the
// current one is consumed.
//
// Scheduling: when the tile count divides evenly over the compute units,
// one workgroup computes one tile.  Otherwise (the 528 lower tiles of
// T T^dagger at d = 2048 land 2 or 3 per CU) the kernel runs stream-K: a
// grid of P workgroups, each taking an equal contiguous share of the
// (tile, K panel) iterations.  A tile cut between workgroups leaves partial
// accumulators in the workspace (at most two per workgroup), and a fix-up
// kernel adds them in K order -- no atomics, so results are deterministic.
#include <algorithm>
#include <cmath>

#include "qst_device.h"
#include "qst_gemm_tiles.h"
#include "qst_kernels.h"
#include "qst_plan.h"

namespace qst {

namespace {

using namespace gemm;

// First iteration owned by stream-K workgroup w of P.
__device__ __forceinline__ int64_t sk_start(int64_t w, int64_t P, int64_t iters) { return (w * iters) / P; }

// Tile output: rho / G' T, or with X0G = g (4..6) the first POVM pass over
// g qubits of a T T^dagger tile.
template <class P, int X0G>
__device__ __forceinline__ void finish_tile(const GemmArgs& g, int tr, int tc, typename P::acc_t (&aR)[2][2],
                                            typename P::acc_t (&aI)[2][2], double scale, void* lds) {
  if constexpr (X0G != 0) {
    x0_tile<P, X0G>(g, tr, tc, aR, aI, scale, static_cast<Cx<typename P::scalar>*>(lds));
  } else {
    epilogue<P>(g, tr, tc, aR, aI, scale);
  }
}

// One tile per workgroup.
template <class P, int X0G>
__global__ __launch_bounds__(256, P::kMinWaves) void gemm_dp_kernel(GemmArgs g) {
  __shared__ __align__(16) unsigned char smem[smem_bytes<P, X0G != 0>()];
  auto& sm = *reinterpret_cast<typename P::Smem*>(smem);
  typename P::acc_t aR[2][2], aI[2][2];
  const double scale = tile_scale<P>(g);
  int tr, tc;
  tile_coords<P>(g, blockIdx.x, tr, tc);
  zero_acc<P>(aR, aI);
  P::run(g, sm, tr, tc, 0, g.kIters, aR, aI);
  finish_tile<P, X0G>(g, tr, tc, aR, aI, scale, smem);
}

// Hybrid schedule: workgroup w first computes the whole tiles w, w + P,
// w + 2P, ... below dp_tiles, then owns the stream-K iterations
// [start(w), start(w+1)) of the K panels of the remaining tiles.
template <class P, int X0G>
__global__ __launch_bounds__(256, P::kMinWaves) void gemm_sk_kernel(GemmArgs g) {
  __shared__ __align__(16) unsigned char smem[smem_bytes<P, X0G != 0>()];
  auto& sm = *reinterpret_cast<typename P::Smem*>(smem);
  typename P::acc_t aR[2][2], aI[2][2];
  // logical workgroup index: consecutive tiles and consecutive segments
  // (neighbours sharing panels) run on one XCD
  const int64_t Pn = gridDim.x, w = xcd_order(blockIdx.x, gridDim.x);
  const double scale = tile_scale<P>(g);
  // one loop over the work items (whole tiles, then the stream-K slice), so
  // that the tile epilogue is instantiated once
  int64_t t = w;
  int64_t it = sk_start(w, Pn, g.iters);
  const int64_t end = sk_start(w + 1, Pn, g.iters);
  const int first_rel = int(it / g.kIters);
  while (t < g.dp_tiles || it < end) {
    int tile, kb, ke, rel = 0;
    if (t < g.dp_tiles) {
      tile = int(t);
      kb = 0;
      ke = g.kIters;
      t += Pn;
    } else {
      rel = int(it / g.kIters);
      kb = int(it % g.kIters);
      ke = int(min(int64_t(g.kIters), int64_t(kb) + (end - it)));
      tile = g.dp_tiles + rel;
      it += ke - kb;
    }
    int tr, tc;
    tile_coords<P>(g, tile, tr, tc);
    zero_acc<P>(aR, aI);
    P::run(g, sm, tr, tc, kb, ke, aR, aI);
    if (kb == 0 && ke == g.kIters) {
      finish_tile<P, X0G>(g, tr, tc, aR, aI, scale, smem);
    } else {
      store_partial<P>(partial_slot<P>(g, int(w), rel == first_rel ? 0 : 1), aR, aI);
    }
  }
}

// Stream-K workgroups owning the first and the last K panel of tile
// dp_tiles + rel.
__device__ __forceinline__ void tile_owners(const GemmArgs& g, int64_t Pn, int rel, int64_t& wlo, int64_t& whi) {
  const int64_t kb = int64_t(rel) * g.kIters, kl = kb + g.kIters - 1;
  wlo = (kb * Pn) / g.iters;
  while (wlo + 1 < Pn && sk_start(wlo + 1, Pn, g.iters) <= kb) ++wlo;
  while (wlo > 0 && sk_start(wlo, Pn, g.iters) > kb) --wlo;
  whi = (kl * Pn) / g.iters;
  while (whi + 1 < Pn && sk_start(whi + 1, Pn, g.iters) <= kl) ++whi;
  while (whi > 0 && sk_start(whi, Pn, g.iters) > kl) --whi;
}

// Partial of workgroup w for tile dp_tiles + rel.
template <class P>
__device__ __forceinline__ typename P::scalar* tile_partial(const GemmArgs& g, int64_t Pn, int64_t w, int rel) {
  const int first_rel = int(sk_start(w, Pn, g.iters) / g.kIters);
  return partial_slot<P>(g, int(w), rel == first_rel ? 0 : 1);
}

// Sum the partials of workgroups [lo, hi] for tile dp_tiles + rel in
// workgroup order, four per memory round trip.
template <class P>
__device__ __forceinline__ void sum_partials(const GemmArgs& g, int64_t Pn, int rel, int64_t lo, int64_t hi,
                                             int64_t step, typename P::acc_t (&aR)[2][2],
                                             typename P::acc_t (&aI)[2][2]) {
  int64_t w = lo;
  for (; w + 3 * step <= hi; w += 4 * step) {
    const typename P::scalar* const src[4] = {tile_partial<P>(g, Pn, w, rel), tile_partial<P>(g, Pn, w + step, rel),
                                              tile_partial<P>(g, Pn, w + 2 * step, rel),
                                              tile_partial<P>(g, Pn, w + 3 * step, rel)};
    add_partials<P, 4>(src, aR, aI);
  }
  for (; w <= hi; w += step) add_partial<P>(tile_partial<P>(g, Pn, w, rel), aR, aI);
}

// First level of the fix-up for tiles cut into many segments: workgroup
// (rel, c) sums the partials of the stream-K workgroups wlo + c*chunk ..
// wlo + (c+1)*chunk - 1 of tile dp_tiles + rel (in order) into the first
// one's partial, so that the fix-up adds one partial per chunk.  A
// workgroup reads and writes only the partials of its own chunk.  (Slicing
// each partial over several workgroups, one 16-byte vector per thread and
// all partials of a chunk in flight at once, measured slower: 20 us against
// 13 us for the 16 tiles of FP64 at N = 11.)
template <class P>
__global__ __launch_bounds__(256) void gemm_chunk_sum_kernel(GemmArgs g, int Pn, int chunk, int groups) {
  const int rel = blockIdx.x / groups, c = blockIdx.x % groups;
  int64_t wlo, whi;
  tile_owners(g, Pn, rel, wlo, whi);
  const int64_t lo = wlo + int64_t(c) * chunk;
  const int64_t hi = min(whi, lo + chunk - 1);
  if (lo >= hi) return;  // empty chunk, or a single partial already in place
  typename P::acc_t aR[2][2], aI[2][2];
  zero_acc<P>(aR, aI);
  sum_partials<P>(g, Pn, rel, lo, hi, 1, aR, aI);
  store_partial<P>(tile_partial<P>(g, Pn, lo, rel), aR, aI);
}

// Sum the partial segments of every stream-K tile that was cut, in K order
// (with chunk > 1, the chunk sums left by gemm_chunk_sum_kernel).
// Workgroup b handles tile dp_tiles + b.
template <class P, int X0G>
__global__ __launch_bounds__(256) void gemm_fixup_kernel(GemmArgs g, int Pn, int chunk) {
  __shared__ __align__(16) unsigned char smem[X0G ? smem_bytes<P, X0G != 0>() : 16];
  const int rel = blockIdx.x;
  int64_t wlo, whi;
  tile_owners(g, Pn, rel, wlo, whi);
  if (wlo == whi) return;  // whole tile inside one workgroup: already written
  const double scale = tile_scale<P>(g);
  typename P::acc_t aR[2][2], aI[2][2];
  zero_acc<P>(aR, aI);
  sum_partials<P>(g, Pn, rel, wlo, whi, chunk, aR, aI);
  int tr, tc;
  tile_coords<P>(g, g.dp_tiles + rel, tr, tc);
  finish_tile<P, X0G>(g, tr, tc, aR, aI, scale, smem);
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
    if constexpr (BF16) {  // d < 64: split bf16 x 3, as the d <= 128 tiles
      const float ahr = bf16_value(float(a.re)), ahi = bf16_value(float(a.im));
      const float alr = bf16_value(float(a.re) - ahr), ali = bf16_value(float(a.im) - ahi);
      const float bhr = bf16_value(float(b.re)), bhi = bf16_value(float(b.im));
      const float blr = bf16_value(float(b.re) - bhr), bli = bf16_value(float(b.im) - bhi);
      sr += (ahr * bhr + ahi * bhi) + (ahr * blr + ahi * bli) + (alr * bhr + ali * bhi);
      si += (ahi * bhr - ahr * bhi) + (ahi * blr - ahr * bli) + (ali * bhr - alr * bhi);
    } else {
      sr += a.re * b.re + a.im * b.im;
      si += a.im * b.re - a.re * b.im;
    }
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

// Compute units of the current device (cached per device).
int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

// Workgroups of gemm_sk_kernel<P, X0G> resident per CU (queried once per process).
template <class P, int X0G>
int sk_occupancy() {
  static int occ = 0;
  if (occ == 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gemm_sk_kernel<P, X0G>, 256, 0) != hipSuccess || n <= 0) n = 1;
    occ = n;
  }
  return occ;
}

// Stream-K grid for a given resident-workgroup count per CU; sets
// g.dp_tiles and g.iters.  Returns 0 when stream-K does not apply.
inline int64_t sk_grid(GemmArgs& g, int cus, int occ) {
  int64_t Pn = 0;
  g.dp_tiles = 0;
  // Whole tiles first when every one of the (CUs x occupancy) workgroups
  // gets at least one: those tiles need no partials.  With fewer tiles than
  // that, lowering the workgroups per CU to make tiles whole costs more
  // (measured at N = 11: 528 tiles at 2 per CU, T T^dagger 245 -> 283 us)
  // than the partials it saves, so every tile is split instead.
  if (g.ntiles / cus >= occ) {
    Pn = int64_t(cus) * occ;
    g.dp_tiles = int((g.ntiles / Pn) * Pn);
  } else {
    const int64_t min_iters = 32;  // at least 32 K panels per stream-K workgroup
    Pn = std::min<int64_t>(int64_t(kStreamKMaxGrid),
                           std::min<int64_t>(int64_t(cus) * occ, int64_t(g.ntiles) * g.kIters / min_iters));
    Pn = (Pn / cus) * cus;  // whole waves of workgroups over the compute units
  }
  if (Pn < cus || Pn > kStreamKMaxGrid) {
    g.dp_tiles = 0;
    return 0;
  }
  g.iters = int64_t(g.ntiles - g.dp_tiles) * g.kIters;
  if (g.iters < Pn) {  // every stream-K workgroup must own at least one K panel
    g.dp_tiles = 0;
    g.iters = int64_t(g.ntiles) * g.kIters;
    return 0;
  }
  return Pn;
}

// Fix-up of the tiles dp_tiles.. cut by the stream-K kernel of Pn
// workgroups.  A tile cut into many segments (32 for the one wave of 16
// leftover tiles in FP64 at N = 11) would leave one workgroup reading them
// all (45 us for FP64 at N = 11); above 8 segments they are first summed
// in chunks of about sqrt(segments) by gemm_chunk_sum_kernel (13 + 18 us).
template <class P, int X0G>
hipError_t launch_fixup(const GemmArgs& g, int64_t Pn, hipStream_t s) {
  const int64_t sk_tiles = g.ntiles - g.dp_tiles;
  // workgroups sharing one tile: at most ceil(kIters / min panels per workgroup) + 1
  const int64_t per_wg = g.iters / Pn;
  const int64_t parts = std::min<int64_t>(Pn, (g.kIters + per_wg - 1) / per_wg + 1);
  int chunk = 1;
  if (parts > 8) {
    chunk = int(std::lround(std::sqrt(double(parts))));
    const int groups = int((parts + chunk - 1) / chunk);
    gemm_chunk_sum_kernel<P><<<unsigned(sk_tiles * groups), 256, 0, s>>>(g, int(Pn), chunk, groups);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  GemmArgs gf = g;
  gf.tau_out = nullptr;
  gemm_fixup_kernel<P, X0G><<<unsigned(sk_tiles), 256, 0, s>>>(gf, int(Pn), chunk);
  return hipGetLastError();
}

template <class P, int X0G = 0>
hipError_t run_gemm(GemmArgs g, hipStream_t s) {
  g.kIters = g.d / P::KP;
  g.iters = int64_t(g.ntiles) * g.kIters;
  const int cus = device_cus();
  g.dp_tiles = 0;
  bool sk = P::kStreamK && g.partial != nullptr && g.ntiles % cus != 0;
  if (sk && X0G != 0) {
    // The POVM epilogue raises the register use of the stream-K kernel.
    // When no workgroup of the plain kernel's grid can finish a whole tile
    // (no data-parallel tiles, every slice shorter than a tile), all tiles
    // are finished by the fix-up: run the plain stream-K kernel (its
    // epilogue is then never reached) and the POVM fix-up.
    GemmArgs gp = g;
    const int64_t Pn = sk_grid(gp, cus, std::min(sk_occupancy<P, 0>(), 4));
    if (Pn > 0 && gp.dp_tiles == 0 && (gp.iters + Pn - 1) / Pn < gp.kIters) {
      gemm_sk_kernel<P, 0><<<unsigned(Pn), 256, 0, s>>>(gp);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      return launch_fixup<P, X0G>(gp, Pn, s);
    }
  }
  int64_t Pn = 0;
  if (sk) {
    const int occ = std::min(sk_occupancy<P, X0G>(), 4);
    Pn = sk_grid(g, cus, occ);
    sk = Pn > 0;
  }
  if (!sk) {
    g.dp_tiles = 0;
    g.iters = int64_t(g.ntiles) * g.kIters;
    gemm_dp_kernel<P, X0G><<<unsigned(g.ntiles), 256, 0, s>>>(g);
    return hipGetLastError();
  }
  gemm_sk_kernel<P, X0G><<<unsigned(Pn), 256, 0, s>>>(g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_fixup<P, X0G>(g, Pn, s);
}

template <int G>
hipError_t run_herk_x0(qst_prec prec, int d, const GemmArgs& g, hipStream_t s, bool planes) {
  if (prec == QST_F64) return run_gemm<CxPolicy<double, true>, G>(g, s);
  if (prec == QST_F32) return run_gemm<CxPolicy<float, true>, G>(g, s);
  if (d <= kBf16SplitMaxDim) return run_gemm<HerkBf16x3Policy, G>(g, s);
  if (planes) return run_gemm<HerkBf16PlanesPolicy, G>(g, s);
  return run_gemm<HerkBf16Policy, G>(g, s);
}

}  // namespace

hipError_t launch_herk(qst_prec prec, const void* T, int64_t ldt, void* rho, int64_t ldr, int n,
                       const double* tau_partials, double* tau_dev, void* sk_partial, hipStream_t s,
                       const Pass0Out* x0, const void* planes) {
  const int d = 1 << n;
  if (prec == QST_F32X6) {
    if (use_x6(prec, n)) return hipErrorInvalidValue;  // launch_x6_herk forms tau itself
    prec = QST_F32;
  }
  if (x0 && (d < BM || x0->g < 4 || x0->g > 6 || !x0->tetra)) return hipErrorInvalidValue;
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
  GemmArgs g{};
  g.A = T;
  g.lda = ldt;
  g.B = T;
  g.ldb = ldt;
  g.C = rho;
  g.ldc = ldr;
  g.d = d;
  g.tau = tau_dev;
  g.up = nullptr;
  g.ntiles = tiles * (tiles + 1) / 2;
  g.partial = sk_partial;
  g.tau_part = tau_partials;
  g.tau_out = tau_partials ? tau_dev : nullptr;
  const bool use_planes = prec == QST_BF16GEMM && d > kBf16SplitMaxDim && planes;
  if (use_planes) {  // operands: bf16 planes of T, row stride d
    g.A = planes;
    g.lda = d;
    g.B = planes;
    g.ldb = d;
  }
  if (x0) {
    g.x0 = x0->X;
    g.x0g = x0->g;
    g.x0up = n - x0->g;
    return x0->g == 6 ? run_herk_x0<6>(prec, d, g, s, use_planes)
           : x0->g == 5 ? run_herk_x0<5>(prec, d, g, s, use_planes)
                        : run_herk_x0<4>(prec, d, g, s, use_planes);
  }
  if (prec == QST_F64) return run_gemm<CxPolicy<double, true>>(g, s);
  if (prec == QST_F32) return run_gemm<CxPolicy<float, true>>(g, s);
  if (d <= kBf16SplitMaxDim) return run_gemm<HerkBf16x3Policy>(g, s);
  if (use_planes) return run_gemm<HerkBf16PlanesPolicy>(g, s);
  return run_gemm<HerkBf16Policy>(g, s);
}

namespace {

// Operand planes of the split-bf16 product, x = hi + lo with hi = bf16(x)
// and lo = bf16(x - hi), for the real and imaginary parts of a d x d complex
// matrix M (leading dimension ld): P[pl][d][d] with pl = re_hi, im_hi,
// re_lo, im_lo; element (r, c) at P[pl][r d + c], or at P[pl][c d + r] with
// TRANSPOSE (through a 64 x 64 LDS tile).  One 64 x 64 tile per workgroup;
// each thread converts two runs of 8 consecutive elements (16-byte stores).
template <bool TRANSPOSE>
__global__ __launch_bounds__(256) void split_planes_kernel(const Cx<float>* __restrict__ M, int64_t ld, int d,
                                                           uint16_t* __restrict__ P) {
  __shared__ Cx<float> tile[TRANSPOSE ? 64 : 1][65];
  const int tiles = d / 64;
  const int64_t r0 = int64_t(blockIdx.x / tiles) * 64, c0 = int64_t(blockIdx.x % tiles) * 64;
  const int64_t dd = int64_t(d) * d;
  const int t = threadIdx.x, rr = t >> 3, cc = (t & 7) * 8;
  auto emit = [&](const Cx<float> (&v)[8], int64_t at) {
    float re[8], im[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      re[i] = v[i].re;
      im[i] = v[i].im;
    }
    u16x8 rh, rl, ih, il;
    bf16x8_split(re, rh, rl);
    bf16x8_split(im, ih, il);
    *reinterpret_cast<u16x8*>(P + at) = rh;
    *reinterpret_cast<u16x8*>(P + dd + at) = ih;
    *reinterpret_cast<u16x8*>(P + 2 * dd + at) = rl;
    *reinterpret_cast<u16x8*>(P + 3 * dd + at) = il;
  };
  Cx<float> v[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const Cx<float>* src = M + (r0 + rr + 32 * h) * ld + c0 + cc;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[h][i] = src[i];
  }
  if constexpr (!TRANSPOSE) {
#pragma unroll
    for (int h = 0; h < 2; ++h) emit(v[h], (r0 + rr + 32 * h) * d + c0 + cc);
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 8; ++i) tile[rr + 32 * h][cc + i] = v[h][i];
    __syncthreads();
    // transposed run: column c of the tile, rows cc .. cc + 7
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = rr + 32 * h;
      Cx<float> u[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) u[i] = tile[cc + i][c];
      emit(u, (c0 + c) * d + r0 + cc);
    }
  }
}

// G' T on the BF16 path for d >= 1024 from the split planes (g.A: planes of
// G', g.B: planes of T^T, both with row stride d): 128 x 128 complex output
// tiles, 512 threads in 8 waves of 64 x 32, panels of 64 k (147 KB of LDS,
// one workgroup per CU); per K step of 32 the three products hi hi + hi lo +
// lo hi of each real product (12 MFMAs per 16 x 16 block).  Per MFMA a 128 x 128 tile moves half the operand bytes of
// a 64 x 64 one, which is what bounds the bf16 form.  Tiles are numbered so
// that each XCD's contiguous range of workgroups covers blocks of 4 x 8
// tiles (4 row panels of G', 8 column panels of T).  Needs d / 128 divisible
// by 8.
constexpr int kWideBM = 128;
__global__ __launch_bounds__(512) void hemm_bf16_wide_kernel(GemmArgs g) {
  constexpr int KP = 64, LD = KP + PADH;   // two MFMA K steps per panel
  __shared__ uint16_t As[4][kWideBM][LD];  // re_hi, im_hi, re_lo, im_lo of G' rows
  __shared__ uint16_t Bt[4][kWideBM][LD];  // the same of T columns: [n][k]
  const uint16_t* A = static_cast<const uint16_t*>(g.A);
  const uint16_t* B = static_cast<const uint16_t*>(g.B);
  const int64_t dd = int64_t(g.d) * g.d;
  const int ts = g.d / kWideBM;
  const int lb = int(xcd_order(blockIdx.x, gridDim.x));
  const int grp = lb / 32, within = lb % 32;
  const int tr = (grp / (ts / 8)) * 4 + within / 8;
  const int tc = (grp % (ts / 8)) * 8 + within % 8;
  const int64_t R0 = int64_t(tr) * kWideBM, C0 = int64_t(tc) * kWideBM;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 2, wc = w & 3;  // rows wr * 64 .., columns wc * 32 ..
  const int li = lane & 15, lq = lane >> 4;
  const int row = t >> 2, kq = (t & 3) * 16;  // 128 rows x 64 k per plane, 16 k per thread
  const int64_t oa = (R0 + row) * g.lda + kq, ob = (C0 + row) * g.ldb + kq;
  u16x8 xa[4][2], xb[4][2];
  f4 aR[4][2], aI[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) aR[i][j] = aI[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto load = [&](int kp) {
    const int64_t k0 = int64_t(kp) * KP;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        xa[pl][h] = *reinterpret_cast<const u16x8*>(A + pl * dd + oa + k0 + 8 * h);
        xb[pl][h] = *reinterpret_cast<const u16x8*>(B + pl * dd + ob + k0 + 8 * h);
      }
  };
  const int kIters = g.d / KP;
  load(0);
  for (int kp = 0; kp < kIters; ++kp) {
    __syncthreads();
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        *reinterpret_cast<u16x8*>(&As[pl][row][kq + 8 * h]) = xa[pl][h];
        *reinterpret_cast<u16x8*>(&Bt[pl][row][kq + 8 * h]) = xb[pl][h];
      }
    __syncthreads();
    if (kp + 1 < kIters) load(kp + 1);
#pragma unroll
    for (int ks = 0; ks < KP / 32; ++ks) {
      const int kk = ks * 32 + lq * 8;
      u16x8 b[2][4];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) b[j][pl] = *reinterpret_cast<const u16x8*>(&Bt[pl][wc * 32 + j * 16 + li][kk]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        u16x8 a[4];
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) a[pl] = *reinterpret_cast<const u16x8*>(&As[pl][wr * 64 + i * 16 + li][kk]);
        const u16x8 nih = bf16_neg(a[1]), nil = bf16_neg(a[3]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // complex: re = ar br - ai bi, im = ar bi + ai br;  hi*hi, hi*lo, lo*hi
          aR[i][j] = mfma_bf16(a[0], b[j][0], aR[i][j]);
          aR[i][j] = mfma_bf16(nih, b[j][1], aR[i][j]);
          aI[i][j] = mfma_bf16(a[0], b[j][1], aI[i][j]);
          aI[i][j] = mfma_bf16(a[1], b[j][0], aI[i][j]);
          aR[i][j] = mfma_bf16(a[0], b[j][2], aR[i][j]);
          aR[i][j] = mfma_bf16(nih, b[j][3], aR[i][j]);
          aI[i][j] = mfma_bf16(a[0], b[j][3], aI[i][j]);
          aI[i][j] = mfma_bf16(a[1], b[j][2], aI[i][j]);
          aR[i][j] = mfma_bf16(a[2], b[j][0], aR[i][j]);
          aR[i][j] = mfma_bf16(nil, b[j][1], aR[i][j]);
          aI[i][j] = mfma_bf16(a[2], b[j][1], aI[i][j]);
          aI[i][j] = mfma_bf16(a[3], b[j][0], aI[i][j]);
        }
      }
    }
  }
  double scale = 2.0 / *g.tau;
  if (g.up) scale *= *g.up;
  const float sc = float(scale);
  Cx<float>* C = static_cast<Cx<float>*>(g.C);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = C0 + wc * 32 + j * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = R0 + wr * 64 + i * 16 + 4 * lq + v;
        C[r * g.ldc + col] = Cx<float>{aR[i][j][v] * sc, aI[i][j][v] * sc};
      }
    }
}

}  // namespace

hipError_t launch_hemm(qst_prec prec, const void* G, int64_t ldg, const void* T, int64_t ldt, void* out,
                       int64_t ldo, int n, const double* tau_dev, const double* upstream_dev,
                       void* sk_partial, hipStream_t s, void* planes) {
  const int d = 1 << n;
  if (prec == QST_F32X6) {
    if (use_x6(prec, n)) return launch_x6_hemm(G, ldg, T, ldt, out, ldo, n, tau_dev, upstream_dev, planes, s);
    prec = QST_F32;
  }
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
  GemmArgs g{};
  g.A = G;
  g.lda = ldg;
  g.B = T;
  g.ldb = ldt;
  g.C = out;
  g.ldc = ldo;
  g.d = d;
  g.tau = tau_dev;
  g.up = upstream_dev;
  g.ntiles = tiles * tiles;
  g.partial = sk_partial;
  g.tau_part = nullptr;
  g.tau_out = nullptr;
  if (prec == QST_F64) return run_gemm<CxPolicy<double, false>>(g, s);
  if (prec == QST_F32) return run_gemm<CxPolicy<float, false>>(g, s);
  if (planes && d % (8 * kWideBM) == 0) {
    uint16_t* pg = static_cast<uint16_t*>(planes);
    uint16_t* pt = pg + 4 * int64_t(d) * d;
    split_planes_kernel<false><<<unsigned(tiles * tiles), 256, 0, s>>>(static_cast<const Cx<float>*>(G), ldg, d, pg);
    split_planes_kernel<true><<<unsigned(tiles * tiles), 256, 0, s>>>(static_cast<const Cx<float>*>(T), ldt, d, pt);
    g.A = pg;
    g.lda = d;
    g.B = pt;
    g.ldb = d;
    const int wt = d / kWideBM;
    hemm_bf16_wide_kernel<<<unsigned(wt * wt), 512, 0, s>>>(g);
    return hipGetLastError();
  }
  return run_gemm<HemmBf16x3Policy>(g, s);
}

}  // namespace qst
