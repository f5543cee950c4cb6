// MFMA micro-kernels of the complex products (T T^dagger and G' T) and the
// shared tile plumbing, used by the product kernels of k_gemm.hip and by the
// batched persistent kernel.  See k_gemm.hip for the tiling and scheduling.
#pragma once

#include "qst_device.h"
#include "qst_plan.h"
#include "qst_povm_rounds.h"

namespace qst {
namespace gemm {

constexpr int BM = 64;    // output tile (complex)
constexpr int PADC = 1;   // LDS row padding (complex elements), fp32/fp64 panels
constexpr int PADH = 8;   // LDS row padding (bf16 elements), bf16 panels
constexpr int TILE = BM * BM;

struct GemmArgs {
  const void* A;
  int64_t lda;
  const void* B;
  int64_t ldb;
  void* C;
  int64_t ldc;
  int d;
  const double* tau;
  const double* up;
  int ntiles;     // output tiles
  int kIters;     // K panels per tile
  int64_t iters;  // stream-K: K panels of the tiles from dp_tiles on
  int dp_tiles;   // stream-K: tiles [0, dp_tiles) are computed whole, one per workgroup and round
  void* partial;  // stream-K partial accumulators [P][2][2 * TILE] (acc scalar)
  const double* tau_part;  // HERK: FP64 partial sums of tau (kReduceBlocks), or NULL to read *tau
  double* tau_out;         // HERK with tau_part: where workgroup 0 stores tau
  // HERK with the first POVM pass in the epilogue (kernels instantiated with
  // X0; tetrahedral POVM): a finished tile of rho is not stored; the pass
  // over its x0g lowest qubits is applied to each of its 2^x0g x 2^x0g
  // sub-tiles and the lower ones go to x0 (the pass output X[(R, C)][k],
  // (R, C) over the x0up remaining qubits).
  void* x0;
  int x0g;
  int x0up;
};

// ---------------------------------------------------------------------------
// Policies: one K-panel loop per (precision, product) with a common
// accumulator shape acc[2][2] re/im, 4 values per lane.
// ---------------------------------------------------------------------------
// M3: three real products per complex product instead of four (Gauss):
// P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); re = P1 - P2,
// im = P3 - P1 - P2.  A quarter fewer MFMAs; the rounding error stays of the
// same order (a few units of eps * sqrt(K) * |A| |B|).  The combination is
// linear, so each K segment (stream-K) combines its own sums.
// DB: two LDS panel buffers (the next panel is stored into one while the
// MFMAs read the other: one barrier per panel step instead of two).  It
// pays where a workgroup's 256-thread groups share every barrier (the
// batched kernel: 0.63 -> 0.60 ms per batch) and costs where independent
// workgroups share a CU (the N = 11 products: 172 -> 167 TFLOP/s).
template <typename R, bool HERK, bool M3 = true, bool DB = false>
struct CxPolicy {
  typedef R scalar;
  typedef typename Mfma<R>::acc acc_t;
  static constexpr int KP = 16;  // complex K per panel
  static constexpr bool kHerk = HERK;
  // waves per SIMD the register allocation must allow (fp64 3M: 2, which
  // caps a lane at 256 registers; it would take 260 unconstrained)
  static constexpr int kMinWaves = 2;
  static constexpr bool kStreamK = true;
  struct Smem {
    Cx<R> As[DB ? 2 : 1][KP][BM + PADC];
    Cx<R> Bs[DB ? 2 : 1][KP][BM + PADC];
  };
  static __device__ __forceinline__ int row(int q, int v) { return Mfma<R>::row(q, v); }

  static __device__ __forceinline__ void run(const GemmArgs& g, Smem& sm, int tr, int tc, int kb, int ke,
                                             acc_t (&aR)[2][2], acc_t (&aI)[2][2]) {
    const Cx<R>* A = static_cast<const Cx<R>*>(g.A);
    const Cx<R>* B = static_cast<const Cx<R>*>(g.B);
    const int64_t R0 = int64_t(tr) * BM, C0 = int64_t(tc) * BM;
    const int t = threadIdx.x & 255;  // index in the 256-thread group computing the tile
    const int lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int li = lane & 15, lk = lane >> 4;
    const int a_row = t >> 2, a_k = (t & 3) * 4;   // A panel: 64 rows x 16 k
    const int hb_k = t >> 4, hb_n = (t & 15) * 4;  // HEMM B panel: 16 k x 64 n
    const Cx<R>* Ap = A + (R0 + a_row) * g.lda + a_k;
    const Cx<R>* Bp = HERK ? (B + (C0 + a_row) * g.ldb + a_k) : (B + int64_t(hb_k) * g.ldb + C0 + hb_n);
    // register prefetch of the next panel (written out, not via a lambda:
    // captured arrays would be kept in scratch memory)
    // (held as native 2-vectors: an aligned struct array would go to scratch)
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2* Av = reinterpret_cast<const v2*>(Ap);
    const v2* Bv = reinterpret_cast<const v2*>(Bp);
    v2 ra[4], rb[4];
#define QST_LOAD_PANEL(kp)                                                   \
  do {                                                                       \
    const int k0_ = (kp) * KP;                                               \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) ra[i] = Av[k0_ + i];       \
    if constexpr (HERK) {                                                    \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) rb[i] = Bv[k0_ + i];     \
    } else {                                                                 \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) rb[i] = Bv[int64_t(k0_) * g.ldb + i]; \
    }                                                                        \
  } while (0)
    // 3M sums (unused by the four-product form).  HERK uses P2' = Ai Bi'
    // with B' = T rows (B = conj B'^T): re = P1 + P2', im = P3 - P1 + P2',
    // P3 = (Ar + Ai)(Br' - Bi').
    acc_t p1[2][2], p2[2][2], p3[2][2];
    if constexpr (M3) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) p1[i][j] = p2[i][j] = p3[i][j] = acc_t{0, 0, 0, 0};
    }
#define QST_STORE_PANEL(buf)                                                                  \
  do {                                                                                        \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) sm.As[buf][a_k + i][a_row] = Cx<R>{ra[i].x, ra[i].y}; \
    if constexpr (HERK) {                                                                     \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) sm.Bs[buf][a_k + i][a_row] = Cx<R>{rb[i].x, rb[i].y}; \
    } else {                                                                                  \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) sm.Bs[buf][hb_k][hb_n + i] = Cx<R>{rb[i].x, rb[i].y}; \
    }                                                                                         \
  } while (0)
    QST_LOAD_PANEL(kb);
    if constexpr (DB) {
      __syncthreads();  // the previous user of the LDS (an epilogue) is done
      QST_STORE_PANEL(0);
      __syncthreads();
    }
    for (int kp = kb; kp < ke; ++kp) {
      int cur = 0;
      if constexpr (DB) {
        cur = (kp - kb) & 1;
      } else {
        __syncthreads();
        QST_STORE_PANEL(0);
        __syncthreads();
      }
      if (kp + 1 < ke) QST_LOAD_PANEL(kp + 1);
#undef QST_LOAD_PANEL
      // operands of the next K step are read from LDS before the MFMAs of
      // the current one, so the LDS latency overlaps them
      Cx<R> an[2], bn[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) an[i] = sm.As[cur][lk][wr * 32 + i * 16 + li];
#pragma unroll
      for (int j = 0; j < 2; ++j) bn[j] = sm.Bs[cur][lk][wc * 32 + j * 16 + li];
#pragma unroll
      for (int ks = 0; ks < KP / 4; ++ks) {
        Cx<R> a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = an[i];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = bn[j];
        if (ks + 1 < KP / 4) {
          const int kn = (ks + 1) * 4 + lk;
#pragma unroll
          for (int i = 0; i < 2; ++i) an[i] = sm.As[cur][kn][wr * 32 + i * 16 + li];
#pragma unroll
          for (int j = 0; j < 2; ++j) bn[j] = sm.Bs[cur][kn][wc * 32 + j * 16 + li];
          __builtin_amdgcn_sched_barrier(0);  // keep these reads ahead of the MFMAs below
        }
        if constexpr (M3) {
          R as[2], bs[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) as[i] = a[i].re + a[i].im;
#pragma unroll
          for (int j = 0; j < 2; ++j) bs[j] = HERK ? b[j].re - b[j].im : b[j].re + b[j].im;
          // twelve independent accumulator chains
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) p1[i][j] = Mfma<R>::step(a[i].re, b[j].re, p1[i][j]);
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) p2[i][j] = Mfma<R>::step(a[i].im, b[j].im, p2[i][j]);
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) p3[i][j] = Mfma<R>::step(as[i], bs[j], p3[i][j]);
        } else {
          // eight independent accumulator chains, each advanced once per sweep
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              aR[i][j] = Mfma<R>::step(a[i].re, b[j].re, aR[i][j]);
              aI[i][j] = Mfma<R>::step(HERK ? a[i].im : a[i].re, HERK ? b[j].re : b[j].im, aI[i][j]);
            }
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              // HERK: re += ai bi, im -= ar bi;  HEMM: re -= ai bi, im += ai br
              aR[i][j] = Mfma<R>::step(HERK ? a[i].im : -a[i].im, b[j].im, aR[i][j]);
              aI[i][j] = Mfma<R>::step(HERK ? -a[i].re : a[i].im, HERK ? b[j].im : b[j].re, aI[i][j]);
            }
        }
      }
      if constexpr (DB) {
        if (kp + 1 < ke) QST_STORE_PANEL(cur ^ 1);
        __syncthreads();
      }
    }
#undef QST_STORE_PANEL
    if constexpr (M3) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // callers pass zeroed accumulators: assign rather than add
          if constexpr (HERK) {
            aR[i][j] = p1[i][j] + p2[i][j];
            aI[i][j] = (p3[i][j] - p1[i][j]) + p2[i][j];
          } else {
            aR[i][j] = p1[i][j] - p2[i][j];
            aI[i][j] = (p3[i][j] - p1[i][j]) - p2[i][j];
          }
        }
    }
  }
};

// T T^dagger with T rounded to bf16 (RNE), fp32 accumulate.
struct HerkBf16Policy {
  static constexpr int kMinWaves = 1;
  typedef float scalar;
  typedef f4 acc_t;
  static constexpr int KP = 32;  // one MFMA K step
  static constexpr bool kHerk = true;
  static constexpr bool kStreamK = false;  // load-bound: splitting K only adds partial traffic
  struct Smem {
    uint16_t Ar[BM][KP + PADH], Ai[BM][KP + PADH], Br[BM][KP + PADH], Bi[BM][KP + PADH];
  };
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }

  static __device__ __forceinline__ void run(const GemmArgs& g, Smem& sm, int tr, int tc, int kb, int ke,
                                             acc_t (&aR)[2][2], acc_t (&aI)[2][2]) {
    const Cx<float>* T = static_cast<const Cx<float>*>(g.A);
    const int64_t R0 = int64_t(tr) * BM, C0 = int64_t(tc) * BM;
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int li = lane & 15, lq = lane >> 4;
    const int row = t >> 2, kq = (t & 3) * 8;  // 64 rows x 32 k, 8 complex per thread
    const Cx<float>* Ap = T + (R0 + row) * g.lda + kq;
    const Cx<float>* Bp = T + (C0 + row) * g.lda + kq;
    Cx<float> ra[8], rb[8];
#define QST_LOAD_PANEL(kp)                                 \
  do {                                                     \
    const int k0_ = (kp) * KP;                             \
    _Pragma("unroll") for (int i = 0; i < 8; ++i) {        \
      ra[i] = Ap[k0_ + i];                                 \
      rb[i] = Bp[k0_ + i];                                 \
    }                                                      \
  } while (0)
    QST_LOAD_PANEL(kb);
    for (int kp = kb; kp < ke; ++kp) {
      __syncthreads();
      {
        float xr[8], xi[8], yr[8], yi[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          xr[i] = ra[i].re;
          xi[i] = ra[i].im;
          yr[i] = rb[i].re;
          yi[i] = rb[i].im;
        }
        *reinterpret_cast<u16x8*>(&sm.Ar[row][kq]) = bf16x8(xr);
        *reinterpret_cast<u16x8*>(&sm.Ai[row][kq]) = bf16x8(xi);
        *reinterpret_cast<u16x8*>(&sm.Br[row][kq]) = bf16x8(yr);
        *reinterpret_cast<u16x8*>(&sm.Bi[row][kq]) = bf16x8(yi);
      }
      __syncthreads();
      if (kp + 1 < ke) QST_LOAD_PANEL(kp + 1);
#undef QST_LOAD_PANEL
      u16x8 a_r[2], a_i[2], b_r[2], b_i[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a_r[i] = *reinterpret_cast<const u16x8*>(&sm.Ar[wr * 32 + i * 16 + li][lq * 8]);
        a_i[i] = *reinterpret_cast<const u16x8*>(&sm.Ai[wr * 32 + i * 16 + li][lq * 8]);
        b_r[i] = *reinterpret_cast<const u16x8*>(&sm.Br[wc * 32 + i * 16 + li][lq * 8]);
        b_i[i] = *reinterpret_cast<const u16x8*>(&sm.Bi[wc * 32 + i * 16 + li][lq * 8]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          aR[i][j] = mfma_bf16(a_r[i], b_r[j], aR[i][j]);
          aI[i][j] = mfma_bf16(a_i[i], b_r[j], aI[i][j]);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const u16x8 na = bf16_neg(a_r[i]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          aR[i][j] = mfma_bf16(a_i[i], b_i[j], aR[i][j]);
          aI[i][j] = mfma_bf16(na, b_i[j], aI[i][j]);
        }
      }
    }
  }
};

// T T^dagger from bf16 planes of T (a re plane and an im plane, d x d
// row-major each, g.A = the re plane, g.lda = d; written by the tau kernel):
// no conversion inside the product and half the operand bytes of fp32 T.
// Panels of 64 k (two MFMA K steps between barriers), fp32 accumulate.
struct HerkBf16PlanesPolicy {
  static constexpr int kMinWaves = 1;
  typedef float scalar;
  typedef f4 acc_t;
  static constexpr int KP = 64;
  static constexpr bool kHerk = true;
  static constexpr bool kStreamK = false;
  struct Smem {
    uint16_t Ar[BM][KP + PADH], Ai[BM][KP + PADH], Br[BM][KP + PADH], Bi[BM][KP + PADH];
  };
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }

  static __device__ __forceinline__ void run(const GemmArgs& g, Smem& sm, int tr, int tc, int kb, int ke,
                                             acc_t (&aR)[2][2], acc_t (&aI)[2][2]) {
    const uint16_t* Pr = static_cast<const uint16_t*>(g.A);
    const uint16_t* Pi = Pr + int64_t(g.d) * g.d;
    const int64_t R0 = int64_t(tr) * BM, C0 = int64_t(tc) * BM;
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int li = lane & 15, lq = lane >> 4;
    const int row = t >> 2, kq = (t & 3) * 16;  // 64 rows x 64 k per plane, 16 k per thread
    const int64_t oa = (R0 + row) * g.lda + kq, ob = (C0 + row) * g.lda + kq;
    u16x8 xr[2], xi[2], yr[2], yi[2];
#define QST_LOAD_PANEL(kp)                                                   \
  do {                                                                       \
    const int64_t k0_ = int64_t(kp) * KP;                                    \
    _Pragma("unroll") for (int h = 0; h < 2; ++h) {                          \
      xr[h] = *reinterpret_cast<const u16x8*>(Pr + oa + k0_ + 8 * h);        \
      xi[h] = *reinterpret_cast<const u16x8*>(Pi + oa + k0_ + 8 * h);        \
      yr[h] = *reinterpret_cast<const u16x8*>(Pr + ob + k0_ + 8 * h);        \
      yi[h] = *reinterpret_cast<const u16x8*>(Pi + ob + k0_ + 8 * h);        \
    }                                                                        \
  } while (0)
    QST_LOAD_PANEL(kb);
    for (int kp = kb; kp < ke; ++kp) {
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        *reinterpret_cast<u16x8*>(&sm.Ar[row][kq + 8 * h]) = xr[h];
        *reinterpret_cast<u16x8*>(&sm.Ai[row][kq + 8 * h]) = xi[h];
        *reinterpret_cast<u16x8*>(&sm.Br[row][kq + 8 * h]) = yr[h];
        *reinterpret_cast<u16x8*>(&sm.Bi[row][kq + 8 * h]) = yi[h];
      }
      __syncthreads();
      if (kp + 1 < ke) QST_LOAD_PANEL(kp + 1);
#undef QST_LOAD_PANEL
#pragma unroll
      for (int ks = 0; ks < KP / 32; ++ks) {
        u16x8 a_r[2], a_i[2], b_r[2], b_i[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a_r[i] = *reinterpret_cast<const u16x8*>(&sm.Ar[wr * 32 + i * 16 + li][ks * 32 + lq * 8]);
          a_i[i] = *reinterpret_cast<const u16x8*>(&sm.Ai[wr * 32 + i * 16 + li][ks * 32 + lq * 8]);
          b_r[i] = *reinterpret_cast<const u16x8*>(&sm.Br[wc * 32 + i * 16 + li][ks * 32 + lq * 8]);
          b_i[i] = *reinterpret_cast<const u16x8*>(&sm.Bi[wc * 32 + i * 16 + li][ks * 32 + lq * 8]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            aR[i][j] = mfma_bf16(a_r[i], b_r[j], aR[i][j]);
            aI[i][j] = mfma_bf16(a_i[i], b_r[j], aI[i][j]);
          }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const u16x8 na = bf16_neg(a_r[i]);
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            aR[i][j] = mfma_bf16(a_i[i], b_i[j], aR[i][j]);
            aI[i][j] = mfma_bf16(na, b_i[j], aI[i][j]);
          }
        }
      }
    }
  }
};

// Eight consecutive complex values -> their re_hi, im_hi, re_lo, im_lo
// bf16 planes at P[plane][row][k0..k0+7] (16-byte stores).
template <int LD>
__device__ __forceinline__ void split_store_planes(uint16_t (*P)[BM][LD], int row, int k0, const Cx<float> (&v)[8]) {
  float re[8], im[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    re[i] = v[i].re;
    im[i] = v[i].im;
  }
  u16x8 h0, h1, l0, l1;
  bf16x8_split(re, h0, l0);
  bf16x8_split(im, h1, l1);
  *reinterpret_cast<u16x8*>(&P[0][row][k0]) = h0;
  *reinterpret_cast<u16x8*>(&P[1][row][k0]) = h1;
  *reinterpret_cast<u16x8*>(&P[2][row][k0]) = l0;
  *reinterpret_cast<u16x8*>(&P[3][row][k0]) = l1;
}

// T T^dagger with T split into bf16 hi + lo (three products: hi hi^dagger +
// hi lo^dagger + lo hi^dagger), fp32 accumulate.  Used for small d, where the
// rounding of plain bf16 T moves the gradient by more than the BF16 bar.
struct HerkBf16x3Policy {
  static constexpr int kMinWaves = 1;
  typedef float scalar;
  typedef f4 acc_t;
  static constexpr int KP = 32;
  static constexpr bool kHerk = true;
  static constexpr bool kStreamK = false;
  struct Smem {
    uint16_t A[4][BM][KP + PADH];  // re_hi, im_hi, re_lo, im_lo of the row block
    uint16_t B[4][BM][KP + PADH];  // same for the column block
  };
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }

  static __device__ __forceinline__ void split_store(uint16_t (*P)[BM][KP + PADH], int row, int kq,
                                                     const Cx<float> (&v)[8]) {
    split_store_planes(P, row, kq, v);
  }

  static __device__ __forceinline__ void run(const GemmArgs& g, Smem& sm, int tr, int tc, int kb, int ke,
                                             acc_t (&aR)[2][2], acc_t (&aI)[2][2]) {
    const Cx<float>* T = static_cast<const Cx<float>*>(g.A);
    const int64_t R0 = int64_t(tr) * BM, C0 = int64_t(tc) * BM;
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int li = lane & 15, lq = lane >> 4;
    const int row = t >> 2, kq = (t & 3) * 8;
    const Cx<float>* Ap = T + (R0 + row) * g.lda + kq;
    const Cx<float>* Bp = T + (C0 + row) * g.lda + kq;
    Cx<float> ra[8], rb[8];
#define QST_LOAD_PANEL(kp)                                 \
  do {                                                     \
    const int k0_ = (kp) * KP;                             \
    _Pragma("unroll") for (int i = 0; i < 8; ++i) {        \
      ra[i] = Ap[k0_ + i];                                 \
      rb[i] = Bp[k0_ + i];                                 \
    }                                                      \
  } while (0)
    QST_LOAD_PANEL(kb);
    for (int kp = kb; kp < ke; ++kp) {
      __syncthreads();
      split_store(sm.A, row, kq, ra);
      split_store(sm.B, row, kq, rb);
      __syncthreads();
      if (kp + 1 < ke) QST_LOAD_PANEL(kp + 1);
#undef QST_LOAD_PANEL
      u16x8 a[2][4], b[2][4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) {
          a[i][pl] = *reinterpret_cast<const u16x8*>(&sm.A[pl][wr * 32 + i * 16 + li][lq * 8]);
          b[i][pl] = *reinterpret_cast<const u16x8*>(&sm.B[pl][wc * 32 + i * 16 + li][lq * 8]);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const u16x8 nrh = bf16_neg(a[i][0]), nrl = bf16_neg(a[i][2]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // A B^dagger: re = ar br + ai bi, im = ai br - ar bi;  hi*hi, hi*lo, lo*hi
          aR[i][j] = mfma_bf16(a[i][0], b[j][0], aR[i][j]);
          aI[i][j] = mfma_bf16(a[i][1], b[j][0], aI[i][j]);
          aR[i][j] = mfma_bf16(a[i][1], b[j][1], aR[i][j]);
          aI[i][j] = mfma_bf16(nrh, b[j][1], aI[i][j]);
          aR[i][j] = mfma_bf16(a[i][0], b[j][2], aR[i][j]);
          aI[i][j] = mfma_bf16(a[i][1], b[j][2], aI[i][j]);
          aR[i][j] = mfma_bf16(a[i][1], b[j][3], aR[i][j]);
          aI[i][j] = mfma_bf16(nrh, b[j][3], aI[i][j]);
          aR[i][j] = mfma_bf16(a[i][2], b[j][0], aR[i][j]);
          aI[i][j] = mfma_bf16(a[i][3], b[j][0], aI[i][j]);
          aR[i][j] = mfma_bf16(a[i][3], b[j][1], aR[i][j]);
          aI[i][j] = mfma_bf16(nrl, b[j][1], aI[i][j]);
        }
      }
    }
  }
};

// G' T with split-bf16 operands: x = hi + lo, hi = bf16(x), lo = bf16(x - hi);
// the product keeps hi*hi + hi*lo + lo*hi (lo*lo is below fp32 rounding).
struct HemmBf16x3Policy {
  static constexpr int kMinWaves = 1;
  typedef float scalar;
  typedef f4 acc_t;
  static constexpr int KP = 32;
  static constexpr bool kHerk = false;
  static constexpr bool kStreamK = true;
  struct Smem {
    uint16_t As[4][BM][KP + PADH];  // re_hi, im_hi, re_lo, im_lo
    uint16_t Bt[4][BM][KP + PADH];  // transposed: [n][k]
  };
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }

  static __device__ __forceinline__ void run(const GemmArgs& g, Smem& sm, int tr, int tc, int kb, int ke,
                                             acc_t (&aR)[2][2], acc_t (&aI)[2][2]) {
    const Cx<float>* G = static_cast<const Cx<float>*>(g.A);
    const Cx<float>* T = static_cast<const Cx<float>*>(g.B);
    const int64_t R0 = int64_t(tr) * BM, C0 = int64_t(tc) * BM;
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int li = lane & 15, lq = lane >> 4;
    const int a_row = t >> 2, a_k = (t & 3) * 8;  // A panel: 64 rows x 32 k, 8 consecutive k per thread
    const int b_n = t & 63, b_k = (t >> 6) * 8;   // B panel: 32 k x 64 n, 8 consecutive k of one column
    const Cx<float>* Ap = G + (R0 + a_row) * g.lda + a_k;
    const Cx<float>* Bp = T + int64_t(b_k) * g.ldb + C0 + b_n;
    Cx<float> ra[8], rb[8];
#define QST_LOAD_PANEL(kp)                                 \
  do {                                                     \
    const int k0_ = (kp) * KP;                             \
    _Pragma("unroll") for (int i = 0; i < 8; ++i) {        \
      ra[i] = Ap[k0_ + i];                                 \
      rb[i] = Bp[int64_t(k0_ + i) * g.ldb];                \
    }                                                      \
  } while (0)
    QST_LOAD_PANEL(kb);
    for (int kp = kb; kp < ke; ++kp) {
      __syncthreads();
      split_store_planes(sm.As, a_row, a_k, ra);
      split_store_planes(sm.Bt, b_n, b_k, rb);
      __syncthreads();
      if (kp + 1 < ke) QST_LOAD_PANEL(kp + 1);
#undef QST_LOAD_PANEL
      u16x8 a[2][4], b[2][4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) {
          a[i][pl] = *reinterpret_cast<const u16x8*>(&sm.As[pl][wr * 32 + i * 16 + li][lq * 8]);
          b[i][pl] = *reinterpret_cast<const u16x8*>(&sm.Bt[pl][wc * 32 + i * 16 + li][lq * 8]);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const u16x8 nih = bf16_neg(a[i][1]), nil = bf16_neg(a[i][3]);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // complex: re = ar br - ai bi, im = ar bi + ai br;  hi*hi, hi*lo, lo*hi
          aR[i][j] = mfma_bf16(a[i][0], b[j][0], aR[i][j]);
          aR[i][j] = mfma_bf16(nih, b[j][1], aR[i][j]);
          aI[i][j] = mfma_bf16(a[i][0], b[j][1], aI[i][j]);
          aI[i][j] = mfma_bf16(a[i][1], b[j][0], aI[i][j]);
          aR[i][j] = mfma_bf16(a[i][0], b[j][2], aR[i][j]);
          aR[i][j] = mfma_bf16(nih, b[j][3], aR[i][j]);
          aI[i][j] = mfma_bf16(a[i][0], b[j][3], aI[i][j]);
          aI[i][j] = mfma_bf16(a[i][1], b[j][2], aI[i][j]);
          aR[i][j] = mfma_bf16(a[i][2], b[j][0], aR[i][j]);
          aR[i][j] = mfma_bf16(nil, b[j][1], aR[i][j]);
          aI[i][j] = mfma_bf16(a[i][2], b[j][1], aI[i][j]);
          aI[i][j] = mfma_bf16(a[i][3], b[j][0], aI[i][j]);
        }
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Shared tile plumbing
// ---------------------------------------------------------------------------
template <class P>
__device__ __forceinline__ void tile_coords(const GemmArgs& g, int tile, int& tr, int& tc) {
  if constexpr (P::kHerk) {
    tri_decode(tile, tr, tc);
  } else {
    const int tiles = g.d / BM;
    tr = tile / tiles;
    tc = tile % tiles;
  }
}

template <class P>
__device__ __forceinline__ void zero_acc(typename P::acc_t (&aR)[2][2], typename P::acc_t (&aI)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      aR[i][j] = typename P::acc_t{0, 0, 0, 0};
      aI[i][j] = typename P::acc_t{0, 0, 0, 0};
    }
}

// Output scale, evaluated by every workgroup at its start: 1/tau for
// T T^dagger, s * 2/tau for G' T.  With tau partials, tau is their sum in a
// fixed order (bitwise the same in every workgroup), and workgroup 0 stores it.
template <class P>
__device__ double tile_scale(const GemmArgs& g) {
  double tau;
  if (g.tau_part) {
    __shared__ double red[4];
    __shared__ double bcast;
    double acc = 0.0;
    for (int b = threadIdx.x; b < kReduceBlocks; b += blockDim.x) acc += g.tau_part[b];
    const double sum = block_sum256(acc, red);
    if (threadIdx.x == 0) {
      bcast = sum;
      if (blockIdx.x == 0 && g.tau_out) *g.tau_out = sum;
    }
    __syncthreads();
    tau = bcast;
  } else {
    tau = *g.tau;
  }
  if constexpr (P::kHerk) {
    return 1.0 / tau;
  } else {
    double s = 2.0 / tau;
    if (g.up) s *= *g.up;
    return s;
  }
}

template <class P>
__device__ __forceinline__ void epilogue(const GemmArgs& g, int tr, int tc, typename P::acc_t (&aR)[2][2],
                                         typename P::acc_t (&aI)[2][2], double scale) {
  typedef typename P::scalar R;
  Cx<R>* C = static_cast<Cx<R>*>(g.C);
  const R sc = R(scale);
  const int lane = threadIdx.x & 63, w = (threadIdx.x & 255) >> 6;  // 256-thread group
  const int wr = w >> 1, wc = w & 1, li = lane & 15, lq = lane >> 4;
  const int64_t R0 = int64_t(tr) * BM, C0 = int64_t(tc) * BM;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = C0 + wc * 32 + j * 16 + li;
      const int64_t rbase = R0 + wr * 32 + i * 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = rbase + P::row(lq, v);
        C[row * g.ldc + col] = Cx<R>{aR[i][j][v] * sc, aI[i][j][v] * sc};
        if (P::kHerk && tr != tc) C[col * g.ldc + row] = Cx<R>{aR[i][j][v] * sc, -aI[i][j][v] * sc};
      }
    }
  }
}

// The tetrahedral fast form reads no mode matrix; this one only fills the
// parameter.
static __constant__ ModeMatrix kTetraNoMatrix = {};

// The first POVM pass over the 2^G x 2^G sub-tiles of a BM x BM tile of rho
// at tile coordinates (tr, tc), held in lds in the sub-tile-major swizzled
// layout lds[((r >> G) * S + (c >> G)) * 4^G + swz<G>(r & M, c & M)], by the
// 256 threads of the workgroup (4^(G-2) per sub-tile); the lower sub-tiles
// (Rhi >= Chi) go to g.x0.  Contains barriers.
template <typename R, int G>
__device__ __forceinline__ void x0_rounds(const GemmArgs& g, int64_t tr, int64_t tc, Cx<R>* lds) {
  constexpr int S = BM >> G;
  constexpr int TG = 1 << (2 * G);
  constexpr int NT = 1 << (2 * (G - 2));
  const int tl = (threadIdx.x & 255) / NT, t = (threadIdx.x & 255) % NT;
  const int64_t Rhi = tr * S + tl / S, Chi = tc * S + tl % S;
  Cx<R>* L = lds + tl * TG;
  const int bq = t & ((1 << (G - 2)) - 1), aq = t >> (G - 2);
  Cx<R> x[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) x[m] = L[swz<G>(4 * aq + blk_ri(m), 4 * bq + blk_ci(m))];
  Cx<R>* out = Rhi >= Chi ? static_cast<Cx<R>*>(g.x0) + ((Rhi << g.x0up) | Chi) * int64_t(TG) : nullptr;
  mat_fwd_rounds<R, true, G>(x, L, t, kTetraNoMatrix, out);
}

// First POVM pass applied to a finished T T^dagger tile (see GemmArgs::x0).
// lds: BM x BM complex values of the workgroup's shared memory (aliasing the
// panel buffers, which the caller no longer reads).
template <class P, int G>
__device__ __forceinline__ void x0_tile(const GemmArgs& g, int tr, int tc, typename P::acc_t (&aR)[2][2],
                                        typename P::acc_t (&aI)[2][2], double scale,
                                        Cx<typename P::scalar>* lds) {
  typedef typename P::scalar R;
  constexpr int S = BM >> G;             // sub-tiles per side
  constexpr int TG = 1 << (2 * G);       // values per sub-tile
  constexpr int NT = 1 << (2 * (G - 2)); // threads per sub-tile
  constexpr int M = (1 << G) - 1;
  const R sc = R(scale);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1, li = lane & 15, lq = lane >> 4;
  __syncthreads();  // every wave is done with the panel buffers
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = wc * 32 + j * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr * 32 + i * 16 + P::row(lq, v);
        lds[((r >> G) * S + (c >> G)) * TG + swz<G>(r & M, c & M)] = Cx<R>{aR[i][j][v] * sc, aI[i][j][v] * sc};
      }
    }
  __syncthreads();
  x0_rounds<R, G>(g, tr, tc, lds);
}

// Shared memory of a product kernel: the policy's panel buffers, and with
// X0 at least one BM x BM complex tile for the POVM epilogue.
template <class P, bool X0>
constexpr size_t smem_bytes() {
  return (X0 && size_t(BM) * BM * sizeof(Cx<typename P::scalar>) > sizeof(typename P::Smem))
             ? size_t(BM) * BM * sizeof(Cx<typename P::scalar>)
             : sizeof(typename P::Smem);
}

// Partial accumulators of one tile segment, stored per lane in the MFMA
// layout: element ((((w*2 + i)*2 + j)*2 + part)*4 + v)*64 + lane.
template <class P>
__device__ __forceinline__ typename P::scalar* partial_slot(const GemmArgs& g, int wg, int which) {
  return static_cast<typename P::scalar*>(g.partial) + (int64_t(wg) * 2 + which) * int64_t(2 * TILE);
}

template <class P>
__device__ __forceinline__ void store_partial(typename P::scalar* dst, typename P::acc_t (&aR)[2][2],
                                              typename P::acc_t (&aI)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        dst[((((w * 2 + i) * 2 + j) * 2 + 0) * 4 + v) * 64 + lane] = aR[i][j][v];
        dst[((((w * 2 + i) * 2 + j) * 2 + 1) * 4 + v) * 64 + lane] = aI[i][j][v];
      }
}

// NB partial tiles at once: all NB are loaded before any is added (one
// memory round trip for the group), then added in the order src[0], src[1], ...
template <class P, int NB>
__device__ __forceinline__ void add_partials(const typename P::scalar* const (&src)[NB],
                                             typename P::acc_t (&aR)[2][2], typename P::acc_t (&aI)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  typename P::acc_t bR[NB][2][2], bI[NB][2][2];
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int o = (((w * 2 + i) * 2 + j) * 2 * 4 + v) * 64 + lane;
          bR[q][i][j][v] = src[q][o];
          bI[q][i][j][v] = src[q][o + 4 * 64];
        }
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          aR[i][j][v] += bR[q][i][j][v];
          aI[i][j][v] += bI[q][i][j][v];
        }
}

template <class P>
__device__ __forceinline__ void add_partial(const typename P::scalar* src, typename P::acc_t (&aR)[2][2],
                                            typename P::acc_t (&aI)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        aR[i][j][v] += src[((((w * 2 + i) * 2 + j) * 2 + 0) * 4 + v) * 64 + lane];
        aI[i][j][v] += src[((((w * 2 + i) * 2 + j) * 2 + 1) * 4 + v) * 64 + lane];
      }
}

}  // namespace gemm
}  // namespace qst
