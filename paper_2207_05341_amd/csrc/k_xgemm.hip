// Complex products of the QST_F32X6 path: FP32 operands, every real product
// computed on the BF16 matrix cores from a three-way split of each operand.
//
//   state map  rho = T T^dagger / tau      (Eq. T_matrix; Eq. unified_DP)
//   gradient   grad = s (2 / tau) G' T     (adjoint of the state map)
//
// Split: x = h + m + l with h = bf16(x), m = bf16(x - h), l = bf16(x - h - m)
// (round to nearest even).  For an FP32 x this is exact: h takes the top 8
// significand bits, m the next 8 and l the last 8, and every difference is
// exact in FP32.  A real product a b then keeps the six partial products
// hh + hm + mh + hl + lh + mm, each exact in FP32; the three dropped ones
// (ml, lm, ll) are below 2^-26 |a||b|, under the FP32 rounding of the
// accumulation itself.  Accumulation is in FP32 inside the MFMA, as in the
// QST_F32 products.
//
// Complex products use three real products (3M form): for C = A B,
// P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi), re = P1 - P2,
// im = P3 - P1 - P2; for S = T T^dagger (B = conj(T) rows),
// P1 = Tr Tr^T, P2 = Ti Ti^T, P3 = (Tr + Ti)(Tr - Ti)^T, re = P1 + P2,
// im = P3 - P1 + P2.  The sums are formed in FP32 before the split.
//
// Operand planes.  A split pass writes each operand once per call as bf16
// planes in the order the v_mfma_f32_32x32x16_bf16 fragments read them: a
// 1 KB unit holds a 32-row x 16-k block of one plane, 16 bytes per lane
// (lane u: row u % 32, k 8 (u / 32) .. + 7), and the units of one (row
// block, K panel) for all groups (re, im, re + im, re - im) and splits
// (h, m, l) are contiguous: unit ((rb * (K / 16) + kb) * NG + g) * 3 + s.
//
// Product kernel: a 128 x 128 complex output tile per 256-thread workgroup
// (four waves of 64 x 64, 2 x 2 MFMA blocks of 32 x 32 each, three
// accumulator sets P1, P2, P3).  The K loop runs over "slabs": one real
// product's three splits of A and B for one 16-deep K panel (24 units,
// 24 KB).  Slabs are copied global -> LDS by the DMA form of the global
// load (no registers), five slabs ahead, into a ring of six LDS slots
// (144 KB); the fragments of slab s+1 are read while the 24 MFMAs of slab s
// run (two MFMAs, one fragment read and one DMA per step).
//
// T T^dagger computes the lower 128 x 128 tiles only (136 at d = 2048),
// which do not divide evenly over the compute units, so it runs stream-K:
// each workgroup takes an equal contiguous share of the (tile, panel)
// sequence; a tile cut between workgroups leaves partial sums (at most two
// per workgroup) that a fix-up kernel adds in K order (deterministic) before
// the tile's epilogue (rho, or the first POVM pass).  G' T has (d / 128)^2
// tiles, one per workgroup, numbered so that each XCD runs 4 x 8 blocks of
// tiles.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "qst_device.h"
#include "qst_gemm_tiles.h"
#include "qst_kernels.h"
#include "qst_plan.h"
#include "qst_split.h"

namespace qst {

namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void_t;

constexpr int XT = kX6Tile;               // output tile (complex)
constexpr int XSLOT = 24 * 1024;          // one slab
constexpr int XNSLOT = 6;                 // LDS ring slots
constexpr int XDIST = 5;                  // slabs loaded ahead of the one being computed
constexpr int XLDS = XSLOT * XNSLOT;      // 147456 bytes of LDS
constexpr int XUNIT = 64;                 // 16-byte vectors per 1 KB unit

static_assert((XDIST - 2) * 6 < 64, "vmcnt immediate");

// ---------------------------------------------------------------------------
// Split (helpers in qst_split.h)
// ---------------------------------------------------------------------------
// Planes of a d x d complex FP32 matrix X (leading dimension ld) as the
// row operand (TRANS false: row r, k = column) or as the rows of X^T (TRANS
// true: row r = column of X, k = row of X).  Groups: re, im, re + im, and
// with NG = 4 also re - im.  One wave per unit block (32 rows x 16 k): lane
// u converts the 8 values of its fragment slot; each plane's unit is one
// coalesced 1 KB store of the wave.
template <bool TRANS, int NG>
__global__ __launch_bounds__(256) void x6_split_kernel(const Cx<float>* __restrict__ X, int64_t ld, int d,
                                                       u16x8* __restrict__ P) {
  const int64_t blk = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);  // unit block (rb, kb)
  const int lane = threadIdx.x & 63;
  const int nkb = d / 16;
  if (blk >= int64_t(d / 32) * nkb) return;
  const int64_t rb = blk / nkb, kb = blk % nkb;
  const int64_t row = rb * 32 + (lane & 31);
  const int64_t k0 = kb * 16 + 8 * (lane >> 5);
  float re[8], im[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const Cx<float> v = TRANS ? X[(k0 + e) * ld + row] : X[row * ld + k0 + e];
    re[e] = v.re;
    im[e] = v.im;
  }
  write_unit_block<NG>(P + blk * (NG * 3 * XUNIT) + lane, re, im);
}

// The planes of T as the row operand of T T^dagger (groups re, im, re + im,
// re - im) and, with TT, of T^T as the column operand of G' T (re, im,
// re + im), with the FP64 partial sums of tau = sum |T_ij|^2 and, with f,
// of F = sum_k f_k: workgroup b of nb writes partials[b] (its 32 x 32
// blocks b, b + nb, ..., four per pass, one per wave) and partials[nb + b]
// (f over [b D / nb, (b + 1) D / nb), D = d^2), each summed in a fixed
// order, so that T is read once.  A wave reads its block as the slots of
// two row-operand unit blocks (lane u: row u % 32, columns 16 h + 8 (u / 32)
// .. + 7, h = 0, 1); with TT it passes the block through LDS (8 KB per
// wave, 16-byte chunks swizzled by row) and reads the two unit blocks of
// T^T (lane u: column u % 32, rows 16 h + 8 (u / 32) .. + 7).  The first 16
// values of f per thread are loaded first, so that their loads are in
// flight together with those of T.
__device__ __forceinline__ int split_swz(int r, int c) {  // (r, c) of a 32 x 32 block, complex index
  return r * 32 + 2 * (((c >> 1) ^ r) & 15) + (c & 1);
}

template <bool WITH_F, bool TT>
__global__ __launch_bounds__(256) void x6_split_tau_kernel(const Cx<float>* __restrict__ X, int64_t ld, int d,
                                                           u16x8* __restrict__ P, u16x8* __restrict__ PT,
                                                           double* __restrict__ partials,
                                                           const float* __restrict__ f) {
  constexpr int NT = 256, NW = NT / 64, U = 16;
  __shared__ double red[NW];
  __shared__ Cx<float> blkL[TT ? NW : 1][TT ? 32 * 32 : 1];
  const int nb = gridDim.x;
  const int64_t D = int64_t(d) * d;
  const int64_t fbeg = D * blockIdx.x / nb, fend = D * (blockIdx.x + 1) / nb;
  float fv[U];
  if constexpr (WITH_F) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = fbeg + threadIdx.x + u * NT;
      fv[u] = e < fend ? f[e] : 0.f;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = lane & 31, hq = lane >> 5;
  const int nkb = d / 16, nb32 = d / 32;
  const int64_t nblk = int64_t(nb32) * nb32;
  double acc = 0.0, accf = 0.0;
  // the loop bound is the same for the whole workgroup (barriers inside)
  for (int64_t b0 = int64_t(blockIdx.x) * NW; b0 < nblk; b0 += int64_t(nb) * NW) {
    const int64_t blk = b0 + wv;
    const bool act = blk < nblk;
    const int64_t br = act ? blk / nb32 : 0, bc = act ? blk % nb32 : 0;
    if (act) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float re[8], im[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const Cx<float> v = X[(32 * br + row) * ld + 32 * bc + 16 * h + 8 * hq + e];
          re[e] = v.re;
          im[e] = v.im;
          acc += double(v.re) * double(v.re) + double(v.im) * double(v.im);
          if constexpr (TT) blkL[wv][split_swz(row, 16 * h + 8 * hq + e)] = v;
        }
        write_unit_block<4>(P + (br * nkb + 2 * bc + h) * (4 * 3 * XUNIT) + lane, re, im);
      }
    }
    if constexpr (TT) {
      __syncthreads();
      if (act) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          float re[8], im[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const Cx<float> v = blkL[wv][split_swz(16 * h + 8 * hq + e, row)];
            re[e] = v.re;
            im[e] = v.im;
          }
          write_unit_block<3>(PT + (bc * nkb + 2 * br + h) * (3 * 3 * XUNIT) + lane, re, im);
        }
      }
      __syncthreads();
    }
  }
  if constexpr (WITH_F) {
#pragma unroll
    for (int u = 0; u < U; ++u) accf += double(fv[u]);
    // the rest of the range (N >= 12), U strided loads per thread at a time
    for (int64_t e0 = fbeg + threadIdx.x + U * NT; e0 < fend; e0 += U * NT) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = e0 + u * NT;
        fv[u] = e < fend ? f[e] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) accf += double(fv[u]);
    }
  }
  const double st = block_sum256(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = st;
  if constexpr (WITH_F) {
    const double sf = block_sum256(accf, red);
    if (threadIdx.x == 0) partials[nb + blockIdx.x] = sf;
  }
}

// ---------------------------------------------------------------------------
// Product kernel
// ---------------------------------------------------------------------------
// A wave-uniform pointer moved into scalar registers.  The builtin takes
// and returns a signed 32-bit value per half; each half is taken back as
// unsigned, so that the high half is not sign-extended over.
__device__ __forceinline__ const u16x8* uniform_ptr(const u16x8* p) {
  const uint64_t u = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(u)));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(u >> 32)));
  return reinterpret_cast<const u16x8*>((uint64_t(hi) << 32) | uint64_t(lo));
}

// global -> LDS copy of one 16-byte vector per lane into the 1 KB at LDS
// byte address lds (wave-uniform).  Written as an asm statement so that the
// compiler's wait-count pass, which cannot tell ring slots apart, does not
// order every LDS read after every such copy; the kernel waits for them
// itself (vmcnt) before the barrier that publishes a slab.  Nothing is
// written to registers.
// sbase: wave-uniform base address (SGPR pair); voff: the lane's byte offset.
__device__ __forceinline__ void dma16(const void* sbase, uint32_t voff, uint32_t lds) {
  uint32_t m0v;  // M0 is an output of the statement, so the compiler keeps no value of its own there
  asm volatile("s_mov_b32 %0, %3\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2"
               : "={m0}"(m0v)
               : "v"(voff), "s"(sbase), "s"(lds)
               : "memory");
  (void)m0v;
}
// LDS byte address of a pointer into the workgroup's shared memory
__device__ __forceinline__ uint32_t lds_address(const char* p) {
  return (uint32_t)(uintptr_t)(lds_void_t*)p;
}
// s_waitcnt vmcnt(n), other counters unconstrained (gfx9 encoding)
#define QST_VMCNT(n) __builtin_amdgcn_s_waitcnt(0x0f70 | ((n) & 15) | (((n) >> 4) << 14))

__device__ __forceinline__ f16v mfma32(u16x8 a, u16x8 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

struct XArgs {
  const u16x8* A;  // planes of the row operand
  const u16x8* B;  // planes of the column operand (rows of B^T)
  int ngA, ngB;    // groups per unit block
  int gA2, gB2;    // group of the third product's operands (re + im, or re - im)
  void* C;         // output (HEMM, or HERK without x0)
  int64_t ldc;
  int d;
  const double* tau;       // tau, or NULL with tau_part
  const double* tau_part;  // FP64 partial sums of tau (kReduceBlocks), folded by every workgroup
  double* tau_out;         // where workgroup 0 of the T T^dagger fix-up stores the folded tau
  const double* up;        // HEMM: upstream scalar or NULL
  float* part;             // HERK partial tiles [slots][re, im][TILE] in the MFMA layout
  int ntiles, kIters;
  X6HerkSched sc;          // HERK schedule (rounds, then slices)
  void* x0;                // HERK: first POVM pass output, or NULL
  int x0g, x0up;
};

constexpr int kXTileVals = XT * XT;  // complex values per tile

// Fold of the tau partials in a fixed order (bitwise the same in every
// workgroup); workgroup 0 of the product kernel stores it.
__device__ double x6_tau(const XArgs& a, bool store) {
  if (!a.tau_part) return *a.tau;
  __shared__ double red[4];
  __shared__ double bcast;
  double acc = 0.0;
  for (int b = threadIdx.x; b < kReduceBlocks; b += 256) acc += a.tau_part[b];
  const double sum = block_sum256(acc, red);
  if (threadIdx.x == 0) {
    bcast = sum;
    if (store && blockIdx.x == 0 && a.tau_out) *a.tau_out = sum;
  }
  __syncthreads();
  return bcast;
}

// Panels per MFMA accumulation chain.  The BF16 MFMA rounds the FP32
// accumulator toward zero when it adds a product block (measured: a Gram
// diagonal accumulated over all 4096 panels of d = 4096 comes out 1.9e-6
// low, against 1.2e-7 for the FP32 MFMA), so a chain is kept short and
// folded into FP32 totals with round-to-nearest adds; a new chain starts
// from a zero accumulator operand.
constexpr int XCHAIN = 32;

// Accumulate the panels [kb, ke) of output tile (tr, tc) into (re, im)
// (which the caller zeroes).  Every thread of the workgroup calls it (it
// contains barriers); on return the LDS ring is idle.
template <bool HERK>
__device__ __forceinline__ void x6_segment(const XArgs& a, char* lds, int tr, int tc, int kb, int ke,
                                           f16v (&re)[2][2], f16v (&im)[2][2]) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = w >> 1, wc = w & 1;
  const int nkb = a.d / 16;
  const uint32_t lbase = __builtin_amdgcn_readfirstlane(lds_address(lds));
  // this wave's six units of every slab: unit q = 6 w + i, A (q < 12) or B,
  // split (q % 12) / 4, row block q % 4; all of it wave-uniform except the
  // lane's 16-byte offset.  cbase[i]: unit i's address at panel 0, group 0
  // (scalar registers: the asm operand requires them); a slab adds
  // (kp ng + g) 3 units.
  const uint32_t voff = uint32_t(lane) * 16;
  const u16x8* cbase[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int q = 6 * w + i;
    const bool isB = q >= 12;
    const int sp = (q % 12) / 4, rb = q % 4;
    const int64_t r0 = int64_t(isB ? tc : tr) * (XT / 32) + rb;
    cbase[i] = uniform_ptr((isB ? a.B : a.A) + ((r0 * nkb * (isB ? a.ngB : a.ngA)) * 3 + sp) * XUNIT);
  }
  const int npan = ke - kb;
  // copies of slab s = 3 kp + prod of the segment (panel clamped to the
  // last); prod is a compile-time constant at every call
  auto dma_slab = [&](int s, int kp, int prod) {
    const int kpa = kb + min(kp, npan - 1);
    const int64_t offA = (int64_t(kpa) * a.ngA + (prod < 2 ? prod : a.gA2)) * 3 * XUNIT;
    const int64_t offB = (int64_t(kpa) * a.ngB + (prod < 2 ? prod : a.gB2)) * 3 * XUNIT;
    const uint32_t slot = lbase + uint32_t((s % XNSLOT) * XSLOT);
    return [=](int i) {
      const int q = 6 * w + i;
      dma16(cbase[i] + (q >= 12 ? offB : offA), voff, slot + uint32_t(q * 1024));
    };
  };
  u16x8 fa[3][3][2], fb[3][3][2];  // [product][split][block]
  f16v acc[3][2][2];
#pragma unroll
  for (int s = 0; s < XDIST; ++s) {
    const auto copy = dma_slab(s, s / 3, s % 3);
#pragma unroll
    for (int i = 0; i < 6; ++i) copy(i);
  }
  QST_VMCNT((XDIST - 1) * 6);
  __builtin_amdgcn_s_barrier();
  {
    const u16x8* L = reinterpret_cast<const u16x8*>(lds);
#pragma unroll
    for (int sp = 0; sp < 3; ++sp)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fa[0][sp][i] = L[(sp * 4 + wr * 2 + i) * XUNIT + lane];
        fb[0][sp][i] = L[(12 + sp * 4 + wc * 2 + i) * XUNIT + lane];
      }
  }
  // combination order hh, hm, hl, mh, mm, lh: the current slab's A_h dies
  // after the third pair, A_m and B_m after the fifth, so the next slab's
  // fragments, read two per step in the second half of the slab (in the
  // order that slab's first MFMAs use them), mostly take freed registers
  constexpr int SA[6] = {0, 0, 0, 1, 1, 2}, SB[6] = {0, 1, 2, 0, 1, 0};
  constexpr int RD_AB[12] = {0, 0, 1, 1, 1, 1, 1, 1, 0, 0, 0, 0};  // 0: A, 1: B
  constexpr int RD_SP[12] = {0, 0, 0, 0, 1, 1, 2, 2, 1, 1, 2, 2};
  for (int c0 = 0; c0 < npan; c0 += XCHAIN) {
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[p][i][j][v] = 0.f;
    const int cend = min(npan, c0 + XCHAIN);
    for (int kp = c0; kp < cend; ++kp) {
#pragma unroll
      for (int prod = 0; prod < 3; ++prod) {
        const int s = 3 * kp + prod;
        // every slab issued six copies per wave, so slab s+1 is complete once
        // at most XDIST-2 newer slabs are outstanding
        QST_VMCNT((XDIST - 2) * 6);
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        const int np = prod == 2 ? 0 : prod + 1;
        const u16x8* L = reinterpret_cast<const u16x8*>(lds + ((s + 1) % XNSLOT) * XSLOT);
        const auto copy = dma_slab(s + XDIST, kp + (prod + XDIST) / 3, (prod + XDIST) % 3);
#pragma unroll
        for (int q = 0; q < 12; ++q) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int m = 2 * q + h;
            const int c = m / 4, i = (m / 2) & 1, j = m & 1;
            acc[prod][i][j] = mfma32(fa[prod][SA[c]][i], fb[prod][SB[c]][j], acc[prod][i][j]);
          }
          if (q >= 6) {
#pragma unroll
            for (int r = 2 * (q - 6); r < 2 * (q - 6) + 2; ++r) {
              const int sp = RD_SP[r], bi = r & 1;
              if (RD_AB[r] == 0) fa[np][sp][bi] = L[(sp * 4 + wr * 2 + bi) * XUNIT + lane];
              else fb[np][sp][bi] = L[(12 + sp * 4 + wc * 2 + bi) * XUNIT + lane];
            }
          } else {
            copy(q);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // close the chain: one 32 x 32 block at a time
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const float p1 = acc[0][i][j][v], p2 = acc[1][i][j][v], p3 = acc[2][i][j][v];
          if constexpr (HERK) {
            re[i][j][v] += p1 + p2;
            im[i][j][v] += (p3 - p1) + p2;
          } else {
            re[i][j][v] += p1 - p2;
            im[i][j][v] += (p3 - p1) - p2;
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
  }
  // the clamped copies issued past the end land before the ring is reused
  // (or the workgroup's LDS is released), and every wave is past its reads
  QST_VMCNT(0);
  __syncthreads();
}

// (row, column) inside the 128 x 128 tile of accumulator value v of block
// (i, j) held by lane `lane` of wave (wr, wc).
__device__ __forceinline__ int x6_row(int wr, int i, int v, int lane) {
  return wr * 64 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}
__device__ __forceinline__ int x6_col(int wc, int j, int lane) { return wc * 64 + j * 32 + (lane & 31); }

// Partial of a tile segment, 16 bytes per lane and store: values
// 4 vq .. 4 vq + 3 of block ij = 2 i + j, part p (re, im) of wave w's lane l
// at floats ((((4 w + ij) 2 + p) 4 + vq) 64 + l) 4 .. + 3 (each store of a
// wave is 1 KB contiguous; wave w's 64 x 64 quadrant is floats
// [8192 w, 8192 (w + 1))).
__device__ __forceinline__ float* x6_slot(const XArgs& a, int64_t slot) {
  return a.part + slot * int64_t(2 * kXTileVals);
}
// slot of a round unit u (sk > 1), and of slice `which` (0: the first unit
// of the worker's range, 1: the last) of slice worker w
__device__ __forceinline__ int64_t x6_unit_slot(int64_t u) { return u; }
__device__ __forceinline__ int64_t x6_slice_slot(const X6HerkSched& sc, int64_t w, int which) {
  return (sc.sk > 1 ? sc.main : 0) + (sc.tq ? w : 2 * w + which);
}
__device__ __forceinline__ void x6_store_partial(float* dst, const f16v (&re)[2][2], const f16v (&im)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  f4v* d4 = reinterpret_cast<f4v*>(dst);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int vq = 0; vq < 4; ++vq) {
        const int64_t o = (((w * 4 + i * 2 + j) * 2) * 4 + vq) * 64 + lane;
        d4[o] = f4v{re[i][j][4 * vq], re[i][j][4 * vq + 1], re[i][j][4 * vq + 2], re[i][j][4 * vq + 3]};
        d4[o + 256] = f4v{im[i][j][4 * vq], im[i][j][4 * vq + 1], im[i][j][4 * vq + 2], im[i][j][4 * vq + 3]};
      }
}

// Tile epilogue.  HEMM: C = scale (re, im).  HERK without x0: rho = (re,
// im) / tau, and the conjugate transpose at the mirror position for an
// off-diagonal tile.  HERK with x0: the first POVM pass over G qubits on
// each 64 x 64 quadrant (the quadrant of wave q, q = 2 qr + qc; the upper
// quadrant of a diagonal tile is the mirror of the lower one and skipped),
// through a 64 x 64 tile in LDS.
template <bool HERK, int X0G>
__device__ __forceinline__ void x6_epilogue(const XArgs& a, int tr, int tc, const f16v (&re)[2][2],
                                            const f16v (&im)[2][2], double scale, char* lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  const float sc = float(scale);
  const int64_t R0 = int64_t(tr) * XT, C0 = int64_t(tc) * XT;
  if constexpr (X0G == 0) {
    Cx<float>* C = static_cast<Cx<float>*>(a.C);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t r = R0 + x6_row(wr, i, v, lane), c = C0 + x6_col(wc, j, lane);
          C[r * a.ldc + c] = Cx<float>{re[i][j][v] * sc, im[i][j][v] * sc};
          if (HERK && tr != tc) C[c * a.ldc + r] = Cx<float>{re[i][j][v] * sc, -im[i][j][v] * sc};
        }
  } else {
    constexpr int G = X0G;
    constexpr int S = 64 >> G;
    constexpr int TG = 1 << (2 * G);
    constexpr int M = (1 << G) - 1;
    Cx<float>* L = reinterpret_cast<Cx<float>*>(lds);
    gemm::GemmArgs g{};
    g.x0 = a.x0;
    g.x0g = a.x0g;
    g.x0up = a.x0up;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int qr = q >> 1, qc = q & 1;
      if (tr == tc && qr < qc) continue;  // uniform across the workgroup
      if (w == q) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int r = i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), c = j * 32 + (lane & 31);
              L[((r >> G) * S + (c >> G)) * TG + swz<G>(r & M, c & M)] = Cx<float>{re[i][j][v] * sc, im[i][j][v] * sc};
            }
      }
      __syncthreads();
      gemm::x0_rounds<float, G>(g, int64_t(2) * tr + qr, int64_t(2) * tc + qc, L);
      __syncthreads();
    }
  }
}

__device__ __forceinline__ void x6_zero(f16v (&re)[2][2], f16v (&im)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) re[i][j][v] = im[i][j][v] = 0.f;
}

// G' T: one tile per workgroup.
__global__ __launch_bounds__(256, 1) void x6_hemm_kernel(XArgs a) {
  extern __shared__ __align__(16) char lds[];
  const int ts = a.d / XT;
  const int lb = int(xcd_order(blockIdx.x, gridDim.x));
  int tr, tc;
  if (ts % 8 == 0) {  // blocks of 4 x 8 tiles per 32 consecutive logical workgroups
    const int grp = lb / 32, within = lb % 32;
    tr = (grp / (ts / 8)) * 4 + within / 8;
    tc = (grp % (ts / 8)) * 8 + within % 8;
  } else {
    tr = lb / ts;
    tc = lb % ts;
  }
  double scale = 2.0 / *a.tau;
  if (a.up) scale *= *a.up;
  f16v re[2][2], im[2][2];
  x6_zero(re, im);
  x6_segment<false>(a, lds, tr, tc, 0, a.kIters, re, im);
  x6_epilogue<false, 0>(a, tr, tc, re, im, scale, lds);
}

__device__ __forceinline__ int64_t x6_slice_start(int64_t w, int64_t Q, int64_t iters) { return (w * iters) / Q; }

// Unit u -> tile and K panels: u = s * ntiles + t covers panels
// [s kh, (s + 1) kh) of lower tile t (the units of a round share s, so
// its workgroups stream the same K range).
__device__ __forceinline__ void x6_unit(const X6HerkSched& sc, int64_t u, int64_t& t, int& k0) {
  t = u % sc.ntiles;
  k0 = int((u / sc.ntiles) * sc.kh);
}

// T T^dagger: logical workgroup w takes round units w, w + P, ...; a whole
// tile (sk = 1) is finished here, a part of one is stored as a partial.
// Then, as slice worker w < Q, the iterations [start(w), start(w + 1)) of
// the remaining units' (unit, panel) sequence.
template <int X0G>
__global__ __launch_bounds__(256, 1) void x6_herk_kernel(XArgs a) {
  extern __shared__ __align__(16) char lds[];
  const X6HerkSched& sc = a.sc;
  const int64_t w = xcd_order(blockIdx.x, gridDim.x);
  // 1 / tau, formed on the first whole tile this workgroup finishes (a
  // split tile's partials are scaled in the fix-up, which stores tau)
  double scale = 0.0;
  auto tile_scale = [&]() {
    if (scale == 0.0) scale = 1.0 / x6_tau(a, false);
    return scale;
  };
  for (int64_t r = 0; r < sc.rounds; ++r) {
    const int64_t u = r * sc.P + w;
    int64_t t;
    int k0;
    x6_unit(sc, u, t, k0);
    int tr, tc;
    tri_decode(t, tr, tc);
    f16v re[2][2], im[2][2];
    x6_zero(re, im);
    x6_segment<true>(a, lds, tr, tc, k0, k0 + int(sc.kh), re, im);
    if (sc.sk == 1) x6_epilogue<true, X0G>(a, tr, tc, re, im, tile_scale(), lds);
    else x6_store_partial(x6_slot(a, x6_unit_slot(u)), re, im);
  }
  if (w >= sc.Q) return;
  // transposed slices: one piece, slice w / left of unit w % left
  int64_t it = sc.tq ? 0 : x6_slice_start(w, sc.Q, sc.left_iters);
  const int64_t end = sc.tq ? 1 : x6_slice_start(w + 1, sc.Q, sc.left_iters);
  const int64_t first_unit = it / sc.kh;
  while (it < end) {
    int64_t j;  // leftover unit
    int kb, ke;
    if (sc.tq) {
      j = w % sc.left;
      kb = int((w / sc.left) * sc.ps);
      ke = kb + int(sc.ps);
      it = end;
    } else {
      j = it / sc.kh;
      kb = int(it % sc.kh);
      ke = int(std::min<int64_t>(sc.kh, kb + (end - it)));
      it += ke - kb;
    }
    int64_t t;
    int k0;
    x6_unit(sc, sc.main + j, t, k0);
    int tr, tc;
    tri_decode(t, tr, tc);
    f16v re[2][2], im[2][2];
    x6_zero(re, im);
    x6_segment<true>(a, lds, tr, tc, k0 + kb, k0 + ke, re, im);
    if (sc.sk == 1 && kb == 0 && ke == sc.kh) {
      x6_epilogue<true, X0G>(a, tr, tc, re, im, tile_scale(), lds);
    } else {
      x6_store_partial(x6_slot(a, x6_slice_slot(sc, w, j == first_unit ? 0 : 1)), re, im);  // slot w with tq
    }
  }
}

// Slice workers holding the first and the last panel of leftover unit j.
__device__ __forceinline__ void x6_owners(const X6HerkSched& sc, int64_t j, int64_t& lo, int64_t& hi) {
  const int64_t f = j * sc.kh, l = f + sc.kh - 1, Q = sc.Q, it = sc.left_iters;
  lo = (f * Q) / it;
  while (lo + 1 < Q && x6_slice_start(lo + 1, Q, it) <= f) ++lo;
  while (lo > 0 && x6_slice_start(lo, Q, it) > f) --lo;
  hi = (l * Q) / it;
  while (hi + 1 < Q && x6_slice_start(hi + 1, Q, it) <= l) ++hi;
  while (hi > 0 && x6_slice_start(hi, Q, it) > l) --hi;
}

// The contributions to lower tile t in K order -- for each of its sk
// units, the round partial, or the slice partials in worker order -- as
// partial slots, one per next() call (-1 at the end).  finished(): a single
// workgroup wrote the tile (no contributions).
struct X6Contrib {
  const X6HerkSched& sc;
  int64_t t, s = 0, wg = 0, hi = -1, j = 0;
  __device__ X6Contrib(const X6HerkSched& sc_, int64_t t_) : sc(sc_), t(t_) {}
  __device__ bool finished() const {
    if (sc.sk != 1) return false;
    if (t < sc.main) return true;  // a round unit: the whole tile
    if (sc.tq) return sc.tq == 1;  // one transposed slice per unit: the whole tile
    int64_t lo, h;
    x6_owners(sc, t - sc.main, lo, h);
    return lo == h;  // inside one worker's slice: finished there
  }
  __device__ int64_t next() {
    while (true) {
      if (wg <= hi) {  // slice partials of leftover unit j
        if (sc.tq) return x6_slice_slot(sc, j + sc.left * wg++, 0);  // slice wg of unit j: worker j + left wg
        const int64_t first_unit = x6_slice_start(wg, sc.Q, sc.left_iters) / sc.kh;
        const int64_t slot = x6_slice_slot(sc, wg, j == first_unit ? 0 : 1);
        ++wg;
        return slot;
      }
      if (s >= sc.sk) return -1;
      const int64_t u = s * sc.ntiles + t;
      ++s;
      if (u < sc.main) return x6_unit_slot(u);
      j = u - sc.main;
      if (sc.tq) {
        wg = 0;
        hi = sc.tq - 1;
      } else {
        x6_owners(sc, j, wg, hi);
      }
    }
  }
};

// Fix-up: workgroup (t, q) adds quadrant q (64 x 64, the data of wave q of
// the product kernel) of the contributions to lower tile t in K order and
// applies the epilogue to it (rho, or the first POVM pass); the upper
// quadrant of a diagonal tile is the mirror of the lower one and skipped.
// Tiles go in reverse order: the leftover units, whose tiles carry the most
// contributions, belong to the last tiles, which thus start first.  Thread
// th holds values 4 (th + 256 m) + c, m < 8, c < 4, of the quadrant's
// 8192-float block (layout of x6_store_partial with w = q), loaded as
// 16-byte vectors; the loads of up to four contributions are in flight
// before they are added, in order.
template <int X0G>
__global__ __launch_bounds__(256, 3) void x6_fixup_kernel(XArgs a) {
  __shared__ __align__(16) Cx<float> L[64 * 64];
  __shared__ double red[4];
  const X6HerkSched& sc = a.sc;
  const int64_t t = sc.ntiles - 1 - (blockIdx.x >> 2);
  const int q = blockIdx.x & 3, qr = q >> 1, qc = q & 1;
  int tr, tc;
  tri_decode(t, tr, tc);
  const bool skip = tr == tc && qr < qc;  // mirror quadrant of a diagonal tile
  const int th = threadIdx.x;
  X6Contrib it(sc, t);
  if (blockIdx.x != 0 && (skip || it.finished())) return;
  // tau's partial sums (x6_tau's order), loaded now so that their latency
  // overlaps the contributions' loads; workgroup 0 also stores tau
  double tp[kReduceBlocks / 256];
#pragma unroll
  for (int k = 0; k < kReduceBlocks / 256; ++k) tp[k] = a.tau_part[th + 256 * k];
  if (blockIdx.x == 0 && (skip || it.finished())) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kReduceBlocks / 256; ++k) acc += tp[k];
    const double tau = block_sum256(acc, red);
    if (th == 0 && a.tau_out) *a.tau_out = tau;
    return;
  }
  f4v acc[8], v[2][8];
#pragma unroll
  for (int m = 0; m < 8; ++m) acc[m] = f4v{0.f, 0.f, 0.f, 0.f};
  // two contributions in flight (most tiles have two), then added in order
  while (true) {
    int64_t sl[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) sl[k] = it.next();
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (sl[k] >= 0) {
        const f4v* src = reinterpret_cast<const f4v*>(x6_slot(a, sl[k]) + q * 8192);
#pragma unroll
        for (int m = 0; m < 8; ++m) v[k][m] = src[th + 256 * m];
      }
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (sl[k] >= 0) {
#pragma unroll
        for (int m = 0; m < 8; ++m) acc[m] += v[k][m];
      }
    if (sl[1] < 0) break;
  }
  double tacc = 0.0;
#pragma unroll
  for (int k = 0; k < kReduceBlocks / 256; ++k) tacc += tp[k];
  const double tau = block_sum256(tacc, red);
  __shared__ double tau_sh;
  if (th == 0) {
    tau_sh = tau;
    if (blockIdx.x == 0 && a.tau_out) *a.tau_out = tau;
  }
  __syncthreads();
  const double scale = 1.0 / tau_sh;
  // vector th + 256 m of the quadrant holds values 4 vq + c of block
  // ij = m / 2, part m % 2, lane th % 64, vq = th / 64
  const float sc32 = float(scale);
  const int lane = th & 63, vq = th >> 6;
  if constexpr (X0G == 0) {
    Cx<float>* C = static_cast<Cx<float>*>(a.C);
    float* Cf = reinterpret_cast<float*>(C);
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) {
        const int part = m & 1, vv = 4 * vq + c4, ij = m >> 1;
        const int i = ij >> 1, j = ij & 1;
        const int64_t r = int64_t(tr) * XT + qr * 64 + i * 32 + 8 * (vv >> 2) + 4 * (lane >> 5) + (vv & 3);
        const int64_t c = int64_t(tc) * XT + qc * 64 + j * 32 + (lane & 31);
        const float x = acc[m][c4] * sc32;
        Cf[2 * (r * a.ldc + c) + part] = x;
        // the mirror: every off-diagonal tile, and the lower-left quadrant
        // of a diagonal tile (whose upper-right quadrant is not computed here)
        if (tr != tc || qr != qc) Cf[2 * (c * a.ldc + r) + part] = part ? -x : x;
      }
  } else {
    constexpr int G = X0G;
    constexpr int S = 64 >> G;
    constexpr int TG = 1 << (2 * G);
    constexpr int M = (1 << G) - 1;
    float* Lf = reinterpret_cast<float*>(L);
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) {
        const int part = m & 1, vv = 4 * vq + c4, ij = m >> 1;
        const int i = ij >> 1, j = ij & 1;
        const int r = i * 32 + 8 * (vv >> 2) + 4 * (lane >> 5) + (vv & 3), c = j * 32 + (lane & 31);
        Lf[2 * (((r >> G) * S + (c >> G)) * TG + swz<G>(r & M, c & M)) + part] = acc[m][c4] * sc32;
      }
    __syncthreads();
    gemm::GemmArgs g{};
    g.x0 = a.x0;
    g.x0g = a.x0g;
    g.x0up = a.x0up;
    gemm::x0_rounds<float, G>(g, int64_t(2) * tr + qr, int64_t(2) * tc + qc, L);
  }
}

// The product kernels use more LDS than the static limit: raise the
// per-kernel limit once per device before the first launch.
template <auto K>
hipError_t x6_allow_lds() {
  static std::mutex mu;  // one flag set per kernel
  static bool done[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!done[dev]) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(K), hipFuncAttributeMaxDynamicSharedMemorySize, XLDS);
    if (e != hipSuccess) return e;
    done[dev] = true;
  }
  return hipSuccess;
}

int x6_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cus;
}

template <int X0G>
hipError_t x6_run_herk(XArgs a, int n, hipStream_t s) {
  hipError_t e = x6_allow_lds<x6_herk_kernel<X0G>>();
  if (e != hipSuccess) return e;
  a.sc = x6_herk_sched(n, x6_cus());
  const int64_t grid = a.sc.rounds > 0 ? a.sc.P : a.sc.Q;
  x6_herk_kernel<X0G><<<unsigned(grid), 256, XLDS, s>>>(a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  x6_fixup_kernel<X0G><<<unsigned(a.ntiles) * 4, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_x6_herk(const void* T, int64_t ldt, void* rho, int64_t ldr, int n, double* tau_partials,
                          const void* f, double* tau_dev, void* planes, void* partials, hipStream_t s,
                          const Pass0Out* x0, void* tt_planes) {
  const int d = 1 << n;
  if (d < kX6Tile || !tau_partials) return hipErrorInvalidValue;
  if (x0 && (x0->g < 4 || x0->g > 6 || !x0->tetra)) return hipErrorInvalidValue;
  u16x8* P = static_cast<u16x8*>(planes);
  {
    ProfScope prof("x6_split_t", s);
    const Cx<float>* Tf = static_cast<const Cx<float>*>(T);
    const float* ff = static_cast<const float*>(f);
    u16x8* PT = static_cast<u16x8*>(tt_planes);
    if (f && PT) x6_split_tau_kernel<true, true><<<kReduceBlocks, 256, 0, s>>>(Tf, ldt, d, P, PT, tau_partials, ff);
    else if (f) x6_split_tau_kernel<true, false><<<kReduceBlocks, 256, 0, s>>>(Tf, ldt, d, P, PT, tau_partials, ff);
    else if (PT) x6_split_tau_kernel<false, true><<<kReduceBlocks, 256, 0, s>>>(Tf, ldt, d, P, PT, tau_partials, ff);
    else x6_split_tau_kernel<false, false><<<kReduceBlocks, 256, 0, s>>>(Tf, ldt, d, P, PT, tau_partials, ff);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  ProfScope prof("herk_x6", s);
  XArgs a{};
  a.A = P;
  a.B = P;
  a.ngA = 4;
  a.ngB = 4;
  a.gA2 = 2;  // re + im
  a.gB2 = 3;  // re - im
  a.C = rho;
  a.ldc = ldr;
  a.d = d;
  a.tau = tau_dev;
  a.tau_part = tau_partials;
  a.tau_out = tau_dev;
  a.part = static_cast<float*>(partials);
  a.ntiles = (d / XT) * (d / XT + 1) / 2;
  a.kIters = d / 16;
  if (x0) {
    a.x0 = x0->X;
    a.x0g = x0->g;
    a.x0up = n - x0->g;
    return x0->g == 6 ? x6_run_herk<6>(a, n, s) : x0->g == 5 ? x6_run_herk<5>(a, n, s) : x6_run_herk<4>(a, n, s);
  }
  return x6_run_herk<0>(a, n, s);
}

hipError_t launch_x6_hemm(const void* G, int64_t ldg, const void* T, int64_t ldt, void* out, int64_t ldo, int n,
                          const double* tau_dev, const double* upstream_dev, void* planes, hipStream_t s,
                          bool g_ready, bool t_ready) {
  const int d = 1 << n;
  if (d < kX6Tile) return hipErrorInvalidValue;
  const int64_t units = int64_t(d / 32) * (d / 16);
  u16x8* PG = static_cast<u16x8*>(planes);
  u16x8* PT = PG + units * 9 * XUNIT;
  hipError_t e;
  if (!g_ready || !t_ready) {
    ProfScope prof("x6_split_gt", s);
    if (!g_ready) {
      x6_split_kernel<false, 3><<<unsigned((units + 3) / 4), 256, 0, s>>>(static_cast<const Cx<float>*>(G), ldg, d, PG);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!t_ready) {
      x6_split_kernel<true, 3><<<unsigned((units + 3) / 4), 256, 0, s>>>(static_cast<const Cx<float>*>(T), ldt, d, PT);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if ((e = x6_allow_lds<x6_hemm_kernel>()) != hipSuccess) return e;
  XArgs a{};
  a.A = PG;
  a.B = PT;
  a.ngA = 3;
  a.ngB = 3;
  a.gA2 = 2;
  a.gB2 = 2;
  a.C = out;
  a.ldc = ldo;
  a.d = d;
  a.tau = tau_dev;
  a.up = upstream_dev;
  a.kIters = d / 16;
  const int ts = d / XT;
  ProfScope prof("hemm_x6", s, true);
  hipExtLaunchKernelGGL(x6_hemm_kernel, dim3(unsigned(ts * ts)), dim3(256), XLDS, s, prof.start(), prof.stop(), 0, a);
  return hipGetLastError();
}

}  // namespace qst
