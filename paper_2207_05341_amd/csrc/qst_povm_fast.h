// Bodies of the specialised product-POVM passes (see k_povm_fast.hip for
// the round structure), as device functions over a logical block and a
// 256-thread group, so that the pass kernels and the batched persistent
// kernel run the same code.  Every thread of the calling workgroup must
// make the same calls: the bodies contain barriers.
#pragma once

#include "qst_device.h"
#include "qst_povm_ops.h"
#include "qst_povm_rounds.h"
#include "qst_split.h"

namespace qst {
namespace fast_pass {

// ---------------------------------------------------------------------------
// Matrix-side pass (pass 0): rho (forward input, lower triangle) or G'
// (adjoint output, written in full); outcome side X'[(Rhi, Chi)][kg].
// 4^(G-2) threads per tile, 256 / 4^(G-2) tiles per 256 threads: the
// call with index wb (thread tid of 256) covers tiles wb * TPW ..; tiles
// past ntiles load nothing and store nothing.  lds holds TPW * 4^G values.
// ---------------------------------------------------------------------------
//
// PLANES (adjoint, FP32, G = 5 or 6): instead of G' itself, G' as the split
// operand planes of the QST_F32X6 gradient product (row operand, groups
// re, im, re + im, three exact bf16 parts; layout of qst_split.h) at
// a.gplanes: each tile, then its conjugate transpose (off the diagonal),
// passes through LDS row-major (16-byte chunks swizzled by row) and every
// thread writes four unit-block slots.
template <typename R, bool ADJ, bool TETRA, int G, bool PLANES = false>
__device__ __forceinline__ void mat_pass_body(const PassArgs& a, const ModeMatrix& A, int64_t ntiles, int64_t wb,
                                              unsigned tid, Cx<R> (&lds)[(256 >> (2 * (G - 2))) << (2 * G)]) {
  static_assert(!PLANES || (ADJ && G >= 5 && sizeof(R) == 4), "planes from FP32 adjoint tiles of 32 or 64 rows");
  constexpr int NT = 1 << (2 * (G - 2));
  constexpr int TPW = 256 / NT;
  constexpr int TILE = 1 << (2 * G);
  using RD = Rounds<G>;
  __builtin_assume(tid < 256);

  const int tl = tid / NT, t = tid % NT;
  const int64_t tile = wb * TPW + tl;
  const bool active = tile < ntiles;
  int Rhi = 0, Chi = 0;
  if (active) tri_decode(tile, Rhi, Chi);
  const int Up = a.U - G;
  Cx<R>* L = lds + tl * TILE;
  const int64_t R0 = int64_t(Rhi) << G, C0 = int64_t(Chi) << G;
  const int64_t obase = ((int64_t(Rhi) << Up) | Chi) * int64_t(TILE);
  const int bq = t & ((1 << (G - 2)) - 1), aq = t >> (G - 2);  // 4 x 4 block (rows 4aq.., cols 4bq..)

  // Fixed part of round rd: the 4 x 4 block corner for round 0 (bits 0, 1
  // vary), otherwise the interleaved enumeration of the other bits by t.
  auto round_fixed = [&](int rd, int& rf, int& cf) {
    if (rd == 0) {
      rf = 4 * aq;
      cf = 4 * bq;
    } else {
      fixed_bits<G>(t, RD::bA[rd], RD::bB[rd], rf, cf);
    }
  };

  Cx<R> x[16];
  if constexpr (!ADJ) {
    Cx<R> blk[4][4];
    if (active) {
      const Cx<R>* M = static_cast<const Cx<R>*>(a.in);
      const bool diag = Rhi == Chi;
      if (diag && aq < bq) {  // block above the diagonal: conjugate of the mirror block
#pragma unroll
        for (int ci = 0; ci < 4; ++ci) {
          const Cx<R>* row = M + (C0 + 4 * bq + ci) * a.ld + R0 + 4 * aq;
#pragma unroll
          for (int ri = 0; ri < 4; ++ri) blk[ri][ci] = Cx<R>{row[ri].re, -row[ri].im};
        }
      } else {
#pragma unroll
        for (int ri = 0; ri < 4; ++ri) {
          const Cx<R>* row = M + (R0 + 4 * aq + ri) * a.ld + C0 + 4 * bq;
#pragma unroll
          for (int ci = 0; ci < 4; ++ci) blk[ri][ci] = row[ci];
        }
        if (diag && aq == bq) {  // diagonal block: upper entries from the lower ones
#pragma unroll
          for (int ri = 0; ri < 4; ++ri)
#pragma unroll
            for (int ci = ri + 1; ci < 4; ++ci) blk[ri][ci] = Cx<R>{blk[ci][ri].re, -blk[ci][ri].im};
        }
      }
    } else {
#pragma unroll
      for (int ri = 0; ri < 4; ++ri)
#pragma unroll
        for (int ci = 0; ci < 4; ++ci) blk[ri][ci] = Cx<R>{R(0), R(0)};
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = blk[blk_ri(m)][blk_ci(m)];
    mat_fwd_rounds<R, TETRA, G>(x, L, t, A, active ? static_cast<Cx<R>*>(a.out) + obase : nullptr);
  } else {
#pragma unroll
    for (int rd = RD::n - 1; rd >= 0; --rd) {
      const int bA = RD::bA[rd], bB = RD::bB[rd];
      int rf, cf;
      round_fixed(rd, rf, cf);
      if (rd == RD::n - 1) {
        const Cx<R>* in = static_cast<const Cx<R>*>(a.in) + obase;
#pragma unroll
        for (int m = 0; m < 16; ++m)
          x[m] = active ? in[t + ((m >> 2) << (2 * bA)) + ((m & 3) << (2 * bB))] : Cx<R>{R(0), R(0)};
      } else {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          int r, c;
          rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
          x[m] = L[swz<G>(r, c)];
        }
      }
      contract16<R, true, TETRA>(x, RD::opA[rd], RD::opB[rd], A);
      if (rd > 0) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          int r, c;
          rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
          L[swz<G>(r, c)] = x[m];
        }
        __syncthreads();
      } else if (active && !PLANES) {
        Cx<R> blk[4][4];
#pragma unroll
        for (int m = 0; m < 16; ++m) blk[blk_ri(m)][blk_ci(m)] = x[m];
        Cx<R>* M = static_cast<Cx<R>*>(a.out);
#pragma unroll
        for (int ri = 0; ri < 4; ++ri) {
          Cx<R>* row = M + (R0 + 4 * aq + ri) * a.ld + C0 + 4 * bq;
#pragma unroll
          for (int ci = 0; ci < 4; ++ci) row[ci] = blk[ri][ci];
        }
        if (Rhi != Chi) {  // mirror tile: conjugate transpose
#pragma unroll
          for (int ci = 0; ci < 4; ++ci) {
            Cx<R>* row = M + (C0 + 4 * bq + ci) * a.ld + R0 + 4 * aq;
#pragma unroll
            for (int ri = 0; ri < 4; ++ri) row[ri] = Cx<R>{blk[ri][ci].re, -blk[ri][ci].im};
          }
        }
      }
    }
    if constexpr (PLANES) {
      constexpr int S = 1 << G;  // tile side
      // (r, c) of the tile in LDS: row-major, 16-byte chunks swizzled by row
      auto at = [](int r, int c) { return r * S + 2 * (((c >> 1) ^ r) & (S / 2 - 1)) + (c & 1); };
      __syncthreads();  // every thread is past its round-0 reads of L
      if (active) {
#pragma unroll
        for (int m = 0; m < 16; ++m) L[at(4 * aq + blk_ri(m), 4 * bq + blk_ci(m))] = x[m];
      }
      __syncthreads();
      if (active) {
        // slots of the tile: 2 (tile, mirror) x (S / 32) row blocks x
        // (S / 16) k blocks x 64 lanes, four per thread
        constexpr int UB = (S / 32) * (S / 16);
        const int64_t nkb = (int64_t(1) << a.n) / 16;
        u16x8* PL = static_cast<u16x8*>(a.gplanes);
#pragma unroll
        for (int i = 0; i < (2 * UB * 64) / NT; ++i) {
          const int it = t + NT * i;
          const bool mir = it >= UB * 64;
          if (mir && Rhi == Chi) continue;  // a diagonal tile is its own mirror
          const int ub = (it / 64) % UB, ln = it % 64;
          const int rbl = ub / (S / 16), kbl = ub % (S / 16);
          const int rr = rbl * 32 + (ln & 31), k0 = kbl * 16 + 8 * (ln >> 5);
          float re[8], im[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            // G'[R0 + rr][C0 + k0 + e], or for the mirror G'[C0 + rr][R0 + k0 + e]
            // = conj(G'[R0 + k0 + e][C0 + rr])
            const Cx<R> v = mir ? L[at(k0 + e, rr)] : L[at(rr, k0 + e)];
            re[e] = v.re;
            im[e] = mir ? -v.im : v.im;
          }
          const int64_t rbg = (mir ? C0 : R0) / 32 + rbl, kbg = (mir ? R0 : C0) / 16 + kbl;
          write_unit_block<3>(PL + (rbg * nkb + kbg) * (3 * 3 * kX6UnitVecs) + ln, re, im);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Outcome-side pass (passes 1..): matrix side is the intermediate
// X[(Rr, Cr)][kdone] (lower triangle of the remaining bits), outcome side is
// X'[(Rhi, Chi)][kg * kd + kdone] or, for the last pass (PSIDE), p itself
// (forward) / g' = F - f/p (adjoint).  A workgroup covers one (Rhi, Chi) pair
// and J consecutive kdone values; lanes run over kdone fastest.  Logical
// block lb, thread tid of 256; lds holds 4^G * J values; inactive (a
// padding call): the same loads, rounds and barriers, no stores.
// ---------------------------------------------------------------------------
template <typename R, bool ADJ, bool TETRA, int G, int J, bool PSIDE>
__device__ __forceinline__ void kd_pass_body(const PassArgs& a, const ModeMatrix& A, int64_t lb, unsigned tid,
                                             Cx<R> (&lds)[J << (2 * G)], bool active) {
  constexpr int TILE = 1 << (2 * G);
  constexpr int NB = TILE * J / 16;  // 16-value blocks per workgroup
  constexpr int BPT = NB / 256;      // blocks per thread
  static_assert(NB % 256 == 0, "tile x chunk must give whole blocks per thread");
  using RD = Rounds<G>;
  __builtin_assume(tid < 256);

  const int U = a.U, Up = U - G;
  const int64_t kd = int64_t(1) << (2 * (a.n - U));
  const int64_t nchunks = kd / J;
  const int64_t ch = lb % nchunks;
  int Rhi, Chi;
  tri_decode(lb / nchunks, Rhi, Chi);
  const int64_t kd0 = ch * J;
  const int64_t obase = ((int64_t(Rhi) << Up) | Chi) * (kd * TILE);
  // adjoint from the outcome side: the cotangent F - f/p of (f, p), or with
  // p == NULL the values of f as given
  double F = 0.0;
  if constexpr (ADJ && PSIDE) F = a.p ? *a.F : 0.0;

#pragma unroll
  for (int step = 0; step < RD::n; ++step) {
    const int rd = ADJ ? RD::n - 1 - step : step;
    const int bA = RD::bA[rd], bB = RD::bB[rd];
    const bool first = step == 0, last = step == RD::n - 1;
#pragma unroll
    for (int bi = 0; bi < BPT; ++bi) {
      const int blk = tid + 256 * bi;
      const int j = blk % J;
      const int u = blk / J;  // fixed-bit enumeration
      int rf, cf;
      fixed_bits<G>(u, bA, bB, rf, cf);
      Cx<R> x[16];
      if (first && !ADJ) {  // matrix side in (forward)
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          int r, c;
          rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
          const int64_t Rr = (int64_t(Rhi) << G) | r, Cr = (int64_t(Chi) << G) | c;
          const bool mir = Rr < Cr;
          const int64_t rr = mir ? Cr : Rr, cc = mir ? Rr : Cr;
          Cx<R> v = static_cast<const Cx<R>*>(a.in)[((rr << U) | cc) * kd + kd0 + j];
          if (mir) v.im = -v.im;
          x[m] = v;
        }
      } else if (first) {  // outcome side in (adjoint)
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          const int kg = u + ((m >> 2) << (2 * bA)) + ((m & 3) << (2 * bB));
          if constexpr (PSIDE) {
            const int64_t k = int64_t(kg) * kd + kd0 + j;
            const R fk = static_cast<const R*>(a.f)[k];
            x[m] = Cx<R>{a.p ? cotangent(F, fk, static_cast<const R*>(a.p)[k]) : fk, R(0)};
          } else {
            x[m] = static_cast<const Cx<R>*>(a.in)[obase + int64_t(kg) * kd + kd0 + j];
          }
        }
      } else {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          int r, c;
          rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
          x[m] = lds[((r << G) | c) * J + j];
        }
      }
      contract16<R, ADJ, TETRA>(x, RD::opA[rd], RD::opB[rd], A);
      if (!last) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          int r, c;
          rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
          lds[((r << G) | c) * J + j] = x[m];
        }
      } else if (!active) {
        // padding call of the batched form: same loads and rounds, no stores
      } else if constexpr (!ADJ) {  // outcome side out (forward)
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          const int kg = u + ((m >> 2) << (2 * bA)) + ((m & 3) << (2 * bB));
          if constexpr (PSIDE) {
            static_cast<R*>(a.out)[int64_t(kg) * kd + kd0 + j] = x[m].re;
          } else {
            static_cast<Cx<R>*>(a.out)[obase + int64_t(kg) * kd + kd0 + j] = x[m];
          }
        }
      } else {  // matrix side out (adjoint): lower triangle only
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          int r, c;
          rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
          const int64_t Rr = (int64_t(Rhi) << G) | r, Cr = (int64_t(Chi) << G) | c;
          if (Rr >= Cr) static_cast<Cx<R>*>(a.out)[((Rr << U) | Cr) * kd + kd0 + j] = x[m];
        }
      }
    }
    if (!last) __syncthreads();
  }
}

// Fused last pass (the kd_fused_pass kernel of k_povm_fast.hip): chunk lb
// of J outcome positions, thread tid of 256, lds of 4^G * J values.  F is
// the sum of f; the NLL terms and the bad-entry counts of the chunk are
// added to L, bad0, bad1.  Reads X = a.out and writes the adjoint
// intermediate in place.  Inactive (a padding call): the same loads,
// rounds and barriers, nothing stored or counted.  FC: the classical
// fidelity terms sqrt(max(p_k, 0) max(pt_k, 0)) against a.pt (loaded
// before the last round's contraction) are added to *fc, the square root in
// the storage precision.
template <typename R, bool TETRA, int G, int J, bool FC = false>
__device__ __forceinline__ void kd_fused_body(const PassArgs& a, const ModeMatrix& Af, const ModeMatrix& Aa, int64_t lb,
                                              unsigned tid, Cx<R> (&lds)[J << (2 * G)], bool active, double F,
                                              double& L, double& bad0, double& bad1, double* fc = nullptr) {
  constexpr int TILE = 1 << (2 * G);
  constexpr int NB = TILE * J / 16;
  constexpr int BPT = NB / 256;
  static_assert(NB % 256 == 0, "tile x chunk must give whole blocks per thread");
  using RD = Rounds<G>;
  static_assert(RD::n >= 2, "the fused pass needs a round to exchange between");
  __builtin_assume(tid < 256);

  const int U = a.U;  // == G
  // element indices of X, f and the target stay below 4^N <= 2^26 (N <= 13):
  // 32-bit, which saves 64-bit vector address arithmetic
  static_assert(QST_MAX_QUBITS <= 15, "32-bit outcome indices");
  const uint32_t kd = 1u << (2 * (a.n - U));
  const uint32_t kd0 = uint32_t(lb) * J;
  Cx<R>* X = static_cast<Cx<R>*>(a.out);  // in place: a.in == a.out
  const R* f = static_cast<const R*>(a.f);
  // f for the outcomes of the last round, loaded now so that it arrives
  // while the forward rounds run
  R fpre[BPT][16];
  {
    constexpr int rl = RD::n - 1;
#pragma unroll
    for (int bi = 0; bi < BPT; ++bi) {
      const int blk = tid + 256 * bi;
      const int j = blk % J;
      const int u = blk / J;
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int kg = u + ((m >> 2) << (2 * RD::bA[rl])) + ((m & 3) << (2 * RD::bB[rl]));
        fpre[bi][m] = f[uint32_t(kg) * kd + kd0 + j];
      }
    }
  }

  // forward rounds; the last one continues into the cotangent and the
  // adjoint of the same round
#pragma unroll
  for (int rd = 0; rd < RD::n; ++rd) {
    const int bA = RD::bA[rd], bB = RD::bB[rd];
    const bool first = rd == 0, last = rd == RD::n - 1;
#pragma unroll
    for (int bi = 0; bi < BPT; ++bi) {
      const int blk = tid + 256 * bi;
      const int j = blk % J;
      const int u = blk / J;
      int rf, cf;
      fixed_bits<G>(u, bA, bB, rf, cf);
      Cx<R> x[16];
      if (first) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          int r, c;
          rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
          const bool mir = r < c;
          const int rr = mir ? c : r, cc = mir ? r : c;
          Cx<R> v = X[((uint32_t(rr) << U) | uint32_t(cc)) * kd + kd0 + j];
          if (mir) v.im = -v.im;
          x[m] = v;
        }
      } else {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          int r, c;
          rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
          x[m] = lds[((r << G) | c) * J + j];
        }
      }
      // F_c target of this block's outcomes (last round only), loaded here
      // so that the forward contraction covers part of its latency and only
      // these 16 values stay live (a prefetch with f measured slower)
      R qk[FC ? 16 : 1];
      if constexpr (FC) {
        if (last) {
#pragma unroll
          for (int m = 0; m < 16; ++m) {
            const int kg = u + ((m >> 2) << (2 * bA)) + ((m & 3) << (2 * bB));
            qk[m] = static_cast<const R*>(a.pt)[uint32_t(kg) * kd + kd0 + j];
          }
        }
      }
      contract16<R, false, TETRA>(x, RD::opA[rd], RD::opB[rd], Af);
      if (last) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          const R fr = fpre[bi][m], pr = x[m].re;
          const double fk = active ? double(fr) : 0.0, pk = double(pr);
          if (fk != 0.0) {
            if (pk > 0.0) {
              L -= fk * ln_prob(pr);
            } else {
              bad0 += 1.0;
            }
          }
          if (active && (pk != pk || fk != fk)) bad1 += 1.0;
          if constexpr (FC) {
            // the square root in the storage precision, the sum in FP64
            const R zero = R(0);
            if (active) *fc += double(sqrt((pr > zero ? pr : zero) * (qk[m] > zero ? qk[m] : zero)));
          }
          x[m] = Cx<R>{cotangent(F, fr, pr), R(0)};
        }
        contract16<R, true, TETRA>(x, RD::opA[rd], RD::opB[rd], Aa);
      }
      // the exchange positions of this block are this thread's alone in the
      // round, so the adjoint values can replace the forward ones directly
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        int r, c;
        rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
        lds[((r << G) | c) * J + j] = x[m];
      }
    }
    __syncthreads();
  }
  // remaining adjoint rounds, last forward round excluded
#pragma unroll
  for (int rd = RD::n - 2; rd >= 0; --rd) {
    const int bA = RD::bA[rd], bB = RD::bB[rd];
#pragma unroll
    for (int bi = 0; bi < BPT; ++bi) {
      const int blk = tid + 256 * bi;
      const int j = blk % J;
      const int u = blk / J;
      int rf, cf;
      fixed_bits<G>(u, bA, bB, rf, cf);
      Cx<R> x[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        int r, c;
        rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
        x[m] = lds[((r << G) | c) * J + j];
      }
      contract16<R, true, TETRA>(x, RD::opA[rd], RD::opB[rd], Aa);
      if (rd > 0) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          int r, c;
          rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
          lds[((r << G) | c) * J + j] = x[m];
        }
      } else if (active) {  // matrix side out: lower triangle only
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          int r, c;
          rc_of(rf, cf, bA, bB, m >> 2, m & 3, r, c);
          if (r >= c) X[((uint32_t(r) << U) | uint32_t(c)) * kd + kd0 + j] = x[m];
        }
      }
    }
    if (rd > 0) __syncthreads();
  }
}


}  // namespace fast_pass
}  // namespace qst
