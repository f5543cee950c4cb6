// Specialised product-POVM passes for the group shapes of N >= 7 (tetrahedral
// and generic POVMs).  Same mathematics and data layout as the generic pass
// kernels in k_povm.hip (see the comment there); what differs is how a
// workgroup moves data:
//
//  * the group size G and chunk J are compile-time constants, so all index
//    arithmetic is shifts and masks;
//  * every thread holds 16 values: all (row, column) combinations of two
//    qubit bits, times one output chunk position.  Two qubits are contracted
//    in registers per round, so a G-qubit group takes ceil(G/2) rounds with
//    one LDS exchange between rounds instead of one per qubit;
//  * the round touching the matrix side reads or writes 4 x 4 blocks of
//    consecutive columns (16- or 32-byte accesses); the round touching the
//    outcome side maps consecutive threads to consecutive outcome indices.
//
// Rounds (bits are the group-local qubit bit positions, 0 = least
// significant; a round holds two bits per thread and applies the per-qubit
// contraction to the listed ones):
//   G=3: {0,1} ops 0,1 | {1,2} op 2
//   G=4: {0,1} ops 0,1 | {2,3} ops 2,3
//   G=5: {0,1} ops 0,1 | {2,3} op 2 | {3,4} ops 3,4
//   G=6: {0,1} ops 0,1 | {2,3} ops 2,3 | {4,5} ops 4,5
// The forward map runs the rounds in this order (matrix side first), the
// adjoint in reverse (outcome side first).
#include "qst_device.h"
#include "qst_kernels.h"
#include "qst_povm_ops.h"
#include "qst_povm_fast.h"
#include "qst_povm_rounds.h"

namespace qst {

namespace {

// ---------------------------------------------------------------------------
// Matrix-side pass (pass 0) and outcome-side passes (passes 1..): one
// logical block per workgroup (fast_pass::mat_pass_body / kd_pass_body).
// ---------------------------------------------------------------------------
template <typename R, bool ADJ, bool TETRA, int G, bool PLANES = false>
__global__ __launch_bounds__(256) void mat_pass(PassArgs a, ModeMatrix A, int64_t ntiles) {
  constexpr int TPW = 256 >> (2 * (G - 2));
  __shared__ Cx<R> lds[TPW << (2 * G)];
  fast_pass::mat_pass_body<R, ADJ, TETRA, G, PLANES>(a, A, ntiles, blockIdx.x, threadIdx.x, lds);
}

template <typename R, bool ADJ, bool TETRA, int G, int J, bool PSIDE>
__global__ __launch_bounds__(256) void kd_pass(PassArgs a, ModeMatrix A) {
  __shared__ Cx<R> lds[J << (2 * G)];
  // J consecutive outcomes are 32..128 bytes; the chunks sharing a cache
  // line must run on the same XCD (see xcd_order)
  fast_pass::kd_pass_body<R, ADJ, TETRA, G, J, PSIDE>(a, A, xcd_order(blockIdx.x, gridDim.x), threadIdx.x, lds,
                                                      true);
}

// ---------------------------------------------------------------------------
// Last pass fused with the likelihood.  The last pass has a single (R, C)
// pair (all remaining qubits are contracted), so a workgroup owns J
// consecutive kdone values of the whole 2^G x 2^G block.  It runs the forward
// rounds (p for 16 outcomes per register block after the last round), the
// NLL terms and the cotangent g'_k = F - f_k / p_k in registers (F from the
// partial sums of the tau kernel, summed in the same fixed order by every
// workgroup), then the adjoint rounds in reverse, starting from the same
// registers (the adjoint's first round is the forward's last round).  Reads X
// and writes Y = adjoint intermediate at the same addresses (in place: every
// address a workgroup writes is one it alone has read, and all its reads
// precede its first write by a barrier).
// ---------------------------------------------------------------------------
// The F_c form holds the target's values besides the rest and would spill
// at two workgroups per CU; it runs at one.
template <typename R, bool TETRA, int G, int J, bool FC = false>
__global__ __launch_bounds__(256, FC ? 1 : 2) void kd_fused_pass(PassArgs a, ModeMatrix Af, ModeMatrix Aa) {
  __shared__ Cx<R> lds[J << (2 * G)];
  __shared__ double red[4];
  __shared__ double Fsh;
  const int64_t lb = xcd_order(blockIdx.x, gridDim.x);
  {
    const double Fsum = sum_partials256(a.Fpart, kReduceBlocks, red);
    if (threadIdx.x == 0) Fsh = Fsum;
    __syncthreads();
  }
  double L = 0.0, bad0 = 0.0, bad1 = 0.0, fc = 0.0;
  fast_pass::kd_fused_body<R, TETRA, G, J, FC>(a, Af, Aa, lb, threadIdx.x, lds, true, Fsh, L, bad0, bad1, &fc);
  // per-workgroup partial sums in a fixed order, slot = logical index
  const int64_t nb = gridDim.x;
  double v = block_sum256(L, red);
  if (threadIdx.x == 0) a.part[lb] = v;
  if constexpr (FC) {
    v = block_sum256(fc, red);
    if (threadIdx.x == 0) a.part[nb + lb] = v;
  }
  v = block_sum256(bad0, red);
  if (threadIdx.x == 0) a.part[2 * nb + lb] = v;
  v = block_sum256(bad1, red);
  if (threadIdx.x == 0) a.part[3 * nb + lb] = v;
}

}  // namespace

// Fused last pass; false when no specialised form covers (g, J).
bool launch_fused_fast(qst_prec prec, bool tetra, const PassArgs& a, const ModeMatrix& Af,
                       const ModeMatrix& Aa, int64_t blocks, hipStream_t s, hipError_t* err) {
  const unsigned grid = unsigned(blocks);
#define QST_FU(R, G, J)                                                              \
  do {                                                                               \
    if (a.pt && tetra) kd_fused_pass<R, true, G, J, true><<<grid, 256, 0, s>>>(a, Af, Aa);   \
    else if (a.pt) kd_fused_pass<R, false, G, J, true><<<grid, 256, 0, s>>>(a, Af, Aa);     \
    else if (tetra) kd_fused_pass<R, true, G, J><<<grid, 256, 0, s>>>(a, Af, Aa);    \
    else kd_fused_pass<R, false, G, J><<<grid, 256, 0, s>>>(a, Af, Aa);              \
  } while (0)
  const int g = a.g, J = a.J;
  if (prec == QST_F64) {
    if (g == 5 && J == 4) QST_FU(double, 5, 4);
    else if (g == 4 && J == 16) QST_FU(double, 4, 16);
    else if (g == 3 && J == 64) QST_FU(double, 3, 64);
    else return false;
  } else {
    if (g == 5 && J == 8) QST_FU(float, 5, 8);
    else if (g == 4 && J == 32) QST_FU(float, 4, 32);
    else if (g == 3 && J == 64) QST_FU(float, 3, 64);
    else return false;
  }
#undef QST_FU
  *err = hipGetLastError();
  return true;
}

// Returns true and launches when a specialised kernel covers the pass.
bool launch_pass_fast(bool adjoint, qst_prec prec, bool tetra, const PassArgs& a, const ModeMatrix& A,
                      bool matside, bool pside, int64_t blocks, hipStream_t s, hipError_t* err) {
  const bool f64 = prec == QST_F64;
#define QST_MAT(R, ADJ, TET, G)                                                                   \
  do {                                                                                            \
    constexpr int TPW = 256 >> (2 * (G - 2));                                                     \
    const unsigned grid = unsigned((blocks + TPW - 1) / TPW);                                     \
    mat_pass<R, ADJ, TET, G><<<grid, 256, 0, s>>>(a, A, blocks);                                  \
  } while (0)
#define QST_MAT_ALL(G)                                                                            \
  do {                                                                                            \
    if (f64) {                                                                                    \
      if (adjoint) { if (tetra) QST_MAT(double, true, true, G); else QST_MAT(double, true, false, G); } \
      else { if (tetra) QST_MAT(double, false, true, G); else QST_MAT(double, false, false, G); }  \
    } else {                                                                                      \
      if (adjoint) { if (tetra) QST_MAT(float, true, true, G); else QST_MAT(float, true, false, G); } \
      else { if (tetra) QST_MAT(float, false, true, G); else QST_MAT(float, false, false, G); }    \
    }                                                                                             \
  } while (0)
  if (matside && adjoint && a.gplanes) {  // G' as split planes: FP32 adjoint, g = 5 or 6
    if (f64 || pside || a.J != 1 || a.g < 5 || a.g > 6) return false;
    const unsigned grid = unsigned((blocks + (256 >> (2 * (a.g - 2))) - 1) / (256 >> (2 * (a.g - 2))));
    if (a.g == 5) {
      if (tetra) mat_pass<float, true, true, 5, true><<<grid, 256, 0, s>>>(a, A, blocks);
      else mat_pass<float, true, false, 5, true><<<grid, 256, 0, s>>>(a, A, blocks);
    } else {
      if (tetra) mat_pass<float, true, true, 6, true><<<grid, 256, 0, s>>>(a, A, blocks);
      else mat_pass<float, true, false, 6, true><<<grid, 256, 0, s>>>(a, A, blocks);
    }
    *err = hipGetLastError();
    return true;
  }
  if (matside && !pside && a.J == 1 && a.g >= 4 && a.g <= 6) {
    if (a.g == 4) QST_MAT_ALL(4);
    else if (a.g == 5) QST_MAT_ALL(5);
    else QST_MAT_ALL(6);
    *err = hipGetLastError();
    return true;
  }
#undef QST_MAT_ALL
#undef QST_MAT
#define QST_KD(R, ADJ, TET, G, J, P) kd_pass<R, ADJ, TET, G, J, P><<<unsigned(blocks), 256, 0, s>>>(a, A)
#define QST_KD_P(R, ADJ, TET, G, J)                                                               \
  do {                                                                                            \
    if (pside) QST_KD(R, ADJ, TET, G, J, true); else QST_KD(R, ADJ, TET, G, J, false);          \
  } while (0)
#define QST_KD_ALL(R, G, J)                                                                       \
  do {                                                                                            \
    if (adjoint) { if (tetra) QST_KD_P(R, true, true, G, J); else QST_KD_P(R, true, false, G, J); } \
    else { if (tetra) QST_KD_P(R, false, true, G, J); else QST_KD_P(R, false, false, G, J); }      \
  } while (0)
  if (!matside) {
    const int g = a.g, J = a.J;
    bool ok = true;
    if (f64) {
      if (g == 5 && J == 4) QST_KD_ALL(double, 5, 4);
      else if (g == 4 && J == 16) QST_KD_ALL(double, 4, 16);
      else if (g == 3 && J == 64) QST_KD_ALL(double, 3, 64);
      else ok = false;
    } else {
      if (g == 5 && J == 8) QST_KD_ALL(float, 5, 8);
      else if (g == 4 && J == 32) QST_KD_ALL(float, 4, 32);
      else if (g == 3 && J == 64) QST_KD_ALL(float, 3, 64);
      else ok = false;
    }
    if (ok) {
      *err = hipGetLastError();
      return true;
    }
  }
#undef QST_KD_ALL
#undef QST_KD_P
#undef QST_KD
  return false;
}

}  // namespace qst
