// Host-side planning shared by the HIP entry points and the HIP-free
// validation unit: argument checks, POVM pass plans, workspace layout.
// Nothing in this header touches the HIP runtime.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "qst.h"

namespace qst {

// Elements of one complex scalar in bytes for a precision's storage type.
inline size_t complex_bytes(qst_prec p) { return p == QST_F64 ? 16 : 8; }
inline size_t real_bytes(qst_prec p) { return p == QST_F64 ? 8 : 4; }
inline bool prec_valid(int p) { return p == QST_F64 || p == QST_F32 || p == QST_BF16GEMM || p == QST_F32X6; }
// Storage and pass arithmetic of a precision (QST_F32X6 differs from
// QST_F32 in its complex products only).
inline qst_prec storage_prec(qst_prec p) { return p == QST_F32X6 ? QST_F32 : p; }

// QST_F32X6 products (k_xgemm.hip): 128 x 128 output tiles; T T^dagger runs
// stream-K on at most kX6MaxGrid workgroups, each leaving at most two
// partial tiles (re, im FP32).  Operand planes: T T^dagger reads the rows of
// T in four groups (re, im, re + im, re - im) of three bf16 splits (24 bytes
// per element); G' T reads G' and T^T in three groups (18 bytes each).
constexpr int kX6Tile = 128;
constexpr int kX6MaxGrid = 256;
inline bool use_x6(qst_prec p, int n) { return p == QST_F32X6 && (int64_t(1) << n) >= kX6Tile; }
// Schedule of the QST_F32X6 T T^dagger (lower 128 x 128 tiles) on P
// workgroups, one per CU.  Each tile's K range is cut into sk equal parts
// ("units"; sk the smallest power of two with tiles x sk >= P, each unit at
// least 8 K panels).  Workgroup w takes units w, w + P, ... for `rounds`
// whole rounds -- every workgroup of a round covers the same K range at the
// same time, so the operand panels it streams are shared in L2 -- and the
// `left` units that remain are shared out as contiguous slices of their
// (unit, panel) sequence (stream-K), at most two slices per workgroup.  A
// tile finished by one workgroup (sk = 1, a whole round unit) is written
// directly; every other contribution is a partial tile that the fix-up adds
// in K order.
struct X6HerkSched {
  int64_t P = 1;  // workgroups of the rounds (one per CU)
  int64_t Q = 1;  // workgroups taking slices
  int64_t ntiles = 0, sk = 1, kh = 0, units = 0, rounds = 0, main = 0, left = 0, left_iters = 0;
  int64_t slots = 0;  // partial tiles: one per round unit when sk > 1, two per slice worker (one with tq)
  int64_t tq = 0;     // transposed slices: slices per leftover unit (0: contiguous slices)
  int64_t ps = 0;     // panels per transposed slice
};
inline X6HerkSched x6_herk_sched(int n, int cus) {
  X6HerkSched s;
  const int64_t d = int64_t(1) << n, t = d / kX6Tile, kiters = d / 16;
  s.P = cus < 1 ? 1 : (cus > kX6MaxGrid ? kX6MaxGrid : cus);
  s.ntiles = t * (t + 1) / 2;
  while (s.ntiles * s.sk < s.P && kiters / (2 * s.sk) >= 8) s.sk *= 2;
  s.kh = kiters / s.sk;
  // rounds only with units of at least 32 panels; otherwise the units are
  // the tiles and all of them are shared out in slices (plain stream-K: a
  // slice then holds whole tiles and at most two partial ones)
  if (s.kh < 32) {
    s.sk = 1;
    s.kh = kiters;
  }
  s.units = s.ntiles * s.sk;
  s.rounds = s.units / s.P;
  s.main = s.rounds * s.P;
  s.left = s.units - s.main;
  s.left_iters = s.left * s.kh;
  // slices of at least 4 panels after rounds (all workgroups share the
  // tail), 16 without them
  const int64_t min_slice = s.rounds > 0 ? 4 : 16;
  s.Q = s.left_iters / min_slice;
  if (s.Q > s.P) s.Q = s.P;
  if (s.Q < 1) s.Q = 1;
  if (s.left_iters == 0) s.Q = 0;
  // After rounds, when the leftover units split evenly into the Q slices,
  // slice worker w takes the (w / left)-th of the tq equal slices of unit
  // w % left: the workers of an XCD (consecutive w) then stream the same K
  // panels of several tiles at once, and every slice lies inside one unit
  // (one partial tile each).
  if (s.rounds > 0 && s.left > 0 && s.Q % s.left == 0 && s.kh % (s.Q / s.left) == 0) {
    s.tq = s.Q / s.left;
    s.ps = s.kh / s.tq;
  }
  s.slots = (s.sk > 1 ? s.main : 0) + (s.tq ? s.Q : 2 * s.Q);
  return s;
}
inline size_t x6_partial_bytes(int n) {
  // the largest schedule over devices with up to kX6MaxGrid compute units
  size_t most = 0;
  for (int cus = 1; cus <= kX6MaxGrid; ++cus) {
    const size_t slots = size_t(x6_herk_sched(n, cus).slots);
    if (slots > most) most = slots;
  }
  return most * 2 * kX6Tile * kX6Tile * sizeof(float);
}
inline size_t x6_herk_plane_bytes(int n) { return (size_t(1) << (2 * n)) * 24; }
inline size_t x6_hemm_plane_bytes(int n) { return (size_t(1) << (2 * n)) * 36; }

// The product-POVM map is applied in passes.  Pass j contracts a group of
// g_j consecutive qubits inside on-chip memory; groups run from the least
// significant qubits (qubit N, N-1, ...) to qubit 1.  Before pass j the
// intermediate is indexed [(R, C)][kdone]: R, C are the row/column bits of
// the U_j qubits not yet contracted and kdone the outcome digits of the
// contracted ones (4^(N-U_j) values, qubit N least significant).
struct PovmPlan {
  int n = 0;           // qubits
  int passes = 0;      // number of passes
  int g[4] = {0};      // group size of pass j (pass 0 = lowest qubits)
  int U[4] = {0};      // remaining qubits before pass j
  int J[4] = {0};      // consecutive kdone values per workgroup in pass j
};

// Largest group a pass may hold on chip: 4^g * J complex values in a 64 KiB
// LDS buffer.
PovmPlan make_povm_plan(int n, qst_prec prec);

// Workgroups launched by a pass (lower block triangle of (R, C) times kdone
// chunks).
int64_t povm_pass_blocks(const PovmPlan& pl, int j);

// Whether pass j has a specialised kernel (k_povm_fast.hip): matrix-side
// passes with g in 4..6; outcome-side passes with (g, J) in
// {(5,4), (4,16), (3,64)} for FP64 and {(5,8), (4,32), (3,64)} otherwise.
bool fast_pass_available(const PovmPlan& pl, int j, qst_prec prec);

// Whether the likelihood call fuses the last POVM pass with the NLL, the
// cotangent and the first adjoint pass: at least two passes, all of them
// specialised.
bool fused_likelihood(const PovmPlan& pl, qst_prec prec);

// Whether adjoint pass 0 of a fused plan can write G' as split operand
// planes (first group of 5 or 6 qubits: tiles of at least 32 rows).
inline bool pass0_writes_planes(const PovmPlan& pl) { return pl.passes >= 2 && (pl.g[0] == 5 || pl.g[0] == 6); }

// Absolute-map workspace (qst_abs_map, qst_abs_map_backward): three d x d
// complex FP64 buffers, d FP64 values (Jacobi norm partials, then
// |lambda|^(P/4)), a few FP64 scalars and the FP64 stream-K partial tiles of
// the complex products (N >= kStreamKMinQubits).
struct AbsMapLayout {
  size_t b0 = 0, b1 = 0, b2 = 0, part = 0, scal = 0, state = 0, sk = 0, sk_bytes = 0, eig = 0, total = 0;
};
// The direct eigensolver's small arrays (offsets from AbsMapLayout::eig):
// the tridiagonal (diagonal, off-diagonal), the reflector scalars, the two
// ping-pong matrix-vector products and their partial sums, the unreduced
// block of every index, scalars and status, and the triangular factors of
// the blocked back-transformation.
constexpr int kEighBlock = 64;          // reflectors per back-transformation block
constexpr int kTrdMaxGroups = 256;      // workgroups of a reduction step
struct EighLayout {
  size_t diag = 0, off = 0, tau = 0, y0 = 0, y1 = 0, p0 = 0, p1 = 0, bstart = 0, bend = 0, scal = 0, tfac = 0,
         pbuf = 0, xbuf = 0, total = 0;
};
EighLayout eigh_layout(int n);
// Rows per partial-sum chunk of the back-transformation (a multiple of 16):
// d / 16 from d = 1024, else 64, so that there are at most 16 chunks (at
// most d / 64 below 1024).
inline int eigh_chunk_rows(int d) { return d / 16 > 64 ? d / 16 : 64; }
// Rows per partial Gram matrix of a block of reflectors, and their number.
constexpr int kEighGramRows = 128;
inline int eigh_gram_chunks(int d) { return (d - 1 + kEighGramRows - 1) / kEighGramRows; }
// Jacobi sweeps the absolute map and the general fidelity allow (the
// graph-capturable calls take a smaller bound of their own).
constexpr int kJacobiMaxSweeps = 40;
AbsMapLayout absmap_layout(int n);
qst_status check_abs_order(double P, std::string& msg);  // P finite and >= 0

// Workspace layout (byte offsets) for each op; see the .cpp for the rules.
struct WsLayout {
  size_t total = 0;
  size_t partials = 0;   // FP64 reduction partials
  size_t scalars = 0;    // small FP64 scalars (F, tau when recomputed, L)
  size_t inter0 = 0;     // first POVM intermediate (4^N complex)
  size_t inter1 = 0;     // second POVM intermediate (4^N complex, >2 passes)
  size_t gmat = 0;       // G' (d x d complex), backward only
  size_t rho = 0;        // rho (d x d complex), recompute mode only
  size_t p = 0;          // p (4^N real), recompute mode only
  size_t sk = 0;         // stream-K partial tiles (0 = not used)
  size_t fpart = 0;      // fused likelihood pass: FP64 partials [4][blocks]
  size_t planes = 0;     // BF16 path: bf16(T) as re and im planes for T T^dagger (d > kBf16SplitMaxDim,
                         // 4 d^2 bytes); split planes of G' and T^T for G' T (d >= 1024, 16 d^2 bytes)
  size_t tplanes = 0;    // combined likelihood-and-gradient call: planes of G' T (G''s, then T^T's)
  bool has_sk = false;
  bool has_planes = false;
  bool has_tplanes = false;
};

WsLayout workspace_layout(int n, qst_prec prec, int op, bool recompute);

constexpr int kReduceBlocks = 1024;  // stage-1 blocks of every FP64 reduction
constexpr int kReduceThreads = 256;

// Stream-K scheduling of the complex products: at most this many
// workgroups, each leaving at most two partial 64 x 64 complex tiles.
constexpr int kStreamKMaxGrid = 1024;
constexpr int kStreamKMinQubits = 10;

// BF16 path: T T^dagger uses plain bf16 T for d > this, split bf16 hi + lo
// (three products) up to it, where plain rounding of T moves the gradient by
// more than 2e-3 relative (measured with the FP64 oracle: up to 4.3e-3 at
// d = 8, 2.9e-3 at d = 64, 1.4e-3 at d = 128, 7.1e-4 at d = 256).
constexpr int kBf16SplitMaxDim = 128;  // smaller products always run one tile per workgroup
inline size_t stream_k_partial_bytes(qst_prec p) {
  return size_t(kStreamKMaxGrid) * 2 * (2 * 64 * 64) * (p == QST_F64 ? 8 : 4);
}

// Fidelity workspace (qst_fidelity_lowrank / qst_fidelity_classical):
// W^dagger T partial sums over nrb row blocks and their total M (complex
// FP64, sized for the largest rank), the r x r Gram matrix, per-workgroup |T|^2 partials and the
// classical-fidelity partials.
constexpr int kFidelityMaxRank = QST_FIDELITY_MAX_RANK;
struct FidelityLayout {
  int nrb = 1;
  size_t mpart = 0, mrow = 0, gram = 0, taup = 0, cpart = 0, total = 0;
};
FidelityLayout fidelity_layout(int n);

// Mapping network workspace: FP64 block partials of the two H-wide sums,
// h and dL/dh_pre (FP64), and the 4^N outputs y (or dL/dy) in storage
// precision.
constexpr int kFnnMaxHidden = 2 * QST_MAX_QUBITS;
constexpr int kFnnBlocks = 1024;
struct FnnLayout {
  size_t part = 0, hvec = 0, dhvec = 0, yvec = 0, total = 0;
};
FnnLayout fnn_layout(int n, size_t real_bytes);

// Argument validation.  Each returns QST_OK or an error status and fills msg.
qst_status check_common(int n, int prec, std::string& msg);
qst_status check_matrix(const void* ptr, int64_t ld, int n, const char* name, std::string& msg);
qst_status check_ptr(const void* ptr, const char* name, std::string& msg);
qst_status check_ws(const void* ws, size_t ws_bytes, size_t need, std::string& msg);
qst_status check_povm(const double* povm_host, std::string& msg);
// Mode and in-place rule of qst_state_premap (Y == X needs ldY == ldX).
qst_status check_premap(int mode, const void* X, int64_t ldX, const void* Y, int64_t ldY, std::string& msg);

// Per-thread last-error message.
void set_error(const std::string& msg);
void clear_error();
const char* last_error_cstr();

// Forward mode matrix W[a][m] (m = 2r + c) = (M_a)_{c,r} and adjoint mode
// matrix V[m][a] = (M_a)_{r,c}, as 4 x 4 complex (re, im) in row-major
// double[32], from a POVM given as in qst_povm_probs.
void povm_mode_matrices(const double* povm_host, double W[32], double V[32]);

// General product POVMs (qst_povm_probs_general, qst_likelihood_general):
// K outcomes per qubit (2 <= K <= kGeneralMaxK), a POVM of its own on each
// qubit, up to kGeneralMaxSettings settings, K^N <= kGeneralMaxOutcomes.
constexpr int kGeneralMaxK = 8;
constexpr int kGeneralMaxSettings = 64;
constexpr int64_t kGeneralMaxOutcomes = int64_t(1) << 30;
// K^N, or -1 when it exceeds kGeneralMaxOutcomes.
int64_t general_outcomes(int n, int K);
// Shape limits and, for every setting and qubit, a POVM: each element
// Hermitian and positive semidefinite, the K elements summing to I
// (povm_host: settings x N x K x 2 x 2 complex (re, im), row-major).
qst_status check_povm_general(int n, int K, int settings, const double* povm_host, std::string& msg);
// Real per-qubit factors C[s][i][k][b] = Tr(M^(s,i)_k P_b) / 2 over the
// Pauli basis P = (I, X, Y, Z): Tr(M_k sigma) = sum_b C[k][b] Tr(P_b sigma).
void general_factors(int n, int K, int settings, const double* povm_host, double* C);
// Mode matrices (as povm_mode_matrices) of the Pauli set (I, X, Y, Z):
// the forward map then gives the Pauli coordinates Tr(P_b rho), the
// adjoint map the synthesis sum_b h_b P_b.
void pauli_mode_matrices(double W[32], double V[32]);

// Workspace of the general-POVM calls (byte offsets).  with_state: the
// likelihood call (state map, rho, settings' probabilities, adjoint);
// otherwise qst_povm_probs_general (Pauli passes and the real passes).
struct GeneralLayout {
  size_t partials = 0, scal = 0, sk = 0, planes = 0, rho = 0, inter0 = 0, inter1 = 0;
  size_t e = 0, h = 0, bufA = 0, bufB = 0, p = 0, total = 0;
  bool has_sk = false, has_planes = false;
};
GeneralLayout general_layout(int n, qst_prec prec, int K, bool with_state);

}  // namespace qst
