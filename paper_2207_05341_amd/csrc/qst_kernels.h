// Launchers of the gfx950 kernels (host side).  Each enqueues work on the
// given stream and returns hipGetLastError().
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "qst.h"
#include "qst_plan.h"

namespace qst {

// Brackets the kernel launched while it is alive with timing events when
// qst_profile_enable(1) is in effect (no-op otherwise).  With in_launch, the
// scope records nothing itself: its one kernel is launched with
// hipExtLaunchKernelGGL(..., start(), stop(), ...), whose events are stamped
// when that dispatch starts and ends (no queue time of separate event
// packets in the interval); start() and stop() are NULL when inactive.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t s, bool in_launch = false);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;
  hipEvent_t start() const { return a_; }
  hipEvent_t stop() const { return b_; }

 private:
  int idx_ = -1;
  hipStream_t s_;
  bool in_launch_ = false;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

// tau = sum |T_ij|^2 (FP64; over bf16-rounded T for QST_BF16GEMM): the
// kReduceBlocks partial sums, and, if tau_dev is not NULL, their total.  With
// f (4^N reals), also the kReduceBlocks partial sums of F = sum f at
// partials + kReduceBlocks.  planes (QST_BF16GEMM with d > kBf16SplitMaxDim,
// else ignored; may be NULL): receives bf16(T) as re and im planes (d x d
// row-major each, 4 d^2 bytes), the operands launch_herk takes.
// Mapping network (workspace laid out by fnn_layout).
hipError_t launch_fnn_forward(qst_prec prec, int n, const void* W1, const void* b1, const void* W2, const void* b2,
                              const void* x, void* h_pre, void* T, int64_t ldT, void* ws, hipStream_t s);
hipError_t launch_fnn_backward(qst_prec prec, int n, const void* W2, const void* x, const void* h_pre, const void* G,
                               int64_t ldG, void* dW1, void* db1, void* dW2, void* db2, void* ws, hipStream_t s);

// One Rprop step over count entries.
hipError_t launch_rprop(qst_prec prec, int64_t count, void* w, const void* g, void* prev, void* step, double eta_minus,
                        double eta_plus, double smin, double smax, hipStream_t s);

// Fidelities (workspace laid out by fidelity_layout).
hipError_t launch_fidelity_lowrank(qst_prec prec, const void* T, int64_t ldT, const void* W, int64_t ldW, int r,
                                   int n, void* ws, double* F, hipStream_t s);
// F_c with the kReduceBlocks partials at part.
hipError_t launch_fidelity_classical_part(qst_prec prec, const void* ph, const void* p, int n, double* part, double* F,
                                          hipStream_t s);
hipError_t launch_fidelity_classical(qst_prec prec, const void* ph, const void* p, int n, void* ws, double* F,
                                     hipStream_t s);

// Direct Hermitian eigensolver (FP64; k_eigh.hip), its small arrays laid
// out by eigh_layout in the absolute map's workspace.
struct EighWork {
  double *diag = nullptr, *off = nullptr, *p0 = nullptr, *p1 = nullptr;
  void *tau = nullptr, *y0 = nullptr, *y1 = nullptr, *scal = nullptr, *tfac = nullptr, *pbuf = nullptr,
       *xbuf = nullptr;
  int *bstart = nullptr, *bend = nullptr, *status = nullptr;
};
EighWork eigh_work(int n, void* eig_area);
// H (d x d complex FP64, Hermitian, both triangles; overwritten) -> the
// tridiagonal (w.diag, w.off), the reflector scalars (w.tau) and the
// reflector rows in V (d x d complex FP64).
hipError_t launch_tridiagonalize(int n, void* A, void* V, const EighWork& w, hipStream_t s);
// Splits the tridiagonal, sets *w.status (0, or -1 if not finite), and the
// eigenvalues (lam, d values; ascending within each unreduced block).
hipError_t launch_tri_eigvals(int n, const EighWork& w, double* lam, hipStream_t s);
// The orthonormal eigenvectors of the tridiagonal as the columns of Z (d x d
// complex FP64, real values); scratch: d x d complex FP64.
hipError_t launch_tri_vectors(int n, const EighWork& w, const double* lam, void* scratch, void* Z, hipStream_t s);
// M = 1.5 I - 0.5 G (the Newton-Schulz matrix), d x d complex FP64.
hipError_t launch_ns_matrix(int n, const void* G, void* M, hipStream_t s);
// Z <- Q_H Z with Q_H the product of the reflectors (V, w.tau), in place;
// W: d x d complex FP64 scratch (the blocks' V T factors).
hipError_t launch_back_transform(int n, const void* V, const EighWork& w, void* Z, void* W, hipStream_t s);
// *out = *w.status.
hipError_t launch_eigh_status(const EighWork& w, int* out, hipStream_t s);

// P-order absolute map and its adjoint (workspace laid out by
// absmap_layout).  At most max_sweeps Jacobi sweeps, the stopping rule
// decided on the device.  sweeps_dev == NULL: synchronous -- the host reads
// the decision after each sweep, stops enqueuing once it holds, and sets
// *sweeps to the sweeps taken or -1 (norm not finite, or not converged;
// nothing after the sweeps is launched then).  Otherwise asynchronous and
// graph-capturable: all max_sweeps are enqueued (the rounds after
// convergence return at once), the rest of the map always runs, and the
// sweeps taken (or -1) land in the device int *sweeps_dev.
hipError_t launch_abs_map(qst_prec prec, int n, double P, const void* T, int64_t ldT, const void* Q0, void* A,
                          int64_t ldA, void* Q, double* lam, void* ws, hipStream_t s, int* sweeps, int max_sweeps,
                          int* sweeps_dev);
// F_q against a general target rho: one eigensolve of T^dagger rho T (the
// absolute-map workspace; sweeps as launch_abs_map).
hipError_t launch_fidelity_general(qst_prec prec, int n, const void* T, int64_t ldT, const void* rho, int64_t ldR,
                                   double* F, void* ws, hipStream_t s, int* sweeps, int max_sweeps, int* sweeps_dev);
hipError_t launch_abs_map_backward(qst_prec prec, int n, double P, const void* Q, const double* lam, const void* GA,
                                   int64_t ldGA, void* GT, int64_t ldGT, void* ws, hipStream_t s);

// State-map pre-map (qst_premap mode) of a d x d complex matrix; Y may be X.
hipError_t launch_premap(qst_prec prec, int mode, const void* X, int64_t ldx, void* Y, int64_t ldy, int n,
                         hipStream_t s);

hipError_t launch_tau(qst_prec prec, const void* T, int64_t ld, int n, double* partials,
                      double* tau_dev, hipStream_t s, const void* f = nullptr, void* planes = nullptr);

// rho = T T^dagger / tau, written in full.  tau comes from tau_partials (the
// partial sums of launch_tau; the kernel also stores the total at tau_dev)
// or, when tau_partials is NULL, from *tau_dev.  sk_partial: stream-K
// partial-tile area of stream_k_partial_bytes(prec) bytes, or NULL (then one
// workgroup per tile).
// First product-POVM pass folded into T T^dagger (tetrahedral POVM, d >= 64):
// instead of rho, each finished tile's pass over the g lowest qubits
// (4 <= g <= 6) is written to X (the pass-0 output of the plan).
struct Pass0Out {
  void* X;
  int g;
  bool tetra;  // must be true
};
// planes: the bf16 planes of T written by launch_tau (BF16 path, d >
// kBf16SplitMaxDim), or NULL to round T inside the product.
hipError_t launch_herk(qst_prec prec, const void* T, int64_t ldt, void* rho, int64_t ldr, int n,
                       const double* tau_partials, double* tau_dev, void* sk_partial, hipStream_t s,
                       const Pass0Out* x0 = nullptr, const void* planes = nullptr);

// out = (upstream ? *upstream : 1) * 2 / *tau_dev * G T.  planes (BF16 path,
// used for d >= 1024; may be NULL): 16 d^2 bytes for the split-bf16 planes
// of G and of T^T, which the 128 x 128-tile product reads.
hipError_t launch_hemm(qst_prec prec, const void* G, int64_t ldg, const void* T, int64_t ldt,
                       void* out, int64_t ldo, int n, const double* tau_dev,
                       const double* upstream_dev, void* sk_partial, hipStream_t s, void* planes = nullptr);

// QST_F32X6 products (k_xgemm.hip), d >= kX6Tile.  T T^dagger: planes
// x6_herk_plane_bytes(n) and partials x6_partial_bytes(n) of workspace; the
// kernel that splits T also writes the kReduceBlocks partial sums of tau at
// tau_partials and, with f (4^N FP32 values), those of F = sum f at
// tau_partials + kReduceBlocks (launch_tau is not called); tau is stored at
// tau_dev; rho and x0 as launch_herk.  With tt_planes (x6_hemm_plane_bytes(n)
// / 2 bytes) the same kernel also writes T^T's planes for G' T there.
// G' T: planes x6_hemm_plane_bytes(n), G''s planes in the first half and
// T^T's in the second; g_ready / t_ready: that half holds its planes
// already (G / T are then not read); as launch_hemm otherwise.
hipError_t launch_x6_herk(const void* T, int64_t ldt, void* rho, int64_t ldr, int n, double* tau_partials,
                          const void* f, double* tau_dev, void* planes, void* partials, hipStream_t s,
                          const Pass0Out* x0, void* tt_planes = nullptr);
hipError_t launch_x6_hemm(const void* G, int64_t ldg, const void* T, int64_t ldt, void* out, int64_t ldo, int n,
                          const double* tau_dev, const double* upstream_dev, void* planes, hipStream_t s,
                          bool g_ready = false, bool t_ready = false);

// Forward (adjoint=false): mat = rho (lower triangle read) -> pvec.
// Adjoint (adjoint=true): g' = F - f/p from (pvec, fvec, F_dev) -> mat = G'
// (written in full).  mode_matrix: W (forward) or V (adjoint) as 4 x 4
// complex; tetra selects the tetrahedral fast form (mode_matrix unused).
hipError_t launch_povm(bool adjoint, qst_prec prec, const PovmPlan& pl, const double* mode_matrix,
                       bool tetra, const void* mat, int64_t ld, void* pvec, const void* fvec,
                       const double* F_dev, void* inter0, void* inter1, hipStream_t s,
                       bool use_fast = true);

// Stage 1 of the NLL over D entries of p and f: FP64 partials [4][kReduceBlocks]
// (L, F, bad0, bad1) as launch_nll's.
hipError_t launch_nll_partials(qst_prec prec, const void* p, const void* f, int64_t D, double* partials,
                               hipStream_t s);

// Workspace pieces of the general-POVM calls (general_layout).
struct GeneralBufs {
  double* partials;  // kReduceBlocks x 4
  double* scal;      // 4 per setting: L_s, F_s, bad0_s, bad1_s
  void *inter0, *inter1;  // product-POVM pass intermediates
  void *e, *h;            // 4^N reals: Pauli coordinates of rho; summed adjoint input
  void *bufA, *bufB;      // max(4, K)^N reals each: the real passes
  void* p;                // K^N reals: one setting's probabilities
};

// p (K^N reals) of a product POVM with real Pauli factors C[i][k][b]
// (general_factors, one setting) from rho.
hipError_t launch_general_probs(qst_prec prec, int n, int K, const double* C, const void* rho, int64_t ld_rho,
                                void* p, const GeneralBufs& b, hipStream_t s);
// Sum over the settings of the NLL (nll_dev = [L, F]) and, with G, the
// adjoint matrix G' = sum_s sum_k (F_s - f^s_k / p^s_k) M^s_k written in
// full; f: settings x K^N reals, setting-major.
hipError_t launch_general_likelihood(qst_prec prec, int n, int K, int settings, const double* C, const void* rho,
                                     int64_t ld_rho, const void* f, void* G, int64_t ldG, double* nll_dev,
                                     unsigned long long* bad_dev, const GeneralBufs& b, hipStream_t s);

// nll[0] = L, nll[1] = F, bad[0..1] counts (bad may be NULL).
hipError_t launch_nll(qst_prec prec, const void* p, const void* f, int n, double* partials,
                      double* nll_dev, unsigned long long* bad_dev, hipStream_t s);

// *F_dev = sum f.
// Stage 2 of qst_likelihood's NLL: L and counters from the fused pass's
// partials [4][nb]; F from the kReduceBlocks F partials of launch_tau.
// With fc_dev, also F_c = (sum of the F_c terms in slot 1)^2.
hipError_t launch_likelihood_finish(const double* part, int nb, const double* Fpart, double* nll_dev,
                                   unsigned long long* bad_dev, hipStream_t s, double* fc_dev = nullptr);

// The POVM part of qst_likelihood when fused_likelihood(pl, prec): forward
// passes 0..P-2 (from pass 1 when pass0_done: its output is already in
// inter0), the fused last pass (+ NLL finish into nll_dev / bad_dev), and, if
// G is not NULL, the adjoint passes P-2..0.  part: FP64 partials [4][blocks
// of the last pass]; Fpart: the kReduceBlocks F partials.  With pt (4^N
// reals), the last pass also forms F_c against pt into fc_dev.  With
// gplanes (FP32 storage, pass0_writes_planes(pl)), adjoint pass 0 writes G'
// as the split planes of the QST_F32X6 gradient product there instead of
// writing G (which may then be NULL).
hipError_t launch_povm_fused(qst_prec prec, const PovmPlan& pl, const double* W, const double* V, bool tetra,
                             const void* rho, int64_t ld_rho, const void* fvec, const double* Fpart, void* G,
                             int64_t ldG, void* inter0, void* inter1, double* part, double* nll_dev,
                             unsigned long long* bad_dev, bool pass0_done, hipStream_t s, const void* pt = nullptr,
                             double* fc_dev = nullptr, void* gplanes = nullptr);

hipError_t launch_fsum(qst_prec prec, const void* f, int n, double* partials, double* F_dev,
                       hipStream_t s);

}  // namespace qst
