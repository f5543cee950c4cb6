/*
 * qst.h -- C ABI of the MI355X (gfx950) likelihood path of neural-network
 * maximum-likelihood quantum state tomography:
 *
 *   T  ->  rho = T T^dagger / Tr(T T^dagger)          (state map)
 *      ->  p_k = Tr(rho M_k), M_k = M_{k_1} (x) ... (x) M_{k_N}   (POVM map)
 *      ->  L = -sum_k f_k ln p_k                        (negative log-likelihood)
 *   and back: dL/dT.
 *
 * Source: Wang, Cheng, Li, Chen, "Ultrafast quantum state tomography with
 * feed-forward neural networks": Sec. 2.1 (Born rule, Eq. MLE), Sec. 2.2.1
 * (Eq. T_matrix, Eq. MLE_T), Sec. 3.2 (Eq. unified_DP, Eq. abs_P at P = 2),
 * Sec. 3.3 (product-structured POVM, Eq. PS), Sec. 4.1 (tetrahedral POVM).
 *
 * Conventions shared by every call
 * --------------------------------
 * - N = n_qubits, d = 2^N, D = 4^N.  1 <= N <= QST_MAX_QUBITS.
 * - Complex values are interleaved (re, im): complex128 for QST_F64,
 *   complex64 for QST_F32 and QST_BF16GEMM.  Matrices are row-major with a
 *   leading dimension (row stride) counted in complex elements, ld >= d.
 * - Qubit 1 is the most significant bit of the row index r and of the column
 *   index c of a d x d matrix (the leftmost Kronecker factor).
 * - Outcome index k = sum_i k_i 4^(N-i), k_i in {0,1,2,3} the single-qubit
 *   outcome a of M_a.
 * - Real vectors (p, f) are float64 for QST_F64, float32 otherwise.
 * - Every pointer named *_dev or described as device memory must be device
 *   memory; povm_host is host memory.  The caller allocates and owns every
 *   buffer; the library never frees or keeps a pointer after a call returns.
 * - stream is a hipStream_t (NULL = the null stream).  Every call only
 *   enqueues work on that stream and returns without synchronising; scalar
 *   results are written to device memory, so call sequences can be captured
 *   into a HIP graph.
 * - Argument errors are detected on the host before anything is enqueued
 *   and returned as a status; a failed launch returns QST_ERR_HIP.  No call
 *   aborts or throws.  qst_last_error() gives a message for the last
 *   failure on the calling thread.
 * - ws / ws_bytes: caller-provided device workspace of at least
 *   qst_workspace_bytes(N, prec, op) bytes (may be NULL when that is 0).
 *   Its content on entry is ignored.
 * - Calls on different streams with distinct buffers may run concurrently.
 */
#ifndef QST_H
#define QST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QST_MAX_QUBITS 13
#define QST_FIDELITY_MAX_RANK 32

typedef enum {
  QST_OK = 0,
  QST_ERR_INVALID_ARG = 1, /* null pointer, N out of range, ld < d, bad POVM */
  QST_ERR_UNSUPPORTED = 2, /* valid request this build does not implement   */
  QST_ERR_WORKSPACE = 3,   /* ws_bytes smaller than qst_workspace_bytes()    */
  QST_ERR_HIP = 4          /* a HIP runtime call or kernel launch failed     */
} qst_status;

typedef enum {
  /* complex128 T and rho, float64 p and f; FP64 MFMA products. */
  QST_F64 = 0,
  /* complex64 T and rho, float32 p and f; FP32 MFMA products with FP32
   * accumulation; tau and the log-likelihood sum in FP64. */
  QST_F32 = 1,
  /* complex64 storage as QST_F32.  For d >= 256, T T^dagger takes T rounded
   * to bfloat16 (round-to-nearest-even) on the BF16 MFMA with FP32
   * accumulation; for d <= 128 T is split into bfloat16 hi + lo (three
   * products), because plain rounding there moves the gradient by more than
   * 2e-3 relative.  tau is the FP64 sum over the same represented T.  The
   * gradient product G' T always uses split bfloat16 operands (hi + lo,
   * three products). */
  QST_BF16GEMM = 2,
  /* complex64 storage, FP32 POVM passes, tau and the log-likelihood sum in
   * FP64, as QST_F32; for d >= 128 the two complex products run on the
   * BF16 MFMA with every FP32 operand split exactly into three bfloat16
   * parts (x = h + m + l) and six partial products per real product (hh,
   * hm, mh, hl, lh, mm: what is dropped is below 2^-26 of |a||b|), FP32
   * accumulation.  Results agree with QST_F32 to the order of FP32
   * rounding; the products run about twice as fast.  Below d = 128 the
   * products are those of QST_F32.  The batched form runs it as QST_F32. */
  QST_F32X6 = 3
} qst_prec;

typedef enum {
  QST_OP_STATE_MAP = 0,
  QST_OP_POVM_PROBS = 1,
  QST_OP_NLL = 2,
  QST_OP_NLL_BACKWARD = 3,
  QST_OP_LIKELIHOOD = 4,
  QST_OP_GRAD_PRODUCT = 5,
  QST_OP_FIDELITY = 6,
  QST_OP_FNN = 7,
  QST_OP_ABS_MAP = 8,
  QST_OP_LIKELIHOOD_GRAD = 9
} qst_op;

/*
 * State map (Eq. T_matrix, with rho = T T^dagger / Tr; for Hermitian T this
 * is the unified map of Eq. unified_DP, and Eq. abs_P at P = 2).
 *   T      [in]  d x d complex, row stride ldT, device.
 *   rho    [out] d x d complex, row stride ld_rho, device.  Written in full
 *                (both triangles; Hermitian to rounding).
 *   tau_dev[out] one double, device: tau = sum_ij |T_ij|^2 accumulated in
 *                FP64 (over the bfloat16-rounded T for QST_BF16GEMM).
 * rho must not overlap T.
 */
qst_status qst_state_map(int n_qubits, qst_prec prec, const void* T, int64_t ldT, void* rho,
                         int64_t ld_rho, double* tau_dev, void* ws, size_t ws_bytes,
                         void* stream);

/*
 * Product-POVM map (Born rule, Sec. 2.1; product structure, Sec. 3.3):
 *   p_k = Tr(rho M_k) for all k in [0, 4^N).
 *   rho      [in]  d x d Hermitian complex, row stride ld_rho, device.  Only
 *                  the lower triangle (row >= column) is read; the upper
 *                  triangle is taken to be its conjugate transpose.
 *   povm_host[in]  NULL for the paper's tetrahedral POVM (Sec. 4.1), else
 *                  host array of 4 Hermitian 2 x 2 complex matrices M_0..M_3,
 *                  32 doubles: M_a[x][y] at (re, im) = [8a + 4x + 2y + {0,1}].
 *                  Each M_a must be Hermitian and sum_a M_a = I, both to
 *                  1e-12 (else QST_ERR_INVALID_ARG).
 *   p        [out] 4^N reals, device.
 */
qst_status qst_povm_probs(int n_qubits, qst_prec prec, const void* rho, int64_t ld_rho,
                          const double* povm_host, void* p, void* ws, size_t ws_bytes,
                          void* stream);

/*
 * Negative log-likelihood (Eq. MLE; loss of Sec. 3.1):
 *   L = -sum_{k: f_k != 0} f_k ln p_k, accumulated in FP64.
 *   p, f     [in]  4^N reals each, device.  f is used as given (counts or
 *                  frequencies; F = sum f is not assumed to be 1).
 *   nll_dev  [out] two doubles, device: nll_dev[0] = L, nll_dev[1] = F.
 *   bad_dev  [out] two uint64, device, or NULL: bad_dev[0] = number of k
 *                  with f_k > 0 and not p_k > 0 (such a term makes L = +inf),
 *                  bad_dev[1] = number of NaN entries in p or f.
 * The reduction order is fixed, so results are bitwise reproducible.
 */
qst_status qst_nll(int n_qubits, qst_prec prec, const void* p, const void* f, double* nll_dev,
                   unsigned long long* bad_dev, void* ws, size_t ws_bytes, void* stream);

/*
 * Adjoint of the whole chain (derived from Eq. MLE_T with rho = T T^dagger/tau):
 *   g'_k = F - f_k / p_k (g'_k = F where f_k = 0),  G' = sum_k g'_k M_k,
 *   gradT = s * (2 / tau) * G' T
 * which is dL/dRe T + i dL/dIm T (the PyTorch convention for complex
 * parameters), times s = *upstream_dev (1 if upstream_dev is NULL).
 *   T        [in]  d x d complex, row stride ldT, device (the same T as the
 *                  forward call).
 *   f        [in]  4^N reals, device.
 *   p        [in]  4^N reals from the forward call, device; or NULL, in
 *                  which case rho and p are recomputed from T inside this
 *                  call (nothing of length 4^N needs to survive the forward).
 *   tau_dev  [in]  the tau written by qst_state_map for this T, device; may
 *                  be NULL only when p is NULL (then tau is recomputed).
 *   nll_dev  [in]  the two doubles written by qst_nll for this f (F is taken
 *                  from nll_dev[1]), device; or NULL, in which case F = sum f
 *                  is reduced here.
 *   povm_host[in]  as in qst_povm_probs.
 *   upstream_dev[in] one double, device, or NULL.
 *   gradT    [out] d x d complex, row stride ldG, device; must not overlap T.
 */
qst_status qst_nll_backward(int n_qubits, qst_prec prec, const void* T, int64_t ldT,
                            const void* f, const void* p, const double* tau_dev,
                            const double* nll_dev, const double* povm_host,
                            const double* upstream_dev, void* gradT, int64_t ldG, void* ws,
                            size_t ws_bytes, void* stream);

/*
 * Likelihood and the adjoint matrix in one call (the chain of Eq. MLE_T with
 * rho = T T^dagger / tau):
 *   tau and rho = T T^dagger / tau          (as qst_state_map),
 *   p_k = Tr(rho M_k) for all k             (as qst_povm_probs),
 *   L = -sum_{f_k != 0} f_k ln p_k, F = sum f, counters (as qst_nll),
 *   and, when G is not NULL, G' = sum_k (F - f_k/p_k) M_k (the matrix that
 *   qst_nll_backward multiplies by T).
 * rho and p stay in the workspace.  For N >= 7 the last stage of the POVM
 * map, the NLL terms, the cotangent and the first stage of the adjoint map
 * run as one kernel per block of outcomes, so p is never written to memory
 * (F is summed beforehand, alongside tau).
 *   T        [in]  d x d complex, row stride ldT, device.
 *   f        [in]  4^N reals, device.
 *   povm_host[in]  as in qst_povm_probs.
 *   tau_dev  [out] one double, device (input of qst_grad_product).
 *   nll_dev  [out] two doubles, device: L and F (as qst_nll).
 *   bad_dev  [out] two uint64, device, or NULL (as qst_nll).
 *   G        [out] d x d complex, row stride ldG, device, written in full;
 *                  or NULL for the value alone.  Must not overlap T.
 * Summation orders are fixed: results are bitwise reproducible.
 */
qst_status qst_likelihood(int n_qubits, qst_prec prec, const void* T, int64_t ldT, const void* f,
                          const double* povm_host, double* tau_dev, double* nll_dev,
                          unsigned long long* bad_dev, void* G, int64_t ldG, void* ws,
                          size_t ws_bytes, void* stream);

/*
 * General product POVMs (Sec. 3.3 with a POVM of its own on each qubit;
 * Sec. 2.1, one POVM per measurement setting): qubit i of setting s is
 * measured with a K-element POVM {M^(s,i)_k}, k = 0..K-1, so a setting has
 * K^N outcomes k = sum_i k_i K^(N-i) (qubit 1 most significant) with
 * p^s_k = Tr(rho M^(s,1)_k1 (x) ... (x) M^(s,N)_kN).  2 <= K <= 8,
 * K^N <= 2^30, 1 <= settings <= 64.
 *   povm_host [in] host, settings x N x K x 2 x 2 complex (re, im),
 *                  row-major: element k of qubit i (0-based) of setting s
 *                  starts at double offset ((s N + i) K + k) 8 as
 *                  M[0][0], M[0][1], M[1][0], M[1][1].  Every element must
 *                  be Hermitian and positive semidefinite and each qubit's
 *                  K elements must sum to I (to 1e-12), else
 *                  QST_ERR_INVALID_ARG.
 * Computed through the Pauli coordinates e_b = Tr(P_b1 (x) ... (x) P_bN rho)
 * of rho (4^N reals, P = I, X, Y, Z) and the real per-qubit factors
 * Tr(M_k P_b) / 2; FP64 arithmetic for QST_F64, FP32 otherwise.
 * Workspace: qst_workspace_bytes_general(N, prec, K, op) with op =
 * QST_OP_POVM_PROBS or QST_OP_LIKELIHOOD (0 for invalid arguments).
 */
size_t qst_workspace_bytes_general(int n_qubits, qst_prec prec, int K, int op);

/*
 * p = K^N probabilities of one general product POVM (settings = 1 layout of
 * povm_host) from rho (d x d complex, row stride ld_rho, device; only the
 * lower triangle is read).  p: K^N reals (storage precision), device.
 */
qst_status qst_povm_probs_general(int n_qubits, qst_prec prec, const void* rho, int64_t ld_rho, int K,
                                  const double* povm_host, void* p, void* ws, size_t ws_bytes, void* stream);

/*
 * The likelihood over several settings (Eq. MLE summed over the
 * measurements of Sec. 2.1):
 *   L = -sum_s sum_k f^s_k ln p^s_k,  rho = T T^dagger / tau,
 * and the adjoint matrix for qst_grad_product,
 *   G' = sum_s sum_k (F_s - f^s_k / p^s_k) M^s_k,  F_s = sum_k f^s_k
 * (each setting's POVM sums to I, which carries the trace normalisation).
 *   f        [in]  settings x K^N reals (storage precision), setting-major, device.
 *   tau_dev  [out] one double, device.
 *   nll_dev  [out] two doubles, device: L (+inf after f_k > 0 with p_k <= 0,
 *                  NaN after a NaN) and F = sum of every f.
 *   bad_dev  [out] two uint64 (as qst_nll, over all settings), or NULL.
 *   G        [out] d x d complex (row stride ldG), written in full, or NULL
 *                  for the value alone.  Must not overlap T.
 * dL/dT then follows from qst_grad_product(G, T, tau).  Summation orders
 * are fixed (settings in order): results are bitwise reproducible.
 */
qst_status qst_likelihood_general(int n_qubits, qst_prec prec, const void* T, int64_t ldT, int settings, int K,
                                  const double* povm_host, const void* f, double* tau_dev, double* nll_dev,
                                  unsigned long long* bad_dev, void* G, int64_t ldG, void* ws, size_t ws_bytes,
                                  void* stream);

/*
 * Bytes of the library's static device scratch: the workspace of
 * qst_likelihood_noalloc, one array per GPU, held until the process ends.
 */
#define QST_STATIC_SCRATCH_BYTES ((size_t)16 << 20)

/*
 * qst_likelihood for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and results, bitwise, with the workspace taken from
 * a static device array of QST_STATIC_SCRATCH_BYTES (16 MiB) instead of a
 * workspace argument.  The call allocates nothing: no hipMalloc, no hipFree,
 * no allocating library routine (with the library's profiler off, its
 * default).  On its first call on a device it looks up that device's copy
 * of the array (hipGetSymbolAddress) with that device current; the stream
 * and every buffer must belong to the current device.
 *   Limit: the workspace qst_likelihood would need, qst_workspace_bytes(N,
 *   prec, QST_OP_LIKELIHOOD), must fit the array: N <= 9 in every
 *   precision.  Larger N returns QST_ERR_WORKSPACE before anything is
 *   launched.
 *   Sharing: every call on one GPU uses that GPU's one array, and a call
 *   leaves its contents behind (nothing in it needs to start at zero).
 *   Calls that overlap on one GPU -- concurrent streams, or host threads
 *   without ordering between their streams -- race on the array and give
 *   undefined results; order them on one stream.
 * Arguments and errors otherwise as qst_likelihood.
 */
qst_status qst_likelihood_noalloc(int n_qubits, qst_prec prec, const void* T, int64_t ldT, const void* f,
                                  const double* povm_host, double* tau_dev, double* nll_dev,
                                  unsigned long long* bad_dev, void* G, int64_t ldG, void* stream);

/*
 * qst_likelihood plus the classical fidelity (Sec. 2.3 Eq. F_CF) of the
 * model's distribution p_k = Tr(M_k rho) against a target distribution:
 *   F_c = (sum_k sqrt(max(p_k, 0) max(p_target_k, 0)))^2.
 * Where qst_likelihood fuses its last POVM pass (N >= 7 with the fused
 * plan), the terms are formed in that pass from the p_k it holds in
 * registers (one more read of 4^N reals, p still never stored); otherwise
 * from the stored p.  tau, F and the counters are those of qst_likelihood
 * bitwise; L and G agree with it to rounding (the fused pass with F_c is a
 * kernel instance of its own, and its FP64 sums may contract into FMAs
 * differently).
 *   p_target [in]  4^N reals (storage precision of f), device; read as
 *                  given (not renormalised).
 *   fc_dev   [out] one double, device.
 * Other arguments, workspace (QST_OP_LIKELIHOOD) and errors as
 * qst_likelihood.
 */
qst_status qst_likelihood_fc(int n_qubits, qst_prec prec, const void* T, int64_t ldT, const void* f,
                             const void* p_target, const double* povm_host, double* tau_dev, double* nll_dev,
                             double* fc_dev, unsigned long long* bad_dev, void* G, int64_t ldG, void* ws,
                             size_t ws_bytes, void* stream);

/*
 * Likelihood and gradient in one call (Eq. MLE_T): tau, L, F and the
 * counters as qst_likelihood, and
 *   gradT = dL/dRe T + i dL/dIm T = (2 / tau) G' T,
 * what qst_likelihood followed by qst_grad_product (upstream 1) gives;
 * G' itself is not returned.  With QST_F32X6 from d = 128 the kernel that
 * splits T for T T^dagger also writes T^T's planes for the gradient
 * product, and where the first POVM stage covers 5 or 6 qubits
 * (tetrahedral POVM, N = 9, 10, 11, 13) the adjoint's last stage writes G'
 * directly as that product's planes.  tau, L, F and the counters equal
 * qst_likelihood's bitwise; gradT equals the two calls' bitwise, except on
 * that last route, where it agrees to rounding (the adjoint stage that
 * writes planes is a kernel instance of its own, whose sums may contract
 * into FMAs differently).
 *   gradT    [out] d x d complex, row stride ld_grad, device; must not
 *                  overlap T.
 * Workspace: qst_workspace_bytes(N, prec, QST_OP_LIKELIHOOD_GRAD).  Other
 * arguments and errors as qst_likelihood.
 */
qst_status qst_likelihood_grad(int n_qubits, qst_prec prec, const void* T, int64_t ldT, const void* f,
                               const double* povm_host, double* tau_dev, double* nll_dev,
                               unsigned long long* bad_dev, void* gradT, int64_t ld_grad, void* ws,
                               size_t ws_bytes, void* stream);

/*
 * Gradient product, the last step of the adjoint (Eq. MLE_T):
 *   gradT = s * (2 / tau) * G' T,  s = *upstream_dev (1 if upstream_dev is NULL),
 * for G' and tau from qst_likelihood (same T).
 *   G        [in]  d x d complex, row stride ldG, device.
 *   T        [in]  d x d complex, row stride ldT, device.
 *   tau_dev  [in]  one double, device.
 *   upstream_dev[in] one double, device, or NULL.
 *   gradT    [out] d x d complex, row stride ld_grad, device; must overlap
 *                  neither G nor T.
 */
qst_status qst_grad_product(int n_qubits, qst_prec prec, const void* G, int64_t ldG, const void* T,
                            int64_t ldT, const double* tau_dev, const double* upstream_dev,
                            void* gradT, int64_t ld_grad, void* ws, size_t ws_bytes, void* stream);

typedef enum {
  /* Y = (X + X^dagger) / 2: the Hermitian part.  Applied to T before the
   * state map it gives Chol_H, the paper's default map (Sec. 3.2
   * Eq. unified_DP, equal to Eq. abs_P at P = 2); the Hermitian part of a
   * non-Hermitian matrix is the remark of Sec. 2.2.2. */
  QST_PREMAP_HERMITIAN = 1,
  /* Y = X on and below the diagonal (row >= column), 0 above: Chol_Delta,
   * the Cholesky-form decomposition with a lower-triangular T (Sec. 2.2.1
   * Eq. T_matrix). */
  QST_PREMAP_LOWER = 2
} qst_premap;

/*
 * Pre-map of a state-map mode, Y = P(X), with P one of qst_premap.  Both
 * maps are orthogonal projections for the real inner product Re Tr(A^dagger
 * B), hence self-adjoint: the same call maps dL/dT' (the gradient of the
 * other calls, taken at T' = P(T)) to dL/dT.
 *   mode     [in]  QST_PREMAP_HERMITIAN or QST_PREMAP_LOWER.
 *   X        [in]  d x d complex, row stride ldX, device.
 *   Y        [out] d x d complex, row stride ldY, device.  Y == X (with
 *                  ldY == ldX) works in place; otherwise Y must not overlap X.
 * Elementwise: the result is bitwise the definition's ((x + conj y) * 0.5 in
 * the storage precision; a copy or a zero).  No workspace.
 */
qst_status qst_state_premap(int n_qubits, qst_prec prec, int mode, const void* X, int64_t ldX, void* Y,
                            int64_t ldY, void* stream);

/*
 * P-order absolute map (Sec. 3.2 Eq. abs_P and the map A(T)_P before it).
 * With H = (T + T^dagger) / 2 = Q Lambda Q^dagger,
 *   A = Q |Lambda|^(P/2) Q^dagger,
 * Hermitian positive semidefinite, so that the state map of A (qst_state_map,
 * qst_likelihood) gives rho = Q |Lambda|^P Q^dagger / Tr |Lambda|^P, the
 * P-order absolute projection; P = 2 is Chol_H (Eq. unified_DP).
 * The eigendecomposition runs in FP64 on the device, whatever prec.  Without
 * Q0 it is a direct solver: Householder reduction to a real tridiagonal
 * matrix, eigenvalues by multisection of Sturm counts, eigenvectors by
 * twisted factorizations (inverse iteration with orthogonalisation within
 * clusters of eigenvalues closer than 1e-7 ||H||), one Newton-Schulz
 * orthogonalisation step, and the blocked back-transformation; a fixed
 * sequence of launches, after which this call reads one status word (one
 * synchronisation).  With Q0 it is a cyclic two-sided Jacobi method on
 * Q0^dagger H Q0: after each sweep a kernel decides on the device whether
 * to stop (off-diagonal norm at 1e-14 of ||H||_F for QST_F64, 1e-10 for the
 * FP32-storage precisions, or at the rounding floor), and this call reads
 * that decision after each sweep to stop enqueuing.  qst_abs_map_async is
 * the same map without any synchronisation.
 *   P      [in]  finite, >= 0.
 *   T      [in]  d x d complex (prec's storage type), row stride ldT, device.
 *   Q0     [in]  NULL (the direct solver), or a warm start for the Jacobi
 *                solver: a unitary d x d complex FP64 matrix laid out as Q
 *                (normally the Q of an earlier call on a nearby T); the
 *                sweeps then run on Q0^dagger H Q0.  The result does not
 *                depend on Q0 beyond rounding as long as Q0 is unitary.  The
 *                direct solver is faster than a warm start from d = 64 on.
 *                Q0 may be Q; it must not overlap T, A or lam.
 *   A      [out] d x d complex (prec's storage type), row stride ldA, device.
 *                A == T with ldA == ldT works in place.
 *   Q      [out] d x d complex FP64 (interleaved re, im), row-major, row
 *                stride d, device: the eigenvectors of H as columns.
 *   lam    [out] d doubles, device: the eigenvalues of H, lam[i] belonging to
 *                column i of Q (no particular order).
 *   sweeps [out] host int, may be NULL: the Jacobi sweeps taken (0 for the
 *                direct solver).
 * Q and lam are what qst_abs_map_backward needs.  Q must not overlap T, A or
 * lam.  Workspace: qst_workspace_bytes(N, prec, QST_OP_ABS_MAP) (three
 * d x d FP64 complex buffers and the solver's smaller arrays).  Returns
 * QST_ERR_INVALID_ARG when H is not finite or the sweeps do not converge.
 */
qst_status qst_abs_map(int n_qubits, qst_prec prec, double P, const void* T, int64_t ldT, const void* Q0, void* A,
                       int64_t ldA, void* Q, double* lam, int* sweeps, void* ws, size_t ws_bytes, void* stream);

/*
 * qst_abs_map for streams that must not be synchronised (HIP graph capture,
 * pipelined training loops).  Nothing is read back and the call returns
 * before the work runs.  Without Q0 the direct solver runs as in
 * qst_abs_map (max_sweeps is checked but not used).  With Q0 at most
 * max_sweeps Jacobi sweeps are enqueued (1 <= max_sweeps <= 40) and the
 * stopping rule is applied on the device after each; rounds after
 * convergence return at once (an empty launch each), and A, Q and lam are
 * then computed as by qst_abs_map.
 *   sweeps_dev [out] one int, device: the sweeps taken (0 for the direct
 *                    solver), or -1 when H was not finite or the warm
 *                    sweeps had not met the stopping rule after max_sweeps
 *                    (A, Q and lam must not be used then).
 * A warm start (Q0 from the previous step) usually needs 2 or 3 sweeps at
 * the training-loop pace (T moved by about 1e-3 of its scale).  Other
 * arguments, workspace and argument errors as qst_abs_map.
 */
qst_status qst_abs_map_async(int n_qubits, qst_prec prec, double P, const void* T, int64_t ldT, const void* Q0,
                             void* A, int64_t ldA, void* Q, double* lam, int max_sweeps, int* sweeps_dev, void* ws,
                             size_t ws_bytes, void* stream);

/*
 * Adjoint of qst_abs_map: dL/dT from dL/dA (both the gradient convention of
 * qst_grad_product, dL/dRe X + i dL/dIm X).  With S = (dL/dA + dL/dA^dagger)/2
 * and Gamma_ij the divided differences (g(l_i) - g(l_j)) / (l_i - l_j) of
 * g(l) = |l|^(P/2) (g'(l_i) where l_i = l_j, 0 at l = 0),
 *   dL/dT = Q (Gamma o (Q^dagger S Q)) Q^dagger,
 * the first-order change of a spectral function, composed with the
 * Hermitian part (both self-adjoint).  Four complex products in FP64.
 *   P, Q, lam  [in] as given to / returned by qst_abs_map.
 *   GA     [in]  d x d complex (prec's storage type), row stride ldGA.
 *   GT     [out] d x d complex (prec's storage type), row stride ldGT.  GT may
 *                be GA (with ldGT == ldGA); it must not overlap Q or lam.
 * Workspace: qst_workspace_bytes(N, prec, QST_OP_ABS_MAP).  No
 * synchronisation.
 */
qst_status qst_abs_map_backward(int n_qubits, qst_prec prec, double P, const void* Q, const double* lam,
                                const void* GA, int64_t ldGA, void* GT, int64_t ldGT, void* ws, size_t ws_bytes,
                                void* stream);

/*
 * Quantum fidelity against a general target (Sec. 2.3 Eq. F_QF, computed
 * with one eigendecomposition as Eq. fq_decom does):
 *   F_q = (Tr sqrt(sqrt(rho_hat) rho sqrt(rho_hat)))^2,
 *   rho_hat = T T^dagger / Tr(T T^dagger).
 * sqrt(rho_hat) rho sqrt(rho_hat) and T^dagger rho T / Tr(T T^dagger) have
 * the same nonzero eigenvalues (rho_hat's factor T stands in for the first
 * decomposition of Eq. fq_decom), so F_q = (sum_i sqrt(lambda_i))^2 / tau
 * with lambda_i the eigenvalues of T^dagger rho T (two FP64 complex
 * products, then the Householder reduction and the multisection of the
 * direct solver of qst_abs_map, eigenvalues only; rounding-level negative
 * eigenvalues read as 0).  For a target of low rank prefer
 * qst_fidelity_lowrank: here each of the d - r zero eigenvalues can add
 * the square root of its rounding error.
 *   T      [in]  d x d complex, row stride ldT, device.
 *   rho    [in]  d x d complex Hermitian positive semidefinite with trace 1
 *                (not checked), row stride ldR, device.
 *   F_dev  [out] one double, device.
 *   sweeps [out] host int, may be NULL: 0 (no Jacobi sweeps).
 * Workspace: qst_workspace_bytes(N, prec, QST_OP_ABS_MAP).  Reads one status
 * word at the end (one synchronisation; qst_fidelity_general_async has
 * none).  QST_ERR_INVALID_ARG when the input is not finite.
 */
qst_status qst_fidelity_general(int n_qubits, qst_prec prec, const void* T, int64_t ldT, const void* rho,
                                int64_t ldR, double* F_dev, int* sweeps, void* ws, size_t ws_bytes, void* stream);

/*
 * qst_fidelity_general without synchronisation; max_sweeps (1..40) is
 * checked but not used (no Jacobi sweeps run); sweeps_dev [out] one device
 * int, 0, or -1 when the input was not finite (F_dev must not be used
 * then).  Other arguments as qst_fidelity_general.
 */
qst_status qst_fidelity_general_async(int n_qubits, qst_prec prec, const void* T, int64_t ldT, const void* rho,
                                      int64_t ldR, double* F_dev, int max_sweeps, int* sweeps_dev, void* ws,
                                      size_t ws_bytes, void* stream);

/*
 * Quantum fidelity against a target of low rank r (Sec. 2.3 Eq. F_QF):
 *   F_q = (Tr sqrt(sqrt(rho_hat) rho sqrt(rho_hat)))^2,
 *   rho_hat = T T^dagger / Tr(T T^dagger)   (the state map of T),
 *   rho     = W W^dagger / Tr(W W^dagger)   (the target, W d x r).
 * sqrt(rho_hat) rho sqrt(rho_hat) and the r x r matrix
 * C = (W^dagger T)(W^dagger T)^dagger / (Tr(T T^dagger) Tr(W W^dagger))
 * have the same nonzero eigenvalues, so F_q = (sum_i sqrt(lambda_i(C)))^2
 * from an r x r Hermitian eigensolve (cyclic Jacobi in FP64; negative
 * rounding-level eigenvalues read as 0).  A pure target psi is r = 1:
 * F_q = |psi^dagger T|^2 / (Tr(T T^dagger) |psi|^2).  Sums in FP64, fixed
 * order (bitwise reproducible).
 *   T      [in]  d x d complex, row stride ldT, device (pass the pre-mapped
 *                T' of a state-map mode).
 *   W      [in]  d x r complex, row stride ldW >= r (row i holds W_i0 ..
 *                W_i,r-1), device.  1 <= r <= QST_FIDELITY_MAX_RANK.
 *   F_dev  [out] one double, device.
 */
qst_status qst_fidelity_lowrank(int n_qubits, qst_prec prec, const void* T, int64_t ldT, const void* W,
                                int64_t ldW, int r, double* F_dev, void* ws, size_t ws_bytes, void* stream);

/*
 * Classical fidelity (Sec. 2.3 Eq. F_CF): F_c = (sum_k sqrt(p_hat_k p_k))^2
 * with negative entries read as 0, summed in FP64 in a fixed order.
 *   p_hat, p [in]  4^N reals each, device.
 *   F_dev    [out] one double, device.
 */
qst_status qst_fidelity_classical(int n_qubits, qst_prec prec, const void* p_hat, const void* p, double* F_dev,
                                  void* ws, size_t ws_bytes, void* stream);

/*
 * The mapping network (Sec. 3.1): a 3-layer feed-forward network from the
 * measured distribution x (4^N inputs) through H = 2N hidden units with a
 * leaky ReLU (negative slope 0.01) to 4^N real outputs y that fill the
 * Hermitian T of Chol_H:
 *   h_pre = W1 x + b1,  y = W2 leaky(h_pre) + b2,  Y = y as a d x d real
 *   matrix (row major),  T_ij = Y_ij + i Y_ji (i > j),  T_ij = Y_ji - i Y_ij
 *   (i < j),  T_ii = Y_ii  (a bijection of R^(d^2) onto Hermitian matrices).
 * Real arrays are float64 for QST_F64, float32 otherwise.
 *   W1 [in]  H x 4^N, row major;  b1 [in] H;  W2 [in] 4^N x H, row major;
 *   b2 [in]  4^N;  x [in] 4^N; all device.
 *   h_pre [out] H reals, device (input of qst_fnn_backward).
 *   T     [out] d x d complex, row stride ldT, device.
 * Sums in FP64 in a fixed order (bitwise reproducible).
 */
qst_status qst_fnn_forward(int n_qubits, qst_prec prec, const void* W1, const void* b1, const void* W2,
                           const void* b2, const void* x, void* h_pre, void* T, int64_t ldT, void* ws,
                           size_t ws_bytes, void* stream);

/*
 * Backward of qst_fnn_forward: from G = dL/dT (the gradient convention of
 * qst_nll_backward, dL/dRe T + i dL/dIm T; only its action on Hermitian
 * directions matters), the gradients of L with respect to the parameters:
 *   dL/dy = fill^*(G):  Re G_ij + Re G_ji (i > j),  Im G_ji - Im G_ij
 *           (i < j),  Re G_ii;
 *   dW2 = dL/dy leaky(h_pre)^T,  db2 = dL/dy,
 *   db1 = (W2^T dL/dy) * leaky'(h_pre),  dW1 = db1 x^T.
 *   W2, x, h_pre [in] as in the forward call;  G [in] d x d complex, row
 *   stride ldG;  dW1 [out] H x 4^N;  db1 [out] H;  dW2 [out] 4^N x H;
 *   db2 [out] 4^N; all device.
 */
qst_status qst_fnn_backward(int n_qubits, qst_prec prec, const void* W2, const void* x, const void* h_pre,
                            const void* G, int64_t ldG, void* dW1, void* db1, void* dW2, void* db2, void* ws,
                            size_t ws_bytes, void* stream);

/*
 * One Rprop step (the optimiser of the paper's setup, Sec. 4.1; the
 * iRprop- rule): for each of count entries,
 *   s = sign(grad) sign(prev),
 *   step <- clamp(step * (s > 0 ? eta_plus : s < 0 ? eta_minus : 1),
 *                 step_min, step_max),
 *   g' = (s < 0 ? 0 : grad),  param <- param - sign(g') step,  prev <- g'.
 * param, prev, step [in/out] and grad [in]: count reals each (float64 for
 * QST_F64, float32 otherwise), device; the caller starts with prev = 0 and
 * step = the learning rate.  Requires 0 < eta_minus < 1 < eta_plus and
 * 0 < step_min <= step_max.  count = 0 does nothing.
 */
qst_status qst_rprop_step(int64_t count, qst_prec prec, void* param, const void* grad, void* prev, void* step,
                          double eta_minus, double eta_plus, double step_min, double step_max, void* stream);

/* Workspace in bytes needed by op (a qst_op) at (n_qubits, prec); 0 for an
 * invalid request. */
size_t qst_workspace_bytes(int n_qubits, qst_prec prec, int op);

/* Static string for a status code. */
const char* qst_status_string(qst_status s);

/* Message describing the last non-OK status returned on this thread ("" if
 * none).  Valid until the next call on the same thread. */
const char* qst_last_error(void);

/* Library version string. */
const char* qst_version(void);

/*
 * Kernel timing for measurement tools.  While enabled (on != 0), each timed
 * kernel scope (one launch, or a short fixed sequence such as a product and
 * its stream-K fix-up, under one name: "hemm_f32", "povm_fwd_p0", ...) is
 * bracketed by two timing-only hipEvents recorded on its launch stream.
 * only == NULL or "" times every scope; otherwise only the scope of that
 * name.  Each event costs several microseconds of queue time between
 * kernels, so a throughput measurement should time only the scope it
 * reports.  Disabled by default; do not enable it while a stream is being
 * captured into a HIP graph.
 */
qst_status qst_profile_enable(int on, const char* only);

/*
 * Waits for the recorded events and writes one line "name calls total_ms"
 * per timed scope name seen since the last reset into buf (NUL-terminated,
 * truncated to len).  Returns the size needed including the NUL.  reset != 0
 * clears the totals afterwards.
 */
size_t qst_profile_report(char* buf, size_t len, int reset);

/*
 * Batched form: many independent instances of mixed qubit counts, forward
 * and adjoint of every instance in one persistent launch (optionally replayed
 * as a captured HIP graph).  Instance i has N_i qubits (1 <= N_i <= 8),
 * d_i = 2^N_i.  Buffers are packed in instance order:
 *   T_all    complex, instance i's d_i x d_i row-major T (ld = d_i) at
 *            complex offset t_off[i];  grad_all: same layout, written;
 *   f_all    real, instance i's 4^N_i frequencies at real offset f_off[i];
 *   nll_out  double [count][2]: (L_i, F_i), written;
 *   bad_out  uint64 [count][2]: the counters of qst_nll, or NULL.
 * t_off and f_off (count + 1 entries each) come from qst_batch_offsets.
 * The plan owns device memory (descriptor table, work counter, per-workgroup
 * scratch) and, in graph mode, a HIP graph, until qst_batch_plan_destroy.
 * On its first run the plan times its candidate launch shapes (workgroup
 * size, the POVM pass plan of N = 7 and 8, grid size, instance order) on the
 * given buffers and keeps the fastest; with a cache
 * file (tune_cache, else the QST_TUNE_CACHE environment variable; NULL/unset
 * = no cache) the choice is appended there and reused by later plans with
 * the same precision, POVM kind, qubit-count histogram and device.
 * A plan must not be run concurrently on two streams.
 */
typedef struct qst_batch_plan qst_batch_plan;

qst_status qst_batch_plan_create(const int* n_qubits_host, int count, qst_prec prec,
                                 const double* povm_host, const char* tune_cache,
                                 qst_batch_plan** plan);

qst_status qst_batch_offsets(const qst_batch_plan* plan, int64_t* t_off_host, int64_t* f_off_host);

/* use_graph != 0 captures (once per buffer set and stream) and replays a HIP
 * graph; stream must then be non-NULL. */
qst_status qst_batch_run(qst_batch_plan* plan, const void* T_all, const void* f_all,
                         double* nll_out, unsigned long long* bad_out, void* grad_all,
                         int use_graph, void* stream);

/* The tuned launch shape: grid (workgroups), sorted_order (1 = largest
 * instances first), tuned_ms (time of one batch when tuned). */
qst_status qst_batch_info(const qst_batch_plan* plan, int* grid, int* sorted_order,
                          double* tuned_ms);

/* The rest of the tuned shape: threads (workgroup size: 512 or 256 for
 * QST_F32, 256 otherwise) and register_round_passes (1: N = 7, 8 run the
 * register-round pair of POVM passes with the likelihood fused into the
 * second, for the tetrahedral POVM in FP64 and FP32; 0: the generic
 * per-qubit passes).  Either pointer may be NULL. */
qst_status qst_batch_shape(const qst_batch_plan* plan, int* threads, int* register_round_passes);

void qst_batch_plan_destroy(qst_batch_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* QST_H */
