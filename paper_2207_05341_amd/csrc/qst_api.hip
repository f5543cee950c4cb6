// extern "C" entry points of libqst: validation, workspace carving and
// kernel dispatch for the likelihood path.  See include/qst.h for the
// contract of each call.
#include <mutex>
#include <string>
#include <vector>

#include "qst_kernels.h"
#include "qst_plan.h"

namespace {

using namespace qst;

inline unsigned char* ws_at(void* ws, size_t off) { return static_cast<unsigned char*>(ws) + off; }

qst_status fail(qst_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

qst_status hip_fail(hipError_t e, const char* what) {
  return fail(QST_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// tau and rho = T T^dagger / tau.  For d >= 64 the product kernel folds the
// tau partial sums itself (and stores tau); below that a finishing kernel
// produces tau first.
// With f, the tau kernel also leaves the partial sums of F = sum f at
// partials + kReduceBlocks.
// With x0, the first POVM pass is applied to rho's tiles in the product
// kernel and rho itself is not written.
// planes: workspace for the bf16 planes of T (BF16 path, d >
// kBf16SplitMaxDim; QST_F32X6 from d = kX6Tile, where the kernel that
// splits T forms the partial sums), or NULL.
// ttplanes (QST_F32X6 only, or NULL): T^T's planes for the gradient product,
// written by the same kernel that splits T.
hipError_t run_state_map(qst_prec prec, const void* T, int64_t ldT, void* rho, int64_t ldr, int n,
                         double* partials, double* tau_dev, void* sk, hipStream_t s, const void* f = nullptr,
                         const Pass0Out* x0 = nullptr, void* planes = nullptr, void* ttplanes = nullptr) {
  if (use_x6(prec, n)) return launch_x6_herk(T, ldT, rho, ldr, n, partials, f, tau_dev, planes, sk, s, x0, ttplanes);
  const bool fold = n >= 6;
  hipError_t e = launch_tau(prec, T, ldT, n, partials, fold ? nullptr : tau_dev, s, f, planes);
  if (e != hipSuccess) return e;
  return launch_herk(prec, T, ldT, rho, ldr, n, fold ? partials : nullptr, tau_dev, sk, s, x0, planes);
}

qst_status likelihood_impl(int n, qst_prec prec, const void* T, int64_t ldT, const void* f, const double* povm_host,
                           double* tau_dev, double* nll_dev, unsigned long long* bad_dev, void* G, int64_t ldG,
                           void* ws, size_t ws_bytes, void* stream, const void* pt, double* fc_dev,
                           void* gplanes = nullptr, void* ttplanes = nullptr);

}  // namespace

extern "C" {

qst_status qst_state_map(int n, qst_prec prec, const void* T, int64_t ldT, void* rho, int64_t ld_rho,
                         double* tau_dev, void* ws, size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(rho, ld_rho, n, "rho", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(tau_dev, "tau_dev", msg)) != QST_OK) return fail(st, msg);
  const WsLayout L = workspace_layout(n, prec, QST_OP_STATE_MAP, false);
  if ((st = check_ws(ws, ws_bytes, L.total, msg)) != QST_OK) return fail(st, msg);
  if (T == rho) return fail(QST_ERR_INVALID_ARG, "rho must not alias T");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* partials = reinterpret_cast<double*>(ws_at(ws, L.partials));
  hipError_t e = run_state_map(prec, T, ldT, rho, ld_rho, n, partials, tau_dev, L.has_sk ? ws_at(ws, L.sk) : nullptr, s,
                               nullptr, nullptr, L.has_planes ? ws_at(ws, L.planes) : nullptr);
  if (e != hipSuccess) return hip_fail(e, "state map");
  clear_error();
  return QST_OK;
}

qst_status qst_state_premap(int n, qst_prec prec, int mode, const void* X, int64_t ldX, void* Y, int64_t ldY,
                            void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(X, ldX, n, "X", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(Y, ldY, n, "Y", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_premap(mode, X, ldX, Y, ldY, msg)) != QST_OK) return fail(st, msg);
  hipError_t e = launch_premap(prec, mode, X, ldX, Y, ldY, n, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "state pre-map");
  clear_error();
  return QST_OK;
}

qst_status qst_abs_map(int n, qst_prec prec, double P, const void* T, int64_t ldT, const void* Q0, void* A,
                       int64_t ldA, void* Q, double* lam, int* sweeps, void* ws, size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(A, ldA, n, "A", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(Q, "Q", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(lam, "lam", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_abs_order(P, msg)) != QST_OK) return fail(st, msg);
  if (A == T && ldA != ldT) return fail(QST_ERR_INVALID_ARG, "in place (A == T) needs ldA == ldT");
  if (Q == T || Q == A || Q == static_cast<void*>(lam)) return fail(QST_ERR_INVALID_ARG, "Q must not alias T, A or lam");
  if (Q0 && (Q0 == T || Q0 == A || Q0 == static_cast<const void*>(lam)))
    return fail(QST_ERR_INVALID_ARG, "Q0 must not alias T, A or lam");
  if ((st = check_ws(ws, ws_bytes, workspace_layout(n, prec, QST_OP_ABS_MAP, false).total, msg)) != QST_OK)
    return fail(st, msg);
  int taken = -1;
  hipError_t e = launch_abs_map(prec, n, P, T, ldT, Q0, A, ldA, Q, lam, ws, static_cast<hipStream_t>(stream), &taken,
                                kJacobiMaxSweeps, nullptr);
  if (e != hipSuccess) return hip_fail(e, "absolute map");
  if (sweeps) *sweeps = taken;
  if (taken < 0)
    return fail(QST_ERR_INVALID_ARG, "absolute map: the eigendecomposition did not converge (is T finite?)");
  clear_error();
  return QST_OK;
}

qst_status qst_fidelity_general(int n, qst_prec prec, const void* T, int64_t ldT, const void* rho, int64_t ldR,
                                double* F_dev, int* sweeps, void* ws, size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(rho, ldR, n, "rho", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(F_dev, "F_dev", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ws(ws, ws_bytes, workspace_layout(n, prec, QST_OP_ABS_MAP, false).total, msg)) != QST_OK)
    return fail(st, msg);
  int taken = -1;
  hipError_t e = launch_fidelity_general(prec, n, T, ldT, rho, ldR, F_dev, ws, static_cast<hipStream_t>(stream), &taken,
                                         kJacobiMaxSweeps, nullptr);
  if (e != hipSuccess) return hip_fail(e, "general fidelity");
  if (sweeps) *sweeps = taken;
  if (taken < 0)
    return fail(QST_ERR_INVALID_ARG, "general fidelity: the eigendecomposition did not converge (are T and rho "
                                     "finite?)");
  clear_error();
  return QST_OK;
}

qst_status qst_abs_map_async(int n, qst_prec prec, double P, const void* T, int64_t ldT, const void* Q0, void* A,
                             int64_t ldA, void* Q, double* lam, int max_sweeps, int* sweeps_dev, void* ws,
                             size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(A, ldA, n, "A", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(Q, "Q", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(lam, "lam", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(sweeps_dev, "sweeps_dev", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_abs_order(P, msg)) != QST_OK) return fail(st, msg);
  if (max_sweeps < 1 || max_sweeps > kJacobiMaxSweeps)
    return fail(QST_ERR_INVALID_ARG, "max_sweeps=" + std::to_string(max_sweeps) + " outside [1, " +
                                         std::to_string(kJacobiMaxSweeps) + "]");
  if (A == T && ldA != ldT) return fail(QST_ERR_INVALID_ARG, "in place (A == T) needs ldA == ldT");
  if (Q == T || Q == A || Q == static_cast<void*>(lam)) return fail(QST_ERR_INVALID_ARG, "Q must not alias T, A or lam");
  if (Q0 && (Q0 == T || Q0 == A || Q0 == static_cast<const void*>(lam)))
    return fail(QST_ERR_INVALID_ARG, "Q0 must not alias T, A or lam");
  if ((st = check_ws(ws, ws_bytes, workspace_layout(n, prec, QST_OP_ABS_MAP, false).total, msg)) != QST_OK)
    return fail(st, msg);
  hipError_t e = launch_abs_map(prec, n, P, T, ldT, Q0, A, ldA, Q, lam, ws, static_cast<hipStream_t>(stream), nullptr,
                                max_sweeps, sweeps_dev);
  if (e != hipSuccess) return hip_fail(e, "absolute map");
  clear_error();
  return QST_OK;
}

qst_status qst_fidelity_general_async(int n, qst_prec prec, const void* T, int64_t ldT, const void* rho, int64_t ldR,
                                      double* F_dev, int max_sweeps, int* sweeps_dev, void* ws, size_t ws_bytes,
                                      void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(rho, ldR, n, "rho", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(F_dev, "F_dev", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(sweeps_dev, "sweeps_dev", msg)) != QST_OK) return fail(st, msg);
  if (max_sweeps < 1 || max_sweeps > kJacobiMaxSweeps)
    return fail(QST_ERR_INVALID_ARG, "max_sweeps=" + std::to_string(max_sweeps) + " outside [1, " +
                                         std::to_string(kJacobiMaxSweeps) + "]");
  if ((st = check_ws(ws, ws_bytes, workspace_layout(n, prec, QST_OP_ABS_MAP, false).total, msg)) != QST_OK)
    return fail(st, msg);
  hipError_t e = launch_fidelity_general(prec, n, T, ldT, rho, ldR, F_dev, ws, static_cast<hipStream_t>(stream),
                                         nullptr, max_sweeps, sweeps_dev);
  if (e != hipSuccess) return hip_fail(e, "general fidelity");
  clear_error();
  return QST_OK;
}

qst_status qst_abs_map_backward(int n, qst_prec prec, double P, const void* Q, const double* lam, const void* GA,
                                int64_t ldGA, void* GT, int64_t ldGT, void* ws, size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(Q, "Q", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(lam, "lam", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(GA, ldGA, n, "GA", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(GT, ldGT, n, "GT", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_abs_order(P, msg)) != QST_OK) return fail(st, msg);
  if (GT == GA && ldGT != ldGA) return fail(QST_ERR_INVALID_ARG, "in place (GT == GA) needs ldGT == ldGA");
  if (GT == Q || GT == static_cast<const void*>(lam)) return fail(QST_ERR_INVALID_ARG, "GT must not alias Q or lam");
  if ((st = check_ws(ws, ws_bytes, workspace_layout(n, prec, QST_OP_ABS_MAP, false).total, msg)) != QST_OK)
    return fail(st, msg);
  hipError_t e = launch_abs_map_backward(prec, n, P, Q, lam, GA, ldGA, GT, ldGT, ws, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "absolute map adjoint");
  clear_error();
  return QST_OK;
}

qst_status qst_fnn_forward(int n, qst_prec prec, const void* W1, const void* b1, const void* W2, const void* b2,
                           const void* x, void* h_pre, void* T, int64_t ldT, void* ws, size_t ws_bytes,
                           void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  const void* ins[] = {W1, b1, W2, b2, x, h_pre};
  const char* names[] = {"W1", "b1", "W2", "b2", "x", "h_pre"};
  for (int i = 0; i < 6; ++i)
    if ((st = check_ptr(ins[i], names[i], msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ws(ws, ws_bytes, workspace_layout(n, prec, QST_OP_FNN, false).total, msg)) != QST_OK)
    return fail(st, msg);
  hipError_t e = launch_fnn_forward(prec, n, W1, b1, W2, b2, x, h_pre, T, ldT, ws, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "network forward");
  clear_error();
  return QST_OK;
}

qst_status qst_fnn_backward(int n, qst_prec prec, const void* W2, const void* x, const void* h_pre, const void* G,
                            int64_t ldG, void* dW1, void* db1, void* dW2, void* db2, void* ws, size_t ws_bytes,
                            void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  const void* ptrs[] = {W2, x, h_pre, dW1, db1, dW2, db2};
  const char* names[] = {"W2", "x", "h_pre", "dW1", "db1", "dW2", "db2"};
  for (int i = 0; i < 7; ++i)
    if ((st = check_ptr(ptrs[i], names[i], msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(G, ldG, n, "G", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ws(ws, ws_bytes, workspace_layout(n, prec, QST_OP_FNN, false).total, msg)) != QST_OK)
    return fail(st, msg);
  hipError_t e = launch_fnn_backward(prec, n, W2, x, h_pre, G, ldG, dW1, db1, dW2, db2, ws,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "network backward");
  clear_error();
  return QST_OK;
}

qst_status qst_rprop_step(int64_t count, qst_prec prec, void* param, const void* grad, void* prev, void* step,
                          double eta_minus, double eta_plus, double step_min, double step_max, void* stream) {
  std::string msg;
  if (!prec_valid(prec)) return fail(QST_ERR_INVALID_ARG, "unknown precision " + std::to_string(prec));
  if (count < 0) return fail(QST_ERR_INVALID_ARG, "count is negative");
  if (!(eta_minus > 0.0 && eta_minus < 1.0 && eta_plus > 1.0))
    return fail(QST_ERR_INVALID_ARG, "Rprop factors need 0 < eta_minus < 1 < eta_plus");
  if (!(step_min > 0.0 && step_min <= step_max))
    return fail(QST_ERR_INVALID_ARG, "Rprop step bounds need 0 < step_min <= step_max");
  if (count > 0) {
    qst_status st;
    const void* ptrs[] = {param, grad, prev, step};
    const char* names[] = {"param", "grad", "prev", "step"};
    for (int i = 0; i < 4; ++i)
      if ((st = check_ptr(ptrs[i], names[i], msg)) != QST_OK) return fail(st, msg);
  }
  hipError_t e = launch_rprop(prec, count, param, grad, prev, step, eta_minus, eta_plus, step_min, step_max,
                              static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "Rprop step");
  clear_error();
  return QST_OK;
}

qst_status qst_fidelity_lowrank(int n, qst_prec prec, const void* T, int64_t ldT, const void* W, int64_t ldW, int r,
                                double* F_dev, void* ws, size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(W, "W", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(F_dev, "F_dev", msg)) != QST_OK) return fail(st, msg);
  if (r < 1 || r > QST_FIDELITY_MAX_RANK)
    return fail(QST_ERR_INVALID_ARG, "rank r=" + std::to_string(r) + " outside [1, " +
                                         std::to_string(QST_FIDELITY_MAX_RANK) + "]");
  if (ldW < r) return fail(QST_ERR_INVALID_ARG, "ldW (" + std::to_string(ldW) + ") is smaller than r");
  if ((st = check_ws(ws, ws_bytes, workspace_layout(n, prec, QST_OP_FIDELITY, false).total, msg)) != QST_OK)
    return fail(st, msg);
  hipError_t e = launch_fidelity_lowrank(prec, T, ldT, W, ldW, r, n, ws, F_dev, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "fidelity");
  clear_error();
  return QST_OK;
}

qst_status qst_fidelity_classical(int n, qst_prec prec, const void* p_hat, const void* p, double* F_dev, void* ws,
                                  size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(p_hat, "p_hat", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(p, "p", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(F_dev, "F_dev", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ws(ws, ws_bytes, workspace_layout(n, prec, QST_OP_FIDELITY, false).total, msg)) != QST_OK)
    return fail(st, msg);
  hipError_t e = launch_fidelity_classical(prec, p_hat, p, n, ws, F_dev, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "classical fidelity");
  clear_error();
  return QST_OK;
}

qst_status qst_povm_probs(int n, qst_prec prec, const void* rho, int64_t ld_rho, const double* povm_host,
                          void* p, void* ws, size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(rho, ld_rho, n, "rho", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(p, "p", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_povm(povm_host, msg)) != QST_OK) return fail(st, msg);
  const WsLayout L = workspace_layout(n, prec, QST_OP_POVM_PROBS, false);
  if ((st = check_ws(ws, ws_bytes, L.total, msg)) != QST_OK) return fail(st, msg);
  double W[32], V[32];
  povm_mode_matrices(povm_host, W, V);
  const PovmPlan pl = make_povm_plan(n, prec);
  hipError_t e = launch_povm(false, prec, pl, W, povm_host == nullptr, rho, ld_rho, p, nullptr, nullptr,
                             ws_at(ws, L.inter0), ws_at(ws, L.inter1), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "POVM map");
  clear_error();
  return QST_OK;
}

qst_status qst_nll(int n, qst_prec prec, const void* p, const void* f, double* nll_dev,
                   unsigned long long* bad_dev, void* ws, size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(p, "p", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(f, "f", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(nll_dev, "nll_dev", msg)) != QST_OK) return fail(st, msg);
  const WsLayout L = workspace_layout(n, prec, QST_OP_NLL, false);
  if ((st = check_ws(ws, ws_bytes, L.total, msg)) != QST_OK) return fail(st, msg);
  hipError_t e = launch_nll(prec, p, f, n, reinterpret_cast<double*>(ws_at(ws, L.partials)), nll_dev, bad_dev,
                            static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "NLL reduction");
  clear_error();
  return QST_OK;
}

qst_status qst_nll_backward(int n, qst_prec prec, const void* T, int64_t ldT, const void* f, const void* p,
                            const double* tau_dev, const double* nll_dev, const double* povm_host,
                            const double* upstream_dev, void* gradT, int64_t ldG, void* ws, size_t ws_bytes,
                            void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(gradT, ldG, n, "gradT", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(f, "f", msg)) != QST_OK) return fail(st, msg);
  if (p && !tau_dev) return fail(QST_ERR_INVALID_ARG, "tau_dev is NULL while p is given");
  if ((st = check_povm(povm_host, msg)) != QST_OK) return fail(st, msg);
  if (T == gradT) return fail(QST_ERR_INVALID_ARG, "gradT must not alias T");
  const bool recompute = (p == nullptr);
  const WsLayout L = workspace_layout(n, prec, QST_OP_NLL_BACKWARD, recompute);
  if ((st = check_ws(ws, ws_bytes, L.total, msg)) != QST_OK) return fail(st, msg);

  hipStream_t s = static_cast<hipStream_t>(stream);
  double* partials = reinterpret_cast<double*>(ws_at(ws, L.partials));
  double* scalars = reinterpret_cast<double*>(ws_at(ws, L.scalars));
  double W[32], V[32];
  povm_mode_matrices(povm_host, W, V);
  const bool tetra = povm_host == nullptr;
  const PovmPlan pl = make_povm_plan(n, prec);
  const int64_t d = int64_t(1) << n;
  hipError_t e;
  if (recompute) {
    // rho and p are rebuilt from T here; rho lives in the G' slot.
    double* tau_ws = scalars + 1;
    e = run_state_map(prec, T, ldT, ws_at(ws, L.rho), d, n, partials, tau_ws, L.has_sk ? ws_at(ws, L.sk) : nullptr, s,
                      nullptr, nullptr, L.has_planes ? ws_at(ws, L.planes) : nullptr);
    if (e != hipSuccess) return hip_fail(e, "state map (recompute)");
    e = launch_povm(false, prec, pl, W, tetra, ws_at(ws, L.rho), d, ws_at(ws, L.p), nullptr, nullptr,
                    ws_at(ws, L.inter0), ws_at(ws, L.inter1), s);
    if (e != hipSuccess) return hip_fail(e, "POVM map (recompute)");
    p = ws_at(ws, L.p);
    tau_dev = tau_ws;
  }
  const double* F_dev = nll_dev ? nll_dev + 1 : scalars;
  if (!nll_dev) {
    e = launch_fsum(prec, f, n, partials, scalars, s);
    if (e != hipSuccess) return hip_fail(e, "F reduction");
  }
  void* G = ws_at(ws, L.gmat);
  e = launch_povm(true, prec, pl, V, tetra, G, d, const_cast<void*>(p), f, F_dev, ws_at(ws, L.inter0),
                  ws_at(ws, L.inter1), s);
  if (e != hipSuccess) return hip_fail(e, "adjoint POVM map");
  e = launch_hemm(prec, G, d, T, ldT, gradT, ldG, n, tau_dev, upstream_dev, L.has_sk ? ws_at(ws, L.sk) : nullptr, s,
                  L.has_planes ? ws_at(ws, L.planes) : nullptr);
  if (e != hipSuccess) return hip_fail(e, "G' T");
  clear_error();
  return QST_OK;
}

qst_status qst_likelihood(int n, qst_prec prec, const void* T, int64_t ldT, const void* f,
                          const double* povm_host, double* tau_dev, double* nll_dev,
                          unsigned long long* bad_dev, void* G, int64_t ldG, void* ws, size_t ws_bytes,
                          void* stream) {
  return likelihood_impl(n, prec, T, ldT, f, povm_host, tau_dev, nll_dev, bad_dev, G, ldG, ws, ws_bytes, stream,
                         nullptr, nullptr);
}

qst_status qst_likelihood_fc(int n, qst_prec prec, const void* T, int64_t ldT, const void* f, const void* p_target,
                             const double* povm_host, double* tau_dev, double* nll_dev, double* fc_dev,
                             unsigned long long* bad_dev, void* G, int64_t ldG, void* ws, size_t ws_bytes,
                             void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_ptr(p_target, "p_target", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(fc_dev, "fc_dev", msg)) != QST_OK) return fail(st, msg);
  return likelihood_impl(n, prec, T, ldT, f, povm_host, tau_dev, nll_dev, bad_dev, G, ldG, ws, ws_bytes, stream,
                         p_target, fc_dev);
}

}  // extern "C"

namespace {

// The workspace of qst_likelihood_noalloc.  In host code `scratch` names a
// host-side stand-in, not device memory: kernels get the device address
// that hipGetSymbolAddress returns for the current device (each GPU holds
// its own copy of the array), looked up once per device and kept here.
__device__ __align__(256) unsigned char scratch[QST_STATIC_SCRATCH_BYTES];

constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchMaxDevices] = {};

qst_status static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchMaxDevices)
    return fail(QST_ERR_UNSUPPORTED, "device ordinal " + std::to_string(dev) + " beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess)
      return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(QST_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return QST_OK;
}

}  // namespace

extern "C" qst_status qst_likelihood_noalloc(int n, qst_prec prec, const void* T, int64_t ldT, const void* f,
                                             const double* povm_host, double* tau_dev, double* nll_dev,
                                             unsigned long long* bad_dev, void* G, int64_t ldG, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  const size_t need = workspace_layout(n, prec, QST_OP_LIKELIHOOD, false).total;
  if (need > QST_STATIC_SCRATCH_BYTES)
    return fail(QST_ERR_WORKSPACE, "N=" + std::to_string(n) + " needs " + std::to_string(need) +
                                       " bytes of workspace, more than the static scratch of " +
                                       std::to_string(QST_STATIC_SCRATCH_BYTES) +
                                       " bytes; use qst_likelihood with a workspace");
  void* ws = nullptr;
  if ((st = static_scratch(&ws)) != QST_OK) return st;
  return likelihood_impl(n, prec, T, ldT, f, povm_host, tau_dev, nll_dev, bad_dev, G, ldG, ws,
                         QST_STATIC_SCRATCH_BYTES, stream, nullptr, nullptr);
}

namespace {

// gplanes / ttplanes (the combined likelihood-and-gradient call, QST_F32X6
// with a fused plan whose pass 0 writes planes): adjoint pass 0 writes G' as
// the gradient product's planes at gplanes (G unused), and the T split writes
// T^T's planes at ttplanes.
qst_status likelihood_impl(int n, qst_prec prec, const void* T, int64_t ldT, const void* f, const double* povm_host,
                           double* tau_dev, double* nll_dev, unsigned long long* bad_dev, void* G, int64_t ldG,
                           void* ws, size_t ws_bytes, void* stream, const void* pt, double* fc_dev,
                           void* gplanes, void* ttplanes) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(f, "f", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(tau_dev, "tau_dev", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(nll_dev, "nll_dev", msg)) != QST_OK) return fail(st, msg);
  if (G && (st = check_matrix(G, ldG, n, "G", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_povm(povm_host, msg)) != QST_OK) return fail(st, msg);
  if (G == T) return fail(QST_ERR_INVALID_ARG, "G must not alias T");
  const WsLayout L = workspace_layout(n, prec, QST_OP_LIKELIHOOD, false);
  if ((st = check_ws(ws, ws_bytes, L.total, msg)) != QST_OK) return fail(st, msg);

  hipStream_t s = static_cast<hipStream_t>(stream);
  double* partials = reinterpret_cast<double*>(ws_at(ws, L.partials));
  double W[32], V[32];
  povm_mode_matrices(povm_host, W, V);
  const bool tetra = povm_host == nullptr;
  const PovmPlan pl = make_povm_plan(n, prec);
  const int64_t d = int64_t(1) << n;
  void* rho = ws_at(ws, L.rho);
  const bool fused = fused_likelihood(pl, prec);
  // tetrahedral POVM: the first pass runs in the epilogue of T T^dagger, so
  // rho is never written (the tile sizes of pass 0 divide the 64 x 64
  // product tiles for every fused plan)
  const bool x0 = fused && tetra && d >= 64 && pl.g[0] >= 4 && pl.g[0] <= 6;
  const Pass0Out p0{ws_at(ws, L.inter0), pl.g[0], true};
  if ((gplanes || ttplanes) && !(use_x6(prec, n) && fused && x0 && pass0_writes_planes(pl)))
    return fail(QST_ERR_INVALID_ARG, "operand planes requested where the plan cannot form them");
  hipError_t e = run_state_map(prec, T, ldT, rho, d, n, partials, tau_dev, L.has_sk ? ws_at(ws, L.sk) : nullptr, s,
                               fused ? f : nullptr, x0 ? &p0 : nullptr, L.has_planes ? ws_at(ws, L.planes) : nullptr,
                               ttplanes);
  if (e != hipSuccess) return hip_fail(e, "state map");
  if (fused) {
    e = launch_povm_fused(prec, pl, W, V, tetra, rho, d, f, partials + kReduceBlocks, G, ldG, ws_at(ws, L.inter0),
                          ws_at(ws, L.inter1), reinterpret_cast<double*>(ws_at(ws, L.fpart)), nll_dev, bad_dev, x0,
                          s, pt, fc_dev, gplanes);
    if (e != hipSuccess) return hip_fail(e, "fused POVM / likelihood passes");
  } else {
    void* p = ws_at(ws, L.p);
    e = launch_povm(false, prec, pl, W, tetra, rho, d, p, nullptr, nullptr, ws_at(ws, L.inter0), ws_at(ws, L.inter1), s);
    if (e != hipSuccess) return hip_fail(e, "POVM map");
    e = launch_nll(prec, p, f, n, partials, nll_dev, bad_dev, s);
    if (e != hipSuccess) return hip_fail(e, "NLL reduction");
    if (pt) {
      e = launch_fidelity_classical_part(prec, p, pt, n, partials, fc_dev, s);
      if (e != hipSuccess) return hip_fail(e, "classical fidelity");
    }
    if (G) {
      e = launch_povm(true, prec, pl, V, tetra, G, ldG, p, f, nll_dev + 1, ws_at(ws, L.inter0), ws_at(ws, L.inter1), s);
      if (e != hipSuccess) return hip_fail(e, "adjoint POVM map");
    }
  }
  clear_error();
  return QST_OK;
}

}  // namespace

namespace {

GeneralBufs general_bufs(void* ws, const GeneralLayout& L) {
  return GeneralBufs{reinterpret_cast<double*>(ws_at(ws, L.partials)), reinterpret_cast<double*>(ws_at(ws, L.scal)),
                     L.inter0 ? ws_at(ws, L.inter0) : nullptr, L.inter1 ? ws_at(ws, L.inter1) : nullptr,
                     ws_at(ws, L.e), L.h ? ws_at(ws, L.h) : nullptr, ws_at(ws, L.bufA), ws_at(ws, L.bufB),
                     L.p ? ws_at(ws, L.p) : nullptr};
}

}  // namespace

extern "C" {

qst_status qst_povm_probs_general(int n, qst_prec prec, const void* rho, int64_t ld_rho, int K,
                                  const double* povm_host, void* p, void* ws, size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(rho, ld_rho, n, "rho", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(p, "p", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_povm_general(n, K, 1, povm_host, msg)) != QST_OK) return fail(st, msg);
  const GeneralLayout L = general_layout(n, prec, K, false);
  if ((st = check_ws(ws, ws_bytes, L.total, msg)) != QST_OK) return fail(st, msg);
  std::vector<double> C(size_t(n) * K * 4);
  general_factors(n, K, 1, povm_host, C.data());
  hipError_t e = launch_general_probs(prec, n, K, C.data(), rho, ld_rho, p, general_bufs(ws, L),
                                      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "general POVM map");
  clear_error();
  return QST_OK;
}

qst_status qst_likelihood_general(int n, qst_prec prec, const void* T, int64_t ldT, int settings, int K,
                                  const double* povm_host, const void* f, double* tau_dev, double* nll_dev,
                                  unsigned long long* bad_dev, void* G, int64_t ldG, void* ws, size_t ws_bytes,
                                  void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(f, "f", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(tau_dev, "tau_dev", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(nll_dev, "nll_dev", msg)) != QST_OK) return fail(st, msg);
  if (G && (st = check_matrix(G, ldG, n, "G", msg)) != QST_OK) return fail(st, msg);
  if (G == T) return fail(QST_ERR_INVALID_ARG, "G must not alias T");
  if ((st = check_povm_general(n, K, settings, povm_host, msg)) != QST_OK) return fail(st, msg);
  const GeneralLayout L = general_layout(n, prec, K, true);
  if ((st = check_ws(ws, ws_bytes, L.total, msg)) != QST_OK) return fail(st, msg);
  std::vector<double> C(size_t(settings) * n * K * 4);
  general_factors(n, K, settings, povm_host, C.data());
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t d = int64_t(1) << n;
  void* rho = ws_at(ws, L.rho);
  hipError_t e = run_state_map(prec, T, ldT, rho, d, n, reinterpret_cast<double*>(ws_at(ws, L.partials)), tau_dev,
                               L.has_sk ? ws_at(ws, L.sk) : nullptr, s, nullptr, nullptr,
                               L.has_planes ? ws_at(ws, L.planes) : nullptr);
  if (e != hipSuccess) return hip_fail(e, "state map");
  e = launch_general_likelihood(prec, n, K, settings, C.data(), rho, d, f, G, ldG, nll_dev, bad_dev,
                                general_bufs(ws, L), s);
  if (e != hipSuccess) return hip_fail(e, "general POVM likelihood");
  clear_error();
  return QST_OK;
}

qst_status qst_grad_product(int n, qst_prec prec, const void* G, int64_t ldG, const void* T, int64_t ldT,
                            const double* tau_dev, const double* upstream_dev, void* gradT, int64_t ld_grad,
                            void* ws, size_t ws_bytes, void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(G, ldG, n, "G", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(gradT, ld_grad, n, "gradT", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_ptr(tau_dev, "tau_dev", msg)) != QST_OK) return fail(st, msg);
  if (gradT == T || gradT == G) return fail(QST_ERR_INVALID_ARG, "gradT must not alias G or T");
  const WsLayout L = workspace_layout(n, prec, QST_OP_GRAD_PRODUCT, false);
  if ((st = check_ws(ws, ws_bytes, L.total, msg)) != QST_OK) return fail(st, msg);
  hipError_t e = launch_hemm(prec, G, ldG, T, ldT, gradT, ld_grad, n, tau_dev, upstream_dev,
                             L.has_sk ? ws_at(ws, L.sk) : nullptr, static_cast<hipStream_t>(stream),
                             L.has_planes ? ws_at(ws, L.planes) : nullptr);
  if (e != hipSuccess) return hip_fail(e, "G' T");
  clear_error();
  return QST_OK;
}

qst_status qst_likelihood_grad(int n, qst_prec prec, const void* T, int64_t ldT, const void* f,
                               const double* povm_host, double* tau_dev, double* nll_dev,
                               unsigned long long* bad_dev, void* gradT, int64_t ld_grad, void* ws, size_t ws_bytes,
                               void* stream) {
  std::string msg;
  qst_status st;
  if ((st = check_common(n, prec, msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(T, ldT, n, "T", msg)) != QST_OK) return fail(st, msg);
  if ((st = check_matrix(gradT, ld_grad, n, "gradT", msg)) != QST_OK) return fail(st, msg);
  if (gradT == T) return fail(QST_ERR_INVALID_ARG, "gradT must not alias T");
  const WsLayout L = workspace_layout(n, prec, QST_OP_LIKELIHOOD_GRAD, false);
  if ((st = check_ws(ws, ws_bytes, L.total, msg)) != QST_OK) return fail(st, msg);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const PovmPlan pl = make_povm_plan(n, prec);
  const int64_t d = int64_t(1) << n;
  void* tp = L.has_tplanes ? ws_at(ws, L.tplanes) : nullptr;
  // QST_F32X6 with the tetrahedral POVM and a plan whose adjoint pass 0
  // writes planes: both operands' planes are formed inside the likelihood
  // (the same bits as the split kernels would write from G' and T)
  const bool in_call = use_x6(prec, n) && povm_host == nullptr && fused_likelihood(pl, prec) &&
                       pass0_writes_planes(pl) && tp != nullptr;
  if (in_call) {
    unsigned char* gpl = static_cast<unsigned char*>(tp);
    unsigned char* tpl = gpl + x6_hemm_plane_bytes(n) / 2;
    if ((st = likelihood_impl(n, prec, T, ldT, f, povm_host, tau_dev, nll_dev, bad_dev, nullptr, 0, ws, ws_bytes,
                              stream, nullptr, nullptr, gpl, tpl)) != QST_OK)
      return st;
    hipError_t e = launch_x6_hemm(nullptr, 0, T, ldT, gradT, ld_grad, n, tau_dev, nullptr, tp, s, true, true);
    if (e != hipSuccess) return hip_fail(e, "G' T");
  } else {
    void* G = ws_at(ws, L.gmat);
    if ((st = likelihood_impl(n, prec, T, ldT, f, povm_host, tau_dev, nll_dev, bad_dev, G, d, ws, ws_bytes, stream,
                              nullptr, nullptr)) != QST_OK)
      return st;
    hipError_t e = launch_hemm(prec, G, d, T, ldT, gradT, ld_grad, n, tau_dev, nullptr,
                               L.has_sk ? ws_at(ws, L.sk) : nullptr, s, tp);
    if (e != hipSuccess) return hip_fail(e, "G' T");
  }
  clear_error();
  return QST_OK;
}

}  // extern "C"
