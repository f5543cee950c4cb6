// HIP-free host logic: argument validation, POVM pass planning and
// workspace layout.  Compiles with g++ alone (no HIP headers), so its tests
// run on machines without a GPU.
#include "qst_plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace qst {

namespace {
thread_local std::string g_last_error;

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
const char* last_error_cstr() { return g_last_error.c_str(); }

PovmPlan make_povm_plan(int n, qst_prec prec) {
  PovmPlan pl;
  pl.n = n;
  const int kFirstMax = 6;  // 4^6 complex in the first (row-tile) pass
  const int kLaterMax = 5;  // 4^5 complex x J in later passes
  int passes = 1;
  if (n > kFirstMax) passes = 1 + (n - kFirstMax + kLaterMax - 1) / kLaterMax;
  pl.passes = passes;
  const int base = n / passes, rem = n % passes;
  for (int j = 0; j < passes; ++j) pl.g[j] = base + (j < rem ? 1 : 0);
  int U = n;
  const size_t cb = complex_bytes(prec);
  for (int j = 0; j < passes; ++j) {
    pl.U[j] = U;
    if (j == 0) {
      pl.J[j] = 1;
    } else {
      const int64_t kd = int64_t(1) << (2 * (n - U));
      int64_t J = int64_t(65536) / ((int64_t(1) << (2 * pl.g[j])) * int64_t(cb));
      if (J > 64) J = 64;
      if (J > kd) J = kd;
      if (J < 1) J = 1;
      pl.J[j] = int(J);
    }
    U -= pl.g[j];
  }
  return pl;
}

int64_t povm_pass_blocks(const PovmPlan& pl, int j) {
  const int Up = pl.U[j] - pl.g[j];
  const int64_t side = int64_t(1) << Up;
  const int64_t pairs = side * (side + 1) / 2;
  const int64_t kd = int64_t(1) << (2 * (pl.n - pl.U[j]));
  return pairs * (kd / pl.J[j]);
}

bool fast_pass_available(const PovmPlan& pl, int j, qst_prec prec) {
  if (j < 0 || j >= pl.passes) return false;
  const int g = pl.g[j], J = pl.J[j];
  if (j == 0) return pl.passes >= 2 && J == 1 && g >= 4 && g <= 6;
  if (prec == QST_F64) return (g == 5 && J == 4) || (g == 4 && J == 16) || (g == 3 && J == 64);
  return (g == 5 && J == 8) || (g == 4 && J == 32) || (g == 3 && J == 64);
}

bool fused_likelihood(const PovmPlan& pl, qst_prec prec) {
  if (pl.passes < 2) return false;
  for (int j = 0; j < pl.passes; ++j)
    if (!fast_pass_available(pl, j, prec)) return false;
  return true;
}

FidelityLayout fidelity_layout(int n) {
  FidelityLayout f;
  const size_t d = size_t(1) << n;
  f.nrb = d >= 64 ? 16 : 1;
  const size_t ncb = d < 64 ? 1 : d / 64;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  f.mpart = take(size_t(f.nrb) * kFidelityMaxRank * d * 2 * sizeof(double));
  f.mrow = take(size_t(kFidelityMaxRank) * d * 2 * sizeof(double));
  f.gram = take(size_t(kFidelityMaxRank) * kFidelityMaxRank * 2 * sizeof(double));
  f.taup = take(ncb * f.nrb * sizeof(double));
  f.cpart = take(size_t(kReduceBlocks) * sizeof(double));
  f.total = off;
  return f;
}

FnnLayout fnn_layout(int n, size_t real_bytes) {
  FnnLayout f;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t H = size_t(2) * n;
  f.part = take(size_t(kFnnBlocks) * H * sizeof(double));
  f.hvec = take(H * sizeof(double));
  f.dhvec = take(H * sizeof(double));
  f.yvec = take((size_t(1) << (2 * n)) * real_bytes);
  f.total = off;
  return f;
}

AbsMapLayout absmap_layout(int n) {
  AbsMapLayout a;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t d = size_t(1) << n;
  a.b0 = take(d * d * 16);
  a.b1 = take(d * d * 16);
  a.b2 = take(d * d * 16);
  // two partials per workgroup of a Jacobi round: d/2 pairs x ceil(d/256)
  // column chunks (at least d values: |lambda|^(P/4) reuses the area)
  const size_t chunks = (d / 2 + 127) / 128;
  a.part = take(std::max(d, d * chunks) * sizeof(double));
  a.scal = take(8 * sizeof(double));
  a.state = take(64);  // the Jacobi sweep state (done flag, sweeps, parity, previous norm)
  if (n >= kStreamKMinQubits) {
    a.sk_bytes = stream_k_partial_bytes(QST_F64);
    a.sk = take(a.sk_bytes);
  }
  a.eig = take(eigh_layout(n).total);
  a.total = off;
  return a;
}

EighLayout eigh_layout(int n) {
  EighLayout e;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t d = size_t(1) << n;
  const size_t blocks = (d - 1 + kEighBlock - 1) / kEighBlock;
  e.diag = take(d * sizeof(double));
  e.off = take(d * sizeof(double));
  e.tau = take(d * 16);
  e.y0 = take(d * 16);
  e.y1 = take(d * 16);
  e.p0 = take(kTrdMaxGroups * sizeof(double));
  e.p1 = take(kTrdMaxGroups * sizeof(double));
  e.bstart = take(d * sizeof(int));
  e.bend = take(d * sizeof(int));
  e.scal = take(8 * sizeof(double));
  e.tfac = take(blocks * kEighBlock * kEighBlock * 16);
  // partial products of the back-transformation, or the blocks' partial
  // Gram matrices, whichever is larger
  const size_t chunks = (d - 1 + eigh_chunk_rows(int(d)) - 1) / eigh_chunk_rows(int(d));
  const size_t grams = blocks * size_t(eigh_gram_chunks(int(d))) * kEighBlock * kEighBlock;
  e.pbuf = take(std::max(std::max<size_t>(chunks, 1) * kEighBlock * d, grams) * 16);
  e.xbuf = take(kEighBlock * d * 16);
  e.total = off;
  return e;
}

WsLayout workspace_layout(int n, qst_prec prec, int op, bool recompute) {
  WsLayout w;
  const size_t cb = complex_bytes(prec), rb = real_bytes(prec);
  const size_t d = size_t(1) << n;
  const size_t D = d * d;
  const PovmPlan pl = make_povm_plan(n, prec);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const bool x6 = use_x6(prec, n);
  // stream-K partial tiles: the QST_F32X6 T T^dagger always, the other
  // products from kStreamKMinQubits
  const bool sk = x6 || n >= kStreamKMinQubits;
  const size_t sk_bytes = x6 ? x6_partial_bytes(n) : stream_k_partial_bytes(prec);
  const bool planes = (prec == QST_BF16GEMM && d > size_t(kBf16SplitMaxDim)) || x6;
  const bool hemm_planes = (prec == QST_BF16GEMM && d >= 1024) || x6;
  // bf16 planes of d x d: the BF16 path's (2 for T T^dagger, 8 for G' T)
  // or the QST_F32X6 split planes (12 and 18)
  const size_t herk_planes = x6 ? 12 : 2, hemm_plane_count = x6 ? 18 : 8;
  auto take_planes = [&](size_t count) {  // count planes of d x d bf16
    w.planes = take(count * D * sizeof(uint16_t));
    w.has_planes = true;
  };
  auto take_sk = [&]() {
    w.sk = take(sk_bytes);
    w.has_sk = true;
  };
  switch (op) {
    case QST_OP_STATE_MAP:
      w.partials = take(size_t(kReduceBlocks) * 4 * sizeof(double));
      if (planes) take_planes(herk_planes);
      if (sk) take_sk();
      break;
    case QST_OP_NLL:
      w.partials = take(size_t(kReduceBlocks) * 4 * sizeof(double));
      break;
    case QST_OP_POVM_PROBS:
      if (pl.passes >= 2) w.inter0 = take(D * cb);
      if (pl.passes >= 3) w.inter1 = take(D * cb);
      break;
    case QST_OP_NLL_BACKWARD:
      w.partials = take(size_t(kReduceBlocks) * 4 * sizeof(double));
      w.scalars = take(8 * sizeof(double));
      if (pl.passes >= 2) w.inter0 = take(D * cb);
      if (pl.passes >= 3) w.inter1 = take(D * cb);
      w.gmat = take(D * cb);
      if (recompute) {
        w.rho = w.gmat;  // rho is dead once p exists; G' reuses its storage
        w.p = take(D * rb);
      }
      if (hemm_planes)
        take_planes(hemm_plane_count);  // also holds T's planes of the recomputed state map
      else if (recompute && planes)
        take_planes(herk_planes);
      if (sk && (recompute || !x6)) take_sk();
      break;
    case QST_OP_LIKELIHOOD: {
      const bool fused = fused_likelihood(pl, prec);
      w.partials = take(size_t(kReduceBlocks) * 4 * sizeof(double));
      if (fused) w.fpart = take(size_t(povm_pass_blocks(pl, pl.passes - 1)) * 4 * sizeof(double));
      w.rho = take(D * cb);
      if (pl.passes >= 2) w.inter0 = take(D * cb);
      if (pl.passes >= 3) w.inter1 = take(D * cb);
      if (!fused) w.p = take(D * rb);
      if (planes) take_planes(herk_planes);
      if (sk) take_sk();
      break;
    }
    case QST_OP_GRAD_PRODUCT:
      if (hemm_planes) take_planes(hemm_plane_count);
      if (sk && !x6) take_sk();
      break;
    case QST_OP_FIDELITY:
      off = fidelity_layout(n).total;
      break;
    case QST_OP_FNN:
      off = fnn_layout(n, rb).total;
      break;
    case QST_OP_ABS_MAP:
      off = absmap_layout(n).total;
      break;
    case QST_OP_LIKELIHOOD_GRAD: {
      // the likelihood's layout (same offsets), then G' for the routes that
      // form it, and the planes of the gradient product (QST_F32X6: G''s
      // then T^T's; BF16 path from d = 1024: split planes of G' and T^T);
      // the likelihood's partial tiles serve the gradient product too
      w = workspace_layout(n, prec, QST_OP_LIKELIHOOD, false);
      off = w.total;
      w.gmat = take(D * cb);
      if (hemm_planes) {
        w.tplanes = take(x6 ? x6_hemm_plane_bytes(n) : hemm_plane_count * D * sizeof(uint16_t));
        w.has_tplanes = true;
      }
      break;
    }
    default:
      return WsLayout{};
  }
  w.total = off;
  return w;
}

qst_status check_common(int n, int prec, std::string& msg) {
  if (n < 1 || n > QST_MAX_QUBITS) {
    msg = "n_qubits=" + std::to_string(n) + " outside [1, " + std::to_string(QST_MAX_QUBITS) + "]";
    return QST_ERR_INVALID_ARG;
  }
  if (!prec_valid(prec)) {
    msg = "unknown precision " + std::to_string(prec);
    return QST_ERR_INVALID_ARG;
  }
  return QST_OK;
}

qst_status check_ptr(const void* ptr, const char* name, std::string& msg) {
  if (!ptr) {
    msg = std::string(name) + " is NULL";
    return QST_ERR_INVALID_ARG;
  }
  return QST_OK;
}

qst_status check_matrix(const void* ptr, int64_t ld, int n, const char* name, std::string& msg) {
  if (check_ptr(ptr, name, msg) != QST_OK) return QST_ERR_INVALID_ARG;
  const int64_t d = int64_t(1) << n;
  if (ld < d) {
    msg = std::string("leading dimension of ") + name + " (" + std::to_string(ld) +
          ") is smaller than d=" + std::to_string(d);
    return QST_ERR_INVALID_ARG;
  }
  return QST_OK;
}

qst_status check_ws(const void* ws, size_t ws_bytes, size_t need, std::string& msg) {
  if (need == 0) return QST_OK;
  if (!ws || ws_bytes < need) {
    msg = "workspace of " + std::to_string(ws ? ws_bytes : 0) + " bytes is smaller than the " +
          std::to_string(need) + " bytes required";
    return QST_ERR_WORKSPACE;
  }
  return QST_OK;
}

qst_status check_povm(const double* M, std::string& msg) {
  if (!M) return QST_OK;
  double sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int a = 0; a < 4; ++a) {
    for (int x = 0; x < 2; ++x) {
      for (int y = 0; y < 2; ++y) {
        const double re = M[8 * a + 4 * x + 2 * y], im = M[8 * a + 4 * x + 2 * y + 1];
        const double tre = M[8 * a + 4 * y + 2 * x], tim = M[8 * a + 4 * y + 2 * x + 1];
        if (!std::isfinite(re) || !std::isfinite(im)) {
          msg = "POVM entry is not finite";
          return QST_ERR_INVALID_ARG;
        }
        if (std::fabs(re - tre) > 1e-12 || std::fabs(im + tim) > 1e-12) {
          msg = "POVM element M_" + std::to_string(a) + " is not Hermitian";
          return QST_ERR_INVALID_ARG;
        }
        sum[4 * x + 2 * y] += re;
        sum[4 * x + 2 * y + 1] += im;
      }
    }
  }
  const double eye[8] = {1, 0, 0, 0, 0, 0, 1, 0};
  for (int i = 0; i < 8; ++i) {
    if (std::fabs(sum[i] - eye[i]) > 1e-12) {
      msg = "POVM elements do not sum to the identity";
      return QST_ERR_INVALID_ARG;
    }
  }
  return QST_OK;
}

qst_status check_abs_order(double P, std::string& msg) {
  if (!std::isfinite(P) || P < 0.0) {
    msg = "absolute-map order P=" + std::to_string(P) + " is not a finite number >= 0";
    return QST_ERR_INVALID_ARG;
  }
  return QST_OK;
}

qst_status check_premap(int mode, const void* X, int64_t ldX, const void* Y, int64_t ldY, std::string& msg) {
  if (mode != QST_PREMAP_HERMITIAN && mode != QST_PREMAP_LOWER) {
    msg = "unknown pre-map mode " + std::to_string(mode);
    return QST_ERR_INVALID_ARG;
  }
  if (X == Y && ldX != ldY) {
    msg = "in place (Y == X) needs ldY == ldX";
    return QST_ERR_INVALID_ARG;
  }
  return QST_OK;
}

void povm_mode_matrices(const double* M, double W[32], double V[32]) {
  // Tetrahedral POVM of Sec. 4.1: M_a = (I + s_a . sigma)/4, s_a = (+-1,+-1,+-1)/sqrt(3).
  double tet[32];
  if (!M) {
    const double t = 1.0 / std::sqrt(3.0);
    const double s[4][3] = {{t, t, t}, {-t, -t, t}, {-t, t, -t}, {t, -t, -t}};
    for (int a = 0; a < 4; ++a) {
      const double sx = s[a][0], sy = s[a][1], sz = s[a][2];
      double* m = tet + 8 * a;
      m[0] = (1 + sz) / 4; m[1] = 0;         // [0][0]
      m[2] = sx / 4;       m[3] = -sy / 4;   // [0][1]
      m[4] = sx / 4;       m[5] = sy / 4;    // [1][0]
      m[6] = (1 - sz) / 4; m[7] = 0;         // [1][1]
    }
    M = tet;
  }
  for (int a = 0; a < 4; ++a) {
    for (int r = 0; r < 2; ++r) {
      for (int c = 0; c < 2; ++c) {
        const int m = 2 * r + c;
        // W[a][m] = M_a[c][r]
        W[2 * (4 * a + m)] = M[8 * a + 4 * c + 2 * r];
        W[2 * (4 * a + m) + 1] = M[8 * a + 4 * c + 2 * r + 1];
        // V[m][a] = M_a[r][c]
        V[2 * (4 * m + a)] = M[8 * a + 4 * r + 2 * c];
        V[2 * (4 * m + a) + 1] = M[8 * a + 4 * r + 2 * c + 1];
      }
    }
  }
}

int64_t general_outcomes(int n, int K) {
  int64_t D = 1;
  for (int i = 0; i < n; ++i) {
    D *= K;
    if (D > kGeneralMaxOutcomes) return -1;
  }
  return D;
}

qst_status check_povm_general(int n, int K, int settings, const double* M, std::string& msg) {
  if (K < 2 || K > kGeneralMaxK) {
    msg = "K=" + std::to_string(K) + " outside [2, " + std::to_string(kGeneralMaxK) + "]";
    return QST_ERR_INVALID_ARG;
  }
  if (settings < 1 || settings > kGeneralMaxSettings) {
    msg = "settings=" + std::to_string(settings) + " outside [1, " + std::to_string(kGeneralMaxSettings) + "]";
    return QST_ERR_INVALID_ARG;
  }
  if (general_outcomes(n, K) < 0) {
    msg = "K^N = " + std::to_string(K) + "^" + std::to_string(n) + " exceeds 2^30 outcomes";
    return QST_ERR_UNSUPPORTED;
  }
  if (!M) {
    msg = "povm_host is NULL";
    return QST_ERR_INVALID_ARG;
  }
  for (int s = 0; s < settings; ++s) {
    for (int i = 0; i < n; ++i) {
      const double* P = M + (int64_t(s) * n + i) * K * 8;
      double sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      const std::string where = "setting " + std::to_string(s) + ", qubit " + std::to_string(i + 1);
      for (int k = 0; k < K; ++k) {
        const double* m = P + 8 * k;  // [0][0], [0][1], [1][0], [1][1] as (re, im)
        for (int j = 0; j < 8; ++j) {
          if (!std::isfinite(m[j])) {
            msg = where + ": POVM entry is not finite";
            return QST_ERR_INVALID_ARG;
          }
          sum[j] += m[j];
        }
        if (std::fabs(m[1]) > 1e-12 || std::fabs(m[7]) > 1e-12 || std::fabs(m[2] - m[4]) > 1e-12 ||
            std::fabs(m[3] + m[5]) > 1e-12) {
          msg = where + ": element " + std::to_string(k) + " is not Hermitian";
          return QST_ERR_INVALID_ARG;
        }
        // smallest eigenvalue of [[a, b], [conj b, c]]
        const double a = m[0], c = m[6], h = 0.5 * (a - c);
        const double lmin = 0.5 * (a + c) - std::sqrt(h * h + m[2] * m[2] + m[3] * m[3]);
        if (lmin < -1e-12) {
          msg = where + ": element " + std::to_string(k) + " is not positive semidefinite";
          return QST_ERR_INVALID_ARG;
        }
      }
      const double eye[8] = {1, 0, 0, 0, 0, 0, 1, 0};
      for (int j = 0; j < 8; ++j) {
        if (std::fabs(sum[j] - eye[j]) > 1e-12) {
          msg = where + ": POVM elements do not sum to the identity";
          return QST_ERR_INVALID_ARG;
        }
      }
    }
  }
  return QST_OK;
}

void general_factors(int n, int K, int settings, const double* M, double* C) {
  for (int s = 0; s < settings; ++s)
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < K; ++k) {
        const double* m = M + ((int64_t(s) * n + i) * K + k) * 8;
        double* c = C + ((int64_t(s) * n + i) * K + k) * 4;
        // Tr(M I), Tr(M X) = 2 Re M01, Tr(M Y) = -2 Im M01, Tr(M Z), halved
        // (M Hermitian: M10 = conj M01)
        c[0] = 0.5 * (m[0] + m[6]);
        c[1] = m[2];
        c[2] = -m[3];
        c[3] = 0.5 * (m[0] - m[6]);
      }
}

void pauli_mode_matrices(double W[32], double V[32]) {
  // I, X, Y = [[0, -i], [i, 0]], Z as K = 4 matrices in the povm_host layout
  const double P[32] = {1, 0, 0, 0, 0, 0, 1, 0,    // I
                        0, 0, 1, 0, 1, 0, 0, 0,    // X
                        0, 0, 0, -1, 0, 1, 0, 0,   // Y
                        1, 0, 0, 0, 0, 0, -1, 0};  // Z
  povm_mode_matrices(P, W, V);
}

GeneralLayout general_layout(int n, qst_prec prec, int K, bool with_state) {
  GeneralLayout w;
  const size_t cb = complex_bytes(prec), rb = real_bytes(prec);
  const size_t d = size_t(1) << n, D = d * d;
  const int64_t DK = general_outcomes(n, K);
  const size_t M = DK < 0 ? D : std::max(D, size_t(DK));  // largest mixed tensor of the real passes
  const PovmPlan pl = make_povm_plan(n, prec);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  w.partials = take(size_t(kReduceBlocks) * 4 * sizeof(double));
  w.scal = take(size_t(4 * kGeneralMaxSettings + 8) * sizeof(double));
  if (pl.passes >= 2) w.inter0 = take(D * cb);
  if (pl.passes >= 3) w.inter1 = take(D * cb);
  w.e = take(D * rb);
  w.bufA = take(M * rb);
  w.bufB = take(M * rb);
  if (with_state) {
    w.h = take(D * rb);
    w.p = take((DK < 0 ? 0 : size_t(DK)) * rb);
    w.rho = take(D * cb);
    if (use_x6(prec, n)) {
      w.planes = take(x6_herk_plane_bytes(n));
      w.has_planes = true;
      w.sk = take(x6_partial_bytes(n));
      w.has_sk = true;
    } else {
      if (prec == QST_BF16GEMM && d > size_t(kBf16SplitMaxDim)) {
        w.planes = take(2 * D * sizeof(uint16_t));
        w.has_planes = true;
      }
      if (n >= kStreamKMinQubits) {
        w.sk = take(stream_k_partial_bytes(prec));
        w.has_sk = true;
      }
    }
  }
  w.total = off;
  return w;
}

}  // namespace qst

extern "C" {

size_t qst_workspace_bytes_general(int n_qubits, qst_prec prec, int K, int op) {
  std::string msg;
  if (qst::check_common(n_qubits, prec, msg) != QST_OK) return 0;
  if (K < 2 || K > qst::kGeneralMaxK || qst::general_outcomes(n_qubits, K) < 0) return 0;
  if (op != QST_OP_POVM_PROBS && op != QST_OP_LIKELIHOOD) return 0;
  return qst::general_layout(n_qubits, prec, K, op == QST_OP_LIKELIHOOD).total;
}

size_t qst_workspace_bytes(int n_qubits, qst_prec prec, int op) {
  std::string msg;
  if (qst::check_common(n_qubits, prec, msg) != QST_OK) return 0;
  if (op < QST_OP_STATE_MAP || op > QST_OP_LIKELIHOOD_GRAD) return 0;
  return qst::workspace_layout(n_qubits, prec, op, /*recompute=*/true).total;
}

const char* qst_status_string(qst_status s) {
  switch (s) {
    case QST_OK: return "QST_OK";
    case QST_ERR_INVALID_ARG: return "QST_ERR_INVALID_ARG";
    case QST_ERR_UNSUPPORTED: return "QST_ERR_UNSUPPORTED";
    case QST_ERR_WORKSPACE: return "QST_ERR_WORKSPACE";
    case QST_ERR_HIP: return "QST_ERR_HIP";
  }
  return "QST_ERR_UNKNOWN";
}

const char* qst_last_error(void) { return qst::last_error_cstr(); }

const char* qst_version(void) { return "qst-mi355x 0.1 (gfx950)"; }

}  // extern "C"
