// Product-POVM map p_k = Tr(rho M_k), M_k = M_{k_1} (x) ... (x) M_{k_N}
// (Born rule, Sec. 2.1; product structure, Sec. 3.3) and its adjoint
// G = sum_k g_k M_k, as a sequence of passes of per-qubit 4 x 4 mode
// contractions.
//
// Data view.  A d x d matrix X is a tensor over per-qubit pair indices
// m_i = 2 r_i + c_i (r_i, c_i the row/column bits of qubit i; qubit 1 is the
// most significant bit).  For one qubit, Tr(M_a X) = sum_m W[a][m] X_m with
// W[a][2r+c] = (M_a)_{c,r}; the full map applies W along every qubit axis,
// and the adjoint applies V[m][a] = (M_a)_{r,c}.  Each pass loads, for one
// workgroup, all 4^g pair values of a group of g qubits (for J consecutive
// values of the already-contracted outcome digits) into LDS, contracts the g
// axes in place, and writes the result; see qst_plan.h for the pass plan.
//
// Hermitian symmetry.  rho, every forward intermediate and every adjoint
// intermediate are Hermitian in the not-yet-contracted (row, column) bits,
// so only entries with row >= column are ever read or written; the others
// are the conjugates.  The forward map therefore reads only the lower
// triangle of rho.
//
// For the paper's tetrahedral POVM (Sec. 4.1), M_a = (I + s_a.sigma)/4 with
// s_a = (+-1, +-1, +-1)/sqrt(3), the 4 x 4 contraction factors as
// (1/4) H diag(1, t, t, t) U with U x = (x0+x3, x1+x2, i(x1-x2), x0-x3),
// H a 4 x 4 Hadamard matrix and t = 1/sqrt(3); the kernels use that form
// (8 complex adds and 3 real-scalar products per 4 values) instead of a
// generic complex 4 x 4 product.
#include "qst_device.h"
#include "qst_kernels.h"
#include "qst_povm_generic.h"
#include "qst_povm_ops.h"

namespace qst {

namespace {

template <typename R, bool TETRA, bool MATSIDE, bool PSIDE>
__global__ __launch_bounds__(256) void povm_fwd_pass(PassArgs a, ModeMatrix A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  generic_pass::fwd_pass_body<R, TETRA, MATSIDE, PSIDE>(a, A, blockIdx.x, reinterpret_cast<Cx<R>*>(smem_raw));
}

template <typename R, bool TETRA, bool MATSIDE, bool PSIDE>
__global__ __launch_bounds__(256) void povm_adj_pass(PassArgs a, ModeMatrix A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  generic_pass::adj_pass_body<R, TETRA, MATSIDE, PSIDE>(a, A, blockIdx.x, reinterpret_cast<Cx<R>*>(smem_raw));
}

template <typename R, bool ADJ, bool TETRA>
hipError_t launch_pass_t(const PassArgs& a, const ModeMatrix& A, bool matside, bool pside,
                         int64_t blocks, hipStream_t s) {
  const size_t lds = (size_t(1) << (2 * a.g)) * size_t(a.J) * sizeof(Cx<R>);
  const dim3 grid{unsigned(blocks), 1, 1}, block{256, 1, 1};
#define QST_POVM_LAUNCH(M, P)                                                              \
  do {                                                                                     \
    if constexpr (ADJ) povm_adj_pass<R, TETRA, M, P><<<grid, block, lds, s>>>(a, A);        \
    else povm_fwd_pass<R, TETRA, M, P><<<grid, block, lds, s>>>(a, A);                      \
  } while (0)
  if (matside && pside) QST_POVM_LAUNCH(true, true);
  else if (matside) QST_POVM_LAUNCH(true, false);
  else if (pside) QST_POVM_LAUNCH(false, true);
  else QST_POVM_LAUNCH(false, false);
#undef QST_POVM_LAUNCH
  return hipGetLastError();
}

}  // namespace

hipError_t launch_povm(bool adjoint, qst_prec prec, const PovmPlan& pl, const double* mode_matrix,
                       bool tetra, const void* mat, int64_t ld, void* pvec, const void* fvec,
                       const double* F_dev, void* inter0, void* inter1, hipStream_t s, bool use_fast) {
  ModeMatrix A;
  for (int i = 0; i < 32; ++i) A.a[i] = mode_matrix[i];
  void* bufs[2] = {inter0, inter1};
  const int P = pl.passes;
  for (int step = 0; step < P; ++step) {
    const int j = adjoint ? (P - 1 - step) : step;
    PassArgs a{};
    a.n = pl.n;
    a.U = pl.U[j];
    a.g = pl.g[j];
    a.J = pl.J[j];
    a.ld = ld;
    const bool matside = (j == 0), pside = (j == P - 1);
    if (!adjoint) {
      a.in = matside ? mat : bufs[(j - 1) & 1];
      a.out = pside ? pvec : bufs[j & 1];
    } else {
      a.in = pside ? nullptr : bufs[j & 1];
      a.out = matside ? const_cast<void*>(mat) : bufs[(j - 1) & 1];
      a.p = pvec;
      a.f = fvec;
      a.F = F_dev;
    }
    const int64_t blocks = povm_pass_blocks(pl, j);
    static const char* kNames[2][4] = {{"povm_fwd_p0", "povm_fwd_p1", "povm_fwd_p2", "povm_fwd_p3"},
                                       {"povm_adj_p0", "povm_adj_p1", "povm_adj_p2", "povm_adj_p3"}};
    ProfScope prof(kNames[adjoint ? 1 : 0][j], s);
    hipError_t e;
    if (use_fast && launch_pass_fast(adjoint, prec, tetra, a, A, matside, pside, blocks, s, &e)) {
      if (e != hipSuccess) return e;
      continue;
    }
    if (prec == QST_F64) {
      if (adjoint) e = tetra ? launch_pass_t<double, true, true>(a, A, matside, pside, blocks, s)
                             : launch_pass_t<double, true, false>(a, A, matside, pside, blocks, s);
      else e = tetra ? launch_pass_t<double, false, true>(a, A, matside, pside, blocks, s)
                     : launch_pass_t<double, false, false>(a, A, matside, pside, blocks, s);
    } else {
      if (adjoint) e = tetra ? launch_pass_t<float, true, true>(a, A, matside, pside, blocks, s)
                             : launch_pass_t<float, true, false>(a, A, matside, pside, blocks, s);
      else e = tetra ? launch_pass_t<float, false, true>(a, A, matside, pside, blocks, s)
                     : launch_pass_t<float, false, false>(a, A, matside, pside, blocks, s);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_povm_fused(qst_prec prec, const PovmPlan& pl, const double* W, const double* V, bool tetra,
                             const void* rho, int64_t ld_rho, const void* fvec, const double* Fpart, void* G,
                             int64_t ldG, void* inter0, void* inter1, double* part, double* nll_dev,
                             unsigned long long* bad_dev, bool pass0_done, hipStream_t s, const void* pt,
                             double* fc_dev, void* gplanes) {
  static const char* kFwd[4] = {"povm_fwd_p0", "povm_fwd_p1", "povm_fwd_p2", "povm_fwd_p3"};
  static const char* kAdj[4] = {"povm_adj_p0", "povm_adj_p1", "povm_adj_p2", "povm_adj_p3"};
  ModeMatrix Af, Aa;
  for (int i = 0; i < 32; ++i) {
    Af.a[i] = W[i];
    Aa.a[i] = V[i];
  }
  void* bufs[2] = {inter0, inter1};
  const int P = pl.passes;
  auto args = [&](int j) {
    PassArgs a{};
    a.n = pl.n;
    a.U = pl.U[j];
    a.g = pl.g[j];
    a.J = pl.J[j];
    return a;
  };
  hipError_t e = hipSuccess;
  for (int j = pass0_done ? 1 : 0; j + 1 < P; ++j) {
    PassArgs a = args(j);
    a.in = j == 0 ? rho : bufs[(j - 1) & 1];
    a.out = bufs[j & 1];
    a.ld = ld_rho;
    ProfScope prof(kFwd[j], s);
    if (!launch_pass_fast(false, prec, tetra, a, Af, j == 0, false, povm_pass_blocks(pl, j), s, &e))
      return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
  }
  {
    PassArgs a = args(P - 1);
    a.in = a.out = bufs[(P - 2) & 1];
    a.f = fvec;
    a.Fpart = Fpart;
    a.part = part;
    a.pt = pt;
    const int64_t nb = povm_pass_blocks(pl, P - 1);
    ProfScope prof("povm_fused", s);
    if (!launch_fused_fast(prec, tetra, a, Af, Aa, nb, s, &e)) return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    if ((e = launch_likelihood_finish(part, int(nb), Fpart, nll_dev, bad_dev, s, pt ? fc_dev : nullptr)) != hipSuccess)
      return e;
  }
  if (!G && !gplanes) return hipSuccess;
  for (int j = P - 2; j >= 0; --j) {
    PassArgs a = args(j);
    a.in = bufs[j & 1];
    a.out = j == 0 ? G : bufs[(j - 1) & 1];
    a.ld = ldG;
    if (j == 0) a.gplanes = gplanes;
    ProfScope prof(kAdj[j], s);
    if (!launch_pass_fast(true, prec, tetra, a, Aa, j == 0, false, povm_pass_blocks(pl, j), s, &e))
      return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace qst
