// General product POVMs: K outcomes per qubit, a K-element POVM of its own
// on each qubit (Sec. 3.3), and several such settings whose negative
// log-likelihoods add (Sec. 2.1: one POVM {M^i_k} per measurement i).
//
// Route through the Pauli coordinates.  Every 2 x 2 Hermitian M is
// M = sum_b C[b] P_b over the Pauli basis P = (I, X, Y, Z) with real
// C[b] = Tr(M P_b) / 2, so for a product POVM
//   p_k = Tr((M^(1)_k1 (x) ... (x) M^(N)_kN) rho) = sum_b prod_i C^(i)[k_i][b_i] e_b,
//   e_b = Tr((P_b1 (x) ... (x) P_bN) rho)   (4^N real Pauli coordinates),
// i.e. p = (C^(1) (x) ... (x) C^(N)) e.  e comes from the product-POVM
// passes run with the Pauli matrices in place of POVM elements (the passes
// take any Hermitian four-element set; only the lower triangle of rho is
// read), and the real K x 4 factors are applied one qubit per launch by
// real_factor_pass.  The adjoint applies the transposed factors (the
// cotangent F_s - f_k / p_k formed on the fly in the first of them, the
// settings' results summed into one 4^N vector h in the last) and then the
// Pauli synthesis G' = sum_b h_b P_b with the adjoint passes.
//
// Tensor layout of a real pass over qubit j: [A][m][B] with A = 4^(j-1)
// (qubits 1..j-1 still in Pauli coordinates), m the qubit's index (4 Pauli
// coordinates or K outcomes) and B = K^(N-j) (qubits j+1..N finished); the
// flat outcome index is k = sum_i k_i K^(N-i), qubit N least significant.
#include <vector>

#include "qst_device.h"
#include "qst_kernels.h"
#include "qst_plan.h"

namespace qst {

namespace {

struct RealFactor {
  double c[kGeneralMaxK][4];  // C[k][b]
};

// MODE 0: forward, [A][4][B] -> [A][K][B], out = C x.
// MODE 1: adjoint, [A][K][B] -> [A][4][B], out (+)= C^T x.
// MODE 2: adjoint whose input is the cotangent F_s - f_k / p_k of the
//         setting's p (in) and f.
template <typename R, int K, int MODE>
__global__ __launch_bounds__(256) void real_factor_pass(const R* __restrict__ in, R* __restrict__ out, int64_t A,
                                                        int64_t B, RealFactor C, const R* __restrict__ f,
                                                        const double* __restrict__ Fs, int accumulate) {
  constexpr int MI = MODE == 0 ? 4 : K, MO = MODE == 0 ? K : 4;
  R c[K][4];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int b = 0; b < 4; ++b) c[k][b] = R(C.c[k][b]);
  double F = 0.0;
  if constexpr (MODE == 2) F = *Fs;
  const int64_t total = A * B;
  for (int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x; t < total; t += int64_t(gridDim.x) * 256) {
    const int64_t a = t / B, b = t - a * B;
    const int64_t ib = a * MI * B + b, ob = a * MO * B + b;
    R x[MI];
#pragma unroll
    for (int m = 0; m < MI; ++m) {
      if constexpr (MODE == 2) x[m] = cotangent(F, f[ib + m * B], in[ib + m * B]);
      else x[m] = in[ib + m * B];
    }
#pragma unroll
    for (int o = 0; o < MO; ++o) {
      R y = R(0);
#pragma unroll
      for (int m = 0; m < MI; ++m) y += (MODE == 0 ? c[o][m] : c[m][o]) * x[m];
      if (accumulate) y += out[ob + o * B];
      out[ob + o * B] = y;
    }
  }
}

template <typename R, int K>
void launch_factor_k(int mode, const R* in, R* out, int64_t A, int64_t B, const RealFactor& C, const R* f,
                     const double* Fs, int accumulate, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((A * B + 255) / 256, 8192);
  const dim3 grid{unsigned(blocks)}, block{256};
  if (mode == 0) real_factor_pass<R, K, 0><<<grid, block, 0, s>>>(in, out, A, B, C, f, Fs, accumulate);
  else if (mode == 1) real_factor_pass<R, K, 1><<<grid, block, 0, s>>>(in, out, A, B, C, f, Fs, accumulate);
  else real_factor_pass<R, K, 2><<<grid, block, 0, s>>>(in, out, A, B, C, f, Fs, accumulate);
}

template <typename R>
hipError_t launch_factor(int K, int mode, const void* in, void* out, int64_t A, int64_t B, const RealFactor& C,
                         const void* f, const double* Fs, int accumulate, hipStream_t s) {
  ProfScope prof("general_factor_pass", s);
  const R* i = static_cast<const R*>(in);
  R* o = static_cast<R*>(out);
  const R* fr = static_cast<const R*>(f);
  switch (K) {
    case 2: launch_factor_k<R, 2>(mode, i, o, A, B, C, fr, Fs, accumulate, s); break;
    case 3: launch_factor_k<R, 3>(mode, i, o, A, B, C, fr, Fs, accumulate, s); break;
    case 4: launch_factor_k<R, 4>(mode, i, o, A, B, C, fr, Fs, accumulate, s); break;
    case 5: launch_factor_k<R, 5>(mode, i, o, A, B, C, fr, Fs, accumulate, s); break;
    case 6: launch_factor_k<R, 6>(mode, i, o, A, B, C, fr, Fs, accumulate, s); break;
    case 7: launch_factor_k<R, 7>(mode, i, o, A, B, C, fr, Fs, accumulate, s); break;
    case 8: launch_factor_k<R, 8>(mode, i, o, A, B, C, fr, Fs, accumulate, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

RealFactor factor_of(const double* C, int K) {
  RealFactor r{};
  for (int k = 0; k < K; ++k)
    for (int b = 0; b < 4; ++b) r.c[k][b] = C[4 * k + b];
  return r;
}

int64_t ipow(int64_t x, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

// Stage 2 of one setting's NLL: scal[0..3] = (L_s, F_s, bad0_s, bad1_s)
// from the [4][nb] partials, in a fixed order.
__global__ __launch_bounds__(256) void setting_sums_kernel(const double* __restrict__ part, int nb,
                                                           double* __restrict__ scal) {
  __shared__ double red[4];
  for (int i = 0; i < 4; ++i) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) acc += part[int64_t(i) * nb + b];
    const double v = block_sum256(acc, red);
    if (threadIdx.x == 0) scal[i] = v;
  }
}

// Totals over the settings, in setting order: nll = (L, F) with L = +inf
// after a term f_k > 0 with p_k <= 0 and NaN after a NaN, and the counters.
__global__ void settings_total_kernel(const double* __restrict__ scal, int settings, double* __restrict__ nll,
                                      unsigned long long* __restrict__ bad) {
  if (threadIdx.x != 0) return;
  double L = 0.0, F = 0.0, b0 = 0.0, b1 = 0.0;
  for (int s = 0; s < settings; ++s) {
    L += scal[4 * s];
    F += scal[4 * s + 1];
    b0 += scal[4 * s + 2];
    b1 += scal[4 * s + 3];
  }
  if (F != F || b1 > 0.0) L = __builtin_nan("");
  else if (b0 > 0.0) L = __builtin_inf();
  nll[0] = L;
  nll[1] = F;
  if (bad) {
    bad[0] = (unsigned long long)b0;
    bad[1] = (unsigned long long)b1;
  }
}

// p of one setting from the Pauli coordinates e: the forward factors of
// qubits N, N-1, .., 1 (ping-pong through bufA / bufB), last one into p.
template <typename R>
hipError_t forward_factors(int n, int K, const double* C, const void* e, void* p, void* bufA, void* bufB,
                           hipStream_t s) {
  void* bufs[2] = {bufA, bufB};
  for (int m = 0; m < n; ++m) {
    const int j = n - m;  // qubit
    const void* in = m == 0 ? e : bufs[(m - 1) & 1];
    void* out = m == n - 1 ? p : bufs[m & 1];
    const hipError_t err = launch_factor<R>(K, 0, in, out, ipow(4, j - 1), ipow(K, n - j),
                                            factor_of(C + int64_t(j - 1) * K * 4, K), nullptr, nullptr, 0, s);
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

// h (+)= the transposed factors of qubits 1..N applied to the cotangent
// F_s - f/p of one setting.
template <typename R>
hipError_t adjoint_factors(int n, int K, const double* C, const void* p, const void* f, const double* Fs, void* h,
                           bool accumulate, void* bufA, void* bufB, hipStream_t s) {
  void* bufs[2] = {bufA, bufB};
  for (int m = 0; m < n; ++m) {
    const int j = m + 1;  // qubit
    const void* in = m == 0 ? p : bufs[(m - 1) & 1];
    void* out = m == n - 1 ? h : bufs[m & 1];
    const hipError_t err =
        launch_factor<R>(K, m == 0 ? 2 : 1, in, out, ipow(4, j - 1), ipow(K, n - j),
                         factor_of(C + int64_t(j - 1) * K * 4, K), m == 0 ? f : nullptr, Fs,
                         (m == n - 1 && accumulate) ? 1 : 0, s);
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_general_probs(qst_prec prec, int n, int K, const double* C, const void* rho, int64_t ld_rho,
                                void* p, const GeneralBufs& b, hipStream_t s) {
  double W[32], V[32];
  pauli_mode_matrices(W, V);
  const PovmPlan pl = make_povm_plan(n, prec);
  ProfScope prof("povm_general", s);
  hipError_t e = launch_povm(false, prec, pl, W, false, rho, ld_rho, b.e, nullptr, nullptr, b.inter0, b.inter1, s);
  if (e != hipSuccess) return e;
  return prec == QST_F64 ? forward_factors<double>(n, K, C, b.e, p, b.bufA, b.bufB, s)
                         : forward_factors<float>(n, K, C, b.e, p, b.bufA, b.bufB, s);
}

hipError_t launch_general_likelihood(qst_prec prec, int n, int K, int settings, const double* C, const void* rho,
                                     int64_t ld_rho, const void* f, void* G, int64_t ldG, double* nll_dev,
                                     unsigned long long* bad_dev, const GeneralBufs& b, hipStream_t s) {
  double W[32], V[32];
  pauli_mode_matrices(W, V);
  const PovmPlan pl = make_povm_plan(n, prec);
  const int64_t DK = ipow(K, n);
  const size_t rb = real_bytes(prec);
  ProfScope prof("likelihood_general", s);
  hipError_t e = launch_povm(false, prec, pl, W, false, rho, ld_rho, b.e, nullptr, nullptr, b.inter0, b.inter1, s);
  if (e != hipSuccess) return e;
  for (int st = 0; st < settings; ++st) {
    const double* Cs = C + int64_t(st) * n * K * 4;
    const void* fs = static_cast<const unsigned char*>(f) + size_t(st) * size_t(DK) * rb;
    double* sc = b.scal + 4 * st;
    e = prec == QST_F64 ? forward_factors<double>(n, K, Cs, b.e, b.p, b.bufA, b.bufB, s)
                        : forward_factors<float>(n, K, Cs, b.e, b.p, b.bufA, b.bufB, s);
    if (e != hipSuccess) return e;
    if ((e = launch_nll_partials(prec, b.p, fs, DK, b.partials, s)) != hipSuccess) return e;
    setting_sums_kernel<<<1, 256, 0, s>>>(b.partials, kReduceBlocks, sc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!G) continue;
    e = prec == QST_F64 ? adjoint_factors<double>(n, K, Cs, b.p, fs, sc + 1, b.h, st > 0, b.bufA, b.bufB, s)
                        : adjoint_factors<float>(n, K, Cs, b.p, fs, sc + 1, b.h, st > 0, b.bufA, b.bufB, s);
    if (e != hipSuccess) return e;
  }
  settings_total_kernel<<<1, 64, 0, s>>>(b.scal, settings, nll_dev, bad_dev);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (!G) return hipSuccess;
  // G' = sum_b h_b P_b: the adjoint passes with the Pauli set, fed h as is
  return launch_povm(true, prec, pl, V, false, G, ldG, nullptr, b.h, nullptr, b.inter0, b.inter1, s);
}

}  // namespace qst
