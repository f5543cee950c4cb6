// The P-order absolute map of Sec. 3.2 (Eq. abs_P) and its adjoint.
//
// Forward: H = (T + T^dagger) / 2 in FP64, H = Q Lambda Q^dagger (by the
// direct solver of k_eigh.hip, or, from a warm start, by the cyclic
// two-sided Jacobi method below), and A = Q |Lambda|^(P/2) Q^dagger =
// U U^dagger with U = Q |Lambda|^(P/4) (one complex product on MFMA).  The
// likelihood path's state map of A, A A^dagger / Tr(A A^dagger) =
// Q |Lambda|^P Q^dagger / Tr |Lambda|^P, is then the P-order absolute
// projection.
//
// The general fidelity takes the eigenvalues of T^dagger rho T from the
// direct solver.
//
// Jacobi: the d indices are paired by the round-robin (circle) schedule, in
// which round t of d - 1 pairs every index once: pair 0 is (0, 1 + t) and
// pair k > 0 is (1 + (k + t) mod (d-1), 1 + (d-1-k+t) mod (d-1)).  All d/2
// rotations of a round are computed from the matrix before the round and
// applied together, A <- J^dagger A J with J block diagonal over the pairs:
// the workgroup of pair (p, q) rewrites rows p and q, each 2 x 2 block of
// them (columns (r, s) of another pair) as J_pq^dagger B J_rs, reading from
// one buffer and writing the other.  The rows of V^T (V the product of the
// rotations, Q at the end) are rotated in place.  The rotation of a pair
// zeroes its off-diagonal entry exactly: with c = |c| e^(i phi) the phase
// diag(1, e^(-i phi)) makes the 2 x 2 block real symmetric and the classical
// rotation angle (tangent t of the smaller root of t^2 + 2 zeta t - 1 = 0,
// zeta = (b - a) / (2 |c|)) diagonalises it.  After each sweep (d - 1
// rounds) a one-workgroup kernel sums the off-diagonal norm and decides on
// the device: the sweeps stop when it is below 1e-14 of ||H||_F (1e-10 for
// FP32 storage), or below 1e-10 of it and no longer falling by half (the
// rounding floor), which Jacobi's quadratic convergence reaches in a few
// sweeps.  The decision sets a flag in the workspace that every later round
// kernel reads first and returns on, so a fixed number of enqueued sweeps
// (the graph-capturable calls) costs one empty launch per skipped round;
// the synchronous calls read the flag on the host after each sweep and
// stop enqueuing.  d - 1 is odd, so the diagonalised matrix sits in the
// first ping-pong buffer after an even number of sweeps and in the second
// after an odd one; the state records which.
//
// Adjoint: for a spectral function A = g(H), g(l) = |l|^(P/2), the
// first-order change is Q (Gamma o (Q^dagger dH Q)) Q^dagger with Gamma the
// divided differences of g on the eigenvalues (g' on ties); both it and
// the Hermitian part are self-adjoint, so dL/dT = Q (Gamma o (Q^dagger S Q))
// Q^dagger with S = (dL/dA + dL/dA^dagger) / 2: four complex products.
//
// A warm start from the eigenvectors Q0 of a nearby matrix (the previous
// step of a training loop) runs the sweeps on Q0^dagger H Q0, nearly
// diagonal, with V starting at Q0: two more products, and the sweeps drop to
// the quadratically convergent tail.
//
// Everything runs in FP64 whatever the storage precision of T, A and the
// gradients: the eigensolver's rounding enters A through g, whose slope is
// unbounded near 0 for P < 2.
#include <hip/hip_runtime.h>

#include <cmath>

#include "qst_device.h"
#include "qst_kernels.h"

namespace qst {

namespace {

using C64 = Cx<double>;

constexpr int kTB = 32;          // tile side of the transposes

__device__ __forceinline__ C64 cmul(C64 a, C64 b) { return C64{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ C64 cscale(C64 a, double s) { return C64{a.re * s, a.im * s}; }
__device__ __forceinline__ C64 csub(C64 a, C64 b) { return C64{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ C64 cadd(C64 a, C64 b) { return C64{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ double cnorm(C64 a) { return a.re * a.re + a.im * a.im; }

// J = [[cs, sn], [-sn ph, cs ph]], ph = e^(-i phi); shift = t |c| (the
// diagonal becomes a - shift, b + shift).
struct Rot {
  double cs, sn;
  C64 ph;
  double shift;
};

__device__ __forceinline__ Rot make_rot(double a, double b, C64 c) {
  Rot r{1.0, 0.0, C64{1.0, 0.0}, 0.0};
  const double ac = hypot(c.re, c.im);
  if (ac == 0.0) return r;
  const double z = (b - a) / (2.0 * ac);
  const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
  r.cs = 1.0 / sqrt(1.0 + t * t);
  r.sn = r.cs * t;
  r.ph = C64{c.re / ac, -c.im / ac};
  r.shift = t * ac;
  return r;
}

__device__ __forceinline__ void pair_at(int k, int t, int m, int& p, int& q) {
  if (k == 0) {
    p = 0;
    q = 1 + t;
  } else {
    p = 1 + (k + t) % m;
    q = 1 + (m - k + t) % m;
  }
}

__device__ __forceinline__ Rot rot_of(const C64* A, int d, int p, int q) {
  return make_rot(A[int64_t(p) * d + p].re, A[int64_t(q) * d + q].re, A[int64_t(p) * d + q]);
}

// One round t: workgroup (k, c) rewrites the column pairs [128c, 128c + 128)
// of rows p, q of pair k (Ain -> Aout), one column pair per thread, and
// rotates columns [2 * 128c, 2 * 128c + 256) of rows p, q of Vt (every
// element of both is touched by exactly one workgroup of the round);
// part[2i], part[2i+1] (i = k * chunks + c) receive the squared off-diagonal
// and diagonal entries it wrote.
constexpr int kRoundThreads = 128;

// Device-side state of the sweeps (in the workspace).
struct JacobiState {
  int done;     // 1 once the stopping rule held (or the norm was not finite)
  int sweeps;   // sweeps taken when done, -1 if not converged or not finite
  int parity;   // buffer of the diagonalised matrix: 0 = first, 1 = second
  int pad;
  double prev;  // relative off-diagonal norm after the previous sweep
};

__global__ void jacobi_reset_kernel(JacobiState* st) {
  st->done = 0;
  st->sweeps = -1;
  st->parity = 0;
  st->prev = HUGE_VAL;
}

__global__ __launch_bounds__(kRoundThreads) void jacobi_round_kernel(const C64* __restrict__ Ain,
                                                                     C64* __restrict__ Aout, C64* __restrict__ Vt,
                                                                     int d, int t, double* __restrict__ part,
                                                                     const JacobiState* __restrict__ st) {
  if (st->done) return;  // converged in an earlier sweep: nothing to rotate
  __shared__ double red[2][kRoundThreads / 64];
  const int m = d - 1, half = d >> 1;
  const int k = blockIdx.x, c = blockIdx.y;
  int p, q;
  pair_at(k, t, m, p, q);
  const Rot J = rot_of(Ain, d, p, q);
  const C64 phc{J.ph.re, -J.ph.im};
  const C64* rp = Ain + int64_t(p) * d;
  const C64* rq = Ain + int64_t(q) * d;
  C64* wp = Aout + int64_t(p) * d;
  C64* wq = Aout + int64_t(q) * d;
  double off = 0.0, dia = 0.0;
  const int R = c * kRoundThreads + int(threadIdx.x);
  if (R < half) {
    int r, s;
    pair_at(R, t, m, r, s);
    if (R == k) {
      const double a = rp[p].re - J.shift, b = rq[q].re + J.shift;
      wp[p] = C64{a, 0.0};
      wq[q] = C64{b, 0.0};
      wp[q] = C64{0.0, 0.0};
      wq[p] = C64{0.0, 0.0};
      dia = a * a + b * b;
    } else {
      const Rot K = rot_of(Ain, d, r, s);
      const C64 xpr = rp[r], xps = rp[s], xqr = rq[r], xqs = rq[s];
      // right: [u, v] J_rs = [u cs - v sn ph, u sn + v cs ph]
      const C64 vp = cmul(xps, K.ph), vq = cmul(xqs, K.ph);
      const C64 ypr = csub(cscale(xpr, K.cs), cscale(vp, K.sn)), yps = cadd(cscale(xpr, K.sn), cscale(vp, K.cs));
      const C64 yqr = csub(cscale(xqr, K.cs), cscale(vq, K.sn)), yqs = cadd(cscale(xqr, K.sn), cscale(vq, K.cs));
      // left: J_pq^dagger = [[cs, -sn conj(ph)], [sn, cs conj(ph)]]
      const C64 ur = cmul(phc, yqr), us = cmul(phc, yqs);
      const C64 zpr = csub(cscale(ypr, J.cs), cscale(ur, J.sn)), zqr = cadd(cscale(ypr, J.sn), cscale(ur, J.cs));
      const C64 zps = csub(cscale(yps, J.cs), cscale(us, J.sn)), zqs = cadd(cscale(yps, J.sn), cscale(us, J.cs));
      wp[r] = zpr;
      wp[s] = zps;
      wq[r] = zqr;
      wq[s] = zqs;
      off = cnorm(zpr) + cnorm(zps) + cnorm(zqr) + cnorm(zqs);
    }
  }
  C64* vpr = Vt + int64_t(p) * d;
  C64* vqr = Vt + int64_t(q) * d;
  const int c0 = 2 * kRoundThreads * c, c1 = min(d, c0 + 2 * kRoundThreads);
  for (int col = c0 + int(threadIdx.x); col < c1; col += kRoundThreads) {
    const C64 u = vpr[col], v = cmul(vqr[col], J.ph);
    vpr[col] = csub(cscale(u, J.cs), cscale(v, J.sn));
    vqr[col] = cadd(cscale(u, J.sn), cscale(v, J.cs));
  }
  off = wave_sum(off);
  dia = wave_sum(dia);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = off;
    red[1][w] = dia;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int i = k * int(gridDim.y) + c;
    part[2 * i] = red[0][0] + red[0][1];
    part[2 * i + 1] = red[1][0] + red[1][1];
  }
}

// out[0] = sum of part[2i] (off-diagonal), out[1] = sum of part[2i+1] over
// the round's workgroups i, in a fixed order.
__global__ __launch_bounds__(256) void jacobi_norms_kernel(const double* __restrict__ part, int count,
                                                           double* __restrict__ out) {
  __shared__ double lds4[4];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < count; k += 256) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  a = block_sum256(a, lds4);
  b = block_sum256(b, lds4);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

// After sweep `sweep` (of at most max_sweeps): the off-diagonal and
// diagonal squared norms from the round partials (fixed order), and the
// stopping rule.  Nothing once done.
__global__ __launch_bounds__(256) void jacobi_check_kernel(const double* __restrict__ part, int count,
                                                           JacobiState* __restrict__ st, double tol, int sweep,
                                                           int max_sweeps) {
  if (st->done) return;
  __shared__ double lds4[4];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < count; k += 256) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  a = block_sum256(a, lds4);
  b = block_sum256(b, lds4);
  if (threadIdx.x != 0) return;
  const double off = a, tot = a + b;
  st->parity = sweep & 1;
  if (!isfinite(off) || !isfinite(tot)) {
    st->done = 1;
    st->sweeps = -1;
    return;
  }
  const double r = tot > 0.0 ? sqrt(off / tot) : 0.0;
  if (r <= tol || (r <= 1e-10 && r > 0.5 * st->prev)) {
    st->done = 1;
    st->sweeps = sweep;
  } else {
    st->prev = r;
    if (sweep >= max_sweeps) st->done = 1;  // sweeps stays -1: not converged
  }
}

__global__ void jacobi_sweeps_out_kernel(const JacobiState* __restrict__ st, int* __restrict__ out) {
  *out = st->sweeps;
}

__global__ void set_scalar_kernel(double* x, double v) { *x = v; }

// lam[i] = A[i][i] (real; A the diagonalised matrix, in A0 or A1 as the
// sweep state says), sc[i] = |lam[i]|^(P/4).
__global__ __launch_bounds__(256) void spectrum_kernel(const C64* __restrict__ A0, const C64* __restrict__ A1,
                                                       const JacobiState* __restrict__ st, int d, double P,
                                                       double* __restrict__ lam, double* __restrict__ sc) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= d) return;
  const C64* A = st->parity ? A1 : A0;
  const double l = A[int64_t(i) * d + i].re;
  lam[i] = l;
  sc[i] = pow(fabs(l), 0.25 * P);
}

// sc[i] = |lam[i]|^(P/4).
__global__ __launch_bounds__(256) void power_scale_kernel(const double* __restrict__ lam, int d, double P,
                                                          double* __restrict__ sc) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < d) sc[i] = pow(fabs(lam[i]), 0.25 * P);
}

// Y[i][j] = op(X[j][i]) * (scale ? scale[j] : 1), op = conj or identity;
// tiles B x B (B = min(d, 32)) staged through LDS.
__global__ __launch_bounds__(256) void transpose64_kernel(const C64* __restrict__ X, int64_t ldx,
                                                          C64* __restrict__ Y, int64_t ldy, int lgB, int conj,
                                                          const double* __restrict__ scale) {
  __shared__ C64 a[kTB][kTB + 1];
  const int B = 1 << lgB;
  const int I = blockIdx.x, Jt = blockIdx.y;  // Y tile (I, Jt) from X tile (Jt, I)
  const int64_t xr0 = int64_t(Jt) << lgB, xc0 = int64_t(I) << lgB;
  const int elems = B * B;
  for (int e = threadIdx.x; e < elems; e += 256) {
    const int r = e >> lgB, c = e & (B - 1);
    a[r][c] = X[(xr0 + r) * ldx + xc0 + c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < elems; e += 256) {
    const int r = e >> lgB, c = e & (B - 1);
    C64 v = a[c][r];  // X[xr0 + c][xc0 + r] = X[j][i] for i = xc0 + r, j = xr0 + c
    if (conj) v.im = -v.im;
    if (scale) v = cscale(v, scale[xr0 + c]);
    Y[(xc0 + r) * ldy + xr0 + c] = v;
  }
}

// Y[j][i] = conj(X[j][i]) * scale[j] (elementwise, d x d contiguous).
__global__ __launch_bounds__(256) void conj_rows_kernel(const C64* __restrict__ X, C64* __restrict__ Y, int n,
                                                        const double* __restrict__ scale) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= (int64_t(1) << (2 * n))) return;
  const double s = scale[e >> n];
  const C64 v = X[e];
  Y[e] = C64{v.re * s, -v.im * s};
}

// S = (X + X^dagger) / 2 in FP64 (d x d contiguous) from X in storage type
// R, over the tile pairs (I, J), I >= J, of B x B tiles.
template <typename R>
__global__ __launch_bounds__(256) void herm_to64_kernel(const Cx<R>* __restrict__ X, int64_t ldx, int lgB,
                                                        C64* __restrict__ S, int64_t lds) {
  __shared__ C64 a[kTB][kTB + 1], b[kTB][kTB + 1];
  const int B = 1 << lgB;
  int I, J;
  tri_decode(blockIdx.x, I, J);
  const int64_t r0 = int64_t(I) << lgB, c0 = int64_t(J) << lgB;
  const int elems = B * B;
  for (int e = threadIdx.x; e < elems; e += 256) {
    const int r = e >> lgB, c = e & (B - 1);
    const Cx<R> x = X[(r0 + r) * ldx + c0 + c], y = X[(c0 + r) * ldx + r0 + c];
    a[r][c] = C64{double(x.re), double(x.im)};
    b[r][c] = C64{double(y.re), double(y.im)};
  }
  __syncthreads();
  for (int e = threadIdx.x; e < elems; e += 256) {
    const int r = e >> lgB, c = e & (B - 1);
    const C64 x = a[r][c], y = b[c][r];
    S[(r0 + r) * lds + c0 + c] = C64{0.5 * (x.re + y.re), 0.5 * (x.im - y.im)};
    if (I != J) {
      const C64 u = b[r][c], v = a[c][r];
      S[(c0 + r) * lds + r0 + c] = C64{0.5 * (u.re + v.re), 0.5 * (u.im - v.im)};
    }
  }
}

// Divided difference of g(l) = |l|^a at (x, y): g' on ties (0 at l = 0); for
// x, y of one sign, |x|^a - |y|^a = |y|^a expm1(a log1p((|x| - |y|) / |y|)),
// free of cancellation when x and y are close.
__device__ __forceinline__ double divided_difference(double x, double y, double a) {
  if (x == y) return x == 0.0 ? 0.0 : (x > 0.0 ? a : -a) * pow(fabs(x), a - 1.0);
  if ((x > 0.0 && y > 0.0) || (x < 0.0 && y < 0.0)) {
    const double ax = fabs(x), ay = fabs(y), dd = ax - ay;
    const double v = pow(ay, a) * expm1(a * log1p(dd / ay)) / dd;
    return x > 0.0 ? v : -v;
  }
  return (pow(fabs(x), a) - pow(fabs(y), a)) / (x - y);
}

__global__ __launch_bounds__(256) void divided_diff_kernel(C64* __restrict__ M, const double* __restrict__ lam,
                                                           int n, double a) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= (int64_t(1) << (2 * n))) return;
  const double g = divided_difference(lam[e >> n], lam[e & ((int64_t(1) << n) - 1)], a);
  M[e] = cscale(M[e], g);
}

template <typename R>
__global__ __launch_bounds__(256) void from64_kernel(const C64* __restrict__ X, int n, Cx<R>* __restrict__ Y,
                                                     int64_t ldy) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= (int64_t(1) << (2 * n))) return;
  const int64_t r = e >> n, c = e & ((int64_t(1) << n) - 1);
  Y[r * ldy + c] = Cx<R>{R(X[e].re), R(X[e].im)};
}

struct Bufs {
  C64 *b0, *b1, *b2;
  double *part, *scal;
  void* sk;
  JacobiState* st;
  void* eig;
};

Bufs carve(int n, void* ws) {
  const AbsMapLayout L = absmap_layout(n);
  unsigned char* w = static_cast<unsigned char*>(ws);
  return Bufs{reinterpret_cast<C64*>(w + L.b0), reinterpret_cast<C64*>(w + L.b1), reinterpret_cast<C64*>(w + L.b2),
              reinterpret_cast<double*>(w + L.part), reinterpret_cast<double*>(w + L.scal),
              L.sk_bytes ? static_cast<void*>(w + L.sk) : nullptr, reinterpret_cast<JacobiState*>(w + L.state),
              static_cast<void*>(w + L.eig)};
}

unsigned elem_blocks(int n) { return unsigned(((int64_t(1) << (2 * n)) + 255) / 256); }

hipError_t herm_to64(qst_prec prec, const void* X, int64_t ldx, C64* S, int n, hipStream_t s) {
  const int lgB = n < 5 ? n : 5;
  const int64_t m = int64_t(1) << (n - lgB);
  const unsigned blocks = unsigned(m * (m + 1) / 2);
  const int64_t d = int64_t(1) << n;
  if (prec == QST_F64)
    herm_to64_kernel<double><<<blocks, 256, 0, s>>>(static_cast<const Cx<double>*>(X), ldx, lgB, S, d);
  else
    herm_to64_kernel<float><<<blocks, 256, 0, s>>>(static_cast<const Cx<float>*>(X), ldx, lgB, S, d);
  return hipGetLastError();
}

hipError_t transpose64(const C64* X, int64_t ldx, C64* Y, int64_t ldy, int n, bool conj, const double* scale,
                       hipStream_t s) {
  const int lgB = n < 5 ? n : 5;
  const unsigned m = 1u << (n - lgB);
  transpose64_kernel<<<dim3(m, m), 256, 0, s>>>(X, ldx, Y, ldy, lgB, conj ? 1 : 0, scale);
  return hipGetLastError();
}

// C = X Y (d x d, FP64, contiguous operands) on the library's complex
// product: its scale 2 up / tau is 1 with tau = 2 (scal[0]) and no up.
hipError_t product64(const C64* X, const C64* Y, void* C, int64_t ldc, int n, const Bufs& b, hipStream_t s) {
  const int64_t d = int64_t(1) << n;
  return launch_hemm(QST_F64, X, d, Y, d, C, ldc, n, b.scal, nullptr, b.sk, s, nullptr);
}

hipError_t store_out(qst_prec prec, const C64* X, void* Y, int64_t ldy, int n, hipStream_t s) {
  if (prec == QST_F64) return hipSuccess;
  from64_kernel<float><<<elem_blocks(n), 256, 0, s>>>(X, n, static_cast<Cx<float>*>(Y), ldy);
  return hipGetLastError();
}

// Relative off-diagonal norm at which the sweeps stop: 1e-14 for FP64
// storage; 1e-10 for FP32 storage, whose outputs are rounded to 6e-8
// (eigenvalue errors are second order in it, A's and the adjoint's first
// order).
double sweep_tol(qst_prec prec) { return prec == QST_F64 ? 1e-14 : 1e-10; }

// Jacobi sweeps on b.b0 (ping-pong with b.b1; V^T rotated in b.b2), at
// most max_sweeps, the stopping rule decided on the device (JacobiState).
// sync: the host reads the state after each sweep and stops enqueuing
// once done (*sweeps then holds the sweeps taken, or -1); otherwise all
// max_sweeps are enqueued and nothing is read back.
hipError_t jacobi_sweeps(const Bufs& b, int n, hipStream_t s, int max_sweeps, double tol, bool sync, int* sweeps) {
  if (sweeps) *sweeps = -1;
  const int d = 1 << n, half = d >> 1;
  const int chunks = (half + kRoundThreads - 1) / kRoundThreads;
  hipError_t e;
  jacobi_reset_kernel<<<1, 1, 0, s>>>(b.st);
  C64 *cur = b.b0, *nxt = b.b1;
  for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
    for (int t = 0; t < d - 1; ++t) {
      jacobi_round_kernel<<<dim3(half, chunks), kRoundThreads, 0, s>>>(cur, nxt, b.b2, d, t, b.part, b.st);
      C64* x = cur;
      cur = nxt;
      nxt = x;
    }
    jacobi_check_kernel<<<1, 256, 0, s>>>(b.part, half * chunks, b.st, tol, sweep, max_sweeps);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (sync) {
      JacobiState host;
      if ((e = hipMemcpyAsync(&host, b.st, sizeof(host), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      if (host.done) {
        if (sweeps) *sweeps = host.sweeps;
        return hipSuccess;
      }
    }
  }
  return hipSuccess;
}

// X (storage type R, row stride ldx) -> FP64, d x d contiguous.
template <typename R>
__global__ __launch_bounds__(256) void to64_kernel(const Cx<R>* __restrict__ X, int64_t ldx, int n,
                                                   C64* __restrict__ Y) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= (int64_t(1) << (2 * n))) return;
  const Cx<R> v = X[(e >> n) * ldx + (e & ((int64_t(1) << n) - 1))];
  Y[e] = C64{double(v.re), double(v.im)};
}

hipError_t to64(qst_prec prec, const void* X, int64_t ldx, C64* Y, int n, hipStream_t s) {
  if (prec == QST_F64)
    to64_kernel<double><<<elem_blocks(n), 256, 0, s>>>(static_cast<const Cx<double>*>(X), ldx, n, Y);
  else
    to64_kernel<float><<<elem_blocks(n), 256, 0, s>>>(static_cast<const Cx<float>*>(X), ldx, n, Y);
  return hipGetLastError();
}

// part[2b] = sum of |X_e|^2 over e = b, b + nb, ... (part[2b+1] = 0).
__global__ __launch_bounds__(256) void sumsq_kernel(const C64* __restrict__ X, int64_t count,
                                                    double* __restrict__ part) {
  __shared__ double lds4[4];
  double a = 0.0;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < count; e += int64_t(gridDim.x) * 256)
    a += cnorm(X[e]);
  a = block_sum256(a, lds4);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = 0.0;
  }
}

// F = (sum_i sqrt(max(lam_i, 0)))^2 / tau over the d eigenvalues, in a
// fixed order (one workgroup).
__global__ __launch_bounds__(256) void fq_eig_finish_kernel(const double* __restrict__ lam, int d,
                                                            const double* __restrict__ tau, double* __restrict__ F) {
  __shared__ double lds4[4];
  double a = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) a += sqrt(fmax(lam[i], 0.0));
  a = block_sum256(a, lds4);
  if (threadIdx.x == 0) *F = a * a / *tau;
}

// Reads the eigensolver's status (0 or -1) on the host: one synchronisation.
hipError_t read_status(const EighWork& w, hipStream_t s, int* out) {
  hipError_t e;
  if ((e = hipMemcpyAsync(out, w.status, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// H (b0, d x d FP64 Hermitian, overwritten) = Q diag(lam) Q^dagger by the
// direct solver: Q (d x d FP64, eigenvectors as columns) and lam; b1 holds
// the reflectors, b2 the tridiagonal's eigenvectors.
hipError_t eigh_direct(const Bufs& b, int n, double* lam, C64* Q, hipStream_t s) {
  const int d = 1 << n;
  const EighWork w = eigh_work(n, b.eig);
  hipError_t e;
  if ((e = launch_tridiagonalize(n, b.b0, b.b1, w, s)) != hipSuccess) return e;
  if ((e = launch_tri_eigvals(n, w, lam, s)) != hipSuccess) return e;
  if ((e = launch_tri_vectors(n, w, lam, b.b0, b.b2, s)) != hipSuccess) return e;
  // one Newton-Schulz step: Z <- Z (1.5 I - 0.5 Z^T Z) (Z real, in b2)
  if ((e = transpose64(b.b2, d, b.b0, d, n, false, nullptr, s)) != hipSuccess) return e;
  if ((e = product64(b.b0, b.b2, Q, d, n, b, s)) != hipSuccess) return e;
  if ((e = launch_ns_matrix(n, Q, b.b0, s)) != hipSuccess) return e;
  if ((e = product64(b.b2, b.b0, Q, d, n, b, s)) != hipSuccess) return e;
  return launch_back_transform(n, b.b1, w, Q, b.b2, s);
}

}  // namespace

hipError_t launch_fidelity_general(qst_prec prec, int n, const void* T, int64_t ldT, const void* rho, int64_t ldR,
                                   double* F, void* ws, hipStream_t s, int* sweeps, int max_sweeps, int* sweeps_dev) {
  const int d = 1 << n, half = d >> 1;
  const Bufs b = carve(n, ws);
  const bool sync = sweeps_dev == nullptr;
  if (sweeps) *sweeps = -1;
  hipError_t e;
  ProfScope prof("fidelity_general", s);
  set_scalar_kernel<<<1, 1, 0, s>>>(b.scal, 2.0);
  if ((e = to64(prec, T, ldT, b.b0, n, s)) != hipSuccess) return e;  // T
  const int nb = half < 256 ? half : 256;                               // 2 nb <= d partials
  sumsq_kernel<<<nb, 256, 0, s>>>(b.b0, int64_t(d) * d, b.part);
  jacobi_norms_kernel<<<1, 256, 0, s>>>(b.part, nb, b.scal + 4);      // tau at scal[4]
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = to64(prec, rho, ldR, b.b2, n, s)) != hipSuccess) return e;                         // rho
  if ((e = product64(b.b2, b.b0, b.b1, d, n, b, s)) != hipSuccess) return e;                  // rho T
  if ((e = transpose64(b.b0, d, b.b2, d, n, true, nullptr, s)) != hipSuccess) return e;      // T^dagger
  if ((e = product64(b.b2, b.b1, b.b0, d, n, b, s)) != hipSuccess) return e;                  // C = T^dagger rho T
  (void)max_sweeps;
  // the eigenvalues of the Hermitian part of C by the direct solver
  const EighWork w = eigh_work(n, b.eig);
  if ((e = herm_to64(QST_F64, b.b0, d, b.b1, n, s)) != hipSuccess) return e;
  if ((e = launch_tridiagonalize(n, b.b1, b.b2, w, s)) != hipSuccess) return e;
  if ((e = launch_tri_eigvals(n, w, b.part, s)) != hipSuccess) return e;
  fq_eig_finish_kernel<<<1, 256, 0, s>>>(b.part, d, b.scal + 4, F);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (sweeps_dev) return launch_eigh_status(w, sweeps_dev, s);
  if (sync) {
    int st = -1;
    if ((e = read_status(w, s, &st)) != hipSuccess) return e;
    if (sweeps) *sweeps = st;
  }
  return hipSuccess;
}

hipError_t launch_abs_map(qst_prec prec, int n, double P, const void* T, int64_t ldT, const void* Q0, void* A,
                          int64_t ldA, void* Q, double* lam, void* ws, hipStream_t s, int* sweeps, int max_sweeps,
                          int* sweeps_dev) {
  const int d = 1 << n;
  const Bufs b = carve(n, ws);
  const bool sync = sweeps_dev == nullptr;
  if (sweeps) *sweeps = -1;
  hipError_t e;
  ProfScope prof("abs_map", s);
  set_scalar_kernel<<<1, 1, 0, s>>>(b.scal, 2.0);
  if ((e = herm_to64(prec, T, ldT, b.b0, n, s)) != hipSuccess) return e;
  if (!Q0) {
    // cold start: the direct solver (a fixed sequence of launches)
    C64* q = static_cast<C64*>(Q);
    if ((e = eigh_direct(b, n, lam, q, s)) != hipSuccess) return e;
    double* sc = b.part;  // |lam|^(P/4), d values
    power_scale_kernel<<<(d + 255) / 256, 256, 0, s>>>(lam, d, P, sc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = transpose64(q, d, b.b2, d, n, false, nullptr, s)) != hipSuccess) return e;  // V^T = Q^T
    if ((e = transpose64(b.b2, d, b.b1, d, n, false, sc, s)) != hipSuccess) return e;  // U = Q diag(sc)
    conj_rows_kernel<<<elem_blocks(n), 256, 0, s>>>(b.b2, b.b0, n, sc);                 // U^dagger
    if ((e = hipGetLastError()) != hipSuccess) return e;
    C64* out64 = prec == QST_F64 ? static_cast<C64*>(A) : b.b2;
    if ((e = product64(b.b1, b.b0, out64, prec == QST_F64 ? ldA : d, n, b, s)) != hipSuccess) return e;
    if ((e = store_out(prec, out64, A, ldA, n, s)) != hipSuccess) return e;
    const EighWork w = eigh_work(n, b.eig);
    if (sweeps_dev) return launch_eigh_status(w, sweeps_dev, s);
    int st = -1;
    if ((e = read_status(w, s, &st)) != hipSuccess) return e;
    if (sweeps) *sweeps = st;
    return hipSuccess;
  }
  {
    // Warm start from a unitary Q0: Jacobi on Q0^dagger H Q0 with V = Q0.
    const C64* q0 = static_cast<const C64*>(Q0);
    if ((e = transpose64(q0, d, b.b1, d, n, true, nullptr, s)) != hipSuccess) return e;  // Q0^dagger
    if ((e = product64(b.b0, q0, b.b2, d, n, b, s)) != hipSuccess) return e;               // H Q0
    if ((e = product64(b.b1, b.b2, b.b0, d, n, b, s)) != hipSuccess) return e;             // Q0^dagger H Q0
    if ((e = transpose64(q0, d, b.b2, d, n, false, nullptr, s)) != hipSuccess) return e;  // V^T = Q0^T
  }
  if ((e = jacobi_sweeps(b, n, s, max_sweeps, sweep_tol(prec), sync, sweeps)) != hipSuccess) return e;
  if (sync && *sweeps < 0) return hipSuccess;
  // the diagonalised matrix is in b0 or b1 (its diagonal read by
  // spectrum_kernel); b.b2 = V^T; b0 and b1 are free afterwards
  double* sc = b.part;  // |lam|^(P/4), d values
  spectrum_kernel<<<(d + 255) / 256, 256, 0, s>>>(b.b0, b.b1, b.st, d, P, lam, sc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = transpose64(b.b2, d, static_cast<C64*>(Q), d, n, false, nullptr, s)) != hipSuccess) return e;
  if ((e = transpose64(b.b2, d, b.b1, d, n, false, sc, s)) != hipSuccess) return e;  // U = Q diag(sc)
  conj_rows_kernel<<<elem_blocks(n), 256, 0, s>>>(b.b2, b.b0, n, sc);                 // U^dagger
  if ((e = hipGetLastError()) != hipSuccess) return e;
  C64* out64 = prec == QST_F64 ? static_cast<C64*>(A) : b.b2;
  if ((e = product64(b.b1, b.b0, out64, prec == QST_F64 ? ldA : d, n, b, s)) != hipSuccess) return e;
  if ((e = store_out(prec, out64, A, ldA, n, s)) != hipSuccess) return e;
  if (sweeps_dev) jacobi_sweeps_out_kernel<<<1, 1, 0, s>>>(b.st, sweeps_dev);
  return hipGetLastError();
}

hipError_t launch_abs_map_backward(qst_prec prec, int n, double P, const void* Q, const double* lam, const void* GA,
                                   int64_t ldGA, void* GT, int64_t ldGT, void* ws, hipStream_t s) {
  const int d = 1 << n;
  const Bufs b = carve(n, ws);
  const C64* q = static_cast<const C64*>(Q);
  hipError_t e;
  ProfScope prof("abs_map_backward", s);
  set_scalar_kernel<<<1, 1, 0, s>>>(b.scal, 2.0);
  if ((e = herm_to64(prec, GA, ldGA, b.b0, n, s)) != hipSuccess) return e;       // S
  if ((e = transpose64(q, d, b.b1, d, n, true, nullptr, s)) != hipSuccess) return e;  // Q^dagger
  if ((e = product64(b.b0, q, b.b2, d, n, b, s)) != hipSuccess) return e;        // S Q
  if ((e = product64(b.b1, b.b2, b.b0, d, n, b, s)) != hipSuccess) return e;     // M = Q^dagger S Q
  divided_diff_kernel<<<elem_blocks(n), 256, 0, s>>>(b.b0, lam, n, 0.5 * P);     // Gamma o M
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = product64(q, b.b0, b.b2, d, n, b, s)) != hipSuccess) return e;        // Q (Gamma o M)
  C64* out64 = prec == QST_F64 ? static_cast<C64*>(GT) : b.b0;
  if ((e = product64(b.b2, b.b1, out64, prec == QST_F64 ? ldGT : d, n, b, s)) != hipSuccess) return e;
  return store_out(prec, out64, GT, ldGT, n, s);
}

}  // namespace qst
