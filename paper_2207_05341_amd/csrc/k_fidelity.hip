// Fidelity of the reconstructed state (Sec. 2.3).
//
// Quantum fidelity against a target of low rank r (Eq. F_QF):
//   F_q = (Tr sqrt(sqrt(rho_hat) rho sqrt(rho_hat)))^2,
//   rho_hat = T T^dagger / tau,  rho = W W^dagger / tw,  W d x r.
// sqrt(rho_hat) rho sqrt(rho_hat) has the nonzero eigenvalues of the r x r
// matrix C = M M^dagger / (tau tw), M = W^dagger T (r x d), so
// F_q = (sum_i sqrt(lambda_i(C)))^2.  Four launches:
//   1. fid_partial_kernel: M over row blocks of T (FP64 sums; also the
//      partial sums of |T|^2 for tau) -- reads T once per 8 or 16 target
//      columns;
//   2. fid_mreduce_kernel: M from the row-block sums, in order;
//   3. fid_gram_kernel: C_ab = sum_j M_aj conj(M_bj), one workgroup per pair;
//   4. fid_jacobi_kernel: tau, tw, C / (tau tw), parallel cyclic Jacobi
//      eigenvalues of the Hermitian C (FP64, one workgroup), F_q.
// Classical fidelity (Eq. F_CF): F_c = (sum_k sqrt(p_hat_k p_k))^2 (negative
// entries read as 0), a two-stage FP64 reduction.
// Every sum has a fixed order: results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "qst_device.h"
#include "qst_kernels.h"
#include "qst_plan.h"

namespace qst {

namespace {

constexpr int kRowChunk = 64;
constexpr int kRowGroup = 8;

struct Zd {
  double re, im;
};

// Workgroup (cb, rb): columns cb*64 .. +63 of T (fewer when d < 64), rows
// rb*RB .. (rb+1)*RB - 1.  Thread t: column c = t & 63, row quarter
// q = t >> 6 (rows i0 + q, i0 + q + 4, ... of each 64-row chunk).  For each
// chunk of AC target columns a0.., W's rows of the chunk are staged in LDS
// and every thread adds conj(W_ia) T_ij over its rows; the quarters are
// summed in order and P[rb][a][j] written.  In the first pass the thread
// also sums |T_ij|^2 (tau), written per workgroup to taup[rb * ncb + cb].
// AC target columns per pass over T (8 for ranks up to 8, else 16).
template <typename R, int AC>
__global__ __launch_bounds__(256) void fid_partial_kernel(const Cx<R>* __restrict__ T, int64_t ldT,
                                                          const Cx<R>* __restrict__ W, int64_t ldW, int r, int d,
                                                          int RB, Zd* __restrict__ P, double* __restrict__ taup) {
  __shared__ Zd wl[kRowChunk][AC];
  __shared__ Zd red[3][64][AC];
  __shared__ double rtau[4];
  const int ncb = d < 64 ? 1 : d / 64;
  const int cb = blockIdx.x % ncb, rb = blockIdx.x / ncb;
  const int t = threadIdx.x, c = t & 63, q = t >> 6;
  const int64_t j = int64_t(cb) * 64 + c;
  const bool col = j < d;
  const int64_t r0 = int64_t(rb) * RB;
  const int chunk = RB < kRowChunk ? RB : kRowChunk;
  double tsum = 0.0;
  for (int a0 = 0; a0 < r; a0 += AC) {
    Zd acc[AC];
#pragma unroll
    for (int a = 0; a < AC; ++a) acc[a] = Zd{0.0, 0.0};
    for (int i0 = 0; i0 < RB; i0 += chunk) {
      __syncthreads();  // the previous chunk's W is no longer read
      for (int e = t; e < chunk * AC; e += 256) {
        const int ii = e / AC, a = e % AC;
        Cx<R> w{R(0), R(0)};
        if (a0 + a < r) w = W[(r0 + i0 + ii) * ldW + a0 + a];
        wl[ii][a] = Zd{double(w.re), double(w.im)};
      }
      __syncthreads();
      if (col) {
        // kRowGroup rows of T loaded before any is used (one memory round
        // trip per group); rows past the chunk are clamped and dropped
        for (int g0 = q; g0 < chunk; g0 += 4 * kRowGroup) {
          Cx<R> xg[kRowGroup];
#pragma unroll
          for (int u = 0; u < kRowGroup; ++u) {
            const int ii = g0 + 4 * u < chunk ? g0 + 4 * u : q;
            xg[u] = T[(r0 + i0 + ii) * ldT + j];
          }
#pragma unroll
          for (int u = 0; u < kRowGroup; ++u) {
            const int ii = g0 + 4 * u;
            if (ii >= chunk) break;
            const double xr = double(xg[u].re), xi = double(xg[u].im);
            if (a0 == 0) tsum += xr * xr + xi * xi;
#pragma unroll
            for (int a = 0; a < AC; ++a) {
              const double wr = wl[ii][a].re, wi = wl[ii][a].im;
              // conj(w) x
              acc[a].re += wr * xr + wi * xi;
              acc[a].im += wr * xi - wi * xr;
            }
          }
        }
      }
    }
    // quarters 1..3 hand their sums to quarter 0, which adds them in order
    __syncthreads();
    if (q > 0) {
#pragma unroll
      for (int a = 0; a < AC; ++a) red[q - 1][c][a] = acc[a];
    }
    __syncthreads();
    if (q == 0 && col) {
#pragma unroll
      for (int a = 0; a < AC; ++a) {
        Zd s = acc[a];
        for (int k = 0; k < 3; ++k) {
          s.re += red[k][c][a].re;
          s.im += red[k][c][a].im;
        }
        if (a0 + a < r) P[(int64_t(rb) * r + a0 + a) * d + j] = s;
      }
    }
  }
  const double ts = block_sum256(tsum, rtau);
  if (t == 0) taup[blockIdx.x] = ts;
}

// M_aj = sum_rb P[rb][a][j] (row blocks in order), one entry per thread.
__global__ __launch_bounds__(256) void fid_mreduce_kernel(const Zd* __restrict__ P, int nrb, int r, int d,
                                                          Zd* __restrict__ M) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= int64_t(r) * d) return;
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < nrb; ++k) {
    const Zd x = P[int64_t(k) * r * d + e];
    sr += x.re;
    si += x.im;
  }
  M[e] = Zd{sr, si};
}

// C_ab = sum_j M_aj conj(M_bj); workgroup b handles the lower pair
// (a, b) = tri_decode(b) and writes C_ab and C_ba.
__global__ __launch_bounds__(256) void fid_gram_kernel(const Zd* __restrict__ M, int r, int d, Zd* __restrict__ C) {
  __shared__ double red[4];
  int a, b;
  tri_decode(blockIdx.x, a, b);
  double sr = 0.0, si = 0.0;
  for (int j = threadIdx.x; j < d; j += 256) {
    const Zd x = M[int64_t(a) * d + j], y = M[int64_t(b) * d + j];
    sr += x.re * y.re + x.im * y.im;
    si += x.im * y.re - x.re * y.im;
  }
  sr = block_sum256(sr, red);
  si = block_sum256(si, red);
  if (threadIdx.x == 0) {
    C[a * r + b] = Zd{sr, si};
    C[b * r + a] = Zd{sr, -si};
  }
}

// tau (the workgroup partials, in order), tw = sum |W|^2, then the
// eigenvalues of C / (tau tw) by parallel cyclic Jacobi and F_q.  A sweep
// takes the r(r-1)/2 pairs in r' - 1 steps of r'/2 disjoint pairs (round-robin
// order, r' = r rounded up to even; pairs with the padding index are
// skipped).  A rotation of the pair (p, q) with C_pq = |c| e, e = c / |c|,
// uses t = sign(x)/(|x| + sqrt(1 + x^2)), x = (C_qq - C_pp) / (2|c|),
// cs = 1/sqrt(1 + t^2), sn = t cs and the unitary G with G_pp = G_qq = cs,
// G_pq = sn e, G_qp = -sn conj(e): C <- G^dagger C G zeroes C_pq.  The
// rotations of one step touch disjoint rows and columns, and each one's
// parameters depend only on its own rows and columns, so applying them
// together equals applying them one after another.  Sweeps stop when the
// off-diagonal mass is below 1e-30 of the diagonal's, or after 40.
__global__ __launch_bounds__(256) void fid_jacobi_kernel(const double* __restrict__ taup, int ntaup,
                                                         const void* __restrict__ Wv, int64_t ldW, int r, int d,
                                                         int f64, const Zd* __restrict__ Cin, double* __restrict__ F) {
  constexpr int RM = kFidelityMaxRank;
  __shared__ Zd C[RM][RM + 1];
  __shared__ double red[4];
  __shared__ double rot[RM / 2][4];  // cs, sn, e.re, e.im per pair
  __shared__ int pq[RM / 2][2];
  __shared__ double colmass[RM];
  __shared__ double scale_sh;
  __shared__ int flag;
  const int t = threadIdx.x;
  double s = 0.0;
  for (int k = t; k < ntaup; k += 256) s += taup[k];
  const double tau = block_sum256(s, red);
  s = 0.0;
  for (int64_t e = t; e < int64_t(d) * r; e += 256) {
    const int64_t i = e / r, a = e % r;
    double wr, wi;
    if (f64) {
      const Cx<double> w = static_cast<const Cx<double>*>(Wv)[i * ldW + a];
      wr = w.re;
      wi = w.im;
    } else {
      const Cx<float> w = static_cast<const Cx<float>*>(Wv)[i * ldW + a];
      wr = double(w.re);
      wi = double(w.im);
    }
    s += wr * wr + wi * wi;
  }
  const double tw = block_sum256(s, red);
  if (t == 0) scale_sh = 1.0 / (tau * tw);
  __syncthreads();
  const double scale = scale_sh;
  for (int e = t; e < r * r; e += 256) {
    const Zd v = Cin[e];
    C[e / r][e % r] = Zd{v.re * scale, v.im * scale};
  }
  __syncthreads();
  const int rp = r + (r & 1), np = rp / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (t < r) {
      double off = 0.0;
      for (int i = 0; i < r; ++i)
        if (i != t) off += C[i][t].re * C[i][t].re + C[i][t].im * C[i][t].im;
      colmass[t] = off;
    }
    __syncthreads();
    if (t == 0) {
      double o = 0.0, g = 0.0;
      for (int k = 0; k < r; ++k) {
        o += colmass[k];
        g += C[k][k].re * C[k][k].re;
      }
      flag = (o == 0.0 || o <= 1e-30 * g) ? 1 : 0;
    }
    __syncthreads();
    if (flag) break;
    for (int step = 0; step < rp - 1; ++step) {
      if (t < np) {
        // round-robin positions t and rp - 1 - t; position 0 stays
        const int u = t, v = rp - 1 - t;
        const int iu = u == 0 ? 0 : ((u - 1 + step) % (rp - 1)) + 1;
        const int iv = ((v - 1 + step) % (rp - 1)) + 1;
        const int p = iu < iv ? iu : iv, q = iu < iv ? iv : iu;
        double cs = 1.0, sn = 0.0, er = 1.0, ei = 0.0;
        if (q < r) {
          const Zd c = C[p][q];
          const double ac = sqrt(c.re * c.re + c.im * c.im);
          if (ac > 1e-300) {
            const double dba = C[q][q].re - C[p][p].re;
            double tt;
            if (fabs(dba) > 1e10 * ac) {
              tt = ac / dba;
            } else {
              const double x = dba / (2.0 * ac);
              tt = (x >= 0.0 ? 1.0 : -1.0) / (fabs(x) + sqrt(1.0 + x * x));
            }
            cs = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * cs;
            er = c.re / ac;
            ei = c.im / ac;
          }
        }
        rot[t][0] = cs;
        rot[t][1] = sn;
        rot[t][2] = er;
        rot[t][3] = ei;
        pq[t][0] = p;
        pq[t][1] = (q < r && sn != 0.0) ? q : -1;
      }
      __syncthreads();
      for (int task = t; task < np * r; task += 256) {  // columns p, q: C G
        const int k = task / r, i = task % r, p = pq[k][0], q = pq[k][1];
        if (q < 0) continue;
        const double cs = rot[k][0], sn = rot[k][1], er = rot[k][2], ei = rot[k][3];
        const Zd cp = C[i][p], cq = C[i][q];
        // cs cp - sn conj(e) cq ;  sn e cp + cs cq
        C[i][p] = Zd{cs * cp.re - sn * (er * cq.re + ei * cq.im), cs * cp.im - sn * (er * cq.im - ei * cq.re)};
        C[i][q] = Zd{sn * (er * cp.re - ei * cp.im) + cs * cq.re, sn * (er * cp.im + ei * cp.re) + cs * cq.im};
      }
      __syncthreads();
      for (int task = t; task < np * r; task += 256) {  // rows p, q: G^dagger (C G)
        const int k = task / r, j = task % r, p = pq[k][0], q = pq[k][1];
        if (q < 0) continue;
        const double cs = rot[k][0], sn = rot[k][1], er = rot[k][2], ei = rot[k][3];
        const Zd rp_ = C[p][j], rq = C[q][j];
        // cs rp - sn e rq ;  sn conj(e) rp + cs rq; the rotated pair's own
        // off-diagonal entries are zero by construction and stored as such
        C[p][j] = j == q ? Zd{0.0, 0.0}
                         : Zd{cs * rp_.re - sn * (er * rq.re - ei * rq.im), cs * rp_.im - sn * (er * rq.im + ei * rq.re)};
        C[q][j] = j == p ? Zd{0.0, 0.0}
                         : Zd{sn * (er * rp_.re + ei * rp_.im) + cs * rq.re, sn * (er * rp_.im - ei * rp_.re) + cs * rq.im};
      }
      __syncthreads();
    }
  }
  if (t == 0) {
    double sq = 0.0;
    for (int k = 0; k < r; ++k) sq += sqrt(fmax(C[k][k].re, 0.0));
    *F = sq * sq;
  }
}

// F_c stage 1: block b sums sqrt(max(p_hat,0) max(p,0)) over its range.
template <typename R>
__global__ __launch_bounds__(256) void fid_classical_partial_kernel(const R* __restrict__ ph, const R* __restrict__ p,
                                                                    int64_t D, double* __restrict__ partials) {
  __shared__ double red[4];
  const int nb = gridDim.x;
  const int64_t chunk = (D + nb - 1) / nb;
  const int64_t beg = int64_t(blockIdx.x) * chunk;
  const int64_t end = beg + chunk < D ? beg + chunk : D;
  constexpr int U = 8;
  double s = 0.0;
  for (int64_t k0 = beg + threadIdx.x; k0 < end; k0 += U * int64_t(blockDim.x)) {
    R a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = k0 + u * int64_t(blockDim.x);
      const bool in = k < end;
      a[u] = in ? ph[k] : R(0);
      b[u] = in ? p[k] : R(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += sqrt(fmax(double(a[u]), 0.0) * fmax(double(b[u]), 0.0));
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void fid_classical_finish_kernel(const double* __restrict__ partials, int nb,
                                                                   double* __restrict__ F) {
  __shared__ double red[4];
  const double s = sum_partials256(partials, nb, red);
  if (threadIdx.x == 0) *F = s * s;
}

template <typename R>
hipError_t run_fidelity_lowrank(const void* T, int64_t ldT, const void* W, int64_t ldW, int r, int n, void* ws,
                                double* F, hipStream_t s) {
  const FidelityLayout fl = fidelity_layout(n);
  const int d = 1 << n;
  unsigned char* base = static_cast<unsigned char*>(ws);
  Zd* P = reinterpret_cast<Zd*>(base + fl.mpart);
  Zd* C = reinterpret_cast<Zd*>(base + fl.gram);
  double* taup = reinterpret_cast<double*>(base + fl.taup);
  const int ncb = d < 64 ? 1 : d / 64;
  if (r <= 8)
    fid_partial_kernel<R, 8><<<unsigned(ncb * fl.nrb), 256, 0, s>>>(static_cast<const Cx<R>*>(T), ldT,
                                                                    static_cast<const Cx<R>*>(W), ldW, r, d,
                                                                    d / fl.nrb, P, taup);
  else
    fid_partial_kernel<R, 16><<<unsigned(ncb * fl.nrb), 256, 0, s>>>(static_cast<const Cx<R>*>(T), ldT,
                                                                     static_cast<const Cx<R>*>(W), ldW, r, d,
                                                                     d / fl.nrb, P, taup);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  Zd* M = reinterpret_cast<Zd*>(base + fl.mrow);
  fid_mreduce_kernel<<<unsigned((int64_t(r) * d + 255) / 256), 256, 0, s>>>(P, fl.nrb, r, d, M);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  fid_gram_kernel<<<unsigned(r * (r + 1) / 2), 256, 0, s>>>(M, r, d, C);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  fid_jacobi_kernel<<<1, 256, 0, s>>>(taup, ncb * fl.nrb, W, ldW, r, d, sizeof(R) == 8, C, F);
  return hipGetLastError();
}

template <typename R>
hipError_t run_fidelity_classical(const void* ph, const void* p, int n, double* part, double* F, hipStream_t s) {
  fid_classical_partial_kernel<R><<<kReduceBlocks, 256, 0, s>>>(static_cast<const R*>(ph), static_cast<const R*>(p),
                                                                int64_t(1) << (2 * n), part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fid_classical_finish_kernel<<<1, 256, 0, s>>>(part, kReduceBlocks, F);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fidelity_lowrank(qst_prec prec, const void* T, int64_t ldT, const void* W, int64_t ldW, int r,
                                   int n, void* ws, double* F, hipStream_t s) {
  if (prec == QST_F64) return run_fidelity_lowrank<double>(T, ldT, W, ldW, r, n, ws, F, s);
  return run_fidelity_lowrank<float>(T, ldT, W, ldW, r, n, ws, F, s);
}

hipError_t launch_fidelity_classical(qst_prec prec, const void* ph, const void* p, int n, void* ws, double* F,
                                     hipStream_t s) {
  double* part = reinterpret_cast<double*>(static_cast<unsigned char*>(ws) + fidelity_layout(n).cpart);
  return launch_fidelity_classical_part(prec, ph, p, n, part, F, s);
}

hipError_t launch_fidelity_classical_part(qst_prec prec, const void* ph, const void* p, int n, double* part, double* F,
                                          hipStream_t s) {
  if (prec == QST_F64) return run_fidelity_classical<double>(ph, p, n, part, F, s);
  return run_fidelity_classical<float>(ph, p, n, part, F, s);
}

}  // namespace qst
