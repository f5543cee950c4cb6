// Direct Hermitian eigensolver (FP64) behind the P-order absolute map of
// Sec. 3.2 (Eq. abs_P) and the general fidelity (Eq. F_QF through one
// eigendecomposition, as Eq. fq_decom does).
//
// H = Q T Q^dagger with T real symmetric tridiagonal (Householder), then
// T = Z Lambda Z^T, and the eigenvectors of H are the columns of Q Z:
//
// 1. Reduction.  Step k forms the reflector I - tau_k v_k v_k^dagger that
//    maps column k below the diagonal onto beta_k e_1 (beta_k real, so T is
//    real), and the Hermitian rank-2 update of the trailing matrix,
//    A22 -= v w^dagger + w v^dagger with w = tau A22 v + alpha v,
//    alpha = -|tau|^2 (v^dagger A22 v) / 2.  One launch per column: step k
//    applies the update of step k-1 on the fly to row k (which every
//    workgroup reads: row k holds column k conjugated, H being Hermitian),
//    forms reflector k from it (redundantly in every workgroup, identically
//    since the data and the order are the same), and then updates its own
//    rows of the trailing matrix while forming their entries of A22 v_k.
//    The trailing matrix is thus read and written once per column.
// 2. Splitting.  Off-diagonal entries below 4 eps sqrt(d) ||T|| are set to
//    zero (a perturbation of the size of the reduction's own rounding); the
//    unreduced blocks are then independent.
// 3. Eigenvalues by multisection: a wave per eigenvalue evaluates the Sturm
//    count (the number of negative pivots of T - x I) of its block at 64
//    points of the current interval and keeps the sub-interval that holds
//    the eigenvalue: about 6 bits per round, full precision in 9 or 10.
// 4. Eigenvectors by twisted factorizations, one thread per eigenvalue:
//    T - lambda I = L+ D+ L+^T (top down) = U- D- U-^T (bottom up); the twist
//    index r minimises |gamma_k| = |D+_k + D-_k - (a_k - lambda)|, and the
//    vector follows from z_r = 1 by z_k = -L+_k z_{k+1} above r and
//    z_{k+1} = -U-_k z_k below it.
// 5. Clusters (eigenvalues of a block closer than 1e-7 ||T||): inverse
//    iteration with Gaussian elimination with partial pivoting on
//    T - sigma I, each member orthogonalised against the members before it
//    (the classical treatment of clusters), one workgroup per cluster.
// 6. One Newton-Schulz step Z <- Z (3 I - Z^T Z) / 2 restores orthogonality
//    to rounding level (the twisted vectors of eigenvalues with a relative
//    gap g are orthogonal to about eps / g).
// 7. Back-transformation Q Z with the reflectors in blocks of 64 in the
//    compact form I - V T_B V^dagger (T_B upper triangular from the Gram
//    matrix of the block's reflectors, W_B = V T_B formed once), applied
//    from the last block to the first: X = V^dagger Z (row-chunk partial
//    sums, then their sum), Z -= W_B X.
//
// The eigenvalues of every block come out in ascending order; across blocks
// there is no particular order.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstddef>

#include "qst_device.h"
#include "qst_kernels.h"

namespace qst {

namespace {

using C64 = Cx<double>;

__device__ __forceinline__ C64 cmul(C64 a, C64 b) { return C64{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
// conj(a) * b
__device__ __forceinline__ C64 cmulc(C64 a, C64 b) { return C64{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }
__device__ __forceinline__ C64 conjg(C64 a) { return C64{a.re, -a.im}; }

constexpr double kEps = DBL_EPSILON;
constexpr double kClusterTol = 1e-7;  // relative gap below which eigenvalues form a cluster

// Sum over a 256-thread block, the result returned to every thread.
__device__ __forceinline__ double block_sum_all(double v, double* lds4) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) lds4[w] = v;
  __syncthreads();
  return ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
}

// Sum over a workgroup of NW waves, the result returned to every thread.
template <int NW>
__device__ __forceinline__ double block_sum_allN(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// ---------------------------------------------------------------------------
// 1. Reduction to tridiagonal form
// ---------------------------------------------------------------------------

struct TrdArgs {
  C64* A;            // d x d working matrix, row-major, Hermitian (both triangles)
  C64* V;            // d x d: row k holds v_k in columns k+1 .. d-1 (v_k[k+1] = 1)
  double* diag;      // d: diagonal of T
  double* off;       // d - 1: off-diagonal of T (beta_k)
  C64* tau;          // d - 1 reflector scalars
  int d, groups;
};

// Step k (0 <= k <= d - 2), d <= DMAX, NT threads (NT / 64 waves) per
// workgroup.  CACHE: v_{k-1} and w_{k-1} are staged in LDS next to v_k
// (3 DMAX complex values); otherwise w_{k-1} is formed from global memory
// where it is used.  yprev / pprev: A22 v_{k-1} (entries k .. d-1) and its
// partial sums from step k - 1; ynext / pnext are this step's.  Rows
// r >= k + 1 belong to workgroup r % groups, and wave w of it takes its
// rows first + (w + i NT/64) groups.  Every load that does not depend on
// this step's arithmetic (the partial sums, row k, v_{k-1} and A22 v_{k-1},
// and with PRE the wave's first row) is issued before any of it, so the
// step waits on memory about once.
template <int DMAX, int NT, bool CACHE>
__global__ __launch_bounds__(NT) void trd_step_kernel(TrdArgs g, int k, const C64* __restrict__ yprev,
                                                      C64* __restrict__ ynext, const double* __restrict__ pprev,
                                                      double* __restrict__ pnext) {
  constexpr int NW = NT / 64;
  constexpr int J2 = (DMAX + NT - 1) / NT;  // row-k slots per thread
  constexpr bool PRE = DMAX <= 2048;        // prefetch the wave's first row
  constexpr int JR = PRE ? DMAX / 64 : 1;   // row slots per lane
  __shared__ C64 lds[(CACHE ? 3 : 1) * DMAX];
  __shared__ double red[NW];
  C64* vs = lds;  // v_k (column index), with x_k before scaling
  C64* vps = lds + (CACHE ? DMAX : 0);
  C64* wps = lds + (CACHE ? 2 * DMAX : 0);
  const int d = g.d, P = g.groups, wg = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int r1 = k + 1;
  const int first = r1 + ((wg - r1 % P) + P) % P;  // first owned row >= k + 1
  if (first >= d && wg != 0) {
    if (tid == 0) pnext[wg] = 0.0;
    return;
  }
  const bool prev = k > 0;
  const C64* vprow = g.V + int64_t(k - 1) * d;  // v_{k-1}; used only when prev
  const C64* rowk = g.A + int64_t(k) * d;
  // ---- independent loads
  double pp = 0.0;
  if (prev)
    for (int p = tid; p < P; p += NT) pp += pprev[p];
  C64 rk[J2], vl[J2], yl[J2];
#pragma unroll
  for (int j = 0; j < J2; ++j) {
    const int c = k + tid + NT * j;
    rk[j] = vl[j] = yl[j] = C64{0.0, 0.0};
    if (c < d) {
      rk[j] = rowk[c];
      if (prev) {
        vl[j] = vprow[c];
        yl[j] = yprev[c];
      }
    }
  }
  C64 vpk{0.0, 0.0}, ypk{0.0, 0.0};
  const int r0 = first + wave * P;
  C64 vr0{0.0, 0.0}, yr0{0.0, 0.0};
  if (prev) {
    vpk = vprow[k];
    ypk = yprev[k];
    if (r0 < d) {
      vr0 = vprow[r0];
      yr0 = yprev[r0];
    }
  }
  C64 ar[JR];
  if (PRE) {
#pragma unroll
    for (int j = 0; j < JR; ++j) {
      const int c = k + 1 + lane + 64 * j;
      ar[j] = (r0 < d && c < d) ? g.A[int64_t(r0) * d + c] : C64{0.0, 0.0};
    }
  }
  // ---- the previous step's alpha and w
  C64 tp{0.0, 0.0};
  double ap = 0.0;
  if (prev) {
    tp = g.tau[k - 1];
    const double s = block_sum_allN<NW>(pp, red);
    ap = -0.5 * (tp.re * tp.re + tp.im * tp.im) * s;
  }
  auto wfrom = [&](C64 v, C64 y) -> C64 {
    const C64 ty = cmul(tp, y);
    return C64{ty.re + ap * v.re, ty.im + ap * v.im};
  };
  const C64 wpk = wfrom(vpk, ypk);
  // row k with the previous update applied; x_c = conj(row_c) is column k
  double nrm = 0.0;
#pragma unroll
  for (int j = 0; j < J2; ++j) {
    const int c = k + tid + NT * j;
    if (c < d) {
      C64 r = rk[j];
      if (prev) {
        const C64 wc = wfrom(vl[j], yl[j]);
        if (CACHE) {
          vps[c] = vl[j];
          wps[c] = wc;
        }
        const C64 t1 = cmulc(wc, vpk);     // v[k] conj(w[c])
        const C64 t2 = cmulc(vl[j], wpk);  // w[k] conj(v[c])
        r.re -= t1.re + t2.re;
        r.im -= t1.im + t2.im;
      }
      rk[j] = conjg(r);
      vs[c] = rk[j];
      if (c >= k + 2) nrm += r.re * r.re + r.im * r.im;
    }
  }
  nrm = block_sum_allN<NW>(nrm, red);  // its barriers also publish vs, vps, wps
  const C64 al = vs[k + 1];
  const double dk = vs[k].re;
  double beta;
  C64 t{0.0, 0.0}, sc{0.0, 0.0};
  if (nrm == 0.0 && al.im == 0.0) {
    beta = al.re;
  } else {
    beta = -copysign(sqrt(al.re * al.re + al.im * al.im + nrm), al.re);
    t = C64{(beta - al.re) / beta, -al.im / beta};
    const C64 den{al.re - beta, al.im};  // 1 / (alpha - beta)
    const double dd = den.re * den.re + den.im * den.im;
    sc = C64{den.re / dd, -den.im / dd};
  }
  __syncthreads();  // everyone has read vs[k], vs[k + 1]
  C64* vrow = g.V + int64_t(k) * d;
#pragma unroll
  for (int j = 0; j < J2; ++j) {
    const int c = k + tid + NT * j;
    if (c > k && c < d) {
      const C64 v = c == k + 1 ? C64{1.0, 0.0} : cmul(rk[j], sc);
      vs[c] = v;
      if (wg == 0) vrow[c] = v;
    }
  }
  if (wg == 0 && tid == 0) {
    g.diag[k] = dk;
    g.off[k] = beta;
    g.tau[k] = t;
  }
  __syncthreads();
  auto vp_at = [&](int c) -> C64 { return CACHE ? vps[c] : vprow[c]; };
  auto wp_at = [&](int c) -> C64 { return CACHE ? wps[c] : wfrom(vprow[c], yprev[c]); };
  // own rows: update with (v_{k-1}, w_{k-1}) on columns >= k + 1, and
  // y_k[r] = sum_c A22[r][c] v_k[c]
  double part = 0.0;
  for (int r = r0, i = 0; r < d; r += NW * P, ++i) {
    C64* row = g.A + int64_t(r) * d;
    C64 vpr{0.0, 0.0}, wpr{0.0, 0.0};
    if (prev) {
      vpr = i == 0 ? vr0 : vprow[r];
      wpr = wfrom(vpr, i == 0 ? yr0 : yprev[r]);
    }
    double yr = 0.0, yi = 0.0;
    auto visit = [&](int c, C64 a) {
      if (prev) {
        const C64 wc = wp_at(c), vc = vp_at(c);
        const C64 t1 = cmulc(wc, vpr), t2 = cmulc(vc, wpr);
        a.re -= t1.re + t2.re;
        a.im -= t1.im + t2.im;
        row[c] = a;
      }
      const C64 v = vs[c];
      yr += a.re * v.re - a.im * v.im;
      yi += a.re * v.im + a.im * v.re;
    };
    if (PRE && i == 0) {
#pragma unroll
      for (int j = 0; j < JR; ++j) {
        const int c = k + 1 + lane + 64 * j;
        if (c < d) visit(c, ar[j]);
      }
    } else {
      for (int c = k + 1 + lane; c < d; c += 64) visit(c, row[c]);
    }
    yr = wave_sum(yr);
    yi = wave_sum(yi);
    if (lane == 0) {
      ynext[r] = C64{yr, yi};
      const C64 v = vs[r];
      part += v.re * yr + v.im * yi;  // Re(conj(v_r) y_r)
    }
  }
  part = block_sum_allN<NW>(part, red);
  if (tid == 0) pnext[wg] = part;
}

constexpr int kTrdThreads = 256;

// The last diagonal entry: A[d-1][d-1] with the update of step d - 2.
__global__ __launch_bounds__(kTrdThreads) void trd_last_kernel(TrdArgs g, const C64* __restrict__ yprev,
                                                               const double* __restrict__ pprev) {
  __shared__ double red[4];
  const int d = g.d, k = d - 1;
  double s = 0.0;
  for (int p = threadIdx.x; p < g.groups; p += kTrdThreads) s += pprev[p];
  s = block_sum_all(s, red);
  if (threadIdx.x != 0) return;
  const C64 tp = g.tau[k - 1];
  const double ap = -0.5 * (tp.re * tp.re + tp.im * tp.im) * s;
  const C64 v = g.V[int64_t(k - 1) * d + k], ty = cmul(tp, yprev[k]);
  const C64 w{ty.re + ap * v.re, ty.im + ap * v.im};
  const C64 a = g.A[int64_t(k) * d + k];
  const C64 u = cmulc(w, v);  // v conj(w); the update is 2 Re of it on the diagonal
  g.diag[k] = a.re - 2.0 * u.re;
}

// ---------------------------------------------------------------------------
// 2. Splitting, norms, status
// ---------------------------------------------------------------------------

struct TriScal {
  double tnorm, pivmin;
  int status;  // 0 finite, -1 not finite
  int pad;
};

// One workgroup of 256 threads: ||T|| (largest Gershgorin bound), zeroes
// negligible off-diagonal entries, the unreduced block [bstart[i], bend[i])
// of every index (each thread scans a contiguous range, then a scan over the
// threads' results), the pivot floor, and whether everything is finite.
__global__ __launch_bounds__(256) void tri_split_kernel(const double* __restrict__ a, double* __restrict__ e, int d,
                                                        int* __restrict__ bstart, int* __restrict__ bend,
                                                        TriScal* __restrict__ ts) {
  __shared__ double mx[3][4];
  __shared__ double bc[2];
  __shared__ int lo_s[256], hi_s[256];
  const int tid = threadIdx.x;
  double tn = 0.0, e2 = 0.0, bad = 0.0;
  for (int k = tid; k < d; k += 256) {
    const double ek = k < d - 1 ? fabs(e[k]) : 0.0, el = k > 0 ? fabs(e[k - 1]) : 0.0;
    const double v = fabs(a[k]) + ek + el;
    if (!isfinite(v)) bad = 1.0;
    tn = fmax(tn, v);
    e2 = fmax(e2, ek * ek);
  }
  tn = wave_max(tn);
  e2 = wave_max(e2);
  bad = wave_max(bad);
  const int w = tid >> 6, l = tid & 63;
  if (l == 0) {
    mx[0][w] = tn;
    mx[1][w] = e2;
    mx[2][w] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    bc[0] = fmax(fmax(mx[0][0], mx[0][1]), fmax(mx[0][2], mx[0][3]));
    bc[1] = fmax(fmax(mx[1][0], mx[1][1]), fmax(mx[1][2], mx[1][3]));
    const double b = fmax(fmax(mx[2][0], mx[2][1]), fmax(mx[2][2], mx[2][3]));
    ts->tnorm = bc[0];
    ts->pivmin = DBL_MIN * fmax(1.0, bc[1]);
    ts->status = b != 0.0 ? -1 : 0;
  }
  __syncthreads();
  const double stol = 4.0 * kEps * sqrt(double(d)) * bc[0];
  // thread tid owns indices [i0, i1); a block starts at 0 and after every
  // zero off-diagonal entry e[k] (at k + 1), and ends after it (at k + 1)
  const int per = (d + 255) / 256, i0 = min(d, tid * per), i1 = min(d, i0 + per);
  int last_start = -1, first_end = d;
  for (int k = i0; k < i1; ++k)
    if (k < d - 1 && fabs(e[k]) <= stol) e[k] = 0.0;
  __syncthreads();  // e[i0 - 1] belongs to the previous thread
  for (int k = i0; k < i1; ++k) {
    const bool starts = k == 0 || e[k - 1] == 0.0;
    if (starts) last_start = k;
  }
  for (int k = i1 - 1; k >= i0; --k) {
    const bool ends = k == d - 1 || e[k] == 0.0;
    if (ends) first_end = k + 1;
  }
  lo_s[tid] = last_start;
  hi_s[tid] = first_end;
  __syncthreads();
  // inclusive max-scan of lo_s (from the left) and min-scan of hi_s (from the right)
  for (int o = 1; o < 256; o <<= 1) {
    const int lv = tid >= o ? lo_s[tid - o] : -1;
    const int hv = tid + o < 256 ? hi_s[tid + o] : d;
    __syncthreads();
    lo_s[tid] = max(lo_s[tid], lv);
    hi_s[tid] = min(hi_s[tid], hv);
    __syncthreads();
  }
  int st = tid > 0 ? lo_s[tid - 1] : -1;
  for (int k = i0; k < i1; ++k) {
    if (k == 0 || e[k - 1] == 0.0) st = k;
    bstart[k] = st;
  }
  int en = tid < 255 ? hi_s[tid + 1] : d;
  for (int k = i1 - 1; k >= i0; --k) {
    if (k == d - 1 || e[k] == 0.0) en = k + 1;
    bend[k] = en;
  }
}

// ---------------------------------------------------------------------------
// 3. Eigenvalues by multisection of Sturm counts
// ---------------------------------------------------------------------------

// Number of eigenvalues of the block [s, t) below x (a and the squared
// off-diagonal e2 in LDS).
__device__ __forceinline__ int sturm_count(const double* a, const double* e2, int s, int t, double x, double pivmin) {
  double q = a[s] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0;
  int k = s + 1;
  for (; k + 8 <= t; k += 8) {  // the LDS reads of 8 steps ahead of their divisions
    double ak[8], ek[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      ak[u] = a[k + u] - x;
      ek[u] = e2[k + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      q = ak[u] - ek[u] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0;
    }
  }
  for (; k < t; ++k) {
    q = (a[k] - x) - e2[k - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// A wave per index i: the (i - s)-th smallest eigenvalue of its block; the
// diagonal and the squared off-diagonal staged in LDS (d <= DMAX).
template <int DMAX>
__global__ __launch_bounds__(256) void tri_eigvals_kernel(const double* __restrict__ a, const double* __restrict__ e,
                                                          int d, const int* __restrict__ bstart,
                                                          const int* __restrict__ bend,
                                                          const TriScal* __restrict__ ts, double* __restrict__ lam) {
  __shared__ double sa[DMAX], se2[DMAX];
  for (int k = threadIdx.x; k < d; k += 256) {
    sa[k] = a[k];
    const double ek = k < d - 1 ? e[k] : 0.0;
    se2[k] = ek * ek;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= d) return;
  const int s = bstart[i], t = bend[i], j = i - s, n = t - s;
  if (n == 1) {
    if (lane == 0) lam[i] = sa[s];
    return;
  }
  const double pivmin = ts->pivmin;
  double gl = HUGE_VAL, gu = -HUGE_VAL;
  for (int k = s + lane; k < t; k += 64) {
    const double r = (k > s ? sqrt(se2[k - 1]) : 0.0) + (k < t - 1 ? sqrt(se2[k]) : 0.0);
    gl = fmin(gl, sa[k] - r);
    gu = fmax(gu, sa[k] + r);
  }
  gl = wave_min(gl);
  gu = wave_max(gu);
  const double tn = fmax(fabs(gl), fabs(gu));
  gl -= 2.0 * kEps * tn * n + 2.0 * pivmin;
  gu += 2.0 * kEps * tn * n + 2.0 * pivmin;
  double lo = gl, hi = gu;
  for (int it = 0; it < 64; ++it) {
    const double x = lo + (hi - lo) * (double(lane + 1) / 65.0);
    const int cnt = sturm_count(sa, se2, s, t, x, pivmin);
    const unsigned long long above = __ballot(cnt > j);  // lanes whose point lies above the eigenvalue
    const int f = above ? __ffsll(above) - 1 : 64;
    const double xl = __shfl(x, f > 0 ? f - 1 : 0, 64), xh = __shfl(x, f < 64 ? f : 63, 64);
    const double nlo = f > 0 ? xl : lo, nhi = f < 64 ? xh : hi;
    lo = nlo;
    hi = nhi;
    if (hi - lo <= 2.0 * kEps * fmax(fabs(lo), fabs(hi)) + pivmin) break;
  }
  if (lane == 0) lam[i] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// 4. Eigenvectors by twisted factorizations
// ---------------------------------------------------------------------------

// Thread i: column i of Z (d x d complex, zero outside the block, written
// as real values).  Scratch: D+ at W[k d + i] and U- at W[d^2 + k d + i];
// the diagonal and off-diagonal staged in LDS (d <= DMAX), the scratch
// read back in batches of 8 so that its loads overlap.
template <int DMAX>
__global__ __launch_bounds__(64) void tri_vectors_kernel(const double* __restrict__ a_g, const double* __restrict__ e_g,
                                                         int d, const int* __restrict__ bstart,
                                                         const int* __restrict__ bend, const TriScal* __restrict__ ts,
                                                         const double* __restrict__ lam, double* __restrict__ W,
                                                         C64* __restrict__ Z) {
  __shared__ double a[DMAX], e[DMAX];
  for (int k = threadIdx.x; k < d; k += 64) {
    a[k] = a_g[k];
    e[k] = k < d - 1 ? e_g[k] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= d) return;
  const int s = bstart[i], t = bend[i];
  if (t - s == 1) {
    Z[int64_t(s) * d + i] = C64{1.0, 0.0};
    return;
  }
  const double pivmin = ts->pivmin, l = lam[i];
  double* Dp = W;
  double* Um = W + int64_t(d) * d;
  // top down: D+_{k+1} = (a_{k+1} - l) - e_k^2 / D+_k
  double dp = a[s] - l;
  if (fabs(dp) < pivmin) dp = -pivmin;
  Dp[int64_t(s) * d + i] = dp;
  for (int k = s; k < t - 1; ++k) {
    const double ek = e[k];
    dp = (a[k + 1] - l) - ek * (ek / dp);
    if (fabs(dp) < pivmin) dp = -pivmin;
    Dp[int64_t(k + 1) * d + i] = dp;
  }
  // bottom up, with the twist index; D+ read back 8 at a time
  double dm = a[t - 1] - l;
  if (fabs(dm) < pivmin) dm = -pivmin;
  double best = fabs(dp);  // gamma_{t-1} = D+_{t-1}
  int r = t - 1;
  for (int k0 = t - 2; k0 >= s; k0 -= 8) {
    double dpb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) dpb[q] = k0 - q >= s ? Dp[int64_t(k0 - q) * d + i] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 - q;
      if (k >= s) {
        const double ek = e[k];
        const double u = ek / dm;
        Um[int64_t(k) * d + i] = u;
        const double ak = a[k] - l;
        dm = ak - u * ek;
        if (fabs(dm) < pivmin) dm = -pivmin;
        const double gam = dpb[q] + dm - ak;
        if (fabs(gam) < best) {
          best = fabs(gam);
          r = k;
        }
      }
    }
  }
  // z_r = 1; z_k = -(e_k / D+_k) z_{k+1} above r, z_{k+1} = -U-_k z_k below
  double nrm = 1.0;
  Z[int64_t(r) * d + i] = C64{1.0, 0.0};
  double z = 1.0;
  for (int k0 = r - 1; k0 >= s; k0 -= 8) {
    double b[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) b[q] = k0 - q >= s ? Dp[int64_t(k0 - q) * d + i] : 1.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 - q;
      if (k >= s) {
        z = -(e[k] / b[q]) * z;
        Z[int64_t(k) * d + i] = C64{z, 0.0};
        nrm += z * z;
      }
    }
  }
  z = 1.0;
  for (int k0 = r; k0 < t - 1; k0 += 8) {
    double b[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) b[q] = k0 + q < t - 1 ? Um[int64_t(k0 + q) * d + i] : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + q;
      if (k < t - 1) {
        z = -b[q] * z;
        Z[int64_t(k + 1) * d + i] = C64{z, 0.0};
        nrm += z * z;
      }
    }
  }
  const double inv = 1.0 / sqrt(nrm);
  for (int k0 = s; k0 < t; k0 += 8) {
    double b[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) b[q] = k0 + q < t ? Z[int64_t(k0 + q) * d + i].re : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (k0 + q < t) Z[int64_t(k0 + q) * d + i].re = b[q] * inv;
  }
}

// ---------------------------------------------------------------------------
// 5. Clusters
// ---------------------------------------------------------------------------

// A deterministic value in [-1, 1) from (i, k) (a 64-bit integer hash).
__device__ __forceinline__ double hash_unit(uint64_t i, uint64_t k) {
  uint64_t x = i * 0x9E3779B97F4A7C15ull + k * 0xBF58476D1CE4E5B9ull;
  x ^= x >> 31;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 29;
  return double(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Solves (T_b - sig I) x = y in place (y: n values), T_b the block of
// (a, e) starting at s, by Gaussian elimination with partial pivoting; dd,
// du, du2: n values each of scratch.  One thread.
__device__ void tri_solve(const double* __restrict__ a, const double* __restrict__ e, int s, int n, double sig,
                          double tiny, double* __restrict__ dd, double* __restrict__ du, double* __restrict__ du2,
                          double* __restrict__ y) {
  for (int k = 0; k < n; ++k) {
    dd[k] = a[s + k] - sig;
    du[k] = k < n - 1 ? e[s + k] : 0.0;
    du2[k] = 0.0;
  }
  for (int k = 0; k < n - 1; ++k) {
    const double ek = e[s + k];
    if (fabs(dd[k]) >= fabs(ek)) {
      if (dd[k] == 0.0) dd[k] = tiny;
      const double m = ek / dd[k];
      dd[k + 1] -= m * du[k];
      y[k + 1] -= m * y[k];
    } else {
      const double m = dd[k] / ek;
      dd[k] = ek;
      const double t = dd[k + 1];
      dd[k + 1] = du[k] - m * t;
      if (k < n - 2) {
        du2[k] = du[k + 1];
        du[k + 1] = -m * du[k + 1];
      }
      du[k] = t;
      const double yk = y[k];
      y[k] = y[k + 1];
      y[k + 1] = yk - m * y[k + 1];
    }
  }
  if (dd[n - 1] == 0.0) dd[n - 1] = tiny;
  y[n - 1] /= dd[n - 1];
  if (n > 1) y[n - 2] = (y[n - 2] - du[n - 2] * y[n - 1]) / dd[n - 2];
  for (int k = n - 3; k >= 0; --k) y[k] = (y[k] - du[k] * y[k + 1] - du2[k] * y[k + 2]) / dd[k];
}

// Workgroup i (64 threads) treats the cluster that starts at index i, if
// one does; 4 n values of scratch at W + 2 d i (clusters start at least two
// indices apart, so the areas do not overlap).
__global__ __launch_bounds__(64) void tri_cluster_kernel(const double* __restrict__ a, const double* __restrict__ e,
                                                         int d, const int* __restrict__ bstart,
                                                         const int* __restrict__ bend, const TriScal* __restrict__ ts,
                                                         const double* __restrict__ lam, double* __restrict__ W,
                                                         C64* __restrict__ Z) {
  const int i = blockIdx.x, lane = threadIdx.x;
  const int s = bstart[i], t = bend[i], n = t - s;
  if (n < 2) return;
  const double tn = ts->tnorm, gap = kClusterTol * tn;
  const bool starts = (i == s || lam[i] - lam[i - 1] > gap) && i + 1 < t && lam[i + 1] - lam[i] <= gap;
  if (!starts) return;
  int c = 1;
  while (i + c < t && lam[i + c] - lam[i + c - 1] <= gap) ++c;
  double* dd = W + int64_t(2) * d * i;
  double* du = dd + n;
  double* du2 = du + n;
  double* y = du2 + n;
  const double pert = 10.0 * kEps * tn, tiny = kEps * tn;
  double prev = -HUGE_VAL;
  for (int m = 0; m < c; ++m) {
    double sig = lam[i + m];
    if (m > 0 && sig - prev < pert) sig = prev + pert;
    prev = sig;
    for (int k = lane; k < n; k += 64) y[k] = hash_unit(uint64_t(i + m), uint64_t(k));
    for (int it = 0; it < 3; ++it) {
      __syncthreads();
      if (lane == 0) tri_solve(a, e, s, n, sig, tiny, dd, du, du2, y);
      __syncthreads();
      for (int q = 0; q < m; ++q) {  // orthogonalise against the earlier members
        const C64* zq = Z + int64_t(s) * d + (i + q);
        double dot = 0.0;
        for (int k = lane; k < n; k += 64) dot += zq[int64_t(k) * d].re * y[k];
        dot = wave_sum(dot);
        for (int k = lane; k < n; k += 64) y[k] -= dot * zq[int64_t(k) * d].re;
      }
      double nrm = 0.0;
      for (int k = lane; k < n; k += 64) nrm += y[k] * y[k];
      nrm = wave_sum(nrm);
      const double inv = 1.0 / sqrt(nrm);
      for (int k = lane; k < n; k += 64) y[k] *= inv;
    }
    C64* zm = Z + int64_t(s) * d + (i + m);
    for (int k = lane; k < n; k += 64) zm[int64_t(k) * d] = C64{y[k], 0.0};
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 6. Newton-Schulz matrix, fills
// ---------------------------------------------------------------------------

// M = 1.5 I - 0.5 G (d x d contiguous).
__global__ __launch_bounds__(256) void ns_matrix_kernel(const C64* __restrict__ G, C64* __restrict__ M, int n) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= (int64_t(1) << (2 * n))) return;
  const int64_t r = e >> n, c = e & ((int64_t(1) << n) - 1);
  const C64 g = G[e];
  M[e] = C64{(r == c ? 1.5 : 0.0) - 0.5 * g.re, -0.5 * g.im};
}

__global__ __launch_bounds__(256) void zero_kernel(C64* __restrict__ X, int64_t count) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e < count) X[e] = C64{0.0, 0.0};
}

// ---------------------------------------------------------------------------
// 7. Back-transformation
// ---------------------------------------------------------------------------

constexpr int kNb = kEighBlock;  // 64
constexpr int kGramRows = kEighGramRows;

// v_{k0 + j}[r] from the reflector rows (0 at and above the diagonal).
__device__ __forceinline__ C64 refl(const C64* __restrict__ V, int d, int k0, int j, int nk, int r) {
  const int k = k0 + j;
  if (j >= nk || r <= k || r >= d) return C64{0.0, 0.0};
  return V[int64_t(k) * d + r];
}

// Partial Gram matrices of the blocks' reflectors: workgroup (b, y) sums
// conj(v_j[r]) v_l[r] over the rows r of chunk y (kGramRows rows from
// k0 + 1) into Gp[(b * gchunks + y)][j][l].
__global__ __launch_bounds__(256) void bt_gram_kernel(const C64* __restrict__ V, int d, int gchunks,
                                                      C64* __restrict__ Gp) {
  __shared__ C64 ch[32][kNb + 1];
  const int b = blockIdx.x, y = blockIdx.y, tid = threadIdx.x;
  const int k0 = b * kNb, nk = min(kNb, d - 1 - k0);
  const int rs = k0 + 1 + y * kGramRows, re = min(d, rs + kGramRows);
  const int tj = tid >> 4, tl = tid & 15;  // entries (4 tj + x, 4 tl + y)
  C64 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int z = 0; z < 4; ++z) acc[x][z] = C64{0.0, 0.0};
  for (int r0 = rs; r0 < re; r0 += 32) {
    __syncthreads();
    for (int q = tid; q < 32 * kNb; q += 256) {
      const int j = q >> 5, rr = q & 31, r = r0 + rr;
      ch[rr][j] = r < re ? refl(V, d, k0, j, nk, r) : C64{0.0, 0.0};
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < 32; ++rr) {
      C64 u[4], w[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        u[x] = ch[rr][4 * tj + x];
        w[x] = ch[rr][4 * tl + x];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int z = 0; z < 4; ++z) {
          const C64 p = cmulc(u[x], w[z]);
          acc[x][z].re += p.re;
          acc[x][z].im += p.im;
        }
    }
  }
  C64* G = Gp + (int64_t(b) * gchunks + y) * kNb * kNb;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int z = 0; z < 4; ++z) G[(4 * tj + x) * kNb + 4 * tl + z] = acc[x][z];
}

// Workgroup b: G = the sum of block b's partial Gram matrices (fixed
// order), then the triangular factor column by column:
// T[j][j] = tau_j, T[0:j][j] = -tau_j T[0:j][0:j] G[0:j][j].
__global__ __launch_bounds__(256) void bt_tmat_kernel(const C64* __restrict__ Gp, int gchunks,
                                                      const C64* __restrict__ tau, int d, C64* __restrict__ Tall) {
  __shared__ C64 gt[kNb][kNb + 1];  // G, then T in place
  __shared__ C64 tmp[kNb];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int k0 = b * kNb, nk = min(kNb, d - 1 - k0);
  for (int q = tid; q < kNb * kNb; q += 256) {
    C64 g{0.0, 0.0};
    for (int y = 0; y < gchunks; ++y) {
      const C64 v = Gp[(int64_t(b) * gchunks + y) * kNb * kNb + q];
      g.re += v.re;
      g.im += v.im;
    }
    gt[q >> 6][q & 63] = g;
  }
  __syncthreads();
  for (int j = 0; j < kNb; ++j) {
    const C64 tj_ = j < nk ? tau[k0 + j] : C64{0.0, 0.0};
    C64 sum{0.0, 0.0};
    if (tid < j) {
      for (int q = tid; q < j; ++q) {
        const C64 p = cmul(gt[tid][q], gt[q][j]);  // T[tid][q] G[q][j]
        sum.re += p.re;
        sum.im += p.im;
      }
    }
    __syncthreads();
    if (tid < kNb) {
      C64 v;
      if (tid < j) {
        const C64 p = cmul(tj_, sum);
        v = C64{-p.re, -p.im};
      } else if (tid == j) {
        v = tj_;
      } else {
        v = C64{0.0, 0.0};
      }
      tmp[tid] = v;
    }
    __syncthreads();
    if (tid < kNb) gt[tid][j] = tmp[tid];
    __syncthreads();
  }
  C64* T = Tall + int64_t(b) * kNb * kNb;
  for (int q = tid; q < kNb * kNb; q += 256) T[q] = gt[q >> 6][q & 63];
}

// W_b = V_b T_b, stored like the reflectors: W[(k0 + j) d + r] =
// sum_{l <= j} v_{k0 + l}[r] T_b[l][j] for r in [k0 + 1, d) (workgroup (b,
// y): rows k0 + 1 + 64 y ...).
__global__ __launch_bounds__(256) void bt_wfactor_kernel(const C64* __restrict__ V, const C64* __restrict__ Tall,
                                                         int d, C64* __restrict__ W) {
  __shared__ C64 vs[64][kNb + 1];  // [row][l]
  __shared__ C64 ts[kNb][kNb + 1];  // [l][j]
  const int b = blockIdx.x, tid = threadIdx.x;
  const int k0 = b * kNb, nk = min(kNb, d - 1 - k0);
  const int r0 = k0 + 1 + blockIdx.y * 64;
  if (r0 >= d) return;
  for (int q = tid; q < 64 * kNb; q += 256) {
    const int l = q >> 6, rr = q & 63;
    vs[rr][l] = refl(V, d, k0, l, nk, r0 + rr);
    ts[q >> 6][q & 63] = Tall[int64_t(b) * kNb * kNb + q];
  }
  __syncthreads();
  const int tr = tid >> 4, tc = tid & 15;  // rows 4 tr + x, columns j = 4 tc + z
  C64 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int z = 0; z < 4; ++z) acc[x][z] = C64{0.0, 0.0};
  for (int l = 0; l < kNb; ++l) {
    C64 u[4], w[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      u[x] = vs[4 * tr + x][l];
      w[x] = ts[l][4 * tc + x];
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 4; ++z) {
        const C64 p = cmul(u[x], w[z]);
        acc[x][z].re += p.re;
        acc[x][z].im += p.im;
      }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int r = r0 + 4 * tr + x;
    if (r >= d) continue;
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const int j = 4 * tc + z;
      if (j < nk) W[int64_t(k0 + j) * d + r] = acc[x][z];
    }
  }
}

// Partial sums of V_b^dagger Z over the row chunk y of R rows (rows from
// k0 + 1): P[y][j][c] for j < 64 and the column tile x of 64.
__global__ __launch_bounds__(256) void bt_partial_kernel(const C64* __restrict__ V, const C64* __restrict__ Z, int d,
                                                         int k0, int nk, int R, C64* __restrict__ P) {
  __shared__ C64 vs[16][kNb + 1];
  __shared__ C64 zs[16][kNb + 1];
  const int tid = threadIdx.x, tj = tid >> 4, tc = tid & 15;
  const int c0 = blockIdx.x * 64, rs = k0 + 1 + blockIdx.y * R, re = min(d, rs + R);
  C64 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = C64{0.0, 0.0};
  for (int r0 = rs; r0 < re; r0 += 16) {
    __syncthreads();
    for (int q = tid; q < 16 * kNb; q += 256) {
      const int j = q >> 4, rr = q & 15, r = r0 + rr;
      vs[rr][j] = r < re ? refl(V, d, k0, j, nk, r) : C64{0.0, 0.0};
      const int rz = q >> 6, cz = q & 63, r2 = r0 + rz, c = c0 + cz;
      zs[rz][cz] = (r2 < re && c < d) ? Z[int64_t(r2) * d + c] : C64{0.0, 0.0};
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < 16; ++rr) {
      C64 u[4], w[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        u[x] = vs[rr][4 * tj + x];
        w[x] = zs[rr][4 * tc + x];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const C64 p = cmulc(u[x], w[y]);
          acc[x][y].re += p.re;
          acc[x][y].im += p.im;
        }
    }
  }
  C64* out = P + int64_t(blockIdx.y) * kNb * d;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int c = c0 + 4 * tc + y;
      if (c < d) out[int64_t(4 * tj + x) * d + c] = acc[x][y];
    }
}

// X[j][c] = sum_y P[y][j][c] (64 d entries, fixed order).
__global__ __launch_bounds__(256) void bt_sum_kernel(const C64* __restrict__ P, int chunks, int d,
                                                     C64* __restrict__ X) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t count = int64_t(kNb) * d;
  if (e >= count) return;
  C64 s{0.0, 0.0};
  for (int y = 0; y < chunks; ++y) {
    const C64 v = P[int64_t(y) * count + e];
    s.re += v.re;
    s.im += v.im;
  }
  X[e] = s;
}

// Z[r][c] -= sum_j w_{k0 + j}[r] X[j][c] on the tile (rows k0 + 1 + 64 y,
// columns 64 x), W = V_b T_b as bt_wfactor_kernel stores it.
__global__ __launch_bounds__(256) void bt_update_kernel(const C64* __restrict__ W, const C64* __restrict__ X, int d,
                                                        int k0, int nk, C64* __restrict__ Z) {
  __shared__ C64 vs[64][17];
  __shared__ C64 xs[16][65];
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const int r0 = k0 + 1 + blockIdx.y * 64, c0 = blockIdx.x * 64;
  C64 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = C64{0.0, 0.0};
  for (int j0 = 0; j0 < kNb; j0 += 16) {
    __syncthreads();
    for (int q = tid; q < 64 * 16; q += 256) {
      const int jj = q >> 6, rr = q & 63;
      const int j = j0 + jj, r = r0 + rr;
      vs[rr][jj] = (j < nk && r < d) ? W[int64_t(k0 + j) * d + r] : C64{0.0, 0.0};
      const int cc = q & 63, c = c0 + cc;
      xs[jj][cc] = c < d ? X[int64_t(j0 + jj) * d + c] : C64{0.0, 0.0};
    }
    __syncthreads();
#pragma unroll 4
    for (int jj = 0; jj < 16; ++jj) {
      C64 u[4], w[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        u[x] = vs[4 * tr + x][jj];
        w[x] = xs[jj][4 * tc + x];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const C64 p = cmul(u[x], w[y]);
          acc[x][y].re += p.re;
          acc[x][y].im += p.im;
        }
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int r = r0 + 4 * tr + x;
    if (r >= d) continue;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int c = c0 + 4 * tc + y;
      if (c < d) {
        C64& z = Z[int64_t(r) * d + c];
        z.re -= acc[x][y].re;
        z.im -= acc[x][y].im;
      }
    }
  }
}

__global__ void status_out_kernel(const TriScal* __restrict__ ts, int* __restrict__ out) { *out = ts->status; }

// Workgroups of a reduction step: one row per wave at the first step (256
// threads up to d = 1024, 512 at 2048, 1024 beyond, so at most 256 groups).
int trd_groups(int d) {
  const int waves = d <= 1024 ? 4 : (d <= 2048 ? 8 : 16);
  const int g = (d + waves - 1) / waves;
  return g > kTrdMaxGroups ? kTrdMaxGroups : g;
}

}  // namespace

EighWork eigh_work(int n, void* eig_area) {
  const EighLayout L = eigh_layout(n);
  unsigned char* w = static_cast<unsigned char*>(eig_area);
  EighWork e;
  e.diag = reinterpret_cast<double*>(w + L.diag);
  e.off = reinterpret_cast<double*>(w + L.off);
  e.tau = w + L.tau;
  e.y0 = w + L.y0;
  e.y1 = w + L.y1;
  e.p0 = reinterpret_cast<double*>(w + L.p0);
  e.p1 = reinterpret_cast<double*>(w + L.p1);
  e.bstart = reinterpret_cast<int*>(w + L.bstart);
  e.bend = reinterpret_cast<int*>(w + L.bend);
  e.scal = w + L.scal;
  e.status = reinterpret_cast<int*>(w + L.scal + offsetof(TriScal, status));
  e.tfac = w + L.tfac;
  e.pbuf = w + L.pbuf;
  e.xbuf = w + L.xbuf;
  return e;
}

hipError_t launch_tridiagonalize(int n, void* A, void* V, const EighWork& w, hipStream_t s) {
  const int d = 1 << n, P = trd_groups(d);
  TrdArgs g{static_cast<C64*>(A), static_cast<C64*>(V), w.diag, w.off, static_cast<C64*>(w.tau), d, P};
  C64* y[2] = {static_cast<C64*>(w.y0), static_cast<C64*>(w.y1)};
  double* p[2] = {w.p0, w.p1};
  for (int k = 0; k <= d - 2; ++k) {
    const int a = k & 1, b = a ^ 1;  // step k reads y[b], p[b] (step k - 1) and writes y[a], p[a]
    if (d <= 512)
      trd_step_kernel<512, 256, true><<<P, 256, 0, s>>>(g, k, y[b], y[a], p[b], p[a]);
    else if (d <= 1024)
      trd_step_kernel<1024, 256, true><<<P, 256, 0, s>>>(g, k, y[b], y[a], p[b], p[a]);
    else if (d <= 2048)
      trd_step_kernel<2048, 512, true><<<P, 512, 0, s>>>(g, k, y[b], y[a], p[b], p[a]);
    else
      trd_step_kernel<8192, 1024, false><<<P, 1024, 0, s>>>(g, k, y[b], y[a], p[b], p[a]);
  }
  const int last = (d - 2) & 1;
  trd_last_kernel<<<1, kTrdThreads, 0, s>>>(g, y[last], p[last]);
  return hipGetLastError();
}

hipError_t launch_tri_eigvals(int n, const EighWork& w, double* lam, hipStream_t s) {
  const int d = 1 << n;
  TriScal* ts = static_cast<TriScal*>(w.scal);
  tri_split_kernel<<<1, 256, 0, s>>>(w.diag, w.off, d, w.bstart, w.bend, ts);
  if (d <= 2048)
    tri_eigvals_kernel<2048><<<(d + 3) / 4, 256, 0, s>>>(w.diag, w.off, d, w.bstart, w.bend, ts, lam);
  else
    tri_eigvals_kernel<8192><<<(d + 3) / 4, 256, 0, s>>>(w.diag, w.off, d, w.bstart, w.bend, ts, lam);
  return hipGetLastError();
}

hipError_t launch_tri_vectors(int n, const EighWork& w, const double* lam, void* scratch, void* Z, hipStream_t s) {
  const int d = 1 << n;
  const int64_t count = int64_t(d) * d;
  const TriScal* ts = static_cast<const TriScal*>(w.scal);
  zero_kernel<<<unsigned((count + 255) / 256), 256, 0, s>>>(static_cast<C64*>(Z), count);
  if (d <= 2048)
    tri_vectors_kernel<2048><<<(d + 63) / 64, 64, 0, s>>>(w.diag, w.off, d, w.bstart, w.bend, ts, lam,
                                                          static_cast<double*>(scratch), static_cast<C64*>(Z));
  else
    tri_vectors_kernel<8192><<<(d + 63) / 64, 64, 0, s>>>(w.diag, w.off, d, w.bstart, w.bend, ts, lam,
                                                          static_cast<double*>(scratch), static_cast<C64*>(Z));
  tri_cluster_kernel<<<d, 64, 0, s>>>(w.diag, w.off, d, w.bstart, w.bend, ts, lam, static_cast<double*>(scratch),
                                      static_cast<C64*>(Z));
  return hipGetLastError();
}

hipError_t launch_ns_matrix(int n, const void* G, void* M, hipStream_t s) {
  const int64_t count = int64_t(1) << (2 * n);
  ns_matrix_kernel<<<unsigned((count + 255) / 256), 256, 0, s>>>(static_cast<const C64*>(G), static_cast<C64*>(M), n);
  return hipGetLastError();
}

hipError_t launch_back_transform(int n, const void* V, const EighWork& w, void* Z, void* Wbuf, hipStream_t s) {
  const int d = 1 << n;
  const int blocks = (d - 1 + kNb - 1) / kNb;
  const C64* v = static_cast<const C64*>(V);
  C64* T = static_cast<C64*>(w.tfac);
  C64* Wm = static_cast<C64*>(Wbuf);
  C64* P = static_cast<C64*>(w.pbuf);
  const int gchunks = eigh_gram_chunks(d);
  bt_gram_kernel<<<dim3(blocks, gchunks), 256, 0, s>>>(v, d, gchunks, P);
  bt_tmat_kernel<<<blocks, 256, 0, s>>>(P, gchunks, static_cast<const C64*>(w.tau), d, T);
  bt_wfactor_kernel<<<dim3(blocks, unsigned((d + 63) / 64)), 256, 0, s>>>(v, T, d, Wm);
  const int R = eigh_chunk_rows(d);
  const unsigned ct = unsigned((d + 63) / 64);
  const unsigned sum_blocks = unsigned((int64_t(kNb) * d + 255) / 256);
  for (int b = blocks - 1; b >= 0; --b) {
    const int k0 = b * kNb, nk = d - 1 - k0 < kNb ? d - 1 - k0 : kNb;
    const int m = d - 1 - k0;  // rows k0 + 1 .. d - 1
    const int chunks = (m + R - 1) / R;
    bt_partial_kernel<<<dim3(ct, chunks), 256, 0, s>>>(v, static_cast<const C64*>(Z), d, k0, nk, R, P);
    bt_sum_kernel<<<sum_blocks, 256, 0, s>>>(P, chunks, d, static_cast<C64*>(w.xbuf));
    bt_update_kernel<<<dim3(ct, unsigned((m + 63) / 64)), 256, 0, s>>>(Wm, static_cast<const C64*>(w.xbuf), d, k0,
                                                                       nk, static_cast<C64*>(Z));
  }
  return hipGetLastError();
}

hipError_t launch_eigh_status(const EighWork& w, int* out, hipStream_t s) {
  status_out_kernel<<<1, 1, 0, s>>>(static_cast<const TriScal*>(w.scal), out);
  return hipGetLastError();
}

}  // namespace qst
