// Batched form: many independent tomography instances of mixed qubit counts
// (N = 1..8) -- forward and adjoint of each -- in ONE persistent launch.
//
// A grid of CUs x occupancy workgroups pulls instance indices from an integer
// work counter, in descending cost order (largest d first, a greedy longest-
// processing-time schedule).  One workgroup carries one instance through
// every step of the path:
//   tau (FP64 block reduction) -> T T^dagger / tau (MFMA tiles of the product
//   kernels, or per-entry loops below d = 64) -> POVM passes -> L, F (FP64
//   block reduction) -> cotangent + adjoint passes -> (2/tau) G' T,
// keeping rho / G', the POVM intermediate and p in a per-workgroup scratch
// region.  Every reduction has a fixed order, so results do not depend on
// which workgroup takes which instance.
//
// The host plan (qst_batch_plan_*) owns the descriptor table, the work
// counter, the scratch and an optional HIP graph of (counter reset + kernel),
// and picks the launch shape with a small autotuner whose choices can be
// cached in a text file: the grid size, the instance order, the workgroup
// size (FP32: 512 threads with two product tiles at a time, or 256 with
// one) and the POVM pass plan of N = 7, 8 (the register-round pair of
// passes with the fused likelihood, or the generic per-qubit passes).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "qst_gemm_tiles.h"
#include "qst_kernels.h"
#include "qst_plan.h"
#include "qst_povm_fast.h"
#include "qst_povm_generic.h"

namespace qst {

namespace {

constexpr int kBatchMaxQubits = 8;

struct BatchItem {
  int n;
  int pad;
  int64_t t_off;  // complex elements into T_all / grad_all
  int64_t f_off;  // reals into f_all
};

struct BatchPlanTable {
  int passes[kBatchMaxQubits + 1];
  int g[kBatchMaxQubits + 1][4];
  int U[kBatchMaxQubits + 1][4];
  int J[kBatchMaxQubits + 1][4];
};

struct BatchArgs {
  const BatchItem* items;
  const int* order;
  int count;
  int* counter;
  const void* T_all;
  const void* f_all;
  double* nll_out;              // [count][2]
  unsigned long long* bad_out;  // [count][2] or NULL
  void* grad_all;
  unsigned char* scratch;
  int64_t stride;  // bytes of scratch per workgroup
  int nmax;
  int fast_forms;  // 1: the register-round pass forms where a plan has one; 0: generic passes
  BatchPlanTable plan;
  ModeMatrix W, V;
};

__global__ void reset_counter_kernel(int* c) { *c = 0; }

// Block-wide FP64 sum over NW waves (wave trees, then the wave sums in
// order), result broadcast to every thread.
template <int NW>
__device__ double block_sum_bcast(double v, double* redw, double* slot) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) redw[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = redw[0];
    for (int i = 1; i < NW; ++i) s += redw[i];
    *slot = s;
  }
  __syncthreads();
  const double r = *slot;
  __syncthreads();
  return r;
}

// Product tiles of the batched kernel: two LDS panel buffers, since the
// 256-thread groups of a workgroup meet at every barrier.
template <typename R>
using BatchHerk = gemm::CxPolicy<R, true, true, true>;
template <typename R>
using BatchHemm = gemm::CxPolicy<R, false, true, true>;

// Barrier after one call of a generic POVM pass.  Between calls of a pass
// that reads another array than it writes, only the LDS buffer is reused:
// fences that order LDS accesses alone (the call's global stores need not
// complete before the next call starts).  After the last call, or when a
// pass reads the array it writes, the full barrier makes the stores
// visible to the whole workgroup.
__device__ __forceinline__ void pass_call_barrier(const PassArgs& a, bool more) {
  if (more && a.in != a.out) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  } else {
    __syncthreads();
  }
}

// Which register-round form covers an instance's POVM plan: 4 (pass 0 over
// 4 qubits, pass 1 over 4 with J = 32 / 16 for FP32 / FP64, N = 8), 3 (4 then
// 3 with J = 64, N = 7), or 0 (the generic passes).
__device__ __forceinline__ int fast_plan(const BatchPlanTable& pl, int n, bool f64) {
  if (pl.passes[n] != 2 || pl.g[n][0] != 4 || pl.J[n][0] != 1) return 0;
  if (pl.g[n][1] == 4 && pl.J[n][1] == (f64 ? 16 : 32)) return 4;
  if (pl.g[n][1] == 3 && pl.J[n][1] == 64) return 3;
  return 0;
}

// Pass args of pass pj of instance n.
__device__ __forceinline__ PassArgs pass_args(const BatchPlanTable& pl, int n, int pj) {
  PassArgs a{};
  a.n = n;
  a.U = pl.U[n][pj];
  a.g = pl.g[n][pj];
  a.J = pl.J[n][pj];
  a.ld = 1 << n;
  return a;
}

// Register-round passes of the two-pass plans.  The SUB 256-thread groups
// of the workgroup take calls sub, sub + SUB, ... of a pass; the call count
// is rounded up to a multiple of SUB (a padding call stores and counts
// nothing), so every group meets the same barriers.  The barrier after
// each call protects the group's LDS area for the next call; the last one
// also makes the pass's stores visible to the next stage.  (The empty asm
// keeps the compiler from hoisting the thread-index arithmetic of the
// unrolled pass bodies out of the call loop, which kept it all live in
// registers across the calls and spilled.)
//
// Pass 0 over 4 qubits: rho -> X (forward) or Y -> G' (adjoint).
template <typename R, bool ADJ, bool TETRA, int SUB, int POOL>
__device__ __forceinline__ void fast_pass0(const BatchArgs& b, int n, Cx<R>* rho, Cx<R>* inter, unsigned char* pool,
                                           int sub, unsigned tid) {
  constexpr int TPW = 256 >> 4;  // tiles of pass 0 (G = 4) per 256 threads
  typedef Cx<R> Lds[TPW << 8];
  static_assert(SUB * sizeof(Lds) <= size_t(POOL), "one pass buffer per 256-thread group must fit the pool");
  PassArgs a = pass_args(b.plan, n, 0);
  a.in = ADJ ? inter : rho;
  a.out = ADJ ? rho : inter;
  const int64_t side = int64_t(1) << (a.U - 4);
  const int64_t tiles = side * (side + 1) / 2;
  const int64_t calls = (tiles + TPW - 1) / TPW;
  Lds& L = reinterpret_cast<Lds*>(pool)[sub];
  for (int64_t c = sub; c < (calls + SUB - 1) / SUB * SUB; c += SUB) {
    unsigned tv = tid;
    asm volatile("" : "+v"(tv));
    fast_pass::mat_pass_body<R, ADJ, TETRA, 4>(a, ADJ ? b.V : b.W, tiles, c, tv, L);
    __syncthreads();
  }
}

// Last pass fused with the likelihood (G1 qubits, chunks of J1): X -> p in
// registers -> NLL terms (added to L, bad0, bad1) and the cotangent
// F - f/p -> adjoint rounds -> Y, in place of X.
template <typename R, bool TETRA, int G1, int J1, int SUB, int POOL>
__device__ __forceinline__ void fast_fused(const BatchArgs& b, int n, Cx<R>* inter, const R* f, double F,
                                           unsigned char* pool, int sub, unsigned tid, double& L, double& bad0,
                                           double& bad1) {
  typedef Cx<R> Lds[J1 << (2 * G1)];
  static_assert(SUB * sizeof(Lds) <= size_t(POOL), "one pass buffer per 256-thread group must fit the pool");
  PassArgs a = pass_args(b.plan, n, 1);
  a.in = inter;
  a.out = inter;
  a.f = f;
  const int64_t calls = (int64_t(1) << (2 * (n - a.U))) / J1;  // one (R, C) pair: the chunks
  Lds& Lb = reinterpret_cast<Lds*>(pool)[sub];
  for (int64_t c = sub; c < (calls + SUB - 1) / SUB * SUB; c += SUB) {
    unsigned tv = tid;
    asm volatile("" : "+v"(tv));
    fast_pass::kd_fused_body<R, TETRA, G1, J1>(a, b.W, b.V, c < calls ? c : calls - 1, tv, Lb, c < calls, F, L, bad0,
                                               bad1);
    __syncthreads();
  }
}

template <typename R, bool TETRA, int SUB, int POOL>
__device__ __forceinline__ void fast_fused_form(const BatchArgs& b, int n, int form, Cx<R>* inter, const R* f,
                                                double F, unsigned char* pool, int sub, unsigned tid, double& L,
                                                double& bad0, double& bad1) {
  constexpr int J4 = sizeof(R) == 8 ? 16 : 32;
  if (form == 4)
    fast_fused<R, TETRA, 4, J4, SUB, POOL>(b, n, inter, f, F, pool, sub, tid, L, bad0, bad1);
  else
    fast_fused<R, TETRA, 3, 64, SUB, POOL>(b, n, inter, f, F, pool, sub, tid, L, bad0, bad1);
}

template <bool BF16>
constexpr int kBatchPoolBytes = BF16 ? 65536 : 131072;

// THREADS = 256 x SUB: the element loops use every thread; the product
// stages run SUB tiles at a time, one per 256-thread group, each with its own
// panel buffers.  Every group makes the same number of tile calls (a tile
// list is padded to a multiple of SUB; a padding call recomputes tile 0 and
// stores nothing), so the barriers inside the tile code stay matched.
template <class PH, class PM, typename R, bool TETRA, bool BF16, int THREADS>
__global__ __launch_bounds__(THREADS) void batch_kernel(BatchArgs b) {
  constexpr int SUB = THREADS / 256, NW = THREADS / 64;
  // POVM element loops: values loaded per thread before any is stored, as
  // many as the registers allow (FP32 at 512 threads: 16; FP64: 8)
  constexpr int kPassLoads = THREADS == 512 ? 16 : (sizeof(R) == 8 ? 8 : generic_pass::kLoadBatch);
  // One LDS pool serves, one stage at a time, the product panels, the POVM
  // pass buffer and the reduction scratch (red, slot, s_idx).  Where the
  // registers already hold the kernel to one workgroup per CU (FP32 at 512
  // threads, FP64) it takes 128 KiB, so a POVM pass needs half the calls;
  // BF16 keeps 64 KiB and two workgroups per CU.
  __shared__ __align__(16) unsigned char pool[kBatchPoolBytes<BF16>];
  static_assert(sizeof(typename PH::Smem) <= sizeof(pool) && sizeof(typename PM::Smem) <= sizeof(pool) &&
                    sizeof(gemm::HerkBf16x3Policy::Smem) <= sizeof(pool),
                "product panels exceed the LDS pool");
  static_assert(SUB * sizeof(typename PH::Smem) <= sizeof(pool) && SUB * sizeof(typename PM::Smem) <= sizeof(pool),
                "one set of panel buffers per 256-thread group must fit the pool");
  double* const red = reinterpret_cast<double*>(pool);
  double* const slotp = red + NW;
  int* const s_idx_p = reinterpret_cast<int*>(red + NW + 1);
  const int sub = threadIdx.x >> 8;
  const int t = threadIdx.x;
  const int64_t dmax = int64_t(1) << b.nmax, Dmax = dmax * dmax;
  unsigned char* scr = b.scratch + int64_t(blockIdx.x) * b.stride;
  Cx<R>* rho = reinterpret_cast<Cx<R>*>(scr);            // rho, then G'
  Cx<R>* inter = rho + Dmax;                             // POVM intermediate
  R* pvec = reinterpret_cast<R*>(inter + Dmax);          // p
  double* Fdev = reinterpret_cast<double*>(pvec + Dmax);  // F for the cotangent

  for (;;) {
    if (t == 0) *s_idx_p = atomicAdd(b.counter, 1);
    __syncthreads();
    const int idx = *s_idx_p;
    __syncthreads();
    if (idx >= b.count) break;
    const int j = b.order[idx];
    const BatchItem it = b.items[j];
    const int n = it.n;
    const int d = 1 << n;
    const int64_t D = int64_t(d) * d;
    const Cx<R>* T = static_cast<const Cx<R>*>(b.T_all) + it.t_off;
    const R* f = static_cast<const R*>(b.f_all) + it.f_off;
    Cx<R>* grad = static_cast<Cx<R>*>(b.grad_all) + it.t_off;

    // 1. tau = sum |T|^2 (FP64, over bf16-rounded T for the BF16 path)
    // (kBatch loads per thread in flight, unconditional: indices past the
    // end are clamped and their values dropped; 16 for FP32 at 512 threads,
    // whose registers allow it)
    // The sum of f (D = 4^n values, as many as T has) is taken in the same
    // loop, in the order of the likelihood stage's own sum: the fused last
    // pass needs F for the cotangent before any probability exists.
    constexpr int kBatch = (THREADS == 512 && sizeof(R) == 4) ? 16 : 4;
    // the two-pass plans of N = 7, 8 run the register-round passes, with the
    // last pass fused with the likelihood (for the tetrahedral POVM in FP32
    // and FP64: with the general 4 x 4 form, or beside the BF16 products,
    // they would cost registers -- spills, or the second BF16 workgroup per CU)
    const int fastp = (TETRA && !BF16 && b.fast_forms) ? fast_plan(b.plan, n, sizeof(R) == 8) : 0;
    double acc = 0.0, facc = 0.0;
    for (int64_t e0 = 0; e0 < D; e0 += kBatch * THREADS) {
      Cx<R> v[kBatch];
      R fv[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int64_t e = e0 + u * THREADS + t;
        v[u] = T[e < D ? e : D - 1];
        fv[u] = f[e < D ? e : D - 1];
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        if (e0 + u * THREADS + t >= D) continue;
        facc += double(fv[u]);
        double x = double(v[u].re), y = double(v[u].im);
        if constexpr (BF16) {
          const float hr = bf16_value(float(v[u].re)), hi = bf16_value(float(v[u].im));
          if (d <= kBf16SplitMaxDim) {  // split bf16 hi + lo
            x = double(hr + bf16_value(float(v[u].re) - hr));
            y = double(hi + bf16_value(float(v[u].im) - hi));
          } else {
            x = double(hr);
            y = double(hi);
          }
        }
        acc += x * x + y * y;
      }
    }
    const double tau = block_sum_bcast<NW>(acc, red, slotp);
    const double Fsum = block_sum_bcast<NW>(facc, red, slotp);

    // 2. rho = T T^dagger / tau
    if (BF16 && d >= 64 && d <= kBf16SplitMaxDim) {
      gemm::GemmArgs g{};
      g.A = T;
      g.lda = d;
      g.B = T;
      g.ldb = d;
      g.C = rho;
      g.ldc = d;
      g.d = d;
      g.kIters = d / gemm::HerkBf16x3Policy::KP;
      const int tiles = d / 64;
      for (int tile = 0; tile < tiles * (tiles + 1) / 2; ++tile) {
        int tr, tc;
        tri_decode(tile, tr, tc);
        f4 aR[2][2], aI[2][2];
        gemm::zero_acc<gemm::HerkBf16x3Policy>(aR, aI);
        gemm::HerkBf16x3Policy::run(g, *reinterpret_cast<gemm::HerkBf16x3Policy::Smem*>(pool), tr, tc, 0,
                                    g.kIters, aR, aI);
        gemm::epilogue<gemm::HerkBf16x3Policy>(g, tr, tc, aR, aI, 1.0 / tau);
      }
    } else if (d >= 64) {
      gemm::GemmArgs g{};
      g.A = T;
      g.lda = d;
      g.B = T;
      g.ldb = d;
      g.C = rho;
      g.ldc = d;
      g.d = d;
      g.kIters = d / PH::KP;
      const int tiles = d / 64, ntl = tiles * (tiles + 1) / 2;
      auto& sm = reinterpret_cast<typename PH::Smem*>(pool)[sub];
      for (int t0 = 0; t0 < ntl; t0 += SUB) {
        const int tile = t0 + sub;
        int tr, tc;
        tri_decode(tile < ntl ? tile : 0, tr, tc);
        typename PH::acc_t aR[2][2], aI[2][2];
        gemm::zero_acc<PH>(aR, aI);
        PH::run(g, sm, tr, tc, 0, g.kIters, aR, aI);
        if (tile < ntl) gemm::epilogue<PH>(g, tr, tc, aR, aI, 1.0 / tau);
      }
    } else {
      for (int64_t e = t; e < D; e += THREADS) {
        const int r = int(e >> n), c = int(e & (d - 1));
        R sr = 0, si = 0;
        for (int k = 0; k < d; ++k) {
          const Cx<R> x = T[int64_t(r) * d + k], y = T[int64_t(c) * d + k];
          if constexpr (BF16) {  // d < 64: split bf16 x 3
            const float ahr = bf16_value(float(x.re)), ahi = bf16_value(float(x.im));
            const float alr = bf16_value(float(x.re) - ahr), ali = bf16_value(float(x.im) - ahi);
            const float bhr = bf16_value(float(y.re)), bhi = bf16_value(float(y.im));
            const float blr = bf16_value(float(y.re) - bhr), bli = bf16_value(float(y.im) - bhi);
            sr += (ahr * bhr + ahi * bhi) + (ahr * blr + ahi * bli) + (alr * bhr + ali * bhi);
            si += (ahi * bhr - ahr * bhi) + (ahi * blr - ahr * bli) + (ali * bhr - alr * bhi);
          } else {
            sr += x.re * y.re + x.im * y.im;
            si += x.im * y.re - x.re * y.im;
          }
        }
        rho[e] = Cx<R>{R(sr / tau), R(si / tau)};
      }
    }
    __syncthreads();

    // 3. POVM map: rho -> p, as many pass blocks at a time as the pool holds
    Cx<R>* buf = reinterpret_cast<Cx<R>*>(pool);
    constexpr int kPoolValues = int(sizeof(pool) / sizeof(Cx<R>));
    const int P = b.plan.passes[n];
    // (two-pass plans of N = 7, 8: pass 0, then the last pass fused with
    // the likelihood and the first adjoint pass; p is never stored)
    double L = 0.0, F = 0.0, bad0 = 0.0, bad1 = 0.0;
    if (fastp) {
      fast_pass0<R, false, TETRA, SUB, int(sizeof(pool))>(b, n, rho, inter, pool, sub, t & 255);
      fast_fused_form<R, TETRA, SUB, int(sizeof(pool))>(b, n, fastp, inter, f, Fsum, pool, sub, t & 255, L, bad0,
                                                       bad1);
    } else
    for (int pj = 0; pj < P; ++pj) {
      PassArgs a{};
      a.n = n;
      a.U = b.plan.U[n][pj];
      a.g = b.plan.g[n][pj];
      a.J = b.plan.J[n][pj];
      a.ld = d;
      const bool ms = pj == 0, ps = pj == P - 1;
      a.in = ms ? static_cast<const void*>(rho) : static_cast<const void*>(inter);
      a.out = ps ? static_cast<void*>(pvec) : static_cast<void*>(inter);
      const int Up = a.U - a.g;
      const int64_t side = int64_t(1) << Up;
      const int64_t blocks = side * (side + 1) / 2 * ((int64_t(1) << (2 * (n - a.U))) / a.J);
      const int per = kPoolValues / ((1 << (2 * a.g)) * a.J);  // blocks the LDS pool holds
      for (int64_t vb = 0; vb < blocks; vb += per) {
        const int nb = int(blocks - vb < per ? blocks - vb : per);
        if (ms && ps) generic_pass::fwd_pass_body<R, TETRA, true, true, kPassLoads>(a, b.W, vb, buf, nb);
        else if (ms) generic_pass::fwd_pass_body<R, TETRA, true, false, kPassLoads>(a, b.W, vb, buf, nb);
        else if (ps) generic_pass::fwd_pass_body<R, TETRA, false, true, kPassLoads>(a, b.W, vb, buf, nb);
        else generic_pass::fwd_pass_body<R, TETRA, false, false, kPassLoads>(a, b.W, vb, buf, nb);
        pass_call_barrier(a, vb + per < blocks);
      }
    }

    // 4. L, F (FP64), counters
    if (fastp) F = Fsum;
    else
    for (int64_t k0 = 0; k0 < D; k0 += kBatch * THREADS) {
      R fv[kBatch], pv[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int64_t k = k0 + u * THREADS + t;
        const int64_t kc = k < D ? k : D - 1;
        fv[u] = f[kc];
        pv[u] = pvec[kc];
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        if (k0 + u * THREADS + t >= D) continue;
        const double fk = double(fv[u]), pk = double(pv[u]);
        F += fk;
        if (fk != 0.0) {
          if (pk > 0.0) L -= fk * ln_prob(pv[u]);
          else bad0 += 1.0;
        }
        if (pk != pk || fk != fk) bad1 += 1.0;
      }
    }
    L = block_sum_bcast<NW>(L, red, slotp);
    if (!fastp) F = block_sum_bcast<NW>(F, red, slotp);
    bad0 = block_sum_bcast<NW>(bad0, red, slotp);
    bad1 = block_sum_bcast<NW>(bad1, red, slotp);
    if (t == 0) {
      double Lo = L;
      if (F != F || bad1 > 0.0) Lo = __builtin_nan("");
      else if (bad0 > 0.0) Lo = __builtin_inf();
      b.nll_out[2 * j] = Lo;
      b.nll_out[2 * j + 1] = F;
      if (b.bad_out) {
        b.bad_out[2 * j] = (unsigned long long)bad0;
        b.bad_out[2 * j + 1] = (unsigned long long)bad1;
      }
      *Fdev = F;
    }
    __syncthreads();

    // 5. cotangent + adjoint map: (p, f) -> G' (in the rho slot); in the
    // fused form only the adjoint pass 0 is left: Y -> G'
    if (fastp) {
      fast_pass0<R, true, TETRA, SUB, int(sizeof(pool))>(b, n, rho, inter, pool, sub, t & 255);
    } else
    for (int pj = P - 1; pj >= 0; --pj) {
      PassArgs a{};
      a.n = n;
      a.U = b.plan.U[n][pj];
      a.g = b.plan.g[n][pj];
      a.J = b.plan.J[n][pj];
      a.ld = d;
      a.p = pvec;
      a.f = f;
      a.F = Fdev;
      const bool ms = pj == 0, ps = pj == P - 1;
      a.in = ps ? nullptr : static_cast<const void*>(inter);
      a.out = ms ? static_cast<void*>(rho) : static_cast<void*>(inter);
      const int Up = a.U - a.g;
      const int64_t side = int64_t(1) << Up;
      const int64_t blocks = side * (side + 1) / 2 * ((int64_t(1) << (2 * (n - a.U))) / a.J);
      const int per = kPoolValues / ((1 << (2 * a.g)) * a.J);
      for (int64_t vb = 0; vb < blocks; vb += per) {
        const int nb = int(blocks - vb < per ? blocks - vb : per);
        if (ms && ps) generic_pass::adj_pass_body<R, TETRA, true, true, kPassLoads>(a, b.V, vb, buf, nb);
        else if (ms) generic_pass::adj_pass_body<R, TETRA, true, false, kPassLoads>(a, b.V, vb, buf, nb);
        else if (ps) generic_pass::adj_pass_body<R, TETRA, false, true, kPassLoads>(a, b.V, vb, buf, nb);
        else generic_pass::adj_pass_body<R, TETRA, false, false, kPassLoads>(a, b.V, vb, buf, nb);
        pass_call_barrier(a, vb + per < blocks);
      }
    }

    // 6. grad = (2/tau) G' T
    const double scale = 2.0 / tau;
    if (d >= 64) {
      gemm::GemmArgs g{};
      g.A = rho;
      g.lda = d;
      g.B = T;
      g.ldb = d;
      g.C = grad;
      g.ldc = d;
      g.d = d;
      g.kIters = d / PM::KP;
      const int tiles = d / 64, ntl = tiles * tiles;
      auto& sm = reinterpret_cast<typename PM::Smem*>(pool)[sub];
      for (int t0 = 0; t0 < ntl; t0 += SUB) {
        const int tile = t0 + sub, tl = tile < ntl ? tile : 0;
        const int tr = tl / tiles, tc = tl % tiles;
        typename PM::acc_t aR[2][2], aI[2][2];
        gemm::zero_acc<PM>(aR, aI);
        PM::run(g, sm, tr, tc, 0, g.kIters, aR, aI);
        if (tile < ntl) gemm::epilogue<PM>(g, tr, tc, aR, aI, scale);
      }
    } else {
      for (int64_t e = t; e < D; e += THREADS) {
        const int r = int(e >> n), c = int(e & (d - 1));
        R sr = 0, si = 0;
        for (int k = 0; k < d; ++k) {
          const Cx<R> x = rho[int64_t(r) * d + k], y = T[int64_t(k) * d + c];
          if constexpr (BF16) {
            const float ahr = bf16_value(float(x.re)), ahi = bf16_value(float(x.im));
            const float alr = bf16_value(float(x.re) - ahr), ali = bf16_value(float(x.im) - ahi);
            const float bhr = bf16_value(float(y.re)), bhi = bf16_value(float(y.im));
            const float blr = bf16_value(float(y.re) - bhr), bli = bf16_value(float(y.im) - bhi);
            sr += (ahr * bhr - ahi * bhi) + (ahr * blr - ahi * bli) + (alr * bhr - ali * bhi);
            si += (ahr * bhi + ahi * bhr) + (ahr * bli + ahi * blr) + (alr * bhi + ali * bhr);
          } else {
            sr += x.re * y.re - x.im * y.im;
            si += x.re * y.im + x.im * y.re;
          }
        }
        grad[e] = Cx<R>{R(sr * scale), R(si * scale)};
      }
    }
    __syncthreads();
  }
}

// Workgroup sizes of the batched kernel: FP32 512 (two tile groups; its
// registers allow two waves per SIMD) or 256; FP64 and BF16 256.
template <typename R, bool BF16, int NT>
void* batch_kernel_fn(bool tetra) {
  using namespace gemm;
  if constexpr (BF16) {
    return tetra ? reinterpret_cast<void*>(&batch_kernel<HerkBf16Policy, HemmBf16x3Policy, float, true, true, NT>)
                 : reinterpret_cast<void*>(&batch_kernel<HerkBf16Policy, HemmBf16x3Policy, float, false, true, NT>);
  } else {
    return tetra ? reinterpret_cast<void*>(&batch_kernel<BatchHerk<R>, BatchHemm<R>, R, true, false, NT>)
                 : reinterpret_cast<void*>(&batch_kernel<BatchHerk<R>, BatchHemm<R>, R, false, false, NT>);
  }
}

template <class PH, class PM, typename R, bool BF16, int NT>
hipError_t launch_batch_t(bool tetra, const BatchArgs& a, int grid, hipStream_t s) {
  if (tetra) batch_kernel<PH, PM, R, true, BF16, NT><<<unsigned(grid), NT, 0, s>>>(a);
  else batch_kernel<PH, PM, R, false, BF16, NT><<<unsigned(grid), NT, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_batch_kernel(qst_prec prec, bool tetra, const BatchArgs& a, int grid, int threads, hipStream_t s) {
  using namespace gemm;
  if (prec == QST_F64)
    return launch_batch_t<BatchHerk<double>, BatchHemm<double>, double, false, 256>(tetra, a, grid, s);
  if (prec == QST_F32) {
    if (threads == 256) return launch_batch_t<BatchHerk<float>, BatchHemm<float>, float, false, 256>(tetra, a, grid, s);
    return launch_batch_t<BatchHerk<float>, BatchHemm<float>, float, false, 512>(tetra, a, grid, s);
  }
  return launch_batch_t<HerkBf16Policy, HemmBf16x3Policy, float, true, 256>(tetra, a, grid, s);
}

// The workgroup sizes a precision offers (the first is the default).
std::vector<int> batch_thread_options(qst_prec prec) {
  if (prec == QST_F32) return {512, 256};
  return {256};
}

int batch_occupancy(qst_prec prec, int threads) {
  void* fn = prec == QST_F64   ? batch_kernel_fn<double, false, 256>(true)
             : prec == QST_F32 ? (threads == 256 ? batch_kernel_fn<float, false, 256>(true)
                                                 : batch_kernel_fn<float, false, 512>(true))
                               : batch_kernel_fn<float, true, 256>(true);
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(fn), threads, 0) != hipSuccess ||
      n <= 0)
    n = 1;
  return n;
}

}  // namespace

}  // namespace qst

// ---------------------------------------------------------------------------
// Host plan
// ---------------------------------------------------------------------------
struct qst_batch_plan {
  int count = 0;
  qst_prec prec = QST_F32;
  bool tetra = true;
  int nmax = 0;
  int device = 0;
  std::vector<int> n;
  std::vector<int64_t> t_off, f_off;  // count + 1 entries
  qst::BatchArgs args{};
  qst::BatchItem* d_items = nullptr;
  int* d_order = nullptr;
  int* d_order_natural = nullptr;
  int* d_counter = nullptr;
  unsigned char* d_scratch = nullptr;
  int cus = 256;
  std::vector<int> thread_options;  // workgroup sizes offered (first: default)
  std::vector<int> occ;             // occupancy of each
  int max_grid = 0;                 // the scratch covers this many workgroups
  // tuning
  std::string cache_path, key;
  bool tuned = false;
  int grid = 0;
  bool sorted_order = true;
  int threads = 256;
  bool fast_forms = true;
  double tuned_ms = 0.0;
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* g_T = nullptr;
  const void* g_f = nullptr;
  void* g_nll = nullptr;
  void* g_bad = nullptr;
  void* g_grad = nullptr;
  hipStream_t g_stream = nullptr;
  int g_grid = 0;
  bool g_sorted = true;
  int g_threads = 0;
  bool g_fast = true;
};

namespace qst {
qst_status fail_status(qst_status st, const std::string& msg) {
  set_error(msg);
  return st;
}
}  // namespace qst

namespace {

std::string device_name(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  return std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

void free_plan(qst_batch_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_order) (void)hipFree(p->d_order);
  if (p->d_order_natural) (void)hipFree(p->d_order_natural);
  if (p->d_counter) (void)hipFree(p->d_counter);
  if (p->d_scratch) (void)hipFree(p->d_scratch);
  delete p;
}

bool read_cache(qst_batch_plan* p) {
  if (p->cache_path.empty()) return false;
  std::ifstream in(p->cache_path);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string key;
    int grid = 0, sorted = 1;
    double ms = 0;
    if (ls >> key >> grid >> sorted >> ms && key == p->key && grid > 0) {
      int threads = p->thread_options[0], fast = 1;
      if (!(ls >> threads >> fast)) {  // a line without the shape fields: the defaults
        threads = p->thread_options[0];
        fast = 1;
      }
      size_t v = 0;
      while (v < p->thread_options.size() && p->thread_options[v] != threads) ++v;
      if (v == p->thread_options.size()) continue;  // a size this precision does not offer
      p->threads = threads;
      p->fast_forms = fast != 0;
      p->grid = std::min(grid, p->cus * p->occ[v]);
      p->sorted_order = sorted != 0;
      p->tuned_ms = ms;
      p->tuned = true;
    }
  }
  return p->tuned;
}

void write_cache(const qst_batch_plan* p) {
  if (p->cache_path.empty()) return;
  std::ofstream out(p->cache_path, std::ios::app);
  out << p->key << " " << p->grid << " " << (p->sorted_order ? 1 : 0) << " " << p->tuned_ms << " " << p->threads
      << " " << (p->fast_forms ? 1 : 0) << "\n";
}

hipError_t enqueue(qst_batch_plan* p, int grid, bool sorted, int threads, bool fast, hipStream_t s) {
  qst::BatchArgs a = p->args;
  a.order = sorted ? p->d_order : p->d_order_natural;
  a.fast_forms = fast ? 1 : 0;
  qst::reset_counter_kernel<<<1, 1, 0, s>>>(p->d_counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return qst::launch_batch_kernel(p->prec, p->tetra, a, grid, threads, s);
}

}  // namespace

extern "C" {

qst_status qst_batch_plan_create(const int* n_qubits, int count, qst_prec prec, const double* povm_host,
                                 const char* tune_cache, qst_batch_plan** out) {
  std::string msg;
  if (!out) return qst::fail_status(QST_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!n_qubits || count <= 0) return qst::fail_status(QST_ERR_INVALID_ARG, "empty batch");
  if (!qst::prec_valid(prec)) return qst::fail_status(QST_ERR_INVALID_ARG, "unknown precision");
  if (qst::check_povm(povm_host, msg) != QST_OK) return qst::fail_status(QST_ERR_INVALID_ARG, msg);
  for (int i = 0; i < count; ++i) {
    if (n_qubits[i] < 1 || n_qubits[i] > qst::kBatchMaxQubits)
      return qst::fail_status(QST_ERR_INVALID_ARG, "batched instances need 1 <= N <= 8 (instance " +
                                                       std::to_string(i) + " has N=" + std::to_string(n_qubits[i]) + ")");
  }
  qst_batch_plan* p = new qst_batch_plan();
  p->count = count;
  p->prec = qst::storage_prec(prec);  // instances have d <= 256: QST_F32X6 runs as QST_F32
  p->tetra = povm_host == nullptr;
  p->n.assign(n_qubits, n_qubits + count);
  p->t_off.assign(count + 1, 0);
  p->f_off.assign(count + 1, 0);
  std::vector<qst::BatchItem> items(count);
  for (int i = 0; i < count; ++i) {
    const int64_t D = int64_t(1) << (2 * p->n[i]);
    p->nmax = std::max(p->nmax, p->n[i]);
    items[i] = qst::BatchItem{p->n[i], 0, p->t_off[i], p->f_off[i]};
    p->t_off[i + 1] = p->t_off[i] + D;
    p->f_off[i + 1] = p->f_off[i] + D;
  }
  // descending cost (N), ties by index: greedy longest-processing-time order
  std::vector<int> order(count), natural(count);
  for (int i = 0; i < count; ++i) order[i] = natural[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p->n[a] > p->n[b]; });

  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) {
    free_plan(p);
    return qst::fail_status(QST_ERR_HIP, std::string("device query: ") + hipGetErrorString(e));
  }
  p->thread_options = qst::batch_thread_options(p->prec);
  int occ_max = 1;
  for (int th : p->thread_options) {
    p->occ.push_back(std::max(1, qst::batch_occupancy(p->prec, th)));
    occ_max = std::max(occ_max, p->occ.back());
  }
  p->threads = p->thread_options[0];
  const int64_t dmax = int64_t(1) << p->nmax, Dmax = dmax * dmax;
  const size_t cb = qst::complex_bytes(p->prec), rb = qst::real_bytes(p->prec);
  const int64_t stride = int64_t((2 * Dmax * cb + Dmax * rb + 64 + 255) / 256 * 256);
  const int max_grid = p->cus * occ_max;
  p->max_grid = max_grid;
  e = hipMalloc(&p->d_items, sizeof(qst::BatchItem) * count);
  if (e == hipSuccess) e = hipMalloc(&p->d_order, sizeof(int) * count);
  if (e == hipSuccess) e = hipMalloc(&p->d_order_natural, sizeof(int) * count);
  if (e == hipSuccess) e = hipMalloc(&p->d_counter, 256);
  if (e == hipSuccess) e = hipMalloc(&p->d_scratch, size_t(stride) * max_grid);
  if (e == hipSuccess) e = hipMemcpy(p->d_items, items.data(), sizeof(qst::BatchItem) * count, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_order, order.data(), sizeof(int) * count, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_order_natural, natural.data(), sizeof(int) * count, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_plan(p);
    return qst::fail_status(QST_ERR_HIP, std::string("batch plan allocation: ") + hipGetErrorString(e));
  }
  qst::BatchArgs& a = p->args;
  a.items = p->d_items;
  a.count = count;
  a.counter = p->d_counter;
  a.scratch = p->d_scratch;
  a.stride = stride;
  a.nmax = p->nmax;
  for (int m = 1; m <= qst::kBatchMaxQubits; ++m) {
    const qst::PovmPlan pl = qst::make_povm_plan(m, p->prec);
    a.plan.passes[m] = pl.passes;
    for (int j = 0; j < 4; ++j) {
      a.plan.g[m][j] = pl.g[j];
      a.plan.U[m][j] = pl.U[j];
      a.plan.J[m][j] = pl.J[j];
    }
  }
  double W[32], V[32];
  qst::povm_mode_matrices(povm_host, W, V);
  for (int i = 0; i < 32; ++i) {
    a.W.a[i] = W[i];
    a.V.a[i] = V[i];
  }
  // tuning key: precision, histogram of qubit counts, device
  int hist[qst::kBatchMaxQubits + 1] = {0};
  for (int i = 0; i < count; ++i) ++hist[p->n[i]];
  std::ostringstream key;
  key << "prec" << int(p->prec) << (p->tetra ? "-tetra" : "-povm") << "-n";
  for (int m = 1; m <= qst::kBatchMaxQubits; ++m) key << (m > 1 ? "." : "") << hist[m];
  key << "-" << device_name(p->device);
  p->key = key.str();
  std::string path = tune_cache ? tune_cache : "";
  if (path.empty()) {
    const char* env = std::getenv("QST_TUNE_CACHE");
    if (env) path = env;
  }
  p->cache_path = path;
  p->grid = p->cus * p->occ[0];
  read_cache(p);
  *out = p;
  qst::clear_error();
  return QST_OK;
}

qst_status qst_batch_offsets(const qst_batch_plan* p, int64_t* t_offsets, int64_t* f_offsets) {
  if (!p || !t_offsets || !f_offsets) return qst::fail_status(QST_ERR_INVALID_ARG, "NULL argument");
  std::copy(p->t_off.begin(), p->t_off.end(), t_offsets);
  std::copy(p->f_off.begin(), p->f_off.end(), f_offsets);
  return QST_OK;
}

qst_status qst_batch_run(qst_batch_plan* p, const void* T_all, const void* f_all, double* nll_out,
                         unsigned long long* bad_out, void* grad_all, int use_graph, void* stream) {
  if (!p) return qst::fail_status(QST_ERR_INVALID_ARG, "plan is NULL");
  if (!T_all || !f_all || !nll_out || !grad_all) return qst::fail_status(QST_ERR_INVALID_ARG, "NULL buffer");
  if (T_all == grad_all) return qst::fail_status(QST_ERR_INVALID_ARG, "grad_all must not alias T_all");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (use_graph && !s) return qst::fail_status(QST_ERR_INVALID_ARG, "graph mode needs a non-null stream");
  p->args.T_all = T_all;
  p->args.f_all = f_all;
  p->args.nll_out = nll_out;
  p->args.bad_out = bad_out;
  p->args.grad_all = grad_all;
  hipError_t e;
  if (!p->tuned) {
    // autotune: workgroup size x POVM pass plan of N = 7, 8 (register-round
    // forms or generic passes; the former exist for the tetrahedral POVM in
    // FP32 and FP64) x grid (CUs x {1..occupancy}) x order (cost-sorted,
    // natural); the fastest of three timed runs after a warm-up each
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    double best = 1e30;
    int best_grid = p->grid, best_threads = p->threads;
    bool best_sorted = true, best_fast = true;
    const bool has_fast = p->tetra && p->prec != QST_BF16GEMM;
    for (size_t v = 0; v < p->thread_options.size() && e == hipSuccess; ++v) {
      const int th = p->thread_options[v];
      for (int fast = 1; fast >= (has_fast ? 0 : 1) && e == hipSuccess; --fast) {
        for (int m = 1; m <= p->occ[v] && e == hipSuccess; ++m) {
          for (int so = 1; so >= 0 && e == hipSuccess; --so) {
            const int grid = p->cus * m;
            e = enqueue(p, grid, so != 0, th, fast != 0, s);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(a, s);
            for (int r = 0; r < 3 && e == hipSuccess; ++r) e = enqueue(p, grid, so != 0, th, fast != 0, s);
            if (e == hipSuccess) e = hipEventRecord(b, s);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (e == hipSuccess && ms / 3.0 < best) {
              best = ms / 3.0;
              best_grid = grid;
              best_sorted = so != 0;
              best_threads = th;
              best_fast = fast != 0;
            }
          }
        }
      }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return qst::fail_status(QST_ERR_HIP, std::string("batch tuning: ") + hipGetErrorString(e));
    p->grid = best_grid;
    p->sorted_order = best_sorted;
    p->threads = best_threads;
    p->fast_forms = best_fast;
    p->tuned_ms = best;
    p->tuned = true;
    write_cache(p);
  }
  if (!use_graph) {
    e = enqueue(p, p->grid, p->sorted_order, p->threads, p->fast_forms, s);
    if (e != hipSuccess) return qst::fail_status(QST_ERR_HIP, std::string("batch launch: ") + hipGetErrorString(e));
    qst::clear_error();
    return QST_OK;
  }
  const bool stale = !p->exec || p->g_T != T_all || p->g_f != f_all || p->g_nll != nll_out || p->g_bad != bad_out ||
                     p->g_grad != grad_all || p->g_stream != s || p->g_grid != p->grid ||
                     p->g_sorted != p->sorted_order || p->g_threads != p->threads || p->g_fast != p->fast_forms;
  if (stale) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t e1 = enqueue(p, p->grid, p->sorted_order, p->threads, p->fast_forms, s);
      e = hipStreamEndCapture(s, &p->graph);
      if (e == hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return qst::fail_status(QST_ERR_HIP, std::string("batch graph capture: ") + hipGetErrorString(e));
    p->g_T = T_all;
    p->g_f = f_all;
    p->g_nll = nll_out;
    p->g_bad = bad_out;
    p->g_grad = grad_all;
    p->g_stream = s;
    p->g_grid = p->grid;
    p->g_sorted = p->sorted_order;
    p->g_threads = p->threads;
    p->g_fast = p->fast_forms;
  }
  e = hipGraphLaunch(p->exec, s);
  if (e != hipSuccess) return qst::fail_status(QST_ERR_HIP, std::string("batch graph launch: ") + hipGetErrorString(e));
  qst::clear_error();
  return QST_OK;
}

qst_status qst_batch_shape(const qst_batch_plan* p, int* threads, int* register_round_passes) {
  if (!p) return qst::fail_status(QST_ERR_INVALID_ARG, "plan is NULL");
  if (threads) *threads = p->threads;
  if (register_round_passes) *register_round_passes = p->fast_forms ? 1 : 0;
  return QST_OK;
}

qst_status qst_batch_info(const qst_batch_plan* p, int* grid, int* sorted_order, double* tuned_ms) {
  if (!p) return qst::fail_status(QST_ERR_INVALID_ARG, "plan is NULL");
  if (grid) *grid = p->grid;
  if (sorted_order) *sorted_order = p->sorted_order ? 1 : 0;
  if (tuned_ms) *tuned_ms = p->tuned_ms;
  return QST_OK;
}

void qst_batch_plan_destroy(qst_batch_plan* p) { free_plan(p); }

}  // extern "C"
