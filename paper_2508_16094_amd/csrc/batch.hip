// gfx950 kernels of the batched interior-point solve.  One workgroup per
// instance for everything that reduces over an instance (its columns and
// rows are contiguous ranges of the block-diagonal problem), elementwise
// kernels read their instance's scalars through the column / row maps.
// Reductions use a fixed order, so the batch is deterministic as well.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

#include "batch.hpp"

namespace pdipm {

namespace {

constexpr int BS = 256;

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + BS - 1) / BS;
  return (unsigned)(b < 1 ? 1 : b);
}

__device__ inline bool lo_b(double l) { return l > -INFINITY; }
__device__ inline bool hi_b(double u) { return u < INFINITY; }

enum { R_SUM = 0, R_MAX = 1, R_MIN = 2 };

__device__ inline double comb(int op, double a, double b) {
  return op == R_SUM ? a + b : (op == R_MAX ? fmax(a, b) : fmin(a, b));
}

// Workgroup reduction of v[0..NQ); every thread receives the results.
template <int NQ>
__device__ void wg_reduce(double (&v)[NQ], const int (&op)[NQ]) {
  __shared__ double sh[NQ][BS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double x = v[q];
    for (int off = 32; off > 0; off >>= 1) x = comb(op[q], x, __shfl_down(x, off, 64));
    if (lane == 0) sh[q][wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double x = sh[q][0];
    for (int w = 1; w < BS / 64; ++w) x = comb(op[q], x, sh[q][w]);
    v[q] = x;
  }
  __syncthreads();
}

__device__ inline void ratio_b(double& a, double val, double d) {
  if (d < 0.0) a = fmin(a, -val / d);
}

__global__ void k_batch_init(BatchDev B, int stay64, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < B.count) {
    B.ist[i * IST_N + IST_STATUS] = PDIPM_MAX_ITER;
    B.ist[i * IST_N + IST_ITERS] = 0;
    B.ist[i * IST_N + IST_DONE] = 0;
    B.ist[i * IST_N + IST_MISS] = 0;
    for (int q = 0; q < BST_N; ++q) B.st[i * BST_N + q] = 0.0;
  }
  if (i < BF_N)
    B.flags[i] = i == BF_RUN ? 1 : (i == BF_STAY64 ? stay64 : (i == BF_FP64_FROM ? -1 : 0));
}

__global__ void k_batch_control(BatchDev B, int max_iter, int allow64, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  if (threadIdx.x != 0) return;
  int32_t* f = B.flags;
  if (!f[BF_RUN]) { f[BF_RUN32] = 0; f[BF_RUN64] = 0; return; }
  const int it = f[BF_STEPS];
  if (it > 0) {
    // factor failures are counted; the switch to FP64 factors follows the
    // running instances' refinement misses alone (a pivot replaced in an
    // ended instance, or one that refinement corrected, costs no accuracy)
    if (*B.bad != INT_MAX) f[BF_FAILURES] += 1;
    if (f[BF_REFINE_MISS] > 0 && !f[BF_STAY64] && allow64) {
      f[BF_STAY64] = 1;
      f[BF_FP64_FROM] = it;
    }
    if (f[BF_REFINE_MISS] > 0) f[BF_MISSES] += 1;
  }
  if (f[BF_ACTIVE] == 0 || it > max_iter) {
    f[BF_RUN] = 0; f[BF_RUN32] = 0; f[BF_RUN64] = 0;
    return;
  }
  f[BF_RUN32] = f[BF_STAY64] ? 0 : 1;
  f[BF_RUN64] = f[BF_STAY64] ? 1 : 0;
  f[BF_STEPS] = it + 1;
}

__global__ void k_batch_push_duals(DevProblem P, BatchDev B, IpmVecs v, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int b = blockIdx.x;
  const int64_t r0 = B.roff[b], r1 = B.roff[b + 1], c0 = B.xoff[b], c1 = B.xoff[b + 1];
  double a[1] = {0.0};
  const int op[1] = {R_SUM};
  for (int64_t k = r0 + threadIdx.x; k < r1; k += BS) a[0] += v.s[k] * v.lam[k];
  wg_reduce<1>(a, op);
  const double mi = (double)(r1 - r0);
  const double mu_w = fmax(1e-4, a[0] / (mi > 0 ? mi : 1.0));
  for (int64_t j = c0 + threadIdx.x; j < c1; j += BS) {
    v.zl[j] = lo_b(P.xl[j]) ? mu_w / (v.x[j] - P.xl[j]) : 0.0;
    v.zu[j] = hi_b(P.xu[j]) ? mu_w / (P.xu[j] - v.x[j]) : 0.0;
  }
}

// P = ||g - s|| / (1 + ||g||), D = ||r_d|| / (1 + ||grad f||), C = comp / (1 + |f|)
// (inf-norms) of one instance; decides its termination.
__global__ void k_batch_stats(DevProblem P, BatchDev B, IpmVecs v, double tol, int max_iter, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int b = blockIdx.x;
  int32_t* is = B.ist + (int64_t)b * IST_N;
  if (is[IST_DONE]) return;
  const int64_t r0 = B.roff[b], r1 = B.roff[b + 1], c0 = B.xoff[b], c1 = B.xoff[b + 1];
  double a[7] = {0, 0, 0, 0, 0, 0, 0};
  const int op[7] = {R_MAX, R_MAX, R_MAX, R_MAX, R_SUM, R_SUM, R_SUM};
  for (int64_t k = r0 + threadIdx.x; k < r1; k += BS) {
    a[0] = fmax(a[0], fabs(v.rp[k]));
    a[1] = fmax(a[1], fabs(v.g[k]));
    a[4] += v.s[k] * v.lam[k];
    if (!isfinite(v.rp[k]) || !isfinite(v.lam[k])) a[6] += 1;
  }
  for (int64_t j = c0 + threadIdx.x; j < c1; j += BS) {
    const double x = v.x[j];
    a[2] = fmax(a[2], fabs(v.rd[j]));
    a[3] = fmax(a[3], fabs(v.gf[j]));
    if (lo_b(P.xl[j])) a[4] += (x - P.xl[j]) * v.zl[j];
    if (hi_b(P.xu[j])) a[4] += (P.xu[j] - x) * v.zu[j];
    a[5] += P.c[j] * x + 0.5 * x * v.qx[j];
    if (!isfinite(v.rd[j]) || !isfinite(x)) a[6] += 1;
  }
  wg_reduce<7>(a, op);
  if (threadIdx.x == 0) {
    double* st = B.st + (int64_t)b * BST_N;
    const double f = a[5];
    const double Pm = a[0] / (1.0 + a[1]), Dm = a[2] / (1.0 + a[3]), Cm = a[4] / (1.0 + fabs(f));
    const double nc = B.nc[b];
    st[BST_F] = f; st[BST_P] = Pm; st[BST_D] = Dm; st[BST_C] = Cm;
    st[BST_MU] = nc > 0 ? a[4] / nc : 0.0;
    st[BST_TARGET] = 1e-2 * tol * (1.0 + a[3]);
    const int it = B.flags[BF_ITER];
    is[IST_ITERS] = it;
    int done = 1;
    if (a[6] > 0 || !isfinite(f)) is[IST_STATUS] = PDIPM_ERR_NUMERICAL;
    else if (Pm <= tol && Dm <= tol && Cm <= tol) is[IST_STATUS] = PDIPM_OK;
    else if (it >= max_iter) is[IST_STATUS] = PDIPM_MAX_ITER;
    else done = 0;
    is[IST_DONE] = done;
    if (!done) atomicAdd(B.flags + BF_ACTIVE, 1);
  }
}

// Largest steps keeping (s, x-l, u-x) and (lambda, z_l, z_u) non-negative
// over one instance (every thread receives them).
__device__ void instance_limits(const DevProblem& P, const BatchDev& B, const IpmVecs& v, int b, const double* dx,
                                const double* ds, const double* dlam, const double* dzl, const double* dzu,
                                double (&lim)[2]) {
  const int64_t r0 = B.roff[b], r1 = B.roff[b + 1], c0 = B.xoff[b], c1 = B.xoff[b + 1];
  lim[0] = INFINITY; lim[1] = INFINITY;
  const int op[2] = {R_MIN, R_MIN};
  for (int64_t k = r0 + threadIdx.x; k < r1; k += BS) {
    ratio_b(lim[0], v.s[k], ds[k]);
    ratio_b(lim[1], v.lam[k], dlam[k]);
  }
  for (int64_t j = c0 + threadIdx.x; j < c1; j += BS) {
    if (lo_b(P.xl[j])) { ratio_b(lim[0], v.x[j] - P.xl[j], dx[j]); ratio_b(lim[1], v.zl[j], dzl[j]); }
    if (hi_b(P.xu[j])) { ratio_b(lim[0], P.xu[j] - v.x[j], -dx[j]); ratio_b(lim[1], v.zu[j], dzu[j]); }
  }
  wg_reduce<2>(lim, op);
}

__global__ void k_batch_predict(DevProblem P, BatchDev B, IpmVecs v, const double* dx, const double* ds,
                                const double* dlam, const double* dzl, const double* dzu, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int b = blockIdx.x;
  if (B.ist[(int64_t)b * IST_N + IST_DONE]) return;
  double lim[2];
  instance_limits(P, B, v, b, dx, ds, dlam, dzl, dzu, lim);
  double ap = fmin(1.0, lim[0]), ad = fmin(1.0, lim[1]);
  if (!B.lp[b]) ap = ad = fmin(ap, ad);
  const int64_t r0 = B.roff[b], r1 = B.roff[b + 1], c0 = B.xoff[b], c1 = B.xoff[b + 1];
  double a[1] = {0.0};
  const int op[1] = {R_SUM};
  for (int64_t k = r0 + threadIdx.x; k < r1; k += BS) a[0] += (v.s[k] + ap * ds[k]) * (v.lam[k] + ad * dlam[k]);
  for (int64_t j = c0 + threadIdx.x; j < c1; j += BS) {
    if (lo_b(P.xl[j])) a[0] += (v.x[j] - P.xl[j] + ap * dx[j]) * (v.zl[j] + ad * dzl[j]);
    if (hi_b(P.xu[j])) a[0] += (P.xu[j] - v.x[j] - ap * dx[j]) * (v.zu[j] + ad * dzu[j]);
  }
  wg_reduce<1>(a, op);
  if (threadIdx.x == 0) {
    double* st = B.st + (int64_t)b * BST_N;
    const double nc = B.nc[b], mu = st[BST_MU];
    const double maff = nc > 0 ? a[0] / nc : 0.0;
    const double sigma = mu > 0 ? fmin(1.0, pow(maff / mu, 3.0)) : 0.0;
    st[BST_SMU] = sigma * mu;
  }
}

__global__ void k_batch_targets(DevProblem P, BatchDev B, const double* dx, const double* ds, const double* dlam,
                                const double* dzl, const double* dzu, double* ts, double* tl, double* tu, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < P.m) ts[i] = B.st[(int64_t)B.ir[i] * BST_N + BST_SMU] - ds[i] * dlam[i];
  if (i < P.n) {
    const double smu = B.st[(int64_t)B.ix[i] * BST_N + BST_SMU];
    tl[i] = lo_b(P.xl[i]) ? smu - dx[i] * dzl[i] : 0.0;
    tu[i] = hi_b(P.xu[i]) ? smu + dx[i] * dzu[i] : 0.0;
  }
}

__global__ void k_batch_correct(DevProblem P, BatchDev B, IpmVecs v, const double* dx, const double* ds,
                                const double* dlam, const double* dzl, const double* dzu, int repeat_on_miss,
                                const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int b = blockIdx.x;
  double* st = B.st + (int64_t)b * BST_N;
  int32_t* is = B.ist + (int64_t)b * IST_N;
  const int miss = is[IST_MISS];
  // a direction whose refined residual missed the instance's target is not
  // taken when FP64 factors can repeat the iteration; a non-finite one ends
  // the instance at its current (finite) iterate
  const bool repeat = repeat_on_miss && miss != MISS_NONE;
  if (is[IST_DONE] || repeat || miss == MISS_NONFINITE) {
    if (threadIdx.x == 0) {
      st[BST_AP] = 0.0; st[BST_AD] = 0.0;
      if (!is[IST_DONE] && !repeat) { is[IST_STATUS] = PDIPM_ERR_NUMERICAL; is[IST_DONE] = 1; }
    }
    return;
  }
  double lim[2];
  instance_limits(P, B, v, b, dx, ds, dlam, dzl, dzu, lim);
  if (threadIdx.x == 0) {
    const double tau = fmax(0.99, 1.0 - st[BST_MU]);
    double ap = fmin(1.0, tau * lim[0]), ad = fmin(1.0, tau * lim[1]);
    if (!B.lp[b]) ap = ad = fmin(ap, ad);
    st[BST_AP] = ap;
    st[BST_AD] = ad;
  }
}

__global__ void k_batch_update(DevProblem P, BatchDev B, IpmVecs v, const double* dx, const double* ds,
                               const double* dlam, const double* dzl, const double* dzu, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  // an instance that takes no step keeps its point exactly: its direction
  // may be non-finite (ended instances are still factored), and 0 * inf is
  // not 0
  if (i < P.m) {
    const double* st = B.st + (int64_t)B.ir[i] * BST_N;
    const double ap = st[BST_AP], ad = st[BST_AD];
    if (ap != 0.0) v.s[i] += ap * ds[i];
    if (ad != 0.0) v.lam[i] += ad * dlam[i];
  }
  if (i < P.n) {
    const double* st = B.st + (int64_t)B.ix[i] * BST_N;
    const double ap = st[BST_AP], ad = st[BST_AD];
    if (ap != 0.0) v.x[i] += ap * dx[i];
    v.zl[i] = lo_b(P.xl[i]) ? (ad != 0.0 ? v.zl[i] + ad * dzl[i] : v.zl[i]) : 0.0;
    v.zu[i] = hi_b(P.xu[i]) ? (ad != 0.0 ? v.zu[i] + ad * dzu[i] : v.zu[i]) : 0.0;
  }
}

__global__ void k_batch_check_residual(BatchDev B, const double* r, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int b = blockIdx.x;
  if (B.ist[(int64_t)b * IST_N + IST_DONE]) return;
  double a[1] = {0.0};
  const int op[1] = {R_MAX};
  for (int64_t j = B.xoff[b] + threadIdx.x; j < B.xoff[b + 1]; j += BS) {
    const double x = fabs(r[j]);
    a[0] = isfinite(x) ? fmax(a[0], x) : INFINITY;
  }
  wg_reduce<1>(a, op);
  if (threadIdx.x == 0 && !(a[0] <= B.st[(int64_t)b * BST_N + BST_TARGET])) {
    int32_t* is = B.ist + (int64_t)b * IST_N;
    if (is[IST_MISS] == MISS_NONE) atomicAdd(B.flags + BF_REFINE_MISS, 1);
    is[IST_MISS] = isfinite(a[0]) ? max(is[IST_MISS], (int32_t)MISS_TARGET) : MISS_NONFINITE;
  }
}

__global__ void k_batch_next(BatchDev B, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  if (threadIdx.x == 0) B.flags[BF_ITER] += 1;
}

__global__ void k_batch_clear_miss(BatchDev B, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < B.count) B.ist[i * IST_N + IST_MISS] = 0;
  if (i == 0) B.flags[BF_REFINE_MISS] = 0;
}

__global__ void k_set_int(int* p, int v, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  if (threadIdx.x == 0) *p = v;
}

}  // namespace

void launch_batch_init(const BatchDev& B, int stay64, hipStream_t s) {
  k_batch_init<<<grid_for(B.count > BF_N ? B.count : BF_N), BS, 0, s>>>(B, stay64, launch_gate());
}
void launch_batch_control(const BatchDev& B, int max_iter, int allow64, hipStream_t s) {
  k_batch_control<<<1, 64, 0, s>>>(B, max_iter, allow64, launch_gate());
}
void launch_batch_push_duals(const DevProblem& P, const BatchDev& B, IpmVecs& v, hipStream_t s) {
  k_batch_push_duals<<<(unsigned)B.count, BS, 0, s>>>(P, B, v, launch_gate());
}
void launch_batch_stats(const DevProblem& P, const BatchDev& B, IpmVecs& v, double tol, int max_iter,
                        hipStream_t s) {
  k_batch_stats<<<(unsigned)B.count, BS, 0, s>>>(P, B, v, tol, max_iter, launch_gate());
}
void launch_batch_predict(const DevProblem& P, const BatchDev& B, IpmVecs& v, const double* dx,
                          const double* ds, const double* dlam, const double* dzl, const double* dzu,
                          hipStream_t s) {
  k_batch_predict<<<(unsigned)B.count, BS, 0, s>>>(P, B, v, dx, ds, dlam, dzl, dzu, launch_gate());
}
void launch_batch_targets(const DevProblem& P, const BatchDev& B, const double* dx, const double* ds,
                          const double* dlam, const double* dzl, const double* dzu, double* ts, double* tl,
                          double* tu, hipStream_t s) {
  k_batch_targets<<<grid_for(P.n > P.m ? P.n : P.m), BS, 0, s>>>(P, B, dx, ds, dlam, dzl, dzu, ts, tl, tu, launch_gate());
}
void launch_batch_correct(const DevProblem& P, const BatchDev& B, IpmVecs& v, const double* dx,
                          const double* ds, const double* dlam, const double* dzl, const double* dzu,
                          int repeat_on_miss, hipStream_t s) {
  k_batch_correct<<<(unsigned)B.count, BS, 0, s>>>(P, B, v, dx, ds, dlam, dzl, dzu, repeat_on_miss, launch_gate());
}
void launch_batch_update(const DevProblem& P, const BatchDev& B, IpmVecs& v, const double* dx,
                         const double* ds, const double* dlam, const double* dzl, const double* dzu,
                         hipStream_t s) {
  k_batch_update<<<grid_for(P.n > P.m ? P.n : P.m), BS, 0, s>>>(P, B, v, dx, ds, dlam, dzl, dzu, launch_gate());
}
void launch_batch_check_residual(const BatchDev& B, const double* r, hipStream_t s) {
  k_batch_check_residual<<<(unsigned)B.count, BS, 0, s>>>(B, r, launch_gate());
}
void launch_batch_next(const BatchDev& B, hipStream_t s) { k_batch_next<<<1, 64, 0, s>>>(B, launch_gate()); }
void launch_batch_clear_miss(const BatchDev& B, hipStream_t s) {
  k_batch_clear_miss<<<grid_for(B.count), BS, 0, s>>>(B, launch_gate());
}
void launch_set_int(int* p, int v, hipStream_t s) { k_set_int<<<1, 64, 0, s>>>(p, v, launch_gate()); }

}  // namespace pdipm
