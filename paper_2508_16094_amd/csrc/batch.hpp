// Per-instance kernels of the batched interior-point solve: many independent
// LP/QP instances stored as one block-diagonal problem, each with its own
// step lengths, centring parameter and termination (implemented in batch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace pdipm {

// per-instance FP64 state, BST_N doubles per instance
enum { BST_MU = 0, BST_F, BST_P, BST_D, BST_C, BST_TARGET, BST_SMU, BST_AP, BST_AD, BST_N = 12 };
// per-instance integer state, IST_N ints per instance (IST_MISS: how a
// direction of this iteration missed the instance's refinement target)
enum { IST_STATUS = 0, IST_ITERS, IST_DONE, IST_MISS, IST_N = 4 };
enum { MISS_NONE = 0, MISS_TARGET = 1, MISS_NONFINITE = 2 };
// global integer flags: running count and refinement misses of the current
// iteration, iterations taken; the control words of a captured solve (RUN:
// stats and steps run, RUN32 / RUN64: the step in that precision runs,
// STAY64: FP64 factors from now on) and its counters
enum {
  BF_ACTIVE = 0, BF_REFINE_MISS, BF_ITER, BF_RUN, BF_RUN32, BF_RUN64, BF_STAY64, BF_STEPS,
  BF_FAILURES, BF_MISSES, BF_FP64_FROM, BF_N = 12
};

struct BatchDev {
  int32_t count;
  const int64_t *xoff, *roff;  // [count + 1] column / row ranges of each instance
  const int32_t *ix, *ir;      // instance of each column / row
  const double* nc;            // complementarity pairs of each instance
  const int32_t* lp;           // 1 for an LP (separate primal and dual steps)
  double* st;                  // [count * BST_N]
  int32_t* ist;                // [count * IST_N]
  int32_t* flags;              // [BF_N]
  const int* bad;              // first non-positive pivot of the last factorisation (INT_MAX: none)
};

// flags: active = refine_miss = iteration = 0; every instance running; the
// control words: RUN = 1, STAY64 = stay64, FP64_FROM = -1
void launch_batch_init(const BatchDev& B, int stay64, hipStream_t s);
// Decision of one iteration, after its termination measures (the host loop's
// decision made on the device, so that a graph holds whole iterations):
// after a step, count a factorisation failure and a refinement miss and
// switch to FP64 factors on either (when allow64); stop (RUN = 0) when no
// instance runs or more than max_iter steps were taken; otherwise open the
// step of the current precision (RUN32 or RUN64) and count it.
void launch_batch_control(const BatchDev& B, int max_iter, int allow64, hipStream_t s);
// push the duals of a warm start: mu_w = max(1e-4, s'lambda / m_i) per instance
void launch_batch_push_duals(const DevProblem& P, const BatchDev& B, IpmVecs& v, hipStream_t s);
// termination measures of every running instance; counts the running ones
void launch_batch_stats(const DevProblem& P, const BatchDev& B, IpmVecs& v, double tol, int max_iter,
                        hipStream_t s);
// predictor: affine step limits, mu_aff and sigma mu per instance
void launch_batch_predict(const DevProblem& P, const BatchDev& B, IpmVecs& v, const double* dx,
                          const double* ds, const double* dlam, const double* dzl, const double* dzu,
                          hipStream_t s);
void launch_batch_targets(const DevProblem& P, const BatchDev& B, const double* dx, const double* ds,
                          const double* dlam, const double* dzl, const double* dzu, double* ts, double* tl,
                          double* tu, hipStream_t s);
// corrector: step lengths per instance (zero for finished instances, and
// with repeat_on_miss for instances whose FP32 direction missed its target
// or when the factorisation met a non-positive pivot: they repeat the
// iteration, with FP64 factors once the control step switches)
void launch_batch_correct(const DevProblem& P, const BatchDev& B, IpmVecs& v, const double* dx,
                          const double* ds, const double* dlam, const double* dzl, const double* dzu,
                          int repeat_on_miss, hipStream_t s);
void launch_batch_update(const DevProblem& P, const BatchDev& B, IpmVecs& v, const double* dx,
                         const double* ds, const double* dlam, const double* dzl, const double* dzu,
                         hipStream_t s);
// flags a running instance whose refined residual r (length n) misses its target
void launch_batch_check_residual(const BatchDev& B, const double* r, hipStream_t s);
void launch_batch_next(const BatchDev& B, hipStream_t s);
void launch_batch_clear_miss(const BatchDev& B, hipStream_t s);
void launch_set_int(int* p, int v, hipStream_t s);

}  // namespace pdipm
