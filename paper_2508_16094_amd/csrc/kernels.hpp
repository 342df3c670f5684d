// Launch wrappers of the gfx950 kernels (implemented in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "host.hpp"

namespace pdipm {

// Device view of the problem patterns and values.
struct DevProblem {
  int64_t n, m, nnz_j, nnz_h;
  const double *c, *b, *q4, *xl, *xu;     // q4 may be null
  const int64_t* jp; const int32_t* jc; const double *ja, *jw;
  const int64_t* jtp; const int32_t *jtr, *jte;
  const int64_t* hp; const int32_t* hc; const double* hq; const int64_t* hdiag;
  const int64_t* hsp; const int32_t *hsc, *hss;
};

// Device view of the plan.
struct DevPlan {
  int64_t ns, n;
  int nb, small_h;
  const int32_t *sfirst, *sw, *sh, *sld, *sldu, *child_ptr, *child, *rel, *level_sn, *sn_rows, *perm;
  const int64_t *spanel, *su, *srow, *suv, *sinv;
  const GemmDesc* gemm; const PotrfDesc* potrf; const ExtAddDesc* ext; const int32_t* small;
  const InvCombDesc* icomb;
  const GatherItem* gitem; const int64_t *grow, *gptr, *gidx;
  const SolveDesc* sdesc; const int32_t *ssmall, *slarge;
  // pivot signs of a signed factorisation P'AP = L S L' (S = diag(sign),
  // permuted numbering; Section 2, SQD matrices); null: Cholesky, S = I
  const signed char* sign;
};

struct DevKMap {
  int64_t nk;
  int64_t npos;   // original indices below npos carry pivot sign +1, the rest -1
  const int32_t *krow, *kc, *kh, *tk, *ta, *tb;
  const int64_t *tp, *pos;
};

// Gate of the kernels this host thread launches: null (every kernel runs),
// or a device int that each kernel reads first, exiting when it is zero.
// A batched solve captures several iterations in one graph and gates their
// kernels by device flags, so iterations it does not need cost no work.
void set_launch_gate(const int* gate);
const int* launch_gate();

// reductions: partial results per block, then one finalising block
constexpr int RED_SUM = 0, RED_MAX = 1, RED_MIN = 2;
constexpr int RED_BLOCKS = 512;
struct RedSpec { int nq; int op[8]; };

void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
void launch_fill_bytes0(void* p, int64_t bytes, hipStream_t s);  // zero via kernel
void launch_finalize(const double* partials, int nblocks, RedSpec spec, double* out, hipStream_t s);

// model evaluation (Section 1 problem form, Section 4 derivative templates).
// A J value array holds 2 nnz_j entries: the values in J's row order, then
// the same values in the transpose's order (written by launch_jac_eval and
// launch_jv_copy, read by the products with J').
void launch_jac_eval(const DevProblem& P, const double* x, double* jv, hipStream_t s);
void launch_jv_copy(const DevProblem& P, double* jv, hipStream_t s);   // constant J (A)
void launch_constraints(const DevProblem& P, const double* x, double* g, hipStream_t s);
void launch_gradient(const DevProblem& P, const double* x, double* qx, double* gf, hipStream_t s);
void launch_hess_eval(const DevProblem& P, const double* x, const double* lam, double* hv, hipStream_t s);
void launch_jt_mul(const DevProblem& P, const double* jv, const double* y, double* out, hipStream_t s);
void launch_j_mul(const DevProblem& P, const double* jv, const double* v, double* out, hipStream_t s);
void launch_h_mul(const DevProblem& P, const double* hv, const double* v, double* out, hipStream_t s);

// assembly of K into panels (T = double or float) and K value copy
template <typename T>
void launch_assemble(const DevKMap& K, const double* hv, const double* jv, const double* sig_s,
                     const double* sig_x, double delta_p, T* panel, double* kval, hipStream_t s);
template <typename T>
void launch_set_values(const DevKMap& K, const double* kval, T* panel, hipStream_t s);

// dual condensed system M = diag(E) + J D J' (Section 3, eq. kkt_dual):
// D = (H + Sigma_x + delta_p)^-1 (H diagonal), E = 1 / Sigma_s
void launch_dual_prep(const DevProblem& P, const double* hv, const double* sig_x, const double* sig_s,
                      double delta_p, double* dd, double* de, hipStream_t s);
void launch_mul_vec(int64_t n, const double* a, const double* b, double* out, hipStream_t s);
// out = d o (r - w)
void launch_dual_finish(int64_t n, const double* d, const double* r, const double* w, double* out,
                        hipStream_t s);
// max_i (1/D_i + sum_k Sigma_s[k] J_ki^2) into the reduction output
void launch_kdiag_max(const DevProblem& P, const double* jv, const double* sig_s, const double* dd,
                      double* partials, hipStream_t s);

// numeric factorisation
template <typename T>
void launch_factor_op(const Op& op, const DevPlan& P, T* panel, T* ubuf, T* inv, int* bad, hipStream_t s);

// triangular solves (vectors FP64, panels T)
void launch_permute_in(const DevPlan& P, const double* rhs, const double* d, double* xperm, hipStream_t s);
void launch_permute_out(const DevPlan& P, const double* xperm, const double* d, double* x, hipStream_t s);
// symmetric scaling of K (FP32 factor): d = |diag(K)|^(-1/2), max |diag|, count
// of diagonal entries whose sign is not their pivot's (indices below npos
// positive, the rest negative)
void launch_diag_scale(int64_t n, const int64_t* kp, const double* kval, double* d, double* partials,
                       hipStream_t s, int64_t npos = INT64_MAX);
// y *= sign (permuted numbering): the middle factor of L S L' solves
void launch_sign_scale(int64_t n, const signed char* sign, double* y, hipStream_t s);
// augmented SQD matrix values in its assembly map's order (x block n first)
void launch_assemble_aug(const DevKMap& K, int64_t n, const double* hv, const double* jv, const double* sig_s,
                         const double* sig_x, double delta_p, double* kval, hipStream_t s);
template <typename T>
void launch_set_scaled(const DevKMap& K, const double* kval, const double* d, double shift, T* panel,
                       hipStream_t s);
template <typename T>
void launch_solve_op(const Op& op, const DevPlan& P, const T* panel, const T* inv, double* xp, double* ys,
                     double* uvec, double* part, hipStream_t s);
// symmetric product with stored K values (lower CSR, original numbering)
void launch_k_mul_stored(int64_t n, const int64_t* kp, const int32_t* kc, const int64_t* ksp,
                         const int32_t* ksc, const int64_t* kss, const double* kval,
                         const double* v, double* out, hipStream_t s);

// interior-point vector steps (Section 3 Newton step, condensed form)
struct IpmVecs {
  double *x, *s, *lam, *zl, *zu;
  double *gf, *qx, *g, *jv, *hv, *rd, *rp, *sig_s, *sig_x;
  double *tmp_n, *tmp_m, *tmp_n2, *tmp_m2;
};
void launch_residuals(const DevProblem& P, IpmVecs& v, hipStream_t s);
void launch_stats_iter(const DevProblem& P, IpmVecs& v, double* partials, hipStream_t s);
void launch_sigmas(const DevProblem& P, IpmVecs& v, double delta_d, hipStream_t s);
// w_m = sig_s (g - ts/lam)  then rhs = -r~_d - J' w_m (ts, tl, tu may be null = 0)
void launch_rhs(const DevProblem& P, IpmVecs& v, const double* ts, const double* tl, const double* tu,
                double* rhs, hipStream_t s);
void launch_recover(const DevProblem& P, IpmVecs& v, const double* dx, const double* ts,
                    const double* tl, const double* tu, double delta_d, double* ds, double* dlam,
                    double* dzl, double* dzu, hipStream_t s);
void launch_step_limits(const DevProblem& P, IpmVecs& v, const double* dx, const double* ds,
                        const double* dlam, const double* dzl, const double* dzu, double* partials,
                        hipStream_t s);
void launch_mu_aff(const DevProblem& P, IpmVecs& v, const double* dx, const double* ds,
                   const double* dlam, const double* dzl, const double* dzu, double ap, double ad,
                   double* partials, hipStream_t s);
void launch_targets(const DevProblem& P, const double* dx, const double* ds, const double* dlam,
                    const double* dzl, const double* dzu, double smu, double* ts, double* tl,
                    double* tu, hipStream_t s);
void launch_axpy_point(const DevProblem& P, IpmVecs& dst, const IpmVecs& src, const double* dx,
                       const double* ds, const double* dlam, const double* dzl, const double* dzu,
                       double ap, double ad, hipStream_t s);
void launch_phi(const DevProblem& P, IpmVecs& v, double smu, double* partials, hipStream_t s);
void launch_init_point(const DevProblem& P, IpmVecs& v, hipStream_t s);
void launch_push_start(const DevProblem& P, IpmVecs& v, const double* xhat, const double* lamhat,
                       double mu_w_unused, hipStream_t s);
void launch_push_duals(const DevProblem& P, IpmVecs& v, double mu_w, hipStream_t s);
void launch_sum_sl(const DevProblem& P, IpmVecs& v, double* partials, hipStream_t s);
// refinement helpers
void launch_k_mul_free(const DevProblem& P, const double* jv, const double* hv, const double* sig_s,
                       const double* sig_x, double delta_p, const double* v, double* out,
                       double* tmp_m, double* tmp_n, hipStream_t s);
void launch_residual_norms(int64_t n, const double* rhs, const double* kx, const double* x, double* r,
                           double* partials, hipStream_t s);
void launch_add(int64_t n, double* x, const double* c, hipStream_t s);
void launch_dot(int64_t n, const double* a, const double* b, double* partials, hipStream_t s);
void launch_cg_step(int64_t n, double alpha, const double* p, const double* q, double* x, double* r,
                    double* partials, hipStream_t s);
void launch_xpby(int64_t n, const double* z, double beta, double* p, hipStream_t s);
void launch_copy(int64_t n, double* dst, const double* src, hipStream_t s);

}  // namespace pdipm
