// gfx950 kernels of the interior-point hot path.
//
// Every reduction is two-pass with a fixed partition (no floating-point
// atomics), assembly and extend-add sum in a fixed order, so repeated runs
// give bitwise-identical results.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.hpp"

namespace pdipm {

namespace {

constexpr int BS = 256;
constexpr int SBS = 512;  // threads of the blocked triangular-solve steps (8 waves)

inline int64_t blocks_for(int64_t n, int bs = BS) {
  int64_t b = (n + bs - 1) / bs;
  return b < 1 ? 1 : b;
}

__device__ inline bool has_lo(double l) { return l > -INFINITY; }
__device__ inline bool has_hi(double u) { return u < INFINITY; }

__device__ inline double red_init(int op) {
  return op == RED_SUM ? 0.0 : (op == RED_MAX ? -INFINITY : INFINITY);
}
__device__ inline double red_comb(int op, double a, double b) {
  return op == RED_SUM ? a + b : (op == RED_MAX ? fmax(a, b) : fmin(a, b));
}

// Reduce v[0..nq) over the block and store one partial per quantity.
template <int NQ>
__device__ void block_reduce_store(double (&v)[NQ], const RedSpec& spec, double* partials) {
  __shared__ double sh[NQ][BS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double x = v[q];
    for (int off = 32; off > 0; off >>= 1) x = red_comb(spec.op[q], x, __shfl_down(x, off, 64));
    if (lane == 0) sh[q][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double x = sh[q][0];
      for (int w = 1; w < BS / 64; ++w) x = red_comb(spec.op[q], x, sh[q][w]);
      partials[(int64_t)q * gridDim.x + blockIdx.x] = x;
    }
  }
}

__global__ void k_finalize(const double* partials, int nblocks, RedSpec spec, double* out, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  __shared__ double sh[BS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = 0; q < spec.nq; ++q) {
    double x = red_init(spec.op[q]);
    for (int b = threadIdx.x; b < nblocks; b += BS) x = red_comb(spec.op[q], x, partials[(int64_t)q * nblocks + b]);
    for (int off = 32; off > 0; off >>= 1) x = red_comb(spec.op[q], x, __shfl_down(x, off, 64));
    if (lane == 0) sh[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      double y = sh[0];
      for (int w = 1; w < BS / 64; ++w) y = red_comb(spec.op[q], y, sh[w]);
      out[q] = y;
    }
    __syncthreads();
  }
}

__global__ void k_fill_f64(double* p, int64_t n, double v, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) p[i] = v;
}

__global__ void k_zero_u32(uint32_t* p, int64_t n, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) p[i] = 0u;
}

// ------------------------------------------------------------ evaluation
__global__ void k_jac_eval(int64_t nnz, const double* ja, const double* jw, const int32_t* jc,
                           const double* x, double* jv, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t e = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (e < nnz) jv[e] = ja[e] - 2.0 * jw[e] * x[jc[e]];
}

__global__ void k_constraints(int64_t m, const int64_t* jp, const int32_t* jc, const double* ja,
                              const double* jw, const double* x, const double* b, double* g, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t k = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (k >= m) return;
  double acc = 0.0;
  for (int64_t e = jp[k]; e < jp[k + 1]; ++e) {
    double xc = x[jc[e]];
    acc += (ja[e] - jw[e] * xc) * xc;
  }
  g[k] = acc - b[k];
}

__global__ void k_gradient(int64_t n, const int64_t* hsp, const int32_t* hsc, const int32_t* hss,
                           const double* hq, const double* c, const double* q4, const double* x,
                           double* qx, double* gf, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int64_t q = hsp[i]; q < hsp[i + 1]; ++q) acc += hq[hss[q]] * x[hsc[q]];
  qx[i] = acc;
  double xi = x[i];
  gf[i] = c[i] + acc + (q4 ? q4[i] * xi * xi * xi : 0.0);
}

__global__ void k_hess_eval(int64_t n, const int64_t* hp, const int64_t* hdiag, const double* hq,
                            const double* q4, const int64_t* jtp, const int32_t* jtr,
                            const int32_t* jte, const double* jw, const double* x, const double* lam,
                            double* hv, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i >= n) return;
  for (int64_t e = hp[i]; e < hp[i + 1]; ++e) hv[e] = hq[e];
  double wl = 0.0;
  for (int64_t q = jtp[i]; q < jtp[i + 1]; ++q) wl += jw[jte[q]] * lam[jtr[q]];
  double xi = x[i];
  hv[hdiag[i]] += (q4 ? 3.0 * q4[i] * xi * xi : 0.0) + 2.0 * wl;
}

// Column-major copy of J's values (the second half of every J value array):
// jvt[q] = jv[jte[q]] in the transpose's order, so that products with J'
// read the values contiguously instead of gathering them.
__global__ void k_jv_transpose(int64_t nnz, const int32_t* jte, const double* jv, double* jvt, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t q = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (q < nnz) jvt[q] = jv[jte[q]];
}

// J' y: one thread per column over the column-major values.
__global__ void k_jt_mul(int64_t n, const int64_t* jtp, const int32_t* jtr, const double* jvt,
                         const double* y, double* out, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int64_t q = jtp[i]; q < jtp[i + 1]; ++q) acc += jvt[q] * y[jtr[q]];
  out[i] = acc;
}

// J v: JROW lanes per row stride over its entries (coalesced), then a fixed
// butterfly sums the lanes.
constexpr int JROW = 8;
__global__ void k_j_mul(int64_t m, const int64_t* jp, const int32_t* jc, const double* jv,
                        const double* v, double* out, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int64_t k = blockIdx.x * (int64_t)(BS / JROW) + threadIdx.x / JROW;
  const int g = threadIdx.x % JROW;
  double acc = 0.0;
  if (k < m)
    for (int64_t e = jp[k] + g; e < jp[k + 1]; e += JROW) acc += jv[e] * v[jc[e]];
#pragma unroll
  for (int o = JROW / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (k < m && g == 0) out[k] = acc;
}

__global__ void k_h_mul(int64_t n, const int64_t* hsp, const int32_t* hsc, const int32_t* hss,
                        const double* hv, const double* v, double* out, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int64_t q = hsp[i]; q < hsp[i + 1]; ++q) acc += hv[hss[q]] * v[hsc[q]];
  out[i] = acc;
}

// ------------------------------------------------------------ assembly
// One thread per entry of K's lower pattern: fixed-order segmented sum of
// the J' Sigma_s J products plus the Hessian and diagonal terms.
template <typename T>
__global__ void k_assemble(DevKMap K, const double* hv, const double* jv, const double* sig_s,
                           const double* sig_x, double delta_p, T* panel, double* kval, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t e = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (e >= K.nk) return;
  double v = 0.0;
  int32_t h = K.kh[e];
  if (h >= 0) v = hv[h];
  int32_t r = K.krow[e];
  if (r == K.kc[e]) v += sig_x[r] + delta_p;
  for (int64_t t = K.tp[e]; t < K.tp[e + 1]; ++t) v += sig_s[K.tk[t]] * jv[K.ta[t]] * jv[K.tb[t]];
  if (panel) panel[K.pos[e]] = (T)v;
  if (kval) kval[e] = v;
}

template <typename T>
__global__ void k_set_values(DevKMap K, const double* kval, T* panel, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t e = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (e < K.nk) panel[K.pos[e]] = (T)kval[e];
}

// Symmetric scaling D = |diag(K)|^(-1/2): partials give max |K_ii| and the
// count of diagonal entries without their pivot's sign (positive below npos,
// negative from npos on; a plain SPD K has npos >= n).
__global__ void k_diag_scale(int64_t n, const int64_t* kp, const double* kval, double* d, double* partials,
                             int64_t npos, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  RedSpec spec{3, {RED_MAX, RED_SUM, RED_MIN}};
  double a[3] = {0.0, 0.0, INFINITY};
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const double kii = (i < npos ? 1.0 : -1.0) * kval[kp[i + 1] - 1];
    if (kii > 0.0 && isfinite(kii)) {
      d[i] = 1.0 / sqrt(kii);
      a[0] = fmax(a[0], kii);
    } else {
      d[i] = 1.0;
      a[1] += 1.0;
      a[2] = fmin(a[2], (double)i);
    }
  }
  block_reduce_store<3>(a, spec, partials);
}

template <typename T>
__global__ void k_set_scaled(DevKMap K, const double* kval, const double* d, double shift, T* panel, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t e = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (e >= K.nk) return;
  const int32_t r = K.krow[e], c = K.kc[e];
  double v = kval[e] * d[r] * d[c];
  if (r == c) v += r < K.npos ? shift : -shift;   // the shift takes the pivot's sign
  panel[K.pos[e]] = (T)v;
}

// Augmented SQD matrix [H + diag(Sigma_x + delta_p), J'; J, -1/Sigma_s] in
// the order of its assembly map: x rows take an H entry, lambda rows a J
// entry (kh) or, on the diagonal, -1/Sigma_s.
__global__ void k_assemble_aug(DevKMap K, int64_t n, const double* hv, const double* jv, const double* sig_s,
                               const double* sig_x, double delta_p, double* kval, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int64_t e = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (e >= K.nk) return;
  const int32_t r = K.krow[e], c = K.kc[e], q = K.kh[e];
  double v;
  if (r < n) {
    v = hv[q];
    if (r == c) v += sig_x[r] + delta_p;
  } else {
    v = r == c ? -1.0 / sig_s[r - n] : jv[q];
  }
  kval[e] = v;
}

__global__ void k_sign_scale(int64_t n, const signed char* sign, double* y, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < n && sign[i] < 0) y[i] = -y[i];
}

__global__ void k_k_mul_stored(int64_t n, const int64_t* ksp, const int32_t* ksc, const int64_t* kss,
                               const double* kval, const double* v, double* out, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int64_t q = ksp[i]; q < ksp[i + 1]; ++q) acc += kval[kss[q]] * v[ksc[q]];
  out[i] = acc;
}

// ------------------------------------------- dual condensed system
// D = (H + Sigma_x + delta_p I)^-1 for a diagonal H and E = Sigma_s^-1
// (= delta_d + s / lambda): the diagonal scalings of M = diag(E) + J D J'.
__global__ void k_dual_prep(int64_t n, int64_t m, const double* hv, const int64_t* hdiag,
                            const double* sig_x, const double* sig_s, double delta_p, double* dd,
                            double* de, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < n) dd[i] = 1.0 / (hv[hdiag[i]] + sig_x[i] + delta_p);
  if (i < m) de[i] = 1.0 / sig_s[i];
}

// out = a o b, and out = d o (r - w): the two diagonal steps of a K solve
// through M (x = D r - D J' M^-1 J D r).
__global__ void k_mul_vec(int64_t n, const double* a, const double* b, double* out, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

__global__ void k_dual_finish(int64_t n, const double* d, const double* r, const double* w, double* out, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < n) out[i] = d[i] * (r[i] - w[i]);
}

// max_i K_ii with K_ii = 1/D_i + sum_k Sigma_s[k] J_ki^2 (the norm estimate
// of K used by the backward error when K itself is never formed)
__global__ void k_kdiag_max(int64_t n, const int64_t* jtp, const int32_t* jtr, const double* jvt,
                            const double* sig_s, const double* dd, double* partials, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  RedSpec spec{1, {RED_MAX}};
  double a[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    double k = 1.0 / dd[i];
    for (int64_t q = jtp[i]; q < jtp[i + 1]; ++q) {
      const double j = jvt[q];
      k += sig_s[jtr[q]] * j * j;
    }
    a[0] = fmax(a[0], k);
  }
  block_reduce_store<1>(a, spec, partials);
}

// ------------------------------------------------------- factorisation
// Small fronts (h <= 64): the whole front in LDS; children's update
// matrices are added in child order, then w columns are eliminated and the
// panel and the new update matrix are written back.
template <typename T>
__global__ void __launch_bounds__(BS) k_small_front(DevPlan P, int64_t d0, T* panel, T* ubuf, int* bad, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  constexpr int LD = 65;
  __shared__ T F[64 * LD];
  const int32_t S = P.small[d0 + blockIdx.x];
  const int h = P.sh[S], w = P.sw[S], ld = P.sld[S];
  const int64_t poff = P.spanel[S];
  for (int idx = threadIdx.x; idx < h * h; idx += BS) {
    int i = idx % h, j = idx / h;
    F[i + j * LD] = (j < w && i >= j) ? panel[poff + i + (int64_t)j * ld] : (T)0;
  }
  __syncthreads();
  for (int32_t q = P.child_ptr[S]; q < P.child_ptr[S + 1]; ++q) {
    const int32_t c = P.child[q];
    const int hu = P.sh[c] - P.sw[c];
    const int32_t* rc = P.rel + P.srow[c] + P.sw[c];
    const T* U = ubuf + P.su[c];
    const int ldu = P.sldu[c];
    for (int idx = threadIdx.x; idx < hu * hu; idx += BS) {
      int i = idx % hu, j = idx / hu;
      if (i >= j) F[rc[i] + rc[j] * LD] += U[i + (int64_t)j * ldu];
    }
    __syncthreads();
  }
  for (int k = 0; k < w; ++k) {
    // signed factorisation (P.sign): L S L' with l_kk = sqrt(s_k a_kk),
    // l_ik = a_ik / (s_k l_kk) and a_ij -= l_ik s_k l_jk
    const T sk = P.sign && P.sign[P.sfirst[S] + k] < 0 ? (T)-1 : (T)1;
    if (threadIdx.x == 0) {
      T d = sk * F[k + k * LD];
      if (!(d > (T)0) || !isfinite((double)d)) {
        atomicMin(bad, P.sfirst[S] + k);
        d = (T)1;
      }
      F[k + k * LD] = sqrt(d);
    }
    __syncthreads();
    const T piv = sk * F[k + k * LD];
    for (int i = k + 1 + threadIdx.x; i < h; i += BS) F[i + k * LD] /= piv;
    __syncthreads();
    const int r = h - k - 1;
    for (int idx = threadIdx.x; idx < r * r; idx += BS) {
      int i = k + 1 + idx % r, j = k + 1 + idx / r;
      if (i >= j) F[i + j * LD] -= sk * F[i + k * LD] * F[j + k * LD];
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < h * w; idx += BS) {
    int i = idx % h, j = idx / h;
    if (i >= j) panel[poff + i + (int64_t)j * ld] = F[i + j * LD];
  }
  const int hu = h - w, ldu = P.sldu[S];
  T* U = ubuf + P.su[S];
  for (int idx = threadIdx.x; idx < hu * hu; idx += BS) {
    int i = idx % hu, j = idx / hu;
    if (i >= j) U[i + (int64_t)j * ldu] = F[(w + i) + (w + j) * LD];
  }
}

// Extend-add for large fronts: a workgroup owns front columns [t0, t1) of
// parent S and adds every child's update matrix entries landing there, one
// child after the other (children may share targets).  The children's
// column ranges inside [t0, t1) (two binary searches in each child's
// relative row map) are found first by one thread per child, a batch at a
// time: searched one child after the other they were a chain of dependent
// loads that set the time of parents with many children (up to 200 per
// front on the block-angular LP; 3-5 ms per launch, mostly latency).
template <typename T>
__global__ void __launch_bounds__(BS) k_extend_add(DevPlan P, int64_t d0, T* panel, T* ubuf, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  constexpr int CB = 256;           // children per batch of searches
  __shared__ int s_lo[CB], s_hi[CB];
  const ExtAddDesc d = P.ext[d0 + blockIdx.x];
  const int32_t S = d.sn;
  const int wP = P.sw[S], ldP = P.sld[S];
  T* pan = panel + P.spanel[S];
  T* UP = ubuf + P.su[S];
  const int64_t ldu = P.sldu[S];
  const int32_t cbeg = P.child_ptr[S], cend = P.child_ptr[S + 1];
  for (int32_t b0 = cbeg; b0 < cend; b0 += CB) {
    const int nb = cend - b0 < CB ? cend - b0 : CB;
    for (int q = threadIdx.x; q < nb; q += BS) {
      const int32_t c = P.child[b0 + q];
      const int hu = P.sh[c] - P.sw[c];
      const int32_t* rc = P.rel + P.srow[c] + P.sw[c];
      int lo = 0, hi = hu;
      while (lo < hi) { int mid = (lo + hi) >> 1; if (rc[mid] < d.t0) lo = mid + 1; else hi = mid; }
      s_lo[q] = lo;
      hi = hu;
      while (lo < hi) { int mid = (lo + hi) >> 1; if (rc[mid] < d.t1) lo = mid + 1; else hi = mid; }
      s_hi[q] = lo;
    }
    __syncthreads();
    for (int q = 0; q < nb; ++q) {
      const int jlo = s_lo[q], jhi = s_hi[q];
      if (jlo >= jhi) continue;      // no columns in [t0, t1): nothing to order
      const int32_t c = P.child[b0 + q];
      const int hu = P.sh[c] - P.sw[c];
      const int32_t* rc = P.rel + P.srow[c] + P.sw[c];
      const T* U = ubuf + P.su[c];
      const int64_t lduc = P.sldu[c];
      for (int j = jlo; j < jhi; ++j) {
        const int tj = rc[j];
        // target column: a panel column of S, or a column of its U (whose
        // rows are counted from wP)
        T* dst = tj < wP ? pan + (int64_t)tj * ldP : UP + (int64_t)(tj - wP) * ldu;
        const int sub = tj < wP ? 0 : wP;
        const T* src = U + (int64_t)j * lduc;
        int i = j + (int)threadIdx.x;
        // four rows per thread at a time, all loads issued before the
        // read-modify-writes
        for (; i + 3 * BS < hu; i += 4 * BS) {
          int t[4];
          T v[4], o[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            t[u] = rc[i + u * BS] - sub;
            v[u] = src[i + u * BS];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) o[u] = dst[t[u]];
#pragma unroll
          for (int u = 0; u < 4; ++u) dst[t[u]] = o[u] + v[u];
        }
        for (; i < hu; i += BS) dst[rc[i] - sub] += src[i];
      }
      __syncthreads();
    }
    __syncthreads();                 // s_lo / s_hi are rewritten by the next batch
  }
}

// Broadcast of lane `src` (wave-uniform) through the scalar unit.
__device__ inline float lane_bcast(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
__device__ inline double lane_bcast(double v, int src) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// 1 / sqrt(x) for x > 0: the hardware estimate refined by Newton's iteration
// y <- y (3 - x y^2) / 2 (once in FP32, twice in FP64), cheaper on the
// factor's dependent chain than a square root and a division.
__device__ inline float rsqrt_newton(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  return y * (1.5f - 0.5f * x * y * y);
}
__device__ inline double rsqrt_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  return y * (1.5 - 0.5 * x * y * y);
}

// Cholesky factor and inverse of one nb x nb diagonal block (bw <= nb
// columns used; the rest is padded with the identity), blocked by panels of
// PB columns in LDS:
//   factor:  wave 0 factors the (nb - c0) x PB panel column by column with
//            lane broadcasts (no workgroup barrier inside a panel), then all
//            waves apply the rank-PB update to the trailing lower part with
//            TS x TS register tiles;
//   inverse: X = inv(L) by recursive doubling: the PB x PB diagonal blocks
//            at once (one thread per column), then log2(nb / PB) levels
//            joining pairs of inverted blocks with two small products each
//            (16-22% faster per block than solving row panels one after
//            the other).
// X is kept transposed in the (zero) upper triangle of the same LDS array
// and its diagonal in xd, so one NB x (NB + 1) array holds both factors.
// PT threads in a (PT / 16) x 16 grid of register tiles.  FP32 launches of
// at most one block per CU take 8 waves (the chain of diagonal blocks of a
// wide supernode is latency-bound: 135 instead of 190 us per block); larger
// launches and FP64 take 4 waves (two workgroups per CU; 8 waves would not
// fit the FP64 panel work in registers).
// SG: signed factorisation L S L' of an SQD block (pivot signs from
// P.sign): l_kk = sqrt(s_k a_kk), l_ik = a_ik / (s_k l_kk), trailing
// a_ij -= l_ik s_k l_jk; the inverse is that of L.
template <typename T, int NB, int PT, bool SG>
__global__ void __launch_bounds__(PT) k_potrf(DevPlan P, int64_t d0, T* panel, T* inv, int* bad, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  constexpr int GR = PT / 16, GC = 16, PB = 16, NP = NB / PB, LDA = NB + 1, S = NB / 64;
  constexpr int TR = NB / GR, TC = NB / GC;   // rows and columns of a thread's tile
  static_assert(GR * GC == PT && TR * GR == NB && TC * GC == NB, "thread grid");
  __shared__ T A[NB * LDA];
  __shared__ T xd[NB];
  __shared__ T rdiag[NB];   // 1 / L(k, k)
  __shared__ T ssg[SG ? NB : 1];   // pivot signs of the block (padding +1)
  const PotrfDesc d = P.potrf[d0 + blockIdx.x];
  const int bw = d.bw;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tr = tid / GC, tc = tid % GC;
  T* g = panel + d.d_off;
  // load the block with CH independent loads in flight per thread (a plain
  // strided loop waits for each load before the next)
  constexpr int PER = NB * NB / PT, CH = PER < 32 ? PER : 32;
  static_assert(PER % CH == 0, "block load chunks");
#pragma unroll
  for (int c0 = 0; c0 < PER; c0 += CH) {
    T v[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int idx = tid + (c0 + u) * PT, i = idx % NB, j = idx / NB;
      v[u] = (i < bw && j < bw && i >= j) ? g[i + (int64_t)j * d.ld] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int idx = tid + (c0 + u) * PT, i = idx % NB, j = idx / NB;
      A[i + j * LDA] = (i < bw && j < bw) ? v[u] : (i == j ? (T)1 : (T)0);
    }
  }
  if (tid < NB) xd[tid] = (T)1;
  if (SG && tid < NB) ssg[tid] = tid < bw && P.sign[d.col0 + tid] < 0 ? (T)-1 : (T)1;
  __syncthreads();
  // ---- factor
  for (int p = 0; p < NP; ++p) {
    const int c0 = p * PB, c1 = c0 + PB;
    if (wave == 0) {
      T a[S][PB];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = c0 + lane + 64 * s;
#pragma unroll
        for (int j = 0; j < PB; ++j) a[s][j] = r < NB ? A[r + (c0 + j) * LDA] : (T)0;
      }
#pragma unroll
      for (int k = 0; k < PB; ++k) {
        const T sk = SG ? ssg[c0 + k] : (T)1;
        T dk = sk * lane_bcast(a[0][k], k);
        if (!(dk > (T)0) || !isfinite((double)dk)) {
          if (lane == 0 && c0 + k < bw) atomicMin(bad, d.col0 + c0 + k);
          dk = (T)1;
        }
        const T rp = rsqrt_newton(dk), piv = dk * rp;
        if (lane == 0) rdiag[c0 + k] = rp;
        const T rs = SG ? sk * rp : rp;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int rel = lane + 64 * s;
          if (rel > k) a[s][k] *= rs;
          else if (rel == k) a[s][k] = piv;
        }
#pragma unroll
        for (int j = k + 1; j < PB; ++j) {
          const T ljk = SG ? sk * lane_bcast(a[0][k], j) : lane_bcast(a[0][k], j);
#pragma unroll
          for (int s = 0; s < S; ++s)
            if (lane + 64 * s > k) a[s][j] -= a[s][k] * ljk;
        }
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int r = c0 + lane + 64 * s;
#pragma unroll
        for (int j = 0; j < PB; ++j)
          if (r < NB && r >= c0 + j) A[r + (c0 + j) * LDA] = a[s][j];
      }
    }
    __syncthreads();
    // trailing update of rows and columns >= c1 (lower part)
    if (c1 < NB && tr * TR + TR - 1 >= tc * TC && tr * TR + TR > c1 && tc * TC + TC > c1) {
      T acc[TR][TC];
#pragma unroll
      for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int c = 0; c < TC; ++c) acc[r][c] = (T)0;
#pragma unroll 4
      for (int t = 0; t < PB; ++t) {
        T li[TR], lj[TC];
        const T st = SG ? ssg[c0 + t] : (T)1;
#pragma unroll
        for (int r = 0; r < TR; ++r) li[r] = A[tr * TR + r + (c0 + t) * LDA];
#pragma unroll
        for (int c = 0; c < TC; ++c) lj[c] = SG ? st * A[tc * TC + c + (c0 + t) * LDA] : A[tc * TC + c + (c0 + t) * LDA];
#pragma unroll
        for (int r = 0; r < TR; ++r)
#pragma unroll
          for (int c = 0; c < TC; ++c) acc[r][c] += li[r] * lj[c];
      }
#pragma unroll
      for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int c = 0; c < TC; ++c) {
          const int i = tr * TR + r, j = tc * TC + c;
          if (j >= c1 && i >= j) A[i + j * LDA] -= acc[r][c];
        }
    }
    __syncthreads();
  }
  // ---- inverse X = inv(L) by recursive doubling: the PB x PB diagonal
  // blocks first (all at once, one thread per column), then pairs of
  // inverted blocks of size s = PB, 2 PB, ... are joined, every pair of a
  // level at once:
  //   inv([L11 0; L21 L22]) = [X11 0; -X22 (L21 X11)  X22].
  // X is kept transposed in the zero upper triangle of A (X(i, j) at
  // A[j + i LDA], i > j) and its diagonal in xd; T = L21 X11 is staged where
  // X21 goes, and X21 is written once every thread has read T.  Depth: PB
  // dependent steps plus log2(NB / PB) joins, against NB dependent steps
  // for row panels one after the other.
  {
    if (tid < NB) {
      const int c0 = (tid / PB) * PB, jj = tid % PB;
      T x[PB];
#pragma unroll
      for (int r = 0; r < PB; ++r) x[r] = r == jj ? (T)1 : (T)0;
#pragma unroll
      for (int t = 0; t < PB; ++t) {
        x[t] *= rdiag[c0 + t];
#pragma unroll
        for (int r = t + 1; r < PB; ++r) x[r] -= A[(c0 + r) + (c0 + t) * LDA] * x[t];
      }
#pragma unroll
      for (int r = 0; r < PB; ++r) {
        if (r > jj) A[(c0 + jj) + (c0 + r) * LDA] = x[r];
        else if (r == jj) xd[c0 + r] = x[r];
      }
    }
    __syncthreads();
    auto X = [&](int i, int j) -> T { return i > j ? A[j + i * LDA] : (i == j ? xd[i] : (T)0); };
    constexpr int LPB = PB == 16 ? 4 : 3, NLEV = (NB == 128 ? 7 : 6) - LPB;
    static_assert((1 << LPB) == PB && (PB << NLEV) == NB, "power-of-two blocks");
    // the joined block's entry (i, j) of pair p: X21(i, j), staged T(i, j)
    auto at21 = [&](int o, int s, int i, int j) -> T& { return A[(o + j) + (o + s + i) * LDA]; };
    if constexpr (NB >= 128) {
      // one 4 x 4 register tile per thread (at most NB^2 / 64 <= PT tiles)
      static_assert(NB * NB / 64 <= PT, "one tile per thread");
#pragma unroll
      for (int lev = 0; lev < NLEV; ++lev) {
        const int lg = LPB + lev, s = 1 << lg, lt = lg - 2, ntile = (NB >> (lg + 1)) << (2 * lt);
        const bool mine = tid < ntile;
        const int p = tid >> (2 * lt), i0 = (tid & ((1 << lt) - 1)) << 2, j0 = ((tid >> lt) & ((1 << lt) - 1)) << 2;
        const int o = p << (lg + 1);
        T acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = (T)0;
        if (mine) {
          // T = L21 X11 (X11(k, j) = 0 for k < j)
          for (int k = j0; k < s; ++k) {
            T l[4], x[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) l[a] = A[(o + s + i0 + a) + (o + k) * LDA];
#pragma unroll
            for (int b = 0; b < 4; ++b) x[b] = X(o + k, o + j0 + b);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < 4; ++b) acc[a][b] += l[a] * x[b];
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) at21(o, s, i0 + a, j0 + b) = acc[a][b];
        }
        __syncthreads();
        if (mine) {
          // X21 = -X22 T (X22(i, k) = 0 for k > i)
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = (T)0;
          for (int k = 0; k < i0 + 4; ++k) {
            T x[4], tv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) x[a] = X(o + s + i0 + a, o + s + k);
#pragma unroll
            for (int b = 0; b < 4; ++b) tv[b] = at21(o, s, k, j0 + b);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * tv[b];
          }
        }
        __syncthreads();
        if (mine) {
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) at21(o, s, i0 + a, j0 + b) = -acc[a][b];
        }
        __syncthreads();
      }
    } else {
      // one entry per thread and round (at most EPT rounds)
      constexpr int EPT = (NB * NB / 4 + PT - 1) / PT;
#pragma unroll
      for (int lev = 0; lev < NLEV; ++lev) {
        const int lg = LPB + lev, s = 1 << lg, ne = NB << (lg - 1);
        T out[EPT];
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          const int e = tid + q * PT;
          if (e < ne) {
            // T = L21 X11 (X11(k, j) = 0 for k < j)
            const int p = e >> (2 * lg), i = e & (s - 1), j = (e >> lg) & (s - 1), o = p << (lg + 1);
            T acc = (T)0;
            for (int k = j; k < s; ++k) acc += A[(o + s + i) + (o + k) * LDA] * X(o + k, o + j);
            at21(o, s, i, j) = acc;
          }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          const int e = tid + q * PT;
          out[q] = (T)0;
          if (e < ne) {
            // X21 = -X22 T (X22(i, k) = 0 for k > i)
            const int p = e >> (2 * lg), i = e & (s - 1), j = (e >> lg) & (s - 1), o = p << (lg + 1);
            T acc = (T)0;
            for (int k = 0; k <= i; ++k) acc += X(o + s + i, o + s + k) * at21(o, s, k, j);
            out[q] = -acc;
          }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          const int e = tid + q * PT;
          if (e < ne) {
            const int p = e >> (2 * lg), i = e & (s - 1), j = (e >> lg) & (s - 1), o = p << (lg + 1);
            at21(o, s, i, j) = out[q];
          }
        }
        __syncthreads();
      }
    }
  }
  // ---- write back L (lower, bw x bw) and X = inv(L) (nb x nb, zero padded)
  T* o = inv + d.inv_off;
  for (int idx = tid; idx < NB * NB; idx += PT) {
    const int i = idx % NB, j = idx / NB;
    if (i < bw && j < bw && i >= j) g[i + (int64_t)j * d.ld] = A[i + j * LDA];
    T x = (T)0;
    if (i < bw && j < bw) x = i > j ? A[j + i * LDA] : (i == j ? xd[i] : (T)0);
    o[i + (int64_t)j * NB] = x;
  }
}

// Tile (ti, tj) of descriptor-local tile index t.  Tile columns are taken in
// groups of TG; inside a group the tiles run row by row, so the tiles one
// XCD holds at a time share the A row block and the group's B blocks in its
// L2.  Lower-masked descriptors (M >= N) enumerate only tiles with ti >= tj:
// a group is a triangle of tg rows followed by full rows of tg tiles.
constexpr int TG = 8;
__host__ __device__ inline void tile_of(const GemmDesc& d, int64_t t, int& ti, int& tj) {
  const int64_t m = d.tiles_m, n = d.tiles_n;
  if (!d.lower) {
    const int64_t full = n / TG;                 // groups of TG columns
    const int64_t per = (int64_t)TG * m;
    int64_t g = t / per;
    if (g > full) g = full;
    const int64_t u = t - g * per;
    const int64_t w = (g < full) ? TG : n - full * TG;
    ti = (int)(u / w);
    tj = (int)(g * TG + u % w);
    return;
  }
  // tiles before group g (all groups before g are full): g (T + TG (m - TG)) - TG^2 g (g - 1) / 2
  const int64_t T = (int64_t)TG * (TG + 1) / 2;
  auto start = [&](int64_t g) { return g * (T + (int64_t)TG * (m - TG)) - (int64_t)TG * TG * g * (g - 1) / 2; };
  const int64_t ng = (n + TG - 1) / TG;
  int64_t lo = 0, hi = ng - 1;                    // last group with start <= t
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (start(mid) <= t) lo = mid; else hi = mid - 1;
  }
  const int64_t g = lo, c0 = g * TG;
  const int64_t w = n - c0 < TG ? n - c0 : TG;
  int64_t u = t - start(g);
  const int64_t tri = w * (w + 1) / 2;
  if (u < tri) {
    int64_t r = 0;
    while ((r + 1) * (r + 2) / 2 <= u) ++r;
    ti = (int)(c0 + r);
    tj = (int)(c0 + (u - r * (r + 1) / 2));
  } else {
    u -= tri;
    ti = (int)(c0 + w + u / w);
    tj = (int)(c0 + u % w);
  }
}

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// run of tiles (neighbouring tiles share A and B panels in that XCD's L2).
__device__ inline int64_t xcd_tile(int64_t bid, int64_t grid) {
  const int64_t per = grid >> 3;   // grid is a multiple of 8
  return (bid & 7) * per + (bid >> 3);
}

// Descriptor of tile bid: the last of d0 .. d1-1 whose first tile is at or
// before bid.  Each wave searches by 64-way splits, one load per lane and
// round (two rounds for up to 4096 descriptors; a binary search was a chain
// of log2(d1 - d0) dependent loads at the start of every tile).  Every wave
// finds the same descriptor.
__device__ inline int64_t find_desc(const GemmDesc* g, int64_t d0, int64_t d1, int64_t bid) {
  const int lane = threadIdx.x & 63;
  int64_t lo = d0, n = d1 - d0;
  while (n > 1) {
    const int64_t step = (n + 63) >> 6;
    const int64_t idx = lo + (int64_t)lane * step;
    // lanes whose split point starts at or before bid form a prefix; lane 0's
    // (lo) always does
    const bool ok = idx < lo + n && g[idx].tile_begin <= bid;
    const int last = 63 - __builtin_clzll((unsigned long long)__ballot(ok));
    lo += (int64_t)last * step;
    n = n - (int64_t)last * step < step ? n - (int64_t)last * step : step;
  }
  return lo;
}

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
// 16-byte vectors that only assume element alignment (panel rows may start
// at any element; the hardware splits misaligned accesses)
typedef float float4u __attribute__((ext_vector_type(4), aligned(4)));
typedef double double2u __attribute__((ext_vector_type(2), aligned(8)));

// Load up to 4 consecutive elements; `valid` of them are in range (<= 0: none).
__device__ inline float4u load4(const float* p, int valid) {
  if (valid >= 4) return *(const float4u*)p;
  float4u v = {0.0f, 0.0f, 0.0f, 0.0f};
  if (valid > 0) v.x = p[0];
  if (valid > 1) v.y = p[1];
  if (valid > 2) v.z = p[2];
  return v;
}
__device__ inline double2u load2(const double* p, int valid) {
  if (valid >= 2) return *(const double2u*)p;
  double2u v = {0.0, 0.0};
  if (valid > 0) v.x = p[0];
  return v;
}

// C (-)= A * B^T, FP64 MFMA 16x16x4.  64 x 64 tile per workgroup of eight
// waves, each a 32 x 16 strip of 2 x 1 MFMA blocks; K chunks of 16 staged
// through LDS with the next chunk prefetched into registers (one 16-byte
// load per operand and thread).  Against 16 x 32 strips and 32-deep chunks
// this ran the rank-512 updates 3-6% faster (55 -> 58.5 TFLOP/s on an
// 8192-row lower update).
// SG: signed factorisation (L S L'): updates subtract A S B' (the sign of
// inner index k, at permuted column kcol + k, applied to A), the panel solve
// scales output column j by the sign at kcol + j.
constexpr int BS64 = 512;  // threads of the FP64 GEMM (8 waves)
template <bool SG>
__global__ void __launch_bounds__(BS64) k_gemm_f64(DevPlan P, int64_t d0, int64_t d1, int64_t ntiles, double* panel,
                                                   double* ubuf, const double* inv, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  constexpr int TM = GEMM_TILE_F64, BX = 2, BY = 1;
  constexpr int WX = TM / (16 * BX);                       // waves along rows
  static_assert(WX * (TM / (16 * BY)) == BS64 / 64, "eight waves per tile");
  // LDS rows padded by 16 doubles: the four 16-lane row groups of an
  // operand read then fall on disjoint banks (padding by 2 left 12% of the
  // LDS cycles in bank conflicts; +2% GEMM rate)
  constexpr int KC = 16, LDS_LD = TM + 16, TPR = TM / 2, KS = BS64 / TPR, PER = KC / KS;
  static_assert(PER >= 1 && PER * KS == KC, "whole rows of the chunk per load round");
  __shared__ double As[KC * LDS_LD];
  __shared__ double Bs[KC * LDS_LD];
  const int64_t bid = xcd_tile(blockIdx.x, gridDim.x);
  if (bid >= ntiles) return;
  const GemmDesc d = P.gemm[find_desc(P.gemm, d0, d1, bid)];
  int ti, tj;
  tile_of(d, bid - d.tile_begin, ti, tj);
  const int i0 = ti * TM, j0 = tj * TM;
  double* C = (d.c_buf ? ubuf : panel) + d.c_off;
  const double* A = panel + d.a_off;
  const double* B = (d.b_buf ? inv : panel) + d.b_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave % WX) * 16 * BX, wn = (wave / WX) * 16 * BY;
  // this thread loads 2 consecutive rows (16-byte loads) at k offsets kb + KS r
  const int ii = (tid % TPR) * 2, kb = tid / TPR;
  const double* Ap = A + (i0 + ii);
  const double* Bp = B + (j0 + ii);
  const int arows = d.M - (i0 + ii), brows = d.N - (j0 + ii);
  doublex4 acc[BX][BY];
#pragma unroll
  for (int x = 0; x < BX; ++x)
#pragma unroll
    for (int y = 0; y < BY; ++y) acc[x][y] = doublex4{0, 0, 0, 0};
  double2u ra[PER], rb[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int gk = k0 + kb + KS * r;
      ra[r] = load2(Ap + (int64_t)gk * d.lda, gk < d.K ? arows : 0);
      rb[r] = load2(Bp + (int64_t)gk * d.ldb, gk < d.K ? brows : 0);
      if constexpr (SG)
        if (d.mode == 0 && gk < d.K && P.sign[d.kcol + gk] < 0) ra[r] = -ra[r];
    }
  };
  load(0);
  for (int k0 = 0; k0 < d.K; k0 += KC) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      *(double2u*)&As[(kb + KS * r) * LDS_LD + ii] = ra[r];
      *(double2u*)&Bs[(kb + KS * r) * LDS_LD + ii] = rb[r];
    }
    __syncthreads();
    if (k0 + KC < d.K) load(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      double a[BX], b[BY];
#pragma unroll
      for (int x = 0; x < BX; ++x) a[x] = As[(kk + (lane >> 4)) * LDS_LD + wm + x * 16 + (lane & 15)];
#pragma unroll
      for (int y = 0; y < BY; ++y) b[y] = Bs[(kk + (lane >> 4)) * LDS_LD + wn + y * 16 + (lane & 15)];
#pragma unroll
      for (int x = 0; x < BX; ++x)
#pragma unroll
        for (int y = 0; y < BY; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[y], a[x], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < BX; ++x)
#pragma unroll
    for (int y = 0; y < BY; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // operands swapped: lanes run along rows of C (contiguous stores)
        const int i = i0 + wm + x * 16 + (lane & 15);
        const int j = j0 + wn + y * 16 + 4 * r + (lane >> 4);
        if (i < d.M && j < d.N && (!d.lower || i >= j)) {
          double* cp = C + i + (int64_t)j * d.ldc;
          if (d.mode == 0) *cp -= acc[x][y][r];
          else *cp = SG && P.sign[d.kcol + j] < 0 ? -acc[x][y][r] : acc[x][y][r];
        }
      }
}

// C (-)= A * B^T, FP32 MFMA 32x32x2 with FP32 accumulation.  128x128 tile
// per workgroup of eight waves, each a 64x32 strip (2x1 MFMA blocks); K is
// staged through LDS in chunks of 16 with the next chunk prefetched into
// registers (chunks of 32 ran the large lower updates 2-4% slower).
constexpr int BS32 = 512;  // threads of the FP32 GEMM (8 waves)
template <bool SG>
__global__ void __launch_bounds__(BS32) k_gemm_f32(DevPlan P, int64_t d0, int64_t d1, int64_t ntiles, float* panel,
                                                   float* ubuf, const float* inv, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  constexpr int TM = GEMM_TILE_F32, KC = 16, LDS_LD = TM + 4, PER = (TM * KC) / BS32;  // 4 per operand
  static_assert(PER % 4 == 0 && KC % 16 == 0, "16-byte loads at k offsets kb + 16 r");
  static_assert(TM == 128, "the FP32 wave layout assumes 128 x 128 tiles");
  __shared__ float As[KC * LDS_LD];
  __shared__ float Bs[KC * LDS_LD];
  const int64_t bid = xcd_tile(blockIdx.x, gridDim.x);
  if (bid >= ntiles) return;
  const GemmDesc d = P.gemm[find_desc(P.gemm, d0, d1, bid)];
  int ti, tj;
  tile_of(d, bid - d.tile_begin, ti, tj);
  const int i0 = ti * TM, j0 = tj * TM;
  float* C = (d.c_buf ? ubuf : panel) + d.c_off;
  const float* A = panel + d.a_off;
  const float* B = (d.b_buf ? inv : panel) + d.b_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // eight waves: wave w owns rows 64 (w mod 2) .. +64 and columns 32 (w / 2) .. +32
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 32;
  // this thread loads 4 consecutive rows (16-byte loads) at k offsets
  // kb + 16 r; edge rows fall back to guarded scalar loads
  const int ii = (tid & 31) * 4, kb = tid >> 5;
  const float* Ap = A + (i0 + ii);
  const float* Bp = B + (j0 + ii);
  const int arows = d.M - (i0 + ii), brows = d.N - (j0 + ii);
  floatx16 acc[2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[a][r] = 0.0f;
  float4u ra[PER / 4], rb[PER / 4];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < PER / 4; ++r) {
      const int gk = k0 + kb + 16 * r;
      ra[r] = load4(Ap + (int64_t)gk * d.lda, gk < d.K ? arows : 0);
      rb[r] = load4(Bp + (int64_t)gk * d.ldb, gk < d.K ? brows : 0);
      if constexpr (SG)
        if (d.mode == 0 && gk < d.K && P.sign[d.kcol + gk] < 0) ra[r] = -ra[r];
    }
  };
  load(0);
  for (int k0 = 0; k0 < d.K; k0 += KC) {
#pragma unroll
    for (int r = 0; r < PER / 4; ++r) {
      *(float4u*)&As[(kb + 16 * r) * LDS_LD + ii] = ra[r];
      *(float4u*)&Bs[(kb + 16 * r) * LDS_LD + ii] = rb[r];
    }
    __syncthreads();
    if (k0 + KC < d.K) load(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 2) {
      float a[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) a[q] = As[(kk + (lane >> 5)) * LDS_LD + wm + q * 32 + (lane & 31)];
      const float b = Bs[(kk + (lane >> 5)) * LDS_LD + wn + (lane & 31)];
#pragma unroll
      for (int x = 0; x < 2; ++x) acc[x] = __builtin_amdgcn_mfma_f32_32x32x2f32(b, a[x], acc[x], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      // operands swapped: lanes run along rows of C (contiguous stores)
      const int i = i0 + wm + x * 32 + (lane & 31);
      const int j = j0 + wn + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (i < d.M && j < d.N && (!d.lower || i >= j)) {
        float* cp = C + i + (int64_t)j * d.ldc;
        if (d.mode == 0) *cp -= acc[x][r];
        else *cp = SG && P.sign[d.kcol + j] < 0 ? -acc[x][r] : acc[x][r];
      }
    }
}

// --------------------------------------------------- triangular solves
__global__ void k_permute_in(int64_t n, const int32_t* perm, const double* rhs, const double* d, double* xp, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t k = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (k < n) xp[k] = d ? rhs[perm[k]] * d[perm[k]] : rhs[perm[k]];
}
__global__ void k_permute_out(int64_t n, const int32_t* perm, const double* xp, const double* d, double* x, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t k = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (k < n) x[perm[k]] = d ? xp[k] * d[perm[k]] : xp[k];
}

// Solve inverses of SOLVE_NB-column diagonal blocks from the FP64
// factorisation's 64-column ones (one workgroup per block):
//   inv([L11 0; L21 L22]) = [X1 0; -X2 (L21 X1)  X2].
// X1, X2 are lower triangular with zeros outside the block's columns, so
// the products run over the triangles only and a partial block (bw <= 64:
// no X2, or bw < 128: zero rows and columns) comes out zero-padded.
__global__ void __launch_bounds__(256) k_inv_combine(DevPlan P, int64_t d0, const double* panel, double* inv,
                                                     const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  constexpr int H = SOLVE_NB / 2, LD = H + 1, NT = 256, PER = H * H / NT;
  __shared__ double X[H * LD], M[H * LD];
  const InvCombDesc d = P.icomb[d0 + blockIdx.x];
  const int tid = threadIdx.x, b2 = d.bw - H;
  double* out = inv + d.out_off;
  const double* X1 = inv + d.x1_off;
  for (int idx = tid; idx < H * H; idx += NT) {
    const int i = idx % H, j = idx / H;
    X[i + j * LD] = X1[i + j * H];
    M[i + j * LD] = i < b2 ? panel[d.l21_off + i + (int64_t)j * d.ld] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < H * H; idx += NT) {
    const int i = idx % H, j = idx / H;
    out[i + (int64_t)j * SOLVE_NB] = X[i + j * LD];
    out[i + (int64_t)(j + H) * SOLVE_NB] = 0.0;
  }
  if (b2 <= 0) {
    for (int idx = tid; idx < H * H; idx += NT) {
      const int i = idx % H, j = idx / H;
      out[(i + H) + (int64_t)j * SOLVE_NB] = 0.0;
      out[(i + H) + (int64_t)(j + H) * SOLVE_NB] = 0.0;
    }
    return;
  }
  // T = L21 X1 (X1(k, j) = 0 for k < j)
  double t[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + NT * q, i = idx % H, j = idx / H;
    double acc = 0.0;
    for (int k = j; k < H; ++k) acc += M[i + k * LD] * X[k + j * LD];
    t[q] = acc;
  }
  __syncthreads();
  const double* X2 = inv + d.x2_off;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = tid + NT * q, i = idx % H, j = idx / H;
    M[i + j * LD] = t[q];
    X[i + j * LD] = X2[i + j * H];
  }
  __syncthreads();
  // Y = -X2 T (X2(i, k) = 0 for k > i), and X2 itself
  for (int idx = tid; idx < H * H; idx += NT) {
    const int i = idx % H, j = idx / H;
    double acc = 0.0;
    for (int k = 0; k <= i; ++k) acc += X[i + k * LD] * M[k + j * LD];
    out[(i + H) + (int64_t)j * SOLVE_NB] = -acc;
    out[(i + H) + (int64_t)(j + H) * SOLVE_NB] = X[i + j * LD];
  }
}

// Forward solve, small supernodes (h <= 64): one workgroup, vector in LDS.
template <typename T>
__global__ void __launch_bounds__(BS) k_fwd_small(DevPlan P, int64_t d0, const T* panel, const double* xp,
                                                 double* ys, double* uvec, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  __shared__ double t[64];
  const int32_t S = P.ssmall[d0 + blockIdx.x];
  const int h = P.sh[S], w = P.sw[S], f = P.sfirst[S], ld = P.sld[S];
  const T* L = panel + P.spanel[S];
  if ((int)threadIdx.x < h) t[threadIdx.x] = (int)threadIdx.x < w ? xp[f + threadIdx.x] : 0.0;
  __syncthreads();
  for (int32_t q = P.child_ptr[S]; q < P.child_ptr[S + 1]; ++q) {
    const int32_t c = P.child[q];
    const int hu = P.sh[c] - P.sw[c];
    const int32_t* rc = P.rel + P.srow[c] + P.sw[c];
    const double* uc = uvec + P.suv[c];
    for (int i = threadIdx.x; i < hu; i += BS) t[rc[i]] += uc[i];
    __syncthreads();
  }
  for (int j = 0; j < w; ++j) {
    const double yj = t[j] / (double)L[j + (int64_t)j * ld];
    if ((int)threadIdx.x > j && (int)threadIdx.x < h) t[threadIdx.x] -= (double)L[threadIdx.x + (int64_t)j * ld] * yj;
    __syncthreads();
  }
  if ((int)threadIdx.x < w) ys[f + threadIdx.x] = t[threadIdx.x] / (double)L[threadIdx.x + (int64_t)threadIdx.x * ld];
  else if ((int)threadIdx.x < h) uvec[P.suv[S] + threadIdx.x - w] = t[threadIdx.x];
}

// Inverse of a diagonal block (lower triangular, column-major, NB x NB
// storage per block, NB = SOLVE_NB) held in registers: wave w
// keeps the columns j = w, w + NW, ... and every lane the rows lane (and
// lane + 64).  The whole block is requested in one round of independent
// loads (the gather kernel issues it before the vector it multiplies is
// known), so a dependent chain of solve steps pays one memory latency here
// instead of one per column group.
template <int NT, typename T>
struct InvBlock {
  static constexpr int NB = SOLVE_NB, NW = NT / 64, JPW = NB / NW, RPL = NB / 64;
  T v[JPW][RPL];
  __device__ void load(const T* I) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < JPW; ++m)
#pragma unroll
      for (int r = 0; r < RPL; ++r) v[m][r] = I[(lane + 64 * r) + (int64_t)(wave + m * NW) * NB];
  }
  // ys[k] = sum over j <= k of inv(k, j) t[j] for k < bw (t in LDS); the
  // waves' partial sums meet in red (NW * NB doubles of LDS) in a fixed
  // order.  Entries outside the triangle are never used.  Must be reached by
  // the whole workgroup.
  __device__ void lower_times(int bw, const double* t, double* red, double* ys) const {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double a[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) a[r] = 0.0;
#pragma unroll
    for (int m = 0; m < JPW; ++m) {
      const int j = wave + m * NW;
      const double tj = j < bw ? t[j] : 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int k = lane + 64 * r;
        const double p = (double)v[m][r] * tj;
        a[r] += (k >= j && k < bw && j < bw) ? p : 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) red[wave * NB + lane + 64 * r] = a[r];
    __syncthreads();
    if (tid < bw) {
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) sum += red[q * NB + tid];
      ys[tid] = sum;
    }
  }
};
// Forward solve, large supernodes: each front row sums its children's
// update-vector entries (the plan's gather map lists them in child order,
// so the sum is deterministic) into x (own columns) or into the front's
// update vector (rows below).  One thread per row; rows of many fronts at
// once, where one workgroup per front adding child after child serialised
// the 200 children of a separator.
__global__ void __launch_bounds__(GATHER_ROWS) k_fwd_gather(DevPlan P, int64_t d0, double* xp, double* uvec,
                                                           const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  const GatherItem g = P.gitem[d0 + blockIdx.x];
  const int32_t S = g.sn;
  const int w = P.sw[S], f = P.sfirst[S];
  const int64_t uo = P.suv[S];
  const int64_t* rp = P.gptr + P.grow[S];
  const int r = g.r0 + (int)threadIdx.x;
  if (r >= g.r1) return;
  double s = 0.0;
  const int64_t k1 = rp[r + 1];
#pragma unroll 4
  for (int64_t k = rp[r]; k < k1; ++k) s += uvec[P.gidx[k]];
  if (r < w) xp[f + r] += s;
  else uvec[uo + r - w] = s;
}

// Forward solve, large supernodes: y of the first column block from the
// gathered right-hand side.
template <typename T>
__global__ void __launch_bounds__(BS) k_fwd_first(DevPlan P, int64_t d0, const T* inv, const double* xp, double* ys,
                                                 const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  typedef InvBlock<BS, T> IB;
  __shared__ double tb[IB::NB], red[IB::NW * IB::NB];
  const int32_t S = P.slarge[d0 + blockIdx.x];
  const int w = P.sw[S], f = P.sfirst[S];
  IB ib;
  ib.load(inv + P.sinv[S]);
  const int bw = w < IB::NB ? w : IB::NB;
  if ((int)threadIdx.x < bw) tb[threadIdx.x] = xp[f + threadIdx.x];
  __syncthreads();
  ib.lower_times(bw, tb, red, ys + f);
}

template <int C>
__device__ inline void halve_step(double* acc, bool upper, int o) {
#pragma unroll
  for (int j = 0; j < C / 2; ++j) {
    const double send = upper ? acc[j] : acc[j + C / 2];
    const double keep = upper ? acc[j + C / 2] : acc[j];
    acc[j] = keep + __shfl_xor(send, o, 64);
  }
}

template <typename T> struct VecOf;
template <> struct VecOf<float> { typedef float4 type; static constexpr int n = 4; };
template <> struct VecOf<double> { typedef double2 type; static constexpr int n = 2; };

// Forward solve step of column block J: every item updates its rows with
// y_J; the owner item (its rows start with block J+1) then forms y_{J+1}.
// Lanes load VEC consecutive rows of a column with one vector load; the eight
// waves split the block's columns and are summed through LDS in a fixed order.
// y_J comes straight from global memory into registers, so the panel and y
// loads of a step are in flight together (the steps of a wide supernode form
// a dependent chain whose length is set by these latencies); the owner loads
// its inverse block in one round after the rows are done (holding it in
// registers through the row loop cost occupancy: 4.5% less bandwidth in the
// large launches).
template <typename T>
__global__ void __launch_bounds__(SBS) k_fwd_step(DevPlan P, int64_t d0, const T* panel, const T* inv,
                                                double* xp, double* ys, double* uvec, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  typedef InvBlock<SBS, T> IB;
  constexpr int VEC = VecOf<T>::n, NW = SBS / 64, CPW = 128 / NW, RW = 64 * VEC;
  typedef typename VecOf<T>::type V;
  __shared__ double tb[IB::NB], red_inv[IB::NW * IB::NB];
  __shared__ double red[NW * RW];
  const SolveDesc d = P.sdesc[d0 + blockIdx.x];
  const int w = d.w, f = d.first, ld = d.ld;
  const int64_t uo = d.uvec_off;
  const int bw = d.bw, c0 = d.c0, nc0 = c0 + bw;
  const T* L = panel + d.panel_off + (int64_t)c0 * ld;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), cb = wave * CPW;
  const int ncol = bw - cb < CPW ? bw - cb : CPW;
  double y[CPW];
#pragma unroll
  for (int m = 0; m < CPW; ++m) y[m] = m < ncol ? ys[f + c0 + cb + m] : 0.0;
  for (int rb = d.r0 & ~(VEC - 1); rb < d.r1; rb += RW) {
    const int i0 = rb + lane * VEC;
    // the row this thread finishes below, read now to overlap the panel loads
    const int io = rb + tid;
    const bool mine = tid < RW && io >= d.r0 && io < d.r1;
    const double old = mine ? (io < w ? xp[f + io] : uvec[uo + io - w]) : 0.0;
    double a[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) a[e] = 0.0;
    const bool full = i0 >= d.r0 && i0 + VEC <= d.r1;
    const bool any = i0 + VEC > d.r0 && i0 < d.r1;
    if (any) {
#pragma unroll
      for (int m = 0; m < CPW; ++m) {
        if (m < ncol) {
          const T* p = L + (int64_t)(cb + m) * ld + i0;
          T v[VEC];
          if (full) {
            const V q = *(const V*)p;
            v[0] = q.x; v[1] = q.y;
            if constexpr (VEC == 4) { v[2] = q.z; v[3] = q.w; }
          } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = (i0 + e >= d.r0 && i0 + e < d.r1) ? p[e] : (T)0;
          }
#pragma unroll
          for (int e = 0; e < VEC; ++e) a[e] += (double)v[e] * y[m];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) red[wave * RW + lane * VEC + e] = a[e];
    __syncthreads();
    if (mine) {
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) sum += red[q * RW + tid];
      const double v = old - sum;
      if (io < w) {
        xp[f + io] = v;
        if (d.owner && io - nc0 < IB::NB) tb[io - nc0] = v;
      } else {
        uvec[uo + io - w] = v;
      }
    }
    __syncthreads();
  }
  if (d.owner) {
    IB ib;
    ib.load(inv + d.inv_off + (int64_t)(nc0 / IB::NB) * IB::NB * IB::NB);
    const int bw2 = w - nc0 < IB::NB ? w - nc0 : IB::NB;
    ib.lower_times(bw2, tb, red_inv, ys + f + nc0);
  }
}

// Backward solve, small supernodes.
template <typename T>
__global__ void __launch_bounds__(BS) k_bwd_small(DevPlan P, int64_t d0, const T* panel, double* ys, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  __shared__ double y[64], xr[64];
  const int32_t S = P.ssmall[d0 + blockIdx.x];
  const int h = P.sh[S], w = P.sw[S], f = P.sfirst[S], ld = P.sld[S];
  const int hu = h - w;
  const T* L = panel + P.spanel[S];
  const int32_t* rows = P.sn_rows + P.srow[S];
  const int tid = threadIdx.x;
  if (tid < w) y[tid] = ys[f + tid];
  if (tid < hu) xr[tid] = ys[rows[w + tid]];
  __syncthreads();
  if (tid < w) {
    double s = 0.0;
    for (int i = 0; i < hu; ++i) s += (double)L[(w + i) + (int64_t)tid * ld] * xr[i];
    y[tid] -= s;
  }
  __syncthreads();
  for (int j = w - 1; j >= 0; --j) {
    const double xj = y[j] / (double)L[j + (int64_t)j * ld];
    if (tid < j) y[tid] -= (double)L[j + (int64_t)tid * ld] * xj;
    __syncthreads();
  }
  if (tid < w) ys[f + tid] = y[tid] / (double)L[tid + (int64_t)tid * ld];
}

// Backward solve, large supernodes: partial products L(rows, J)' x(rows)
// over a row range below column block J.  Each lane loads VEC consecutive
// rows of a column with one vector load (coalesced along the column), each
// of the eight waves owns 16 columns of the block and keeps one FP64
// accumulator per column; the 64 lanes are combined by recursive halving
// (17 exchanges in all instead of 6 per column).
template <typename T>
__global__ void __launch_bounds__(SBS) k_bwd_part(DevPlan P, int64_t d0, const T* panel, const double* ys,
                                                double* part, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  constexpr int CPW = 16, VEC = VecOf<T>::n;   // eight waves of 16 columns
  typedef typename VecOf<T>::type V;
  const SolveDesc d = P.sdesc[d0 + blockIdx.x];
  const int w = d.w, f = d.first, ld = d.ld;
  const T* L = panel + d.panel_off + (int64_t)d.c0 * ld;   // 16-byte aligned columns
  const int32_t* rows = P.sn_rows + d.row_off;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cb = wave * CPW;
  double acc[CPW];
#pragma unroll
  for (int m = 0; m < CPW; ++m) acc[m] = 0.0;
  if (cb < d.bw) {
    const int ncol = d.bw - cb < CPW ? d.bw - cb : CPW;
    for (int rb = d.r0 & ~(VEC - 1); rb < d.r1; rb += 64 * VEC) {
      const int i0 = rb + lane * VEC;
      double xv[VEC];
      bool any = false;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int i = i0 + e;
        const bool in = i >= d.r0 && i < d.r1;
        xv[e] = in ? (i < w ? ys[f + i] : ys[rows[i]]) : 0.0;
        any |= in;
      }
      const bool full = i0 >= d.r0 && i0 + VEC <= d.r1;
      if (!any) continue;
#pragma unroll
      for (int m = 0; m < CPW; ++m) {
        if (m < ncol) {
          const T* p = L + (int64_t)(cb + m) * ld + i0;
          T v[VEC];
          if (full) {
            const V q = *(const V*)p;
            v[0] = q.x; v[1] = q.y;
            if constexpr (VEC == 4) { v[2] = q.z; v[3] = q.w; }
          } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = (i0 + e >= d.r0 && i0 + e < d.r1) ? p[e] : (T)0;
          }
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[m] += (double)v[e] * xv[e];
        }
      }
    }
  }
  halve_step<16>(acc, lane & 32, 32);
  halve_step<8>(acc, lane & 16, 16);
  halve_step<4>(acc, lane & 8, 8);
  halve_step<2>(acc, lane & 4, 4);
  acc[0] += __shfl_xor(acc[0], 2, 64);
  acc[0] += __shfl_xor(acc[0], 1, 64);
  const int c = cb + ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
  if ((lane & 3) == 0 && c < d.bw) part[d.part_off + c] = acc[0];
}

// Backward solve, diagonal block: x_J = inv(L_JJ)' (y_J - sum of partials).
// All memory traffic is requested up front: each wave's 16 columns of the
// inverse (column k contiguous, lanes along it), y_J, and the partials, of
// which every thread sums one column's share with up to 16 loads in flight
// (groups of threads per column, combined in a fixed order).  Each wave then
// reduces its 16 columns by recursive halving.
template <typename T>
__global__ void __launch_bounds__(SBS) k_bwd_diag(DevPlan P, int64_t d0, const T* inv, double* ys,
                                                const double* part, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  constexpr int NB = SOLVE_NB, CPW = 16, RPL = NB / 64;
  constexpr int NG = SBS / NB, PU = 16;   // thread groups per column; partial loads per round
  __shared__ double z[NB], zp[NG * NB];
  const SolveDesc d = P.sdesc[d0 + blockIdx.x];
  const int f = d.first, bw = d.bw;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), cb = wave * CPW;
  const T* I = inv + d.inv_off + (int64_t)(d.c0 / NB) * NB * NB;
  T v[CPW][RPL];
  if (cb < NB) {
#pragma unroll
    for (int m = 0; m < CPW; ++m)
#pragma unroll
      for (int r = 0; r < RPL; ++r) v[m][r] = I[(lane + 64 * r) + (int64_t)(cb + m) * NB];
  }
  const int c = tid % NB, g = tid / NB;
  const double yv = (g == 0 && c < bw) ? ys[f + d.c0 + c] : 0.0;
  double sp = 0.0;
  if (c < bw) {
    const double* pp = part + d.part_off + c;
    for (int q0 = g; q0 < d.nparts; q0 += NG * PU) {
      double t[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int q = q0 + u * NG;
        t[u] = q < d.nparts ? pp[(int64_t)q * NB] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PU; ++u) sp += t[u];
    }
  }
  zp[g * NB + c] = sp;
  __syncthreads();
  if (g == 0) {
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < NG; ++q) tot += zp[q * NB + c];
    z[c] = c < bw ? yv - tot : 0.0;
  }
  __syncthreads();
  double acc[CPW];
#pragma unroll
  for (int m = 0; m < CPW; ++m) {
    acc[m] = 0.0;
    if (cb < NB) {
      const int k = cb + m;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        const double p = (double)v[m][r] * z[i];
        acc[m] += (k < bw && i >= k && i < bw) ? p : 0.0;
      }
    }
  }
  halve_step<16>(acc, lane & 32, 32);
  halve_step<8>(acc, lane & 16, 16);
  halve_step<4>(acc, lane & 8, 8);
  halve_step<2>(acc, lane & 4, 4);
  acc[0] += __shfl_xor(acc[0], 2, 64);
  acc[0] += __shfl_xor(acc[0], 1, 64);
  const int col = cb + ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
  if ((lane & 3) == 0 && col < bw) ys[f + d.c0 + col] = acc[0];
}

// -------------------------------------------------------- IPM vectors
__global__ void k_residuals(DevProblem P, const double* jtl, const double* gf, const double* zl,
                            const double* zu, const double* g, const double* s, double* rd, double* rp, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < P.n) rd[i] = gf[i] - jtl[i] - (has_lo(P.xl[i]) ? zl[i] : 0.0) + (has_hi(P.xu[i]) ? zu[i] : 0.0);
  if (i < P.m) rp[i] = g[i] - s[i];
}

// Per-iteration statistics: max|r_p|, max|g|, max|r_d|, max|grad f|,
// complementarity sum, objective sum, count of non-finite values.
__global__ void k_stats_iter(DevProblem P, IpmVecs v, double* partials, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  RedSpec spec{7, {RED_MAX, RED_MAX, RED_MAX, RED_MAX, RED_SUM, RED_SUM, RED_SUM}};
  double a[7] = {0, 0, 0, 0, 0, 0, 0};
  const int64_t N = P.n > P.m ? P.n : P.m;
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < N; i += (int64_t)gridDim.x * BS) {
    if (i < P.m) {
      a[0] = fmax(a[0], fabs(v.rp[i]));
      a[1] = fmax(a[1], fabs(v.g[i]));
      a[4] += v.s[i] * v.lam[i];
      if (!isfinite(v.rp[i]) || !isfinite(v.lam[i])) a[6] += 1;
    }
    if (i < P.n) {
      const double x = v.x[i];
      a[2] = fmax(a[2], fabs(v.rd[i]));
      a[3] = fmax(a[3], fabs(v.gf[i]));
      if (has_lo(P.xl[i])) a[4] += (x - P.xl[i]) * v.zl[i];
      if (has_hi(P.xu[i])) a[4] += (P.xu[i] - x) * v.zu[i];
      a[5] += P.c[i] * x + 0.5 * x * v.qx[i] + (P.q4 ? 0.25 * P.q4[i] * x * x * x * x : 0.0);
      if (!isfinite(v.rd[i]) || !isfinite(x)) a[6] += 1;
    }
  }
  block_reduce_store<7>(a, spec, partials);
}

__global__ void k_sigmas(DevProblem P, IpmVecs v, double dd, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < P.m) v.sig_s[i] = v.lam[i] / (v.s[i] + dd * v.lam[i]);
  if (i < P.n) {
    double sx = 0.0;
    if (has_lo(P.xl[i])) sx += v.zl[i] / (v.x[i] - P.xl[i]);
    if (has_hi(P.xu[i])) sx += v.zu[i] / (P.xu[i] - v.x[i]);
    v.sig_x[i] = sx;
  }
}

__global__ void k_rhs_m(DevProblem P, IpmVecs v, const double* ts, double* wm, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t k = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (k < P.m) wm[k] = v.sig_s[k] * (v.g[k] - (ts ? ts[k] / v.lam[k] : 0.0));
}

__global__ void k_rhs_n(DevProblem P, IpmVecs v, const double* jtw, const double* tl, const double* tu,
                        double* rhs, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i >= P.n) return;
  double rt = v.rd[i];
  if (has_lo(P.xl[i])) rt += -(tl ? tl[i] : 0.0) / (v.x[i] - P.xl[i]) + v.zl[i];
  if (has_hi(P.xu[i])) rt += (tu ? tu[i] : 0.0) / (P.xu[i] - v.x[i]) - v.zu[i];
  rhs[i] = -rt - jtw[i];
}

__global__ void k_recover_m(DevProblem P, IpmVecs v, const double* jdx, const double* ts, double dd,
                            double* ds, double* dlam, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t k = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (k >= P.m) return;
  const double dl = v.sig_s[k] * ((ts ? ts[k] / v.lam[k] : 0.0) - v.g[k] - jdx[k]);
  dlam[k] = dl;
  ds[k] = jdx[k] + v.rp[k] + dd * dl;
}

__global__ void k_recover_n(DevProblem P, IpmVecs v, const double* dx, const double* tl, const double* tu,
                            double* dzl, double* dzu, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i >= P.n) return;
  if (has_lo(P.xl[i])) {
    const double gap = v.x[i] - P.xl[i];
    dzl[i] = (tl ? tl[i] : 0.0) / gap - v.zl[i] - v.zl[i] / gap * dx[i];
  } else {
    dzl[i] = 0.0;
  }
  if (has_hi(P.xu[i])) {
    const double gap = P.xu[i] - v.x[i];
    dzu[i] = (tu ? tu[i] : 0.0) / gap - v.zu[i] + v.zu[i] / gap * dx[i];
  } else {
    dzu[i] = 0.0;
  }
}

__device__ inline void ratio(double& a, double val, double d) {
  if (d < 0.0) a = fmin(a, -val / d);
}

// Largest steps keeping (s, x-l, u-x) and (lambda, z_l, z_u) non-negative.
__global__ void k_step_limits(DevProblem P, IpmVecs v, const double* dx, const double* ds,
                              const double* dlam, const double* dzl, const double* dzu, double* partials, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  RedSpec spec{2, {RED_MIN, RED_MIN}};
  double a[2] = {INFINITY, INFINITY};
  const int64_t N = P.n > P.m ? P.n : P.m;
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < N; i += (int64_t)gridDim.x * BS) {
    if (i < P.m) {
      ratio(a[0], v.s[i], ds[i]);
      ratio(a[1], v.lam[i], dlam[i]);
    }
    if (i < P.n) {
      if (has_lo(P.xl[i])) { ratio(a[0], v.x[i] - P.xl[i], dx[i]); ratio(a[1], v.zl[i], dzl[i]); }
      if (has_hi(P.xu[i])) { ratio(a[0], P.xu[i] - v.x[i], -dx[i]); ratio(a[1], v.zu[i], dzu[i]); }
    }
  }
  block_reduce_store<2>(a, spec, partials);
}

__global__ void k_mu_aff(DevProblem P, IpmVecs v, const double* dx, const double* ds, const double* dlam,
                         const double* dzl, const double* dzu, double ap, double ad, double* partials, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  RedSpec spec{1, {RED_SUM}};
  double a[1] = {0.0};
  const int64_t N = P.n > P.m ? P.n : P.m;
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < N; i += (int64_t)gridDim.x * BS) {
    if (i < P.m) a[0] += (v.s[i] + ap * ds[i]) * (v.lam[i] + ad * dlam[i]);
    if (i < P.n) {
      if (has_lo(P.xl[i])) a[0] += (v.x[i] - P.xl[i] + ap * dx[i]) * (v.zl[i] + ad * dzl[i]);
      if (has_hi(P.xu[i])) a[0] += (P.xu[i] - v.x[i] - ap * dx[i]) * (v.zu[i] + ad * dzu[i]);
    }
  }
  block_reduce_store<1>(a, spec, partials);
}

__global__ void k_targets(DevProblem P, const double* dx, const double* ds, const double* dlam,
                          const double* dzl, const double* dzu, double smu, double* ts, double* tl,
                          double* tu, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < P.m) ts[i] = smu - ds[i] * dlam[i];
  if (i < P.n) {
    tl[i] = has_lo(P.xl[i]) ? smu - dx[i] * dzl[i] : 0.0;
    tu[i] = has_hi(P.xu[i]) ? smu + dx[i] * dzu[i] : 0.0;
  }
}

__global__ void k_axpy_point(DevProblem P, IpmVecs dst, IpmVecs src, const double* dx, const double* ds,
                             const double* dlam, const double* dzl, const double* dzu, double ap, double ad, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < P.m) {
    dst.s[i] = src.s[i] + ap * ds[i];
    dst.lam[i] = src.lam[i] + ad * dlam[i];
  }
  if (i < P.n) {
    dst.x[i] = src.x[i] + ap * dx[i];
    dst.zl[i] = has_lo(P.xl[i]) ? src.zl[i] + ad * dzl[i] : 0.0;
    dst.zu[i] = has_hi(P.xu[i]) ? src.zu[i] + ad * dzu[i] : 0.0;
  }
}

// Squared residual norm of the perturbed KKT conditions (NLP line search).
__global__ void k_phi(DevProblem P, IpmVecs v, double smu, double* partials, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  RedSpec spec{1, {RED_SUM}};
  double a[1] = {0.0};
  const int64_t N = P.n > P.m ? P.n : P.m;
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < N; i += (int64_t)gridDim.x * BS) {
    if (i < P.m) {
      const double c = v.s[i] * v.lam[i] - smu;
      a[0] += v.rp[i] * v.rp[i] + c * c;
    }
    if (i < P.n) {
      a[0] += v.rd[i] * v.rd[i];
      if (has_lo(P.xl[i])) { const double c = (v.x[i] - P.xl[i]) * v.zl[i] - smu; a[0] += c * c; }
      if (has_hi(P.xu[i])) { const double c = (P.xu[i] - v.x[i]) * v.zu[i] - smu; a[0] += c * c; }
    }
  }
  block_reduce_store<1>(a, spec, partials);
}

__global__ void k_init_point(DevProblem P, IpmVecs v, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < P.n) {
    const bool lo = has_lo(P.xl[i]), hi = has_hi(P.xu[i]);
    double x = 0.0;
    if (lo && hi) x = 0.5 * (P.xl[i] + P.xu[i]);
    else if (lo) x = P.xl[i] + 1.0;
    else if (hi) x = P.xu[i] - 1.0;
    v.x[i] = x;
    v.zl[i] = lo ? 1.0 : 0.0;
    v.zu[i] = hi ? 1.0 : 0.0;
  }
  if (i < P.m) v.lam[i] = 1.0;
}

__global__ void k_slack_from_g(DevProblem P, IpmVecs v, int warm, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t k = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (k >= P.m) return;
  const double g = v.g[k];
  v.s[k] = warm ? fmax(g, 1e-2 * fmax(1.0, fabs(g))) : fmax(g, 1.0);
}

// Interior push of a supplied point (bound-push rule of Waechter-Biegler).
__global__ void k_push_x(DevProblem P, IpmVecs v, const double* xhat, const double* lamhat, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < P.n) {
    const bool lo = has_lo(P.xl[i]), hi = has_hi(P.xu[i]);
    const double width = (lo && hi) ? P.xu[i] - P.xl[i] : INFINITY;
    double x = xhat[i];
    if (lo) x = fmax(x, P.xl[i] + fmin(1e-2 * fmax(1.0, fabs(P.xl[i])), 1e-2 * width));
    if (hi) x = fmin(x, P.xu[i] - fmin(1e-2 * fmax(1.0, fabs(P.xu[i])), 1e-2 * width));
    v.x[i] = x;
  }
  if (i < P.m) v.lam[i] = fmax(lamhat[i], 1e-2);
}

__global__ void k_push_duals(DevProblem P, IpmVecs v, double mu_w, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i >= P.n) return;
  v.zl[i] = has_lo(P.xl[i]) ? mu_w / (v.x[i] - P.xl[i]) : 0.0;
  v.zu[i] = has_hi(P.xu[i]) ? mu_w / (P.xu[i] - v.x[i]) : 0.0;
}

__global__ void k_sum_sl(DevProblem P, IpmVecs v, double* partials, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  RedSpec spec{1, {RED_SUM}};
  double a[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < P.m; i += (int64_t)gridDim.x * BS)
    a[0] += v.s[i] * v.lam[i];
  block_reduce_store<1>(a, spec, partials);
}

// K v = H v + (Sigma_x + delta_p) v + J'(Sigma_s (J v)), second part
__global__ void k_kfree_m(int64_t m, const double* sig_s, double* jv_tmp, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t k = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (k < m) jv_tmp[k] *= sig_s[k];
}
__global__ void k_kfree_n(int64_t n, const double* hv_v, const double* jt, const double* sig_x, double dp,
                          const double* v, double* out, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < n) out[i] = hv_v[i] + jt[i] + (sig_x[i] + dp) * v[i];
}

__global__ void k_residual_norms(int64_t n, const double* rhs, const double* kx, const double* x, double* r,
                                 double* partials, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  RedSpec spec{3, {RED_MAX, RED_MAX, RED_MAX}};
  double a[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const double ri = rhs[i] - kx[i];
    r[i] = ri;
    a[0] = fmax(a[0], fabs(ri));
    a[1] = fmax(a[1], fabs(rhs[i]));
    a[2] = fmax(a[2], fabs(x[i]));
    if (!isfinite(ri)) a[0] = INFINITY;
  }
  block_reduce_store<3>(a, spec, partials);
}

__global__ void k_dot(int64_t n, const double* a, const double* b, double* partials, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  RedSpec spec{1, {RED_SUM}};
  double acc[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) acc[0] += a[i] * b[i];
  block_reduce_store<1>(acc, spec, partials);
}

// x += alpha p, r -= alpha q; reports max|r| and max|x|.
__global__ void k_cg_step(int64_t n, double alpha, const double* p, const double* q, double* x, double* r,
                          double* partials, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  RedSpec spec{2, {RED_MAX, RED_MAX}};
  double a[2] = {0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const double xi = x[i] + alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    x[i] = xi;
    r[i] = ri;
    a[0] = fmax(a[0], fabs(ri));
    a[1] = fmax(a[1], fabs(xi));
    if (!isfinite(ri)) a[0] = INFINITY;
  }
  block_reduce_store<2>(a, spec, partials);
}

__global__ void k_xpby(int64_t n, const double* z, double beta, double* p, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < n) p[i] = z[i] + beta * p[i];
}

__global__ void k_add(int64_t n, double* x, const double* c, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < n) x[i] += c[i];
}
__global__ void k_copy(int64_t n, double* d, const double* s, const int* gate) {
  if (gate && *gate == 0) return;   // gated launch whose gate is closed
  int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x;
  if (i < n) d[i] = s[i];
}

inline int red_grid(int64_t N) {
  int64_t b = blocks_for(N);
  return (int)(b < RED_BLOCKS ? b : RED_BLOCKS);
}

}  // namespace

// ============================================================ wrappers
namespace {
thread_local const int* g_launch_gate = nullptr;
}  // namespace
void set_launch_gate(const int* gate) { g_launch_gate = gate; }
const int* launch_gate() { return g_launch_gate; }

void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = blocks_for(n);
  if (g > 65536) g = 65536;
  k_fill_f64<<<(unsigned)g, BS, 0, s>>>(p, n, v, launch_gate());
}
void launch_fill_bytes0(void* p, int64_t bytes, hipStream_t s) {
  int64_t n = bytes / 4;
  if (n <= 0) return;
  int64_t g = blocks_for(n);
  if (g > 65536) g = 65536;
  k_zero_u32<<<(unsigned)g, BS, 0, s>>>((uint32_t*)p, n, launch_gate());
}
void launch_finalize(const double* partials, int nblocks, RedSpec spec, double* out, hipStream_t s) {
  k_finalize<<<1, BS, 0, s>>>(partials, nblocks, spec, out, launch_gate());
}

void launch_jv_copy(const DevProblem& P, double* jv, hipStream_t s) {
  if (P.nnz_j == 0) return;
  launch_copy(P.nnz_j, jv, P.ja, s);
  k_jv_transpose<<<(unsigned)blocks_for(P.nnz_j), BS, 0, s>>>(P.nnz_j, P.jte, jv, jv + P.nnz_j, launch_gate());
}
void launch_jac_eval(const DevProblem& P, const double* x, double* jv, hipStream_t s) {
  if (P.nnz_j == 0) return;
  k_jac_eval<<<(unsigned)blocks_for(P.nnz_j), BS, 0, s>>>(P.nnz_j, P.ja, P.jw, P.jc, x, jv, launch_gate());
  k_jv_transpose<<<(unsigned)blocks_for(P.nnz_j), BS, 0, s>>>(P.nnz_j, P.jte, jv, jv + P.nnz_j, launch_gate());
}
void launch_constraints(const DevProblem& P, const double* x, double* g, hipStream_t s) {
  if (P.m == 0) return;
  k_constraints<<<(unsigned)blocks_for(P.m), BS, 0, s>>>(P.m, P.jp, P.jc, P.ja, P.jw, x, P.b, g, launch_gate());
}
void launch_gradient(const DevProblem& P, const double* x, double* qx, double* gf, hipStream_t s) {
  k_gradient<<<(unsigned)blocks_for(P.n), BS, 0, s>>>(P.n, P.hsp, P.hsc, P.hss, P.hq, P.c, P.q4, x, qx, gf, launch_gate());
}
void launch_hess_eval(const DevProblem& P, const double* x, const double* lam, double* hv, hipStream_t s) {
  k_hess_eval<<<(unsigned)blocks_for(P.n), BS, 0, s>>>(P.n, P.hp, P.hdiag, P.hq, P.q4, P.jtp, P.jtr, P.jte,
                                                        P.jw, x, lam, hv, launch_gate());
}
void launch_jt_mul(const DevProblem& P, const double* jv, const double* y, double* out, hipStream_t s) {
  k_jt_mul<<<(unsigned)blocks_for(P.n), BS, 0, s>>>(P.n, P.jtp, P.jtr, jv + P.nnz_j, y, out, launch_gate());
}
void launch_j_mul(const DevProblem& P, const double* jv, const double* v, double* out, hipStream_t s) {
  if (P.m == 0) return;
  const int64_t g = (P.m + BS / JROW - 1) / (BS / JROW);
  if (g > 0) k_j_mul<<<(unsigned)g, BS, 0, s>>>(P.m, P.jp, P.jc, jv, v, out, launch_gate());
}
void launch_h_mul(const DevProblem& P, const double* hv, const double* v, double* out, hipStream_t s) {
  k_h_mul<<<(unsigned)blocks_for(P.n), BS, 0, s>>>(P.n, P.hsp, P.hsc, P.hss, hv, v, out, launch_gate());
}

template <typename T>
void launch_assemble(const DevKMap& K, const double* hv, const double* jv, const double* sig_s,
                     const double* sig_x, double delta_p, T* panel, double* kval, hipStream_t s) {
  k_assemble<T><<<(unsigned)blocks_for(K.nk), BS, 0, s>>>(K, hv, jv, sig_s, sig_x, delta_p, panel, kval, launch_gate());
}
template void launch_assemble<double>(const DevKMap&, const double*, const double*, const double*,
                                      const double*, double, double*, double*, hipStream_t);
template void launch_assemble<float>(const DevKMap&, const double*, const double*, const double*,
                                     const double*, double, float*, double*, hipStream_t);
template <typename T>
void launch_set_values(const DevKMap& K, const double* kval, T* panel, hipStream_t s) {
  k_set_values<T><<<(unsigned)blocks_for(K.nk), BS, 0, s>>>(K, kval, panel, launch_gate());
}
template void launch_set_values<double>(const DevKMap&, const double*, double*, hipStream_t);
template void launch_set_values<float>(const DevKMap&, const double*, float*, hipStream_t);

void launch_k_mul_stored(int64_t n, const int64_t*, const int32_t*, const int64_t* ksp, const int32_t* ksc,
                         const int64_t* kss, const double* kval, const double* v, double* out, hipStream_t s) {
  k_k_mul_stored<<<(unsigned)blocks_for(n), BS, 0, s>>>(n, ksp, ksc, kss, kval, v, out, launch_gate());
}

template <typename T>
void launch_factor_op(const Op& op, const DevPlan& P, T* panel, T* ubuf, T* inv, int* bad, hipStream_t s) {
  if (op.grid <= 0) return;
  const unsigned g = (unsigned)op.grid;
  switch (op.type) {
    case OP_EXTEND_ADD: k_extend_add<T><<<g, BS, 0, s>>>(P, op.begin, panel, ubuf, launch_gate()); break;
    case OP_SMALL: k_small_front<T><<<g, BS, 0, s>>>(P, op.begin, panel, ubuf, bad, launch_gate()); break;
    case OP_POTRF:
      if (P.sign) {
        if constexpr (sizeof(T) == 8) k_potrf<T, 64, 256, true><<<g, 256, 0, s>>>(P, op.begin, panel, inv, bad, launch_gate());
        else k_potrf<T, 128, 256, true><<<g, 256, 0, s>>>(P, op.begin, panel, inv, bad, launch_gate());
      } else {
        if constexpr (sizeof(T) == 8) k_potrf<T, 64, 256, false><<<g, 256, 0, s>>>(P, op.begin, panel, inv, bad, launch_gate());
        else if (op.grid <= 256) k_potrf<T, 128, 512, false><<<g, 512, 0, s>>>(P, op.begin, panel, inv, bad, launch_gate());
        else k_potrf<T, 128, 256, false><<<g, 256, 0, s>>>(P, op.begin, panel, inv, bad, launch_gate());
      }
      break;
    case OP_TRSM:
    case OP_UPDATE: {
      const unsigned g8 = (unsigned)((op.grid + 7) / 8 * 8);
      if (P.sign) {
        if constexpr (sizeof(T) == 8)
          k_gemm_f64<true><<<g8, BS64, 0, s>>>(P, op.begin, op.end, op.grid, panel, ubuf, inv, launch_gate());
        else k_gemm_f32<true><<<g8, BS32, 0, s>>>(P, op.begin, op.end, op.grid, panel, ubuf, inv, launch_gate());
      } else {
        if constexpr (sizeof(T) == 8)
          k_gemm_f64<false><<<g8, BS64, 0, s>>>(P, op.begin, op.end, op.grid, panel, ubuf, inv, launch_gate());
        else k_gemm_f32<false><<<g8, BS32, 0, s>>>(P, op.begin, op.end, op.grid, panel, ubuf, inv, launch_gate());
      }
      break;
    }
    case OP_INV_COMBINE:
      if constexpr (sizeof(T) == 8) k_inv_combine<<<g, 256, 0, s>>>(P, op.begin, panel, inv, launch_gate());
      break;
  }
}
template void launch_factor_op<double>(const Op&, const DevPlan&, double*, double*, double*, int*, hipStream_t);
template void launch_factor_op<float>(const Op&, const DevPlan&, float*, float*, float*, int*, hipStream_t);

void launch_sign_scale(int64_t n, const signed char* sign, double* y, hipStream_t s) {
  if (n > 0) k_sign_scale<<<(unsigned)blocks_for(n), BS, 0, s>>>(n, sign, y, launch_gate());
}
void launch_assemble_aug(const DevKMap& K, int64_t n, const double* hv, const double* jv, const double* sig_s,
                         const double* sig_x, double delta_p, double* kval, hipStream_t s) {
  k_assemble_aug<<<(unsigned)blocks_for(K.nk), BS, 0, s>>>(K, n, hv, jv, sig_s, sig_x, delta_p, kval, launch_gate());
}
void launch_permute_in(const DevPlan& P, const double* rhs, const double* d, double* xp, hipStream_t s) {
  k_permute_in<<<(unsigned)blocks_for(P.n), BS, 0, s>>>(P.n, P.perm, rhs, d, xp, launch_gate());
}
void launch_permute_out(const DevPlan& P, const double* xp, const double* d, double* x, hipStream_t s) {
  k_permute_out<<<(unsigned)blocks_for(P.n), BS, 0, s>>>(P.n, P.perm, xp, d, x, launch_gate());
}
void launch_diag_scale(int64_t n, const int64_t* kp, const double* kval, double* d, double* partials,
                       hipStream_t s, int64_t npos) {
  int g = red_grid(n);
  k_diag_scale<<<g, BS, 0, s>>>(n, kp, kval, d, partials, npos, launch_gate());
  RedSpec spec{3, {RED_MAX, RED_SUM, RED_MIN}};
  launch_finalize(partials, g, spec, partials + 8 * RED_BLOCKS, s);
}
template <typename T>
void launch_set_scaled(const DevKMap& K, const double* kval, const double* d, double shift, T* panel,
                       hipStream_t s) {
  k_set_scaled<T><<<(unsigned)blocks_for(K.nk), BS, 0, s>>>(K, kval, d, shift, panel, launch_gate());
}
template void launch_set_scaled<float>(const DevKMap&, const double*, const double*, double, float*, hipStream_t);
template void launch_set_scaled<double>(const DevKMap&, const double*, const double*, double, double*, hipStream_t);
template <typename T>
void launch_solve_op(const Op& op, const DevPlan& P, const T* panel, const T* inv, double* xp, double* ys,
                     double* uvec, double* part, hipStream_t s) {
  if (op.grid <= 0) return;
  const unsigned g = (unsigned)op.grid;
  switch (op.type) {
    case OP_FWD_SMALL: k_fwd_small<T><<<g, BS, 0, s>>>(P, op.begin, panel, xp, ys, uvec, launch_gate()); break;
    case OP_FWD_GATHER: k_fwd_gather<<<g, GATHER_ROWS, 0, s>>>(P, op.begin, xp, uvec, launch_gate()); break;
    case OP_FWD_FIRST: k_fwd_first<T><<<g, BS, 0, s>>>(P, op.begin, inv, xp, ys, launch_gate()); break;
    case OP_FWD_STEP: k_fwd_step<T><<<g, SBS, 0, s>>>(P, op.begin, panel, inv, xp, ys, uvec, launch_gate()); break;
    case OP_BWD_SMALL: k_bwd_small<T><<<g, BS, 0, s>>>(P, op.begin, panel, ys, launch_gate()); break;
    case OP_BWD_PART: k_bwd_part<T><<<g, SBS, 0, s>>>(P, op.begin, panel, ys, part, launch_gate()); break;
    case OP_BWD_DIAG: k_bwd_diag<T><<<g, SBS, 0, s>>>(P, op.begin, inv, ys, part, launch_gate()); break;
  }
}
template void launch_solve_op<double>(const Op&, const DevPlan&, const double*, const double*, double*, double*,
                                      double*, double*, hipStream_t);
template void launch_solve_op<float>(const Op&, const DevPlan&, const float*, const float*, double*, double*,
                                     double*, double*, hipStream_t);

void launch_residuals(const DevProblem& P, IpmVecs& v, hipStream_t s) {
  // J' lambda into tmp_n
  launch_jt_mul(P, v.jv, v.lam, v.tmp_n, s);
  int64_t N = P.n > P.m ? P.n : P.m;
  k_residuals<<<(unsigned)blocks_for(N), BS, 0, s>>>(P, v.tmp_n, v.gf, v.zl, v.zu, v.g, v.s, v.rd, v.rp, launch_gate());
}
void launch_stats_iter(const DevProblem& P, IpmVecs& v, double* partials, hipStream_t s) {
  int64_t N = P.n > P.m ? P.n : P.m;
  int g = red_grid(N);
  k_stats_iter<<<g, BS, 0, s>>>(P, v, partials, launch_gate());
  RedSpec spec{7, {RED_MAX, RED_MAX, RED_MAX, RED_MAX, RED_SUM, RED_SUM, RED_SUM}};
  launch_finalize(partials, g, spec, partials + 8 * RED_BLOCKS, s);
}
void launch_sigmas(const DevProblem& P, IpmVecs& v, double dd, hipStream_t s) {
  int64_t N = P.n > P.m ? P.n : P.m;
  k_sigmas<<<(unsigned)blocks_for(N), BS, 0, s>>>(P, v, dd, launch_gate());
}
void launch_rhs(const DevProblem& P, IpmVecs& v, const double* ts, const double* tl, const double* tu,
                double* rhs, hipStream_t s) {
  if (P.m > 0) k_rhs_m<<<(unsigned)blocks_for(P.m), BS, 0, s>>>(P, v, ts, v.tmp_m, launch_gate());
  launch_jt_mul(P, v.jv, v.tmp_m, v.tmp_n, s);
  k_rhs_n<<<(unsigned)blocks_for(P.n), BS, 0, s>>>(P, v, v.tmp_n, tl, tu, rhs, launch_gate());
}
void launch_recover(const DevProblem& P, IpmVecs& v, const double* dx, const double* ts, const double* tl,
                    const double* tu, double dd, double* ds, double* dlam, double* dzl, double* dzu,
                    hipStream_t s) {
  if (P.m > 0) {
    launch_j_mul(P, v.jv, dx, v.tmp_m, s);
    k_recover_m<<<(unsigned)blocks_for(P.m), BS, 0, s>>>(P, v, v.tmp_m, ts, dd, ds, dlam, launch_gate());
  }
  k_recover_n<<<(unsigned)blocks_for(P.n), BS, 0, s>>>(P, v, dx, tl, tu, dzl, dzu, launch_gate());
}
void launch_step_limits(const DevProblem& P, IpmVecs& v, const double* dx, const double* ds, const double* dlam,
                        const double* dzl, const double* dzu, double* partials, hipStream_t s) {
  int64_t N = P.n > P.m ? P.n : P.m;
  int g = red_grid(N);
  k_step_limits<<<g, BS, 0, s>>>(P, v, dx, ds, dlam, dzl, dzu, partials, launch_gate());
  RedSpec spec{2, {RED_MIN, RED_MIN}};
  launch_finalize(partials, g, spec, partials + 8 * RED_BLOCKS, s);
}
void launch_mu_aff(const DevProblem& P, IpmVecs& v, const double* dx, const double* ds, const double* dlam,
                   const double* dzl, const double* dzu, double ap, double ad, double* partials, hipStream_t s) {
  int64_t N = P.n > P.m ? P.n : P.m;
  int g = red_grid(N);
  k_mu_aff<<<g, BS, 0, s>>>(P, v, dx, ds, dlam, dzl, dzu, ap, ad, partials, launch_gate());
  RedSpec spec{1, {RED_SUM}};
  launch_finalize(partials, g, spec, partials + 8 * RED_BLOCKS, s);
}
void launch_targets(const DevProblem& P, const double* dx, const double* ds, const double* dlam,
                    const double* dzl, const double* dzu, double smu, double* ts, double* tl, double* tu,
                    hipStream_t s) {
  int64_t N = P.n > P.m ? P.n : P.m;
  k_targets<<<(unsigned)blocks_for(N), BS, 0, s>>>(P, dx, ds, dlam, dzl, dzu, smu, ts, tl, tu, launch_gate());
}
void launch_axpy_point(const DevProblem& P, IpmVecs& dst, const IpmVecs& src, const double* dx, const double* ds,
                       const double* dlam, const double* dzl, const double* dzu, double ap, double ad,
                       hipStream_t s) {
  int64_t N = P.n > P.m ? P.n : P.m;
  k_axpy_point<<<(unsigned)blocks_for(N), BS, 0, s>>>(P, dst, src, dx, ds, dlam, dzl, dzu, ap, ad, launch_gate());
}
void launch_phi(const DevProblem& P, IpmVecs& v, double smu, double* partials, hipStream_t s) {
  int64_t N = P.n > P.m ? P.n : P.m;
  int g = red_grid(N);
  k_phi<<<g, BS, 0, s>>>(P, v, smu, partials, launch_gate());
  RedSpec spec{1, {RED_SUM}};
  launch_finalize(partials, g, spec, partials + 8 * RED_BLOCKS, s);
}
void launch_init_point(const DevProblem& P, IpmVecs& v, hipStream_t s) {
  int64_t N = P.n > P.m ? P.n : P.m;
  k_init_point<<<(unsigned)blocks_for(N), BS, 0, s>>>(P, v, launch_gate());
  launch_constraints(P, v.x, v.g, s);
  if (P.m > 0) k_slack_from_g<<<(unsigned)blocks_for(P.m), BS, 0, s>>>(P, v, 0, launch_gate());
}
void launch_push_start(const DevProblem& P, IpmVecs& v, const double* xhat, const double* lamhat, double,
                       hipStream_t s) {
  int64_t N = P.n > P.m ? P.n : P.m;
  k_push_x<<<(unsigned)blocks_for(N), BS, 0, s>>>(P, v, xhat, lamhat, launch_gate());
  launch_constraints(P, v.x, v.g, s);
  if (P.m > 0) k_slack_from_g<<<(unsigned)blocks_for(P.m), BS, 0, s>>>(P, v, 1, launch_gate());
}
void launch_push_duals(const DevProblem& P, IpmVecs& v, double mu_w, hipStream_t s) {
  k_push_duals<<<(unsigned)blocks_for(P.n), BS, 0, s>>>(P, v, mu_w, launch_gate());
}
void launch_sum_sl(const DevProblem& P, IpmVecs& v, double* partials, hipStream_t s) {
  int g = red_grid(P.m > 0 ? P.m : 1);
  k_sum_sl<<<g, BS, 0, s>>>(P, v, partials, launch_gate());
  RedSpec spec{1, {RED_SUM}};
  launch_finalize(partials, g, spec, partials + 8 * RED_BLOCKS, s);
}
void launch_k_mul_free(const DevProblem& P, const double* jv, const double* hv, const double* sig_s,
                       const double* sig_x, double dp, const double* v, double* out, double* tmp_m,
                       double* tmp_n, hipStream_t s) {
  // out <- H v ; tmp_m <- Sigma_s J v ; tmp_n <- J' tmp_m ; out <- out + tmp_n + (Sigma_x + dp) v
  launch_h_mul(P, hv, v, out, s);
  if (P.m > 0) {
    launch_j_mul(P, jv, v, tmp_m, s);
    k_kfree_m<<<(unsigned)blocks_for(P.m), BS, 0, s>>>(P.m, sig_s, tmp_m, launch_gate());
    launch_jt_mul(P, jv, tmp_m, tmp_n, s);
  } else {
    launch_fill_f64(tmp_n, P.n, 0.0, s);
  }
  k_kfree_n<<<(unsigned)blocks_for(P.n), BS, 0, s>>>(P.n, out, tmp_n, sig_x, dp, v, out, launch_gate());
}
void launch_residual_norms(int64_t n, const double* rhs, const double* kx, const double* x, double* r,
                           double* partials, hipStream_t s) {
  int g = red_grid(n);
  k_residual_norms<<<g, BS, 0, s>>>(n, rhs, kx, x, r, partials, launch_gate());
  RedSpec spec{3, {RED_MAX, RED_MAX, RED_MAX}};
  launch_finalize(partials, g, spec, partials + 8 * RED_BLOCKS, s);
}
void launch_dot(int64_t n, const double* a, const double* b, double* partials, hipStream_t s) {
  int g = red_grid(n);
  k_dot<<<g, BS, 0, s>>>(n, a, b, partials, launch_gate());
  RedSpec spec{1, {RED_SUM}};
  launch_finalize(partials, g, spec, partials + 8 * RED_BLOCKS, s);
}
void launch_cg_step(int64_t n, double alpha, const double* p, const double* q, double* x, double* r,
                    double* partials, hipStream_t s) {
  int g = red_grid(n);
  k_cg_step<<<g, BS, 0, s>>>(n, alpha, p, q, x, r, partials, launch_gate());
  RedSpec spec{2, {RED_MAX, RED_MAX}};
  launch_finalize(partials, g, spec, partials + 8 * RED_BLOCKS, s);
}
void launch_xpby(int64_t n, const double* z, double beta, double* p, hipStream_t s) {
  k_xpby<<<(unsigned)blocks_for(n), BS, 0, s>>>(n, z, beta, p, launch_gate());
}
void launch_dual_prep(const DevProblem& P, const double* hv, const double* sig_x, const double* sig_s,
                      double delta_p, double* dd, double* de, hipStream_t s) {
  const int64_t len = P.n > P.m ? P.n : P.m;
  k_dual_prep<<<(unsigned)blocks_for(len), BS, 0, s>>>(P.n, P.m, hv, P.hdiag, sig_x, sig_s, delta_p, dd, de, launch_gate());
}
void launch_mul_vec(int64_t n, const double* a, const double* b, double* out, hipStream_t s) {
  if (n > 0) k_mul_vec<<<(unsigned)blocks_for(n), BS, 0, s>>>(n, a, b, out, launch_gate());
}
void launch_dual_finish(int64_t n, const double* d, const double* r, const double* w, double* out,
                        hipStream_t s) {
  if (n > 0) k_dual_finish<<<(unsigned)blocks_for(n), BS, 0, s>>>(n, d, r, w, out, launch_gate());
}
void launch_kdiag_max(const DevProblem& P, const double* jv, const double* sig_s, const double* dd,
                      double* partials, hipStream_t s) {
  int g = red_grid(P.n);
  k_kdiag_max<<<g, BS, 0, s>>>(P.n, P.jtp, P.jtr, jv + P.nnz_j, sig_s, dd, partials, launch_gate());
  RedSpec spec{1, {RED_MAX}};
  launch_finalize(partials, g, spec, partials + 8 * RED_BLOCKS, s);
}
void launch_add(int64_t n, double* x, const double* c, hipStream_t s) {
  k_add<<<(unsigned)blocks_for(n), BS, 0, s>>>(n, x, c, launch_gate());
}
void launch_copy(int64_t n, double* d, const double* src, hipStream_t s) {
  if (n > 0) k_copy<<<(unsigned)blocks_for(n), BS, 0, s>>>(n, d, src, launch_gate());
}

}  // namespace pdipm
