// Learned warm start on gfx950: a ReLU multilayer perceptron trained and
// evaluated with BF16 MFMA products (FP32 accumulation), FP32 loss,
// gradients and Adam state (interface and formulas in pdipm_mlp.h).
//
// Every product C = A B' runs through one tiled kernel: 128 x 128 output
// tiles, eight waves of 64 x 32 (2 x 1 blocks of the 32x32x16 BF16 MFMA), K
// staged through LDS in chunks of 32 with operands loaded either along K or
// along the row index (so the transposed products of the backward pass need
// no transposed copies).  Long reductions are split over workgroups; the
// partial tiles are summed in split order by an epilogue kernel that also
// applies bias, ReLU, the ReLU mask of the backward pass and the BF16 cast,
// so every result is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pdipm_mlp.h"

namespace {

constexpr int BS = 256;
constexpr int GBS = 512;                         // threads of the product kernel (8 waves)
constexpr int TM = 128, KC = 32, LDK = KC + 8;  // LDS rows of 40 BF16 (80 bytes, 16-byte aligned)
constexpr int RB = 512;                          // blocks of the loss reduction

typedef uint16_t bf16;
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline float bf2f(bf16 v) { return __uint_as_float((uint32_t)v << 16); }
// FP32 -> BF16, round to nearest even (NaN stays NaN, overflow goes to inf)
__device__ inline bf16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}

struct GemmArgs {
  const bf16* a; int64_t sam, sak;  // A(m, k) = a[m * sam + k * sak]
  const bf16* b; int64_t sbn, sbk;  // B(n, k) = b[n * sbn + k * sbk]
  float* out;                       // out[z * M * N + m * N + n]: partial sums of split z
  int M, N, K, kper, tiles_n;
};

// Stage rows [r0, r0 + 128) x k [k0, k0 + 32) of an operand into S[row][k].
__device__ inline void stage(const bf16* p, int64_t sr, int64_t sk, int r0, int R, int k0, int kend, bf16* S) {
  const int tid = threadIdx.x;
  if (sk == 1) {
#pragma unroll
    for (int q = 0; q < (TM * KC / 8) / GBS; ++q) {
      const int c = tid + q * GBS;
      const int row = c >> 2, kk = (c & 3) * 8;
      const int r = r0 + row, k = k0 + kk;
      const bf16* src = p + (int64_t)r * sr + k;
      uint4 v = {0u, 0u, 0u, 0u};
      if (r < R) {
        if (k + 8 <= kend && ((uintptr_t)src & 15) == 0) {
          v = *(const uint4*)src;
        } else {
          bf16 t[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) t[e] = k + e < kend ? src[e] : (bf16)0;
          memcpy(&v, t, 16);
        }
      }
      *(uint4*)(S + row * LDK + kk) = v;
    }
  } else {
#pragma unroll
    for (int q = 0; q < (TM * KC / 8) / GBS; ++q) {
      const int c = tid + q * GBS;
      const int kk = c >> 4, rr = (c & 15) * 8;
      const int r = r0 + rr, k = k0 + kk;
      const bf16* src = p + (int64_t)k * sk + (int64_t)r * sr;
      bf16 t[8];
      if (k < kend && sr == 1 && r + 8 <= R && ((uintptr_t)src & 15) == 0) {
        const uint4 v = *(const uint4*)src;
        memcpy(t, &v, 16);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = (k < kend && r + e < R) ? src[(int64_t)e * sr] : (bf16)0;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) S[(rr + e) * LDK + kk] = t[e];
    }
  }
}

__global__ void __launch_bounds__(GBS) k_gemm_bf16(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) bf16 As[TM * LDK];
  __shared__ __attribute__((aligned(16))) bf16 Bs[TM * LDK];
  const int tm = blockIdx.x / g.tiles_n, tn = blockIdx.x % g.tiles_n;
  const int m0 = tm * TM, n0 = tn * TM;
  const int kb = blockIdx.y * g.kper, ke = std::min(g.K, kb + g.kper);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // eight waves: wave w owns rows 64 (w mod 2) .. +64 and columns 32 (w / 2) .. +32
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 32;
  floatx16 acc[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[i][e] = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += KC) {
    stage(g.a, g.sam, g.sak, m0, g.M, k0, ke, As);
    stage(g.b, g.sbn, g.sbk, n0, g.N, k0, ke, Bs);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC; ks += 16) {
      bf16x8 af[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const uint4 va = *(const uint4*)(As + (wm + i * 32 + (lane & 31)) * LDK + ks + 8 * (lane >> 5));
        af[i] = __builtin_bit_cast(bf16x8, va);
      }
      const uint4 vb = *(const uint4*)(Bs + (wn + (lane & 31)) * LDK + ks + 8 * (lane >> 5));
      const bf16x8 bfr = __builtin_bit_cast(bf16x8, vb);
#pragma unroll
      for (int i = 0; i < 2; ++i) acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr, acc[i], 0, 0, 0);
    }
    __syncthreads();
  }
  float* out = g.out + (int64_t)blockIdx.y * g.M * g.N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int m = m0 + wm + i * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      const int n = n0 + wn + (lane & 31);
      if (m < g.M && n < g.N) out[(int64_t)m * g.N + n] = acc[i][e];
    }
}

enum { EP_HIDDEN = 0, EP_OUTPUT = 1, EP_GRAD = 2, EP_MASKED = 3 };

// y = sum of the split partials in order (+ bias[n]); hidden: relu -> BF16;
// output: FP32; grad: FP32; masked: y * (mask > 0) -> FP32 and BF16.
__global__ void k_epilogue(const float* P, int splits, int64_t MN, int N, const float* bias, int mode,
                           const bf16* mask, bf16* ob, float* of) {
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < MN; i += (int64_t)gridDim.x * BS) {
    float y = P[i];
    for (int z = 1; z < splits; ++z) y += P[(int64_t)z * MN + i];
    if (bias) y += bias[i % N];
    if (mode == EP_HIDDEN) {
      ob[i] = f2bf(fmaxf(y, 0.0f));
    } else if (mode == EP_MASKED) {
      if (!(bf2f(mask[i]) > 0.0f)) y = 0.0f;
      of[i] = y;
      ob[i] = f2bf(y);
    } else {
      of[i] = y;
    }
  }
}

__global__ void k_to_bf16(const float* x, bf16* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) y[i] = f2bf(x[i]);
}

__device__ inline float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ inline float softp(float z) { return z > 20.0f ? z : log1pf(expf(z)); }

__global__ void k_transform(const float* z, float* out, int64_t n, int D, int n_x, float xs) {
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const int col = (int)(i % D);
    out[i] = col < n_x ? xs * sigm(z[i]) : softp(z[i]);
  }
}

// Loss terms and dL/dz; per-block partial sums of the two squared errors.
__global__ void __launch_bounds__(BS) k_loss(const float* z, const float* t, int64_t n, int D, int n_x, float xs,
                                            float wx, float wl, float* dz, bf16* dzb, double* part) {
  double ax = 0.0, al = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const int col = (int)(i % D);
    const float zi = z[i];
    float d;
    if (col < n_x) {
      const float s = sigm(zi), e = s - t[i] / xs;
      ax += (double)e * e;
      d = 2.0f * wx * e * s * (1.0f - s);
    } else {
      const float sp = softp(zi), e = logf(sp + 1e-6f) - logf(t[i] + 1e-6f);
      al += (double)e * e;
      d = 2.0f * wl * e / (sp + 1e-6f) * sigm(zi);
    }
    dz[i] = d;
    dzb[i] = f2bf(d);
  }
  __shared__ double sx[BS / 64], sl[BS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    ax += __shfl_down(ax, off, 64);
    al += __shfl_down(al, off, 64);
  }
  if (lane == 0) { sx[wave] = ax; sl[wave] = al; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0, l = 0;
    for (int w = 0; w < BS / 64; ++w) { x += sx[w]; l += sl[w]; }
    part[blockIdx.x] = x;
    part[RB + blockIdx.x] = l;
  }
}

__global__ void k_loss_final(const double* part, int nb, double wx, double wl, float* loss) {
  if (threadIdx.x == 0) {
    double x = 0, l = 0;
    for (int b = 0; b < nb; ++b) { x += part[b]; l += part[RB + b]; }
    *loss = (float)(wx * x + wl * l);
  }
}

// db[n] = sum over rows of dY[b][n] (rows in order)
__global__ void k_colsum(const float* dy, int B, int N, float* db) {
  const int n = blockIdx.x * BS + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int b = 0; b < B; ++b) s += dy[(int64_t)b * N + n];
  db[n] = s;
}

__global__ void k_adam(float* p, float* m, float* v, const float* g, bf16* pb, int64_t n, float lr, float c1,
                       float c2) {
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    p[i] = pi;
    pb[i] = f2bf(pi);
  }
}

__global__ void k_zero_f32(float* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) p[i] = 0.0f;
}

inline unsigned grid_of(int64_t n, int cap = 4096) {
  int64_t b = (n + BS - 1) / BS;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

thread_local std::string g_mlp_error;

struct Reg {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};

}  // namespace

struct mlp_handle {
  int L = 0, n_x = 0, bmax = 0;
  float xs = 10.0f;
  double xw = 1.0;  // weight of the x term of the loss
  std::vector<int> dims;
  std::vector<int64_t> woff, boff;  // parameter offsets (elements) of W_l, b_l
  int64_t np = 0;
  int maxd = 0, maxh = 1;
  size_t part_elems = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t need = 0;
  struct { size_t p, m, v, g, pb, xin, h, z, dz, dzb, dh, dhb, part, lpart, loss; } o{};
  int adam_t = 0;
  std::string err;
  template <typename T> T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
  bf16* hbuf(int l) { return at<bf16>(o.h) + (size_t)(l - 1) * bmax * maxh; }  // hidden activation l >= 1
};

namespace {

int mfail(mlp_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_mlp_error = msg;
  return code;
}

#define MCHK(h, call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return mfail((h), PDIPM_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// split count of a product so that tiles x splits fills the chip
int splits_for(int M, int N, int K) {
  const int tiles = ((M + TM - 1) / TM) * ((N + TM - 1) / TM);
  int s = 1;
  while (tiles * s < 512 && K / (s * 2) >= 256) s *= 2;
  return s;
}

size_t part_need(int M, int N, int K) { return (size_t)splits_for(M, N, K) * M * N; }

// C partials of A B' (strides as in GemmArgs), then the epilogue.
void product(mlp_handle* h, const bf16* a, int64_t sam, int64_t sak, const bf16* b, int64_t sbn, int64_t sbk, int M,
             int N, int K, int mode, const float* bias, const bf16* mask, bf16* ob, float* of) {
  GemmArgs g;
  g.a = a; g.sam = sam; g.sak = sak; g.b = b; g.sbn = sbn; g.sbk = sbk;
  g.M = M; g.N = N; g.K = K;
  const int splits = splits_for(M, N, K);
  g.kper = ((K + splits - 1) / splits + KC - 1) / KC * KC;
  const int zs = (K + g.kper - 1) / g.kper;
  g.tiles_n = (N + TM - 1) / TM;
  g.out = h->at<float>(h->o.part);
  dim3 grid((unsigned)(((M + TM - 1) / TM) * g.tiles_n), (unsigned)zs);
  k_gemm_bf16<<<grid, GBS, 0, h->stream>>>(g);
  const int64_t MN = (int64_t)M * N;
  k_epilogue<<<grid_of(MN), BS, 0, h->stream>>>(g.out, zs, MN, N, bias, mode, mask, ob, of);
}

void forward_pass(mlp_handle* h, const float* theta, int B) {
  const int L = h->L;
  const auto& d = h->dims;
  k_to_bf16<<<grid_of((int64_t)B * d[0]), BS, 0, h->stream>>>(theta, h->at<bf16>(h->o.xin), (int64_t)B * d[0]);
  const bf16* pb = h->at<bf16>(h->o.pb);
  const float* p = h->at<float>(h->o.p);
  for (int l = 1; l <= L; ++l) {
    const bf16* in = l == 1 ? h->at<bf16>(h->o.xin) : h->hbuf(l - 1);
    const bf16* W = pb + h->woff[l - 1];
    const float* bias = p + h->boff[l - 1];
    if (l < L)
      product(h, in, d[l - 1], 1, W, d[l - 1], 1, B, d[l], d[l - 1], EP_HIDDEN, bias, nullptr, h->hbuf(l), nullptr);
    else
      product(h, in, d[l - 1], 1, W, d[l - 1], 1, B, d[l], d[l - 1], EP_OUTPUT, bias, nullptr, nullptr,
              h->at<float>(h->o.z));
  }
}

// loss (device) and gradients into o.g
void backward_pass(mlp_handle* h, const float* target, int B) {
  const int L = h->L;
  const auto& d = h->dims;
  const int D = d[L];
  const int64_t n = (int64_t)B * D;
  const int nl = D - h->n_x;
  const float wx = h->n_x ? (float)(h->xw / ((double)B * h->n_x)) : 0.0f;
  const float wl = nl ? 1.0f / ((float)B * nl) : 0.0f;
  double* lp = h->at<double>(h->o.lpart);
  k_loss<<<RB, BS, 0, h->stream>>>(h->at<float>(h->o.z), target, n, D, h->n_x, h->xs, wx, wl, h->at<float>(h->o.dz),
                                   h->at<bf16>(h->o.dzb), lp);
  k_loss_final<<<1, 64, 0, h->stream>>>(lp, RB, h->n_x ? h->xw / ((double)B * h->n_x) : 0.0,
                                        nl ? 1.0 / ((double)B * nl) : 0.0, h->at<float>(h->o.loss));
  float* g = h->at<float>(h->o.g);
  const bf16* pb = h->at<bf16>(h->o.pb);
  const float* dyf = h->at<float>(h->o.dz);
  const bf16* dyb = h->at<bf16>(h->o.dzb);
  int cur = 0;
  for (int l = L; l >= 1; --l) {
    const bf16* hin = l == 1 ? h->at<bf16>(h->o.xin) : h->hbuf(l - 1);
    // dW_l = dY' h_{l-1}: rows of dW are outputs, the reduction runs over the batch
    product(h, dyb, 1, d[l], hin, 1, d[l - 1], d[l], d[l - 1], B, EP_GRAD, nullptr, nullptr, nullptr,
            g + h->woff[l - 1]);
    k_colsum<<<(unsigned)((d[l] + BS - 1) / BS), BS, 0, h->stream>>>(dyf, B, d[l], g + h->boff[l - 1]);
    if (l > 1) {
      // dh_{l-1} = (dY W_l) * (h_{l-1} > 0)
      float* nf = h->at<float>(h->o.dh) + (size_t)cur * h->bmax * h->maxh;
      bf16* nb = h->at<bf16>(h->o.dhb) + (size_t)cur * h->bmax * h->maxh;
      product(h, dyb, d[l], 1, pb + h->woff[l - 1], 1, d[l - 1], B, d[l - 1], d[l], EP_MASKED, nullptr,
              h->hbuf(l - 1), nb, nf);
      dyf = nf;
      dyb = nb;
      cur ^= 1;
    }
  }
}

int check_batch(mlp_handle* h, int B) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  if (!h->ws) return mfail(h, PDIPM_ERR_NOT_ANALYZED, "workspace not set");
  if (B < 1 || B > h->bmax) return mfail(h, PDIPM_ERR_INVALID_ARG, "batch size outside 1..max_batch");
  return PDIPM_OK;
}

}  // namespace

extern "C" {

int mlp_create(int32_t n_layers, const int32_t* dims, int32_t n_x, double x_scale, double x_weight,
               int32_t max_batch, mlp_handle** out) {
  if (!out) return mfail(nullptr, PDIPM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_layers < 1 || !dims || max_batch < 1) return mfail(nullptr, PDIPM_ERR_INVALID_ARG, "bad layer count or batch");
  for (int l = 0; l <= n_layers; ++l)
    if (dims[l] < 1 || dims[l] > (1 << 24)) return mfail(nullptr, PDIPM_ERR_INVALID_ARG, "bad layer size");
  if (n_x < 0 || n_x > dims[n_layers]) return mfail(nullptr, PDIPM_ERR_INVALID_ARG, "n_x outside 0..dims[L]");
  if (!(x_scale > 0)) return mfail(nullptr, PDIPM_ERR_INVALID_ARG, "x_scale must be positive");
  if (!(x_weight > 0) || !std::isfinite(x_weight)) return mfail(nullptr, PDIPM_ERR_INVALID_ARG, "x_weight must be positive");
  mlp_handle* h = new (std::nothrow) mlp_handle();
  if (!h) return mfail(nullptr, PDIPM_ERR_OUT_OF_MEMORY, "host allocation failed");
  h->L = n_layers;
  h->dims.assign(dims, dims + n_layers + 1);
  h->n_x = n_x;
  h->xs = (float)x_scale;
  h->xw = x_weight;
  h->bmax = max_batch;
  int64_t off = 0;
  for (int l = 0; l < n_layers; ++l) {
    h->woff.push_back(off);
    off += (int64_t)dims[l + 1] * dims[l];
    h->boff.push_back(off);
    off += dims[l + 1];
  }
  h->np = off;
  h->maxd = *std::max_element(h->dims.begin(), h->dims.end());
  for (int l = 1; l < n_layers; ++l) h->maxh = std::max(h->maxh, dims[l]);
  // partial buffer: the largest split product of a forward or training pass
  const int B = max_batch;
  size_t pn = 1;
  for (int l = 1; l <= n_layers; ++l) {
    pn = std::max(pn, part_need(B, dims[l], dims[l - 1]));
    pn = std::max(pn, part_need(dims[l], dims[l - 1], B));
    if (l > 1) pn = std::max(pn, part_need(B, dims[l - 1], dims[l]));
  }
  // smaller batches may split further: tiles x splits < 1024 bounds any split product
  h->part_elems = std::max(pn, (size_t)1024 * TM * TM);
  pn = h->part_elems;
  Reg r;
  auto& o = h->o;
  o.p = r.take(h->np * 4); o.m = r.take(h->np * 4); o.v = r.take(h->np * 4); o.g = r.take(h->np * 4);
  o.pb = r.take(h->np * 2);
  o.xin = r.take((size_t)B * dims[0] * 2);
  o.h = r.take((size_t)std::max(1, n_layers - 1) * B * h->maxh * 2);
  o.z = r.take((size_t)B * dims[n_layers] * 4);
  o.dz = r.take((size_t)B * dims[n_layers] * 4);
  o.dzb = r.take((size_t)B * dims[n_layers] * 2);
  o.dh = r.take((size_t)2 * B * h->maxh * 4);
  o.dhb = r.take((size_t)2 * B * h->maxh * 2);
  o.part = r.take(pn * 4);
  o.lpart = r.take(2 * RB * 8);
  o.loss = r.take(16);
  h->need = r.off;
  *out = h;
  return PDIPM_OK;
}

int mlp_num_params(mlp_handle* h, int64_t* count) {
  if (!h || !count) return PDIPM_ERR_INVALID_ARG;
  *count = h->np;
  return PDIPM_OK;
}

int mlp_workspace_query(mlp_handle* h, size_t* bytes) {
  if (!h || !bytes) return PDIPM_ERR_INVALID_ARG;
  *bytes = h->need;
  return PDIPM_OK;
}

int mlp_set_workspace(mlp_handle* h, void* ws, size_t bytes) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  if (!ws || bytes < h->need) return mfail(h, PDIPM_ERR_OUT_OF_MEMORY, "workspace needs " + std::to_string(h->need) + " bytes");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return mfail(h, PDIPM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  h->ws = (char*)ws;
  return PDIPM_OK;
}

int mlp_set_stream(mlp_handle* h, void* stream) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  h->stream = (hipStream_t)stream;
  return PDIPM_OK;
}

int mlp_set_params(mlp_handle* h, const float* hp) {
  if (!h || !hp) return PDIPM_ERR_INVALID_ARG;
  if (!h->ws) return mfail(h, PDIPM_ERR_NOT_ANALYZED, "workspace not set");
  MCHK(h, hipMemcpyAsync(h->at<float>(h->o.p), hp, h->np * 4, hipMemcpyHostToDevice, h->stream));
  k_to_bf16<<<grid_of(h->np), BS, 0, h->stream>>>(h->at<float>(h->o.p), h->at<bf16>(h->o.pb), h->np);
  k_zero_f32<<<grid_of(h->np), BS, 0, h->stream>>>(h->at<float>(h->o.m), h->np);
  k_zero_f32<<<grid_of(h->np), BS, 0, h->stream>>>(h->at<float>(h->o.v), h->np);
  h->adam_t = 0;
  MCHK(h, hipGetLastError());
  MCHK(h, hipStreamSynchronize(h->stream));
  return PDIPM_OK;
}

int mlp_get_params(mlp_handle* h, float* hp) {
  if (!h || !hp) return PDIPM_ERR_INVALID_ARG;
  if (!h->ws) return mfail(h, PDIPM_ERR_NOT_ANALYZED, "workspace not set");
  MCHK(h, hipMemcpyAsync(hp, h->at<float>(h->o.p), h->np * 4, hipMemcpyDeviceToHost, h->stream));
  MCHK(h, hipStreamSynchronize(h->stream));
  return PDIPM_OK;
}

int mlp_forward(mlp_handle* h, const float* theta, float* out, int32_t B) {
  int rc = check_batch(h, B);
  if (rc) return rc;
  forward_pass(h, theta, B);
  const int D = h->dims[h->L];
  k_transform<<<grid_of((int64_t)B * D), BS, 0, h->stream>>>(h->at<float>(h->o.z), out, (int64_t)B * D, D, h->n_x, h->xs);
  MCHK(h, hipGetLastError());
  return PDIPM_OK;
}

int mlp_gradients(mlp_handle* h, const float* theta, const float* target, int32_t B, float* loss, float* grads) {
  int rc = check_batch(h, B);
  if (rc) return rc;
  forward_pass(h, theta, B);
  backward_pass(h, target, B);
  MCHK(h, hipGetLastError());
  if (loss) MCHK(h, hipMemcpyAsync(loss, h->at<float>(h->o.loss), 4, hipMemcpyDeviceToHost, h->stream));
  if (grads) MCHK(h, hipMemcpyAsync(grads, h->at<float>(h->o.g), h->np * 4, hipMemcpyDeviceToHost, h->stream));
  if (loss || grads) MCHK(h, hipStreamSynchronize(h->stream));
  return PDIPM_OK;
}

int mlp_train_step(mlp_handle* h, const float* theta, const float* target, int32_t B, float lr, float* loss) {
  int rc = check_batch(h, B);
  if (rc) return rc;
  forward_pass(h, theta, B);
  backward_pass(h, target, B);
  h->adam_t += 1;
  const float c1 = 1.0f - std::pow(0.9f, (float)h->adam_t), c2 = 1.0f - std::pow(0.999f, (float)h->adam_t);
  k_adam<<<grid_of(h->np), BS, 0, h->stream>>>(h->at<float>(h->o.p), h->at<float>(h->o.m), h->at<float>(h->o.v),
                                               h->at<float>(h->o.g), h->at<bf16>(h->o.pb), h->np, lr, c1, c2);
  MCHK(h, hipGetLastError());
  if (loss) {
    MCHK(h, hipMemcpyAsync(loss, h->at<float>(h->o.loss), 4, hipMemcpyDeviceToHost, h->stream));
    MCHK(h, hipStreamSynchronize(h->stream));
  }
  return PDIPM_OK;
}

double mlp_flops(mlp_handle* h, int32_t B, int32_t training) {
  if (!h) return 0.0;
  double f = 0.0;
  for (int l = 1; l <= h->L; ++l) {
    const double mac = (double)B * h->dims[l] * h->dims[l - 1];
    f += 2.0 * mac;                                  // forward
    if (training) f += 2.0 * mac * (l > 1 ? 2.0 : 1.0);  // weight gradient, input gradient
  }
  return f;
}

const char* mlp_last_error(const mlp_handle* h) { return h ? h->err.c_str() : g_mlp_error.c_str(); }

void mlp_destroy(mlp_handle* h) { delete h; }

}  // extern "C"
