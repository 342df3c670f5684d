// C ABI of the interior-point hot path: handles, workspace, factorisation,
// triangular solves with FP64 refinement, and the predictor-corrector loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "host.hpp"
#include "kernels.hpp"
#include "pdipm.h"

using namespace pdipm;

namespace {

thread_local std::string g_create_error;

struct Region {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};

template <typename T>
size_t bytes_of(const std::vector<T>& v) { return v.size() * sizeof(T); }

// Largest plan arrays over the blocking candidates of a batch (the
// workspace is laid out for all of them, so switching needs no new memory).
struct PlanCaps {
  size_t gemm = 0, potrf = 0, ext = 0, small = 0, sdesc = 0, ssmall = 0, slarge = 0, icomb = 0;
  size_t gitem = 0, grow = 0, gptr = 0, gidx = 0;
  int64_t inv = 0, part = 1;
  void add(const Plan& P) {
    gemm = std::max(gemm, bytes_of(P.gemm)); potrf = std::max(potrf, bytes_of(P.potrf));
    ext = std::max(ext, bytes_of(P.ext)); small = std::max(small, bytes_of(P.small));
    sdesc = std::max(sdesc, bytes_of(P.sdesc)); ssmall = std::max(ssmall, bytes_of(P.ssmall));
    slarge = std::max(slarge, bytes_of(P.slarge)); icomb = std::max(icomb, bytes_of(P.icomb));
    gitem = std::max(gitem, bytes_of(P.gitem)); grow = std::max(grow, bytes_of(P.grow));
    gptr = std::max(gptr, bytes_of(P.gptr)); gidx = std::max(gidx, bytes_of(P.gidx));
    inv = std::max(inv, P.inv_elems); part = std::max(part, P.part_elems);
  }
};

}  // namespace

struct ipm_handle {
  int device = 0;
  hipStream_t stream = 0;
  ipm_options opt{};
  bool standalone = false;
  bool dual = false;            // steps through the dual condensed system M
  bool aug = false;             // steps through the augmented SQD system (signed L S L')
  bool sym_ready = false;       // symbolic analysis already done at create (automatic form)
  std::vector<signed char> psign;  // pivot signs, permuted numbering (augmented form)
  HostProblem hp;
  Graph graph;
  Symbolic sym;
  KMap km;
  Plan plan64, plan32;
  bool need64 = true, need32 = false;
  // standalone: symmetric map of K's lower pattern
  std::vector<int64_t> ksp, kss;
  std::vector<int32_t> ksc;
  std::string err;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_need = 0;
  bool ws_ready = false;
  struct Off {
    size_t c, b, q4, xl, xu, jp, jc, ja, jw, jtp, jtr, jte, hp, hc, hq, hdiag, hsp, hsc, hss;
    size_t kmrow, kmc, kmh, kmtp, kmtk, kmta, kmtb, kmpos, ksp, ksc, kss, kval, kmkp, dscale;
    size_t sfirst, sw, sh, sld, sldu, cptr, child, rel, lsn, snrows, perm, spanel, su, srow, suv;
    size_t gemm64, potrf64, gemm32, potrf32, ext, small, icomb64;
    size_t sdesc64, sdesc32, ssmall64, ssmall32, slarge64, slarge32;
    size_t gitem[2], grow[2], gptr[2], gidx[2];   // forward gather map (FP64, FP32 plan)
    size_t panel, ubuf, inv, bad, partials, xperm, uvec, ysol, part, sinv64, sinv32;
    size_t vec[55];
    size_t sign;
  } o{};
  DevProblem dp{};
  DevPlan dpl64{}, dpl32{};
  DevKMap dk{};
  void* panel = nullptr;
  void* ubuf = nullptr;
  void* inv = nullptr;
  int* bad = nullptr;
  double* partials = nullptr;
  double* xperm = nullptr;
  double* uvec = nullptr;
  double* kval = nullptr;
  double* dscale = nullptr;     // symmetric scaling of the FP32 factor
  double* ysol = nullptr;       // forward/backward solution (permuted)
  double* part = nullptr;       // backward partial sums
  bool scaled = false;          // current factor is of D K D
  double kmax = 1.0;            // max diagonal of K (norm estimate)
  double shift = 0.0;           // diagonal shift of the scaled FP32 factor
  int64_t bad_diag_col = -1;    // permuted column of a non-positive diagonal
  IpmVecs v{}, tv{};
  double *dxa, *dsa, *dla, *dzla, *dzua, *dx, *ds, *dl, *dzl, *dzu, *ts, *tl, *tu, *rhs, *ir_r, *ir_c,
      *ir_kx, *xhat, *lamhat, *cg_p;
  double *dual_d = nullptr, *dual_e = nullptr, *dual_tn = nullptr, *dual_tm = nullptr;
  double *aug_in = nullptr, *aug_out = nullptr;
  // factor state
  int assembled_prec = -1, factor_prec = -1;
  bool values_set = false, factored = false;
  double cur_delta_p = 0;  // delta_p used by the last assembly
  // result
  bool solved = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // optional per-launch timing of the GEMM kernel and phase totals
  bool profiling = false;
  std::vector<hipEvent_t> pev;
  ipm_profile prof{};
  // batched solve: bcount > 0 when the handle holds a block-diagonal batch
  int32_t bcount = 0;
  std::vector<int64_t> bxoff, broff;
  std::vector<int32_t> bix, bir, blp;
  std::vector<double> bnc;
  std::vector<Blocking> bcand;
  int32_t bblocking = 0;
  PlanCaps cap64, cap32;
  BatchDev bd{};
  hipStream_t own_stream = nullptr;
  hipGraphExec_t gsolve = nullptr;  // whole batched iterations, one graph
  struct BOff { size_t xoff, roff, ix, ir, nc, lp, st, ist, flags; } bo{};
};

namespace {

int fail(ipm_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return code;
}

#define HIPCHK(h, call)                                                                 \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((h), PDIPM_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// Autotuned blockings remembered for the rest of the process, per size
// bucket of a batch: precision, instance count, order, nnz(L) and largest
// front, each as its power-of-two exponent.  A batch created later in a
// bucket starts with the blocking its last autotune chose.
using TuneKey = std::array<int, 5>;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;

TuneKey tune_key(const ipm_handle* h) {
  auto lg = [](double v) { return v < 1 ? 0 : (int)std::ilogb(v); };
  const Symbolic& s = h->sym;
  int64_t maxf = 0;
  for (size_t k = 0; k + 1 < s.sn_start.size(); ++k) maxf = std::max<int64_t>(maxf, s.sn_rowptr[k + 1] - s.sn_rowptr[k]);
  return TuneKey{h->opt.precision, lg(h->bcount), lg((double)s.n), lg((double)s.nnz_L), lg((double)maxf)};
}

void finish_analysis(ipm_handle* h) {
  if (h->bcount > 0) {
    // blocking candidates of the autotuner; the workspace fits each of them
    for (int sh : {64, 32})
      for (int ob : {4, 2, 1}) h->bcand.push_back(Blocking{sh, ob});
    for (const Blocking& b : h->bcand) {
      Plan t;
      build_plan(h->sym, 8, &t, b);
      h->cap64.add(t);
      build_plan(h->sym, 4, &t, b);
      h->cap32.add(t);
    }
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tuned.find(tune_key(h));
      h->bblocking = it == g_tuned.end() ? 0 : it->second;
    }
    build_plan(h->sym, 8, &h->plan64, h->bcand[h->bblocking]);
    build_plan(h->sym, 4, &h->plan32, h->bcand[h->bblocking]);
    map_k_to_panels(h->sym, h->plan64, &h->km);
  } else {
    // the FP32 plan on a second host thread while the FP64 plan and the map
    // of K entries to panel positions (same layout in both precisions) are
    // built here
    std::string plan32_error;
    std::thread plan32_thread([&]() {
      try {
        build_plan(h->sym, 4, &h->plan32);
      } catch (const std::exception& ex) {
        plan32_error = ex.what();
      }
    });
    try {
      build_plan(h->sym, 8, &h->plan64);
      map_k_to_panels(h->sym, h->plan64, &h->km);
    } catch (...) {
      plan32_thread.join();
      throw;
    }
    plan32_thread.join();
    if (!plan32_error.empty()) throw std::runtime_error(plan32_error);
  }
  if (h->standalone) {
    // symmetric pattern of the stored lower K for products K v
    const int64_t n = h->km.n;
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t e = 0; e < (int64_t)h->km.kc.size(); ++e) {
      int32_t i = h->km.krow[e], j = h->km.kc[e];
      cnt[i + 1]++;
      if (i != j) cnt[j + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    h->ksp = cnt;
    h->ksc.resize(cnt[n]);
    h->kss.resize(cnt[n]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < (int64_t)h->km.kc.size(); ++e) {
      int32_t i = h->km.krow[e], j = h->km.kc[e];
      int64_t q = fill[i]++;
      h->ksc[q] = j; h->kss[q] = e;
      if (i != j) { q = fill[j]++; h->ksc[q] = i; h->kss[q] = e; }
    }
  }
}

void layout(ipm_handle* h) {
  Region r;
  auto& o = h->o;
  const HostProblem& p = h->hp;
  const int64_t n = h->sym.n, m = h->standalone ? 0 : p.m;
  if (!h->standalone) {
    o.c = r.take(bytes_of(p.c)); o.b = r.take(bytes_of(p.b)); o.q4 = r.take(bytes_of(p.q4));
    o.xl = r.take(bytes_of(p.xl)); o.xu = r.take(bytes_of(p.xu));
    o.jp = r.take(bytes_of(p.jp)); o.jc = r.take(bytes_of(p.jc)); o.ja = r.take(bytes_of(p.ja));
    o.jw = r.take(bytes_of(p.jw)); o.jtp = r.take(bytes_of(p.jtp)); o.jtr = r.take(bytes_of(p.jtr));
    o.jte = r.take(bytes_of(p.jte)); o.hp = r.take(bytes_of(p.hp)); o.hc = r.take(bytes_of(p.hc));
    o.hq = r.take(bytes_of(p.hq)); o.hdiag = r.take(bytes_of(p.hdiag)); o.hsp = r.take(bytes_of(p.hsp));
    o.hsc = r.take(bytes_of(p.hsc)); o.hss = r.take(bytes_of(p.hss));
    o.kmh = r.take(bytes_of(h->km.kh)); o.kmtp = r.take(bytes_of(h->km.tp));
    o.kmtk = r.take(bytes_of(h->km.tk)); o.kmta = r.take(bytes_of(h->km.ta)); o.kmtb = r.take(bytes_of(h->km.tb));
  } else {
    o.ksp = r.take(bytes_of(h->ksp)); o.ksc = r.take(bytes_of(h->ksc)); o.kss = r.take(bytes_of(h->kss));
  }
  o.kmrow = r.take(bytes_of(h->km.krow)); o.kmc = r.take(bytes_of(h->km.kc)); o.kmpos = r.take(bytes_of(h->km.pos));
  o.kval = r.take(h->km.kc.size() * 8);
  o.kmkp = r.take(bytes_of(h->km.kp));
  o.dscale = r.take(n * 8);
  const Plan& P = h->plan64;
  o.sfirst = r.take(bytes_of(P.sfirst)); o.sw = r.take(bytes_of(P.sw)); o.sh = r.take(bytes_of(P.sh));
  o.sld = r.take(bytes_of(P.sld)); o.sldu = r.take(bytes_of(P.sldu));
  o.cptr = r.take(bytes_of(P.child_ptr)); o.child = r.take(bytes_of(P.child)); o.rel = r.take(bytes_of(P.rel));
  o.lsn = r.take(bytes_of(P.level_sn)); o.snrows = r.take(bytes_of(h->sym.sn_rows));
  o.perm = r.take(bytes_of(h->sym.perm)); o.spanel = r.take(bytes_of(P.spanel)); o.su = r.take(bytes_of(P.su));
  o.srow = r.take(bytes_of(P.srow)); o.suv = r.take(bytes_of(P.suv));
  // plan arrays: a batch reserves the largest size over its blocking candidates
  PlanCaps c64, c32;
  c64.add(h->plan64);
  c32.add(h->plan32);
  if (h->bcount > 0) { c64 = h->cap64; c32 = h->cap32; }
  o.ext = r.take(std::max(c64.ext, c32.ext)); o.small = r.take(std::max(c64.small, c32.small));
  if (h->need64) {
    o.gemm64 = r.take(c64.gemm); o.potrf64 = r.take(c64.potrf);
    o.sdesc64 = r.take(c64.sdesc); o.ssmall64 = r.take(c64.ssmall);
    o.sinv64 = r.take(bytes_of(h->plan64.sinv));
    o.slarge64 = r.take(c64.slarge);
    o.icomb64 = r.take(c64.icomb);
    o.gitem[0] = r.take(c64.gitem); o.grow[0] = r.take(c64.grow);
    o.gptr[0] = r.take(c64.gptr); o.gidx[0] = r.take(c64.gidx);
  }
  if (h->need32) {
    o.gemm32 = r.take(c32.gemm); o.potrf32 = r.take(c32.potrf);
    o.sdesc32 = r.take(c32.sdesc); o.ssmall32 = r.take(c32.ssmall);
    o.sinv32 = r.take(bytes_of(h->plan32.sinv));
    o.slarge32 = r.take(c32.slarge);
    o.gitem[1] = r.take(c32.gitem); o.grow[1] = r.take(c32.grow);
    o.gptr[1] = r.take(c32.gptr); o.gidx[1] = r.take(c32.gidx);
  }
  const size_t es = h->need64 ? 8 : 4;
  o.panel = r.take((size_t)P.panel_elems * es);
  o.ubuf = r.take((size_t)std::max<int64_t>(1, P.u_elems) * es);
  size_t inv64 = h->need64 ? (size_t)c64.inv * 8 : 0;
  size_t inv32 = h->need32 ? (size_t)c32.inv * 4 : 0;
  o.inv = r.take(std::max(inv64, inv32));
  o.bad = r.take(64);
  o.partials = r.take((8 * RED_BLOCKS + 16) * sizeof(double));
  o.xperm = r.take(n * 8);
  o.uvec = r.take((size_t)std::max<int64_t>(1, P.uv_elems) * 8);
  o.ysol = r.take(n * 8);
  o.part = r.take((size_t)std::max(h->need64 ? c64.part : 1, h->need32 ? c32.part : 1) * 8);
  // vectors: 0..52 (n or m sized; n of the problem, which for the dual
  // condensed system differs from the order of the factored matrix)
  const int64_t nv = std::max<int64_t>(h->standalone ? n : p.n, 1), mv = std::max<int64_t>(m, 1);
  const int64_t jn = std::max<int64_t>((int64_t)p.jc.size(), 1), hn = std::max<int64_t>((int64_t)p.hc.size(), 1);
  const int64_t sizes[] = {
      nv, mv, mv, nv, nv,          // 0 x, 1 s, 2 lam, 3 zl, 4 zu
      nv, nv, mv, 2 * jn, hn,      // 5 gf, 6 qx, 7 g, 8 jv (row order, then transposed), 9 hv
      nv, mv, mv, nv,              // 10 rd, 11 rp, 12 sig_s, 13 sig_x
      nv, mv, nv, mv,              // 14 tmp_n, 15 tmp_m, 16 tmp_n2, 17 tmp_m2
      nv, mv, mv, nv, nv,          // 18..22 trial x, s, lam, zl, zu
      nv, nv, mv, 2 * jn, nv, mv,  // 23 gf, 24 qx, 25 g, 26 jv (as 8), 27 rd, 28 rp
      nv, mv, mv, nv, nv,          // 29..33 affine dx, ds, dlam, dzl, dzu
      nv, mv, mv, nv, nv,          // 34..38 dx, ds, dlam, dzl, dzu
      mv, nv, nv, nv,              // 39 ts, 40 tl, 41 tu, 42 rhs
      nv, nv, nv, nv, mv,          // 43 ir_r, 44 ir_c, 45 ir_kx, 46 xhat, 47 lamhat
      nv,                          // 48 cg direction
      nv, mv, nv, mv,              // 49 D, 50 E, 51..52 dual solve temporaries
      std::max<int64_t>(n, 1), std::max<int64_t>(n, 1)};  // 53..54 augmented solve vectors
  static_assert(sizeof(sizes) / sizeof(sizes[0]) == sizeof(o.vec) / sizeof(o.vec[0]), "vector table");
  for (int i = 0; i < 55; ++i) o.vec[i] = r.take((size_t)sizes[i] * 8);
  o.sign = r.take(std::max<size_t>(1, h->psign.size()));
  if (h->bcount > 0) {
    auto& b = h->bo;
    b.xoff = r.take(bytes_of(h->bxoff)); b.roff = r.take(bytes_of(h->broff));
    b.ix = r.take(bytes_of(h->bix)); b.ir = r.take(std::max<size_t>(4, bytes_of(h->bir)));
    b.nc = r.take(bytes_of(h->bnc)); b.lp = r.take(bytes_of(h->blp));
    b.st = r.take((size_t)h->bcount * BST_N * 8); b.ist = r.take((size_t)h->bcount * IST_N * 4);
    b.flags = r.take(BF_N * 4);
  }
  h->ws_need = r.off;
}

template <typename T>
T* at(ipm_handle* h, size_t off) { return reinterpret_cast<T*>(h->ws + off); }

int upload(ipm_handle* h, size_t off, const void* src, size_t bytes) {
  if (bytes == 0) return PDIPM_OK;
  HIPCHK(h, hipMemcpyAsync(h->ws + off, src, bytes, hipMemcpyHostToDevice, h->stream));
  return PDIPM_OK;
}

#define UP(off, vec) do { int rc_ = upload(h, h->o.off, vec.data(), bytes_of(vec)); if (rc_) return rc_; } while (0)

// Launch descriptors of the current plans (they change with the blocking).
int upload_plans(ipm_handle* h) {
  const Plan& P = h->plan64;
  UP(ext, P.ext); UP(small, P.small);
  if (h->need64) {
    UP(gemm64, h->plan64.gemm); UP(potrf64, h->plan64.potrf); UP(sdesc64, h->plan64.sdesc); UP(sinv64, h->plan64.sinv);
    UP(ssmall64, h->plan64.ssmall); UP(slarge64, h->plan64.slarge); UP(icomb64, h->plan64.icomb);
    UP(gitem[0], h->plan64.gitem); UP(grow[0], h->plan64.grow); UP(gptr[0], h->plan64.gptr);
    UP(gidx[0], h->plan64.gidx);
  }
  if (h->need32) {
    UP(gemm32, h->plan32.gemm); UP(potrf32, h->plan32.potrf); UP(sdesc32, h->plan32.sdesc); UP(sinv32, h->plan32.sinv);
    UP(ssmall32, h->plan32.ssmall); UP(slarge32, h->plan32.slarge);
    UP(gitem[1], h->plan32.gitem); UP(grow[1], h->plan32.grow); UP(gptr[1], h->plan32.gptr);
    UP(gidx[1], h->plan32.gidx);
  }
  return PDIPM_OK;
}

int bind_workspace(ipm_handle* h) {
  auto& o = h->o;
  const HostProblem& p = h->hp;
  if (!h->standalone) {
    UP(c, p.c); UP(b, p.b); UP(q4, p.q4); UP(xl, p.xl); UP(xu, p.xu); UP(jp, p.jp); UP(jc, p.jc);
    UP(ja, p.ja); UP(jw, p.jw); UP(jtp, p.jtp); UP(jtr, p.jtr); UP(jte, p.jte); UP(hp, p.hp); UP(hc, p.hc);
    UP(hq, p.hq); UP(hdiag, p.hdiag); UP(hsp, p.hsp); UP(hsc, p.hsc); UP(hss, p.hss);
    UP(kmh, h->km.kh); UP(kmtp, h->km.tp); UP(kmtk, h->km.tk); UP(kmta, h->km.ta); UP(kmtb, h->km.tb);
  } else {
    UP(ksp, h->ksp); UP(ksc, h->ksc); UP(kss, h->kss);
  }
  UP(kmrow, h->km.krow); UP(kmc, h->km.kc); UP(kmpos, h->km.pos); UP(kmkp, h->km.kp);
  const Plan& P = h->plan64;
  UP(sfirst, P.sfirst); UP(sw, P.sw); UP(sh, P.sh); UP(sld, P.sld); UP(sldu, P.sldu); UP(cptr, P.child_ptr); UP(child, P.child);
  UP(rel, P.rel); UP(lsn, P.level_sn); UP(snrows, h->sym.sn_rows); UP(perm, h->sym.perm);
  UP(spanel, P.spanel); UP(su, P.su); UP(srow, P.srow); UP(suv, P.suv);
  if (!h->psign.empty()) UP(sign, h->psign);
  int rcp = upload_plans(h);
  if (rcp) return rcp;
  if (h->bcount > 0) {
    auto& b = h->bo;
    int rc2;
    if ((rc2 = upload(h, b.xoff, h->bxoff.data(), bytes_of(h->bxoff)))) return rc2;
    if ((rc2 = upload(h, b.roff, h->broff.data(), bytes_of(h->broff)))) return rc2;
    if ((rc2 = upload(h, b.ix, h->bix.data(), bytes_of(h->bix)))) return rc2;
    if ((rc2 = upload(h, b.ir, h->bir.data(), bytes_of(h->bir)))) return rc2;
    if ((rc2 = upload(h, b.nc, h->bnc.data(), bytes_of(h->bnc)))) return rc2;
    if ((rc2 = upload(h, b.lp, h->blp.data(), bytes_of(h->blp)))) return rc2;
    BatchDev& d = h->bd;
    d.count = h->bcount;
    d.xoff = at<int64_t>(h, b.xoff); d.roff = at<int64_t>(h, b.roff);
    d.ix = at<int32_t>(h, b.ix); d.ir = at<int32_t>(h, b.ir);
    d.nc = at<double>(h, b.nc); d.lp = at<int32_t>(h, b.lp);
    d.st = at<double>(h, b.st); d.ist = at<int32_t>(h, b.ist); d.flags = at<int32_t>(h, b.flags);
    d.bad = at<int>(h, o.bad);
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  // device views
  DevProblem& d = h->dp;
  d.n = p.n; d.m = p.m; d.nnz_j = (int64_t)p.jc.size(); d.nnz_h = (int64_t)p.hc.size();
  if (!h->standalone) {
    d.c = at<double>(h, o.c); d.b = at<double>(h, o.b); d.q4 = p.q4.empty() ? nullptr : at<double>(h, o.q4);
    d.xl = at<double>(h, o.xl); d.xu = at<double>(h, o.xu);
    d.jp = at<int64_t>(h, o.jp); d.jc = at<int32_t>(h, o.jc); d.ja = at<double>(h, o.ja); d.jw = at<double>(h, o.jw);
    d.jtp = at<int64_t>(h, o.jtp); d.jtr = at<int32_t>(h, o.jtr); d.jte = at<int32_t>(h, o.jte);
    d.hp = at<int64_t>(h, o.hp); d.hc = at<int32_t>(h, o.hc); d.hq = at<double>(h, o.hq);
    d.hdiag = at<int64_t>(h, o.hdiag); d.hsp = at<int64_t>(h, o.hsp); d.hsc = at<int32_t>(h, o.hsc);
    d.hss = at<int32_t>(h, o.hss);
  }
  DevKMap& k = h->dk;
  k.nk = (int64_t)h->km.kc.size();
  k.npos = h->aug ? p.n : INT64_MAX;
  k.krow = at<int32_t>(h, o.kmrow); k.kc = at<int32_t>(h, o.kmc); k.pos = at<int64_t>(h, o.kmpos);
  if (!h->standalone) {
    k.kh = at<int32_t>(h, o.kmh); k.tp = at<int64_t>(h, o.kmtp); k.tk = at<int32_t>(h, o.kmtk);
    k.ta = at<int32_t>(h, o.kmta); k.tb = at<int32_t>(h, o.kmtb);
  }
  for (int prec = 0; prec < 2; ++prec) {
    DevPlan& q = prec == 0 ? h->dpl64 : h->dpl32;
    const Plan& PP = prec == 0 ? h->plan64 : h->plan32;
    q.ns = PP.ns; q.n = PP.n; q.nb = PP.nb; q.small_h = PP.small_h;
    q.sfirst = at<int32_t>(h, o.sfirst); q.sw = at<int32_t>(h, o.sw); q.sh = at<int32_t>(h, o.sh);
    q.sld = at<int32_t>(h, o.sld); q.sldu = at<int32_t>(h, o.sldu);
    q.child_ptr = at<int32_t>(h, o.cptr); q.child = at<int32_t>(h, o.child); q.rel = at<int32_t>(h, o.rel);
    q.level_sn = at<int32_t>(h, o.lsn); q.sn_rows = at<int32_t>(h, o.snrows); q.perm = at<int32_t>(h, o.perm);
    q.spanel = at<int64_t>(h, o.spanel); q.su = at<int64_t>(h, o.su); q.srow = at<int64_t>(h, o.srow);
    q.suv = at<int64_t>(h, o.suv); q.ext = at<ExtAddDesc>(h, o.ext); q.small = at<int32_t>(h, o.small);
    q.gemm = at<GemmDesc>(h, prec == 0 ? o.gemm64 : o.gemm32);
    q.potrf = at<PotrfDesc>(h, prec == 0 ? o.potrf64 : o.potrf32);
    q.sdesc = at<SolveDesc>(h, prec == 0 ? o.sdesc64 : o.sdesc32);
    q.ssmall = at<int32_t>(h, prec == 0 ? o.ssmall64 : o.ssmall32);
    q.slarge = at<int32_t>(h, prec == 0 ? o.slarge64 : o.slarge32);
    q.sinv = at<int64_t>(h, prec == 0 ? o.sinv64 : o.sinv32);
    q.icomb = prec == 0 ? at<InvCombDesc>(h, o.icomb64) : nullptr;
    q.gitem = at<GatherItem>(h, o.gitem[prec]); q.grow = at<int64_t>(h, o.grow[prec]);
    q.gptr = at<int64_t>(h, o.gptr[prec]); q.gidx = at<int64_t>(h, o.gidx[prec]);
    q.sign = h->psign.empty() ? nullptr : at<signed char>(h, o.sign);
  }
  h->panel = h->ws + o.panel; h->ubuf = h->ws + o.ubuf; h->inv = h->ws + o.inv;
  h->bad = at<int>(h, o.bad); h->partials = at<double>(h, o.partials);
  h->xperm = at<double>(h, o.xperm); h->uvec = at<double>(h, o.uvec); h->kval = at<double>(h, o.kval);
  h->dscale = at<double>(h, o.dscale);
  h->ysol = at<double>(h, o.ysol);
  h->part = at<double>(h, o.part);
  double* V[55];
  for (int i = 0; i < 55; ++i) V[i] = at<double>(h, o.vec[i]);
  IpmVecs& v = h->v;
  v.x = V[0]; v.s = V[1]; v.lam = V[2]; v.zl = V[3]; v.zu = V[4]; v.gf = V[5]; v.qx = V[6]; v.g = V[7];
  v.jv = V[8]; v.hv = V[9]; v.rd = V[10]; v.rp = V[11]; v.sig_s = V[12]; v.sig_x = V[13];
  v.tmp_n = V[14]; v.tmp_m = V[15]; v.tmp_n2 = V[16]; v.tmp_m2 = V[17];
  IpmVecs& t = h->tv;
  t = v;
  t.x = V[18]; t.s = V[19]; t.lam = V[20]; t.zl = V[21]; t.zu = V[22]; t.gf = V[23]; t.qx = V[24]; t.g = V[25];
  t.jv = V[26]; t.rd = V[27]; t.rp = V[28];
  h->dxa = V[29]; h->dsa = V[30]; h->dla = V[31]; h->dzla = V[32]; h->dzua = V[33];
  h->dx = V[34]; h->ds = V[35]; h->dl = V[36]; h->dzl = V[37]; h->dzu = V[38];
  h->ts = V[39]; h->tl = V[40]; h->tu = V[41]; h->rhs = V[42];
  h->ir_r = V[43]; h->ir_c = V[44]; h->ir_kx = V[45]; h->xhat = V[46]; h->lamhat = V[47];
  h->cg_p = V[48];
  h->dual_d = V[49]; h->dual_e = V[50]; h->dual_tn = V[51]; h->dual_tm = V[52];
  h->aug_in = V[53]; h->aug_out = V[54];
  h->ws_ready = true;
  h->assembled_prec = h->factor_prec = -1;
  h->factored = h->values_set = false;
  return PDIPM_OK;
}

int read_back(ipm_handle* h, const double* dev, double* host, int count) {
  HIPCHK(h, hipMemcpyAsync(host, dev, count * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PDIPM_OK;
}

double* red_out(ipm_handle* h) { return h->partials + 8 * RED_BLOCKS; }

// ------------------------------------------------------------- factor
int factor_now(ipm_handle* h, int prec, kkt_factor_info* info) {
  const Plan& P = prec == PDIPM_FP64 ? h->plan64 : h->plan32;
  const DevPlan& D = prec == PDIPM_FP64 ? h->dpl64 : h->dpl32;
  const size_t es = prec == PDIPM_FP64 ? 8 : 4;
  int big = INT_MAX;
  HIPCHK(h, hipMemcpyAsync(h->bad, &big, sizeof(int), hipMemcpyHostToDevice, h->stream));
  launch_fill_bytes0(h->ubuf, (int64_t)std::max<int64_t>(1, P.u_elems) * es, h->stream);
  const bool prof = h->profiling;
  if (prof && (int64_t)h->pev.size() < 2 * P.gemm_launches) {
    size_t old = h->pev.size();
    h->pev.resize(2 * P.gemm_launches);
    for (size_t i = old; i < h->pev.size(); ++i) HIPCHK(h, hipEventCreate(&h->pev[i]));
  }
  const bool timing = h->ev0 != nullptr;   // no events on a handle never given a workspace
  if (timing) HIPCHK(h, hipEventRecord(h->ev0, h->stream));
  int64_t gl = 0;
  for (const Op& op : P.ops) {
    const bool timed = prof && (op.type == OP_TRSM || op.type == OP_UPDATE);
    if (timed) HIPCHK(h, hipEventRecord(h->pev[2 * gl], h->stream));
    if (prec == PDIPM_FP64)
      launch_factor_op<double>(op, D, (double*)h->panel, (double*)h->ubuf, (double*)h->inv, h->bad, h->stream);
    else
      launch_factor_op<float>(op, D, (float*)h->panel, (float*)h->ubuf, (float*)h->inv, h->bad, h->stream);
    if (timed) { HIPCHK(h, hipEventRecord(h->pev[2 * gl + 1], h->stream)); ++gl; }
  }
  if (timing) HIPCHK(h, hipEventRecord(h->ev1, h->stream));
  HIPCHK(h, hipGetLastError());
  int badcol = INT_MAX;
  HIPCHK(h, hipMemcpyAsync(&badcol, h->bad, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  float ms = 0;
  if (timing) hipEventElapsedTime(&ms, h->ev0, h->ev1);
  if (prof) {
    double gms = 0;
    // optional diagnostic: GEMM time and rate by launch class (panel solve,
    // updates at K <= nb, updates at larger K) and by grid size
    static const bool breakdown = std::getenv("PDIPM_GEMM_BREAKDOWN") != nullptr;
    double cls_ms[3][3] = {}, cls_fl[3][3] = {};
    int64_t cls_n[3][3] = {};
    int64_t li = 0;
    for (const Op& op : P.ops) {
      if (op.type != OP_TRSM && op.type != OP_UPDATE) continue;
      float t = 0;
      hipEventElapsedTime(&t, h->pev[2 * li], h->pev[2 * li + 1]);
      ++li;
      gms += t;
      if (breakdown) {
        const int c = op.type == OP_TRSM ? 0 : (P.gemm[op.begin].K <= P.nb ? 1 : 2);
        const int b = op.grid < 512 ? 0 : (op.grid < 4096 ? 1 : 2);
        double fl = 0;
        for (int64_t q = op.begin; q < op.end; ++q) fl += gemm_desc_flops(P.gemm[q]);
        cls_ms[c][b] += t; cls_fl[c][b] += fl; cls_n[c][b]++;
      }
    }
    if (breakdown) {
      static const char* cn[3] = {"panel-solve", "update K<=nb", "update K>nb"};
      static const char* bn[3] = {"<512", "<4096", ">=4096"};
      for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
          if (cls_n[c][b])
            fprintf(stderr, "gemm%s %-13s tiles %-6s launches %6lld  %9.2f ms  %7.1f TFLOP/s\n",
                    prec == PDIPM_FP64 ? "64" : "32", cn[c], bn[b], (long long)cls_n[c][b], cls_ms[c][b],
                    cls_fl[c][b] / (cls_ms[c][b] * 1e9));
    }
    if (prec == PDIPM_FP32) {
      h->prof.gemm32_launches += gl; h->prof.gemm32_ms += gms; h->prof.gemm32_flops += P.gemm_flops;
      h->prof.gemm32_bytes += P.gemm_bytes;
      h->prof.factorizations32 += 1;
    } else {
      h->prof.gemm64_launches += gl; h->prof.gemm64_ms += gms; h->prof.gemm64_flops += P.gemm_flops;
      h->prof.gemm64_bytes += P.gemm_bytes;
      h->prof.factorizations64 += 1;
    }
    h->prof.factor_ms += ms;
    h->prof.factor_flops += h->sym.flops;
  }
  h->factor_prec = prec;
  h->factored = badcol == INT_MAX;
  if (info) {
    info->status = h->factored ? PDIPM_OK : PDIPM_ERR_NOT_PD;
    info->first_bad_col = h->factored ? -1 : badcol;
    info->ms = ms;
    info->flops = h->sym.flops;
  }
  return h->factored ? PDIPM_OK : fail(h, PDIPM_ERR_NOT_PD, "non-positive pivot at permuted column " + std::to_string(badcol));
}

void trisolve(ipm_handle* h, const double* rhs, double* out) {
  const int prec = h->factor_prec;
  const Plan& P = prec == PDIPM_FP64 ? h->plan64 : h->plan32;
  const DevPlan& D = prec == PDIPM_FP64 ? h->dpl64 : h->dpl32;
  const double* d = h->scaled ? h->dscale : nullptr;
  if (h->profiling) {
    h->prof.solves += 1;
    h->prof.solve_bytes += 2.0 * (double)h->sym.nnz_L * (prec == PDIPM_FP64 ? 8 : 4) + 4.0 * h->sym.n * 8;
  }
  launch_permute_in(D, rhs, d, h->xperm, h->stream);
  for (const std::vector<Op>* ops : {&P.fwd_ops, &P.bwd_ops}) {
    // L S L' (signed factor): between L y = b and L' x = z comes z = S y
    if (ops == &P.bwd_ops && D.sign) launch_sign_scale(D.n, D.sign, h->ysol, h->stream);
    for (const Op& op : *ops) {
      if (prec == PDIPM_FP64)
        launch_solve_op<double>(op, D, (const double*)h->panel, (const double*)h->inv, h->xperm, h->ysol,
                                h->uvec, h->part, h->stream);
      else
        launch_solve_op<float>(op, D, (const float*)h->panel, (const float*)h->inv, h->xperm, h->ysol,
                               h->uvec, h->part, h->stream);
    }
  }
  launch_permute_out(D, h->ysol, d, out, h->stream);
}

// Solve K x = rhs with the current factor.  Primal condensed form: the
// factor is of K.  Dual condensed form (Section 3, eq. kkt_dual): the factor
// is of M = diag(E) + J D J', and K^-1 = D - D J' M^-1 J D, so
// x = D (rhs - J' M^-1 J D rhs).
void ksolve(ipm_handle* h, const double* rhs, double* out) {
  if (h->aug) {
    // augmented form (Section 3, eq. augmentedKKT): [H' J'; J -1/Sigma_s] (x, w)
    // = (rhs, 0) gives w = Sigma_s J x and (H' + J' Sigma_s J) x = rhs
    const int64_t n = h->dp.n, m = h->dp.m;
    launch_copy(n, h->aug_in, rhs, h->stream);
    if (m > 0) launch_fill_f64(h->aug_in + n, m, 0.0, h->stream);
    trisolve(h, h->aug_in, h->aug_out);
    launch_copy(n, out, h->aug_out, h->stream);
    return;
  }
  if (!h->dual) { trisolve(h, rhs, out); return; }
  const DevProblem& P = h->dp;
  launch_mul_vec(P.n, h->dual_d, rhs, h->dual_tn, h->stream);
  launch_j_mul(P, h->v.jv, h->dual_tn, h->dual_tm, h->stream);
  trisolve(h, h->dual_tm, h->dual_tm);
  launch_jt_mul(P, h->v.jv, h->dual_tm, h->dual_tn, h->stream);
  launch_dual_finish(P.n, h->dual_d, rhs, h->dual_tn, out, h->stream);
}

void kmul(ipm_handle* h, const double* x, double* out) {
  if (h->standalone)
    launch_k_mul_stored(h->sym.n, nullptr, nullptr, at<int64_t>(h, h->o.ksp), at<int32_t>(h, h->o.ksc),
                        at<int64_t>(h, h->o.kss), h->kval, x, out, h->stream);
  else
    launch_k_mul_free(h->dp, h->v.jv, h->v.hv, h->v.sig_s, h->v.sig_x, h->cur_delta_p, x, out, h->v.tmp_m2,
                      h->v.tmp_n2, h->stream);
}

// Solve with the current factor and refine in FP64: plain iterative
// refinement while the residual halves each step, then (FP32 factor)
// preconditioned conjugate gradients on K (SPD) with the factor as
// preconditioner.  Converged when ||r||_inf <= target (target <= 0: the
// backward-error target ir_tol (kmax ||x|| + ||b||)); refinement also stops
// when the residual stagnates.
int solve_refined(ipm_handle* h, const double* rhs, double* out, kkt_solve_info* info, double target,
                  bool* converged) {
  const int64_t n = h->hp.n;   // order of K
  ksolve(h, rhs, out);
  int steps = 0;
  double omega = 0, rnorm = 0, nb = 0, nx = 0;
  const bool fp32 = h->factor_prec == PDIPM_FP32;
  auto goal = [&]() { return target > 0 ? target : h->opt.ir_tol * (h->kmax * nx + nb); };
  double prev = INFINITY;
  for (int it = 0;; ++it) {
    kmul(h, out, h->ir_kx);
    launch_residual_norms(n, rhs, h->ir_kx, out, h->ir_r, h->partials, h->stream);
    double nr[3];
    int rc = read_back(h, red_out(h), nr, 3);
    if (rc) return rc;
    rnorm = nr[0]; nb = nr[1]; nx = nr[2];
    if (!std::isfinite(rnorm) || rnorm <= goal() || it >= h->opt.ir_max || !(rnorm < 0.5 * prev)) break;
    prev = rnorm;
    ksolve(h, h->ir_r, h->ir_c);
    launch_add(n, out, h->ir_c, h->stream);
    ++steps;
  }
  int cg = 0;
  if (fp32 && std::isfinite(rnorm) && rnorm > goal()) {
    // PCG from the refined point; ir_r holds its residual
    double* r = h->ir_r; double* z = h->ir_c; double* q = h->ir_kx; double* p = h->cg_p;
    ksolve(h, r, z);
    launch_copy(n, p, z, h->stream);
    launch_dot(n, r, z, h->partials, h->stream);
    double rho;
    int rc = read_back(h, red_out(h), &rho, 1);
    if (rc) return rc;
    const int max_cg = 5 * std::max(1, h->opt.ir_max);
    double best = rnorm;
    int since_best = 0;
    for (cg = 0; cg < max_cg && rho > 0; ++cg) {
      kmul(h, p, q);
      launch_dot(n, p, q, h->partials, h->stream);
      double pq;
      if ((rc = read_back(h, red_out(h), &pq, 1))) return rc;
      if (!(pq > 0)) break;
      const double alpha = rho / pq;
      launch_cg_step(n, alpha, p, q, out, r, h->partials, h->stream);
      double nr[2];
      if ((rc = read_back(h, red_out(h), nr, 2))) return rc;
      rnorm = nr[0]; nx = nr[1];
      if (rnorm <= goal() || !std::isfinite(rnorm)) { ++cg; break; }
      if (rnorm < 0.9 * best) { best = rnorm; since_best = 0; }
      else if (++since_best >= 8) { ++cg; break; }   // stagnation
      ksolve(h, r, z);
      launch_dot(n, r, z, h->partials, h->stream);
      double rho2;
      if ((rc = read_back(h, red_out(h), &rho2, 1))) return rc;
      launch_xpby(n, z, rho2 / rho, p, h->stream);
      rho = rho2;
    }
  }
  omega = rnorm / (h->kmax * nx + nb + 1e-300);
  if (converged) *converged = std::isfinite(rnorm) && rnorm <= goal();
  if (h->opt.print_level > 2)
    fprintf(stderr, "      refine: prec %s residual %.3e goal %.3e ir %d cg %d |b| %.3e |x| %.3e\n",
            fp32 ? "fp32" : "fp64", rnorm, goal(), steps, cg, nb, nx);
  if (info) { info->ir_steps = steps + cg; info->residual = omega; info->fallback = 0; }
  if (!std::isfinite(rnorm)) return fail(h, PDIPM_ERR_NUMERICAL, "non-finite solve residual");
  return PDIPM_OK;
}

// K values (FP64, K pattern order) for the point held in the vectors.
// Dual condensed form: the values of M = diag(1 / Sigma_s) + J D J' with
// D = (H + Sigma_x + delta_p)^-1 (the assembly map of M has no Hessian term;
// its triples scale by D and its diagonal adds E = 1 / Sigma_s).
void assemble_values(ipm_handle* h, double delta_p) {
  if (h->aug) {
    launch_assemble_aug(h->dk, h->dp.n, h->v.hv, h->v.jv, h->v.sig_s, h->v.sig_x, delta_p, h->kval, h->stream);
    // diagonal part of K's (1,1) block, for the norm estimate of K
    launch_dual_prep(h->dp, h->v.hv, h->v.sig_x, h->v.sig_s, delta_p, h->dual_d, h->dual_e, h->stream);
  } else if (h->dual) {
    launch_dual_prep(h->dp, h->v.hv, h->v.sig_x, h->v.sig_s, delta_p, h->dual_d, h->dual_e, h->stream);
    launch_assemble<double>(h->dk, h->v.hv, h->v.jv, h->dual_d, h->dual_e, 0.0, nullptr, h->kval, h->stream);
  } else {
    launch_assemble<double>(h->dk, h->v.hv, h->v.jv, h->v.sig_s, h->v.sig_x, delta_p, nullptr, h->kval, h->stream);
  }
  h->cur_delta_p = delta_p;
}

// Load the panels from the K values: FP64 as is; FP32 as D K D + shift I with
// D = diag(K)^(-1/2).  Returns NOT_PD when a diagonal entry is not positive.
int load_panels(ipm_handle* h, int prec, double shift) {
  if (prec == PDIPM_FP64 && !h->need64) return fail(h, PDIPM_ERR_INVALID_ARG, "workspace has no FP64 factor space");
  if (prec == PDIPM_FP32 && !h->need32) return fail(h, PDIPM_ERR_INVALID_ARG, "workspace has no FP32 plan");
  const size_t es = prec == PDIPM_FP64 ? 8 : 4;
  launch_fill_bytes0(h->panel, (int64_t)h->plan64.panel_elems * es, h->stream);
  launch_diag_scale(h->sym.n, at<int64_t>(h, h->o.kmkp), h->kval, h->dscale, h->partials, h->stream, h->dk.npos);
  double dd[3];
  int rc = read_back(h, red_out(h), dd, 3);
  if (rc) return rc;
  h->kmax = dd[0] > 0 ? dd[0] : 1.0;
  if ((h->dual || h->aug) && dd[1] == 0) {
    // the backward error refers to K, whose largest diagonal entry is
    // formed from D, Sigma_s and J
    launch_kdiag_max(h->dp, h->v.jv, h->v.sig_s, h->dual_d, h->partials, h->stream);
    double km;
    if ((rc = read_back(h, red_out(h), &km, 1))) return rc;
    h->kmax = km > 0 && std::isfinite(km) ? km : 1.0;
  }
  if (dd[1] > 0) {
    h->factored = false;
    h->bad_diag_col = h->sym.pinv[(int64_t)dd[2]];
    return fail(h, PDIPM_ERR_NOT_PD, "non-positive diagonal entry of K at permuted column " +
                                         std::to_string(h->bad_diag_col));
  }
  if (prec == PDIPM_FP64) {
    launch_set_values<double>(h->dk, h->kval, (double*)h->panel, h->stream);
    h->scaled = false;
  } else {
    launch_set_scaled<float>(h->dk, h->kval, h->dscale, shift, (float*)h->panel, h->stream);
    h->scaled = true;
  }
  h->shift = shift;
  h->assembled_prec = prec;
  h->factored = false;
  return PDIPM_OK;
}

// Factor K in the requested precision.  FP32: on a non-positive pivot the
// scaled factor is retried with diagonal shifts 1e-7, 1e-6, ... 1e-3 (the
// shifted factor only preconditions refinement against the true K) unless
// allow_shift is false (a problem that may be nonconvex: the failed pivot
// may reveal an indefinite K, which the FP64 factor decides and the
// inertia correction treats).
int factor_k(ipm_handle* h, int prec, kkt_factor_info* fi, double* ms_acc, int* shifts,
             bool allow_shift = true) {
  double shift = 0.0;
  for (int attempt = 0;; ++attempt) {
    int rc = load_panels(h, prec, shift);
    if (rc == PDIPM_ERR_NOT_PD && fi) {
      fi->status = rc;
      fi->first_bad_col = h->bad_diag_col;
      fi->ms = 0;
      fi->flops = h->sym.flops;
    }
    if (rc) return rc;
    rc = factor_now(h, prec, fi);
    if (ms_acc) *ms_acc += fi->ms;
    if (rc != PDIPM_ERR_NOT_PD || prec == PDIPM_FP64 || !allow_shift) return rc;
    if (attempt >= 5) return rc;
    shift = shift == 0.0 ? 1e-7 : shift * 10.0;
    if (shifts) ++*shifts;
  }
}

int assemble(ipm_handle* h, int prec, double delta_p) {
  assemble_values(h, delta_p);
  return load_panels(h, prec, 0.0);
}

int check_ready(ipm_handle* h) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  if (!h->ws_ready) return fail(h, PDIPM_ERR_NOT_ANALYZED, "workspace not set");
  return PDIPM_OK;
}

// ------------------------------------------------------------ IPM loop
struct Scalars { double maxrp, maxg, maxrd, maxgf, comp, f, nonfinite; };

// Modelled device time (seconds) of one factorisation and of one refinement
// step (triangular-solve pair, matrix-free K v, residual norms) of the
// current plans in each precision.  The FP32 form decides from these counts
// when FP64 factors take over, so the decision, and with it the whole
// iterate sequence, is the same on every run.  Model constants for gfx950:
// about 6 us of launch and dependency latency per kernel, sustained MFMA
// rates of 100 (FP32) and 50 (FP64) TFLOP/s on the Schur updates, and
// 3 TB/s for the streaming triangular solves and sparse products.
struct CostModel { double fac32, fac64, step32, step64; };

CostModel cost_model(const ipm_handle* h) {
  constexpr double lat = 6e-6, r32 = 100e12, r64 = 50e12, bw = 3e12;
  const double F = h->sym.flops, nl = (double)h->sym.nnz_L, n = (double)h->sym.n;
  const double kv_bytes = 8.0 * (3.0 * (double)h->hp.jc.size() + 2.0 * (double)h->hp.hc.size()) + 96.0 * n;
  auto fac = [&](const Plan& P, double r) { return lat * (double)P.ops.size() + F / r; };
  auto step = [&](const Plan& P, double w) {
    return lat * (double)(P.fwd_ops.size() + P.bwd_ops.size() + 8) + (2.0 * nl * w + 32.0 * n + kv_bytes) / bw;
  };
  return CostModel{fac(h->plan32, r32), fac(h->plan64, r64), step(h->plan32, 4.0), step(h->plan64, 8.0)};
}

int evaluate_point(ipm_handle* h, IpmVecs& v, bool hess) {
  const DevProblem& P = h->dp;
  if (h->hp.kind == KIND_NLP) launch_jac_eval(P, v.x, v.jv, h->stream);
  launch_constraints(P, v.x, v.g, h->stream);
  launch_gradient(P, v.x, v.qx, v.gf, h->stream);
  if (hess && h->hp.kind == KIND_NLP) launch_hess_eval(P, v.x, v.lam, v.hv, h->stream);
  launch_residuals(P, v, h->stream);
  return PDIPM_OK;
}

int run_ipm(ipm_handle* h, const ipm_start* st, ipm_result* res) {
  using clk = std::chrono::steady_clock;
  const auto t_start = clk::now();
  const DevProblem& P = h->dp;
  IpmVecs& v = h->v;
  const int64_t n = P.n, m = P.m;
  const int kind = h->hp.kind;
  int64_t nbnd = 0;
  for (int64_t i = 0; i < n; ++i) nbnd += std::isfinite(h->hp.xl[i]) + std::isfinite(h->hp.xu[i]);
  const double nc = (double)(m + nbnd);
  const ipm_options& O = h->opt;
  const int prec = O.precision;
  ipm_result R{};
  auto ms_since = [&](clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); };
  // constant derivatives for LP/QP
  if (kind != KIND_NLP) {
    launch_jv_copy(P, v.jv, h->stream);
    launch_copy(P.nnz_h, v.hv, P.hq, h->stream);
    launch_jv_copy(P, h->tv.jv, h->stream);
  }
  if (st) {
    const hipMemcpyKind kd = st->memspace == PDIPM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(h, hipMemcpyAsync(h->xhat, st->x, n * 8, kd, h->stream));
    if (m) HIPCHK(h, hipMemcpyAsync(h->lamhat, st->lam, m * 8, kd, h->stream));
    launch_push_start(P, v, h->xhat, h->lamhat, 0, h->stream);
    launch_sum_sl(P, v, h->partials, h->stream);
    double sl;
    int rc = read_back(h, red_out(h), &sl, 1);
    if (rc) return rc;
    launch_push_duals(P, v, std::max(1e-4, sl / std::max<int64_t>(1, m)), h->stream);
  } else {
    launch_init_point(P, v, h->stream);
  }
  double delta_w_last = 0.0;
  const CostModel cm = cost_model(h);
  bool stay64 = false;  // FP32 form: switched to FP64 factors for the rest of the solve
  int ntri_prev = 0;    // triangular solves of the previous FP32 iteration
  int status = PDIPM_MAX_ITER;
  int it = 0;
  double Pm = 0, Dm = 0, Cm = 0, mu = 0, f = 0;
  while (true) {
    auto te = clk::now();
    evaluate_point(h, v, true);
    launch_stats_iter(P, v, h->partials, h->stream);
    double s7[7];
    int rc = read_back(h, red_out(h), s7, 7);
    if (rc) return rc;
    R.ms_eval += ms_since(te);
    Scalars S{s7[0], s7[1], s7[2], s7[3], s7[4], s7[5], s7[6]};
    f = S.f;
    Pm = S.maxrp / (1.0 + S.maxg);
    Dm = S.maxrd / (1.0 + S.maxgf);
    Cm = S.comp / (1.0 + std::fabs(f));
    mu = nc > 0 ? S.comp / nc : 0.0;
    if (O.print_level > 0)
      fprintf(stderr, "it %3d f %+.10e P %.2e D %.2e C %.2e mu %.2e fac %s ir %d\n", it, f, Pm, Dm, Cm, mu,
              stay64 || prec == PDIPM_FP64 ? "fp64" : "fp32", R.ir_steps);
    if (S.nonfinite > 0 || !std::isfinite(f)) { status = PDIPM_ERR_NUMERICAL; break; }
    if (Pm <= O.tol && Dm <= O.tol && Cm <= O.tol) { status = PDIPM_OK; break; }
    if (it >= O.max_iter) { status = PDIPM_MAX_ITER; break; }
    if (ms_since(t_start) > O.max_wall_time * 1e3) { status = PDIPM_TIME_LIMIT; break; }
    launch_sigmas(P, v, O.delta_d, h->stream);
    // assemble + factor.  FP32: scaled factor with shift retries, then an
    // FP64 refactor when allowed; a non-positive pivot in FP64 triggers the
    // inertia correction (delta_w added to the diagonal of K).
    int fprec = stay64 ? PDIPM_FP64 : prec;
    double delta_w = 0.0;
    auto ta = clk::now();
    const int ir_before = R.ir_steps;
    const bool fp32_iter = !stay64 && prec == PDIPM_FP32;
    assemble_values(h, O.delta_p);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    R.ms_assemble += ms_since(ta);
    kkt_factor_info fi{};
    int shifts = 0;
    rc = factor_k(h, fprec, &fi, &R.ms_factor, &shifts, h->hp.convex);
    if (rc == PDIPM_ERR_NOT_PD && fprec == PDIPM_FP32 && h->need64) {
      fprec = PDIPM_FP64;
      stay64 = true;
      R.fp64_refactors++;
      rc = factor_k(h, fprec, &fi, &R.ms_factor, nullptr);
    }
    if (rc == PDIPM_ERR_NOT_PD && (h->dual || h->aug)) {
      // the dual condensed form needs H + Sigma_x + delta_p > 0 and the
      // augmented one an SQD matrix; the inertia correction belongs to the
      // primal condensed form
      status = PDIPM_ERR_NUMERICAL;
      break;
    }
    if (rc == PDIPM_ERR_NOT_PD) {
      delta_w = delta_w_last == 0.0 ? 1e-4 : std::max(1e-20, delta_w_last / 3.0);
      const bool first = delta_w_last == 0.0;
      while (true) {
        assemble_values(h, O.delta_p + delta_w);
        rc = factor_k(h, fprec, &fi, &R.ms_factor, nullptr);
        if (rc == PDIPM_OK) { delta_w_last = delta_w; break; }
        if (rc != PDIPM_ERR_NOT_PD) return rc;
        delta_w *= first ? 100.0 : 8.0;
        if (delta_w > 1e40) { status = PDIPM_ERR_NUMERICAL; break; }
      }
      if (status == PDIPM_ERR_NUMERICAL) break;
      R.inertia_corrections++;
    } else if (rc) {
      return rc;
    }
    auto ts0 = clk::now();
    kkt_solve_info si{};
    // refinement target: the stationarity error a solve leaves behind stays
    // below 1% of the larger of the tolerance and the current scaled dual
    // infeasibility (an inexact Newton step: far from the solution a direction
    // needs only be accurate relative to the residual it removes); the affine
    // predictor, which only sets sigma and the second-order term of the
    // corrector, stops at 10%
    const double target = 1e-2 * std::max(O.tol, Dm) * (1.0 + S.maxgf);
    auto direction = [&](const double* tsv, const double* tlv, const double* tuv, double* dx, double* ds,
                         double* dl, double* dzl, double* dzu) -> int {
      launch_rhs(P, v, tsv, tlv, tuv, h->rhs, h->stream);
      bool conv = false;
      int r2 = solve_refined(h, h->rhs, dx, &si, tsv ? target : 10.0 * target, &conv);
      if (r2) return r2;
      if (!conv && h->factor_prec == PDIPM_FP32 && h->need64) {
        // FP32 refinement cannot reach the target: FP64 factors from here on
        kkt_factor_info f64{};
        r2 = factor_k(h, PDIPM_FP64, &f64, &R.ms_factor, nullptr);
        if (r2) return r2;
        R.fp64_refactors++;
        stay64 = true;
        r2 = solve_refined(h, h->rhs, dx, &si, target, &conv);
        if (r2) return r2;
      }
      R.ir_steps += si.ir_steps;
      R.max_ir_residual = std::max(R.max_ir_residual, si.residual);
      launch_recover(P, v, dx, tsv, tlv, tuv, O.delta_d, ds, dl, dzl, dzu, h->stream);
      return PDIPM_OK;
    };
    rc = direction(nullptr, nullptr, nullptr, h->dxa, h->dsa, h->dla, h->dzla, h->dzua);
    if (rc) return rc;
    launch_step_limits(P, v, h->dxa, h->dsa, h->dla, h->dzla, h->dzua, h->partials, h->stream);
    double lim[2];
    if ((rc = read_back(h, red_out(h), lim, 2))) return rc;
    double apa = std::min(1.0, lim[0]), ada = std::min(1.0, lim[1]);
    if (kind != KIND_LP) apa = ada = std::min(apa, ada);
    launch_mu_aff(P, v, h->dxa, h->dsa, h->dla, h->dzla, h->dzua, apa, ada, h->partials, h->stream);
    double maff;
    if ((rc = read_back(h, red_out(h), &maff, 1))) return rc;
    maff /= nc;
    const double sigma = mu > 0 ? std::min(1.0, std::pow(maff / mu, 3.0)) : 0.0;
    const double smu = sigma * mu;
    launch_targets(P, h->dxa, h->dsa, h->dla, h->dzla, h->dzua, smu, h->ts, h->tl, h->tu, h->stream);
    rc = direction(h->ts, h->tl, h->tu, h->dx, h->ds, h->dl, h->dzl, h->dzu);
    if (rc) return rc;
    launch_step_limits(P, v, h->dx, h->ds, h->dl, h->dzl, h->dzu, h->partials, h->stream);
    if ((rc = read_back(h, red_out(h), lim, 2))) return rc;
    const double solve_ms = ms_since(ts0);
    R.ms_solve += solve_ms;
    // Cost-based switch of the FP32 form: once the next FP32 iteration is
    // predicted to cost more than an FP64 one, FP64 factors take over for
    // the remaining iterations, where the condition number and with it the
    // refinement work only grow.  FP32 prediction: this iteration's
    // factorisations (shift retries included) plus its solves, their count
    // grown by the ratio to the previous FP32 iteration (between 1 and 2).
    // FP64 prediction: one factorisation plus two solves.  Both from the
    // cost model (counts, not clocks).
    if (fp32_iter && !stay64 && O.fp64_fallback && h->need64) {
      const int ntri = 2 + (R.ir_steps - ir_before);
      const double grow = ntri_prev > 0 ? std::min(2.0, std::max(1.0, (double)ntri / ntri_prev)) : 1.0;
      if ((1 + shifts) * cm.fac32 + grow * ntri * cm.step32 > cm.fac64 + 2.0 * cm.step64) {
        stay64 = true;
        R.fp64_refactors++;
      }
      ntri_prev = ntri;
    }
    if (O.print_level > 1)
      fprintf(stderr, "    solve: ir %d omega %.2e shifts %d fp64 %d delta_w %.1e kmax %.2e sigma %.2e\n",
              si.ir_steps, si.residual, shifts, R.fp64_refactors, delta_w, h->kmax, sigma);
    const double tau = std::max(0.99, 1.0 - mu);
    double ap = std::min(1.0, tau * lim[0]), ad = std::min(1.0, tau * lim[1]);
    if (kind != KIND_LP) ap = ad = std::min(ap, ad);
    if (kind == KIND_NLP) {
      launch_phi(P, v, smu, h->partials, h->stream);
      double phi0;
      if ((rc = read_back(h, red_out(h), &phi0, 1))) return rc;
      phi0 = std::sqrt(phi0);
      double a = ap;
      bool ok = false;
      for (int k = 0; k < 31; ++k) {
        launch_axpy_point(P, h->tv, v, h->dx, h->ds, h->dl, h->dzl, h->dzu, a, a, h->stream);
        evaluate_point(h, h->tv, false);
        launch_phi(P, h->tv, smu, h->partials, h->stream);
        double phi1;
        if ((rc = read_back(h, red_out(h), &phi1, 1))) return rc;
        if (std::sqrt(phi1) <= (1.0 - 1e-4 * a) * phi0) { ok = true; break; }
        a *= 0.5;
      }
      if (!ok) { status = PDIPM_STALLED; break; }
      ap = ad = a;
    }
    launch_axpy_point(P, v, v, h->dx, h->ds, h->dl, h->dzl, h->dzu, ap, ad, h->stream);
    ++it;
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  R.status = status;
  R.iterations = it;
  R.f = f; R.P = Pm; R.D = Dm; R.C = Cm; R.mu = mu;
  R.ms_total = ms_since(t_start);
  h->solved = true;
  if (res) *res = R;
  return status;
}

// ------------------------------------------------------------ batched solve
// Many LP/QP instances are held as one block-diagonal problem: symbolic
// analysis, assembly, factorisation and triangular solves treat them as
// one matrix (instances are independent diagonal blocks, so every level of
// the plan is one launch over all instances), while step lengths, centring
// and termination are per instance.  The whole solve is one captured HIP
// graph of graph_iters iterations, replayed until every instance has ended:
// a control kernel on the device decides, from device flags, whether the
// next iteration runs and in which precision, and every other launch of the
// graph reads its gate word first.

int set_blocking(ipm_handle* h, int idx) {
  if (idx < 0 || idx >= (int)h->bcand.size()) return fail(h, PDIPM_ERR_INVALID_ARG, "blocking index out of range");
  build_plan(h->sym, 8, &h->plan64, h->bcand[idx]);
  build_plan(h->sym, 4, &h->plan32, h->bcand[idx]);
  h->bblocking = idx;
  if (h->gsolve) { hipGraphExecDestroy(h->gsolve); h->gsolve = nullptr; }
  if (!h->ws_ready) return PDIPM_OK;
  int rc = upload_plans(h);
  if (rc) return rc;
  h->dpl64.small_h = h->plan64.small_h;
  h->dpl32.small_h = h->plan32.small_h;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PDIPM_OK;
}

// Panels of the current K values and the factorisation, all on the device
// (a non-positive pivot is recorded in h->bad and replaced by one).
void batch_factor(ipm_handle* h, int prec) {
  const Plan& P = prec == PDIPM_FP64 ? h->plan64 : h->plan32;
  const DevPlan& D = prec == PDIPM_FP64 ? h->dpl64 : h->dpl32;
  const size_t es = prec == PDIPM_FP64 ? 8 : 4;
  launch_fill_bytes0(h->panel, (int64_t)h->plan64.panel_elems * es, h->stream);
  if (prec == PDIPM_FP64) {
    launch_set_values<double>(h->dk, h->kval, (double*)h->panel, h->stream);
    h->scaled = false;
  } else {
    launch_diag_scale(h->sym.n, at<int64_t>(h, h->o.kmkp), h->kval, h->dscale, h->partials, h->stream);
    launch_set_scaled<float>(h->dk, h->kval, h->dscale, 0.0, (float*)h->panel, h->stream);
    h->scaled = true;
  }
  launch_set_int(h->bad, INT_MAX, h->stream);
  launch_fill_bytes0(h->ubuf, (int64_t)std::max<int64_t>(1, P.u_elems) * es, h->stream);
  for (const Op& op : P.ops) {
    if (prec == PDIPM_FP64)
      launch_factor_op<double>(op, D, (double*)h->panel, (double*)h->ubuf, (double*)h->inv, h->bad, h->stream);
    else
      launch_factor_op<float>(op, D, (float*)h->panel, (float*)h->ubuf, (float*)h->inv, h->bad, h->stream);
  }
  h->factor_prec = prec;
}

// Solve with a fixed number of FP64 refinement steps, then flag the running
// instances whose residual misses their target.
void batch_solve_fixed(ipm_handle* h, const double* rhs, double* out, int steps) {
  const int64_t n = h->hp.n;
  ksolve(h, rhs, out);
  for (int k = 0; k < steps; ++k) {
    kmul(h, out, h->ir_kx);
    launch_residual_norms(n, rhs, h->ir_kx, out, h->ir_r, h->partials, h->stream);
    ksolve(h, h->ir_r, h->ir_c);
    launch_add(n, out, h->ir_c, h->stream);
  }
  kmul(h, out, h->ir_kx);
  launch_residual_norms(n, rhs, h->ir_kx, out, h->ir_r, h->partials, h->stream);
  launch_batch_check_residual(h->bd, h->ir_r, h->stream);
}

void batch_stats_ops(ipm_handle* h) {
  evaluate_point(h, h->v, true);
  launch_set_int(h->bd.flags + BF_ACTIVE, 0, h->stream);
  launch_batch_stats(h->dp, h->bd, h->v, h->opt.tol, h->opt.max_iter, h->stream);
}

void batch_step_ops(ipm_handle* h, int prec) {
  const DevProblem& P = h->dp;
  IpmVecs& v = h->v;
  const ipm_options& O = h->opt;
  const int steps = prec == PDIPM_FP64 ? 1 : std::max(1, std::min(O.ir_max, 3));
  launch_batch_clear_miss(h->bd, h->stream);
  launch_sigmas(P, v, O.delta_d, h->stream);
  assemble_values(h, O.delta_p);
  batch_factor(h, prec);
  auto direction = [&](const double* tsv, const double* tlv, const double* tuv, double* dx, double* ds,
                       double* dl, double* dzl, double* dzu) {
    launch_rhs(P, v, tsv, tlv, tuv, h->rhs, h->stream);
    batch_solve_fixed(h, h->rhs, dx, steps);
    launch_recover(P, v, dx, tsv, tlv, tuv, O.delta_d, ds, dl, dzl, dzu, h->stream);
  };
  direction(nullptr, nullptr, nullptr, h->dxa, h->dsa, h->dla, h->dzla, h->dzua);
  launch_batch_predict(P, h->bd, v, h->dxa, h->dsa, h->dla, h->dzla, h->dzua, h->stream);
  launch_batch_targets(P, h->bd, h->dxa, h->dsa, h->dla, h->dzla, h->dzua, h->ts, h->tl, h->tu, h->stream);
  direction(h->ts, h->tl, h->tu, h->dx, h->ds, h->dl, h->dzl, h->dzu);
  // an FP32 direction that missed its target is not taken: the instance
  // repeats the iteration with FP64 factors (which the control step then
  // switches to)
  const int repeat = prec == PDIPM_FP32 && O.fp64_fallback && h->need64;
  launch_batch_correct(P, h->bd, v, h->dx, h->ds, h->dl, h->dzl, h->dzu, repeat, h->stream);
  launch_batch_update(P, h->bd, v, h->dx, h->ds, h->dl, h->dzl, h->dzu, h->stream);
  launch_batch_next(h->bd, h->stream);
}

template <typename F>
int capture(ipm_handle* h, hipGraphExec_t* out, F&& record) {
  hipGraph_t g = nullptr;
  HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
  record();
  hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (e != hipSuccess) return fail(h, PDIPM_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return fail(h, PDIPM_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  return PDIPM_OK;
}

int ensure_stream(ipm_handle* h) {
  if (h->stream) return PDIPM_OK;
  if (!h->own_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking));
  HIPCHK(h, hipDeviceSynchronize());
  h->stream = h->own_stream;
  return PDIPM_OK;
}

// Start point of every instance (cold, or a pushed warm start).
int batch_start(ipm_handle* h, const ipm_start* st) {
  const DevProblem& P = h->dp;
  IpmVecs& v = h->v;
  launch_jv_copy(P, v.jv, h->stream);
  launch_copy(P.nnz_h, v.hv, P.hq, h->stream);
  launch_batch_init(h->bd, h->opt.precision == PDIPM_FP64 ? 1 : 0, h->stream);
  if (st) {
    const hipMemcpyKind kd = st->memspace == PDIPM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(h, hipMemcpyAsync(h->xhat, st->x, P.n * 8, kd, h->stream));
    if (P.m) HIPCHK(h, hipMemcpyAsync(h->lamhat, st->lam, P.m * 8, kd, h->stream));
    launch_push_start(P, v, h->xhat, h->lamhat, 0, h->stream);
    launch_batch_push_duals(P, h->bd, v, h->stream);
  } else {
    launch_init_point(P, v, h->stream);
  }
  return PDIPM_OK;
}

int run_batch(ipm_handle* h, const ipm_start* st, ipm_result* res, ipm_batch_info* info) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto ms_since = [&](clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); };
  int rc = ensure_stream(h);
  if (rc) return rc;
  h->profiling = false;
  const ipm_options& O = h->opt;
  ipm_batch_info I{};
  I.blocking = h->bblocking;
  if ((rc = batch_start(h, st))) return rc;
  const bool graphs = O.use_graphs != 0;
  const int allow64 = O.precision == PDIPM_FP32 && O.fp64_fallback && h->need64 ? 1 : 0;
  const bool with32 = O.precision == PDIPM_FP32, with64 = O.precision == PDIPM_FP64 || allow64;
  int32_t hflags[BF_N];
  bool timed_out = false;
  if (graphs) {
    if (!h->gsolve) {
      const auto tc = clk::now();
      rc = capture(h, &h->gsolve, [&] {
        // each iteration holds the termination measures, the control step
        // and both precisions' Newton steps, all gated by device flags
        for (int k = 0; k < O.graph_iters; ++k) {
          set_launch_gate(h->bd.flags + BF_RUN);
          batch_stats_ops(h);
          set_launch_gate(nullptr);
          launch_batch_control(h->bd, O.max_iter, allow64, h->stream);
          if (with32) { set_launch_gate(h->bd.flags + BF_RUN32); batch_step_ops(h, PDIPM_FP32); }
          if (with64) { set_launch_gate(h->bd.flags + BF_RUN64); batch_step_ops(h, PDIPM_FP64); }
        }
        set_launch_gate(nullptr);
      });
      set_launch_gate(nullptr);
      if (rc) return rc;
      I.ms_capture += ms_since(tc);
    }
    while (true) {
      HIPCHK(h, hipGraphLaunch(h->gsolve, h->stream));
      I.graph_launches++;
      HIPCHK(h, hipMemcpyAsync(hflags, h->bd.flags, sizeof(hflags), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      if (!hflags[BF_RUN]) break;
      if (ms_since(t0) > O.max_wall_time * 1e3) { timed_out = true; break; }
    }
  } else {
    // the same sequence launched directly, the host reading the control words
    while (true) {
      batch_stats_ops(h);
      launch_batch_control(h->bd, O.max_iter, allow64, h->stream);
      HIPCHK(h, hipGetLastError());
      HIPCHK(h, hipMemcpyAsync(hflags, h->bd.flags, sizeof(hflags), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      if (O.print_level > 0)
        fprintf(stderr, "batch it %3d running %d refine-miss %d fac %s\n", hflags[BF_STEPS], hflags[BF_ACTIVE],
                hflags[BF_REFINE_MISS], hflags[BF_RUN64] ? "fp64" : "fp32");
      if (!hflags[BF_RUN]) break;
      if (ms_since(t0) > O.max_wall_time * 1e3) { timed_out = true; break; }
      batch_step_ops(h, hflags[BF_RUN64] ? PDIPM_FP64 : PDIPM_FP32);
      HIPCHK(h, hipGetLastError());
    }
  }
  const int it = hflags[BF_ITER];
  I.fp64_from = hflags[BF_FP64_FROM];
  I.factor_failures = hflags[BF_FAILURES];
  I.refine_misses = hflags[BF_MISSES];
  std::vector<double> hst((size_t)h->bcount * BST_N);
  std::vector<int32_t> hist((size_t)h->bcount * IST_N);
  HIPCHK(h, hipMemcpyAsync(hst.data(), h->bd.st, hst.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(hist.data(), h->bd.ist, hist.size() * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  I.iterations = it;
  I.ms_total = ms_since(t0);
  for (int32_t b = 0; b < h->bcount; ++b) {
    const double* s = hst.data() + (size_t)b * BST_N;
    const int32_t* q = hist.data() + (size_t)b * IST_N;
    int status = q[IST_STATUS];
    if (!q[IST_DONE]) status = timed_out ? PDIPM_TIME_LIMIT : PDIPM_MAX_ITER;
    if (status == PDIPM_OK) I.solved++;
    if (res) {
      ipm_result R{};
      R.status = status;
      R.iterations = q[IST_ITERS];
      R.f = s[BST_F]; R.P = s[BST_P]; R.D = s[BST_D]; R.C = s[BST_C]; R.mu = s[BST_MU];
      R.ms_total = I.ms_total;
      res[b] = R;
    }
  }
  h->solved = true;
  if (info) *info = I;
  return PDIPM_OK;
}

// Time one factorisation per blocking candidate at the cold start point and
// keep the fastest (ties: the lower index).
int batch_autotune(ipm_handle* h, int32_t* chosen, double* ms_out, int reps) {
  int rc = ensure_stream(h);
  if (rc) return rc;
  const int prec = h->opt.precision;
  double best = INFINITY;
  int besti = 0;
  for (int c = 0; c < (int)h->bcand.size(); ++c) {
    if ((rc = set_blocking(h, c))) return rc;
    if ((rc = batch_start(h, nullptr))) return rc;
    evaluate_point(h, h->v, true);
    launch_sigmas(h->dp, h->v, h->opt.delta_d, h->stream);
    assemble_values(h, h->opt.delta_p);
    double tmin = INFINITY;
    for (int r = 0; r < std::max(1, reps); ++r) {
      HIPCHK(h, hipEventRecord(h->ev0, h->stream));
      batch_factor(h, prec);
      HIPCHK(h, hipEventRecord(h->ev1, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      float ms = 0;
      hipEventElapsedTime(&ms, h->ev0, h->ev1);
      tmin = std::min(tmin, (double)ms);
    }
    if (ms_out) ms_out[c] = tmin;
    if (tmin < best) { best = tmin; besti = c; }
  }
  if ((rc = set_blocking(h, besti))) return rc;
  if (chosen) *chosen = besti;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[tune_key(h)] = besti;
  return PDIPM_OK;
}

// ------------------------------------------------ allocation-free solve
// The device memory of ipm_solve_static: one array per GPU that the library
// runs on, held until the process ends and shared by every such call on
// that GPU (each call re-uploads its handle's data; calls that overlap on
// one GPU race).  Host code never passes the array's name to a kernel or a
// copy: it uses the address hipGetSymbolAddress returns on each device.
constexpr size_t STATIC_WS_BYTES = (size_t)64 << 20;
constexpr int STATIC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[STATIC_MAX_DEVICES] = {};

// Address of the current device's array (looked up once per device).
int static_scratch(ipm_handle* h, void** out) {
  int dev = -1;
  HIPCHK(h, hipGetDevice(&dev));
  if (dev != h->device) return fail(h, PDIPM_ERR_INVALID_ARG, "call ipm_solve_static on the handle's device");
  if (dev < 0 || dev >= STATIC_MAX_DEVICES) return fail(h, PDIPM_ERR_INVALID_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(h, PDIPM_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PDIPM_OK;
}

}  // namespace

// ================================================================= ABI
extern "C" {

void ipm_default_options(ipm_options* o) {
  if (!o) return;
  o->tol = 1e-6;
  o->max_iter = 500;
  o->max_wall_time = 900.0;
  o->delta_p = 1e-8;
  o->delta_d = 1e-8;
  o->precision = PDIPM_FP64;
  o->ir_max = 10;
  o->ir_tol = 1e-14;
  o->nd_leaf = 64;
  o->amalg_menu = 0;
  o->print_level = 0;
  o->fp64_fallback = 1;
  o->use_graphs = 1;
  o->graph_iters = 20;
  o->kkt_form = PDIPM_KKT_PRIMAL;
  o->ordering = PDIPM_ORDER_LEVELS;
}

const char* ipm_status_string(int s) {
  switch (s) {
    case PDIPM_OK: return "optimal";
    case PDIPM_MAX_ITER: return "iteration limit";
    case PDIPM_TIME_LIMIT: return "time limit";
    case PDIPM_STALLED: return "stalled";
    case PDIPM_ERR_INVALID_ARG: return "invalid argument";
    case PDIPM_ERR_OUT_OF_MEMORY: return "workspace too small";
    case PDIPM_ERR_NOT_PD: return "not positive definite";
    case PDIPM_ERR_NUMERICAL: return "numerical failure";
    case PDIPM_ERR_DEVICE: return "device error";
    case PDIPM_ERR_NOT_ANALYZED: return "not analyzed";
    default: return "unknown";
  }
}

const char* ipm_last_error(const ipm_handle* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

// Host-side phase timing on stderr when PDIPM_TIMING is set.
static void create_lap(const char* what) {
  static const bool on = std::getenv("PDIPM_TIMING") != nullptr;
  static auto t0 = std::chrono::steady_clock::now();
  if (!on) return;
  const auto t1 = std::chrono::steady_clock::now();
  fprintf(stderr, "[create] %s %.3f s\n", what, std::chrono::duration<double>(t1 - t0).count());
  t0 = t1;
}

static int finish_create(ipm_handle* h, const ipm_options* opts, ipm_handle** out) {
  if (h->opt.ordering != PDIPM_ORDER_LEVELS && h->opt.ordering != PDIPM_ORDER_MULTILEVEL) {
    delete h;
    return fail(nullptr, PDIPM_ERR_INVALID_ARG, "ordering must be PDIPM_ORDER_LEVELS or PDIPM_ORDER_MULTILEVEL");
  }
  if (h->opt.precision == PDIPM_PRECISION_AUTO && h->standalone) {
    delete h;
    return fail(nullptr, PDIPM_ERR_INVALID_ARG, "kkt_factor takes its precision per call: no PDIPM_PRECISION_AUTO");
  }
  const bool auto_prec = h->opt.precision == PDIPM_PRECISION_AUTO;
  try {
    if (auto_prec) h->opt.fp64_fallback = 1;
    h->need64 = h->opt.precision == PDIPM_FP64 || h->opt.fp64_fallback;
    h->need32 = h->opt.precision == PDIPM_FP32 || auto_prec;
    if (!h->sym_ready) analyze(h->graph, h->opt.nd_leaf, h->opt.amalg_menu, &h->sym, h->opt.ordering);
    create_lap("symbolic analysis");
    if (h->aug) {
      // SQD: the pivot of an x variable is positive, of a lambda one negative
      h->psign.resize(h->sym.n);
      for (int64_t k = 0; k < h->sym.n; ++k) h->psign[k] = h->sym.perm[k] < h->hp.n ? 1 : -1;
    }
    finish_analysis(h);
    create_lap("plans and K map");
    if (auto_prec) {
      // FP32 factors pay when the factorisation time they save exceeds the
      // extra refinement solves an iteration needs: at least one per
      // direction for a single instance; for a batch, whose FP32 directions
      // take a fixed min(ir_max, 3) refinement steps against one with FP64
      // factors, that difference per direction
      const CostModel cm = cost_model(h);
      const double extra = h->bcount > 0 ? 2.0 * std::max(1, std::min(h->opt.ir_max, 3) - 1) : 2.0;
      h->opt.precision = cm.fac64 - cm.fac32 > extra * cm.step32 ? PDIPM_FP32 : PDIPM_FP64;
    }
    layout(h);
    create_lap("workspace layout");
    hipGetDevice(&h->device);
  } catch (const std::exception& e) {
    g_create_error = e.what();
    delete h;
    return PDIPM_ERR_INVALID_ARG;
  }
  (void)opts;
  *out = h;
  return PDIPM_OK;
}

int ipm_create(const ipm_problem_desc* prob, const ipm_options* opts, ipm_handle** out) {
  if (!out) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ipm_handle* h = new (std::nothrow) ipm_handle();
  if (!h) return fail(nullptr, PDIPM_ERR_OUT_OF_MEMORY, "host allocation failed");
  if (opts) h->opt = *opts; else ipm_default_options(&h->opt);
  if (h->opt.precision != PDIPM_FP64 && h->opt.precision != PDIPM_FP32 && h->opt.precision != PDIPM_PRECISION_AUTO) {
    delete h;
    return fail(nullptr, PDIPM_ERR_INVALID_ARG, "precision must be PDIPM_FP64, PDIPM_FP32 or PDIPM_PRECISION_AUTO");
  }
  if (h->opt.kkt_form != PDIPM_KKT_PRIMAL && h->opt.kkt_form != PDIPM_KKT_DUAL &&
      h->opt.kkt_form != PDIPM_KKT_AUGMENTED && h->opt.kkt_form != PDIPM_KKT_AUTO) {
    delete h;
    return fail(nullptr, PDIPM_ERR_INVALID_ARG, "kkt_form must be PDIPM_KKT_PRIMAL, _DUAL, _AUGMENTED or _AUTO");
  }
  create_lap("start");
  std::string e = build_problem(prob, &h->hp);
  if (!e.empty()) { delete h; return fail(nullptr, PDIPM_ERR_INVALID_ARG, e); }
  create_lap("problem copy and patterns");
  if (h->opt.kkt_form == PDIPM_KKT_AUTO) {
    // the condensed system with less factorisation work: the dual one needs
    // a diagonal Hessian and at least one row
    h->opt.kkt_form = PDIPM_KKT_PRIMAL;
    if ((int64_t)h->hp.hc.size() == h->hp.n && h->hp.m > 0) {
      try {
        Graph gd;
        KMap kd;
        Symbolic sd;
        build_dual_structures(h->hp, &gd, &kd);
        analyze(gd, h->opt.nd_leaf, h->opt.amalg_menu, &sd, h->opt.ordering);
        build_graph_from_problem(h->hp, &h->graph);
        build_kmap_problem(h->hp, &h->km);
        analyze(h->graph, h->opt.nd_leaf, h->opt.amalg_menu, &h->sym, h->opt.ordering);
        if (sd.flops < h->sym.flops) {
          h->graph = std::move(gd);
          h->km = std::move(kd);
          h->sym = std::move(sd);
          h->dual = true;
          h->opt.kkt_form = PDIPM_KKT_DUAL;
        }
        h->sym_ready = true;
      } catch (const std::exception& ex) {
        delete h;
        return fail(nullptr, PDIPM_ERR_INVALID_ARG, ex.what());
      }
      create_lap("both condensed systems analysed");
      return finish_create(h, opts, out);
    }
  }
  if (h->opt.kkt_form == PDIPM_KKT_AUGMENTED) {
    h->aug = true;
    try {
      build_augmented_structures(h->hp, &h->graph, &h->km);
    } catch (const std::exception& ex) {
      delete h;
      return fail(nullptr, PDIPM_ERR_INVALID_ARG, ex.what());
    }
    create_lap("graph of the augmented matrix and its map");
    return finish_create(h, opts, out);
  }
  if (h->opt.kkt_form == PDIPM_KKT_DUAL) {
    if ((int64_t)h->hp.hc.size() != h->hp.n) {
      delete h;
      return fail(nullptr, PDIPM_ERR_INVALID_ARG, "the dual condensed form needs a diagonal Hessian (Q diagonal or empty)");
    }
    if (h->hp.m == 0) {
      delete h;
      return fail(nullptr, PDIPM_ERR_INVALID_ARG, "the dual condensed form needs at least one constraint row");
    }
    h->dual = true;
    try {
      build_dual_structures(h->hp, &h->graph, &h->km);
    } catch (const std::exception& ex) {
      delete h;
      return fail(nullptr, PDIPM_ERR_INVALID_ARG, ex.what());
    }
    create_lap("graph of M and M map");
    return finish_create(h, opts, out);
  }
  try {
    // the graph of K (for the ordering) and the K map (for assembly) both
    // only read the problem: build them on two host threads
    std::string kmap_error;
    std::thread kmap_thread([&]() {
      try {
        build_kmap_problem(h->hp, &h->km);
      } catch (const std::exception& ex) {
        kmap_error = ex.what();
      }
    });
    try {
      build_graph_from_problem(h->hp, &h->graph);
    } catch (...) {
      kmap_thread.join();
      throw;
    }
    kmap_thread.join();
    if (!kmap_error.empty()) throw std::runtime_error(kmap_error);
    create_lap("graph of K and K map");
  } catch (const std::exception& ex) {
    delete h;
    return fail(nullptr, PDIPM_ERR_INVALID_ARG, ex.what());
  }
  return finish_create(h, opts, out);
}

int kkt_create_csr(int64_t n, const int64_t* rp, const int32_t* ci, const ipm_options* opts, ipm_handle** out) {
  if (!out) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n <= 0 || n >= (1ll << 31) || !rp || !ci) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "bad K pattern");
  if (rp[0] != 0) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "rowptr[0] != 0");
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "rowptr not monotone");
    bool diag = false;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      if (ci[e] < 0 || ci[e] > i) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "entry outside the lower triangle");
      if (e > rp[i] && ci[e - 1] >= ci[e]) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "columns not sorted");
      diag |= ci[e] == i;
    }
    if (!diag) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "every row needs its diagonal entry");
  }
  ipm_handle* h = new (std::nothrow) ipm_handle();
  if (!h) return fail(nullptr, PDIPM_ERR_OUT_OF_MEMORY, "host allocation failed");
  if (opts) h->opt = *opts; else ipm_default_options(&h->opt);
  h->standalone = true;
  h->hp.n = n;
  h->hp.m = 0;
  build_graph_from_lower(n, rp, ci, &h->graph);
  build_kmap_lower(n, rp, ci, &h->km);
  return finish_create(h, opts, out);
}

int kkt_analyze(ipm_handle* h, kkt_symbolic_stats* s) {
  if (!h || !s) return PDIPM_ERR_INVALID_ARG;
  s->n = h->sym.n;
  s->nnz_K = (int64_t)h->km.kc.size();
  s->nnz_L = h->sym.nnz_L;
  s->nnz_L_stored = 0;
  for (int64_t k = 0; k < h->plan64.ns; ++k) s->nnz_L_stored += (int64_t)h->plan64.sh[k] * h->plan64.sw[k];
  s->n_super = h->sym.nsuper();
  s->max_front = h->plan64.max_front;
  s->n_levels = h->plan64.nlevels;
  s->n_triples = (int64_t)h->km.tk.size();
  s->flops = h->sym.flops;
  s->update_bytes = (double)h->plan64.u_elems * (h->need64 ? 8 : 4);
  s->kkt_form = h->standalone ? -1 : (h->aug ? PDIPM_KKT_AUGMENTED : (h->dual ? PDIPM_KKT_DUAL : PDIPM_KKT_PRIMAL));
  s->precision = h->opt.precision;
  return PDIPM_OK;
}

int kkt_get_symbolic(ipm_handle* h, int32_t* perm, int32_t* etree, int64_t* cc, int32_t* sn_start,
                     int64_t* sn_rowptr, int32_t* sn_rows) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  const Symbolic& s = h->sym;
  if (perm) memcpy(perm, s.perm.data(), bytes_of(s.perm));
  if (etree) memcpy(etree, s.etree.data(), bytes_of(s.etree));
  if (cc) memcpy(cc, s.colcount.data(), bytes_of(s.colcount));
  if (sn_start) memcpy(sn_start, s.sn_start.data(), bytes_of(s.sn_start));
  if (sn_rowptr) memcpy(sn_rowptr, s.sn_rowptr.data(), bytes_of(s.sn_rowptr));
  if (sn_rows) memcpy(sn_rows, s.sn_rows.data(), bytes_of(s.sn_rows));
  return PDIPM_OK;
}

int kkt_get_pattern(ipm_handle* h, int64_t* rp, int32_t* ci) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  if (rp) memcpy(rp, h->km.kp.data(), bytes_of(h->km.kp));
  if (ci) memcpy(ci, h->km.kc.data(), bytes_of(h->km.kc));
  return PDIPM_OK;
}

int ipm_workspace_query(ipm_handle* h, size_t* bytes) {
  if (!h || !bytes) return PDIPM_ERR_INVALID_ARG;
  *bytes = h->ws_need;
  return PDIPM_OK;
}

int ipm_set_stream(ipm_handle* h, void* stream) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  h->stream = (hipStream_t)stream;
  return PDIPM_OK;
}

int ipm_set_workspace(ipm_handle* h, void* ws, size_t bytes) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  if (!ws || bytes < h->ws_need)
    return fail(h, PDIPM_ERR_OUT_OF_MEMORY, "workspace needs " + std::to_string(h->ws_need) + " bytes");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(h, PDIPM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  h->ws = (char*)ws;
  h->ws_bytes = bytes;
  if (!h->ev0) {
    HIPCHK(h, hipEventCreate(&h->ev0));
    HIPCHK(h, hipEventCreate(&h->ev1));
  }
  return bind_workspace(h);
}

int kkt_set_values(ipm_handle* h, const double* d_kval) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->standalone) return fail(h, PDIPM_ERR_INVALID_ARG, "kkt_set_values needs a kkt_create_csr handle");
  HIPCHK(h, hipMemcpyAsync(h->kval, d_kval, h->km.kc.size() * 8, hipMemcpyDeviceToDevice, h->stream));
  h->values_set = true;
  h->factored = false;
  h->cur_delta_p = 0.0;
  return PDIPM_OK;
}

int kkt_assemble(ipm_handle* h, const double* x, const double* lam, const double* sig_s, const double* sig_x,
                 int prec) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (h->standalone) return fail(h, PDIPM_ERR_INVALID_ARG, "kkt_assemble needs an ipm_create handle");
  const DevProblem& P = h->dp;
  IpmVecs& v = h->v;
  launch_copy(P.n, v.x, x, h->stream);
  launch_copy(P.m, v.lam, lam, h->stream);
  launch_copy(P.m, v.sig_s, sig_s, h->stream);
  launch_copy(P.n, v.sig_x, sig_x, h->stream);
  launch_jac_eval(P, v.x, v.jv, h->stream);
  launch_hess_eval(P, v.x, v.lam, v.hv, h->stream);
  rc = assemble(h, prec, h->opt.delta_p);
  if (rc) return rc;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PDIPM_OK;
}

int kkt_get_values(ipm_handle* h, double* out) {
  int rc = check_ready(h);
  if (rc) return rc;
  HIPCHK(h, hipMemcpyAsync(out, h->kval, h->km.kc.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PDIPM_OK;
}

int kkt_factor(ipm_handle* h, int prec, kkt_factor_info* info) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (prec != PDIPM_FP64 && prec != PDIPM_FP32) return fail(h, PDIPM_ERR_INVALID_ARG, "bad precision");
  if ((prec == PDIPM_FP64 && !h->need64) || (prec == PDIPM_FP32 && !h->need32))
    return fail(h, PDIPM_ERR_INVALID_ARG, "the workspace was not sized for this precision");
  if (h->standalone ? !h->values_set : h->assembled_prec < 0)
    return fail(h, PDIPM_ERR_NOT_ANALYZED, "no K values (kkt_set_values / kkt_assemble)");
  kkt_factor_info fi{};
  rc = factor_k(h, prec, &fi, nullptr, nullptr);
  if (rc == PDIPM_ERR_NOT_PD && fi.first_bad_col < 0) fi.status = PDIPM_ERR_NOT_PD;
  if (info) *info = fi;
  return rc;
}

int kkt_get_factor(ipm_handle* h, double* out) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (h->factor_prec < 0) return fail(h, PDIPM_ERR_NOT_ANALYZED, "no factor");
  const Plan& P = h->plan64;
  const int64_t ne = P.panel_elems;
  std::vector<double> pan(ne);
  if (h->factor_prec == PDIPM_FP64) {
    HIPCHK(h, hipMemcpyAsync(pan.data(), h->panel, ne * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
  } else {
    std::vector<float> tmp(ne);
    HIPCHK(h, hipMemcpyAsync(tmp.data(), h->panel, ne * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int64_t i = 0; i < ne; ++i) pan[i] = tmp[i];
  }
  std::vector<double> d;
  if (h->scaled) {
    // the device factor is of D P'KP D: row k of L is divided by d[perm[k]]
    d.resize(h->sym.n);
    HIPCHK(h, hipMemcpyAsync(d.data(), h->dscale, d.size() * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  int64_t o = 0;
  for (int64_t k = 0; k < P.ns; ++k) {
    const int32_t* rows = h->sym.sn_rows.data() + h->sym.sn_rowptr[k];
    for (int32_t c = 0; c < P.sw[k]; ++c)
      for (int32_t r = 0; r < P.sh[k]; ++r) {
        double v = pan[P.spanel[k] + (int64_t)c * P.sld[k] + r];
        if (h->scaled) v /= d[h->sym.perm[rows[r]]];
        out[o++] = v;
      }
  }
  return PDIPM_OK;
}

int kkt_solve(ipm_handle* h, const double* rhs, double* x, kkt_solve_info* info) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->factored) return fail(h, PDIPM_ERR_NOT_ANALYZED, "no valid factor");
  HIPCHK(h, hipEventRecord(h->ev0, h->stream));
  kkt_solve_info si{};
  bool conv = false;
  rc = solve_refined(h, rhs, x, &si, 0.0, &conv);
  if (rc == PDIPM_OK && !conv && h->factor_prec == PDIPM_FP32 && h->need64) {
    // FP32 refinement missed the backward-error target: refactor in FP64
    // and solve again (the handle keeps the FP64 factor afterwards)
    const int steps32 = si.ir_steps;
    kkt_factor_info f64{};
    rc = factor_k(h, PDIPM_FP64, &f64, nullptr, nullptr);
    if (rc == PDIPM_OK) rc = solve_refined(h, rhs, x, &si, 0.0, &conv);
    si.ir_steps += steps32;
    si.fallback = 1;
  }
  HIPCHK(h, hipEventRecord(h->ev1, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  float ms = 0;
  hipEventElapsedTime(&ms, h->ev0, h->ev1);
  si.ms = ms;
  if (info) *info = si;
  return rc;
}

int ipm_evaluate(ipm_handle* h, const double* x, const double* lam, double* f, double* grad, double* g,
                 double* jval, double* hval) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (h->standalone) return fail(h, PDIPM_ERR_INVALID_ARG, "needs an ipm_create handle");
  const DevProblem& P = h->dp;
  IpmVecs& v = h->v;
  launch_copy(P.n, v.x, x, h->stream);
  launch_copy(P.m, v.lam, lam, h->stream);
  launch_jac_eval(P, v.x, v.jv, h->stream);
  launch_constraints(P, v.x, v.g, h->stream);
  launch_gradient(P, v.x, v.qx, v.gf, h->stream);
  launch_hess_eval(P, v.x, v.lam, v.hv, h->stream);
  if (f) {
    // objective through the iteration statistics (rd/rp contents are irrelevant here)
    launch_fill_f64(v.zl, P.n, 0.0, h->stream);
    launch_fill_f64(v.zu, P.n, 0.0, h->stream);
    launch_residuals(P, v, h->stream);
    launch_stats_iter(P, v, h->partials, h->stream);
    double s7[7];
    if ((rc = read_back(h, red_out(h), s7, 7))) return rc;
    *f = s7[5];
  }
  if (grad) HIPCHK(h, hipMemcpyAsync(grad, v.gf, P.n * 8, hipMemcpyDeviceToDevice, h->stream));
  if (g && P.m) HIPCHK(h, hipMemcpyAsync(g, v.g, P.m * 8, hipMemcpyDeviceToDevice, h->stream));
  if (jval && P.nnz_j) HIPCHK(h, hipMemcpyAsync(jval, v.jv, P.nnz_j * 8, hipMemcpyDeviceToDevice, h->stream));
  if (hval) HIPCHK(h, hipMemcpyAsync(hval, v.hv, P.nnz_h * 8, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PDIPM_OK;
}

int ipm_set_profiling(ipm_handle* h, int enable) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  h->profiling = enable != 0;
  h->prof = ipm_profile{};
  return PDIPM_OK;
}

int ipm_get_profile(ipm_handle* h, ipm_profile* out) {
  if (!h || !out) return PDIPM_ERR_INVALID_ARG;
  *out = h->prof;
  return PDIPM_OK;
}

int ipm_pattern_sizes(ipm_handle* h, int64_t* nj, int64_t* nh) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  if (nj) *nj = (int64_t)h->hp.jc.size();
  if (nh) *nh = (int64_t)h->hp.hc.size();
  return PDIPM_OK;
}

int ipm_get_patterns(ipm_handle* h, int64_t* jrp, int32_t* jci, int64_t* hrp, int32_t* hci) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  if (jrp) memcpy(jrp, h->hp.jp.data(), bytes_of(h->hp.jp));
  if (jci) memcpy(jci, h->hp.jc.data(), bytes_of(h->hp.jc));
  if (hrp) memcpy(hrp, h->hp.hp.data(), bytes_of(h->hp.hp));
  if (hci) memcpy(hci, h->hp.hc.data(), bytes_of(h->hp.hc));
  return PDIPM_OK;
}

int ipm_solve_static(ipm_handle* h, const ipm_start* st, ipm_result* res) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  if (h->standalone || h->bcount > 0) return fail(h, PDIPM_ERR_INVALID_ARG, "needs an ipm_create handle");
  if (h->ws_need > STATIC_WS_BYTES)
    return fail(h, PDIPM_ERR_OUT_OF_MEMORY, "workspace needs " + std::to_string(h->ws_need) +
                                                " bytes; the static array holds " + std::to_string(STATIC_WS_BYTES));
  void* p = nullptr;
  int rc = static_scratch(h, &p);
  if (rc) return rc;
  // every call binds afresh: another handle may have used the array since
  h->ws = (char*)p;
  h->ws_bytes = STATIC_WS_BYTES;
  h->profiling = false;
  if ((rc = bind_workspace(h))) return rc;
  return run_ipm(h, st, res);
}

int ipm_set_precision(ipm_handle* h, int precision) {
  if (!h) return PDIPM_ERR_INVALID_ARG;
  if (precision != PDIPM_FP64 && precision != PDIPM_FP32)
    return fail(h, PDIPM_ERR_INVALID_ARG, "precision must be PDIPM_FP64 or PDIPM_FP32");
  if ((precision == PDIPM_FP64 && !h->need64) || (precision == PDIPM_FP32 && !h->need32))
    return fail(h, PDIPM_ERR_INVALID_ARG, "the handle was not created with space for this precision");
  h->opt.precision = precision;
  return PDIPM_OK;
}

int ipm_solve(ipm_handle* h, const ipm_start* st, ipm_result* res) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (h->standalone) return fail(h, PDIPM_ERR_INVALID_ARG, "needs an ipm_create handle");
  return run_ipm(h, st, res);
}

int ipm_get_solution(ipm_handle* h, double* x, double* s, double* lam, double* zl, double* zu, int memspace) {
  int rc = check_ready(h);
  if (rc) return rc;
  const hipMemcpyKind k = memspace == PDIPM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const IpmVecs& v = h->v;
  const int64_t n = h->dp.n, m = h->dp.m;
  if (x) HIPCHK(h, hipMemcpyAsync(x, v.x, n * 8, k, h->stream));
  if (s && m) HIPCHK(h, hipMemcpyAsync(s, v.s, m * 8, k, h->stream));
  if (lam && m) HIPCHK(h, hipMemcpyAsync(lam, v.lam, m * 8, k, h->stream));
  if (zl) HIPCHK(h, hipMemcpyAsync(zl, v.zl, n * 8, k, h->stream));
  if (zu) HIPCHK(h, hipMemcpyAsync(zu, v.zu, n * 8, k, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PDIPM_OK;
}

void ipm_destroy(ipm_handle* h) {
  if (!h) return;
  if (h->gsolve) hipGraphExecDestroy(h->gsolve);
  if (h->ev0) hipEventDestroy(h->ev0);
  if (h->ev1) hipEventDestroy(h->ev1);
  for (hipEvent_t e : h->pev) hipEventDestroy(e);
  if (h->own_stream) {
    hipStreamSynchronize(h->own_stream);
    hipStreamDestroy(h->own_stream);
  }
  delete h;
}

// ------------------------------------------------------------ batch ABI
struct ipm_batch {
  ipm_handle* h = nullptr;
};

int ipm_batch_create(int32_t count, const ipm_problem_desc* probs, const ipm_options* opts, ipm_batch** out) {
  if (!out) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (count < 1 || !probs) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "count must be >= 1 with problems");
  int64_t N = 0, M = 0, nnzA = 0, nnzQ = 0;
  for (int32_t i = 0; i < count; ++i) {
    const ipm_problem_desc& d = probs[i];
    if (d.n <= 0 || d.m < 0) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": bad sizes");
    if (d.W.rowptr && d.W.rowptr[d.m] > 0)
      return fail(nullptr, PDIPM_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": batches take LP/QP instances (W empty)");
    if (d.q4)
      for (int64_t j = 0; j < d.n; ++j)
        if (d.q4[j] != 0.0)
          return fail(nullptr, PDIPM_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": batches take LP/QP instances (q4 zero)");
    if (d.m > 0 && (!d.A.rowptr || !d.b))
      return fail(nullptr, PDIPM_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": rows need A and b");
    N += d.n; M += d.m;
    nnzA += d.A.rowptr ? d.A.rowptr[d.m] : 0;
    nnzQ += d.Q.rowptr ? d.Q.rowptr[d.n] : 0;
  }
  if (N >= (1ll << 31) || M >= (1ll << 31)) return fail(nullptr, PDIPM_ERR_INVALID_ARG, "batch too large for int32 indices");
  // concatenated block-diagonal problem
  std::vector<double> c(N), b(M), xl(N), xu(N), av, qv;
  std::vector<int64_t> arp(M + 1, 0), qrp(N + 1, 0);
  std::vector<int32_t> aci, qci;
  av.reserve(nnzA); aci.reserve(nnzA); qv.reserve(nnzQ); qci.reserve(nnzQ);
  ipm_handle* h = new (std::nothrow) ipm_handle();
  if (!h) return fail(nullptr, PDIPM_ERR_OUT_OF_MEMORY, "host allocation failed");
  if (opts) h->opt = *opts; else ipm_default_options(&h->opt);
  if (h->opt.precision != PDIPM_FP64 && h->opt.precision != PDIPM_FP32 && h->opt.precision != PDIPM_PRECISION_AUTO) {
    delete h;
    return fail(nullptr, PDIPM_ERR_INVALID_ARG, "precision must be PDIPM_FP64, PDIPM_FP32 or PDIPM_PRECISION_AUTO");
  }
  if (h->opt.kkt_form != PDIPM_KKT_PRIMAL) {
    delete h;
    return fail(nullptr, PDIPM_ERR_INVALID_ARG, "batches use the primal condensed form (kkt_form 0)");
  }
  if (h->opt.graph_iters < 1 || h->opt.graph_iters > 1000) {
    delete h;
    return fail(nullptr, PDIPM_ERR_INVALID_ARG, "graph_iters must be in 1..1000");
  }
  h->bcount = count;
  h->bxoff.assign(count + 1, 0);
  h->broff.assign(count + 1, 0);
  h->bix.resize(N);
  h->bir.resize(M);
  h->blp.resize(count);
  h->bnc.resize(count);
  int64_t x0 = 0, r0 = 0;
  for (int32_t i = 0; i < count; ++i) {
    const ipm_problem_desc& d = probs[i];
    if (!d.c) { delete h; return fail(nullptr, PDIPM_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": c is required"); }
    int64_t nb = 0;
    for (int64_t j = 0; j < d.n; ++j) {
      c[x0 + j] = d.c[j];
      xl[x0 + j] = d.xl ? d.xl[j] : -INFINITY;
      xu[x0 + j] = d.xu ? d.xu[j] : INFINITY;
      nb += std::isfinite(xl[x0 + j]) + std::isfinite(xu[x0 + j]);
      h->bix[x0 + j] = i;
      const int64_t e0 = d.Q.rowptr ? d.Q.rowptr[j] : 0, e1 = d.Q.rowptr ? d.Q.rowptr[j + 1] : 0;
      for (int64_t e = e0; e < e1; ++e) {
        qci.push_back((int32_t)(d.Q.colind[e] + x0));
        qv.push_back(d.Q.val[e]);
      }
      qrp[x0 + j + 1] = (int64_t)qci.size();
    }
    for (int64_t k = 0; k < d.m; ++k) {
      b[r0 + k] = d.b[k];
      h->bir[r0 + k] = i;
      for (int64_t e = d.A.rowptr[k]; e < d.A.rowptr[k + 1]; ++e) {
        if (d.A.colind[e] < 0 || d.A.colind[e] >= d.n) {
          delete h;
          return fail(nullptr, PDIPM_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": A column out of range");
        }
        aci.push_back((int32_t)(d.A.colind[e] + x0));
        av.push_back(d.A.val[e]);
      }
      arp[r0 + k + 1] = (int64_t)aci.size();
    }
    h->blp[i] = (d.Q.rowptr && d.Q.rowptr[d.n] > 0) ? 0 : 1;
    h->bnc[i] = (double)(d.m + nb);
    x0 += d.n; r0 += d.m;
    h->bxoff[i + 1] = x0;
    h->broff[i + 1] = r0;
  }
  ipm_problem_desc u{};
  u.n = N; u.m = M; u.c = c.data(); u.b = M ? b.data() : nullptr;
  u.A = pdipm_csr{M, N, arp.data(), aci.data(), av.data()};
  if (nnzQ > 0) u.Q = pdipm_csr{N, N, qrp.data(), qci.data(), qv.data()};
  u.xl = xl.data(); u.xu = xu.data();
  std::string e = build_problem(&u, &h->hp);
  if (!e.empty()) { delete h; return fail(nullptr, PDIPM_ERR_INVALID_ARG, e); }
  try {
    build_graph_from_problem(h->hp, &h->graph);
    build_kmap_problem(h->hp, &h->km);
  } catch (const std::exception& ex) {
    delete h;
    return fail(nullptr, PDIPM_ERR_INVALID_ARG, ex.what());
  }
  ipm_handle* hh = nullptr;
  int rc = finish_create(h, opts, &hh);
  if (rc) return rc;
  ipm_batch* bt = new (std::nothrow) ipm_batch();
  if (!bt) { ipm_destroy(hh); return fail(nullptr, PDIPM_ERR_OUT_OF_MEMORY, "host allocation failed"); }
  bt->h = hh;
  *out = bt;
  return PDIPM_OK;
}

int ipm_batch_analyze(ipm_batch* b, kkt_symbolic_stats* out) {
  if (!b) return PDIPM_ERR_INVALID_ARG;
  return kkt_analyze(b->h, out);
}

int ipm_batch_offsets(ipm_batch* b, int64_t* xoff, int64_t* roff) {
  if (!b) return PDIPM_ERR_INVALID_ARG;
  if (xoff) memcpy(xoff, b->h->bxoff.data(), bytes_of(b->h->bxoff));
  if (roff) memcpy(roff, b->h->broff.data(), bytes_of(b->h->broff));
  return PDIPM_OK;
}

int ipm_batch_workspace_query(ipm_batch* b, size_t* bytes) {
  if (!b) return PDIPM_ERR_INVALID_ARG;
  return ipm_workspace_query(b->h, bytes);
}

int ipm_batch_set_workspace(ipm_batch* b, void* ws, size_t bytes) {
  if (!b) return PDIPM_ERR_INVALID_ARG;
  ipm_handle* h = b->h;
  if (h->gsolve) { hipGraphExecDestroy(h->gsolve); h->gsolve = nullptr; }
  int rc = ensure_stream(h);
  if (rc) return rc;
  return ipm_set_workspace(h, ws, bytes);
}

int ipm_batch_set_stream(ipm_batch* b, void* stream) {
  if (!b) return PDIPM_ERR_INVALID_ARG;
  ipm_handle* h = b->h;
  if (h->gsolve) { hipGraphExecDestroy(h->gsolve); h->gsolve = nullptr; }
  h->stream = (hipStream_t)stream;
  return ensure_stream(h);
}

int ipm_batch_blockings(ipm_batch* b, int32_t* count, int32_t* small_h, int32_t* outer_blocks) {
  if (!b) return PDIPM_ERR_INVALID_ARG;
  const auto& c = b->h->bcand;
  if (count) *count = (int32_t)c.size();
  for (size_t i = 0; i < c.size(); ++i) {
    if (small_h) small_h[i] = c[i].small_h;
    if (outer_blocks) outer_blocks[i] = c[i].outer_blocks;
  }
  return PDIPM_OK;
}

int ipm_batch_set_blocking(ipm_batch* b, int32_t index) {
  if (!b) return PDIPM_ERR_INVALID_ARG;
  return set_blocking(b->h, index);
}

int ipm_batch_autotune(ipm_batch* b, int32_t reps, int32_t* chosen, double* ms) {
  if (!b) return PDIPM_ERR_INVALID_ARG;
  int rc = check_ready(b->h);
  if (rc) return rc;
  return batch_autotune(b->h, chosen, ms, reps);
}

int ipm_batch_solve(ipm_batch* b, const ipm_start* start, ipm_result* res, ipm_batch_info* info) {
  if (!b) return PDIPM_ERR_INVALID_ARG;
  int rc = check_ready(b->h);
  if (rc) return rc;
  return run_batch(b->h, start, res, info);
}

int ipm_batch_set_b(ipm_batch* b, const double* hb) {
  if (!b || !hb) return PDIPM_ERR_INVALID_ARG;
  ipm_handle* h = b->h;
  int rc = check_ready(h);
  if (rc) return rc;
  for (int64_t k = 0; k < h->hp.m; ++k)
    if (!std::isfinite(hb[k])) return fail(h, PDIPM_ERR_INVALID_ARG, "non-finite b");
  std::copy(hb, hb + h->hp.m, h->hp.b.begin());
  if ((rc = upload(h, h->o.b, h->hp.b.data(), bytes_of(h->hp.b)))) return rc;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PDIPM_OK;
}

int ipm_batch_get_solution(ipm_batch* b, double* x, double* s, double* lam, double* zl, double* zu, int memspace) {
  if (!b) return PDIPM_ERR_INVALID_ARG;
  return ipm_get_solution(b->h, x, s, lam, zl, zu, memspace);
}

const char* ipm_batch_last_error(const ipm_batch* b) {
  return b ? b->h->err.c_str() : g_create_error.c_str();
}

void ipm_batch_destroy(ipm_batch* b) {
  if (!b) return;
  ipm_destroy(b->h);
  delete b;
}

}  // extern "C"
