// Problem ingestion, K pattern and assembly map, supernodal plan (host).
#include "host.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <numeric>
#include <sstream>
#include <stdexcept>
#include <thread>
#include <tuple>

#include "pdipm.h"

namespace pdipm {

namespace {

std::string check_csr(const pdipm_csr& a, int64_t nr, int64_t nc, const char* name, bool lower) {
  if (!a.rowptr) return "";
  std::ostringstream os;
  if (a.nrows != nr || a.ncols != nc) {
    os << name << ": shape " << a.nrows << "x" << a.ncols << " expected " << nr << "x" << nc;
    return os.str();
  }
  if (a.rowptr[0] != 0) return std::string(name) + ": rowptr[0] != 0";
  for (int64_t i = 0; i < nr; ++i) {
    if (a.rowptr[i + 1] < a.rowptr[i]) return std::string(name) + ": rowptr not monotone";
    for (int64_t e = a.rowptr[i]; e < a.rowptr[i + 1]; ++e) {
      int32_t j = a.colind[e];
      if (j < 0 || j >= nc) return std::string(name) + ": column index out of range";
      if (e > a.rowptr[i] && a.colind[e - 1] >= j)
        return std::string(name) + ": columns not sorted or duplicated";
      if (lower && j > i) return std::string(name) + ": entry above the diagonal";
      if (!std::isfinite(a.val[e])) return std::string(name) + ": non-finite value";
    }
  }
  return "";
}

}  // namespace

std::string build_problem(const ipm_problem_desc* d, HostProblem* p) {
  if (!d) return "problem is NULL";
  if (d->n <= 0 || d->m < 0) return "n must be positive and m non-negative";
  if (d->n >= (1ll << 31) || d->m >= (1ll << 31)) return "n and m must fit int32";
  if (!d->c) return "c is required";
  if (d->m > 0 && !d->b) return "b is required when m > 0";
  const int64_t n = d->n, m = d->m;
  std::string e;
  if (!(e = check_csr(d->A, m, n, "A", false)).empty()) return e;
  if (!(e = check_csr(d->W, m, n, "W", false)).empty()) return e;
  if (!(e = check_csr(d->Q, n, n, "Q", true)).empty()) return e;
  p->n = n;
  p->m = m;
  p->c.assign(d->c, d->c + n);
  p->b.assign(d->b ? d->b : d->c, d->b ? d->b + m : d->c);
  if (!d->b) p->b.clear();
  for (double v : p->c)
    if (!std::isfinite(v)) return "non-finite c";
  for (double v : p->b)
    if (!std::isfinite(v)) return "non-finite b";
  p->xl.assign(n, -INFINITY);
  p->xu.assign(n, INFINITY);
  if (d->xl) p->xl.assign(d->xl, d->xl + n);
  if (d->xu) p->xu.assign(d->xu, d->xu + n);
  for (int64_t i = 0; i < n; ++i) {
    if (std::isnan(p->xl[i]) || std::isnan(p->xu[i]) || p->xl[i] == INFINITY || p->xu[i] == -INFINITY)
      return "invalid bound";
    if (!(p->xl[i] < p->xu[i])) return "lower bound must be below upper bound";
  }
  p->has_q4 = false;
  if (d->q4) {
    p->q4.assign(d->q4, d->q4 + n);
    for (double v : p->q4) {
      if (!std::isfinite(v) || v < 0) return "q4 must be finite and non-negative";
      if (v != 0) p->has_q4 = true;
    }
  }
  if (!p->has_q4) p->q4.clear();
  p->has_w = d->W.rowptr && d->W.rowptr[m] > 0;
  // convexity that can be certified cheaply: W >= 0 (g concave) and Q
  // symmetric diagonally dominant with a non-negative diagonal (PSD by
  // Gershgorin); otherwise the Hessian may be indefinite and the primal
  // condensed K needs inertia correction
  p->convex = true;
  if (p->has_w)
    for (int64_t e2 = 0; e2 < d->W.rowptr[m]; ++e2)
      if (d->W.val[e2] < 0) p->convex = false;
  bool has_q = d->Q.rowptr && d->Q.rowptr[n] > 0;
  if (has_q) {
    std::vector<double> diag(n, 0.0), off(n, 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e2 = d->Q.rowptr[i]; e2 < d->Q.rowptr[i + 1]; ++e2) {
        const int32_t j = d->Q.colind[e2];
        const double v = d->Q.val[e2];
        if (j == i) diag[i] += v;
        else { off[i] += std::fabs(v); off[j] += std::fabs(v); }
      }
    for (int64_t i = 0; i < n; ++i)
      if (diag[i] < off[i]) p->convex = false;
  }
  p->kind = (p->has_w || p->has_q4) ? KIND_NLP : (has_q ? KIND_QP : KIND_LP);
  // J union pattern
  p->jp.assign(m + 1, 0);
  p->jc.clear(); p->ja.clear(); p->jw.clear();
  for (int64_t k = 0; k < m; ++k) {
    int64_t ea = d->A.rowptr ? d->A.rowptr[k] : 0, eA = d->A.rowptr ? d->A.rowptr[k + 1] : 0;
    int64_t ew = d->W.rowptr ? d->W.rowptr[k] : 0, eW = d->W.rowptr ? d->W.rowptr[k + 1] : 0;
    while (ea < eA || ew < eW) {
      int32_t ca = ea < eA ? d->A.colind[ea] : INT32_MAX;
      int32_t cw = ew < eW ? d->W.colind[ew] : INT32_MAX;
      int32_t cmin = std::min(ca, cw);
      p->jc.push_back(cmin);
      p->ja.push_back(ca == cmin ? d->A.val[ea++] : 0.0);
      p->jw.push_back(cw == cmin ? d->W.val[ew++] : 0.0);
    }
    p->jp[k + 1] = (int64_t)p->jc.size();
  }
  if ((int64_t)p->jc.size() >= (1ll << 31)) return "J has too many entries";
  // transpose of J
  p->jtp.assign(n + 1, 0);
  for (int32_t j : p->jc) p->jtp[j + 1]++;
  for (int64_t j = 0; j < n; ++j) p->jtp[j + 1] += p->jtp[j];
  p->jtr.resize(p->jc.size());
  p->jte.resize(p->jc.size());
  {
    std::vector<int64_t> fill(p->jtp.begin(), p->jtp.end() - 1);
    for (int64_t k = 0; k < m; ++k)
      for (int64_t e2 = p->jp[k]; e2 < p->jp[k + 1]; ++e2) {
        int64_t q = fill[p->jc[e2]]++;
        p->jtr[q] = (int32_t)k;
        p->jte[q] = (int32_t)e2;
      }
  }
  // H lower pattern = lower(Q) plus the diagonal
  p->hp.assign(n + 1, 0);
  p->hc.clear(); p->hq.clear();
  p->hdiag.assign(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    bool diag_done = false;
    if (d->Q.rowptr) {
      for (int64_t e2 = d->Q.rowptr[i]; e2 < d->Q.rowptr[i + 1]; ++e2) {
        int32_t j = d->Q.colind[e2];
        if (j == i) { p->hdiag[i] = (int64_t)p->hc.size(); diag_done = true; }
        p->hc.push_back(j);
        p->hq.push_back(d->Q.val[e2]);
      }
    }
    if (!diag_done) {
      p->hdiag[i] = (int64_t)p->hc.size();
      p->hc.push_back((int32_t)i);
      p->hq.push_back(0.0);
    }
    p->hp[i + 1] = (int64_t)p->hc.size();
  }
  // symmetric pattern of H with sources
  {
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e2 = p->hp[i]; e2 < p->hp[i + 1]; ++e2) {
        cnt[i + 1]++;
        if (p->hc[e2] != i) cnt[p->hc[e2] + 1]++;
      }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    p->hsp = cnt;
    p->hsc.resize(cnt[n]);
    p->hss.resize(cnt[n]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    // entries (i, j<=i) go to row i; (j, i) for j<i go to row j.  Rows come
    // out sorted because row i first receives the transposed entries from
    // rows < i... collect then sort per row.
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e2 = p->hp[i]; e2 < p->hp[i + 1]; ++e2) {
        int32_t j = p->hc[e2];
        int64_t q = fill[i]++;
        p->hsc[q] = j; p->hss[q] = (int32_t)e2;
        if (j != i) { q = fill[j]++; p->hsc[q] = (int32_t)i; p->hss[q] = (int32_t)e2; }
      }
    for (int64_t i = 0; i < n; ++i) {
      std::vector<std::pair<int32_t, int32_t>> row;
      for (int64_t q = p->hsp[i]; q < p->hsp[i + 1]; ++q) row.push_back({p->hsc[q], p->hss[q]});
      std::sort(row.begin(), row.end());
      for (size_t t = 0; t < row.size(); ++t) {
        p->hsc[p->hsp[i] + t] = row[t].first;
        p->hss[p->hsp[i] + t] = row[t].second;
      }
    }
  }
  return "";
}

void build_graph_from_problem(const HostProblem& p, Graph* g) {
  const int64_t n = p.n;
  g->n = n;
  // Adjacency rows are independent: contiguous column ranges, balanced by
  // the J entries they visit, on up to 8 host threads, concatenated in order.
  std::vector<int64_t> work(n + 1, 0);
  for (int64_t j = 0; j < n; ++j) {
    int64_t w = 1 + (p.hsp[j + 1] - p.hsp[j]);
    for (int64_t q = p.jtp[j]; q < p.jtp[j + 1]; ++q) w += p.jp[p.jtr[q] + 1] - p.jp[p.jtr[q]];
    work[j + 1] = work[j] + w;
  }
  const int64_t nt = host_threads(work[n], 1 << 22);
  std::vector<int64_t> cut(nt + 1, n);
  cut[0] = 0;
  for (int64_t t = 1; t < nt; ++t)
    cut[t] = std::lower_bound(work.begin(), work.end(), work[n] * t / nt) - work.begin();
  for (int64_t t = 1; t <= nt; ++t) cut[t] = std::max(cut[t], cut[t - 1]);
  std::vector<std::vector<int32_t>> adj(nt);
  std::vector<std::vector<int64_t>> len(nt);
  auto run = [&](int64_t t) {
    std::vector<int32_t> mark(n, -1), row;
    for (int64_t j = cut[t]; j < cut[t + 1]; ++j) {
      row.clear();
      mark[j] = (int32_t)j;
      for (int64_t q = p.jtp[j]; q < p.jtp[j + 1]; ++q) {
        int32_t k = p.jtr[q];
        for (int64_t e = p.jp[k]; e < p.jp[k + 1]; ++e) {
          int32_t i = p.jc[e];
          if (mark[i] != j) { mark[i] = (int32_t)j; row.push_back(i); }
        }
      }
      for (int64_t q = p.hsp[j]; q < p.hsp[j + 1]; ++q) {
        int32_t i = p.hsc[q];
        if (mark[i] != j) { mark[i] = (int32_t)j; row.push_back(i); }
      }
      std::sort(row.begin(), row.end());
      adj[t].insert(adj[t].end(), row.begin(), row.end());
      len[t].push_back((int64_t)row.size());
    }
  };
  std::vector<std::thread> pool;
  for (int64_t t = 1; t < nt; ++t) pool.emplace_back(run, t);
  run(0);
  for (std::thread& th : pool) th.join();
  g->ptr.assign(n + 1, 0);
  g->adj.clear();
  int64_t total = 0;
  for (const auto& a : adj) total += (int64_t)a.size();
  g->adj.reserve(total);
  int64_t col = 0;
  for (int64_t t = 0; t < nt; ++t) {
    g->adj.insert(g->adj.end(), adj[t].begin(), adj[t].end());
    for (int64_t c : len[t]) { g->ptr[col + 1] = g->ptr[col] + c; ++col; }
  }
}

void build_graph_from_lower(int64_t n, const int64_t* rp, const int32_t* ci, Graph* g) {
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
      if (ci[e] != i) { cnt[i + 1]++; cnt[ci[e] + 1]++; }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  g->n = n;
  g->ptr = cnt;
  g->adj.resize(cnt[n]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
      if (ci[e] != i) { g->adj[fill[i]++] = ci[e]; g->adj[fill[ci[e]]++] = (int32_t)i; }
  for (int64_t i = 0; i < n; ++i) std::sort(g->adj.begin() + g->ptr[i], g->adj.begin() + g->ptr[i + 1]);
}

void build_kmap_problem(const HostProblem& p, KMap* km) {
  const int64_t n = p.n;
  km->n = n;
  // Columns are independent: contiguous column ranges, balanced by the J
  // entries they visit, are mapped on up to 8 host threads into arrays of
  // their own and concatenated in column order (the result does not depend
  // on the number of threads).
  struct Part {
    std::vector<int32_t> kc, krow, kh, tk, ta, tb;
    std::vector<int64_t> tend;    // triples of the part up to each entry
    std::vector<int64_t> ncol;    // entries of each column of the range
  };
  std::vector<int64_t> work(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    int64_t w = 1 + (p.hp[i + 1] - p.hp[i]);
    for (int64_t q = p.jtp[i]; q < p.jtp[i + 1]; ++q) w += p.jp[p.jtr[q] + 1] - p.jp[p.jtr[q]];
    work[i + 1] = work[i] + w;
  }
  const int64_t nt = host_threads(work[n], 1 << 22);
  std::vector<int64_t> cut(nt + 1, n);
  cut[0] = 0;
  for (int64_t t = 1; t < nt; ++t)
    cut[t] = std::lower_bound(work.begin(), work.end(), work[n] * t / nt) - work.begin();
  for (int64_t t = 1; t <= nt; ++t) cut[t] = std::max(cut[t], cut[t - 1]);
  std::vector<Part> parts(nt);
  auto run = [&](int64_t t) {
    Part& q = parts[t];
    struct Item { int32_t j, k, a, b; };
    std::vector<Item> items;
    for (int64_t i = cut[t]; i < cut[t + 1]; ++i) {
      items.clear();
      for (int64_t r = p.jtp[i]; r < p.jtp[i + 1]; ++r) {
        int32_t k = p.jtr[r], a = p.jte[r];
        for (int64_t e = p.jp[k]; e < p.jp[k + 1]; ++e) {
          int32_t j = p.jc[e];
          if (j > i) break;
          items.push_back({j, k, a, (int32_t)e});
        }
      }
      std::sort(items.begin(), items.end(), [](const Item& x, const Item& y) {
        return x.j != y.j ? x.j < y.j : x.k < y.k;
      });
      // merge with the H row (lower, sorted; includes the diagonal)
      const size_t before = q.kc.size();
      size_t u = 0;
      int64_t eh = p.hp[i];
      while (u < items.size() || eh < p.hp[i + 1]) {
        int32_t jt = u < items.size() ? items[u].j : INT32_MAX;
        int32_t jh = eh < p.hp[i + 1] ? p.hc[eh] : INT32_MAX;
        int32_t j = std::min(jt, jh);
        q.kc.push_back(j);
        q.krow.push_back((int32_t)i);
        q.kh.push_back(jh == j ? (int32_t)eh++ : -1);
        while (u < items.size() && items[u].j == j) {
          q.tk.push_back(items[u].k);
          q.ta.push_back(items[u].a);
          q.tb.push_back(items[u].b);
          ++u;
        }
        q.tend.push_back((int64_t)q.tk.size());
      }
      q.ncol.push_back((int64_t)(q.kc.size() - before));
    }
  };
  std::vector<std::thread> pool;
  for (int64_t t = 1; t < nt; ++t) pool.emplace_back(run, t);
  run(0);
  for (std::thread& th : pool) th.join();
  int64_t ne = 0, ntr = 0;
  for (const Part& q : parts) { ne += (int64_t)q.kc.size(); ntr += (int64_t)q.tk.size(); }
  km->kp.assign(n + 1, 0);
  km->kc.clear(); km->krow.clear(); km->kh.clear(); km->tk.clear(); km->ta.clear(); km->tb.clear();
  km->kc.reserve(ne); km->krow.reserve(ne); km->kh.reserve(ne);
  km->tk.reserve(ntr); km->ta.reserve(ntr); km->tb.reserve(ntr);
  km->tp.assign(1, 0);
  km->tp.reserve(ne + 1);
  int64_t col = 0;
  for (const Part& q : parts) {
    const int64_t base = (int64_t)km->tk.size();
    km->kc.insert(km->kc.end(), q.kc.begin(), q.kc.end());
    km->krow.insert(km->krow.end(), q.krow.begin(), q.krow.end());
    km->kh.insert(km->kh.end(), q.kh.begin(), q.kh.end());
    km->tk.insert(km->tk.end(), q.tk.begin(), q.tk.end());
    km->ta.insert(km->ta.end(), q.ta.begin(), q.ta.end());
    km->tb.insert(km->tb.end(), q.tb.begin(), q.tb.end());
    for (int64_t v : q.tend) km->tp.push_back(base + v);
    for (int64_t c : q.ncol) { km->kp[col + 1] = km->kp[col] + c; ++col; }
  }
}

void build_dual_structures(const HostProblem& p, Graph* g, KMap* km) {
  // A structural view of the problem whose constraint matrix is J' (its rows
  // are the columns of J) and whose Hessian is diagonal: the primal builders
  // then give the pattern of diag + (J')' D (J') = diag + J D J', the dual
  // condensed matrix, and its assembly triples, with entry indices in J'
  // order that are mapped back to J's CSR order below.
  HostProblem t;
  t.n = p.m;
  t.m = p.n;
  t.jp = p.jtp;
  t.jc = p.jtr;
  t.jtp = p.jp;
  t.jtr = p.jc;
  const int64_t nnz = (int64_t)p.jc.size();
  t.jte.resize(nnz);
  for (int64_t q = 0; q < nnz; ++q) t.jte[p.jte[q]] = (int32_t)q;
  t.hp.resize(p.m + 1);
  t.hc.resize(p.m);
  t.hsp.resize(p.m + 1);
  t.hsc.resize(p.m);
  t.hss.resize(p.m);
  for (int64_t k = 0; k <= p.m; ++k) t.hp[k] = t.hsp[k] = k;
  for (int64_t k = 0; k < p.m; ++k) t.hc[k] = t.hsc[k] = t.hss[k] = (int32_t)k;
  build_graph_from_problem(t, g);
  build_kmap_problem(t, km);
  for (int32_t& h : km->kh) h = -1;                 // M has no Hessian term
  for (int32_t& a : km->ta) a = p.jte[a];
  for (int32_t& b : km->tb) b = p.jte[b];
}

void build_augmented_structures(const HostProblem& p, Graph* g, KMap* km) {
  const int64_t n = p.n, m = p.m, N = n + m;
  // graph: x_i ~ x_j through H, x_j ~ lambda_k through J (lambda_k = n + k)
  g->n = N;
  g->ptr.assign(N + 1, 0);
  g->adj.clear();
  std::vector<int32_t> row;
  for (int64_t i = 0; i < n; ++i) {
    row.clear();
    for (int64_t q = p.hsp[i]; q < p.hsp[i + 1]; ++q)
      if (p.hsc[q] != i) row.push_back(p.hsc[q]);
    for (int64_t q = p.jtp[i]; q < p.jtp[i + 1]; ++q) row.push_back((int32_t)(n + p.jtr[q]));
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    g->adj.insert(g->adj.end(), row.begin(), row.end());
    g->ptr[i + 1] = (int64_t)g->adj.size();
  }
  for (int64_t k = 0; k < m; ++k) {
    for (int64_t e = p.jp[k]; e < p.jp[k + 1]; ++e) g->adj.push_back(p.jc[e]);
    g->ptr[n + k + 1] = (int64_t)g->adj.size();
  }
  // lower pattern: x rows = H's lower rows; lambda row k = J row k, then its
  // diagonal.  kh holds the H entry (x rows) or the J entry (lambda rows,
  // -1 on the diagonal); there are no product triples.
  km->n = N;
  km->kp.assign(N + 1, 0);
  km->kc.clear(); km->krow.clear(); km->kh.clear();
  km->tk.clear(); km->ta.clear(); km->tb.clear();
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = p.hp[i]; e < p.hp[i + 1]; ++e) {
      km->kc.push_back(p.hc[e]);
      km->krow.push_back((int32_t)i);
      km->kh.push_back((int32_t)e);
    }
    km->kp[i + 1] = (int64_t)km->kc.size();
  }
  for (int64_t k = 0; k < m; ++k) {
    for (int64_t e = p.jp[k]; e < p.jp[k + 1]; ++e) {
      km->kc.push_back(p.jc[e]);
      km->krow.push_back((int32_t)(n + k));
      km->kh.push_back((int32_t)e);
    }
    km->kc.push_back((int32_t)(n + k));
    km->krow.push_back((int32_t)(n + k));
    km->kh.push_back(-1);
    km->kp[n + k + 1] = (int64_t)km->kc.size();
  }
  km->tp.assign(km->kc.size() + 1, 0);
}

void build_kmap_lower(int64_t n, const int64_t* rp, const int32_t* ci, KMap* km) {
  km->n = n;
  km->kp.assign(rp, rp + n + 1);
  km->kc.assign(ci, ci + rp[n]);
  km->krow.resize(rp[n]);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) km->krow[e] = (int32_t)i;
  km->kh.clear(); km->tk.clear(); km->ta.clear(); km->tb.clear();
  km->tp.clear();
}

double gemm_desc_flops(const GemmDesc& g) {
  if (g.mode == 1) return (double)g.M * g.K * g.K;   // triangular solve
  if (g.lower) {
    const double n = std::min(g.M, g.N);
    return 2.0 * g.K * ((double)g.M * g.N - n * (n - 1) / 2);
  }
  return 2.0 * g.K * (double)g.M * g.N;
}

void build_plan(const Symbolic& s, int esize, Plan* pl, const Blocking& blk) {
  Plan& P = *pl;
  P = Plan();
  P.esize = esize;
  P.nb = esize == 8 ? 64 : 128;            // diagonal block / panel-solve width
  // outer block: rank of the trailing update (a multiple of nb); by default
  // 512 columns in both precisions (FP64: eight 64-column blocks)
  const int nbo = P.nb * (blk.outer_blocks > 0 ? blk.outer_blocks : (esize == 8 ? 8 : 4));
  P.small_h = blk.small_h > 0 && blk.small_h <= SMALL_H_MAX ? blk.small_h : SMALL_H_MAX;
  const int64_t ns = s.nsuper();
  P.ns = ns;
  P.n = s.n;
  P.sfirst.resize(ns); P.sw.resize(ns); P.sh.resize(ns); P.sld.resize(ns); P.sparent.assign(ns, -1);
  P.slevel.assign(ns, 0); P.spanel.resize(ns); P.su.resize(ns); P.srow.resize(ns + 1); P.suv.resize(ns);
  std::vector<int32_t> col2sn(s.n);
  for (int64_t k = 0; k < ns; ++k) {
    P.sfirst[k] = s.sn_start[k];
    P.sw[k] = s.sn_start[k + 1] - s.sn_start[k];
    P.sh[k] = (int32_t)(s.sn_rowptr[k + 1] - s.sn_rowptr[k]);
    // columns of fronts taller than any small-front limit start on 128-byte
    // boundaries (the GEMM tiles then touch no partial cache lines: +5% GEMM
    // rate), the others on 16-byte ones.  The rule must not depend on the
    // blocking: the map of K entries to panel positions is built once and
    // serves every blocking the autotuner tries.
    P.sld[k] = P.sh[k] > SMALL_H_MAX ? (P.sh[k] + 31) & ~31 : (P.sh[k] + 3) & ~3;
    P.srow[k] = s.sn_rowptr[k];
    for (int32_t j = s.sn_start[k]; j < s.sn_start[k + 1]; ++j) col2sn[j] = (int32_t)k;
  }
  P.srow[ns] = s.sn_rowptr[ns];
  int64_t off = 0, uoff = 0, uvoff = 0;
  P.sldu.resize(ns);
  for (int64_t k = 0; k < ns; ++k) {
    // the panels of fronts taller than the small-front limit and the update
    // matrices with more than that many rows start on 32-element boundaries
    // and keep their columns there (leading dimensions multiples of 32);
    // rules of h and h - w alone, so the layout serves every blocking
    if (P.sh[k] > SMALL_H_MAX) off = (off + 31) & ~(int64_t)31;
    P.spanel[k] = off;
    off += (int64_t)P.sld[k] * P.sw[k];
    int64_t hu = P.sh[k] - P.sw[k];
    P.sldu[k] = (int32_t)(hu > SMALL_H_MAX ? (hu + 31) & ~31 : hu);
    if (hu > SMALL_H_MAX) uoff = (uoff + 31) & ~(int64_t)31;
    P.su[k] = uoff;
    uoff += hu * P.sldu[k];
    P.suv[k] = uvoff;
    uvoff += hu;
    P.max_front = std::max<int64_t>(P.max_front, P.sh[k]);
    int32_t last = s.sn_start[k + 1] - 1;
    if (s.etree[last] >= 0) P.sparent[k] = col2sn[s.etree[last]];
  }
  P.panel_elems = off;
  P.u_elems = uoff;
  P.uv_elems = uvoff;
  P.update_bytes = (double)uoff * esize;
  // children (increasing) and levels
  P.child_ptr.assign(ns + 1, 0);
  for (int64_t k = 0; k < ns; ++k)
    if (P.sparent[k] >= 0) P.child_ptr[P.sparent[k] + 1]++;
  for (int64_t k = 0; k < ns; ++k) P.child_ptr[k + 1] += P.child_ptr[k];
  P.child.resize(P.child_ptr[ns]);
  {
    std::vector<int32_t> fill(P.child_ptr.begin(), P.child_ptr.end() - 1);
    for (int64_t k = 0; k < ns; ++k)
      if (P.sparent[k] >= 0) P.child[fill[P.sparent[k]]++] = (int32_t)k;
  }
  for (int64_t k = 0; k < ns; ++k)
    if (P.sparent[k] >= 0) P.slevel[P.sparent[k]] = std::max(P.slevel[P.sparent[k]], P.slevel[k] + 1);
  P.nlevels = 0;
  for (int64_t k = 0; k < ns; ++k) P.nlevels = std::max(P.nlevels, P.slevel[k] + 1);
  P.level_ptr.assign(P.nlevels + 1, 0);
  for (int64_t k = 0; k < ns; ++k) P.level_ptr[P.slevel[k] + 1]++;
  for (int l = 0; l < P.nlevels; ++l) P.level_ptr[l + 1] += P.level_ptr[l];
  P.level_sn.resize(ns);
  {
    std::vector<int32_t> fill(P.level_ptr.begin(), P.level_ptr.end() - 1);
    for (int64_t k = 0; k < ns; ++k) P.level_sn[fill[P.slevel[k]]++] = (int32_t)k;
  }
  // relative row positions in the parent front
  P.rel.assign(s.sn_rows.size(), -1);
  for (int64_t k = 0; k < ns; ++k) {
    int32_t par = P.sparent[k];
    if (par < 0) continue;
    const int32_t* pr = s.sn_rows.data() + s.sn_rowptr[par];
    int64_t ph = s.sn_rowptr[par + 1] - s.sn_rowptr[par];
    int64_t q = 0;
    for (int64_t e = s.sn_rowptr[k] + P.sw[k]; e < s.sn_rowptr[k + 1]; ++e) {
      int32_t r = s.sn_rows[e];
      while (q < ph && pr[q] < r) ++q;
      if (q >= ph || pr[q] != r) throw std::runtime_error("child row missing from parent front");
      P.rel[e] = (int32_t)q;
    }
  }
  // permanent storage of the inverses of the diagonal blocks (large fronts):
  // nb-column blocks for the factorisation's panel solves (finv), then, in
  // FP64, the SOLVE_NB-column blocks of the triangular solves (sinv; the
  // same blocks in FP32, where nb = SOLVE_NB)
  const int nb = P.nb;
  std::vector<int64_t> finv(ns, -1);
  int64_t ioff = 0;
  for (int64_t k = 0; k < ns; ++k) {
    if (P.sh[k] <= P.small_h) continue;
    finv[k] = ioff;
    ioff += (int64_t)((P.sw[k] + nb - 1) / nb) * nb * nb;
  }
  if (nb == SOLVE_NB) {
    P.sinv = finv;
  } else {
    if (SOLVE_NB != 2 * nb) throw std::runtime_error("solve blocks must pair factor blocks");
    P.sinv.assign(ns, -1);
    for (int64_t k = 0; k < ns; ++k) {
      if (finv[k] < 0) continue;
      P.sinv[k] = ioff;
      for (int32_t c0 = 0; c0 < P.sw[k]; c0 += SOLVE_NB) {
        InvCombDesc d{};
        d.bw = std::min(SOLVE_NB, P.sw[k] - c0);
        d.x1_off = finv[k] + (int64_t)(c0 / nb) * nb * nb;
        d.x2_off = d.bw > nb ? d.x1_off + (int64_t)nb * nb : -1;
        d.ld = P.sld[k];
        d.l21_off = P.spanel[k] + (int64_t)c0 * P.sld[k] + c0 + nb;
        d.out_off = ioff;
        P.icomb.push_back(d);
        ioff += (int64_t)SOLVE_NB * SOLVE_NB;
      }
    }
  }
  P.inv_elems = std::max<int64_t>(1, ioff);
  // launch schedule, level by level
  for (int l = 0; l < P.nlevels; ++l) {
    std::vector<int32_t> large;
    int64_t small_begin = (int64_t)P.small.size();
    for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; ++q) {
      int32_t k = P.level_sn[q];
      if (P.sh[k] <= P.small_h) P.small.push_back(k);
      else large.push_back(k);
    }
    if (!large.empty()) {
      int64_t zb = (int64_t)P.ext.size();
      for (int32_t k : large) {
        if (P.child_ptr[k + 1] == P.child_ptr[k]) continue;
        for (int32_t t0 = 0; t0 < P.sh[k]; t0 += 16)
          P.ext.push_back({k, t0, std::min<int32_t>(t0 + 16, P.sh[k]), 0});
      }
      if ((int64_t)P.ext.size() > zb)
        P.ops.push_back({OP_EXTEND_ADD, zb, (int64_t)P.ext.size(), (int64_t)P.ext.size() - zb});
    }
    if ((int64_t)P.small.size() > small_begin)
      P.ops.push_back({OP_SMALL, small_begin, (int64_t)P.small.size(), (int64_t)P.small.size() - small_begin});
    if (large.empty()) continue;
    int32_t maxw = 0;
    for (int32_t k : large) maxw = std::max(maxw, P.sw[k]);
    const int tm = esize == 8 ? GEMM_TILE_F64 : GEMM_TILE_F32;
    auto add_gemm = [&](int64_t c_off, int64_t a_off, int64_t b_off, int32_t ldc, int32_t lda, int32_t ldb,
                        int32_t M, int32_t N, int32_t K, int32_t c_buf, int32_t b_buf, int32_t mode,
                        int32_t lower, int32_t kcol, int64_t& tiles) {
      GemmDesc g{};
      g.kcol = kcol;
      g.c_off = c_off; g.a_off = a_off; g.b_off = b_off;
      g.ldc = ldc; g.lda = lda; g.ldb = ldb;
      g.M = M; g.N = N; g.K = K;
      g.c_buf = c_buf; g.b_buf = b_buf; g.mode = mode; g.lower = lower;
      g.tiles_m = (M + tm - 1) / tm; g.tiles_n = (N + tm - 1) / tm;
      g.tile_begin = tiles;
      // lower-masked blocks start on the diagonal (M >= N): only tiles on or
      // below the diagonal are enumerated
      if (lower) tiles += (int64_t)g.tiles_n * g.tiles_m - (int64_t)g.tiles_n * (g.tiles_n - 1) / 2;
      else tiles += (int64_t)g.tiles_m * g.tiles_n;
      P.gemm.push_back(g);
    };
    // two-level blocking: inner blocks of nb columns, each first updated by
    // the earlier inner blocks of its outer block (left-looking: one update
    // of rank c0 - o0 instead of one rank-nb update per earlier block, so the
    // block's columns are read and written once), then diagonal factor and
    // panel solve; after the outer block, one rank-nbo update of everything
    // to its right
    for (int32_t o0 = 0; o0 < maxw; o0 += nbo) {
      for (int32_t c0 = o0; c0 < std::min(o0 + nbo, maxw); c0 += nb) {
        if (c0 > o0) {
          int64_t gb = (int64_t)P.gemm.size(), tiles = 0;
          for (int32_t k : large) {
            if (P.sw[k] <= c0) continue;
            const int32_t h = P.sh[k], ld = P.sld[k], bw = std::min(nb, P.sw[k] - c0);
            add_gemm(P.spanel[k] + (int64_t)c0 * ld + c0, P.spanel[k] + (int64_t)o0 * ld + c0,
                     P.spanel[k] + (int64_t)o0 * ld + c0, ld, ld, ld, h - c0, bw, c0 - o0, 0, 0, 0, 1,
                     P.sfirst[k] + o0, tiles);
          }
          if (tiles) P.ops.push_back({OP_UPDATE, gb, (int64_t)P.gemm.size(), tiles});
        }
        int64_t pb = (int64_t)P.potrf.size();
        std::vector<int64_t> inv_of(large.size(), -1);
        for (size_t q = 0; q < large.size(); ++q) {
          int32_t k = large[q];
          if (P.sw[k] <= c0) continue;
          int32_t bw = std::min(nb, P.sw[k] - c0);
          PotrfDesc d;
          d.d_off = P.spanel[k] + (int64_t)c0 * P.sld[k] + c0;
          d.inv_off = finv[k] + (int64_t)(c0 / nb) * nb * nb;
          d.ld = P.sld[k];
          d.bw = bw;
          d.col0 = P.sfirst[k] + c0;
          d.pad = 0;
          inv_of[q] = d.inv_off;
          P.potrf.push_back(d);
        }
        P.ops.push_back({OP_POTRF, pb, (int64_t)P.potrf.size(), (int64_t)P.potrf.size() - pb});
        // panel solve below the diagonal block, in place: C = A * inv(L_JJ)^T
        int64_t gb = (int64_t)P.gemm.size(), tiles = 0;
        for (size_t q = 0; q < large.size(); ++q) {
          int32_t k = large[q];
          if (inv_of[q] < 0) continue;
          int32_t bw = std::min(nb, P.sw[k] - c0);
          int32_t M = P.sh[k] - c0 - bw;
          if (M <= 0) continue;
          int64_t off = P.spanel[k] + (int64_t)c0 * P.sld[k] + c0 + bw;
          add_gemm(off, off, inv_of[q], P.sld[k], P.sld[k], nb, M, bw, bw, 0, 1, 1, 0, P.sfirst[k] + c0, tiles);
        }
        if (tiles) P.ops.push_back({OP_TRSM, gb, (int64_t)P.gemm.size(), tiles});
      }
      // rank-(outer block) update of the trailing panel columns and of U
      int64_t gb = (int64_t)P.gemm.size(), tiles = 0;
      for (size_t q = 0; q < large.size(); ++q) {
        int32_t k = large[q];
        int32_t h = P.sh[k], w = P.sw[k], ld = P.sld[k];
        if (w <= o0) continue;
        int32_t o1 = std::min(o0 + nbo, w), K = o1 - o0;
        if (w - o1 > 0)
          add_gemm(P.spanel[k] + (int64_t)o1 * ld + o1, P.spanel[k] + (int64_t)o0 * ld + o1,
                   P.spanel[k] + (int64_t)o0 * ld + o1, ld, ld, ld, h - o1, w - o1, K, 0, 0, 0, 1,
                   P.sfirst[k] + o0, tiles);
        if (h - w > 0)
          add_gemm(P.su[k], P.spanel[k] + (int64_t)o0 * ld + w, P.spanel[k] + (int64_t)o0 * ld + w, P.sldu[k], ld,
                   ld, h - w, h - w, K, 1, 0, 0, 1, P.sfirst[k] + o0, tiles);
      }
      if (tiles) P.ops.push_back({OP_UPDATE, gb, (int64_t)P.gemm.size(), tiles});
    }
  }
  for (const Op& op : P.ops) {
    if (op.type != OP_TRSM && op.type != OP_UPDATE) continue;
    ++P.gemm_launches;
    for (int64_t q = op.begin; q < op.end; ++q) {
      const GemmDesc& g = P.gemm[q];
      {
        const double n = std::min(g.M, g.N);
        const double c = g.lower ? (double)g.M * g.N - n * (n - 1) / 2 : (double)g.M * g.N;
        P.gemm_bytes += (double)esize * ((double)g.M * g.K + (g.mode == 1 ? (double)g.K * g.K : (double)g.N * g.K) +
                                         (g.mode == 1 ? 1.0 : 2.0) * c);
      }
      P.gemm_flops += gemm_desc_flops(g);
    }
  }
  if (!P.icomb.empty())
    P.ops.push_back({OP_INV_COMBINE, 0, (int64_t)P.icomb.size(), (int64_t)P.icomb.size()});
  // ---- gather map of the forward solve: for each front row of a large
  // supernode, its children's update-vector entries in child order
  P.grow.assign(ns, -1);
  for (int64_t k = 0; k < ns; ++k) {
    if (P.sh[k] <= P.small_h) continue;
    const int64_t base = (int64_t)P.gptr.size();
    P.grow[k] = base;
    P.gptr.resize(base + P.sh[k] + 1, 0);
    int64_t* rp = P.gptr.data() + base;
    for (int32_t q = P.child_ptr[k]; q < P.child_ptr[k + 1]; ++q) {
      const int32_t c = P.child[q];
      for (int64_t e = P.srow[c] + P.sw[c]; e < P.srow[c + 1]; ++e) rp[P.rel[e] + 1]++;
    }
    rp[0] = (int64_t)P.gidx.size();
    for (int32_t r = 0; r < P.sh[k]; ++r) rp[r + 1] += rp[r];
    P.gidx.resize(rp[P.sh[k]]);
    std::vector<int64_t> pos(rp, rp + P.sh[k]);
    for (int32_t q = P.child_ptr[k]; q < P.child_ptr[k + 1]; ++q) {
      const int32_t c = P.child[q];
      for (int64_t e = P.srow[c] + P.sw[c]; e < P.srow[c + 1]; ++e)
        P.gidx[pos[P.rel[e]]++] = P.suv[c] + (e - P.srow[c] - P.sw[c]);
    }
  }
  if (P.gptr.empty()) P.gptr.push_back(0);
  if (P.gidx.empty()) P.gidx.push_back(0);
  // ---- triangular solve schedule (same levels; large fronts blocked by
  // SOLVE_NB columns)
  const int snb = SOLVE_NB;
  const int RB = 128;  // rows per forward work item
  for (int l = 0; l < P.nlevels; ++l) {
    std::vector<int32_t> large;
    int64_t sb = (int64_t)P.ssmall.size();
    for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; ++q) {
      int32_t k = P.level_sn[q];
      if (P.sh[k] <= P.small_h) P.ssmall.push_back(k);
      else large.push_back(k);
    }
    if ((int64_t)P.ssmall.size() > sb)
      P.fwd_ops.push_back({OP_FWD_SMALL, sb, (int64_t)P.ssmall.size(), (int64_t)P.ssmall.size() - sb});
    if (large.empty()) continue;
    int64_t gb = (int64_t)P.slarge.size();
    for (int32_t k : large) P.slarge.push_back(k);
    // children's update vectors into the fronts (one row per thread), then
    // y of each front's first column block
    const int64_t ib = (int64_t)P.gitem.size();
    for (int32_t k : large)
      for (int32_t r0 = 0; r0 < P.sh[k]; r0 += GATHER_ROWS)
        P.gitem.push_back({k, r0, std::min(r0 + GATHER_ROWS, P.sh[k]), 0});
    P.fwd_ops.push_back({OP_FWD_GATHER, ib, (int64_t)P.gitem.size(), (int64_t)P.gitem.size() - ib});
    P.fwd_ops.push_back({OP_FWD_FIRST, gb, (int64_t)P.slarge.size(), (int64_t)large.size()});
    int32_t maxw = 0;
    for (int32_t k : large) maxw = std::max(maxw, P.sw[k]);
    for (int32_t c0 = 0; c0 < maxw; c0 += snb) {
      int64_t db = (int64_t)P.sdesc.size();
      for (int32_t k : large) {
        if (P.sw[k] <= c0) continue;
        int32_t bw = std::min(snb, P.sw[k] - c0);
        for (int32_t r0 = c0 + bw; r0 < P.sh[k]; r0 += RB) {
          SolveDesc d{};
          d.sn = k; d.c0 = c0; d.bw = bw; d.r0 = r0; d.r1 = std::min(r0 + RB, P.sh[k]);
          d.owner = (r0 == c0 + bw && c0 + bw < P.sw[k]) ? 1 : 0;
          P.sdesc.push_back(d);
        }
      }
      if ((int64_t)P.sdesc.size() > db)
        P.fwd_ops.push_back({OP_FWD_STEP, db, (int64_t)P.sdesc.size(), (int64_t)P.sdesc.size() - db});
    }
  }
  // backward: levels from the root down; column blocks from the last one:
  // partial products over row ranges below the block, then the block solve
  const int RBB = 128;  // rows per backward partial item
  for (int l = P.nlevels - 1; l >= 0; --l) {
    std::vector<int32_t> large;
    int64_t sb = (int64_t)P.ssmall.size();
    for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; ++q) {
      int32_t k = P.level_sn[q];
      if (P.sh[k] <= P.small_h) P.ssmall.push_back(k);
      else large.push_back(k);
    }
    if ((int64_t)P.ssmall.size() > sb)
      P.bwd_ops.push_back({OP_BWD_SMALL, sb, (int64_t)P.ssmall.size(), (int64_t)P.ssmall.size() - sb});
    if (large.empty()) continue;
    int32_t maxw = 0;
    for (int32_t k : large) maxw = std::max(maxw, P.sw[k]);
    const int32_t nsteps = (maxw + snb - 1) / snb;
    for (int32_t step = nsteps - 1; step >= 0; --step) {
      const int32_t c0 = step * snb;
      int64_t pb = (int64_t)P.sdesc.size();
      int64_t part = 0;
      std::vector<SolveDesc> diag;
      for (int32_t k : large) {
        if (P.sw[k] <= c0) continue;
        int32_t bw = std::min(snb, P.sw[k] - c0);
        SolveDesc dd{};
        dd.sn = k; dd.c0 = c0; dd.bw = bw; dd.owner = 1; dd.part_off = part;
        int32_t np = 0;
        for (int32_t r0 = c0 + bw; r0 < P.sh[k]; r0 += RBB) {
          SolveDesc d{};
          d.sn = k; d.c0 = c0; d.bw = bw; d.r0 = r0; d.r1 = std::min(r0 + RBB, P.sh[k]);
          d.part_off = part;
          part += snb;
          ++np;
          P.sdesc.push_back(d);
        }
        dd.nparts = np;
        diag.push_back(dd);
      }
      P.part_elems = std::max(P.part_elems, part);
      if ((int64_t)P.sdesc.size() > pb)
        P.bwd_ops.push_back({OP_BWD_PART, pb, (int64_t)P.sdesc.size(), (int64_t)P.sdesc.size() - pb});
      int64_t qb = (int64_t)P.sdesc.size();
      for (auto& d : diag) P.sdesc.push_back(d);
      P.bwd_ops.push_back({OP_BWD_DIAG, qb, (int64_t)P.sdesc.size(), (int64_t)P.sdesc.size() - qb});
    }
  }
  for (SolveDesc& d : P.sdesc) {
    const int32_t k = d.sn;
    d.w = P.sw[k]; d.first = P.sfirst[k]; d.ld = P.sld[k];
    d.panel_off = P.spanel[k]; d.uvec_off = P.suv[k]; d.inv_off = P.sinv[k]; d.row_off = P.srow[k];
  }
}

void map_k_to_panels(const Symbolic& s, const Plan& P, KMap* km) {
  const int64_t nk = (int64_t)km->kc.size();
  km->pos.resize(nk);
  std::vector<int32_t> col2sn(s.n);
  for (int64_t k = 0; k < P.ns; ++k)
    for (int32_t j = s.sn_start[k]; j < s.sn_start[k + 1]; ++j) col2sn[j] = (int32_t)k;
  // entries are independent: contiguous ranges on up to 8 host threads
  std::atomic<bool> outside{false};
  auto range = [&](int64_t e0, int64_t e1) {
    for (int64_t e = e0; e < e1; ++e) {
      int32_t a = s.pinv[km->krow[e]], b = s.pinv[km->kc[e]];
      int32_t r = std::max(a, b), c = std::min(a, b);
      int32_t k = col2sn[c];
      const int32_t* rows = s.sn_rows.data() + s.sn_rowptr[k];
      int64_t h = s.sn_rowptr[k + 1] - s.sn_rowptr[k];
      const int32_t* it = std::lower_bound(rows, rows + h, r);
      if (it == rows + h || *it != r) { outside = true; return; }
      km->pos[e] = P.spanel[k] + (int64_t)(c - P.sfirst[k]) * P.sld[k] + (it - rows);
    }
  };
  const int64_t nt = host_threads(nk, 1 << 20);
  std::vector<std::thread> pool;
  for (int64_t t = 1; t < nt; ++t) pool.emplace_back(range, nk * t / nt, nk * (t + 1) / nt);
  range(0, nk / nt);
  for (std::thread& th : pool) th.join();
  if (outside) throw std::runtime_error("K entry outside the factor structure");
}

}  // namespace pdipm
