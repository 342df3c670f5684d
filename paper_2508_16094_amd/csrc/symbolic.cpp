// Fill-reducing ordering and supernodal symbolic factorisation (host).
#include "symbolic.hpp"

#include <algorithm>
#include <cstring>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <stdexcept>
#include <thread>

namespace pdipm {

int64_t host_threads(int64_t work, int64_t work_min) {
  if (const char* e = std::getenv("PDIPM_HOST_THREADS")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1) return std::min<long>(v, 64);
  }
  if (work < work_min) return 1;
  return std::min<int64_t>(8, std::max(1u, std::thread::hardware_concurrency()));
}

AmalgamationRule amalgamation_rule(int menu) {
  switch (menu) {
    case 1: return {128, 16, 1, 20};
    case 2: return {64, 8, 1, 10};
    case -1: return {1, 0, 0, 1};  // no amalgamation
    default: return {1 << 30, 8, 1, 10};
  }
}

namespace {

// Work item of the dissection: a vertex list to order, or to emit as is.
struct Task {
  bool emit;
  std::vector<int32_t> v;
};

struct NdState {
  const Graph& g;
  std::vector<int32_t> mark;   // membership stamp of the current task
  std::vector<int32_t> seen;   // BFS stamp
  std::vector<int32_t> deg;    // degree inside the current component
  int32_t stamp = 0, bstamp = 0;
  explicit NdState(const Graph& gr)
      : g(gr), mark(gr.n, -1), seen(gr.n, -1), deg(gr.n, 0) {}

  // BFS levels from root inside vertices marked `stamp`; levels stored flat.
  int bfs(int32_t root, std::vector<int32_t>& order, std::vector<int64_t>& lvl_ptr) {
    ++bstamp;
    order.clear();
    lvl_ptr.clear();
    order.push_back(root);
    seen[root] = bstamp;
    lvl_ptr.push_back(0);
    size_t begin = 0;
    while (true) {
      size_t end = order.size();
      lvl_ptr.push_back((int64_t)end);
      for (size_t q = begin; q < end; ++q) {
        int32_t u = order[q];
        for (int64_t e = g.ptr[u]; e < g.ptr[u + 1]; ++e) {
          int32_t w = g.adj[e];
          if (mark[w] == stamp && seen[w] != bstamp) {
            seen[w] = bstamp;
            order.push_back(w);
          }
        }
      }
      if (order.size() == end) break;
      begin = end;
    }
    return (int)lvl_ptr.size() - 1;  // number of levels
  }
};

int32_t min_degree_vertex(const std::vector<int32_t>& deg, const int32_t* v, size_t cnt) {
  int32_t best = v[0];
  for (size_t i = 1; i < cnt; ++i) {
    int32_t u = v[i];
    if (deg[u] < deg[best] || (deg[u] == deg[best] && u < best)) best = u;
  }
  return best;
}

// Exact minimum degree on at most 64 vertices with bitmask adjacency.
void leaf_minimum_degree(NdState& st, const std::vector<int32_t>& comp, std::vector<int32_t>& out) {
  const int k = (int)comp.size();
  uint64_t nb[64];
  for (int a = 0; a < k; ++a) {
    nb[a] = 0;
    int32_t v = comp[a];
    for (int64_t e = st.g.ptr[v]; e < st.g.ptr[v + 1]; ++e) {
      int32_t w = st.g.adj[e];
      if (st.mark[w] != st.stamp) continue;
      auto it = std::lower_bound(comp.begin(), comp.end(), w);
      if (it != comp.end() && *it == w) nb[a] |= 1ull << (it - comp.begin());
    }
  }
  uint64_t alive = (k == 64) ? ~0ull : ((1ull << k) - 1);
  for (int step = 0; step < k; ++step) {
    int best = -1, bdeg = 1 << 30;
    for (uint64_t m = alive; m; m &= m - 1) {
      int a = __builtin_ctzll(m);
      int d = __builtin_popcountll(nb[a] & alive);
      if (d < bdeg) { bdeg = d; best = a; }   // ascending a: ties keep smallest
    }
    out.push_back(comp[best]);
    uint64_t clique = nb[best] & alive & ~(1ull << best);
    for (uint64_t m = clique; m; m &= m - 1) {
      int a = __builtin_ctzll(m);
      nb[a] |= clique;
      nb[a] &= ~(1ull << a);
    }
    alive &= ~(1ull << best);
  }
}

// Order a component by increasing degree inside it (st.deg), ties by index.
std::vector<int32_t> degree_order(const NdState& st, const std::vector<int32_t>& comp) {
  std::vector<int32_t> out(comp);
  std::stable_sort(out.begin(), out.end(), [&](int32_t a, int32_t b) {
    return st.deg[a] != st.deg[b] ? st.deg[a] < st.deg[b] : a < b;
  });
  return out;
}

// ---------------------------------------------- multilevel bisection
// Separators from multilevel graph bisection in the style of METIS (Karypis
// and Kumar): heavy-edge matching down to a small graph, a BFS-grown
// bisection there, greedy boundary refinement on every level on the way
// back, and the smaller boundary side of the edge cut as the vertex
// separator.  Integer weights and explicit tie-breaks throughout, so the
// result is reproducible bit for bit by an independent implementation.
constexpr int64_t ML_COARSEN_TO = 64;
constexpr int64_t ML_SHRINK_NUM = 9, ML_SHRINK_DEN = 10;
constexpr int ML_PASSES = 8;
constexpr int64_t ML_BAL_NUM = 11, ML_BAL_DEN = 20;

struct MlGraph {
  std::vector<int64_t> ptr;
  std::vector<int32_t> adj;
  std::vector<int64_t> ew, vw;
  int64_t n() const { return (int64_t)vw.size(); }
};

// Heavy-edge matching in increasing vertex order (partner: largest edge
// weight, then smaller vertex weight, then smaller index); coarse ids in
// order of the first member's visit; parallel edges and weights add.
void ml_coarsen(const MlGraph& f, std::vector<int32_t>& cmap, MlGraph& c) {
  const int64_t n = f.n();
  std::vector<char> matched(n, 0);
  cmap.assign(n, -1);
  std::vector<int32_t> first, second;
  for (int64_t v = 0; v < n; ++v) {
    if (matched[v]) continue;
    int32_t best = -1;
    int64_t bw = 0, bvw = 0;
    for (int64_t e = f.ptr[v]; e < f.ptr[v + 1]; ++e) {
      const int32_t u = f.adj[e];
      if (matched[u]) continue;
      const int64_t w = f.ew[e];
      if (best < 0 || w > bw || (w == bw && (f.vw[u] < bvw || (f.vw[u] == bvw && u < best)))) {
        best = u; bw = w; bvw = f.vw[u];
      }
    }
    matched[v] = 1;
    cmap[v] = (int32_t)first.size();
    if (best >= 0) { matched[best] = 1; cmap[best] = (int32_t)first.size(); }
    first.push_back((int32_t)v);
    second.push_back(best);
  }
  const int64_t nc = (int64_t)first.size();
  c.ptr.assign(nc + 1, 0);
  c.adj.clear(); c.ew.clear(); c.vw.assign(nc, 0);
  std::vector<int64_t> acc(nc, 0);
  std::vector<int32_t> touched;
  for (int64_t k = 0; k < nc; ++k) {
    touched.clear();
    for (int32_t v : {first[k], second[k]}) {
      if (v < 0) continue;
      c.vw[k] += f.vw[v];
      for (int64_t e = f.ptr[v]; e < f.ptr[v + 1]; ++e) {
        const int32_t cu = cmap[f.adj[e]];
        if (cu == k) continue;
        if (acc[cu] == 0) touched.push_back(cu);
        acc[cu] += f.ew[e];
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int32_t cu : touched) { c.adj.push_back(cu); c.ew.push_back(acc[cu]); acc[cu] = 0; }
    c.ptr[k + 1] = (int64_t)c.adj.size();
  }
}

// BFS levels (discovery order) from root, flat with level pointers.
int ml_bfs(const MlGraph& g, int32_t root, std::vector<int32_t>& order, std::vector<int64_t>& lp,
           std::vector<int32_t>& seen, int32_t stamp) {
  order.clear(); lp.clear();
  order.push_back(root);
  seen[root] = stamp;
  lp.push_back(0);
  size_t begin = 0;
  while (true) {
    const size_t end = order.size();
    lp.push_back((int64_t)end);
    for (size_t q = begin; q < end; ++q)
      for (int64_t e = g.ptr[order[q]]; e < g.ptr[order[q] + 1]; ++e) {
        const int32_t w = g.adj[e];
        if (seen[w] != stamp) { seen[w] = stamp; order.push_back(w); }
      }
    if (order.size() == end) break;
    begin = end;
  }
  return (int)lp.size() - 1;
}

// Part 0 = the shortest prefix of a BFS order from a pseudo-peripheral vertex
// whose weight reaches half the total.
std::vector<int8_t> ml_initial(const MlGraph& g) {
  const int64_t n = g.n();
  int64_t total = 0;
  for (int64_t w : g.vw) total += w;
  auto deg = [&](int32_t v) { return g.ptr[v + 1] - g.ptr[v]; };
  int32_t r = 0;
  for (int32_t v = 1; v < n; ++v)
    if (deg(v) < deg(r)) r = v;
  std::vector<int32_t> seen(n, 0), order, order2;
  std::vector<int64_t> lp, lp2;
  int32_t stamp = 1;
  int nl = ml_bfs(g, r, order, lp, seen, stamp);
  while (true) {
    int32_t v = order[lp[nl - 1]];
    for (int64_t q = lp[nl - 1]; q < lp[nl]; ++q) {
      const int32_t u = order[q];
      if (deg(u) < deg(v) || (deg(u) == deg(v) && u < v)) v = u;
    }
    const int nl2 = ml_bfs(g, v, order2, lp2, seen, ++stamp);
    if (nl2 > nl) { std::swap(order, order2); std::swap(lp, lp2); nl = nl2; }
    else break;
  }
  std::vector<int8_t> part(n, 1);
  int64_t w0 = 0;
  for (int32_t v : order) {
    if (2 * w0 >= total) break;
    part[v] = 0;
    w0 += g.vw[v];
  }
  return part;
}

// Greedy boundary refinement: boundary vertices by decreasing gain (ties by
// index) with gains kept current; a vertex moves when its gain is positive
// and the target part stays within the balance bound, or its gain is zero
// and the move strictly narrows the weight difference.
void ml_refine(const MlGraph& g, std::vector<int8_t>& part) {
  const int64_t n = g.n();
  int64_t total = 0;
  for (int64_t w : g.vw) total += w;
  const int64_t maxw = ML_BAL_NUM * total / ML_BAL_DEN;
  int64_t pw[2] = {0, 0};
  for (int64_t v = 0; v < n; ++v) pw[part[v]] += g.vw[v];
  std::vector<int64_t> ext(n, 0), inn(n, 0);
  for (int64_t v = 0; v < n; ++v)
    for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e)
      (part[g.adj[e]] == part[v] ? inn[v] : ext[v]) += g.ew[e];
  std::vector<int32_t> cands;
  for (int pass = 0; pass < ML_PASSES; ++pass) {
    cands.clear();
    for (int64_t v = 0; v < n; ++v)
      if (ext[v] > 0) cands.push_back((int32_t)v);
    std::sort(cands.begin(), cands.end(), [&](int32_t a, int32_t b) {
      const int64_t ka = inn[a] - ext[a], kb = inn[b] - ext[b];
      return ka != kb ? ka < kb : a < b;
    });
    bool moved = false;
    for (int32_t v : cands) {
      const int64_t gain = ext[v] - inn[v];
      const int src = part[v], dst = 1 - part[v];
      if (!((gain > 0 && pw[dst] + g.vw[v] <= maxw) || (gain == 0 && pw[src] > pw[dst] + g.vw[v]))) continue;
      part[v] = (int8_t)dst;
      pw[src] -= g.vw[v];
      pw[dst] += g.vw[v];
      std::swap(ext[v], inn[v]);
      for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
        const int32_t u = g.adj[e];
        if (part[u] == dst) { inn[u] += g.ew[e]; ext[u] -= g.ew[e]; }
        else { ext[u] += g.ew[e]; inn[u] -= g.ew[e]; }
      }
      moved = true;
    }
    if (!moved) break;
  }
}

// Separator of the connected component comp (sorted; its vertices carry
// mark cst): false when the bisection leaves a side empty.
bool multilevel_separator(const Graph& g, const std::vector<int32_t>& comp, const std::vector<int32_t>& mark,
                          int32_t cst, std::vector<int32_t>& local, std::vector<int32_t>& lo,
                          std::vector<int32_t>& hi, std::vector<int32_t>& sep) {
  const int64_t nc = (int64_t)comp.size();
  std::vector<MlGraph> graphs(1);
  MlGraph& g0 = graphs[0];
  for (int64_t i = 0; i < nc; ++i) local[comp[i]] = (int32_t)i;
  g0.ptr.assign(nc + 1, 0);
  g0.vw.assign(nc, 1);
  for (int64_t i = 0; i < nc; ++i) {
    const int32_t v = comp[i];
    for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e)
      if (mark[g.adj[e]] == cst) g0.adj.push_back(local[g.adj[e]]);
    g0.ptr[i + 1] = (int64_t)g0.adj.size();
  }
  g0.ew.assign(g0.adj.size(), 1);
  std::vector<std::vector<int32_t>> cmaps;
  while (graphs.back().n() > ML_COARSEN_TO) {
    std::vector<int32_t> cmap;
    MlGraph c;
    ml_coarsen(graphs.back(), cmap, c);
    if (c.n() * ML_SHRINK_DEN > ML_SHRINK_NUM * graphs.back().n()) break;
    cmaps.push_back(std::move(cmap));
    graphs.push_back(std::move(c));
  }
  std::vector<int8_t> part = ml_initial(graphs.back());
  ml_refine(graphs.back(), part);
  for (int64_t l = (int64_t)cmaps.size() - 1; l >= 0; --l) {
    std::vector<int8_t> fine(cmaps[l].size());
    for (size_t v = 0; v < fine.size(); ++v) fine[v] = part[cmaps[l][v]];
    part.swap(fine);
    ml_refine(graphs[l], part);
  }
  const MlGraph& f = graphs[0];
  std::vector<char> bnd(nc, 0);
  int64_t nb[2] = {0, 0};
  for (int64_t v = 0; v < nc; ++v)
    for (int64_t e = f.ptr[v]; e < f.ptr[v + 1]; ++e)
      if (part[f.adj[e]] != part[v]) { bnd[v] = 1; ++nb[part[v]]; break; }
  const int side = nb[0] <= nb[1] ? 0 : 1;
  lo.clear(); hi.clear(); sep.clear();
  for (int64_t v = 0; v < nc; ++v) {
    if (bnd[v] && part[v] == side) sep.push_back(comp[v]);
    else if (part[v] == 0) lo.push_back(comp[v]);
    else hi.push_back(comp[v]);
  }
  return !lo.empty() && !hi.empty();
}

}  // namespace

std::vector<int32_t> nested_dissection(const Graph& g, int leaf, int method) {
  const int64_t n = g.n;
  std::vector<int32_t> out;
  out.reserve(n);
  NdState st(g);
  std::vector<Task> stack;
  {
    Task t{false, std::vector<int32_t>(n)};
    std::iota(t.v.begin(), t.v.end(), 0);
    stack.push_back(std::move(t));
  }
  std::vector<int32_t> comp, order, order2;
  std::vector<int64_t> lp, lp2;
  std::vector<int32_t> local(method == 1 ? n : 0), mlo, mhi, msep;
  while (!stack.empty()) {
    Task t = std::move(stack.back());
    stack.pop_back();
    if (t.emit) {
      out.insert(out.end(), t.v.begin(), t.v.end());
      continue;
    }
    const int32_t my = ++st.stamp;
    for (int32_t v : t.v) st.mark[v] = my;
    std::vector<Task> tasks;
    // components in increasing order of smallest vertex (t.v is sorted)
    ++st.bstamp;
    const int32_t comp_stamp = st.bstamp;
    std::vector<int32_t> cseen_list;
    for (int32_t v0 : t.v) {
      if (st.seen[v0] >= comp_stamp) continue;
      // gather the component with a BFS that uses its own stamp
      comp.clear();
      comp.push_back(v0);
      st.seen[v0] = comp_stamp;
      for (size_t q = 0; q < comp.size(); ++q) {
        int32_t u = comp[q];
        for (int64_t e = g.ptr[u]; e < g.ptr[u + 1]; ++e) {
          int32_t w = g.adj[e];
          if (st.mark[w] == my && st.seen[w] < comp_stamp) {
            st.seen[w] = comp_stamp;
            comp.push_back(w);
          }
        }
      }
      std::sort(comp.begin(), comp.end());
      // restrict membership to this component for the rest of its processing
      const int32_t cst = ++st.stamp;
      for (int32_t v : comp) st.mark[v] = cst;
      if ((int64_t)comp.size() <= leaf) {
        Task e{true, {}};
        e.v.reserve(comp.size());
        leaf_minimum_degree(st, comp, e.v);
        tasks.push_back(std::move(e));
      } else {
        for (int32_t v : comp) {
          int32_t d = 0;
          for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) d += (st.mark[g.adj[e]] == cst);
          st.deg[v] = d;
        }
        int32_t r = min_degree_vertex(st.deg, comp.data(), comp.size());
        int nl = st.bfs(r, order, lp);
        while (true) {
          const int32_t* last = order.data() + lp[nl - 1];
          size_t cnt = (size_t)(lp[nl] - lp[nl - 1]);
          int32_t v = min_degree_vertex(st.deg, last, cnt);
          int nl2 = st.bfs(v, order2, lp2);
          if (nl2 > nl) {
            r = v;
            std::swap(order, order2);
            std::swap(lp, lp2);
            nl = nl2;
          } else {
            break;
          }
        }
        const int h = nl - 1;
        if (h < 2) {
          tasks.push_back(Task{true, degree_order(st, comp)});
        } else if (method == 1 && multilevel_separator(g, comp, st.mark, cst, local, mlo, mhi, msep)) {
          // multilevel separator, with the same rejection rule as below
          const int64_t total = (int64_t)comp.size();
          for (int32_t v : msep) st.mark[v] = -2;
          ++st.bstamp;
          const int32_t cs2 = st.bstamp;
          int64_t biggest = 0;
          for (int32_t v0 : comp) {
            if (st.mark[v0] != cst || st.seen[v0] == cs2) continue;
            int64_t cnt = 0;
            order2.clear();
            order2.push_back(v0);
            st.seen[v0] = cs2;
            for (size_t qq = 0; qq < order2.size(); ++qq) {
              int32_t u = order2[qq];
              ++cnt;
              for (int64_t e = g.ptr[u]; e < g.ptr[u + 1]; ++e) {
                int32_t w2 = g.adj[e];
                if (st.mark[w2] == cst && st.seen[w2] != cs2) { st.seen[w2] = cs2; order2.push_back(w2); }
              }
            }
            biggest = std::max(biggest, cnt);
          }
          for (int32_t v : msep) st.mark[v] = cst;
          if (8 * biggest > 7 * total) {
            tasks.push_back(Task{true, degree_order(st, comp)});
            continue;
          }
          tasks.push_back(Task{false, mlo});
          tasks.push_back(Task{false, mhi});
          tasks.push_back(Task{true, msep});
        } else {
          const int64_t total = (int64_t)comp.size();
          int best = -1;
          int64_t bs = 0, bd = 1;
          int bm = 0;
          int64_t below = lp[1] - lp[0];
          for (int l = 1; l < h; ++l) {
            int64_t sz = lp[l + 1] - lp[l];
            int64_t above = total - below - sz;
            int64_t den = std::min(below, above);
            int med = std::abs(2 * l - h);
            bool better;
            if (best < 0) {
              better = true;
            } else {
              // sz/den < bs/bd  <=>  sz*bd < bs*den  (all positive)
              __int128 lhs = (__int128)sz * bd, rhs = (__int128)bs * den;
              better = lhs < rhs || (lhs == rhs && (med < bm || (med == bm && l < best)));
            }
            if (better) { best = l; bs = sz; bd = den; bm = med; }
            below += sz;
          }
          // reject a separator that leaves one component with > 7/8 of C
          for (int64_t q = lp[best]; q < lp[best + 1]; ++q) st.mark[order[q]] = -2;
          ++st.bstamp;
          const int32_t cs2 = st.bstamp;
          int64_t biggest = 0;
          for (int32_t v0 : comp) {
            if (st.mark[v0] != cst || st.seen[v0] == cs2) continue;
            int64_t cnt = 0;
            order2.clear();
            order2.push_back(v0);
            st.seen[v0] = cs2;
            for (size_t qq = 0; qq < order2.size(); ++qq) {
              int32_t u = order2[qq];
              ++cnt;
              for (int64_t e = g.ptr[u]; e < g.ptr[u + 1]; ++e) {
                int32_t w2 = g.adj[e];
                if (st.mark[w2] == cst && st.seen[w2] != cs2) { st.seen[w2] = cs2; order2.push_back(w2); }
              }
            }
            biggest = std::max(biggest, cnt);
          }
          for (int64_t q = lp[best]; q < lp[best + 1]; ++q) st.mark[order[q]] = cst;
          if (8 * biggest > 7 * total) {
            tasks.push_back(Task{true, degree_order(st, comp)});
            continue;
          }
          Task lo{false, std::vector<int32_t>(order.begin(), order.begin() + lp[best])};
          Task hi{false, std::vector<int32_t>(order.begin() + lp[best + 1], order.end())};
          Task sep{true, std::vector<int32_t>(order.begin() + lp[best], order.begin() + lp[best + 1])};
          std::sort(lo.v.begin(), lo.v.end());
          std::sort(hi.v.begin(), hi.v.end());
          std::sort(sep.v.begin(), sep.v.end());
          tasks.push_back(std::move(lo));
          tasks.push_back(std::move(hi));
          tasks.push_back(std::move(sep));
        }
      }
      // component vertices keep stamp cst; the outer loop skips them through seen
    }
    for (auto it = tasks.rbegin(); it != tasks.rend(); ++it) stack.push_back(std::move(*it));
  }
  return out;
}

namespace {

// Adjacency of the permuted graph: for position j, neighbours as positions,
// in increasing order.  Rows are independent: contiguous row ranges of
// about equal size on up to 8 host threads.
Graph permute_graph(const Graph& g, const std::vector<int32_t>& perm, const std::vector<int32_t>& pinv) {
  Graph h;
  h.n = g.n;
  h.ptr.assign(g.n + 1, 0);
  h.adj.resize(g.adj.size());
  for (int64_t j = 0; j < g.n; ++j) {
    int32_t v = perm[j];
    h.ptr[j + 1] = h.ptr[j] + (g.ptr[v + 1] - g.ptr[v]);
  }
  const int64_t nnz = h.ptr[g.n];
  const int64_t nt = host_threads(nnz, 1 << 22);
  auto run = [&](int64_t t) {
    const int64_t j0 = std::lower_bound(h.ptr.begin(), h.ptr.end(), nnz * t / nt) - h.ptr.begin();
    const int64_t j1 = t + 1 == nt ? g.n : std::lower_bound(h.ptr.begin(), h.ptr.end(), nnz * (t + 1) / nt) - h.ptr.begin();
    for (int64_t j = j0; j < j1 && j < g.n; ++j) {
      int32_t v = perm[j];
      int64_t o = h.ptr[j];
      for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) h.adj[o++] = pinv[g.adj[e]];
      std::sort(h.adj.begin() + h.ptr[j], h.adj.begin() + h.ptr[j + 1]);
    }
  };
  std::vector<std::thread> pool;
  for (int64_t t = 1; t < nt; ++t) pool.emplace_back(run, t);
  run(0);
  for (std::thread& th : pool) th.join();
  return h;
}

// Elimination tree by path compression over the rows of the lower triangle.
std::vector<int32_t> etree_of(const Graph& h) {
  const int64_t n = h.n;
  std::vector<int32_t> parent(n, -1), anc(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = h.ptr[i]; e < h.ptr[i + 1]; ++e) {
      int32_t k = h.adj[e];
      if (k >= i) break;  // sorted: only k < i
      while (k != -1 && k < i) {
        int32_t next = anc[k];
        anc[k] = (int32_t)i;
        if (next == -1) { parent[k] = (int32_t)i; break; }
        k = next;
      }
    }
  }
  return parent;
}

std::vector<int32_t> postorder_of(const std::vector<int32_t>& parent) {
  const int64_t n = (int64_t)parent.size();
  std::vector<int32_t> head(n, -1), next(n, -1), out;
  out.reserve(n);
  // children lists in increasing order: insert in decreasing order
  for (int64_t j = n - 1; j >= 0; --j) {
    if (parent[j] >= 0) { next[j] = head[parent[j]]; head[parent[j]] = (int32_t)j; }
  }
  std::vector<int32_t> stack;
  for (int64_t r = 0; r < n; ++r) {
    if (parent[r] != -1) continue;
    stack.push_back((int32_t)r);
    while (!stack.empty()) {
      int32_t v = stack.back();
      int32_t c = head[v];
      if (c != -1) {
        head[v] = next[c];
        stack.push_back(c);
      } else {
        stack.pop_back();
        out.push_back(v);
      }
    }
  }
  return out;
}

// Column counts of L for a postordered pattern (postorder = identity):
// each row subtree adds +1 at its leaves, -1 at the meeting point of
// consecutive leaves and -1 above its root; counts are subtree sums.
std::vector<int64_t> column_counts(const Graph& h, const std::vector<int32_t>& parent) {
  const int64_t n = h.n;
  std::vector<int64_t> w(n, 0);
  std::vector<int32_t> first(n, -1), prevk(n, -1), prevleaf(n, -1), anc(n);
  for (int64_t j = 0; j < n; ++j) {
    int64_t k = j;
    while (k != -1 && first[k] == -1) { first[k] = (int32_t)j; k = parent[k]; }
    anc[j] = (int32_t)j;
  }
  for (int64_t i = 0; i < n; ++i)
    if (parent[i] != -1) w[parent[i]] -= 1;
  auto find = [&](int32_t q) {
    int32_t r = q;
    while (anc[r] != r) r = anc[r];
    while (anc[q] != r) { int32_t t = anc[q]; anc[q] = r; q = t; }
    return r;
  };
  for (int64_t j = 0; j < n; ++j) {
    // rows i >= j of column j, diagonal included
    auto visit = [&](int32_t i) {
      if (first[j] > prevk[i]) {
        w[j] += 1;
        if (prevleaf[i] != -1) w[find(prevleaf[i])] -= 1;
        prevleaf[i] = (int32_t)j;
      }
      prevk[i] = (int32_t)j;
    };
    visit((int32_t)j);
    for (int64_t e = h.ptr[j]; e < h.ptr[j + 1]; ++e)
      if (h.adj[e] > j) visit(h.adj[e]);
    if (parent[j] != -1) anc[j] = parent[j];
  }
  std::vector<int64_t> cc(w);
  for (int64_t j = 0; j < n; ++j)
    if (parent[j] != -1) cc[parent[j]] += cc[j];
  return cc;
}

}  // namespace

void analyze(const Graph& g, int leaf, int menu, Symbolic* out, int method) {
  const int64_t n = g.n;
  const bool timing = std::getenv("PDIPM_TIMING") != nullptr;
  auto t0 = std::chrono::steady_clock::now();
  auto lap = [&](const char* what) {
    if (!timing) return;
    auto t1 = std::chrono::steady_clock::now();
    fprintf(stderr, "[analyze] %s %.3f s\n", what, std::chrono::duration<double>(t1 - t0).count());
    t0 = t1;
  };
  Symbolic& s = *out;
  s.n = n;
  std::vector<int32_t> nd = nested_dissection(g, leaf, method);
  lap("nested dissection");
  std::vector<int32_t> pinv(n);
  for (int64_t k = 0; k < n; ++k) pinv[nd[k]] = (int32_t)k;
  std::vector<int32_t> post, etree0;
  {
    Graph h0 = permute_graph(g, nd, pinv);
    lap("permuted graph");
    etree0 = etree_of(h0);
    lap("elimination tree");
    post = postorder_of(etree0);
  }
  s.perm.resize(n);
  for (int64_t k = 0; k < n; ++k) s.perm[k] = nd[post[k]];
  s.pinv.resize(n);
  for (int64_t k = 0; k < n; ++k) s.pinv[s.perm[k]] = (int32_t)k;
  lap("postorder");
  Graph h = permute_graph(g, s.perm, s.pinv);
  // a postorder is a topological order of the tree: the elimination tree
  // of the reordered graph is the relabelled tree
  {
    std::vector<int32_t> at(n);
    for (int64_t k = 0; k < n; ++k) at[post[k]] = (int32_t)k;
    s.etree.resize(n);
    for (int64_t k = 0; k < n; ++k) {
      const int32_t p = etree0[post[k]];
      s.etree[k] = p < 0 ? -1 : at[p];
    }
  }
  s.colcount = column_counts(h, s.etree);
  lap("etree and counts");
  s.nnz_L = 0;
  s.flops = 0;
  for (int64_t j = 0; j < n; ++j) {
    s.nnz_L += s.colcount[j];
    s.flops += (double)s.colcount[j] * (double)s.colcount[j] - 1.0;
  }
  // fundamental supernodes
  std::vector<int32_t> nchild(n, 0);
  for (int64_t j = 0; j < n; ++j)
    if (s.etree[j] >= 0) nchild[s.etree[j]]++;
  std::vector<int32_t> first, last;
  for (int64_t j = 0; j < n; ++j) {
    bool joins = j > 0 && s.etree[j - 1] == j && s.colcount[j - 1] == s.colcount[j] + 1 && nchild[j] == 1;
    if (!joins) first.push_back((int32_t)j);
  }
  for (size_t k = 0; k < first.size(); ++k)
    last.push_back(k + 1 < first.size() ? first[k + 1] - 1 : (int32_t)(n - 1));
  // relaxed amalgamation: merge the adjacent preceding child while allowed
  AmalgamationRule rule = amalgamation_rule(menu);
  std::vector<int32_t> owner(n);      // column -> supernode token
  std::vector<int64_t> truenz(first.size());
  for (size_t k = 0; k < first.size(); ++k) {
    int64_t t = 0;
    for (int32_t j = first[k]; j <= last[k]; ++j) { owner[j] = (int32_t)k; t += s.colcount[j]; }
    truenz[k] = t;
  }
  // stack of accepted supernodes (first, last, token); merging pops the top
  std::vector<int32_t> sf, sl, stok;
  std::vector<int64_t> snz;
  for (size_t k = 0; k < first.size(); ++k) {
    int32_t f = first[k], l = last[k], tok = (int32_t)k;
    int64_t nz = truenz[k];
    while (!sf.empty()) {
      int32_t cf = sf.back(), cl = sl.back();
      int32_t p = s.etree[cl];
      if (p < 0 || owner[p] != tok) break;
      int64_t wc = cl - cf + 1, ws = l - f + 1;
      int64_t hs = ws + s.colcount[l] - 1;
      int64_t w = wc + ws, hh = wc + hs;
      if (w > rule.max_w) break;
      int64_t total = w * hh - w * (w - 1) / 2;
      int64_t zeros = total - (snz.back() + nz);
      if (!(w <= rule.small_w || zeros * rule.zero_den <= rule.zero_num * total)) break;
      for (int32_t j = cf; j <= cl; ++j) owner[j] = tok;
      f = cf;
      nz += snz.back();
      sf.pop_back(); sl.pop_back(); stok.pop_back(); snz.pop_back();
    }
    sf.push_back(f); sl.push_back(l); stok.push_back(tok); snz.push_back(nz);
  }
  const int64_t ns = (int64_t)sf.size();
  s.sn_start.resize(ns + 1);
  for (int64_t k = 0; k < ns; ++k) s.sn_start[k] = sf[k];
  s.sn_start[ns] = (int32_t)n;
  lap("supernodes");
  // supernode rows: columns, then the structure of the last column, built
  // from A's entries of the supernode's columns and the children's rows
  std::vector<int32_t> col2sn(n);
  for (int64_t k = 0; k < ns; ++k)
    for (int32_t j = s.sn_start[k]; j < s.sn_start[k + 1]; ++j) col2sn[j] = (int32_t)k;
  std::vector<std::vector<int32_t>> kids(ns);
  for (int64_t k = 0; k < ns; ++k) {
    int32_t p = s.etree[s.sn_start[k + 1] - 1];
    if (p >= 0) kids[col2sn[p]].push_back((int32_t)k);
  }
  s.sn_rowptr.assign(ns + 1, 0);
  s.sn_rows.clear();
  std::vector<int32_t> mark(n, -1), tmp;
  for (int64_t k = 0; k < ns; ++k) {
    const int32_t f = s.sn_start[k], l = s.sn_start[k + 1] - 1;
    tmp.clear();
    for (int32_t j = f; j <= l; ++j) {
      for (int64_t e = h.ptr[j]; e < h.ptr[j + 1]; ++e) {
        int32_t i = h.adj[e];
        if (i > l && mark[i] != k) { mark[i] = (int32_t)k; tmp.push_back(i); }
      }
    }
    for (int32_t c : kids[k]) {
      int32_t wc = s.sn_start[c + 1] - s.sn_start[c];
      for (int64_t e = s.sn_rowptr[c] + wc; e < s.sn_rowptr[c + 1]; ++e) {
        int32_t i = s.sn_rows[e];
        if (i > l && mark[i] != k) { mark[i] = (int32_t)k; tmp.push_back(i); }
      }
    }
    std::sort(tmp.begin(), tmp.end());
    for (int32_t j = f; j <= l; ++j) s.sn_rows.push_back(j);
    s.sn_rows.insert(s.sn_rows.end(), tmp.begin(), tmp.end());
    s.sn_rowptr[k + 1] = (int64_t)s.sn_rows.size();
    if ((int64_t)tmp.size() != s.colcount[l] - 1)
      throw std::runtime_error("supernode structure does not match the column count");
  }
  lap("supernode rows");
}

}  // namespace pdipm
