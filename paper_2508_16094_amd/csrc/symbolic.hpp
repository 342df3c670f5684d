// Host-side symbolic analysis of the condensed KKT matrix.
//
// The factorisation P'KP = LL' uses a fill-reducing permutation computed
// once on the host and reused every iteration (Section 2: ordering is serial
// and amortised).  The ordering rule (nested dissection by BFS level
// structures, exact minimum degree on small components, postorder) and the
// supernode rule (fundamental supernodes plus relaxed amalgamation) are
// fixed so that an independent implementation reproduces them bit for bit.
#pragma once
#include <cstdint>
#include <vector>

namespace pdipm {

// Symmetric pattern without diagonal: CSR adjacency, sorted rows.
struct Graph {
  int64_t n = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> adj;
};

struct AmalgamationRule {
  int32_t max_w, small_w;
  int64_t zero_num, zero_den;  // explicit zeros <= num/den of the trapezoid
};
AmalgamationRule amalgamation_rule(int menu_index);

struct Symbolic {
  int64_t n = 0;
  std::vector<int32_t> perm;      // perm[k] = original index at position k
  std::vector<int32_t> pinv;      // pinv[orig] = position
  std::vector<int32_t> etree;     // parent in permuted numbering, -1 = root
  std::vector<int64_t> colcount;  // |column of L| incl. diagonal
  std::vector<int32_t> sn_start;  // nsuper + 1
  std::vector<int64_t> sn_rowptr; // nsuper + 1
  std::vector<int32_t> sn_rows;   // permuted row indices, own columns first
  int64_t nnz_L = 0;              // sum colcount
  double flops = 0;               // sum (c_j^2 - 1)
  int64_t nsuper() const { return (int64_t)sn_start.size() - 1; }
};

// Nested dissection order (before postordering).
// Host threads for a parallel setup loop of the given work: the value of
// PDIPM_HOST_THREADS when set (1 to 64, at any size; the results never
// depend on it), else up to 8 once the work reaches work_min.
int64_t host_threads(int64_t work, int64_t work_min);
// method 0: separators are BFS levels; 1: separators from multilevel
// bisection (heavy-edge coarsening, boundary refinement), the level rule
// where the bisection leaves a side empty.
std::vector<int32_t> nested_dissection(const Graph& g, int leaf, int method = 0);
// Full analysis: order, postorder, etree, column counts, supernodes.
void analyze(const Graph& g, int leaf, int menu, Symbolic* out, int method = 0);

}  // namespace pdipm
