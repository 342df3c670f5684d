// Host-side structures: problem data on fixed patterns, the K pattern with
// its assembly map, and the numeric plan of the supernodal factorisation.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "pdipm.h"
#include "symbolic.hpp"

namespace pdipm {

enum Kind { KIND_LP = 0, KIND_QP = 1, KIND_NLP = 2 };

// Problem (1) with bounds, stored on the patterns the derivative kernels use.
struct HostProblem {
  int64_t n = 0, m = 0;
  int kind = KIND_LP;
  std::vector<double> c, b, q4, xl, xu;  // q4 empty when absent; bounds +-inf
  bool has_q4 = false, has_w = false;
  bool convex = true;    // certified convex: W >= 0 and Q diagonally dominant
  // J = A - 2 W diag(x) on the union pattern of A and W (m x n, CSR)
  std::vector<int64_t> jp;
  std::vector<int32_t> jc;
  std::vector<double> ja, jw;
  // J transposed: for column j the rows k (ascending) and J entry indices
  std::vector<int64_t> jtp;
  std::vector<int32_t> jtr, jte;
  // H lower pattern (original numbering): Q's lower triangle plus the full
  // diagonal; hq = Q values (0 on added diagonal entries); hdiag[i] = index
  std::vector<int64_t> hp;
  std::vector<int32_t> hc;
  std::vector<double> hq;
  std::vector<int64_t> hdiag;
  // symmetric H pattern for products H v: column indices and source entry
  std::vector<int64_t> hsp;
  std::vector<int32_t> hsc, hss;
};

// Lower CSR pattern of K (original numbering) and the assembly map:
//   K(e) = H(kh[e]) + [row == col](Sigma_x + delta_p)
//        + sum_{t in tp[e]..tp[e+1]} Sigma_s[tk[t]] J[ta[t]] J[tb[t]]
struct KMap {
  int64_t n = 0;
  std::vector<int64_t> kp;
  std::vector<int32_t> kc, krow, kh;
  std::vector<int64_t> tp;
  std::vector<int32_t> tk, ta, tb;
  std::vector<int64_t> pos;  // element offset of the entry in the panels
};

// Largest front height factored by the one-workgroup small-front kernel.
constexpr int SMALL_H_MAX = 64;

// Square tile edge of the Schur-update / panel-solve GEMM kernels.  FP64
// 128 x 128 tiles ran the largest rank-512 updates up to 4% faster than
// 64 x 64 but the 4096-row ones 20% slower and wasted half of every tile of
// the 64-column panel solves and inner updates (the block-angular LP's
// solve took 4% longer), so FP64 keeps 64 x 64.
constexpr int GEMM_TILE_F32 = 128;
constexpr int GEMM_TILE_F64 = 64;

// Launch descriptors (offsets are element offsets in the named buffers).
struct GemmDesc {          // C (-)= A * B^T on an M x N block, K inner
  int64_t c_off, a_off, b_off;
  int32_t ldc, lda, ldb;
  int32_t M, N, K;
  int32_t c_buf;           // 0 panels, 1 update matrices
  int32_t b_buf;           // 0 panels, 1 inverse-diagonal scratch
  int32_t mode;            // 0 subtract (lower masked when lower=1), 1 set
  int32_t lower;
  int32_t tiles_m, tiles_n;
  int32_t kcol;            // permuted column of inner index 0 (mode 0) or of
                           // output column 0 (mode 1): the pivot signs of a
                           // signed (SQD) factorisation
  int64_t tile_begin;      // first tile of this descriptor in its launch
};

struct PotrfDesc {         // factor the bw x bw diagonal block, write inverse
  int64_t d_off;           // panel offset of the block's (0,0)
  int64_t inv_off;         // scratch offset of the inverse (ld = nb)
  int32_t ld, bw;
  int32_t col0;            // permuted column of the block's first column
  int32_t pad;
};

struct ExtAddDesc {        // parent front, target front columns [t0, t1)
  int32_t sn, t0, t1, pad;
};

// Column-block width of the blocked triangular solves, both precisions.
// FP64 factorisations block by 64 columns; their solve inverses are formed
// from pairs of 64 x 64 inverses after the factorisation:
//   inv([L11 0; L21 L22]) = [X1 0; -X2 L21 X1  X2],  X1 = inv(L11), X2 = inv(L22).
constexpr int SOLVE_NB = 128;
// Front rows per forward gather item (one per thread of its workgroup).
constexpr int GATHER_ROWS = 256;

struct InvCombDesc {       // one SOLVE_NB x SOLVE_NB solve inverse from two nb x nb ones
  int64_t x1_off, x2_off;  // inverse-scratch offsets of X1 and X2 (x2_off < 0: bw <= nb)
  int64_t l21_off;         // panel offset of L21 (rows c0 + nb .., columns c0 ..)
  int64_t out_off;         // inverse-scratch offset of the result (ld SOLVE_NB)
  int32_t ld, bw;          // panel leading dimension; columns of the block (<= SOLVE_NB)
};

// Blocked triangular-solve work item of supernode sn and column block
// [c0, c0 + bw) over rows [r0, r1) below the block.  Forward: the owner
// item also forms y of the next block.  Backward: partial products go to
// part[part_off ..]; a diagonal item sums its nparts partials and solves.
// The supernode's own fields are copied in, so that a solve kernel reaches
// its data after one dependent load (the descriptor) instead of two.
struct SolveDesc {
  int32_t sn, c0, bw, r0, r1, owner;
  int64_t part_off;
  int32_t nparts, w;       // w: supernode width
  int64_t panel_off;       // panel offset of the supernode
  int64_t uvec_off;        // its update-vector offset
  int64_t inv_off;         // its diagonal-block inverses
  int64_t row_off;         // its row list
  int32_t first, ld;       // first column, panel leading dimension
};

// Forward solve: rows [r0, r1) of the front of large supernode sn collect
// their children's update-vector entries.
struct GatherItem {
  int32_t sn, r0, r1, pad;
};

enum OpType {
  OP_EXTEND_ADD = 0, OP_SMALL, OP_POTRF, OP_TRSM, OP_UPDATE,   // factorisation
  OP_INV_COMBINE,                                                // solve inverses (FP64)
  OP_FWD_SMALL, OP_FWD_GATHER, OP_FWD_FIRST, OP_FWD_STEP,        // forward solve
  OP_BWD_SMALL, OP_BWD_PART, OP_BWD_DIAG                         // backward solve
};

struct Op {
  int type;
  int64_t begin, end;      // descriptor range in the pool of its type
  int64_t grid;            // workgroups
};

struct Plan {
  int64_t ns = 0, n = 0;
  int nb = 64;             // panel block width of the blocked path
  int small_h = 64;        // fronts with h <= small_h use the one-workgroup path
  int esize = 8;           // bytes per panel element (8 FP64, 4 FP32)
  std::vector<int32_t> sfirst, sw, sh, sld, sparent, slevel;  // sld: panel leading dim (h rounded up to 4)
  std::vector<int32_t> sldu;          // update-matrix leading dim (h - w, rounded up to 32 above 64)
  std::vector<int64_t> spanel, su, srow, suv;  // panel / U / row / update-vector offsets
  std::vector<int32_t> child_ptr, child;
  std::vector<int32_t> rel;           // parallel to sn_rows: row position in the parent
  int nlevels = 0;
  std::vector<int32_t> level_ptr, level_sn;  // supernodes by level
  int64_t panel_elems = 0, u_elems = 0, uv_elems = 0;
  int64_t inv_elems = 0;              // inverse-diagonal scratch
  int64_t max_front = 0;
  std::vector<Op> ops;
  std::vector<GemmDesc> gemm;
  std::vector<PotrfDesc> potrf;
  std::vector<ExtAddDesc> ext;
  std::vector<int32_t> small;
  double update_bytes = 0;
  // permanent inverses of the SOLVE_NB-column diagonal blocks of large
  // supernodes (the triangular solves' blocks; -1 for small supernodes)
  std::vector<int64_t> sinv;
  std::vector<InvCombDesc> icomb;     // FP64: their formation from 64-column inverses
  // triangular solves
  std::vector<Op> fwd_ops, bwd_ops;
  std::vector<SolveDesc> sdesc;
  std::vector<int32_t> ssmall, slarge; // supernode lists used by the solve ops
  // forward gather of large supernodes: per front row, the update-vector
  // offsets of the children's entries for that row in child order (rows of
  // supernode k at gptr[grow[k] ..], -1 for small supernodes)
  std::vector<GatherItem> gitem;
  std::vector<int64_t> grow, gptr, gidx;
  int64_t part_elems = 1;              // backward partial sums (max per step)
  // algorithmic work of the Schur-update / panel-solve GEMM launches of one
  // factorisation (useful multiply-add flops, triangles not double counted)
  double gemm_flops = 0;
  double gemm_bytes = 0;   // operand blocks read once, C read and written once
  int64_t gemm_launches = 0;
};

std::string build_problem(const ::ipm_problem_desc* d, HostProblem* p);
void build_graph_from_problem(const HostProblem& p, Graph* g);
void build_graph_from_lower(int64_t n, const int64_t* rp, const int32_t* ci, Graph* g);
void build_kmap_problem(const HostProblem& p, KMap* km);
void build_kmap_lower(int64_t n, const int64_t* rp, const int32_t* ci, KMap* km);
// Graph and assembly map of the dual condensed matrix M = diag + J D J'
// (m x m; Section 3, eq. kkt_dual): M(e) = [row == col] E_row
// + sum_t D[tk[t]] J[ta[t]] J[tb[t]], tk a column of J, ta/tb J entries.
void build_dual_structures(const HostProblem& p, Graph* g, KMap* km);
// Graph and assembly map of the augmented SQD matrix (Section 3, eq.
// augmentedKKT) of order n + m, x block first:
//   [ H + diag(Sigma_x + delta_p)   J'           ]
//   [ J                             -1 / Sigma_s ]
// x rows: kh = H entry; lambda rows: kh = J entry, -1 on the diagonal.
void build_augmented_structures(const HostProblem& p, Graph* g, KMap* km);
// Blocking of the numeric plan: fronts of height <= small_h (at most 64) use
// the one-workgroup LDS kernel; larger fronts take rank-(outer_blocks * nb)
// trailing updates.
struct Blocking {
  int small_h = 64;
  int outer_blocks = 0;  // 0: the precision's default (8 FP64, 4 FP32)
};
// Useful flops of one GEMM descriptor (lower-masked blocks count only the
// entries on or below the diagonal; the panel solve counts M K^2).
double gemm_desc_flops(const GemmDesc& g);
void build_plan(const Symbolic& s, int precision_bytes, Plan* plan, const Blocking& blk = Blocking());
void map_k_to_panels(const Symbolic& s, const Plan& plan, KMap* km);

}  // namespace pdipm
