// Host planner: cluster tree, block tree, host assembly, device layout and
// the static schedules of factorisation, solve and matvec.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "ops.h"

namespace hlu {

struct Params {
  int kernel = 0;          // 0 weighted, 1 point
  double eta = 2.0;
  int leaf = 32;
  int fixed_rank = 0;
  double eps_f = 1e-6;
  int cap_f = 32;
  double eps_mv = 1e-12;
  int cap_mv = 64;
  int mixed = 0;
  double refine_tol = 0.0;
  int refine_max_iter = 10;
  int max_nrhs = 32;
  uint64_t scratch_cap = 0;   // 0: no reuse of H-GEMM temporaries
  int device_asm = 0;         // 1: blocks built on the device (hlu_assemble)
  // 0: H-LU of the kernel matrix.  1 and 2: a doubled matrix on two copies
  // of the points, M = [M11 M12; M21 M22] with every quadrant on the
  // original block tree; 1 (product): M12 = A, M21 = B (kernel_b), M11 =
  // M22 = 0, schedule M11 -= M12 M21, so M11 = -A B; 2 (inverse): M11 = A,
  // M12 = M21 = I, M22 = 0, schedule LU(M11), M12 := L^-1 P M12,
  // M21 := M21 U^-1, M22 -= M21 M12, so M22 = -A^-1.
  int operation = 0;
  int kernel_b = 0;
};

// Device assembly of the low-rank blocks in chunks that share one ACA
// workspace: blocks [b0, b1) of the low-rank table, their recompression ops
// [op0, op1) of asm_ops.
struct AsmChunk {
  int b0, b1, op0, op1;
};

struct Cluster {
  int off = 0, size = 0;
  double lo[3], hi[3];
  int son[2] = {-1, -1};
  int leaf = -1;           // leaf index if a leaf
  int first_leaf = 0, nleaves = 0;
};

struct BNode {
  int t, s;
  char kind;               // 'F', 'R', 'H'
  int son[4] = {-1, -1, -1, -1};
  int blk = -1;            // leaf block index (F or R)
};

struct LBlock {
  int t, s;
  char kind;
  int m, n;
  uint64_t offF = 0;       // dense (FP64, ld m)
  uint64_t offU = 0, offV = 0, offRank = 0;   // factor copy (capacity cap_f)
  uint64_t offT = 0;       // solve: V^T X of this block (cap_f x max_nrhs, FP64)
  int objF = -1, objU = -1, objV = -1, objRank = -1;
  // matvec copy
  uint64_t mvU = 0, mvV = 0;
  int mvk = 0;
  int kf = 0;              // assembled rank of the factor copy
};

struct Batch {
  int wave, type, start, count;
  uint32_t mask;           // op types present (bit per type)
};

struct Schedule {
  std::vector<Op> ops;     // sorted by (wave, type); pointers are byte offsets
  std::vector<Batch> batches;      // one per (wave, type)
  std::vector<Batch> waves_list;   // one per wave (all types)
  std::vector<Term> terms;         // term table of the truncation / row-update ops
  int waves = 0;
  // dependency graph in schedule order (for the dataflow executor):
  // successors of op i are succ[succ_off[i] .. succ_off[i+1]), indeg0[i]
  // its number of predecessors; ready0 lists the ops without any
  std::vector<int32_t> succ_off, succ, indeg0, ready0;
};

struct Plan {
  Params prm;
  int n = 0;
  std::vector<double> xyz, area;   // cluster order
  std::vector<int64_t> perm;       // perm[p] = original index
  std::vector<Cluster> cl;
  std::vector<int> leaves;         // cluster ids of leaves in order
  std::vector<BNode> bn;
  std::vector<LBlock> blk;
  int broot = 0;
  int n_orig = 0;                  // points per copy (n / 2 for doubled plans)
  int result_node = -1;            // block node of the result quadrant (operation 1, 2)

  // device layout (byte offsets from the bound base)
  uint64_t off_status = 0;         // int32 info, int32 flags, ...
  uint64_t off_work = 0, size_work = 0;      // ranks | dense | low-rank
  uint64_t off_pristine = 0;
  uint64_t off_piv = 0;
  // inverses of the diagonal leaves for the solve: the leaf at rows
  // [o, o + b) keeps L^{-1} P at off_inv_l + 512 o and U^{-1} at
  // off_inv_u + 512 o (b x b FP64, leading dimension b)
  uint64_t off_inv_l = 0, off_inv_u = 0;
  uint64_t off_mv = 0, size_mv = 0;
  uint64_t off_scratch = 0, size_scratch = 0;
  uint64_t off_cost = 0;           // per-op records of the factor schedule
  uint64_t off_cost_s = 0;         // per-op records of the solve schedule
  uint64_t off_ws = 0;             // solve / refinement workspace
  uint64_t off_nrhs = 0;           // int32 nrhs slot used by solve panels
  uint64_t off_Y = 0, off_X = 0, off_B = 0, off_eta = 0;
  uint64_t off_mvT = 0;
  uint64_t off_ops_f = 0, off_ops_s = 0, off_terms_f = 0, off_terms_s = 0;
  // dataflow executor state of the factor schedule
  uint64_t off_df_succ_off = 0, off_df_succ = 0, off_df_indeg0 = 0, off_df_indeg = 0,
           off_df_queue = 0, off_df_ready0 = 0, off_df_ctrl = 0;
  // the same arrays for the solve schedule
  uint64_t off_dfs_succ_off = 0, off_dfs_succ = 0, off_dfs_indeg0 = 0, off_dfs_indeg = 0,
           off_dfs_queue = 0, off_dfs_ready0 = 0, off_dfs_ctrl = 0;
  uint64_t off_mv_lr = 0, off_mv_terms = 0, off_mv_rows = 0, off_perm = 0;
  uint64_t total = 0;

  std::vector<char> img_work;      // host image of the work region
  std::vector<char> img_mv;        // host image of the matvec region

  Schedule fsched, ssched;
  std::vector<MvLR> mv_lr;
  std::vector<MvTerm> mv_terms;
  std::vector<MvRow> mv_rows;

  // points in cluster order on the device (x, y, z interleaved; then area)
  uint64_t off_pts = 0;
  // device assembly (prm.device_asm)
  std::vector<AsmBlock> asm_dense, asm_lr;   // offsets relative to the base
  std::vector<AsmChunk> asm_chunks;
  std::vector<Op> asm_ops;                   // recompression (OP_TRUNC), one per low-rank block
  std::vector<Term> asm_terms;
  uint64_t off_asm_dense = 0, off_asm_lr = 0, off_asm_ranks = 0, off_asm_ops = 0,
           off_asm_terms = 0, off_asm_ws = 0, size_asm_ws = 0;
  int asm_kmax = 64;
  double asm_eps = 0.0;                      // cross-approximation tolerance

  double anorm_inf = 0.0;          // max row sum of |A| (exact)
  double flops_model = 0.0;
  int64_t max_rank_f = 0;
  std::string err;
};

// Build everything on the host; returns false and sets p.err on failure.
bool build_plan(Plan& p, const double* xyz, const double* area, int64_t n,
                const Params& prm);

}  // namespace hlu
