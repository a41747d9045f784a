// C-ABI of the H-LU library: planning, binding, assembly upload, the
// wave-by-wave executor of the static schedules, solve with iterative
// refinement, matvec and the single-kernel test entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <memory>
#include <vector>

#include "../../include/hlu.h"
#include "plan.hpp"

extern "C" hipError_t hlu_launch_ops(int type, const void* ops, int count, hipStream_t s);
extern "C" hipError_t hlu_launch_mv(const void* lr, int nlr, const void* rows, int nrows,
                                    const void* terms, const double* X, int ldx, const double* B,
                                    double beta, double alpha, double* Y, int nrhs,
                                    hipStream_t s);
extern "C" hipError_t hlu_launch_vec(int what, const double* a, int64_t lda, double* y, int ldy,
                                     const int64_t* perm, int n, int nrhs, hipStream_t s);
extern "C" hipError_t hlu_launch_colmax(const double* R, const double* X, const double* B, int ld,
                                        int n, int nrhs, double* out, hipStream_t s);
extern "C" hipError_t hlu_launch_set_int(int32_t* p, int v, hipStream_t s);
extern "C" size_t hlu_static_scratch_bytes(void);
extern "C" hipError_t hlu_launch_asm(const void* dense, int ndense, const void* lr, int nlr,
                                     const double* pts, int npts, int kernel, double eps,
                                     int kmax, int32_t* caphits, hipStream_t s);
extern "C" hipError_t hlu_launch_direct_mv(const double* pts, int npts, int kernel,
                                           const double* X, int ld, const double* B, double beta,
                                           double alpha, double* Y, int nrhs, int absmode,
                                           hipStream_t s);
extern "C" hipError_t hlu_static_scratch(void** out);
extern "C" hipError_t hlu_launch_build_trunc(void* dst, const double* U, const double* V,
                                             int32_t* rank, const double* X, const double* Y, int m,
                                             int n, int kx, int w, int cap, double eps,
                                             int fixed_rank, hipStream_t s);
extern "C" hipError_t hlu_launch_keep_flag(const int32_t* src, int32_t* dst, hipStream_t s);
extern "C" hipError_t hlu_launch_axpy_masked(const double* d, double* x, int ld, int n, int nrhs,
                                             const int32_t* active, hipStream_t s);
extern "C" hipError_t hlu_launch_wave(const void* ops, int count, size_t lds, hipStream_t s);
extern "C" size_t hlu_lds_bytes(int type);
extern "C" hipError_t hlu_build_wave_graph(const void* ops_base, const int* starts,
                                           const int* counts, const size_t* lds, int nwaves,
                                           int32_t* status, hipGraphExec_t* out);
extern "C" hipError_t hlu_launch_dataflow(int kind, const void* parts, int np, int* queue,
                                          const int* ready0, int nready, int* ctrl, int n,
                                          int nhigh, int nhw, int workers, long long timeout,
                                          int32_t* status, hipStream_t s);
extern "C" hipError_t hlu_build_df_graph(int kind, const void* parts, int np, int* queue,
                                         const int* ready0, int nready, int* ctrl, int n,
                                         int nhigh, int nhw, int workers, long long timeout,
                                         int32_t* status, hipGraphExec_t* out);

namespace {

thread_local std::string g_err;

const char* df_error_text(int32_t e) {
  switch (e) {
    case 2: return "dataflow executor: queue overflow";
    case 3: return "dataflow executor: op type outside the executor's set";
    default: return "dataflow executor: a wait exceeded its time limit";
  }
}

hlu_status fail(hlu_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(HLU_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

void relocate(hlu::PRef& r, uint64_t base) {
  if (r.ptr && r.kind != hlu::PK_IDENT) r.ptr += base;
  if (r.rankp) r.rankp += base;
}

void relocate(hlu::Op& op, uint64_t base) {
  for (auto& r : op.p) relocate(r, base);
  if (op.cost) op.cost += base;
}

// Host-side check of a schedule before anything is launched: every panel a
// kernel may touch (at full capacity) lies inside the buffer, dynamic column
// counts point at an int inside the buffer, and operand shapes agree with
// what each kernel assumes.  Offsets are relative to the buffer start.
bool panel_ok(const hlu::PRef& r, uint64_t total, std::string& why, bool allow_ident = false) {
  if (r.kind == hlu::PK_IDENT) {
    // identity panels are implicit; only the dense update's operands and the
    // truncation's stacked terms evaluate them, every other body reads
    // stored panels only
    if (!allow_ident) { why = "identity panel outside a truncation term"; return false; }
    return r.rows >= 0 && r.cols >= 0;
  }
  if (r.kind != hlu::PK_MAT) { why = "unknown panel kind"; return false; }
  if (r.rows < 0 || r.cols < 0 || r.ld < 1) { why = "bad panel dims"; return false; }
  if (r.rows == 0 || r.cols == 0) return true;
  uint64_t es = r.dt == hlu::DT_F64 ? 8 : 4;
  uint64_t last = r.trans ? (uint64_t)(r.cols - 1) + (uint64_t)(r.rows - 1) * r.ld
                          : (uint64_t)(r.rows - 1) + (uint64_t)(r.cols - 1) * r.ld;
  if (!r.trans && r.ld < r.rows) { why = "ld < rows"; return false; }
  if (r.trans && r.ld < r.cols) { why = "ld < cols (transposed)"; return false; }
  if (r.ptr < 512 || r.ptr + (last + 1) * es > total) { why = "panel outside buffer"; return false; }
  if (r.rankp && (r.rankp < 256 || r.rankp + 4 > total)) { why = "rank pointer outside buffer"; return false; }
  return true;
}

bool validate(const hlu::Plan& p, const hlu::Schedule& sc, std::string& why) {
  const uint64_t T = p.total;
  for (size_t i = 0; i < sc.ops.size(); ++i) {
    const hlu::Op& o = sc.ops[i];
    auto bad = [&](const char* w) {
      why = "op " + std::to_string(i) + " (type " + std::to_string(o.type) + "): " + w;
      return false;
    };
    if (o.cost && o.cost + hlu::kCostRecBytes > T) return bad("cost record outside buffer");
    switch (o.type) {
      case hlu::OP_GETRF:
        if (!panel_ok(o.p[0], T, why)) return bad(why.c_str());
        if (o.p[0].rows != o.p[0].cols || o.p[0].rows < 1 || o.p[0].rows > 64) return bad("leaf size");
        if (o.p[1].ptr < 512 || o.p[1].ptr + 4 * o.p[0].rows > T) return bad("pivots");
        break;
      case hlu::OP_TRSM_L:
      case hlu::OP_TRSM_UT:
      case hlu::OP_TRSM_U:
        if (!panel_ok(o.p[0], T, why) || !panel_ok(o.p[1], T, why)) return bad(why.c_str());
        if (o.p[0].rows != o.p[0].cols || o.p[0].rows > 64 || o.p[1].rows != o.p[0].rows)
          return bad("leaf solve shapes");
        if (o.type == hlu::OP_TRSM_L && (o.p[2].ptr < 512 || o.p[2].ptr + 4 * o.p[0].rows > T))
          return bad("pivots");
        break;
      case hlu::OP_PGEMM: {
        const hlu::PRef &X = o.p[2], &Y = o.p[3];
        if (!panel_ok(X, T, why) || !panel_ok(Y, T, why)) return bad(why.c_str());
        bool tr = o.i1 != 0;
        if (o.i0 == 0) {
          const hlu::PRef& M = o.p[0];
          if (!panel_ok(M, T, why)) return bad(why.c_str());
          int mr = tr ? M.cols : M.rows, mc = tr ? M.rows : M.cols;
          if (mr != Y.rows || mc != X.rows) return bad("dense product shapes");
        } else {
          const hlu::PRef &U = o.p[0], &V = o.p[1];
          if (!panel_ok(U, T, why) || !panel_ok(V, T, why)) return bad(why.c_str());
          const hlu::PRef& A = tr ? V : U;
          const hlu::PRef& B = tr ? U : V;
          if (A.rows != Y.rows || B.rows != X.rows) return bad("low-rank product shapes");
          if (U.cols > 64 || !U.rankp) return bad("low-rank operand rank");
        }
        if (X.cols != Y.cols && !(X.rankp && X.rankp == Y.rankp)) {
          // static / dynamic mix: the kernel uses the smaller live count
          if (!X.rankp && !Y.rankp) return bad("panel column counts differ");
        }
        break;
      }
      case hlu::OP_TRUNC: {
        const hlu::PRef &U = o.p[0], &V = o.p[1];
        for (int q = 0; q < 2; ++q)
          if (!panel_ok(o.p[q], T, why)) return bad(why.c_str());
        int cap = o.i2 & 0xffff;
        if (!U.rankp || U.rankp != V.rankp || U.cols != cap || V.cols != cap || cap > 32)
          return bad("truncation target");
        if (o.i1 < 1 || o.i1 > 16 || o.i0 < 0 || (size_t)(o.i0 + o.i1) > sc.terms.size())
          return bad("truncation term list");
        if (o.p[2].ptr != p.off_terms_f) return bad("truncation term table");
        for (int t = o.i0; t < o.i0 + o.i1; ++t) {
          const hlu::Term& tm = sc.terms[t];
          if (!panel_ok(tm.X, T, why, true) || !panel_ok(tm.Y, T, why, true))
            return bad(why.c_str());
          if (tm.xo < 0 || tm.yo < 0 || tm.xo + tm.X.rows > U.rows || tm.yo + tm.Y.rows > V.rows)
            return bad("truncation term placement");
          if (tm.X.cols != tm.Y.cols) return bad("truncation term widths");
          if (cap + tm.X.cols > 64) return bad("term wider than the stack allows");
          if (tm.X.rankp != tm.Y.rankp) return bad("truncation term rank pointers differ");
        }
        break;
      }
      case hlu::OP_ADDD: {
        const hlu::PRef &Cm = o.p[0], &X = o.p[1], &Y = o.p[2];
        for (int q = 0; q < 3; ++q)
          if (!panel_ok(o.p[q], T, why, q > 0)) return bad(why.c_str());
        if (X.rows != Cm.rows || Y.rows != Cm.cols || X.cols != Y.cols) return bad("dense update shapes");
        if (Cm.dt != hlu::DT_F64 || Cm.trans || Cm.rankp) return bad("dense update target");
        break;
      }
      case hlu::OP_ZERO:
        if (!panel_ok(o.p[0], T, why) || o.p[0].rankp) return bad(why.c_str());
        break;
      case hlu::OP_TRINV: {
        const hlu::PRef &A = o.p[0], &W = o.p[2], &Ui = o.p[3];
        for (int q : {0, 2, 3})
          if (!panel_ok(o.p[q], T, why)) return bad(why.c_str());
        const int b = A.rows;
        if (A.cols != b || b < 1 || b > 64 || A.dt != hlu::DT_F64 || A.trans) return bad("leaf");
        for (const hlu::PRef* q : {&W, &Ui})
          if (q->rows != b || q->cols != b || q->ld != b || q->dt != hlu::DT_F64 || q->trans ||
              q->rankp)
            return bad("leaf inverse target");
        if (o.p[1].ptr < 512 || o.p[1].ptr + 4 * b > T) return bad("pivots");
        break;
      }
      case hlu::OP_INVAPPLY: {
        const hlu::PRef &W = o.p[0], &Y = o.p[1];
        if (!panel_ok(W, T, why) || !panel_ok(Y, T, why)) return bad(why.c_str());
        if (W.rows != W.cols || W.rows > 64 || W.dt != hlu::DT_F64 || W.trans || W.rankp)
          return bad("leaf inverse");
        if (Y.rows != W.rows || Y.dt != hlu::DT_F64 || Y.trans || Y.cols > 64)
          return bad("leaf inverse operand");
        break;
      }
      case hlu::OP_MVT: {
        const hlu::PRef &V = o.p[0], &X = o.p[2], &Tt = o.p[3];
        if (!panel_ok(V, T, why) || !panel_ok(X, T, why) || !panel_ok(Tt, T, why))
          return bad(why.c_str());
        if (V.cols > 64 || V.trans || X.rows != V.rows || X.cols > 64 || X.dt != hlu::DT_F64 ||
            X.trans)
          return bad("V^T X operands");
        if (Tt.dt != hlu::DT_F64 || Tt.trans || Tt.rankp || Tt.rows < V.cols || Tt.cols < X.cols)
          return bad("V^T X target");
        if (o.i2 != 0 && o.i2 != 1) return bad("V^T X accumulate flag");
        break;
      }
      case hlu::OP_MVROW: {
        const hlu::PRef& Y = o.p[3];
        if (!panel_ok(Y, T, why)) return bad(why.c_str());
        if (Y.rows > 64 || Y.cols > 64 || Y.dt != hlu::DT_F64 || Y.trans) return bad("row target");
        auto term_ok = [&](const hlu::PRef& X, const hlu::PRef& Yt) {
          if (!panel_ok(X, T, why) || !panel_ok(Yt, T, why)) return bad(why.c_str());
          if (X.rows != Y.rows || X.cols > 64 || X.trans) return bad("row term factor");
          if (Yt.dt != hlu::DT_F64 || Yt.trans || Yt.rows < X.cols || Yt.cols < Y.cols)
            return bad("row term operand");
          return true;
        };
        if (o.i0 == -1) {   // one term inline: factor in p1, operand in p2
          if (o.i1 != 1) return bad("inline row term count");
          if (!term_ok(o.p[1], o.p[2])) return false;
        } else {
          if (o.i1 < 1 || o.i1 > 256 || o.i0 < 0 || (size_t)o.i0 + o.i1 > sc.terms.size())
            return bad("row update term list");
          if (o.p[2].ptr != p.off_terms_s) return bad("row update term table");
          for (int t = o.i0; t < o.i0 + o.i1; ++t)
            if (!term_ok(sc.terms[t].X, sc.terms[t].Y)) return false;
        }
        if (o.i2 != 0 && o.i2 != 1) return bad("row update flag");
        if (o.i2 == 1) {   // fused leaf inverse in p0
          const hlu::PRef& W = o.p[0];
          if (!panel_ok(W, T, why)) return bad(why.c_str());
          if (W.rows != Y.rows || W.cols != Y.rows || W.dt != hlu::DT_F64 || W.trans || W.rankp)
            return bad("fused leaf inverse");
        }
        break;
      }
      default:
        return bad("unknown op type");
    }
  }
  return true;
}

}  // namespace

// Device offsets of one schedule's dataflow arrays.
// (the schedule's DfPart descriptor lives at ctrl + 64)
static_assert(HLU_OP_TYPES == hlu::OP_NTYPES, "op type count of the C-ABI");

struct DfArrays {
  const hlu::Schedule* sc;
  uint64_t ops, succ_off, succ, indeg0, indeg, queue, ready0, ctrl;
  uint64_t part() const { return ctrl + 64; }
};
static DfArrays df_factor(const hlu::Plan& p) {
  return {&p.fsched, p.off_ops_f, p.off_df_succ_off, p.off_df_succ, p.off_df_indeg0,
          p.off_df_indeg, p.off_df_queue, p.off_df_ready0, p.off_df_ctrl};
}
static DfArrays df_solve(const hlu::Plan& p) {
  return {&p.ssched, p.off_ops_s, p.off_dfs_succ_off, p.off_dfs_succ, p.off_dfs_indeg0,
          p.off_dfs_indeg, p.off_dfs_queue, p.off_dfs_ready0, p.off_dfs_ctrl};
}

struct hlu_handle_s {
  // The plan (schedules, layout, host images of the assembled data) is
  // immutable once built and shared by the clones of a handle.
  std::shared_ptr<hlu::Plan> shared;
  hlu::Plan& plan;
  explicit hlu_handle_s(std::shared_ptr<hlu::Plan> p) : shared(std::move(p)), plan(*shared) {}
  char* base = nullptr;
  size_t bytes = 0;
  bool assembled = false;
  bool factored = false;
  double anorm = 0.0;
  int iters = 0;
  double eta_hist[16] = {0};
  double eta_final = 0.0;
  bool not_converged = false;
  int32_t asm_cap_hits = 0;           // cross approximations stopped at their rank limit
  double refine_tol = 0.0;            // refinement target of hlu_solve (0: none)
  int refine_max_iter = 0;
  hlu_params params;
  bool use_graph = true;
  int executor = 0;                   // 0: waves, 1: dataflow
  int workers = 0;                    // dataflow workgroups (0: one per compute unit)
  int tune = 0;                       // tuning word of the factor part (DfPart::tune)
  int n_high = 0;                     // factor ops flagged near-critical (high ring)
  int high_workers = 0;               // workgroups serving the high ring
  hipGraphExec_t graph_f = nullptr;   // factor schedule (with status reset)
  hipGraphExec_t graph_s = nullptr;   // solve schedule
  hipGraphExec_t graph_df = nullptr;  // factor by the dataflow executor
  hipGraphExec_t graph_dfs = nullptr; // solve by the dataflow executor
  void drop_graphs() {
    if (graph_f) hipGraphExecDestroy(graph_f);
    if (graph_s) hipGraphExecDestroy(graph_s);
    if (graph_df) hipGraphExecDestroy(graph_df);
    if (graph_dfs) hipGraphExecDestroy(graph_dfs);
    graph_f = graph_s = graph_df = graph_dfs = nullptr;
  }
  ~hlu_handle_s() { drop_graphs(); }
};

extern "C" {

const char* hlu_last_error(void) { return g_err.c_str(); }

hlu_status hlu_plan(const double* xyz, const double* area, int64_t n, const hlu_params* p,
                    hlu_handle* out) {
  g_err.clear();
  if (!xyz || !area || !p || !out) return fail(HLU_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (n < 1 || n > (1LL << 30)) return fail(HLU_ERR_ARG, "n out of range");
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(xyz[i])) return fail(HLU_ERR_ARG, "non-finite coordinate");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(area[i]) || area[i] < 0) return fail(HLU_ERR_ARG, "bad area");
  if (p->leaf_size < 1 || p->leaf_size > 64) return fail(HLU_ERR_ARG, "leaf_size must be in [1, 64]");
  if (!(p->eta >= 0) || !std::isfinite(p->eta)) return fail(HLU_ERR_ARG, "eta must be >= 0");
  if (p->rank_cap_factor < 1 || p->rank_cap_factor > 32)
    return fail(HLU_ERR_ARG, "rank_cap_factor must be in [1, 32]");
  if (p->rank_cap_matvec < 0 || p->rank_cap_matvec > 64)
    return fail(HLU_ERR_ARG, "rank_cap_matvec must be in [0, 64]");
  if (p->device_assembly != 0 && p->device_assembly != 1)
    return fail(HLU_ERR_ARG, "device_assembly must be 0 or 1");
  if (p->operation < HLU_OP_LU || p->operation > HLU_OP_INVERSE)
    return fail(HLU_ERR_ARG, "unknown operation");
  if (p->operation != HLU_OP_LU) {
    if (p->rank_cap_matvec != 0 || p->device_assembly != 0 || p->refine_tol != 0.0)
      return fail(HLU_ERR_ARG, "products and inverses take rank_cap_matvec = 0, host "
                               "assembly and no refinement");
    if (n > (1LL << 28)) return fail(HLU_ERR_ARG, "n out of range for a doubled plan");
    if (p->operation == HLU_OP_PRODUCT &&
        (p->kernel_b < HLU_KERNEL_LAPLACE3D_WEIGHTED || p->kernel_b > HLU_KERNEL_LAPLACE2D_LOG))
      return fail(HLU_ERR_ARG, "unknown kernel_b");
  }
  if (p->device_assembly == 1 && p->rank_cap_matvec != 0)
    return fail(HLU_ERR_ARG, "device assembly builds no operator copy: rank_cap_matvec must be 0");
  if (p->scratch_cap_bytes < 0) return fail(HLU_ERR_ARG, "scratch_cap_bytes must be >= 0");
  if (p->fixed_rank < 0 || p->fixed_rank > p->rank_cap_factor)
    return fail(HLU_ERR_ARG, "fixed_rank must be in [0, rank_cap_factor]");
  if (p->fixed_rank == 0 && !(p->eps_factor > 0 && p->eps_factor < 1))
    return fail(HLU_ERR_ARG, "eps_factor must be in (0, 1)");
  // the device truncation orthogonalises the stacked factors through FP64
  // Gram matrices, which resolve singular values only down to about 1e-8 of
  // the largest: tighter tolerances would be met in name only
  if (p->fixed_rank == 0 && p->eps_factor < 1e-8)
    return fail(HLU_ERR_ARG, "eps_factor must be >= 1e-8 (FP64 Gram truncation)");
  if (p->rank_cap_matvec > 0 && !(p->eps_matvec > 0 && p->eps_matvec < 1))
    return fail(HLU_ERR_ARG, "eps_matvec must be in (0, 1)");
  if (p->max_nrhs < 1 || p->max_nrhs > 64) return fail(HLU_ERR_ARG, "max_nrhs must be in [1, 64]");
  if (p->kernel != HLU_KERNEL_LAPLACE3D_WEIGHTED && p->kernel != HLU_KERNEL_LAPLACE3D_POINT &&
      p->kernel != HLU_KERNEL_LAPLACE1D_LOG && p->kernel != HLU_KERNEL_LAPLACE2D_LOG)
    return fail(HLU_ERR_ARG, "unknown kernel");
  if (p->kernel == HLU_KERNEL_LAPLACE1D_LOG || p->kernel == HLU_KERNEL_LAPLACE2D_LOG)
    for (int64_t i = 0; i < n; ++i)
      if (!(area[i] > 0)) return fail(HLU_ERR_ARG, "panel lengths must be > 0");
  if (p->precision != HLU_PREC_FP64 && p->precision != HLU_PREC_MIXED)
    return fail(HLU_ERR_ARG, "unknown precision");
  if (p->refine_max_iter < 0 || p->refine_max_iter > 15)
    return fail(HLU_ERR_ARG, "refine_max_iter must be in [0, 15]");
  hlu_handle h = nullptr;
  try {
    h = new hlu_handle_s(std::make_shared<hlu::Plan>());
  } catch (const std::bad_alloc&) {
    return fail(HLU_ERR_NOMEM, "host allocation failed");
  }
  h->params = *p;
  h->refine_tol = p->refine_tol;
  h->refine_max_iter = p->refine_max_iter;
  hlu::Params prm;
  prm.kernel = p->kernel;
  prm.eta = p->eta;
  prm.leaf = p->leaf_size;
  prm.fixed_rank = p->fixed_rank;
  prm.eps_f = p->fixed_rank > 0 ? 0.0 : p->eps_factor;
  prm.cap_f = p->rank_cap_factor;
  prm.eps_mv = p->eps_matvec;
  prm.cap_mv = p->rank_cap_matvec;
  prm.mixed = p->precision == HLU_PREC_MIXED;
  prm.refine_tol = p->refine_tol;
  prm.refine_max_iter = p->refine_max_iter;
  prm.max_nrhs = p->max_nrhs;
  prm.scratch_cap = (uint64_t)p->scratch_cap_bytes;
  prm.device_asm = p->device_assembly;
  prm.operation = p->operation;
  prm.kernel_b = p->operation == HLU_OP_PRODUCT ? p->kernel_b : p->kernel;
  try {
    if (!hlu::build_plan(h->plan, xyz, area, n, prm)) {
      std::string e = h->plan.err;
      delete h;
      return fail(HLU_ERR_ARG, "planning failed: " + e);
    }
    if (prm.device_asm)
      for (const auto& b : h->plan.blk)
        if (b.kind == 'R' && (b.m > 65536 || b.n > 65536)) {
          delete h;
          return fail(HLU_ERR_ARG, "device assembly: an admissible block exceeds 65536 rows");
        }
  } catch (const std::bad_alloc&) {
    delete h;
    return fail(HLU_ERR_NOMEM, "host allocation failed while planning");
  }
  *out = h;
  return HLU_OK;
}

hlu_status hlu_clone(hlu_handle src, hlu_handle* out) {
  if (!src || !out) return fail(HLU_ERR_ARG, "NULL argument");
  *out = nullptr;
  hlu_handle h = nullptr;
  try {
    h = new hlu_handle_s(src->shared);
  } catch (const std::bad_alloc&) {
    return fail(HLU_ERR_NOMEM, "host allocation failed");
  }
  h->params = src->params;
  h->refine_tol = src->refine_tol;
  h->refine_max_iter = src->refine_max_iter;
  h->use_graph = src->use_graph;
  h->executor = src->executor;
  h->workers = src->workers;
  *out = h;
  return HLU_OK;
}

size_t hlu_required_bytes(hlu_handle h) { return h ? (size_t)h->plan.total : 0; }

hlu_status hlu_validate(hlu_handle h) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  std::string why;
  if (!validate(h->plan, h->plan.fsched, why)) return fail(HLU_ERR_ARG, "factor schedule: " + why);
  if (!validate(h->plan, h->plan.ssched, why)) return fail(HLU_ERR_ARG, "solve schedule: " + why);
  const hlu::Plan& p = h->plan;
  // dependency graph: successors lie later in schedule order (acyclic), and
  // every in-degree equals the number of edges pointing at the op
  for (const hlu::Schedule* scp : {&p.fsched, &p.ssched}) {
    const hlu::Schedule& sc = *scp;
    const size_t N = sc.ops.size();
    if (sc.succ_off.size() != N + 1 || sc.indeg0.size() != N)
      return fail(HLU_ERR_ARG, "dependency graph size");
    // op types the dataflow executor of this schedule runs
    const unsigned allowed =
        scp == &p.fsched
            ? (1u << hlu::OP_GETRF) | (1u << hlu::OP_TRSM_L) | (1u << hlu::OP_TRSM_UT) |
                  (1u << hlu::OP_TRSM_U) | (1u << hlu::OP_PGEMM) | (1u << hlu::OP_TRUNC) |
                  (1u << hlu::OP_ADDD) | (1u << hlu::OP_ZERO) | (1u << hlu::OP_TRINV)
            : (1u << hlu::OP_MVT) | (1u << hlu::OP_MVROW) | (1u << hlu::OP_INVAPPLY);
    for (const auto& op : sc.ops)
      if (!((allowed >> op.type) & 1))
        return fail(HLU_ERR_ARG, "op type " + std::to_string(op.type) + " outside the " +
                                     (scp == &p.fsched ? "factor" : "solve") + " executor's set");
    // wave of every op (the wave executor runs a wave's ops concurrently,
    // so every dependency edge must cross waves)
    std::vector<int32_t> wv(N, 0);
    for (const auto& w : sc.waves_list)
      for (int q = 0; q < w.count; ++q) wv[w.start + q] = w.wave;
    std::vector<int32_t> cnt(N, 0);
    for (size_t i = 0; i < N; ++i)
      for (int32_t e = sc.succ_off[i]; e < sc.succ_off[i + 1]; ++e) {
        int32_t s = sc.succ[e];
        if (s <= (int64_t)i || s >= (int64_t)N) return fail(HLU_ERR_ARG, "dependency edge order");
        if (wv[s] <= wv[i]) return fail(HLU_ERR_ARG, "dependency edge inside one wave");
        cnt[s]++;
      }
    size_t nready = 0;
    for (size_t i = 0; i < N; ++i) {
      if (cnt[i] != sc.indeg0[i]) return fail(HLU_ERR_ARG, "dependency in-degree");
      nready += sc.indeg0[i] == 0;
    }
    if (nready != sc.ready0.size()) return fail(HLU_ERR_ARG, "initial ready list");
  }
  // matvec tables
  for (const auto& e : p.mv_lr) {
    if (e.k > 0 && (e.U < 512 || e.U + (uint64_t)e.m * e.k * 8 > p.total ||
                    e.V + (uint64_t)e.n * e.k * 8 > p.total ||
                    e.T + (uint64_t)e.kcap * p.prm.max_nrhs * 8 > p.total ||
                    e.c0 + e.n > p.n || e.r0 + e.m > p.n))
      return fail(HLU_ERR_ARG, "matvec low-rank table");
  }
  for (const auto& r : p.mv_rows) {
    if (r.r0 < 0 || r.r0 + r.rows > p.n || r.t0 + r.nt > (int64_t)p.mv_terms.size())
      return fail(HLU_ERR_ARG, "matvec row table");
    for (int q = 0; q < r.nt; ++q) {
      const auto& t = p.mv_terms[r.t0 + q];
      if (t.roff < 0 || t.roff + r.rows > t.lda) return fail(HLU_ERR_ARG, "matvec term rows");
      if (t.A + ((uint64_t)t.lda * t.ncol) * 8 > p.total) return fail(HLU_ERR_ARG, "matvec term extent");
      if (t.T == 0 && t.c0 + t.ncol > p.n) return fail(HLU_ERR_ARG, "matvec term columns");
    }
  }
  // device assembly: every block inside the buffer and the points, every
  // recompression op's panels and its term inside the buffer
  if (p.prm.device_asm) {
    for (const auto& a : p.asm_dense)
      if (a.U < 512 || a.U + (uint64_t)a.m * a.n * 8 > p.total || a.r0 < 0 || a.c0 < 0 ||
          a.r0 + a.m > p.n || a.c0 + a.n > p.n)
        return fail(HLU_ERR_ARG, "assembly dense table");
    for (const auto& a : p.asm_lr)
      if (a.U < p.off_asm_ws || a.U + (uint64_t)a.m * p.asm_kmax * 8 > p.off_asm_ws + p.size_asm_ws ||
          a.V < p.off_asm_ws || a.V + (uint64_t)a.n * p.asm_kmax * 8 > p.off_asm_ws + p.size_asm_ws ||
          a.rank < 256 || a.rank + 4 > p.total || a.r0 < 0 || a.c0 < 0 || a.r0 + a.m > p.n ||
          a.c0 + a.n > p.n || a.m > 65536 || a.n > 65536)
        return fail(HLU_ERR_ARG, "assembly low-rank table");
    if (p.asm_ops.size() != p.asm_lr.size() || p.asm_terms.size() != p.asm_lr.size())
      return fail(HLU_ERR_ARG, "assembly op count");
    for (size_t i = 0; i < p.asm_ops.size(); ++i) {
      const hlu::Op& o = p.asm_ops[i];
      const hlu::Term& t = p.asm_terms[i];
      if (o.type != hlu::OP_TRUNC || o.i0 != (int32_t)i || o.i1 != 1 ||
          !panel_ok(o.p[0], p.total, why) || !panel_ok(o.p[1], p.total, why) ||
          !panel_ok(t.X, p.total, why) || !panel_ok(t.Y, p.total, why) ||
          t.X.rows != o.p[0].rows || t.Y.rows != o.p[1].rows || t.X.cols + 0 > 64 ||
          o.p[2].ptr != p.off_asm_terms)
        return fail(HLU_ERR_ARG, "assembly recompression op: " + why);
    }
  }
  return HLU_OK;
}

hlu_status hlu_get_stats(hlu_handle h, hlu_plan_stats* o) {
  if (!h || !o) return fail(HLU_ERR_ARG, "NULL argument");
  const hlu::Plan& p = h->plan;
  std::memset(o, 0, sizeof(*o));
  o->n = p.n;
  o->leaves = (int64_t)p.leaves.size();
  for (auto& b : p.blk) (b.kind == 'F' ? o->dense_blocks : o->lowrank_blocks)++;
  o->ops_factor = (int64_t)p.fsched.ops.size();
  o->waves_factor = p.fsched.waves;
  o->ops_solve = (int64_t)p.ssched.ops.size();
  o->waves_solve = p.ssched.waves;
  o->bytes_factor_region = (int64_t)p.size_work;
  o->bytes_matvec_region = (int64_t)p.size_mv;
  o->bytes_scratch = (int64_t)p.size_scratch;
  o->bytes_total = (int64_t)p.total;
  o->offset_scratch = (int64_t)p.off_scratch;
  return HLU_OK;
}

hlu_status hlu_get_perm(hlu_handle h, int64_t* perm) {
  if (!h || !perm) return fail(HLU_ERR_ARG, "NULL argument");
  // doubled plans (products, inverses): the first copy's order (the second
  // copy's is the same)
  std::memcpy(perm, h->plan.perm.data(), sizeof(int64_t) * h->plan.n_orig);
  return HLU_OK;
}

hlu_status hlu_bind(hlu_handle h, void* dev_ptr, size_t bytes) {
  if (!h || !dev_ptr) return fail(HLU_ERR_ARG, "NULL argument");
  if (((uintptr_t)dev_ptr) & 255) return fail(HLU_ERR_ARG, "buffer must be 256-byte aligned");
  if (bytes < h->plan.total) return fail(HLU_ERR_NOMEM, "bound buffer smaller than required bytes");
  hlu::Plan& p = h->plan;
  {
    hlu_status vs = hlu_validate(h);
    if (vs != HLU_OK) return vs;
  }
  uint64_t base = (uint64_t)dev_ptr;
  // relocated copies of the schedules and the matvec tables
  std::vector<hlu::Op> f = p.fsched.ops, s = p.ssched.ops;
  for (auto& op : f) relocate(op, base);
  for (auto& op : s) relocate(op, base);
  for (int q = 0; q < 2; ++q) {
    std::vector<hlu::Term> tf = q ? p.ssched.terms : p.fsched.terms;
    for (auto& t : tf) {
      relocate(t.X, base);
      relocate(t.Y, base);
    }
    if (!tf.empty())
      HIPCHK(hipMemcpy((char*)dev_ptr + (q ? p.off_terms_s : p.off_terms_f), tf.data(),
                       tf.size() * sizeof(hlu::Term), hipMemcpyHostToDevice));
  }
  for (const DfArrays& da : {df_factor(p), df_solve(p)}) {
    const hlu::Schedule& sc = *da.sc;
    char* d = (char*)dev_ptr;
    HIPCHK(hipMemcpy(d + da.succ_off, sc.succ_off.data(), sc.succ_off.size() * 4,
                     hipMemcpyHostToDevice));
    if (!sc.succ.empty())
      HIPCHK(hipMemcpy(d + da.succ, sc.succ.data(), sc.succ.size() * 4, hipMemcpyHostToDevice));
    if (!sc.indeg0.empty())
      HIPCHK(hipMemcpy(d + da.indeg0, sc.indeg0.data(), sc.indeg0.size() * 4,
                       hipMemcpyHostToDevice));
    if (!sc.ready0.empty())
      HIPCHK(hipMemcpy(d + da.ready0, sc.ready0.data(), sc.ready0.size() * 4,
                       hipMemcpyHostToDevice));
    HIPCHK(hipMemset(d + da.ctrl, 0, 256));
    hlu::DfPart pt;
    pt.ops = base + da.ops;
    pt.succ_off = base + da.succ_off;
    pt.succ = base + da.succ;
    pt.indeg0 = base + da.indeg0;
    pt.indeg = base + da.indeg;
    pt.base = 0;
    pt.n = (int32_t)sc.ops.size();
    pt.tune = da.sc == &p.fsched ? h->tune : 0;
    pt.pad = 0;
    HIPCHK(hipMemcpy(d + da.part(), &pt, sizeof(pt), hipMemcpyHostToDevice));
  }
  std::vector<hlu::MvLR> lr = p.mv_lr;
  for (auto& e : lr) {
    if (e.U) e.U += base;
    if (e.V) e.V += base;
    if (e.T) e.T += base;
  }
  std::vector<hlu::MvTerm> tm = p.mv_terms;
  for (auto& t : tm) {
    if (t.A) t.A += base;
    if (t.T) t.T += base;
  }
  char* b = (char*)dev_ptr;
  if (!f.empty()) HIPCHK(hipMemcpy(b + p.off_ops_f, f.data(), f.size() * sizeof(hlu::Op), hipMemcpyHostToDevice));
  if (!s.empty()) HIPCHK(hipMemcpy(b + p.off_ops_s, s.data(), s.size() * sizeof(hlu::Op), hipMemcpyHostToDevice));
  if (!lr.empty()) HIPCHK(hipMemcpy(b + p.off_mv_lr, lr.data(), lr.size() * sizeof(hlu::MvLR), hipMemcpyHostToDevice));
  if (!tm.empty()) HIPCHK(hipMemcpy(b + p.off_mv_terms, tm.data(), tm.size() * sizeof(hlu::MvTerm), hipMemcpyHostToDevice));
  if (!p.mv_rows.empty())
    HIPCHK(hipMemcpy(b + p.off_mv_rows, p.mv_rows.data(), p.mv_rows.size() * sizeof(hlu::MvRow), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b + p.off_perm, p.perm.data(), sizeof(int64_t) * p.n, hipMemcpyHostToDevice));
  {
    // points in cluster order (x y z interleaved, then the panel weights)
    std::vector<double> pts((size_t)4 * p.n);
    std::memcpy(pts.data(), p.xyz.data(), sizeof(double) * 3 * (size_t)p.n);
    std::memcpy(pts.data() + 3 * (size_t)p.n, p.area.data(), sizeof(double) * (size_t)p.n);
    HIPCHK(hipMemcpy(b + p.off_pts, pts.data(), pts.size() * 8, hipMemcpyHostToDevice));
  }
  if (p.prm.device_asm) {
    std::vector<hlu::AsmBlock> ad = p.asm_dense, al = p.asm_lr;
    for (auto& a : ad) a.U += base;
    for (auto& a : al) {
      a.U += base;
      a.V += base;
      a.rank += base;
    }
    std::vector<hlu::Op> ao = p.asm_ops;
    for (auto& op : ao) relocate(op, base);
    std::vector<hlu::Term> at = p.asm_terms;
    for (auto& t : at) {
      relocate(t.X, base);
      relocate(t.Y, base);
    }
    if (!ad.empty())
      HIPCHK(hipMemcpy(b + p.off_asm_dense, ad.data(), ad.size() * sizeof(hlu::AsmBlock), hipMemcpyHostToDevice));
    if (!al.empty())
      HIPCHK(hipMemcpy(b + p.off_asm_lr, al.data(), al.size() * sizeof(hlu::AsmBlock), hipMemcpyHostToDevice));
    if (!ao.empty())
      HIPCHK(hipMemcpy(b + p.off_asm_ops, ao.data(), ao.size() * sizeof(hlu::Op), hipMemcpyHostToDevice));
    if (!at.empty())
      HIPCHK(hipMemcpy(b + p.off_asm_terms, at.data(), at.size() * sizeof(hlu::Term), hipMemcpyHostToDevice));
  }
  HIPCHK(hipMemset(b + p.off_status, 0, 256));
  h->drop_graphs();
  h->base = b;
  h->bytes = bytes;
  h->assembled = false;
  h->factored = false;
  return HLU_OK;
}

static hlu_status run_mv(hlu_handle h, const double* X, const double* B, double beta, double alpha,
                         double* Y, int nrhs, hipStream_t s) {
  hlu::Plan& p = h->plan;
  if (p.prm.cap_mv == 0) {
    // no operator copy: the exact matrix by direct summation
    HIPCHK(hlu_launch_direct_mv((const double*)(h->base + p.off_pts), p.n, p.prm.kernel, X, p.n, B,
                                beta, alpha, Y, nrhs, 0, s));
    return HLU_OK;
  }
  HIPCHK(hlu_launch_mv(h->base + p.off_mv_lr, (int)p.mv_lr.size(), h->base + p.off_mv_rows,
                       (int)p.mv_rows.size(), h->base + p.off_mv_terms, X, p.n, B, beta, alpha,
                       Y, nrhs, s));
  return HLU_OK;
}

hlu_status hlu_assemble(hlu_handle h, void* stream) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  if (!h->base) return fail(HLU_ERR_STATE, "hlu_bind first");
  hipStream_t s = (hipStream_t)stream;
  hlu::Plan& p = h->plan;
  char* b = h->base;
  h->asm_cap_hits = 0;
  if (p.prm.device_asm) {
    // the blocks are built on the device from the points: dense entries,
    // cross approximations chunk by chunk (sharing one workspace), each
    // chunk recompressed into the factored copy by the truncation kernel
    int32_t* caphits = (int32_t*)(b + p.off_status + 16);
    HIPCHK(hipMemsetAsync(b + p.off_work, 0, p.size_work, s));
    HIPCHK(hipMemsetAsync(b + p.off_status, 0, 256, s));
    const double* pts = (const double*)(b + p.off_pts);
    HIPCHK(hlu_launch_asm(b + p.off_asm_dense, (int)p.asm_dense.size(), nullptr, 0, pts, p.n,
                          p.prm.kernel, p.asm_eps, p.asm_kmax, caphits, s));
    for (const hlu::AsmChunk& c : p.asm_chunks) {
      HIPCHK(hlu_launch_asm(nullptr, 0, b + p.off_asm_lr + (uint64_t)c.b0 * sizeof(hlu::AsmBlock),
                            c.b1 - c.b0, pts, p.n, p.prm.kernel, p.asm_eps, p.asm_kmax, caphits, s));
      HIPCHK(hlu_launch_ops(hlu::OP_TRUNC, b + p.off_asm_ops + (uint64_t)c.op0 * sizeof(hlu::Op),
                            c.op1 - c.op0, s));
    }
    HIPCHK(hipMemcpyAsync(b + p.off_pristine, b + p.off_work, p.size_work,
                          hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(&h->asm_cap_hits, caphits, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemsetAsync(b + p.off_status, 0, 256, s));
  } else {
    HIPCHK(hipMemcpyAsync(b + p.off_work, p.img_work.data(), p.size_work, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(b + p.off_pristine, p.img_work.data(), p.size_work, hipMemcpyHostToDevice, s));
    if (p.size_mv)
      HIPCHK(hipMemcpyAsync(b + p.off_mv, p.img_mv.data(), p.size_mv, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(b + p.off_status, 0, 256, s));
  }
  if (p.prm.operation != 0) {
    // products and inverses: no solve, no backward error
    HIPCHK(hipStreamSynchronize(s));
    h->anorm = 0.0;
    h->assembled = true;
    h->factored = false;
    return HLU_OK;
  }
  if (p.prm.cap_mv == 0) {
    // |A|_inf of the exact matrix by direct summation
    double* Y = (double*)(b + p.off_Y);
    HIPCHK(hlu_launch_direct_mv((const double*)(b + p.off_pts), p.n, p.prm.kernel, nullptr, p.n,
                                nullptr, 0.0, 1.0, Y, 1, 1, s));
    std::vector<double> rs(p.n);
    HIPCHK(hipMemcpyAsync(rs.data(), Y, sizeof(double) * p.n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    h->anorm = *std::max_element(rs.begin(), rs.end());
    h->assembled = true;
    h->factored = false;
    return HLU_OK;
  }
  // |A|_inf: all entries of both kernels are positive, so it is the
  // largest entry of A * ones (with the accurate matvec copy)
  std::vector<double> ones(p.n, 1.0);
  double* X = (double*)(b + p.off_X);
  double* Y = (double*)(b + p.off_Y);
  HIPCHK(hipMemcpyAsync(X, ones.data(), sizeof(double) * p.n, hipMemcpyHostToDevice, s));
  hlu_status st = run_mv(h, X, nullptr, 0.0, 1.0, Y, 1, s);
  if (st != HLU_OK) return st;
  double* out = (double*)(b + p.off_eta);
  HIPCHK(hlu_launch_colmax(Y, X, X, p.n, p.n, 1, out, s));
  double mx[3];
  HIPCHK(hipMemcpyAsync(mx, out, sizeof(mx), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  h->anorm = mx[0];
  h->assembled = true;
  h->factored = false;
  return HLU_OK;
}

hlu_status hlu_assemble_from(hlu_handle h, hlu_handle src, void* stream) {
  if (!h || !src) return fail(HLU_ERR_ARG, "NULL handle");
  if (h->shared != src->shared) return fail(HLU_ERR_ARG, "handles do not share one plan");
  if (!h->base) return fail(HLU_ERR_STATE, "hlu_bind first");
  if (!src->assembled) return fail(HLU_ERR_STATE, "source not assembled");
  hipStream_t s = (hipStream_t)stream;
  const hlu::Plan& p = h->plan;
  char* b = h->base;
  HIPCHK(hipMemcpyAsync(b + p.off_work, src->base + p.off_pristine, p.size_work,
                        hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(b + p.off_pristine, src->base + p.off_pristine, p.size_work,
                        hipMemcpyDeviceToDevice, s));
  if (p.size_mv)
    HIPCHK(hipMemcpyAsync(b + p.off_mv, src->base + p.off_mv, p.size_mv, hipMemcpyDeviceToDevice,
                          s));
  HIPCHK(hlu_launch_set_int((int32_t*)(b + p.off_status), 0, s));
  h->anorm = src->anorm;
  h->assembled = true;
  h->factored = false;
  return HLU_OK;
}

// Blocks of an H-matrix built elsewhere (the file format is declared in
// hlu.h): every leaf block of this handle's block tree is replaced, in the
// factored copy and its pristine copy, by the file's block of the same rows
// and columns.  The refinement operator copy keeps the handle's own blocks.
namespace {
struct ImportFile {
  FILE* f = nullptr;
  ~ImportFile() { if (f) std::fclose(f); }
  bool read(void* dst, size_t bytes) { return std::fread(dst, 1, bytes, f) == bytes; }
};
}  // namespace

hlu_status hlu_import_blocks(hlu_handle h, const char* path) {
  if (!h || !path) return fail(HLU_ERR_ARG, "NULL argument");
  hlu::Plan& p = h->plan;
  ImportFile in;
  in.f = std::fopen(path, "rb");
  if (!in.f) return fail(HLU_ERR_ARG, std::string("cannot open ") + path);
  char magic[8];
  int64_t hdr[2];
  if (!in.read(magic, 8) || std::memcmp(magic, "HLUBLK01", 8) != 0)
    return fail(HLU_ERR_ARG, "not an H-matrix block file (magic HLUBLK01)");
  if (!in.read(hdr, sizeof(hdr))) return fail(HLU_ERR_ARG, "truncated header");
  if (hdr[0] != p.n) return fail(HLU_ERR_ARG, "block file is for another n");
  if (hdr[1] != (int64_t)p.blk.size())
    return fail(HLU_ERR_ARG, "block file has another number of leaf blocks");
  std::vector<int64_t> perm(p.n);
  if (!in.read(perm.data(), sizeof(int64_t) * p.n)) return fail(HLU_ERR_ARG, "truncated permutation");
  if (perm != p.perm) return fail(HLU_ERR_ARG, "block file was built on another cluster tree");
  std::unordered_map<uint64_t, int> at;
  for (size_t i = 0; i < p.blk.size(); ++i) {
    const hlu::LBlock& b = p.blk[i];
    at[((uint64_t)p.cl[b.t].off << 32) | (uint64_t)p.cl[b.s].off] = (int)i;
  }
  std::vector<char> img(p.size_work, 0);
  std::vector<char> seen(p.blk.size(), 0);
  std::vector<double> buf;
  const int cap = p.prm.cap_f;
  for (size_t q = 0; q < p.blk.size(); ++q) {
    int64_t d[6];
    if (!in.read(d, sizeof(d))) return fail(HLU_ERR_ARG, "truncated block header");
    const int64_t r0 = d[0], c0 = d[1], m = d[2], nc = d[3], kind = d[4], k = d[5];
    if (r0 < 0 || c0 < 0 || r0 >= p.n || c0 >= p.n)
      return fail(HLU_ERR_ARG, "block offset out of range");
    auto it = at.find(((uint64_t)r0 << 32) | (uint64_t)c0);
    if (it == at.end()) return fail(HLU_ERR_ARG, "block not in this block tree");
    const hlu::LBlock& b = p.blk[it->second];
    if (seen[it->second]) return fail(HLU_ERR_ARG, "block given twice");
    seen[it->second] = 1;
    if (m != b.m || nc != b.n) return fail(HLU_ERR_ARG, "block shape differs from the block tree");
    if (kind != (b.kind == 'R' ? 1 : 0)) return fail(HLU_ERR_ARG, "block kind differs (dense/low-rank)");
    if (kind == 0) {
      buf.resize((size_t)m * nc);
      if (!in.read(buf.data(), 8 * buf.size())) return fail(HLU_ERR_ARG, "truncated dense block");
      std::memcpy(img.data() + (b.offF - p.off_work), buf.data(), 8 * buf.size());
      continue;
    }
    if (k < 0 || k > cap) return fail(HLU_ERR_ARG, "rank above the rank capacity");
    *(int32_t*)(img.data() + (b.offRank - p.off_work)) = (int32_t)k;
    for (int side = 0; side < 2; ++side) {
      const int64_t rows = side ? nc : m;
      buf.resize((size_t)rows * k);
      if (!in.read(buf.data(), 8 * buf.size())) return fail(HLU_ERR_ARG, "truncated factor");
      char* dst = img.data() + ((side ? b.offV : b.offU) - p.off_work);
      if (p.prm.mixed) {
        float* f = (float*)dst;
        for (size_t e = 0; e < buf.size(); ++e) f[e] = (float)buf[e];
      } else {
        std::memcpy(dst, buf.data(), 8 * buf.size());
      }
    }
  }
  if (!h->base) return fail(HLU_ERR_STATE, "hlu_bind first");
  if (!h->assembled) return fail(HLU_ERR_STATE, "hlu_assemble first (the operator copy)");
  HIPCHK(hipMemcpy(h->base + p.off_work, img.data(), p.size_work, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->base + p.off_pristine, img.data(), p.size_work, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(h->base + p.off_status, 0, 256));
  h->factored = false;
  return HLU_OK;
}

hlu_status hlu_set_workers(hlu_handle h, int workers) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  if (workers < 0 || workers > 65536) return fail(HLU_ERR_ARG, "workers must be in [0, 65536]");
  if (workers != h->workers) h->drop_graphs();
  h->workers = workers;
  return HLU_OK;
}

// The factored copy's blocks as they are now on the device, in the file
// format hlu_import_blocks reads (FP32 factors widened to FP64).
hlu_status hlu_export_blocks(hlu_handle h, const char* path) {
  if (!h || !path) return fail(HLU_ERR_ARG, "NULL argument");
  if (!h->base) return fail(HLU_ERR_STATE, "hlu_bind first");
  const hlu::Plan& p = h->plan;
  std::vector<char> img(p.size_work);
  HIPCHK(hipMemcpy(img.data(), h->base + p.off_work, p.size_work, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(HLU_ERR_ARG, std::string("cannot create ") + path);
  bool ok = std::fwrite("HLUBLK01", 1, 8, f) == 8;
  int64_t hdr[2] = {p.n, (int64_t)p.blk.size()};
  ok = ok && std::fwrite(hdr, sizeof(hdr), 1, f) == 1;
  ok = ok && std::fwrite(p.perm.data(), 8, p.n, f) == (size_t)p.n;
  std::vector<double> buf;
  for (size_t i = 0; ok && i < p.blk.size(); ++i) {
    const hlu::LBlock& b = p.blk[i];
    const int64_t kind = b.kind == 'R' ? 1 : 0;
    const int64_t k = kind ? *(const int32_t*)(img.data() + (b.offRank - p.off_work)) : 0;
    int64_t d[6] = {p.cl[b.t].off, p.cl[b.s].off, b.m, b.n, kind, k};
    ok = std::fwrite(d, sizeof(d), 1, f) == 1;
    if (!kind) {
      ok = ok && std::fwrite(img.data() + (b.offF - p.off_work), 8, (size_t)b.m * b.n, f) ==
                     (size_t)b.m * b.n;
      continue;
    }
    for (int side = 0; ok && side < 2; ++side) {
      const int64_t rows = side ? b.n : b.m;
      const char* src = img.data() + ((side ? b.offV : b.offU) - p.off_work);
      buf.resize((size_t)rows * k);
      if (p.prm.mixed)
        for (size_t e = 0; e < buf.size(); ++e) buf[e] = ((const float*)src)[e];
      else
        std::memcpy(buf.data(), src, 8 * buf.size());
      ok = std::fwrite(buf.data(), 8, buf.size(), f) == buf.size();
    }
  }
  if (std::fclose(f) != 0) ok = false;
  if (!ok) return fail(HLU_ERR_ARG, std::string("write failed: ") + path);
  return HLU_OK;
}

// Result of a product or inverse plan after hlu_factor: the result
// quadrant (which holds -A B, or -A^-1) expanded densely with the sign
// restored, in the original point order (out: n x n column-major, ld).
hlu_status hlu_export_result(hlu_handle h, double* out, int64_t ld) {
  if (!h || !out) return fail(HLU_ERR_ARG, "NULL argument");
  const hlu::Plan& p = h->plan;
  if (p.prm.operation == 0) return fail(HLU_ERR_STATE, "not a product or inverse plan");
  if (!h->base || !h->factored) return fail(HLU_ERR_STATE, "hlu_factor first");
  const int n1 = p.n_orig;
  if (n1 > 16384) return fail(HLU_ERR_ARG, "n too large for a dense export");
  if (ld < n1) return fail(HLU_ERR_ARG, "ld < n");
  std::vector<char> w(p.size_work);
  HIPCHK(hipMemcpy(w.data(), h->base + p.off_work, p.size_work, hipMemcpyDeviceToHost));
  for (int j = 0; j < n1; ++j) std::memset(out + (size_t)j * ld, 0, sizeof(double) * n1);
  const int q = p.prm.operation == 1 ? 0 : 1;   // quadrant (q, q)
  for (const auto& b : p.blk) {
    const int r0 = p.cl[b.t].off - q * n1, c0 = p.cl[b.s].off - q * n1;
    if (r0 < 0 || c0 < 0 || r0 >= n1 || c0 >= n1) continue;
    auto put = [&](int i, int j, double v) {
      out[(size_t)p.perm[r0 + i] + (size_t)p.perm[c0 + j] * ld] = -v;
    };
    if (b.kind == 'F') {
      const double* F = (const double*)(w.data() + (b.offF - p.off_work));
      for (int j = 0; j < b.n; ++j)
        for (int i = 0; i < b.m; ++i) put(i, j, F[i + (size_t)j * b.m]);
      continue;
    }
    const int k = *(const int32_t*)(w.data() + (b.offRank - p.off_work));
    const char* U = w.data() + (b.offU - p.off_work);
    const char* V = w.data() + (b.offV - p.off_work);
    auto at = [&](const char* base, size_t e) {
      return p.prm.mixed ? (double)((const float*)base)[e] : ((const double*)base)[e];
    };
    for (int j = 0; j < b.n; ++j)
      for (int i = 0; i < b.m; ++i) {
        double v = 0.0;
        for (int l = 0; l < k; ++l) v += at(U, i + (size_t)l * b.m) * at(V, j + (size_t)l * b.n);
        put(i, j, v);
      }
  }
  return HLU_OK;
}

hlu_status hlu_set_tuning(hlu_handle h, int trunc_width) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  if (trunc_width != 0 && (trunc_width < 16 || trunc_width > 64))
    return fail(HLU_ERR_ARG, "trunc_width must be 0 or in [16, 64]");
  h->tune = trunc_width;
  if (h->base) {
    // the factor part's tuning word, in place (read by every later launch)
    const hlu::Plan& p = h->plan;
    const uint64_t at = df_factor(p).part() + offsetof(hlu::DfPart, tune);
    int32_t v = h->tune;
    HIPCHK(hipMemcpy(h->base + at, &v, 4, hipMemcpyHostToDevice));
  }
  h->drop_graphs();
  return HLU_OK;
}

hlu_status hlu_reset(hlu_handle h, void* stream) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  if (!h->assembled) return fail(HLU_ERR_STATE, "hlu_assemble first");
  hipStream_t s = (hipStream_t)stream;
  hlu::Plan& p = h->plan;
  HIPCHK(hipMemcpyAsync(h->base + p.off_work, h->base + p.off_pristine, p.size_work,
                        hipMemcpyDeviceToDevice, s));
  HIPCHK(hlu_launch_set_int((int32_t*)(h->base + p.off_status), 0, s));
  h->factored = false;
  return HLU_OK;
}

static size_t wave_lds(uint32_t mask) {
  size_t l = 0;
  for (int t = 0; t < hlu::OP_NTYPES; ++t)
    if (mask & (1u << t)) l = std::max(l, hlu_lds_bytes(t));
  return l;
}

static hlu_status build_graph(hlu_handle h, const hlu::Schedule& sc, uint64_t off_ops,
                              int32_t* status, hipGraphExec_t* out) {
  std::vector<int> st, ct;
  std::vector<size_t> lds;
  for (const hlu::Batch& w : sc.waves_list) {
    st.push_back(w.start);
    ct.push_back(w.count);
    lds.push_back(wave_lds(w.mask));
  }
  hipError_t e = hlu_build_wave_graph(h->base + off_ops, st.data(), ct.data(), lds.data(),
                                      (int)st.size(), status, out);
  if (e != hipSuccess) return fail(HLU_ERR_DEVICE, std::string("graph: ") + hipGetErrorString(e));
  return HLU_OK;
}

// One launch per wave (all op types of the wave together), or one replay of
// the schedule's graph.  `status` (factor only) is reset first.
static hlu_status run_schedule(hlu_handle h, const hlu::Schedule& sc, uint64_t off_ops,
                               hipStream_t s, int32_t* status, hipGraphExec_t* graph) {
  if (h->use_graph && graph) {
    if (!*graph) {
      hlu_status st = build_graph(h, sc, off_ops, status, graph);
      if (st != HLU_OK) return st;
    }
    HIPCHK(hipGraphLaunch(*graph, s));
    return HLU_OK;
  }
  if (status) HIPCHK(hlu_launch_set_int(status, 0, s));
  const char* ops = h->base + off_ops;
  for (const hlu::Batch& w : sc.waves_list) {
    hipError_t e = hlu_launch_wave(ops + (size_t)w.start * sizeof(hlu::Op), w.count,
                                   wave_lds(w.mask), s);
    if (e != hipSuccess) return fail(HLU_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  }
  return HLU_OK;
}

// device facts for the dataflow executor: workgroups (one per compute
// unit: the largest op type's LDS allows one resident workgroup) and the
// wall-clock ticks per second
static hlu_status device_facts(int* cus, long long* ticks_per_s) {
  int dev = 0, cu = 0, rate_khz = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
  *cus = cu > 0 ? cu : 1;
  *ticks_per_s = rate_khz > 0 ? (long long)rate_khz * 1000 : 100000000LL;
  return HLU_OK;
}

// Runs one schedule with the persistent dataflow executor.  The factor
// schedule also clears the status word first (the solve leaves it alone).
static hlu_status run_dataflow(hlu_handle h, const DfArrays& da, hipStream_t s,
                               hipGraphExec_t* graph) {
  hlu::Plan& p = h->plan;
  const hlu::Schedule& sc = *da.sc;
  char* b = h->base;
  int cus = 0;
  long long tps = 0;
  hlu_status st = device_facts(&cus, &tps);
  if (st != HLU_OK) return st;
  const long long timeout = 20 * tps;   // no single wait may exceed 20 s
  if (h->workers > 0) cus = h->workers;
  const bool factor = da.sc == &p.fsched;
  int32_t* status = factor ? (int32_t*)(b + p.off_status) : nullptr;
  int* queue = (int*)(b + da.queue);
  const int* ready0 = (const int*)(b + da.ready0);
  int* ctrl = (int*)(b + da.ctrl);
  const void* part = b + da.part();
  const int n = (int)sc.ops.size(), nready = (int)sc.ready0.size();
  if (n == 0) return HLU_OK;
  const int nhigh = factor && h->high_workers > 0 && h->high_workers < cus ? h->n_high : 0;
  const int nhw = nhigh > 0 ? h->high_workers : 0;
  if (h->use_graph) {
    if (!*graph)
      HIPCHK(hlu_build_df_graph(factor ? 0 : 1, part, 1, queue, ready0, nready, ctrl, n, nhigh,
                                nhw, cus, timeout, status, graph));
    HIPCHK(hipGraphLaunch(*graph, s));
    return HLU_OK;
  }
  HIPCHK(hlu_launch_dataflow(factor ? 0 : 1, part, 1, queue, ready0, nready, ctrl, n, nhigh, nhw,
                             cus, timeout, status, s));
  return HLU_OK;
}

// Word of the status region that keeps the first error flag any solve
// sweep of the current hlu_solve raised (every dataflow launch clears its
// own control words, so a later sweep would otherwise hide an earlier one).
static int32_t* solve_error_word(hlu_handle h) {
  return (int32_t*)(h->base + h->plan.off_status + 8);
}

// One forward/backward sweep of the solve schedule (Y := A_H^{-1} Y).
static hlu_status run_solve(hlu_handle h, hipStream_t s) {
  hlu::Plan& p = h->plan;
  if (h->executor == 1) {
    hlu_status st = run_dataflow(h, df_solve(p), s, &h->graph_dfs);
    if (st != HLU_OK) return st;
    HIPCHK(hlu_launch_keep_flag((const int32_t*)(h->base + p.off_dfs_ctrl + 8),
                                solve_error_word(h), s));
    return HLU_OK;
  }
  return run_schedule(h, p.ssched, p.off_ops_s, s, nullptr, &h->graph_s);
}

hlu_status hlu_factor(hlu_handle h, void* stream) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  if (!h->assembled) return fail(HLU_ERR_STATE, "hlu_assemble first");
  if (h->factored) return fail(HLU_ERR_STATE, "already factored: hlu_reset first");
  hipStream_t s = (hipStream_t)stream;
  hlu_status st = h->executor == 1
                      ? run_dataflow(h, df_factor(h->plan), s, &h->graph_df)
                      : run_schedule(h, h->plan.fsched, h->plan.off_ops_f, s,
                                     (int32_t*)(h->base + h->plan.off_status), &h->graph_f);
  if (st != HLU_OK) return st;
  h->factored = true;
  return HLU_OK;
}

hlu_status hlu_set_executor(hlu_handle h, int mode) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  if (mode != 0 && mode != 1) return fail(HLU_ERR_ARG, "executor must be 0 (waves) or 1 (dataflow)");
  h->executor = mode;
  return HLU_OK;
}

// Near-critical ops of the factor schedule from the last factorisation's op
// records: with d the recorded durations and a fixed hand-off time per edge,
// top(u) is the longest path to u's start and bottom(u) the longest path
// from u's start to the end; an op whose slack L - top - bottom is at most
// slack_frac * L (L the longest path) and that has predecessors is flagged
// (bit 30 of its initial in-degree on the device) and goes to the high
// ring, served by high_workers workgroups.  high_workers = 0 clears the
// flags.
hlu_status hlu_set_priorities(hlu_handle h, double slack_frac, int high_workers,
                              int32_t* n_flagged) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  if (!h->base) return fail(HLU_ERR_STATE, "hlu_bind first");
  if (high_workers < 0 || high_workers > 1024)
    return fail(HLU_ERR_ARG, "high_workers must be in [0, 1024]");
  if (!(slack_frac >= 0.0 && slack_frac <= 1.0))
    return fail(HLU_ERR_ARG, "slack_frac must be in [0, 1]");
  const hlu::Schedule& sc = h->plan.fsched;
  const size_t n = sc.ops.size();
  std::vector<int32_t> deg(sc.indeg0.begin(), sc.indeg0.end());
  int nh = 0;
  if (high_workers > 0 && n > 0) {
    if (!h->factored) return fail(HLU_ERR_STATE, "factor once first (its op records give the durations)");
    int cus = 0;
    long long tps = 0;
    hlu_status st = device_facts(&cus, &tps);
    if (st != HLU_OK) return st;
    HIPCHK(hipDeviceSynchronize());
    std::vector<double> rec(n * (hlu::kCostRecBytes / 8));
    HIPCHK(hipMemcpy(rec.data(), h->base + h->plan.off_cost, n * hlu::kCostRecBytes,
                     hipMemcpyDeviceToHost));
    const size_t w = hlu::kCostRecBytes / 8;
    const double hop = 8e-6 * (double)tps;   // hand-off of one edge, in ticks
    std::vector<double> d(n), top(n, 0.0), bot(n, 0.0);
    for (size_t i = 0; i < n; ++i) d[i] = std::max(0.0, rec[i * w + 5] - rec[i * w + 4]);
    // the schedule is in topological order (every edge points forward)
    for (size_t u = 0; u < n; ++u)
      for (int e = sc.succ_off[u]; e < sc.succ_off[u + 1]; ++e) {
        const int v = sc.succ[e];
        top[v] = std::max(top[v], top[u] + d[u] + hop);
      }
    double L = 0.0;
    for (size_t u = n; u-- > 0;) {
      double b = 0.0;
      for (int e = sc.succ_off[u]; e < sc.succ_off[u + 1]; ++e)
        b = std::max(b, hop + bot[sc.succ[e]]);
      bot[u] = d[u] + b;
      L = std::max(L, top[u] + bot[u]);
    }
    for (size_t u = 0; u < n; ++u)
      if (deg[u] > 0 && L - top[u] - bot[u] <= slack_frac * L) {
        deg[u] |= 1 << 30;
        ++nh;
      }
  }
  const DfArrays da = df_factor(h->plan);
  if (n > 0)
    HIPCHK(hipMemcpy(h->base + da.indeg0, deg.data(), n * 4, hipMemcpyHostToDevice));
  h->n_high = nh;
  h->high_workers = nh > 0 ? high_workers : 0;
  h->drop_graphs();
  if (n_flagged) *n_flagged = nh;
  return HLU_OK;
}

hlu_status hlu_set_refinement(hlu_handle h, double refine_tol, int refine_max_iter) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  if (!(refine_tol >= 0.0) || !std::isfinite(refine_tol))
    return fail(HLU_ERR_ARG, "refine_tol must be >= 0");
  if (refine_max_iter < 0 || refine_max_iter > 15)
    return fail(HLU_ERR_ARG, "refine_max_iter must be in [0, 15]");
  h->refine_tol = refine_tol;
  h->refine_max_iter = refine_max_iter;
  return HLU_OK;
}

hlu_status hlu_set_graph(hlu_handle h, int enable) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  h->use_graph = enable != 0;
  return HLU_OK;
}

hlu_status hlu_factor_profile(hlu_handle h, void* stream, double* ms_per_type,
                              int64_t* launches_per_type) {
  if (!h || !ms_per_type || !launches_per_type) return fail(HLU_ERR_ARG, "NULL argument");
  if (!h->assembled) return fail(HLU_ERR_STATE, "hlu_assemble first");
  if (h->factored) return fail(HLU_ERR_STATE, "already factored: hlu_reset first");
  hipStream_t s = (hipStream_t)stream;
  const hlu::Schedule& sc = h->plan.fsched;
  const char* ops = h->base + h->plan.off_ops_f;
  std::vector<hipEvent_t> ev(2 * sc.batches.size());
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  HIPCHK(hlu_launch_set_int((int32_t*)(h->base + h->plan.off_status), 0, s));
  hipError_t err = hipSuccess;
  for (size_t i = 0; i < sc.batches.size() && err == hipSuccess; ++i) {
    const hlu::Batch& bt = sc.batches[i];
    err = hipEventRecord(ev[2 * i], s);
    if (err == hipSuccess)
      err = hlu_launch_ops(bt.type, ops + (size_t)bt.start * sizeof(hlu::Op), bt.count, s);
    if (err == hipSuccess) err = hipEventRecord(ev[2 * i + 1], s);
  }
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  for (int t = 0; t < HLU_OP_TYPES; ++t) { ms_per_type[t] = 0.0; launches_per_type[t] = 0; }
  for (size_t i = 0; i < sc.batches.size() && err == hipSuccess; ++i) {
    float ms = 0.f;
    err = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
    ms_per_type[sc.batches[i].type] += ms;
    launches_per_type[sc.batches[i].type]++;
  }
  for (auto& e : ev) hipEventDestroy(e);
  if (err != hipSuccess) return fail(HLU_ERR_DEVICE, hipGetErrorString(err));
  h->factored = true;
  return HLU_OK;
}

// ---- batched factorisation: the union of several handles' factor
// schedules run by one persistent executor launch.  The batch owns only the
// part table, a queue over all ops and the initial ready list; every op keeps
// reading and writing its own handle's buffer.
struct hlu_batch_s {
  std::vector<hlu_handle> hs;
  std::vector<int32_t> base;
  std::vector<int32_t> ready0;    // global indices, the handles' ready lists interleaved
  int64_t ntot = 0;
  uint64_t off_parts = 0, off_queue = 0, off_ready0 = 0, off_ctrl = 0, total = 0;
  char* dev = nullptr;
  int tune = 0;                   // tuning word of every part (DfPart::tune)
  int workers = 0;                // workgroups of the launch (0: one per compute unit)
};

hlu_status hlu_batch_create(const hlu_handle* hs, int count, hlu_batch* out) {
  if (!hs || !out || count < 1) return fail(HLU_ERR_ARG, "bad handle list");
  *out = nullptr;
  auto* b = new (std::nothrow) hlu_batch_s;
  if (!b) return fail(HLU_ERR_NOMEM, "host allocation failed");
  int64_t tot = 0;
  for (int i = 0; i < count; ++i) {
    if (!hs[i]) {
      delete b;
      return fail(HLU_ERR_ARG, "NULL handle");
    }
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) {
        delete b;
        return fail(HLU_ERR_ARG, "a handle appears twice in the batch");
      }
    b->hs.push_back(hs[i]);
    b->base.push_back((int32_t)tot);
    tot += (int64_t)hs[i]->plan.fsched.ops.size();
    if (tot >= (int64_t)1 << 31) {
      delete b;
      return fail(HLU_ERR_ARG, "too many ops in one batch");
    }
  }
  b->ntot = tot;
  // round-robin over the handles so that every matrix starts at once
  std::vector<size_t> cur(count, 0);
  for (bool more = true; more;) {
    more = false;
    for (int i = 0; i < count; ++i) {
      const auto& r = hs[i]->plan.fsched.ready0;
      if (cur[i] < r.size()) {
        b->ready0.push_back(b->base[i] + r[cur[i]++]);
        more = true;
      }
    }
  }
  uint64_t c = 0;
  auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
  b->off_parts = c;
  c = al(c + (uint64_t)count * sizeof(hlu::DfPart));
  b->off_queue = c;
  c = al(c + (uint64_t)std::max<int64_t>(1, tot) * 4);
  b->off_ready0 = c;
  c = al(c + (uint64_t)std::max<size_t>(1, b->ready0.size()) * 4);
  b->off_ctrl = c;
  c = al(c + 256);
  b->total = c;
  *out = b;
  return HLU_OK;
}

size_t hlu_batch_required_bytes(hlu_batch b) { return b ? (size_t)b->total : 0; }

hlu_status hlu_batch_bind(hlu_batch b, void* dev_ptr, size_t bytes) {
  if (!b || !dev_ptr) return fail(HLU_ERR_ARG, "NULL argument");
  if (bytes < b->total) return fail(HLU_ERR_ARG, "buffer smaller than hlu_batch_required_bytes");
  if (((uint64_t)dev_ptr & 255) != 0) return fail(HLU_ERR_ARG, "buffer not 256-byte aligned");
  std::vector<hlu::DfPart> parts(b->hs.size());
  for (size_t i = 0; i < b->hs.size(); ++i) {
    hlu_handle h = b->hs[i];
    if (!h->base) return fail(HLU_ERR_STATE, "every handle must be bound first");
    const hlu::Plan& p = h->plan;
    const uint64_t hb = (uint64_t)h->base;
    parts[i].ops = hb + p.off_ops_f;
    parts[i].succ_off = hb + p.off_df_succ_off;
    parts[i].succ = hb + p.off_df_succ;
    parts[i].indeg0 = hb + p.off_df_indeg0;
    parts[i].indeg = hb + p.off_df_indeg;
    parts[i].base = b->base[i];
    parts[i].n = (int32_t)p.fsched.ops.size();
    parts[i].tune = b->tune;
    parts[i].pad = 0;
  }
  char* d = (char*)dev_ptr;
  HIPCHK(hipMemcpy(d + b->off_parts, parts.data(), parts.size() * sizeof(hlu::DfPart),
                   hipMemcpyHostToDevice));
  if (!b->ready0.empty())
    HIPCHK(hipMemcpy(d + b->off_ready0, b->ready0.data(), b->ready0.size() * 4,
                     hipMemcpyHostToDevice));
  HIPCHK(hipMemset(d + b->off_ctrl, 0, 256));
  b->dev = d;
  return HLU_OK;
}

hlu_status hlu_batch_set_tuning(hlu_batch b, int trunc_width, int workers) {
  if (!b) return fail(HLU_ERR_ARG, "NULL batch");
  if (trunc_width != 0 && (trunc_width < 16 || trunc_width > 64))
    return fail(HLU_ERR_ARG, "trunc_width must be 0 or in [16, 64]");
  if (workers < 0 || workers > 65536) return fail(HLU_ERR_ARG, "workers must be in [0, 65536]");
  b->tune = trunc_width;
  b->workers = workers;
  if (b->dev) {
    for (size_t i = 0; i < b->hs.size(); ++i) {
      const uint64_t at = b->off_parts + i * sizeof(hlu::DfPart) + offsetof(hlu::DfPart, tune);
      int32_t v = b->tune;
      HIPCHK(hipMemcpy(b->dev + at, &v, 4, hipMemcpyHostToDevice));
    }
  }
  return HLU_OK;
}

hlu_status hlu_batch_factor(hlu_batch b, void* stream) {
  if (!b) return fail(HLU_ERR_ARG, "NULL batch");
  if (!b->dev) return fail(HLU_ERR_STATE, "hlu_batch_bind first");
  for (hlu_handle h : b->hs) {
    if (!h->assembled) return fail(HLU_ERR_STATE, "hlu_assemble first");
    if (h->factored) return fail(HLU_ERR_STATE, "already factored: hlu_reset first");
  }
  hipStream_t s = (hipStream_t)stream;
  int cus = 0;
  long long tps = 0;
  hlu_status st = device_facts(&cus, &tps);
  if (st != HLU_OK) return st;
  if (b->workers > 0) cus = b->workers;
  for (hlu_handle h : b->hs)
    HIPCHK(hlu_launch_set_int((int32_t*)(h->base + h->plan.off_status), 0, s));
  HIPCHK(hlu_launch_dataflow(0, b->dev + b->off_parts, (int)b->hs.size(), (int*)(b->dev + b->off_queue),
                             (const int*)(b->dev + b->off_ready0), (int)b->ready0.size(),
                             (int*)(b->dev + b->off_ctrl), (int)b->ntot, 0, 0, cus, 20 * tps,
                             nullptr, s));
  for (hlu_handle h : b->hs) h->factored = true;
  return HLU_OK;
}

hlu_status hlu_batch_sync(hlu_batch b, void* stream) {
  if (!b) return fail(HLU_ERR_ARG, "NULL batch");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  if (!b->dev) return HLU_OK;
  int32_t err = 0;
  HIPCHK(hipMemcpy(&err, b->dev + b->off_ctrl + 8, 4, hipMemcpyDeviceToHost));
  if (err)
    return fail(HLU_ERR_DEVICE, df_error_text(err));
  return HLU_OK;
}

void hlu_batch_destroy(hlu_batch b) { delete b; }

hlu_status hlu_solve(hlu_handle h, const double* b_dev, double* x_dev, int nrhs, int64_t ld,
                     void* stream) {
  if (!h || !b_dev || !x_dev) return fail(HLU_ERR_ARG, "NULL argument");
  if (!h->factored) return fail(HLU_ERR_STATE, "hlu_factor first");
  hlu::Plan& p = h->plan;
  if (p.prm.operation != 0) return fail(HLU_ERR_STATE, "not an LU plan");
  if (nrhs < 1 || nrhs > p.prm.max_nrhs) return fail(HLU_ERR_ARG, "nrhs out of range");
  if (ld < p.n) return fail(HLU_ERR_ARG, "ld < n");
  hipStream_t s = (hipStream_t)stream;
  char* b = h->base;
  const int n = p.n;
  double* Y = (double*)(b + p.off_Y);
  double* X = (double*)(b + p.off_X);
  double* B = (double*)(b + p.off_B);
  const int64_t* perm = (const int64_t*)(b + p.off_perm);
  HIPCHK(hlu_launch_set_int((int32_t*)(b + p.off_nrhs), nrhs, s));
  HIPCHK(hlu_launch_set_int(solve_error_word(h), 0, s));
  HIPCHK(hlu_launch_vec(0, b_dev, ld, B, n, perm, n, nrhs, s));        // B = P b
  HIPCHK(hlu_launch_vec(3, B, n, Y, n, nullptr, n, nrhs, s));          // Y = B
  hlu_status st = run_solve(h, s);
  if (st != HLU_OK) return st;
  HIPCHK(hlu_launch_vec(3, Y, n, X, n, nullptr, n, nrhs, s));          // X = Y
  h->iters = 0;
  h->not_converged = false;
  h->eta_final = 0.0;
  const double tol = h->refine_tol;
  if (tol > 0.0) {
    // Each column is refined until its own backward error meets the
    // tolerance and is left alone afterwards, so a column's result does not
    // depend on the other columns solved with it.
    double* out = (double*)(b + p.off_eta);
    int32_t* active_dev = (int32_t*)(out + 3 * p.prm.max_nrhs);
    std::vector<double> mx(3 * nrhs);
    std::vector<int32_t> active(nrhs);
    int32_t sweep_err = 0;
    for (int it = 0;; ++it) {
      st = run_mv(h, X, B, 1.0, -1.0, Y, nrhs, s);                       // Y = B - A X
      if (st != HLU_OK) return st;
      HIPCHK(hlu_launch_colmax(Y, X, B, n, n, nrhs, out, s));
      HIPCHK(hipMemcpyAsync(mx.data(), out, sizeof(double) * 3 * nrhs, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(&sweep_err, solve_error_word(h), 4, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      // a failed sweep leaves Y undefined: stop refining (hlu_sync reports it)
      if (sweep_err) break;
      double eta = 0.0;
      for (int j = 0; j < nrhs; ++j) {
        double den = h->anorm * mx[3 * j + 1] + mx[3 * j + 2];
        double e = den > 0 ? mx[3 * j] / den : (mx[3 * j] > 0 ? INFINITY : 0.0);
        if (!(e <= INFINITY)) e = INFINITY;  // NaN
        // a column stays converged once it was (its X no longer changes)
        if (it > 0 && !active[j]) e = std::min(e, tol);
        active[j] = e > tol;
        eta = std::max(eta, e);
      }
      if (it < 16) h->eta_hist[it] = eta;
      h->eta_final = eta;
      if (eta <= tol) break;
      if (it >= h->refine_max_iter) { h->not_converged = true; break; }
      HIPCHK(hipMemcpyAsync(active_dev, active.data(), sizeof(int32_t) * nrhs,
                            hipMemcpyHostToDevice, s));
      st = run_solve(h, s);                                              // Y = A_H^{-1} Y
      if (st != HLU_OK) return st;
      // X += Y (active columns); `active` is next written after the stream
      // synchronisation of the following iteration, which follows this copy
      HIPCHK(hlu_launch_axpy_masked(Y, X, n, n, nrhs, active_dev, s));
      h->iters = it + 1;
    }
  }
  HIPCHK(hlu_launch_vec(1, X, ld, x_dev, n, perm, n, nrhs, s));        // x = P^T X
  return HLU_OK;
}

hlu_status hlu_matvec(hlu_handle h, const double* x_dev, double* y_dev, int nrhs, int64_t ld,
                      void* stream) {
  if (!h || !x_dev || !y_dev) return fail(HLU_ERR_ARG, "NULL argument");
  if (!h->assembled) return fail(HLU_ERR_STATE, "hlu_assemble first");
  hlu::Plan& p = h->plan;
  if (p.prm.operation != 0) return fail(HLU_ERR_STATE, "not an LU plan");
  if (nrhs < 1 || nrhs > p.prm.max_nrhs) return fail(HLU_ERR_ARG, "nrhs out of range");
  if (ld < p.n) return fail(HLU_ERR_ARG, "ld < n");
  hipStream_t s = (hipStream_t)stream;
  char* b = h->base;
  const int n = p.n;
  double* X = (double*)(b + p.off_B);
  double* Y = (double*)(b + p.off_Y);
  const int64_t* perm = (const int64_t*)(b + p.off_perm);
  HIPCHK(hlu_launch_vec(0, x_dev, ld, X, n, perm, n, nrhs, s));
  hlu_status st = run_mv(h, X, nullptr, 0.0, 1.0, Y, nrhs, s);
  if (st != HLU_OK) return st;
  HIPCHK(hlu_launch_vec(1, Y, ld, y_dev, n, perm, n, nrhs, s));
  return HLU_OK;
}

hlu_status hlu_sync(hlu_handle h, void* stream, hlu_info* out) {
  if (!h) return fail(HLU_ERR_ARG, "NULL handle");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipStreamSynchronize(s));
  hlu_info inf;
  std::memset(&inf, 0, sizeof(inf));
  int32_t df_error = 0;
  if (h->base) {
    int32_t st = 0;
    HIPCHK(hipMemcpy(&st, h->base + h->plan.off_status, 4, hipMemcpyDeviceToHost));
    if (st > 0) inf.info = h->plan.perm[st - 1] + 1;
    HIPCHK(hipMemcpy(&df_error, h->base + h->plan.off_df_ctrl + 8, 4, hipMemcpyDeviceToHost));
    if (!df_error)
      HIPCHK(hipMemcpy(&df_error, solve_error_word(h), 4, hipMemcpyDeviceToHost));
  }
  inf.iters = h->iters;
  for (int i = 0; i < 16; ++i) inf.eta_hist[i] = h->eta_hist[i];
  inf.eta_final = h->eta_final;
  if (h->factored && h->base && !h->plan.fsched.ops.empty()) {
    size_t no = h->plan.fsched.ops.size();
    const int R = hlu::kCostRecDoubles;
    std::vector<double> c(no * R);
    HIPCHK(hipMemcpy(c.data(), h->base + h->plan.off_cost, no * hlu::kCostRecBytes,
                     hipMemcpyDeviceToHost));
    for (size_t i = 0; i < no; ++i) inf.cap_hits += (int64_t)c[R * i + 2];
    inf.cap_hits += h->asm_cap_hits;
    // ranks of the low-rank blocks live at the start of the work region
    size_t nr = 0;
    for (const auto& b : h->plan.blk) nr += b.kind == 'R';
    std::vector<int32_t> rk(nr);
    if (nr) HIPCHK(hipMemcpy(rk.data(), h->base + h->plan.off_work, nr * 4, hipMemcpyDeviceToHost));
    int64_t mr = 0;
    for (int32_t r : rk) mr = std::max<int64_t>(mr, r);
    inf.max_rank = mr;
  }
  if (out) *out = inf;
  if (df_error)
    return fail(HLU_ERR_DEVICE, df_error_text(df_error));
  if (inf.info) return fail(HLU_ERR_SINGULAR, "zero pivot");
  if (h->not_converged) return fail(HLU_ERR_NOT_CONVERGED, "refinement did not converge");
  return HLU_OK;
}

// Sum of the per-op records of the last factorisation: flops, algorithmic
// bytes and capacity hits, per op type (arrays of length 8).
hlu_status hlu_factor_cost(hlu_handle h, double* flops, double* bytes, int64_t* counts) {
  if (!h || !flops || !bytes || !counts) return fail(HLU_ERR_ARG, "NULL argument");
  if (!h->base) return fail(HLU_ERR_STATE, "hlu_bind first");
  size_t no = h->plan.fsched.ops.size();
  const int R = hlu::kCostRecDoubles;
  std::vector<double> c(no * R);
  if (no)
    HIPCHK(hipMemcpy(c.data(), h->base + h->plan.off_cost, no * hlu::kCostRecBytes,
                     hipMemcpyDeviceToHost));
  for (int t = 0; t < HLU_OP_TYPES; ++t) { flops[t] = 0; bytes[t] = 0; counts[t] = 0; }
  for (size_t i = 0; i < no; ++i) {
    int t = h->plan.fsched.ops[i].type;
    flops[t] += c[R * i];
    bytes[t] += c[R * i + 1];
    counts[t]++;
  }
  return HLU_OK;
}

// Per-op records of the last factorisation in schedule order (8 doubles per
// op) and static op information (type, wave, rows of p0, rows of p1).
hlu_status hlu_factor_records(hlu_handle h, double* recs, int32_t* info) {
  return hlu_schedule_records(h, 0, recs, info);
}

// The same for either schedule (0: factor, 1: solve, whose records hold the
// last solve sweep).
hlu_status hlu_schedule_records(hlu_handle h, int which, double* recs, int32_t* info) {
  if (!h || !recs || !info) return fail(HLU_ERR_ARG, "NULL argument");
  if (which != 0 && which != 1) return fail(HLU_ERR_ARG, "schedule must be 0 or 1");
  if (!h->base) return fail(HLU_ERR_STATE, "hlu_bind first");
  const hlu::Schedule& sc = which ? h->plan.ssched : h->plan.fsched;
  size_t no = sc.ops.size();
  if (no)
    HIPCHK(hipMemcpy(recs, h->base + (which ? h->plan.off_cost_s : h->plan.off_cost),
                     no * hlu::kCostRecBytes, hipMemcpyDeviceToHost));
  for (const auto& w : sc.waves_list)
    for (int q = 0; q < w.count; ++q) {
      const hlu::Op& o = sc.ops[w.start + q];
      int32_t* r = info + 4 * (size_t)(w.start + q);
      r[0] = o.type;
      r[1] = w.wave;
      r[2] = o.p[0].rows;
      r[3] = o.p[1].rows;
    }
  return HLU_OK;
}

// Dependency graph of the factor schedule in schedule order (CSR):
// succ_off (ops+1 int32) and succ (edges int32); returns the edge count in
// *nedges (pass succ = NULL to query it).
hlu_status hlu_factor_graph(hlu_handle h, int32_t* succ_off, int32_t* succ, int64_t* nedges) {
  return hlu_schedule_graph(h, 0, succ_off, succ, nedges);
}

// The op descriptors of a schedule in schedule order (offsets relative to
// the device buffer), the wave of each op and the term table; sizes in
// *nops / *nterms.
hlu_status hlu_schedule_ops(hlu_handle h, int which, void* ops, int32_t* waves, int64_t* nops,
                            void* terms, int64_t* nterms) {
  if (!h || !nops || !nterms) return fail(HLU_ERR_ARG, "NULL argument");
  if (which != 0 && which != 1) return fail(HLU_ERR_ARG, "schedule must be 0 or 1");
  const hlu::Schedule& sc = which ? h->plan.ssched : h->plan.fsched;
  *nops = (int64_t)sc.ops.size();
  *nterms = (int64_t)sc.terms.size();
  if (ops) std::memcpy(ops, sc.ops.data(), sc.ops.size() * sizeof(hlu::Op));
  if (waves)
    for (const auto& w : sc.waves_list)
      for (int q = 0; q < w.count; ++q) waves[w.start + q] = w.wave;
  if (terms) std::memcpy(terms, sc.terms.data(), sc.terms.size() * sizeof(hlu::Term));
  return HLU_OK;
}

hlu_status hlu_schedule_graph(hlu_handle h, int which, int32_t* succ_off, int32_t* succ,
                              int64_t* nedges) {
  if (!h || !nedges) return fail(HLU_ERR_ARG, "NULL argument");
  if (which != 0 && which != 1) return fail(HLU_ERR_ARG, "schedule must be 0 or 1");
  const hlu::Schedule& sc = which ? h->plan.ssched : h->plan.fsched;
  *nedges = (int64_t)sc.succ.size();
  if (succ_off) std::memcpy(succ_off, sc.succ_off.data(), sc.succ_off.size() * 4);
  if (succ) std::memcpy(succ, sc.succ.data(), sc.succ.size() * 4);
  return HLU_OK;
}

// Number of launches per op type in the factor schedule (HLU_OP_TYPES).
hlu_status hlu_factor_batches(hlu_handle h, int64_t* launches) {
  if (!h || !launches) return fail(HLU_ERR_ARG, "NULL argument");
  for (int t = 0; t < HLU_OP_TYPES; ++t) launches[t] = 0;
  for (const auto& b : h->plan.fsched.batches) launches[b.type]++;
  return HLU_OK;
}

hlu_status hlu_export_pivots(hlu_handle h, int32_t* piv, void* stream) {
  if (!h || !piv) return fail(HLU_ERR_ARG, "NULL argument");
  if (!h->base) return fail(HLU_ERR_STATE, "hlu_bind first");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  HIPCHK(hipMemcpy(piv, h->base + h->plan.off_piv, sizeof(int32_t) * h->plan.n, hipMemcpyDeviceToHost));
  return HLU_OK;
}

hlu_status hlu_export_factors(hlu_handle h, double* lhat, double* u, void* stream) {
  if (!h || !lhat || !u) return fail(HLU_ERR_ARG, "NULL argument");
  if (!h->base) return fail(HLU_ERR_STATE, "hlu_bind first");
  const hlu::Plan& p = h->plan;
  const int n = p.n;
  if (p.prm.operation != 0) return fail(HLU_ERR_STATE, "not an LU plan (use hlu_export_result)");
  if (n > 8192) return fail(HLU_ERR_ARG, "n too large for a dense export");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  std::vector<char> w(p.size_work);
  HIPCHK(hipMemcpy(w.data(), h->base + p.off_work, p.size_work, hipMemcpyDeviceToHost));
  std::vector<int32_t> piv(n);
  HIPCHK(hipMemcpy(piv.data(), h->base + p.off_piv, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  std::memset(lhat, 0, sizeof(double) * (size_t)n * n);
  std::memset(u, 0, sizeof(double) * (size_t)n * n);
  const bool mixed = p.prm.mixed;
  for (const auto& b : p.blk) {
    const hlu::Cluster &ct = p.cl[b.t], &cs = p.cl[b.s];
    std::vector<double> M((size_t)b.m * b.n, 0.0);
    if (b.kind == 'F') {
      const double* F = (const double*)(w.data() + (b.offF - p.off_work));
      std::memcpy(M.data(), F, sizeof(double) * M.size());
    } else {
      int k = *(const int32_t*)(w.data() + (b.offRank - p.off_work));
      for (int j = 0; j < b.n; ++j)
        for (int i = 0; i < b.m; ++i) {
          double s = 0;
          for (int l = 0; l < k; ++l) {
            double uu, vv;
            if (mixed) {
              uu = ((const float*)(w.data() + (b.offU - p.off_work)))[i + (size_t)l * b.m];
              vv = ((const float*)(w.data() + (b.offV - p.off_work)))[j + (size_t)l * b.n];
            } else {
              uu = ((const double*)(w.data() + (b.offU - p.off_work)))[i + (size_t)l * b.m];
              vv = ((const double*)(w.data() + (b.offV - p.off_work)))[j + (size_t)l * b.n];
            }
            s += uu * vv;
          }
          M[i + (size_t)j * b.m] = s;
        }
    }
    if (b.t == b.s) {
      // Lhat leaf = P^T L: undo the leaf's row swaps on the unit lower part
      std::vector<double> L((size_t)b.m * b.m, 0.0);
      for (int j = 0; j < b.m; ++j)
        for (int i = 0; i < b.m; ++i) {
          L[i + (size_t)j * b.m] = i > j ? M[i + (size_t)j * b.m] : (i == j ? 1.0 : 0.0);
          u[(ct.off + i) + (size_t)(cs.off + j) * n] = i <= j ? M[i + (size_t)j * b.m] : 0.0;
        }
      // rows of P L: P applies swaps k <-> piv[k] in order; P^T L undoes
      // them in reverse order
      for (int k = b.m - 1; k >= 0; --k) {
        int q = piv[ct.off + k];
        if (q != k)
          for (int j = 0; j < b.m; ++j) std::swap(L[k + (size_t)j * b.m], L[q + (size_t)j * b.m]);
      }
      for (int j = 0; j < b.m; ++j)
        for (int i = 0; i < b.m; ++i) lhat[(ct.off + i) + (size_t)(cs.off + j) * n] = L[i + (size_t)j * b.m];
    } else {
      double* dst = ct.off > cs.off ? lhat : u;
      for (int j = 0; j < b.n; ++j)
        for (int i = 0; i < b.m; ++i) dst[(ct.off + i) + (size_t)(cs.off + j) * n] = M[i + (size_t)j * b.m];
    }
  }
  return HLU_OK;
}

void hlu_destroy(hlu_handle h) { delete h; }

// ---------------------------------------------------------------- test entry points
static hlu_status run_single(const std::vector<hlu::Op>& ops, int type, hipStream_t s) {
  void* d = nullptr;
  HIPCHK(hipMalloc(&d, ops.size() * sizeof(hlu::Op)));
  hipError_t e = hipMemcpyAsync(d, ops.data(), ops.size() * sizeof(hlu::Op), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hlu_launch_ops(type, d, (int)ops.size(), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(d);
  if (e != hipSuccess) return fail(HLU_ERR_DEVICE, hipGetErrorString(e));
  return HLU_OK;
}

hlu_status hlu_getrf_batched(double* a_dev, int32_t* piv_dev, int32_t* info_dev, int b, int count,
                             void* stream) {
  if (!a_dev || !piv_dev || !info_dev) return fail(HLU_ERR_ARG, "NULL argument");
  if (b < 1 || b > 64 || count < 0) return fail(HLU_ERR_ARG, "b must be in [1, 64]");
  if (count == 0) return HLU_OK;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipMemsetAsync(info_dev, 0, sizeof(int32_t) * count, s));
  std::vector<hlu::Op> ops(count);
  for (int i = 0; i < count; ++i) {
    hlu::Op& o = ops[i];
    std::memset(&o, 0, sizeof(o));
    o.type = hlu::OP_GETRF;
    o.p[0].ptr = (uint64_t)(a_dev + (size_t)i * b * b);
    o.p[0].ld = b;
    o.p[0].rows = b;
    o.p[0].cols = b;
    o.p[1].ptr = (uint64_t)(piv_dev + (size_t)i * b);
    o.p[1].rankp = (uint64_t)(info_dev + i);
    o.i0 = 0;
  }
  return run_single(ops, hlu::OP_GETRF, s);
}

hlu_status hlu_truncate_add(double* U_dev, double* V_dev, int32_t* rank_dev, const double* X_dev,
                            const double* Y_dev, int m, int n, int kc, int kx, int cap, double eps,
                            int fixed_rank, void* stream) {
  if (!U_dev || !V_dev || !rank_dev || (kx > 0 && (!X_dev || !Y_dev)))
    return fail(HLU_ERR_ARG, "NULL argument");
  const int w = 64 - cap;   // widest term the stack admits
  if (m < 1 || n < 1 || kc < 0 || kx < 0 || kc > cap || cap < 1 || cap > 32 ||
      kx > 16 * w || fixed_rank < 0 || fixed_rank > cap)
    return fail(HLU_ERR_ARG, "sizes out of range");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hlu_launch_set_int(rank_dev, kc, s));
  // the update is split into terms of at most w columns; the kernel adds
  // them in passes whose stacked width stays <= 64
  std::vector<hlu::Term> terms;
  for (int c0 = 0; c0 < kx; c0 += w) {
    hlu::Term t;
    std::memset(&t, 0, sizeof(t));
    int cw = std::min(w, kx - c0);
    t.X.ptr = (uint64_t)(X_dev + (size_t)c0 * m);
    t.X.ld = m;
    t.X.rows = m;
    t.X.cols = cw;
    t.Y.ptr = (uint64_t)(Y_dev + (size_t)c0 * n);
    t.Y.ld = n;
    t.Y.rows = n;
    t.Y.cols = cw;
    terms.push_back(t);
  }
  hlu::Op o;
  std::memset(&o, 0, sizeof(o));
  o.type = hlu::OP_TRUNC;
  o.p[0].ptr = (uint64_t)U_dev;
  o.p[0].rankp = (uint64_t)rank_dev;
  o.p[0].ld = m;
  o.p[0].rows = m;
  o.p[0].cols = cap;
  o.p[1].ptr = (uint64_t)V_dev;
  o.p[1].rankp = (uint64_t)rank_dev;
  o.p[1].ld = n;
  o.p[1].rows = n;
  o.p[1].cols = cap;
  o.i0 = 0;
  o.i1 = (int)terms.size();
  o.i2 = cap | (fixed_rank << 16);
  o.d0 = eps;
  if (terms.empty()) return HLU_OK;
  void* d = nullptr;
  const size_t bytes = sizeof(hlu::Op) + terms.size() * sizeof(hlu::Term);
  HIPCHK(hipMalloc(&d, bytes));
  o.p[2].ptr = (uint64_t)((char*)d + sizeof(hlu::Op));
  hipError_t e = hipMemcpyAsync(d, &o, sizeof(o), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync((char*)d + sizeof(hlu::Op), terms.data(), terms.size() * sizeof(hlu::Term),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hlu_launch_ops(hlu::OP_TRUNC, d, 1, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(d);
  if (e != hipSuccess) return fail(HLU_ERR_DEVICE, hipGetErrorString(e));
  return HLU_OK;
}

// The same truncated addition without any allocation: the descriptor and
// its term table are written by a kernel into the library's static device
// scratch (hlu_static_scratch), and everything runs asynchronously on the
// stream.  Calls that overlap on one device share that scratch.
hlu_status hlu_truncate_add_noalloc(double* U_dev, double* V_dev, int32_t* rank_dev,
                                    const double* X_dev, const double* Y_dev, int m, int n,
                                    int kc, int kx, int cap, double eps, int fixed_rank,
                                    void* stream) {
  if (!U_dev || !V_dev || !rank_dev || (kx > 0 && (!X_dev || !Y_dev)))
    return fail(HLU_ERR_ARG, "NULL argument");
  const int w = 64 - cap;
  if (m < 1 || n < 1 || kc < 0 || kx < 0 || kc > cap || cap < 1 || cap > 32 ||
      kx > 16 * w || fixed_rank < 0 || fixed_rank > cap)
    return fail(HLU_ERR_ARG, "sizes out of range");
  const size_t nterms = (size_t)(kx + w - 1) / w;
  const size_t need = sizeof(hlu::Op) + nterms * sizeof(hlu::Term);
  if (need > hlu_static_scratch_bytes())
    return fail(HLU_ERR_ARG, "update needs " + std::to_string(need) +
                                 " bytes of descriptors, above the static scratch of " +
                                 std::to_string(hlu_static_scratch_bytes()) + " bytes");
  hipStream_t s = (hipStream_t)stream;
  void* scr = nullptr;
  HIPCHK(hlu_static_scratch(&scr));
  HIPCHK(hlu_launch_set_int(rank_dev, kc, s));
  if (kx == 0) return HLU_OK;
  HIPCHK(hlu_launch_build_trunc(scr, U_dev, V_dev, rank_dev, X_dev, Y_dev, m, n, kx, w, cap, eps,
                                fixed_rank, s));
  HIPCHK(hlu_launch_ops(hlu::OP_TRUNC, scr, 1, s));
  return HLU_OK;
}

}  // extern "C"
