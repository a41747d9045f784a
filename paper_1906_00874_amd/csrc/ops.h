// Device-visible descriptors of the static H-LU schedule.
//
// The host planner walks the recursive H-LU (the O1.1-O5.5 sequence of the
// paper's Sec. 3.1, with the partitioned solves of Sec. 5.2) once, emits one
// descriptor per primitive operation on dense leaf blocks and on the factor
// panels of low-rank blocks, and groups independent operations of the same
// type into waves.  Every kernel processes one descriptor per workgroup.
#pragma once
#include <stdint.h>

namespace hlu {

enum DType : uint8_t { DT_F64 = 0, DT_F32 = 1 };
enum PKind : uint8_t { PK_MAT = 0, PK_IDENT = 1 };

// A column-major panel (or the transpose of one) in device memory.
// Element (i, j) of the panel is at ptr[i + j*ld] (trans = 0) or
// ptr[j + i*ld] (trans = 1).  cols is static when rankp == 0, otherwise the
// column count is the int32 at rankp (the live rank of a low-rank block or
// the right-hand-side count of a solve).  kind == PK_IDENT stands for the
// rows x rows identity (ptr unused).
struct PRef {
  uint64_t ptr;
  uint64_t rankp;
  int32_t ld;
  int32_t rows;
  int32_t cols;
  uint8_t dt, trans, kind, pad;
};

enum OpType : int32_t {
  OP_GETRF = 0,    // p0: b x b leaf (FP64) in place; p1.ptr: int32 piv[b];
                   // p1.rankp: int32 info word; i0: first row of the leaf
  OP_TRSM_L = 1,   // p0: factored leaf; p2.ptr: piv; p1 := L^{-1} P p1
  OP_TRSM_UT = 2,  // p0: factored leaf; p1 := U^{-T} p1
  OP_TRSM_U = 3,   // p0: factored leaf; p1 := U^{-1} p1
  OP_PGEMM = 4,    // p3 += d0 * op(M) p2; i0 = 0: M dense p0;
                   // i0 = 1: M = p0 p1^T (low-rank); i1: transpose M;
                   // i2 bit 0: p3 := d0 * op(M) p2 (first write of a fresh panel)
  OP_TRUNC = 5,    // C = p0 p1^T (rank at p0.rankp, capacity i2 & 0xffff,
                   // fixed rank i2 >> 16); C := best approx of C - sum X Y^T
                   // over the terms [i0, i0 + i1) of the term table at
                   // p2.ptr (X placed at row xo of C, Y at row yo); d0 = eps
  OP_ADDD = 6,     // p0 (dense FP64) -= p1 p2^T
  OP_ZERO = 7,     // p0 := 0 (static columns)
  OP_MVT = 8,      // solve: p3 (FP64, rows = live cols of p0) := p0^T p2
                   // (i2 = 1: p3 += p0^T p2)
  OP_MVROW = 9,    // solve: p3 += d0 * sum over the terms [i0, i0 + i1) of the
                   // table at p2.ptr of X_t Y_t (X_t: rows of p3 x live cols,
                   // Y_t: FP64 with at least that many rows); i0 = -1: one
                   // term carried in the op, X in p1 and Y in p2; i2 = 1:
                   // then p3 := p0 p3 with the leaf inverse p0 (rows x rows)
  OP_TRINV = 10,   // factor: from the factored leaf p0 (b x b) and its pivots
                   // at p1.ptr, p2 := L^{-1} P and p3 := U^{-1} (FP64, b x b)
  OP_INVAPPLY = 11,  // solve: p1 := p0 p1 (p0: b x b FP64, p1: b x live cols)
  OP_NTYPES = 12
};

// Bytes of the per-op record a kernel writes at Op::cost: doubles {model
// flops, algorithmic bytes, rank-capacity hit, rank, start tick, end tick,
// stack width, detail}; a truncation's detail packs passes * 1e9 + Jacobi
// sweeps * 1e6 + largest Cholesky rank of the left stack * 1e3 + largest
// column count of the SVD core.
constexpr int kCostRecBytes = 64;
constexpr int kCostRecDoubles = kCostRecBytes / 8;

struct Op {
  int32_t type;
  int32_t i0, i1, i2;
  double d0;
  uint64_t cost;   // device address of this op's {flops, bytes} record (0: none)
  PRef p[4];
};

// One low-rank update term of a truncation: C -= X Y^T with X at row xo of
// C and Y at row yo (zero elsewhere).
struct Term {
  PRef X, Y;
  int32_t xo, yo;
  int32_t pad[2];
};

// One schedule of a dataflow run.  Ops, successor lists and in-degrees use
// the schedule's own numbering; the run numbers all ops of all its parts
// consecutively, part i owning [base, base + n).
struct DfPart {
  uint64_t ops;        // const Op[n]
  uint64_t succ_off;   // const int32[n + 1]
  uint64_t succ;       // const int32[edges] (local indices)
  uint64_t indeg0;     // const int32[n]
  uint64_t indeg;      // int32[n], consumed by the run
  int32_t base, n;
  int32_t tune;        // tile shapes of this part's ops: bits 0-7 the widest
                       // stack a truncation pass takes (0: 64)
  int32_t pad;
};

// Device assembly: one block to build from the points.  Dense: its entries
// into U (ld m).  Low-rank: adaptive cross approximation into the FP64
// workspace panels U (m x kmax, ld m) and V (n x kmax, ld n), the rank
// reached written to the int32 at `rank`; the block is then U V^T with
// U's columns negated (the form the truncation that recompresses it into
// the factored copy takes).
struct AsmBlock {
  uint64_t U, V, rank;
  int32_t r0, c0, m, n;
};

// Matvec with the refinement copy: per low-rank block, T = V^T X[s];
// per leaf row cluster, y = b - sum(F X[s]) - sum(U T).
struct MvLR {        // one low-rank block of the matvec copy (FP64)
  uint64_t U, V, T;  // U: m x k (ld m), V: n x k (ld n), T: k x nrhs (ld kcap)
  int32_t m, n, k, kcap;
  int32_t r0, c0;    // first row / column (cluster order)
};
struct MvTerm {      // one contribution to a leaf row cluster
  uint64_t A;        // dense: block pointer (ld = lda); low-rank: U pointer
  uint64_t T;        // low-rank: T of the block (0 for dense)
  int32_t lda;       // leading dimension of A
  int32_t roff;      // row of the leaf inside the block
  int32_t ncol;      // dense: block columns; low-rank: rank
  int32_t c0;        // dense: first column (cluster order); low-rank: kcap (ld of T)
};
struct MvRow {       // one leaf row cluster
  int32_t r0, rows, t0, nt;   // rows [r0, r0+rows); terms [t0, t0+nt)
};

}  // namespace hlu
