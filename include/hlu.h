/*
 * hlu.h -- C-ABI of the MI355X (gfx950) hierarchical-matrix LU library.
 *
 * The library builds an H-matrix for the d=3 Laplace kernel of the paper's
 * BEM problems (Sec. 6.1) from surface points, an admissibility parameter
 * eta and a leaf size (cluster tree: Algorithm 1; block tree: Algorithm 2),
 * factors it with the recursive H-LU (the O1.1-O5.5 sequence of Sec. 3.1,
 * with low-rank arithmetic of Sec. 3.1 "Low-rank blocks"), and solves with
 * the factors, optionally refining the solution against an accurate H-matrix
 * copy of the operator.
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (hipMalloc / torch CUDA
 *    tensors on the current device); every other pointer is host memory.
 *  - Device calls take a hipStream_t (passed as void*) and are asynchronous
 *    on that stream.  Errors the device detects (zero pivots, refinement
 *    that does not converge) surface at hlu_sync.
 *  - Matrices and vectors are FP64, column-major, in the caller's original
 *    point order, with a leading dimension `ld` >= n.
 *  - No exception crosses the ABI; every call returns an hlu_status and
 *    hlu_last_error() gives a thread-local message for the last failure.
 *  - Ownership: host inputs are copied at plan time; the device buffer
 *    passed to hlu_bind belongs to the caller, must stay alive until
 *    hlu_destroy, and is never freed by the library.
 *  - One handle may be used by one host thread at a time; distinct handles
 *    are independent.
 */
#ifndef HLU_H
#define HLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hlu_handle_s* hlu_handle;

/* Number of op types of the schedules (length of the per-type arrays of the
 * diagnostic calls): 0 leaf LU, 1-3 leaf solves (L, U^T, U), 4 panel
 * product, 5 truncation, 6 dense update, 7 zeroing, 8 V^T X, 9 row update,
 * 10 leaf inverses, 11 inverse application. */
#define HLU_OP_TYPES 12

typedef enum {
    HLU_OK = 0,
    HLU_ERR_ARG = 1,            /* invalid argument (NULL, n<1, NaN input, ...) */
    HLU_ERR_NOMEM = 2,          /* bound buffer smaller than hlu_required_bytes */
    HLU_ERR_DEVICE = 3,         /* a HIP runtime call failed */
    HLU_ERR_SINGULAR = 4,       /* zero pivot in a diagonal leaf (info = row) */
    HLU_ERR_NOT_CONVERGED = 5,  /* refinement stopped above refine_tol */
    HLU_ERR_STATE = 6           /* call out of order (e.g. solve before factor) */
} hlu_status;

/* Entries of the collocation matrix for the Laplace kernels of Sec. 6.1
 * between panel midpoints x_i (xyz rows; unused coordinates zero), with the
 * identity added (second-kind form I + V_h):
 *   d = 3, g(x,y) = 1/(4 pi |x-y|), `area` = panel areas:
 *     LAPLACE3D_WEIGHTED: A_ij = area_j / (4 pi |x_i - x_j|) (one-point
 *                         quadrature over panel j)
 *     LAPLACE3D_POINT:    A_ij = 1 / (4 pi |x_i - x_j|)
 *     both: A_ii = 2 sqrt(area_i/pi)/(4 pi) sqrt(pi) + 1;
 *   d = 1, g(x,y) = -log|x-y|, `area` = panel lengths h_j > 0:
 *     LAPLACE1D_LOG: A_ij = -h_j log|x_i - x_j|,
 *                    A_ii = h_i (1 - log(h_i / 2)) + 1 (exact panel integral);
 *   d = 2, g(x,y) = -log|x-y| / (2 pi), `area` = panel lengths h_j > 0:
 *     LAPLACE2D_LOG: A_ij = -h_j log|x_i - x_j| / (2 pi),
 *                    A_ii = h_i (1 - log(h_i / 2)) / (2 pi) + 1.
 * The backward error of hlu_solve takes ||A||_inf as max_i (A_mv 1)_i with
 * the matvec copy, exact when every entry is >= 0 (all d = 3 inputs; d = 1
 * and d = 2 points within unit distance of each other) and a lower bound
 * otherwise, which makes the reported backward error an overestimate;
 * without the copy it is max_i sum_j |A_ij| summed directly. */
typedef enum {
    HLU_KERNEL_LAPLACE3D_WEIGHTED = 0,
    HLU_KERNEL_LAPLACE3D_POINT = 1,
    HLU_KERNEL_LAPLACE1D_LOG = 2,
    HLU_KERNEL_LAPLACE2D_LOG = 3
} hlu_kernel;

/* FP64: all factors and all arithmetic FP64.  MIXED: the factors of
 * low-rank blocks and the H-GEMM product panels are stored in FP32, and the
 * operations that produce them run in FP32: panel products into an FP32
 * panel on the FP32 matrix cores with FP32 accumulation (FP64 near-field
 * operands rounded to FP32), leaf triangular solves on FP32 panels in FP32,
 * and the low-rank part of dense-block updates as an FP32 matrix-core
 * product subtracted in FP64.  Diagonal-leaf LU and pivoting, the dense
 * near field, the truncation (FP64 Gram, Cholesky and SVD core from the
 * FP32 panels) and the refinement residual stay FP64. */
typedef enum { HLU_PREC_FP64 = 0, HLU_PREC_MIXED = 1 } hlu_precision;

/* What hlu_factor computes.  LU: the H-LU factorisation (Sec. 3.1).
 * PRODUCT and INVERSE: the other H-arithmetic operations on the same kernels,
 * on a doubled H-matrix over two copies of the points, M = [M11 M12; M21
 * M22], every quadrant on the original block tree (2n unknowns):
 *   PRODUCT: M12 = A (kernel), M21 = B (kernel_b), M11 = M22 = 0; the
 *     schedule is the H-GEMM M11 -= M12 M21, so M11 = -A B, truncated to
 *     eps_factor / rank_cap_factor like every update of the H-LU;
 *   INVERSE: M11 = A, M12 = M21 = I, M22 = 0; the schedule is the first
 *     steps of the H-LU of M (LU of M11, the two triangular solves on M12
 *     and M21, the Schur-complement update of M22), so
 *     M22 = -M21 U^-1 L^-1 P M12 = -A^-1.
 * Such plans take rank_cap_matvec = 0, host assembly and no refinement;
 * hlu_solve, hlu_matvec and hlu_export_factors refuse them
 * (HLU_ERR_STATE). */
typedef enum { HLU_OP_LU = 0, HLU_OP_PRODUCT = 1, HLU_OP_INVERSE = 2 } hlu_operation;

typedef struct {
    hlu_kernel kernel;
    double eta;               /* admissibility: min(diam) <= eta * dist (Sec. 2) */
    int leaf_size;            /* C_lf of Algorithm 1: split while size > C_lf   */
    int fixed_rank;           /* > 0: every truncation keeps this rank          */
    double eps_factor;        /* truncation tolerance of the factored copy,
                                 in [1e-8, 1) unless fixed_rank > 0            */
    int rank_cap_factor;      /* rank capacity of the factored copy (<= 32)     */
    double eps_matvec;        /* tolerance of the refinement operator copy      */
    int rank_cap_matvec;      /* rank capacity of that copy (<= 64); 0: no copy
                                 (then the refinement residual, hlu_matvec and
                                 ||A||_inf are summed directly over the exact
                                 entries on the device: O(n^2 nrhs) work)      */
    hlu_precision precision;
    double refine_tol;        /* backward-error target of hlu_solve (0: no IR)  */
    int refine_max_iter;      /* at most this many refinement steps              */
    int max_nrhs;             /* largest nrhs hlu_solve / hlu_matvec will see   */
    uint64_t seed;            /* reserved for randomised construction           */
    int64_t scratch_cap_bytes;/* 0: every H-GEMM temporary has its own region;
                                 > 0: temporaries share a ring of this many
                                 bytes (a region is reused only after every op
                                 touching its previous tenant has run)          */
    int operation;            /* HLU_OP_LU (0): the H-LU of the kernel matrix;
                                 HLU_OP_PRODUCT (1) / HLU_OP_INVERSE (2): see
                                 hlu_export_result                             */
    int kernel_b;             /* HLU_OP_PRODUCT: kernel of the right factor B  */
    int device_assembly;      /* 0: hlu_plan assembles the blocks on the host
                                 (cross approximation + QR/SVD recompression)
                                 and hlu_assemble uploads them; 1: hlu_plan
                                 builds trees, layout and schedules only, and
                                 hlu_assemble builds every block on the device
                                 (requires rank_cap_matvec = 0)               */
} hlu_params;

typedef struct {
    int64_t info;             /* first zero pivot (1-based, original order) or 0 */
    int iters;                /* refinement steps taken by the last solve        */
    double eta_hist[16];      /* backward error per refinement step              */
    double eta_final;
    int64_t cap_hits;         /* truncations that hit the rank capacity          */
    int64_t max_rank;         /* largest rank in the factored copy               */
} hlu_info;

/* Plan statistics (host side, available right after hlu_plan). */
typedef struct {
    int64_t n, leaves, dense_blocks, lowrank_blocks;
    int64_t ops_factor, waves_factor, ops_solve, waves_solve;
    double flops_factor_model;   /* model flops at capacity ranks (upper bound) */
    int64_t bytes_factor_region, bytes_matvec_region, bytes_scratch, bytes_total;
    int64_t offset_scratch;      /* byte offset of the scratch region in the buffer */
} hlu_plan_stats;

/* Build the cluster tree and block tree for n points (xyz: n x 3 row-major,
 * area: n, host), assemble all blocks on the host (dense near field exactly;
 * far-field blocks by adaptive cross approximation followed by QR + SVD
 * recompression to eps_factor and eps_matvec), and build the static op
 * schedule of the factorisation, the solve and the matvec.
 * Returns HLU_ERR_ARG for NULL pointers, n < 1, non-finite input, leaf < 1,
 * eta < 0, caps outside [1,32] / [1,64], max_nrhs outside [1,64], or
 * eps_factor below 1e-8 without fixed_rank (the device truncation forms FP64
 * Gram matrices of the stacked factors, which resolve singular values only
 * down to about 1e-8 of the largest). */
hlu_status hlu_plan(const double* xyz, const double* area, int64_t n,
                    const hlu_params* p, hlu_handle* out);

/* Device bytes the handle needs (factor copy, pristine copy, matvec copy,
 * scratch, schedules and solve workspace).  0 for a NULL handle. */
size_t hlu_required_bytes(hlu_handle h);

/* Bind a caller-owned device buffer of at least hlu_required_bytes bytes
 * (256-byte aligned) and upload the schedules.  HLU_ERR_NOMEM if too small. */
hlu_status hlu_bind(hlu_handle h, void* dev_ptr, size_t bytes);

/* Host assembly (device_assembly = 0): copy the H-matrix assembled by
 * hlu_plan (factor copy, its pristine copy and the matvec copy) into the
 * bound buffer on `stream`.  Device assembly (device_assembly = 1): build
 * it on the device from the points -- dense blocks entry by entry, every
 * admissible block by adaptive cross approximation with partial pivoting
 * (to eps/10, at most 64 terms) recompressed by the truncation of
 * Sec. 3.1's truncated addition to eps_factor and rank_cap_factor -- then
 * keep the pristine copy.  Both compute ||A||_inf and synchronise the
 * stream before returning.  Requires hlu_bind.  Cross approximations that
 * stop at 64 terms are counted in hlu_info.cap_hits. */
hlu_status hlu_assemble(hlu_handle h, void* stream);

/* Restore the factor copy from the pristine copy (device-to-device). */
hlu_status hlu_reset(hlu_handle h, void* stream);

/* A second handle over the same plan (cluster tree, block tree, schedules
 * and host images are shared, read-only, not copied): it needs a buffer of
 * its own (hlu_bind) and is filled either by hlu_assemble or, without any
 * host-to-device traffic, by hlu_assemble_from.  Executor, graph and worker
 * settings are copied.  Clones and the original may be used concurrently on
 * different streams; each is destroyed by hlu_destroy (the plan lives until
 * the last one is gone). */
hlu_status hlu_clone(hlu_handle src, hlu_handle* out);

/* Fill h's bound buffer from the assembled handle src of the same plan: the
 * factor copy and its pristine copy from src's pristine copy, and the
 * matvec copy, device to device on `stream`.  src's pristine and matvec
 * copies are only read (src may be factoring meanwhile).  HLU_ERR_ARG if
 * the two do not share a plan, HLU_ERR_STATE if h is unbound or src is not
 * assembled. */
hlu_status hlu_assemble_from(hlu_handle h, hlu_handle src, void* stream);

/* Replace the assembled blocks of the factored copy (and of its pristine
 * copy, so hlu_reset restores them) by the blocks of an H-matrix built
 * elsewhere on the same cluster and block trees (Algorithms 1 and 2), e.g.
 * by the CPU oracle, so that two factorisations of one A_H can be compared
 * (test path).  Synchronous (the null stream); the handle must be bound and
 * assembled (the refinement operator copy and ||A||_inf stay the handle's
 * own); afterwards the handle is unfactored.
 * File (host path, little-endian):
 *   char magic[8] = "HLUBLK01"; int64 n; int64 nblocks;
 *   int64 perm[n]              cluster position -> original point index
 *   nblocks times: int64 r0, c0, m, nc, kind, k
 *                  (rows r0..r0+m-1 and columns c0..c0+nc-1 in cluster
 *                  order; kind 0 dense, 1 low-rank of rank k)
 *     dense:    double F[m*nc] column-major
 *     low-rank: double U[m*k], double V[nc*k] column-major (block = U V^T)
 * Returns HLU_ERR_ARG when the file cannot be read, its permutation, block
 * set, shapes or kinds differ from the handle's trees, or a rank exceeds
 * rank_cap_factor; HLU_ERR_STATE when unbound or unassembled. */
hlu_status hlu_import_blocks(hlu_handle h, const char* path);

/* After hlu_factor on a PRODUCT or INVERSE plan: the result (A B, or A^-1)
 * expanded densely in the original point order into host memory (out:
 * n x n column-major, leading dimension ld >= n, n <= 16384).  Synchronous.
 * HLU_ERR_STATE for an LU plan or before hlu_factor. */
hlu_status hlu_export_result(hlu_handle h, double* out, int64_t ld);

/* Diagnostic: write the factored copy's blocks as they are on the device
 * (after hlu_assemble: the assembled A_H; after hlu_factor: the L and U
 * blocks in place) to a host file in the format hlu_import_blocks reads,
 * FP32 factors widened to FP64.  Synchronous.  HLU_ERR_STATE when unbound,
 * HLU_ERR_ARG when the file cannot be written. */
hlu_status hlu_export_blocks(hlu_handle h, const char* path);

/* Tile shape of this handle's factorisation by the dataflow executor
 * (hlu_set_executor(h, 1)): trunc_width is the widest stacked factor pair a
 * truncation pass takes (the K of its Gram, Cholesky and SVD core tiles;
 * Sec. 3.1 truncated addition), 0 for the default of 64, otherwise in
 * [16, 64].  The rank rule is unchanged; a narrower stack means more passes
 * over smaller cores, so results agree with the default within the
 * truncation tolerance rather than bit for bit.  Chosen per workload by the
 * autotuner (paper_1906_00874_amd/autotune.py). */
hlu_status hlu_set_tuning(hlu_handle h, int trunc_width);

/* Workgroups of the dataflow executor for this handle's factor and solve
 * launches: 0 (the default) one per compute unit; a smaller count leaves
 * compute units to launches of other handles on other streams. */
hlu_status hlu_set_workers(hlu_handle h, int workers);

/* Scheduling of the factorisation by the dataflow executor (the early start
 * of each operation once its own predecessors are done, Secs. 4-5; the
 * priorities are this library's refinement of it).  From the op records of
 * the last factorisation of h (durations, plus a fixed hand-off per
 * dependency edge), every op's slack against the longest path L is
 * computed; ops with predecessors and slack <= slack_frac * L are flagged
 * near-critical and from then on go to a second ready ring that
 * high_workers workgroups serve exclusively.  high_workers = 0 clears the
 * flags (one ring).  The flags live in h's device buffer (bit 30 of each
 * op's initial in-degree); batched launches ignore them.  *n_flagged
 * (optional) receives the number of flagged ops.  HLU_ERR_STATE if h is
 * unbound or, with high_workers > 0, not factored since its last reset;
 * HLU_ERR_ARG for slack_frac outside [0, 1] or high_workers outside
 * [0, 1024].  Synchronises the device. */
hlu_status hlu_set_priorities(hlu_handle h, double slack_frac, int high_workers,
                              int32_t* n_flagged);

/* H-LU of the factor copy in place (Sec. 3.1 sequence, recursive), one
 * launch per kernel type per wave of the static schedule.  Zero pivots are
 * recorded on the device and reported by hlu_sync. */
hlu_status hlu_factor(hlu_handle h, void* stream);

/* enable != 0 (the default): hlu_factor and the solves replay a HIP graph
 * of the schedule (built on first use, one kernel node per wave); 0: one
 * launch per wave from the host.  Both execute the same kernels in the same
 * order. */
hlu_status hlu_set_graph(hlu_handle h, int enable);

/* Executor of hlu_factor.  0 (the default): one launch per wave of the
 * static schedule.  1: one persistent launch that runs each op as soon as
 * its own predecessors in the dependency graph have finished (a device-side
 * dataflow executor: the analogue of nested tasks with weak dependencies and
 * early release, Sec. 5.2).  Both give bitwise identical factors.  A wait in
 * the dataflow executor that exceeds 20 s raises an error flag that makes
 * every workgroup exit; hlu_sync then returns HLU_ERR_DEVICE. */
hlu_status hlu_set_executor(hlu_handle h, int mode);

/* hlu_factor with a HIP event pair around every launch on `stream`;
 * returns the summed launch durations (ms) and launch counts per op type
 * (arrays of HLU_OP_TYPES).  Synchronises the stream; used for roofline
 * figures. */
hlu_status hlu_factor_profile(hlu_handle h, void* stream, double* ms_per_type,
                              int64_t* launches_per_type);

/* Batched factorisation of independent matrices: the union of the handles'
 * factor schedules (the recursive H-LU of Sec. 3.1 for each matrix) run by
 * one launch of the persistent dataflow executor, so ops of every matrix
 * share the machine as soon as their own predecessors are done.
 *
 * hlu_batch_create: host only; `hs` are planned handles, each listed at most
 * once (a handle's in-degree counters are consumed by the run, so a handle
 * must not be factored elsewhere while its batch runs).  The batch copies
 * the handle list; the handles must outlive it.
 * hlu_batch_required_bytes: device bytes of the batch workspace (part table,
 * queue over all ops, initial ready list).
 * hlu_batch_bind: caller-owned, 256-byte aligned device buffer; every handle
 * must already be bound.  Synchronous.
 * hlu_batch_factor: every handle assembled and not factored (hlu_reset in
 * between); asynchronous on `stream`.  Zero pivots are reported per handle
 * by hlu_sync(h).
 * hlu_batch_sync: waits for `stream`; HLU_ERR_DEVICE if the executor
 * stopped on its time limit or a queue overflow. */
typedef struct hlu_batch_s* hlu_batch;
hlu_status hlu_batch_create(const hlu_handle* hs, int count, hlu_batch* out);
size_t hlu_batch_required_bytes(hlu_batch b);
hlu_status hlu_batch_bind(hlu_batch b, void* dev_ptr, size_t bytes);
hlu_status hlu_batch_factor(hlu_batch b, void* stream);
hlu_status hlu_batch_sync(hlu_batch b, void* stream);
void hlu_batch_destroy(hlu_batch b);

/* Tile shape and launch width of a batch's later launches: trunc_width as in
 * hlu_set_tuning (0: 64) for every matrix of the batch, workers the number
 * of persistent workgroups (0: one per compute unit).  Synchronous when the
 * batch is bound.  HLU_ERR_ARG for values outside those ranges. */
hlu_status hlu_batch_set_tuning(hlu_batch b, int trunc_width, int workers);

/* x = A^{-1} b for nrhs right-hand sides (b_dev, x_dev: n x nrhs, leading
 * dimension ld, original order; they may alias).  With refine_tol > 0 the
 * solution is refined with FP64 residuals of the matvec copy (without a
 * copy: of the exact matrix by direct summation) until the
 * backward error max_j |r_j|_inf / (|A|_inf |x_j|_inf + |b_j|_inf) <=
 * refine_tol (this call then synchronises the stream once per step).  Each
 * column is corrected only while its own backward error exceeds refine_tol,
 * so a column's result is the same whatever other columns share the call.
 * HLU_ERR_STATE before hlu_factor; HLU_ERR_ARG if nrhs > max_nrhs. */
hlu_status hlu_solve(hlu_handle h, const double* b_dev, double* x_dev, int nrhs,
                     int64_t ld, void* stream);

/* Refinement settings of this handle's later hlu_solve calls (initially
 * refine_tol / refine_max_iter of its parameters): refine_tol = 0 gives the
 * plain solve with the factors.  HLU_ERR_ARG for refine_tol < 0 or
 * refine_max_iter outside [0, 15]. */
hlu_status hlu_set_refinement(hlu_handle h, double refine_tol, int refine_max_iter);

/* y = A_mv x with the matvec copy (original order, n x nrhs); without a
 * copy, y = A x with the exact entries by direct summation. */
hlu_status hlu_matvec(hlu_handle h, const double* x_dev, double* y_dev, int nrhs,
                      int64_t ld, void* stream);

/* Wait for the stream work of this handle and report device-side status:
 * HLU_ERR_DEVICE if the dataflow executor stopped (time limit or queue
 * overflow) in the last factorisation or in any solve sweep of the last
 * hlu_solve, else HLU_ERR_SINGULAR (info set), else HLU_ERR_NOT_CONVERGED
 * from the last solve. */
hlu_status hlu_sync(hlu_handle h, void* stream, hlu_info* out);

/* Host-side check of the schedules and matvec tables (every panel inside
 * the buffer at full capacity, operand shapes consistent).  hlu_bind runs
 * it too and refuses to bind an invalid plan.  HLU_ERR_ARG on failure. */
hlu_status hlu_validate(hlu_handle h);

/* Plan statistics. */
hlu_status hlu_get_stats(hlu_handle h, hlu_plan_stats* out);

/* Per-op-type totals of the last factorisation (arrays of HLU_OP_TYPES,
 * indexed by op type as listed at HLU_OP_TYPES): model flops, algorithmic
 * bytes and op counts, summed from the records each kernel writes.
 * Synchronous. */
hlu_status hlu_factor_cost(hlu_handle h, double* flops, double* bytes, int64_t* counts);

/* Number of kernel launches per op type in the factor schedule
 * (HLU_OP_TYPES int64). */
hlu_status hlu_factor_batches(hlu_handle h, int64_t* launches);

/* Diagnostics: the per-op records of the last factorisation in schedule
 * order (8 doubles per op: model flops, algorithmic bytes, rank-capacity hit,
 * rank, start and end tick of the device wall clock, stack width, detail;
 * a truncation's detail packs passes * 1e9 + Jacobi sweeps * 1e6 + largest
 * left Cholesky rank * 1e3 + largest SVD core width)
 * and static op information (4 int32 per op: type, wave, rows of the first
 * and second operand).  recs: ops_factor*8, info: ops_factor*4.  Synchronous. */
hlu_status hlu_factor_records(hlu_handle h, double* recs, int32_t* info);

/* Diagnostics: the dependency graph of the factor schedule in schedule
 * order as CSR successor lists (succ_off: ops_factor+1 int32, succ: edges
 * int32); *nedges receives the edge count (call with succ == NULL first). */
hlu_status hlu_factor_graph(hlu_handle h, int32_t* succ_off, int32_t* succ, int64_t* nedges);

/* Diagnostics for either schedule (which: 0 factor, 1 solve): the per-op
 * records (as hlu_factor_records; the solve's hold its last sweep) and the
 * dependency graph (as hlu_factor_graph). */
hlu_status hlu_schedule_records(hlu_handle h, int which, double* recs, int32_t* info);
hlu_status hlu_schedule_graph(hlu_handle h, int which, int32_t* succ_off, int32_t* succ,
                              int64_t* nedges);
/* Diagnostics: the op descriptors (struct Op of the kernels' header, offsets
 * relative to the device buffer), the wave of each op (int32) and the term
 * table of a schedule, in schedule order; pass NULL buffers to query the
 * counts. */
hlu_status hlu_schedule_ops(hlu_handle h, int which, void* ops, int32_t* waves, int64_t* nops,
                            void* terms, int64_t* nterms);

/* Cluster-order permutation: perm[p] = original index of position p (host
 * array of n int64). */
hlu_status hlu_get_perm(hlu_handle h, int64_t* perm);

/* Export the factor copy (after hlu_factor, or the assembled one before) as
 * a dense n x n column-major FP64 host array in cluster order: the lower
 * part holds Lhat (diagonal leaf blocks P^T L), the upper part U, so
 * A_H ~= Lhat * U.  For n <= 8192 only; synchronises the stream. */
hlu_status hlu_export_factors(hlu_handle h, double* lhat, double* u, void* stream);

/* Export the diagonal leaf pivots (n int32, 0-based row within the leaf,
 * LAPACK order) after hlu_factor; synchronises the stream. */
hlu_status hlu_export_pivots(hlu_handle h, int32_t* piv, void* stream);

/* Release host-side state.  Never frees the caller's device buffer. */
void hlu_destroy(hlu_handle h);

/* Message for the last failing call on this thread ("" if none). */
const char* hlu_last_error(void);

/* ---- single-kernel entry points used by the kernel parity tests -------- */

/* Batched LU with partial pivoting of `count` dense b x b column-major FP64
 * blocks stored back to back (a_dev: count*b*b), pivots to piv_dev
 * (count*b int32, 0-based LAPACK order) and the first zero pivot of each
 * block (1-based, 0 if none) to info_dev (count int32).  b in [1, 64]. */
hlu_status hlu_getrf_batched(double* a_dev, int32_t* piv_dev, int32_t* info_dev,
                             int b, int count, void* stream);

/* Best low-rank approximation of C - X Y^T (Sec. 3.1, truncated addition):
 * U (m x kc), V (n x kc) hold C = U V^T on entry (kc <= cap <= 32); X
 * (m x kx), Y (n x kx) the update, kx <= 16 (64 - cap) (the update is taken
 * in passes whose stacked width stays <= 64).  On exit U, V (capacity cap
 * columns, leading dimensions m and n) hold the truncated result and
 * *rank_dev its rank; fixed_rank > 0 keeps that rank, otherwise the
 * smallest rank whose discarded singular values have Frobenius norm <=
 * eps times the norm of the sum, capped at cap.  All FP64.  Allocates a
 * device descriptor buffer and synchronises the stream before returning. */
hlu_status hlu_truncate_add(double* U_dev, double* V_dev, int32_t* rank_dev,
                            const double* X_dev, const double* Y_dev, int m, int n,
                            int kc, int kx, int cap, double eps, int fixed_rank,
                            void* stream);

/* hlu_truncate_add for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops): the same arguments and
 * result, bit for bit, but no hipMalloc / hipFree or allocating call of any
 * kind and no synchronisation -- it only launches kernels on `stream`.
 * The truncation descriptor and its term table are built by a kernel in a
 * static device array of 4096 bytes (hlu_static_scratch_bytes) that each
 * device holds for the life of the process; an update whose descriptors
 * would not fit returns HLU_ERR_ARG (with kx <= 16 (64 - cap) they always
 * fit).  Every call on one device shares that array and it keeps the last
 * call's contents: calls that overlap on one device (different streams or
 * threads without ordering between them) race and must not be issued. */
hlu_status hlu_truncate_add_noalloc(double* U_dev, double* V_dev, int32_t* rank_dev,
                                    const double* X_dev, const double* Y_dev, int m, int n,
                                    int kc, int kx, int cap, double eps, int fixed_rank,
                                    void* stream);

/* Size in bytes of the static device scratch of hlu_truncate_add_noalloc. */
size_t hlu_static_scratch_bytes(void);

#ifdef __cplusplus
}
#endif
#endif /* HLU_H */
