/*
 * rlb -- right-looking blocked (RLB) supernodal sparse Cholesky, A = L L^T,
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Karsavuran, Ng, Peyton, Peyton, "Some new techniques to use in
 * serial sparse Cholesky factorization algorithms" -- the RLB factorization of
 * Section 2.2.2 (Algorithm 5), preceded by the symbolic steps of Section 2.1.2
 * and Section 3.1 (ordering, supernodes, merging, reordering within
 * supernodes) and followed by the forward/backward solves of step 4 of the
 * solution process (Section 1).
 *
 * Conventions
 *  - rlb_status is int32: 0 = success, negative = error (RLB_ERR_*),
 *    positive k = the matrix is not positive definite: the pivot of column k
 *    (1-based, factored order) is not positive. Columns 1..k-1 of L are valid.
 *  - Input matrices are the LOWER triangle (diagonal included) in CSC form
 *    with 0-based int64 indices, rows strictly ascending in every column, the
 *    diagonal present in every column, no duplicates. Values are FP64.
 *  - Host pointers are marked (host); device pointers (device). Device work is
 *    enqueued on the caller's HIP stream (a hipStream_t passed as void*); no
 *    call synchronizes except where stated. A device pointer may be NULL
 *    when its buffer holds no element (n = 0, nrhs = 0 or no entries); the
 *    matrix of order 0 goes through every call.
 *  - Handles are not thread-safe; one handle must not be used from two host
 *    threads at once.
 *  - Errors leave outputs unspecified; rlb_last_error() returns a message.
 */
#ifndef RLB_H
#define RLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rlb_status;

#define RLB_OK 0
#define RLB_ERR_ARG (-1)            /* bad argument or option value */
#define RLB_ERR_PATTERN (-2)        /* malformed CSC (unsorted, duplicate, upper, missing diagonal) */
#define RLB_ERR_ALLOC (-3)          /* host or device allocation failed */
#define RLB_ERR_WORKSPACE (-4)      /* caller workspace too small */
#define RLB_ERR_HIP (-5)            /* a HIP runtime call failed */
#define RLB_ERR_STATE (-6)          /* handle not in a state for this call (e.g. factor failed) */
#define RLB_ERR_NOT_CONVERGED (-7)  /* refinement did not reach the tolerance */
#define RLB_ERR_UNSUPPORTED (-8)    /* option combination not implemented */

/* Orderings (step 1 of the solution process, Section 1). */
#define RLB_ORDER_NATURAL 0
#define RLB_ORDER_GRID_ND 1 /* geometric nested dissection on grid[] */
#define RLB_ORDER_USER 2
#define RLB_ORDER_GRAPH_ND 3 /* nested dissection of the adjacency graph: level-structure
                                bisection from pseudo-peripheral roots, components apart
                                (general sparse input; no grid needed) */

/* Arithmetic of the bulk SYRK/GEMM updates (POTRF and TRSM are FP64 always). */
#define RLB_PREC_FP64 0
#define RLB_PREC_FP32_UPDATES 1 /* SYRK/GEMM operands in FP32, FP32 accumulation */
#define RLB_PREC_BF16_UPDATES 2 /* operands BF16 with per-panel power-of-two scales */
#define RLB_PREC_FP16_UPDATES 3 /* operands FP16 with per-panel power-of-two scales */

typedef struct rlb_options {
  int32_t struct_size;      /* sizeof(rlb_options) */
  int32_t ordering;         /* RLB_ORDER_* */
  const int64_t* user_perm; /* (host) perm[new] = old, for RLB_ORDER_USER */
  int64_t grid[4];          /* nx, ny, nz, dofs per node, for RLB_ORDER_GRID_ND;
                               node (x,y,z) dof d is index d + dofs*(x + nx*(y + ny*z)) */
  double merge_cap;         /* supernode merging stops before storage grows by more
                               than this fraction (Section 3.1: 0.125); 0 = no merging */
  int32_t reorder;          /* 1 = partition-refinement reordering inside supernodes
                               (Section 1, Fig. 2; Section 3.1), 0 = none */
  int32_t maximal_blocks;   /* 1 = merge contiguous GEMM blocks (Alg. 5, "maximal") */
  int32_t precision;        /* RLB_PREC_* used by rlb_numeric_create */
  int32_t panel_spread;     /* panel launches with more 64-row tiles than this give a
                               workgroup several consecutive row tiles; 0 = 512 */
  int32_t deterministic;    /* 1 (default): no floating-point atomics in the
                               factorization -- every target tile of an update launch has
                               one owner that sums its contributions in a fixed order, so
                               repeated factorizations of the same values give the same
                               bits, and a batch gives each matrix the bits of its own
                               factorization; 0: tiles with many contributions are cut
                               into parts added atomically (rounding order varies) */
  int32_t outer_block;      /* columns of the outer block of wide supernodes: the
                               trailing columns right of an outer block are updated once,
                               with inner dimension outer_block, after its last 64-column
                               panel; a multiple of 64; 0 = 256; 64 = after every panel */
  int32_t big_tile_min;     /* the long updates of a step (trailing updates by an outer
                               block, updates into ancestors) take 128x128 target tiles
                               when there are at least this many; <= 0 (default): never
                               (on the grid workloads the 64x64 tiles are faster) */
  int32_t method;           /* RLB_METHOD_RLB (default): Algorithm 5, every update written
                               straight into the ancestors' storage; RLB_METHOD_RL:
                               Algorithm 4 (Section 2.2.1), each supernode's updates
                               formed in an update matrix U_J (working storage after the
                               factor in the workspace) and assembled into the ancestors
                               through relative indices (one writer per target column,
                               a fixed order); RLB_METHOD_HYBRID: per step, the RL route
                               for the supernodes whose rectangles meet many more 64x64
                               target tiles than U_J has (a cost model of the planner),
                               Algorithm 5 for the rest. The two others are FP64 only
                               and not batched */
  int32_t tile_order;       /* target tiles of an update launch of its own:
                               RLB_TILE_ORDER_WEIGHT (0): heaviest first, dealt round-robin
                               to the XCDs as dispatched; RLB_TILE_ORDER_XCD (1): in 8x8
                               blocks of neighbouring tiles of each target supernode, and
                               each XCD takes a contiguous eighth of that order, so the
                               tiles running on one XCD (one L2) share their source rows */
  int32_t tall_tile_min;    /* the long updates of a step (updates into ancestors, and the
                               trailing update after an outer block) take 128x64 target
                               tiles in the FP64 form when there are at least this many;
                               <= 0: never (the other forms run the same work in 64x64
                               tiles) */
  double hybrid_step_us;    /* RLB_METHOD_HYBRID: the time (microseconds, by the planner's
                               model) the update-matrix route must save in a step to be
                               taken there; 0 (default): 30, about the step's two extra
                               launches; < 0: any saving */
  int32_t split_chunks;     /* deterministic form: an update launch lasts at least as long
                               as its heaviest target tile, which one workgroup sums.
                               0 (default): no tile is cut; every update is written
                               straight into its target (Alg. 5: no floating-point
                               working storage). < 0: in a launch whose heaviest tile
                               holds more than twice its balanced share of 16-deep K
                               chunks (its chunks over min(tiles, 1024 resident
                               workgroups)), the tiles above that share are cut along
                               their contribution list into parts of about half the
                               share; each part writes its sum into a 64x64 block of the
                               workspace (factor_bytes counts them) and a reduce launch
                               adds the parts into the tile in part order, so repeated
                               factorizations stay bitwise equal. > 0: every tile of more
                               chunks than this, in parts of this many */
} rlb_options;

#define RLB_TILE_ORDER_WEIGHT 0
#define RLB_TILE_ORDER_XCD 1

#define RLB_METHOD_RLB 0
#define RLB_METHOD_RL 1
#define RLB_METHOD_HYBRID 2

typedef struct rlb_info {
  int64_t n, nnz_a;
  int64_t n_supernodes, n_fundamental, n_levels;
  int64_t nnz_exact;     /* entries of L in the exact structure of the final order */
  int64_t nnz_stored;    /* entries of L in supernodal storage (lower trapezoids) */
  double flops_exact;    /* sum over columns of (column count)^2, exact structure */
  double flops_padded;   /* the same over the stored (supernodal) structure */
  int64_t n_blocks;      /* blocks of all supernodes (Section 2.2.2) */
  int64_t n_pairs;       /* (J, ancestor P) update pairs */
  int64_t n_calls;       /* SYRK + GEMM block updates of Alg. 5 */
  int64_t merge_added, merge_base; /* merging: added stored entries, fundamental entries */
  int64_t factor_bytes;  /* device workspace needed by rlb_factor (FP64 factor storage,
                            and for RL its update-matrix working storage after it) */
  int64_t n_panel_tiles;  /* workgroups of all panel launches */
  int64_t n_update_tiles; /* target tiles of all update launches */
  int64_t n_merged_tiles; /* target tiles that sum contributions of several supernodes */
  int64_t n_split_tiles;  /* update workgroups of tiles cut for load balance (atomic adds,
                             or deterministic parts summed by a reduce launch) */
  int64_t n_launches;
  double flops_tiles;    /* flops the update kernels execute (16x16 MFMA blocks touched) */
  double flops_upd_alg;  /* algorithmic flops of the updates: 2 * inner dimension *
                            entries written, summed over contributions */
  double flops_panel;    /* flops of the panel (POTRF + TRSM) steps */
  double flops_upd_launch; /* the part of flops_upd_alg run by update launches of their
                              own (the rest runs inside panel launches) */
  int64_t u_bytes;       /* RL: floating-point working storage of the update matrices
                            (part of factor_bytes); 0 for RLB */
} rlb_info;

typedef struct rlb_symbolic_s* rlb_symbolic;
typedef struct rlb_numeric_s* rlb_numeric;

/* Fill *opt with the defaults of the paper: grid ND ordering (grid must still
 * be set), merge cap 0.125, reordering on, maximal blocks on, FP64; and
 * deterministic = 1. */
rlb_status rlb_default_options(rlb_options* opt);

/* Symbolic phase (host only, no device use): ordering, elimination tree,
 * postorder, fundamental supernodes (Section 2.1.2), merging (Section 3.1),
 * reordering within supernodes (Section 1, Section 3.1), glbind / relind /
 * blocks / relindB (Section 2.1.2, Section 2.2.2), and the device work plan.
 *   n, colptr[n+1], rowidx[colptr[n]] : (host) lower-triangle CSC pattern
 *   opt   : (host) options, may be NULL for defaults with natural ordering
 *   out   : receives a new handle owned by the caller (rlb_symbolic_free)
 * Errors: RLB_ERR_PATTERN, RLB_ERR_ARG, RLB_ERR_ALLOC. */
rlb_status rlb_analyze(int64_t n, const int64_t* colptr, const int64_t* rowidx,
                       const rlb_options* opt, rlb_symbolic* out);

rlb_status rlb_symbolic_info(rlb_symbolic sym, rlb_info* out);

/* Copy one integer array of the analysis into caller memory (host).
 * which: "perm", "perm_nd", "perm_post", "etree_post", "etree", "fund_ptr",
 * "sn_ptr", "sn_parent", "gl_ptr", "gl", "rel_ptr", "rel", "blk_ptr", "blk",
 * "rbp_ptr", "rbp_anc", "rbv_ptr", "rbv", "colcount", "level", "off", "amap",
 * and the device work lists "update_tiles" (7 values per target tile:
 * target offset, ldc, m, n, flags, first contribution, contribution count),
 * "update_segs" (9 per contribution: X and Y source offsets, source ld, k,
 * tile rows [ra, rb), tile columns [ca, cb), source supernode),
 * "diag_tiles" (3 per 64-column step: diagonal offset, ld, nb),
 * "panel_tiles" (11 per workgroup: diagonal offset, ld, nb, nrows, row0,
 * column, status slot, group counter, group size, first row below the
 * diagonal block, number of 64-row tiles from row0) and "launches" (12 per
 * launch: kind 0 panel (POTRF+TRSM) / 1 update, level, step, first tile, tile
 * count, variant, pre, ustart, ucount, ncount, alt_start, alt_count). If out is NULL only *len is set. All arrays are returned as int64. */
rlb_status rlb_symbolic_array(rlb_symbolic sym, const char* which, int64_t* out, int64_t* len);

void rlb_symbolic_free(rlb_symbolic sym);

/* Upload the work plan of `sym` to the current HIP device. The numeric handle
 * borrows `sym`, which must outlive it. precision: RLB_PREC_*. In every form
 * the 64x64 diagonal-tile POTRF, the panel TRSM, the factor storage and the
 * solves are FP64; the reduced forms change the operands of the SYRK/GEMM
 * updates (the in-supernode trailing updates and the updates written into
 * ancestors), which accumulate in FP32 and are added to FP64 targets. The
 * FP32 form keeps an FP32 copy of the finished entries below the diagonal
 * tiles (a library buffer of factor_bytes / 2), from which the updates read
 * their operands.
 * Errors: RLB_ERR_HIP, RLB_ERR_ALLOC, RLB_ERR_ARG. */
rlb_status rlb_numeric_create(rlb_symbolic sym, int32_t precision, rlb_numeric* out);

/* Numeric factorization (Alg. 5): A-load, then per level of the supernodal
 * elimination tree the cdiv (POTRF + TRSM) of every supernode and its
 * SYRK/GEMM updates written directly into ancestor storage.
 *   values    : (device) FP64 values of the analysed CSC, in its entry order
 *   workspace : (device) caller-owned buffer of >= info.factor_bytes bytes,
 *               8-byte aligned; receives the factor and must stay alive and
 *               unmodified while `num` is used for solves
 *   stream    : hipStream_t (void*), may be NULL for the default stream
 * Asynchronous; call rlb_factor_status for the outcome.
 * Errors: RLB_ERR_WORKSPACE, RLB_ERR_ARG, RLB_ERR_HIP. */
rlb_status rlb_factor(rlb_numeric num, const double* values, void* workspace,
                      size_t workspace_bytes, void* stream);

/* Synchronize the factor's stream and return 0 or k > 0 (first non-positive
 * pivot, 1-based column of the factored order); *info receives the same. */
rlb_status rlb_factor_status(rlb_numeric num, int64_t* info);

/* Reduced-precision forms: the number of pivots of the last factorization
 * that fell to u * A_jj or below (u: unit roundoff of the update operands)
 * and were replaced by u * max_i A_ii, so that the FP64 POTRF of the diagonal
 * tile continues; the refinement then works against the patched factor.
 * Always 0 in the FP64 form. Synchronizes the factor's stream.
 * Errors: RLB_ERR_ARG, RLB_ERR_STATE (no factorization enqueued), RLB_ERR_HIP. */
rlb_status rlb_factor_pivots_patched(rlb_numeric num, int64_t* count);

/* Solve A X = B in place with the computed factor (forward solve with L,
 * backward solve with L^T, Section 1 step 4).
 *   B : (device) n x nrhs column-major FP64 in the ORIGINAL order, ld = ldb
 * Uses a library scratch buffer of n*nrhs doubles (allocated on first use).
 * If rlb_factor_status has not been called since the last rlb_factor, the
 * pivot status is read first (this synchronizes the factor's stream once).
 * Errors: RLB_ERR_ARG, RLB_ERR_STATE (no factor, or the last one failed),
 * RLB_ERR_HIP. */
rlb_status rlb_solve(rlb_numeric num, int64_t nrhs, double* B, int64_t ldb, void* stream);

/* rlb_solve without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same forward/backward solve kernels, with their three work
 * vectors in a fixed per-GPU library array of 3 x 2^21 doubles (48 MiB, held
 * by every GPU the library runs on until the process ends) instead of the
 * lazily allocated per-handle buffers. Calls no hipMalloc, hipFree or other
 * allocating routine.
 *   B : (device) n x nrhs column-major FP64, ORIGINAL order, ld = ldb; solved
 *       in place; requires nrhs <= 16 and n * nrhs <= 2^21
 * The handle's device must be current. Every call on one GPU shares that
 * GPU's array (the previous call's contents are overwritten; nothing needs to
 * start at zero): calls that overlap on one GPU -- on different streams or
 * host threads -- race and must be serialized by the caller.
 * Errors: RLB_ERR_ARG (sizes beyond the capacity, bad arguments, wrong
 * device), RLB_ERR_STATE (no factor, or the last one failed), RLB_ERR_HIP. */
rlb_status rlb_solve_noalloc(rlb_numeric num, int64_t nrhs, double* B, int64_t ldb, void* stream);

typedef struct rlb_refine_report {
  int32_t iterations;       /* refinement steps taken after the first solve */
  int32_t converged;        /* 1 if every column reached tol */
  double backward_error[16];/* final ||b - A x||_inf / (||A||_inf ||x||_inf) per column */
  double history[64];       /* max backward error after the first solve and each step */
  int32_t pcg_from;         /* step at which PCG took over, or -1 */
  int32_t reserved;
} rlb_refine_report;

/* Iterative refinement in FP64 on the device (the mixed forms): X = solve(B),
 * then repeat r = B - A X (FP64 residual), d = solve(r), X += d until every
 * column's backward error is <= tol or max_iter steps were taken. When the
 * correction fails to halve (max over columns of ||d||_2) at two steps, the
 * iteration continues as conjugate gradients in FP64 preconditioned by the
 * computed factor (M = L L^T), per column, from the current iterate (residual
 * by recurrence; the stopping test always uses the true residual B - A X, and
 * CG restarts from it when the backward error has not halved in 8 steps).
 *   values : (device) the same FP64 values that were factored (for A X)
 *   B, X   : (device) n x nrhs column-major, ORIGINAL order, ld = ld; nrhs <= 16
 * Like rlb_solve, reads the factor's pivot status first if it has not been
 * read. Returns RLB_ERR_NOT_CONVERGED (X holds the last iterate) if tol is not
 * met, RLB_ERR_STATE if the last factorization failed. */
rlb_status rlb_refine(rlb_numeric num, const double* values, int64_t nrhs, const double* B,
                      double* X, int64_t ld, double tol, int32_t max_iter, void* stream,
                      rlb_refine_report* rep);

/* Backward error ||B - A X||_inf / (||A||_inf ||X||_inf) per column (device
 * FP64 residual; synchronizes). ||A||_inf is formed from `values` on every
 * call. out: (host) nrhs doubles. */
rlb_status rlb_backward_error(rlb_numeric num, const double* values, int64_t nrhs,
                              const double* B, const double* X, int64_t ld, void* stream,
                              double* out);

/* Copy the factor out of factor storage into a host CSC with the stored
 * supernodal structure (final order): colptr[n+1], rowidx, vals sized by
 * info.nnz_stored. Synchronizes. For tests and inspection. */
rlb_status rlb_factor_export(rlb_numeric num, int64_t* colptr, int64_t* rowidx, double* vals);

void rlb_numeric_free(rlb_numeric num);

/* Batched form: factor many independent matrices with one merged level
 * schedule (level h of every matrix in the same launches).
 *   count           : number of matrices
 *   syms[count]     : (host) analysed patterns, borrowed: each must outlive
 *                     the batch (its schedules and solves read them)
 *   values[count]   : (host array of device pointers) FP64 values of each
 *   workspace       : (device) >= rlb_batch_bytes() bytes, caller-owned
 * rlb_batch_create builds the merged plan once; rlb_batch_factor runs it and
 * may be called again with new values. Per-matrix status via rlb_batch_status.
 * precision must be RLB_PREC_FP64 (RLB_ERR_UNSUPPORTED otherwise: the reduced
 * forms are single-matrix).
 */
typedef struct rlb_batch_s* rlb_batch;
rlb_status rlb_batch_create(int32_t count, const rlb_symbolic* syms, int32_t precision,
                            rlb_batch* out, int64_t* workspace_bytes);
rlb_status rlb_batch_factor(rlb_batch b, const double* const* values, void* workspace,
                            size_t workspace_bytes, void* stream);
/* info[count] (host): 0 or the failing column of each matrix. Synchronizes. */
rlb_status rlb_batch_status(rlb_batch b, int64_t* info);
/* Solve matrix i of the batch in place (B in its original order). Reads the
 * batch's statuses first if rlb_batch_status has not been called since the
 * last rlb_batch_factor; RLB_ERR_STATE if matrix i's factorization failed. */
rlb_status rlb_batch_solve(rlb_batch b, int32_t i, int64_t nrhs, double* B, int64_t ldb,
                           void* stream);
void rlb_batch_free(rlb_batch b);

/* Level schedule of a batch: which levels of the matrices share a launch.
 * LEAVES aligns every matrix's leaves (level 0 of all matrices together),
 * ROOTS aligns the roots, CENTERED shifts each matrix by half the difference.
 * Every schedule gives the same factors; they differ in launch count and
 * balance. rlb_batch_create starts with LEAVES. Synchronizes the device and
 * drops the captured graph; a factorization already in the workspace stays
 * valid (the factor storage does not depend on the schedule).
 * Errors: RLB_ERR_ARG, RLB_ERR_HIP, RLB_ERR_ALLOC. */
#define RLB_BATCH_SCHED_LEAVES 0
#define RLB_BATCH_SCHED_ROOTS 1
#define RLB_BATCH_SCHED_CENTERED 2
rlb_status rlb_batch_set_schedule(rlb_batch b, int32_t schedule);

/* A merged launch of the batch with at least min_items narrow work items
 * (update tiles and panel members of at most 16 columns) runs them one per
 * wavefront, four per workgroup, instead of one per 256-thread workgroup;
 * min_items <= 0: never. Default 1024. The factor storage does not depend on
 * it. Errors: RLB_ERR_ARG, RLB_ERR_HIP. */
rlb_status rlb_batch_set_narrow_min(rlb_batch b, int64_t min_items);

/* The batch's current level schedule and narrow-item threshold (0: never). */
rlb_status rlb_batch_get_tuning(rlb_batch b, int32_t* schedule, int64_t* narrow_min);

/* Autotune the level schedule and the narrow-item threshold (256, 1024,
 * 4096 or never): factor the batch (same arguments as rlb_batch_factor) once
 * untimed and `reps` times timed with HIP events under each pair, keep the
 * fastest pair. *chosen (may be NULL) receives its schedule and ms (may be
 * NULL, 3 entries) the best mean milliseconds of each schedule; the chosen
 * threshold is read back with rlb_batch_get_tuning. The workspace holds a
 * valid factorization afterwards. Errors: as rlb_batch_factor. */
rlb_status rlb_batch_autotune(rlb_batch b, const double* const* values, void* workspace,
                              size_t ws_bytes, void* stream, int32_t reps, int32_t* chosen,
                              double* ms);

/* Record the factor's launch sequence in a HIP graph on first use and replay
 * it on later rlb_factor / rlb_batch_factor calls with the same buffers. */
rlb_status rlb_set_graph_mode(rlb_numeric num, int32_t on);
rlb_status rlb_batch_set_graph_mode(rlb_batch b, int32_t on);

/* Device time of the dominant kernel family, measured with HIP events on the
 * factor's stream during the last rlb_factor: total ms of the update launches
 * and of the panel launches, and the number of each. Enabled by
 * rlb_set_profiling(num, 1) (adds one event pair per launch). */
rlb_status rlb_set_profiling(rlb_numeric num, int32_t on);
rlb_status rlb_last_profile(rlb_numeric num, double* update_ms, double* panel_ms,
                            int64_t* n_update, int64_t* n_panel);
/* The same profiled factorization launch by launch, in the order of the
 * "launches" array (ms may be NULL; on entry *count is its capacity, on
 * return the number of launches). */
rlb_status rlb_last_profile_launches(rlb_numeric num, double* ms, int64_t* count);

const char* rlb_status_string(rlb_status s);
const char* rlb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RLB_H */
