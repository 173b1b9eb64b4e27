/*
 * hec.h -- C ABI of the HEC level-scheduled triangular-solve library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library implements the method of Chen, Liu and Yang, "Parallel
 * Triangular Solvers on GPU": sparse lower and upper triangular solves on the
 * HEC (hybrid ELL + CSR) format, scheduled by level sets, applied as ILU(0),
 * ILU(k), ILUT, block ILU and Restricted Additive Schwarz preconditioners
 * inside restarted GMRES and BiCGSTAB, plus a device refactorization of
 * ILU(0)/ILU(k) factors and an SOR / Gauss-Seidel smoother on the same solves.
 *
 * Conventions shared by every entry point:
 *  - Indices are int32_t and 0-based.  Host CSR inputs (rowptr[n+1], col[nnz],
 *    val[nnz]) must have each row sorted by strictly ascending column; they are
 *    copied, and the caller keeps ownership.
 *  - Vectors are caller-owned DEVICE pointers on the device that was current
 *    when the handle was created, laid out [n][nrhs] with the right-hand-side
 *    index fastest.  Input and output vectors must not overlap unless a
 *    function says otherwise.
 *  - Every device call takes a hipStream_t and is asynchronous on it, except
 *    krylov_solve, krylov_solve_batch and ilu_refactor, which synchronize the
 *    stream to return their outcome.
 *  - Every function returns hec_status_t; on error the handle outputs are left
 *    untouched and hec_last_error() returns a thread-local description.  No
 *    C++ exception crosses this interface.
 *  - Opaque handles are owned by the library until their *_destroy call.
 *    Destroy functions accept NULL.
 */
#ifndef HEC_H
#define HEC_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hec_status {
    HEC_OK = 0,
    HEC_ERR_INVALID_ARG = 1,    /* bad size, NULL pointer, wrong handle kind */
    HEC_ERR_NOT_TRIANGULAR = 2, /* an entry on the wrong side of the diagonal */
    HEC_ERR_UNSORTED = 3,       /* a row not sorted by strictly ascending column */
    HEC_ERR_MISSING_DIAG = 4,   /* a row without its diagonal (non-unit solve) */
    HEC_ERR_ZERO_PIVOT = 5,     /* a zero or non-finite diagonal / pivot */
    HEC_ERR_ALLOC = 6,          /* host or device allocation failed */
    HEC_ERR_HIP = 7,            /* HIP runtime error; text kept in hec_last_error */
    HEC_ERR_NOT_CONVERGED = 8,  /* Krylov solver hit maxit */
    HEC_ERR_BREAKDOWN = 9,      /* Krylov breakdown (zero inner product) */
    HEC_ERR_CAPACITY = 10,      /* persistent grid larger than co-residency */
    HEC_ERR_TIMEOUT = 11,       /* a device-side wait exceeded its spin limit */
    HEC_ERR_NO_DEVICE = 12      /* handle built host-only, or no GPU */
} hec_status_t;

typedef enum hec_dtype { HEC_F64 = 0, HEC_F32 = 1 } hec_dtype_t;
typedef enum hec_uplo { HEC_LOWER = 0, HEC_UPPER = 1 } hec_uplo_t;

/* How the level sets are executed on the device (all give bit-identical
 * results for the same plan, since every row is computed the same way). */
typedef enum hec_schedule {
    HEC_SCHED_AUTO = 0,              /* the owner schedule on the dataflow kernel when its LDS
                                        holds every part for max_nrhs right-hand sides, else
                                        the system queue, the barrier-free kernel or one
                                        launch per level (see kernel_variant) */
    HEC_SCHED_LEVEL_LAUNCH = 1,      /* one kernel launch per level (Algorithm 2 shape) */
    HEC_SCHED_LEVEL_PERSISTENT = 2,  /* one persistent launch; each level split into
                                        per-workgroup chunks; a chunk polls the values it
                                        reads from other chunks */
    HEC_SCHED_OWNER_PERSISTENT = 3   /* one persistent launch; each workgroup owns a
                                        connected set of rows across all levels and
                                        keeps their solution in LDS */
} hec_schedule_t;

typedef enum hec_ilu_kind { HEC_ILU0 = 0, HEC_ILUK = 1, HEC_ILUT = 2 } hec_ilu_kind_t;
typedef enum hec_krylov { HEC_GMRES = 0, HEC_FGMRES = 1, HEC_BICGSTAB = 2 } hec_krylov_t;
typedef enum hec_precond_kind {
    HEC_PRECOND_NONE = 0, HEC_PRECOND_ILU = 1, HEC_PRECOND_RAS = 2
} hec_precond_kind_t;

/* Tuning knobs for the analysis / execution layout.  Fill with
 * hec_tune_default() and override fields. */
typedef struct hec_tune {
    int32_t ell_width;      /* HEC ELL width w; -1 = smallest w with at most half the
                               rows having more than w off-diagonals */
    int32_t schedule;       /* hec_schedule_t */
    int32_t num_groups;     /* persistent workgroups; 0 = one per compute unit (at most the
                               co-resident capacity; larger requests fail with CAPACITY) */
    int32_t merge_rows;     /* level-merge threshold: a level with fewer rows than this
                               is not split across workgroups */
    int32_t group_lanes;    /* lanes cooperating on one row when a step holds long
                               CSR tails (1, 2, 4, 8, 16, 32 or 64); 0 = auto */
    int32_t long_row;       /* CSR-tail length from which a step is run with
                               group_lanes cooperating lanes per row */
    int32_t part_rows;      /* owner schedule: target rows per owned part (0 = auto) */
    int32_t host_only;      /* 1 = build the host plan only (no device upload) */
    int32_t max_nrhs;       /* workspace is allocated for up to this many RHS (grows on demand);
                               plans run by the dataflow kernel accept at most this many */
    int32_t block_threads;  /* threads per workgroup (64..1024, multiple of 64) */
    int32_t chunk_rows;     /* owner schedule: rows of matrix data staged in LDS per chunk
                               (1, 2 or 4 times block_threads; 0 = the smallest of
                               those that is at least 256) */
    int32_t partition;      /* owner schedule parts: 0 = auto (blocks of a detected
                               structured grid, else contiguous), 1 = contiguous ranges of the
                               problem order, 2 = recursive graph bisection, 3 = grid blocks */
    int32_t kernel_variant; /* persistent kernel: 0 = auto (owner schedule: the dataflow kernel
                               when its LDS fits, else 2; with schedule AUTO the fallback is one
                               launch per level), 1 = generic row-per-thread kernel,
                               2 = owner kernel with LDS-staged chunks, 3 = owner kernel with
                               separate compute and fetch waves (one RHS), 4 = dataflow owner
                               kernel: no per-level barrier, each row waits only for its own
                               inputs; block_threads sets its compute wavefronts (at most 384;
                               two more run beside them); ELL width 1..8, 10, 12 or 16 (others round
                               up; the automatic width covers the longest row, up to 16);
                               max_nrhs at most 64; 5 = barrier-free kernel over the
                               level-ordered layout in global memory (schedule AUTO or
                               LEVEL_LAUNCH): one launch, each (row, rhs) waits only for its
                               own inputs; 6 = the dataflow kernel with more parts than
                               workgroups (schedule AUTO or OWNER_PERSISTENT): every
                               independent system (batch_setup's systems, RAS subdomains, or
                               the whole matrix) is cut into contiguous ranges of its problem
                               order that fit the LDS (part_rows sets a first cut), systems
                               with the most levels first, and the workgroups take parts from
                               a queue in that order: a part reads only from earlier parts,
                               so the solve needs no co-residency (on request only);
                               7 = system queue (schedule AUTO or LEVEL_PERSISTENT): the
                               workgroups take whole independent systems (batch_setup's
                               systems, RAS subdomains, or the whole matrix), largest first,
                               from a queue and solve each level by level with a workgroup
                               barrier between levels, the last levels of the system held in
                               an LDS ring (no co-residency needed).  Without a CSR tail, with
                               ELL width 1..8 (the automatic width covers the longest row up
                               to 8) and a multiple of 4 right-hand sides, a pipelined kernel of 512
                               threads prefetches each level's rows several levels ahead;
                               otherwise block_threads sets the workgroup.
                               Schedule AUTO picks the dataflow kernel when its LDS holds
                               every part, else 7 for at least half as many independent
                               systems as compute units, else 5 unless the levels are very
                               wide (2^20 (row, rhs) items per level on average or more),
                               else one launch per level */
} hec_tune_t;

/* Per-RHS outcome of krylov_solve. */
typedef struct hec_krylov_info {
    int32_t status;          /* HEC_OK (true relative residual <= rtol), HEC_ERR_NOT_CONVERGED
                                (maxit reached) or HEC_ERR_BREAKDOWN (a zero or non-finite
                                scalar or residual stopped this RHS; a b holding a NaN or an
                                infinity is not iterated at all) */
    int32_t iters;           /* Krylov iterations (Arnoldi steps / BiCGSTAB steps) */
    int32_t restarts;        /* completed restart cycles */
    int32_t precond_applies; /* preconditioner applications (GMRES with delayed
                                re-orthogonalization: iters or iters + 1) */
    double relres;           /* final true ||b - A x||_2 / ||b||_2, computed in FP64 (||b - A x||_2
                                for b = 0; NaN when b is not finite) */
} hec_krylov_info_t;

/* Statistics of a triangular plan. */
typedef struct tri_stats {
    int32_t n, nlev, ell_width, ld, num_groups, nsteps, nexport, schedule;
    int64_t nnz_offdiag;     /* stored off-diagonal entries */
    int64_t nnz_tail;        /* off-diagonals in the CSR remainder */
    int64_t lds_rows;        /* largest per-workgroup LDS window, in rows */
    int64_t nremote;         /* dependency entries read across workgroups */
    int32_t unit_diag, dtype;
    int32_t crit_hops;       /* most workgroup-to-workgroup handoffs along one dependency chain */
    int32_t dataflow;        /* 1 when the plan runs on the dataflow owner kernel */
    int32_t syncfree;        /* 1 when the plan runs on the barrier-free global-memory kernel */
    int32_t queue;           /* 1 when the dataflow kernel takes its parts from a queue
                                (num_groups then counts parts, not workgroups) */
    int32_t sysq;            /* 1 when the plan runs on the system-queue kernel (num_groups
                                then counts independent systems) */
} tri_stats_t;

typedef struct hec_matrix_s *hec_matrix_t;
typedef struct tri_plan_s *tri_plan_t;
typedef struct ilu_s *ilu_t;
typedef struct ras_s *ras_t;
typedef struct hec_graph_s *hec_graph_t;

typedef struct hec_precond {
    int32_t kind;   /* hec_precond_kind_t */
    void *handle;   /* ilu_t or ras_t (borrowed) */
} hec_precond_t;

/* Thread-local text of the last error on this thread ("" if none). */
const char *hec_last_error(void);

/* Default tuning: ell_width -1, schedule AUTO, all other knobs auto. */
hec_status_t hec_tune_default(hec_tune_t *tune);

/* ---------------------------------------------------------------------------
 * HEC matrix (Section 2.1): an ELL part of width w stored column-major with
 * leading dimension ld (n rounded up to 64 rows, so each ELL column starts on
 * a 256-byte boundary for the 4-byte indices), padded with value 0 and column
 * n, plus a CSR remainder holding the entries past the first w of each row.
 * This general form backs the Krylov residual b - A x.
 * ell_width: -1 = median row length.  dt: storage type of the values; val
 * points to double (HEC_F64) or float (HEC_F32).
 * ------------------------------------------------------------------------- */
hec_status_t hec_from_csr(int32_t n, const int32_t *rowptr, const int32_t *col, const void *val,
                          hec_dtype_t dt, int32_t ell_width, hec_matrix_t *out);
/* y = A x (FP64 vectors, [n][nrhs]). */
hec_status_t hec_spmv(hec_matrix_t A, const double *x, double *y, int32_t nrhs, hipStream_t stream);
/* Copy the HEC arrays back to host memory.  Pass NULL arrays to query sizes:
 * *width, *ld and *tail_nnz are always written.  ell_col/ell_val hold
 * width*ld entries (column-major), csr_ptr n+1, csr_col/csr_val tail_nnz;
 * ell_val/csr_val are double. */
hec_status_t hec_matrix_export(hec_matrix_t A, int32_t *width, int32_t *ld, int64_t *tail_nnz,
                               int32_t *ell_col, double *ell_val, int32_t *csr_ptr,
                               int32_t *csr_col, double *csr_val);
void hec_matrix_destroy(hec_matrix_t A);

/* ---------------------------------------------------------------------------
 * Triangular plans: Algorithm 1 (preprocessing) of Section 2.2.
 *  1. level of every row by eq. (2) (structural: every stored off-diagonal
 *     entry counts; levels are 1-based);
 *  2. the map m of eq. (3): rows sorted by level, ascending index inside a
 *     level (an upper triangle is first reversed by t(i) = n-1-i, so its rows
 *     inside a level come in descending original index);
 *  3. L reordered to L' (entry order inside a row kept, diagonal last);
 *  4. L' converted to HEC; the first min(w, len-1) off-diagonals of a row go
 *     to ELL, the rest and the diagonal (last) to the CSR remainder, so every
 *     CSR row holds at least one element.
 * The device copy additionally holds the execution layout chosen by the
 * schedule (see hec_schedule_t).
 * uplo: HEC_LOWER needs col <= row for every entry, HEC_UPPER col >= row.
 * unit_diag: 1 = the diagonal is 1 and is neither required nor read.
 * val: double (HEC_F64) or float (HEC_F32); FP32 plans store factors and solve
 * in FP32.  tune may be NULL (defaults).
 * Errors: INVALID_ARG, UNSORTED, NOT_TRIANGULAR, MISSING_DIAG, ZERO_PIVOT,
 * ALLOC, HIP, CAPACITY.
 * ------------------------------------------------------------------------- */
hec_status_t tri_analyze(int32_t n, const int32_t *rowptr, const int32_t *col, const void *val,
                         hec_dtype_t dt, hec_uplo_t uplo, int32_t unit_diag,
                         const hec_tune_t *tune, tri_plan_t *out);
/* Level data of eq. (2)-(3): *nlev; levelptr[nlev+1] (first position of each
 * level); perm[n] (new position -> original row).  Arrays may be NULL. */
hec_status_t tri_plan_info(tri_plan_t plan, int32_t *n, int32_t *nlev, int32_t *levelptr,
                           int32_t *perm);
/* The HEC of L' (level order, paper layout: diagonal last in the CSR part),
 * copied to host; same size-query convention as hec_matrix_export. */
hec_status_t tri_plan_hec(tri_plan_t plan, int32_t *width, int32_t *ld, int64_t *tail_nnz,
                          int32_t *ell_col, double *ell_val, int32_t *csr_ptr, int32_t *csr_col,
                          double *csr_val);
hec_status_t tri_plan_stats(tri_plan_t plan, tri_stats_t *stats);
/* Execution order chosen for the device: xperm[n] (device position -> original
 * row) and the workgroup owning each device position (owner[n]); may be NULL. */
hec_status_t tri_plan_layout(tri_plan_t plan, int32_t *xperm, int32_t *owner);

/* Profiling hook: while `trace` is non-NULL, persistent launches of this plan
 * write, for workgroup g and its j-th step, the device's constant-rate
 * real-time counter (100 MHz on gfx950, one time base for all CUs) at the
 * step's start and end to trace[2*(g*stride + j)] and trace[2*(g*stride + j) + 1]
 * (uint64, device memory of 2*groups*stride entries owned by the caller); steps
 * beyond `stride` are not recorded.  The dataflow kernel keeps entry stride-1
 * of each workgroup for the times its set-up ended and its last step finished
 * (steps beyond stride-1 are not recorded) and needs 16 bytes of LDS per
 * recorded step.  Pass NULL to stop tracing. */
hec_status_t tri_plan_trace(tri_plan_t plan, void *trace, int32_t stride);

/* Bounded waits.  Every device-side wait of a persistent launch (a row's
 * input from another workgroup or wavefront) gives up after a number of
 * polls; the launch then raises the plan's abort flag, every workgroup exits,
 * the output of that launch is unspecified, and the next call on the plan
 * (tri_solve_*, ilu_apply, ras_apply, krylov_solve, or tri_plan_check)
 * returns HEC_ERR_TIMEOUT and clears the flag, so the call after it runs
 * normally.  tri_plan_set_wait_limit sets the plan's limit in polls (0 = the
 * default 2^22, about a second; at most 2^27): a smaller limit detects a hung
 * solve sooner, and a limit of a few polls makes any wait give up (to test a
 * caller's handling of the TIMEOUT path).  Errors: INVALID_ARG.
 * tri_plan_check reports (and clears) an abort of an earlier launch without
 * launching anything: call it after synchronizing the stream to learn whether
 * the last solve completed.  Returns HEC_OK or HEC_ERR_TIMEOUT. */
hec_status_t tri_plan_set_wait_limit(tri_plan_t plan, uint32_t polls);
hec_status_t tri_plan_check(tri_plan_t plan);

/* Solve L x = b (Algorithm 2): b is gathered into level order, the levels are
 * solved in order with all rows of a level computed simultaneously, and x is
 * scattered back to the original order.  b, x: device, [n][nrhs] of vec_dt
 * (HEC_F64 or HEC_F32; FP64 vectors with an FP32 plan are converted on load and
 * store).  Errors: INVALID_ARG (plan kind, sizes), NO_DEVICE, HIP, TIMEOUT
 * (reported by the next call on the plan, since the solve is asynchronous). */
hec_status_t tri_solve_lower(tri_plan_t L, const void *b, void *x, int32_t nrhs, hec_dtype_t vec_dt,
                             hipStream_t stream);
/* Solve U x = b; the plan was built from U reversed by t(i) = n-1-i. */
hec_status_t tri_solve_upper(tri_plan_t U, const void *b, void *x, int32_t nrhs, hec_dtype_t vec_dt,
                             hipStream_t stream);
void tri_plan_destroy(tri_plan_t plan);

/* ---------------------------------------------------------------------------
 * ILU preconditioners (Section 3): the host factors A (ILU(0): A's pattern;
 * ILU(k): level-of-fill k; ILUT(p, tol): dual dropping with tol relative to the
 * row's 2-norm and at most p entries in each of L and U) into a unit lower L
 * and an upper U, and builds the two triangular plans.  factor_dt = HEC_F32
 * rounds the FP64 factors once to FP32.
 * Errors: as tri_analyze, plus ZERO_PIVOT from the factorization.
 * ------------------------------------------------------------------------- */
hec_status_t ilu_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                       hec_ilu_kind_t kind, int32_t k, double tol, int32_t p,
                       hec_dtype_t factor_dt, const hec_tune_t *tune, ilu_t *out);
/* Copy a factor (which = 0: L with its unit diagonal stored last in each row;
 * 1: U, diagonal first) to host in FP64.  Pass NULL arrays to query *nnz. */
hec_status_t ilu_factor(ilu_t ilu, int32_t which, int64_t *nnz, int32_t *rowptr, int32_t *col,
                        double *val);
/* Borrowed plan handles of L and U (destroyed with the ilu). */
hec_status_t ilu_plans(ilu_t ilu, tri_plan_t *L, tri_plan_t *U);
/* z = (LU)^{-1} r by eq. (1): L y = r, then U z = y; y never leaves the device
 * and stays in level order between the two solves.  r, z: device [n][nrhs] of
 * vec_dt; r and z may alias. */
hec_status_t ilu_apply(ilu_t ilu, const void *r, void *z, int32_t nrhs, hec_dtype_t vec_dt,
                       hipStream_t stream);
/* ilu_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solves, with the intermediate vector and the U solve's workspace
 * in a fixed 64 MiB device array of the library (one per GPU, held until the
 * process ends) instead of the handle's workspace, and no hipMalloc, hipFree
 * or other allocating call.  The handle's own per-plan state (mailboxes,
 * counters) is used as sized at setup, so nrhs must not exceed the handle's
 * max_nrhs.  Needs 2 * ceil256((n + 1) * nrhs * s) bytes of the array
 * (s = 8 for FP64 factors, 4 for FP32): n * nrhs up to about 4.19 million
 * with FP64 factors (one 128^3 right-hand side fits), 8.38 million with FP32.
 * Nothing in the array needs to start at any value.  All calls on one GPU
 * share the array: calls that overlap in time on one GPU (different streams
 * or threads) race and must be ordered by the caller.
 * Errors: INVALID_ARG (as ilu_apply, or nrhs above max_nrhs), CAPACITY
 * (the sizes above exceed the array), NO_DEVICE, HIP, TIMEOUT. */
hec_status_t ilu_apply_noalloc(ilu_t ilu, const void *r, void *z, int32_t nrhs, hec_dtype_t vec_dt,
                               hipStream_t stream);
void ilu_destroy(ilu_t ilu);
/* Numeric refactorization on the device (Section 3's ILU(0) / ILU(k), computed
 * over the level sets of eq. (2): the rows of one level of L are independent).
 * For a handle from ilu_setup or batch_setup with kind HEC_ILU0 or HEC_ILUK:
 * new values `val` (device FP64 [nnz], in the order of rowptr/col) of a matrix
 * whose pattern (host rowptr[n+1], col[nnz], sorted rows) lies inside the
 * factor pattern built at setup (A's own pattern qualifies) are factored on
 * the device and written into both plans in place; the factors equal those a
 * new setup would compute, bit for bit.  The first call for a pattern builds
 * its device maps (host work); later calls with the same pattern reuse them,
 * and rowptr = col = NULL names the previous call's pattern without comparing.
 * Runs on `stream` and synchronizes it (to report a zero pivot; the plans are
 * then left unchanged).  Solves on other streams must be ordered by the caller.
 * ilu_factor returns the refactored values afterwards.
 * Errors: INVALID_ARG (ILUT handle, NULL arrays, no earlier pattern, an entry
 * outside the factor pattern), ZERO_PIVOT, CAPACITY (a factor row longer than 1024 entries),
 * NO_DEVICE for a host-only setup. */
hec_status_t ilu_refactor(ilu_t ilu, const int32_t *rowptr, const int32_t *col, const double *val,
                          hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Restricted Additive Schwarz (Section 3, eq. (4)): subdomain s owns the rows
 * with owner[i] == s; it is extended by `overlap` rings of graph neighbours in
 * A; A_s = A[ext_s, ext_s] is factored by ILU(0); the block-diagonal
 * diag(L_1..L_s) and diag(U_1..U_s) are solved as one system, with one
 * persistent launch per triangle.  Apply: restrict r to every extended
 * subdomain, solve, and write only owned rows back (restricted prolongation).
 * r, z: device FP64 [n][nrhs]; must not alias.
 * ------------------------------------------------------------------------- */
hec_status_t ras_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                       int32_t nsub, const int32_t *owner, int32_t overlap, hec_dtype_t factor_dt,
                       const hec_tune_t *tune, ras_t *out);
/* Block ILU(k) and block ILUT (Section 3), and RAS with those subdomain
 * factorizations: as ras_setup, but every A_s is factored by `kind` (k: fill
 * level for HEC_ILUK; tol, p: drop tolerance relative to the row's 2-norm and
 * entries kept per row in each of L and U for HEC_ILUT) instead of ILU(0).
 * overlap = 0 gives the block-Jacobi forms (BILU(k), BILUT): every row is in
 * exactly one block and the couplings between blocks are dropped.  The
 * returned handle is a ras_t (ras_apply, ras_info, ras_plans, krylov_solve).
 * Errors: as ras_setup, plus INVALID_ARG for an unknown kind, k < 0, p < 0 or
 * tol < 0. */
hec_status_t ras_setup_ilu(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                           int32_t nsub, const int32_t *owner, int32_t overlap, hec_ilu_kind_t kind,
                           int32_t k, double tol, int32_t p, hec_dtype_t factor_dt,
                           const hec_tune_t *tune, ras_t *out);
hec_status_t ras_apply(ras_t ras, const double *r, double *z, int32_t nrhs, hipStream_t stream);
/* Device refactorization of a RAS / block ILU handle built with ILU(0) or
 * ILU(k) subdomain factors, as ilu_refactor: `val` (device FP64, in the order
 * of A's host pattern rowptr/col) holds new values of A; every subdomain
 * matrix A_s = A[ext_s, ext_s] is gathered from them on the device and
 * refactored over its fixed pattern, and the plans are rewritten in place
 * (bit-identical to a new setup with these values).  rowptr = col = NULL
 * reuses the previous call's pattern.  Synchronizes `stream`.
 * Errors: INVALID_ARG (ILUT subdomains, NULL arrays, no earlier pattern, an
 * entry of a subdomain matrix missing from A's pattern), ZERO_PIVOT, CAPACITY,
 * NO_DEVICE for a host-only setup. */
hec_status_t ras_refactor(ras_t ras, const int32_t *rowptr, const int32_t *col, const double *val,
                          hipStream_t stream);
/* Extended-subdomain sizes (ext[nsub], may be NULL) and total extended rows. */
hec_status_t ras_info(ras_t ras, int32_t *nsub, int64_t *total_ext, int32_t *ext_sizes);
/* Borrowed plan handles of the block-diagonal L and U. */
hec_status_t ras_plans(ras_t ras, tri_plan_t *L, tri_plan_t *U);
void ras_destroy(ras_t ras);

/* ---------------------------------------------------------------------------
 * Batched independent systems (eq. (4)): the block-diagonal matrix
 * diag(A_1..A_s) given as one CSR of n = sum n_i rows whose rows
 * sys_ptr[i]..sys_ptr[i+1]-1 form system i (no coupling across systems),
 * factored block by block (ILU kind as ilu_setup) and solved with one launch
 * per triangle (or per level, see HEC_SCHED_AUTO) for all systems together.  The
 * returned handle is an ilu_t: ilu_apply, ilu_plans, ilu_factor, krylov_solve
 * and krylov_solve_batch apply.
 * ------------------------------------------------------------------------- */
hec_status_t batch_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                         int32_t nsys, const int32_t *sys_ptr, hec_ilu_kind_t kind, int32_t k,
                         double tol, int32_t p, hec_dtype_t factor_dt, const hec_tune_t *tune,
                         ilu_t *out);

/* ---------------------------------------------------------------------------
 * SOR / Gauss-Seidel smoother (Section 1: Gauss-Seidel smoothers of algebraic
 * multigrid are among the users of triangular solves).  With A = D + L + U
 * (diagonal, strict lower and strict upper parts) a forward sweep is
 *     x <- (D/omega + L)^{-1} (b - (U + (1 - 1/omega) D) x),
 * one HEC SpMV followed by one level-scheduled lower solve (Algorithm 2); a
 * backward sweep exchanges L and U.  omega = 1 is Gauss-Seidel.
 * sor_setup: host CSR A (rows sorted, every diagonal stored and nonzero),
 * 0 < omega < 2; builds the plans of D/omega + L and D/omega + U (tune as
 * tri_analyze; NULL = defaults) and the two SpMV operators, all FP64.  The host
 * arrays are copied.
 * sor_apply: `sweeps` >= 0 sweeps on x in place (x holds the initial guess);
 * symmetric = 0: forward sweeps; 1: forward then backward per sweep (SSOR).
 * b, x: device FP64 [n][nrhs]; must not alias.  Asynchronous on `stream`.
 * Errors: INVALID_ARG (omega outside (0, 2), nrhs < 1, sweeps < 0, aliasing),
 * MISSING_DIAG, ZERO_PIVOT, UNSORTED, NOT_TRIANGULAR as tri_analyze,
 * NO_DEVICE for a host-only setup.
 * ------------------------------------------------------------------------- */
typedef struct sor_s *sor_t;
hec_status_t sor_setup(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, double omega,
                       const hec_tune_t *tune, sor_t *out);
hec_status_t sor_apply(sor_t sor, const double *b, double *x, int32_t nrhs, int32_t sweeps, int32_t symmetric,
                       hipStream_t stream);
void sor_destroy(sor_t sor);

/* ---------------------------------------------------------------------------
 * Restarted Krylov solvers (Section 4 uses restarted GMRES) for A x = b with
 * right preconditioning by M; every RHS is an independent system sharing the
 * operator.  Residual, inner products, norms and updates are FP64 on the
 * device; with an FP32 preconditioner the outer loop is iterative refinement
 * (use HEC_FGMRES).  GMRES/FGMRES(m): classical Gram-Schmidt with one
 * re-orthogonalization, Givens rotations, x updated at the end of each cycle.
 * For nrhs a power of two up to 16 the re-orthogonalization of each basis
 * vector is delayed into the next step (the preconditioner is applied to the
 * once-projected vector and the Hessenberg column is finished one step
 * later), so the last step before convergence applies M once more than the
 * iteration count.
 * BiCGSTAB: van der Vorst's right-preconditioned recurrence.  Convergence is
 * declared on the true residual ||b - A x|| / ||b|| <= rtol.  b, x: device FP64
 * [n][nrhs]; x holds x0 on entry.  info: host array of nrhs entries.
 * A NaN never counts as converged: each RHS stops on its own at a non-finite
 * value, and its x is then left as it was before the step that produced it.
 * Returns HEC_OK if every RHS converged; else BREAKDOWN if any RHS broke
 * down, else NOT_CONVERGED (per-RHS outcome in info); INVALID_ARG and the
 * other codes report an unusable call (info is then not filled).
 * ------------------------------------------------------------------------- */
hec_status_t krylov_solve(hec_matrix_t A, hec_precond_t M, hec_krylov_t method, int32_t m,
                          const double *b, double *x, int32_t nrhs, double rtol, int32_t maxit,
                          hec_krylov_info_t *info, hipStream_t stream);

/* Independent systems solved together (eq. (4) form): A (and M) block-diagonal
 * with blocks sys_ptr[s]..sys_ptr[s+1]-1 (host array of nsys+1 entries, 0 to n;
 * an entry of A coupling two blocks is INVALID_ARG).  Every (system, rhs) pair is
 * its own Krylov problem: its own inner products, Hessenberg matrix, step sizes
 * and stopping test ||b_s - A_s x_s|| / ||b_s|| <= rtol, as if each system were
 * solved alone, while every operator and preconditioner application covers all
 * systems at once.  info: host array of nsys*nrhs entries, entry s*nrhs + k for
 * system s and right-hand side k.  At most 16384 pairs.  Other arguments and
 * errors as krylov_solve. */
hec_status_t krylov_solve_batch(hec_matrix_t A, hec_precond_t M, hec_krylov_t method, int32_t m,
                                int32_t nsys, const int32_t *sys_ptr, const double *b, double *x,
                                int32_t nrhs, double rtol, int32_t maxit, hec_krylov_info_t *info,
                                hipStream_t stream);

/* ---------------------------------------------------------------------------
 * HIP graph of one preconditioner application (kind HEC_PRECOND_ILU or
 * HEC_PRECOND_RAS) on fixed vectors r -> z, captured from the same launches
 * ilu_apply / ras_apply issue, for callers that replay it in a loop.
 * ------------------------------------------------------------------------- */
hec_status_t hec_graph_capture(hec_precond_t M, const void *r, void *z, int32_t nrhs,
                               hec_dtype_t vec_dt, hipStream_t stream, hec_graph_t *out);
hec_status_t hec_graph_launch(hec_graph_t g, hipStream_t stream);
void hec_graph_destroy(hec_graph_t g);

/* ---------------------------------------------------------------------------
 * Autotuner: times candidate execution layouts of the solve L x = b (or
 * U x = b) with nrhs right-hand sides on the current device and writes the
 * fastest tuning to *best (its time per solve in microseconds to *best_us).
 * Candidates, cheapest first: the automatic choice; the dataflow kernel with
 * one part per workgroup for 2, 4 and 6 compute wavefronts (the rows each
 * wavefront walks per level) and automatic, contiguous and bisection parts;
 * the part queue (kernel_variant 6) for 4 and 6 wavefronts and automatic,
 * 1024 and 4096 rows per part; the system queue with 512 and 1024 threads
 * per workgroup; the barrier-free kernel; one launch per level; the
 * level-persistent schedule at two level-merge thresholds; and
 * wider ELL parts when rows overflow the automatic width.  nsys > 0 with
 * sys_ptr[nsys+1] marks independent diagonal blocks (batch_setup's systems,
 * RAS subdomains), as the setups pass them.  max_seconds > 0 stops starting
 * new candidates after that much time (the automatic choice is always
 * timed).  cache_path (may be NULL): a file of JSON lines keyed by a
 * signature of the problem (n, nnz, triangle, unit diagonal, nrhs, type,
 * blocks and the histogram of level sizes); a hit returns the stored tuning
 * without timing anything, a miss appends the new result.  The inputs are
 * those of tri_analyze.  Errors: as tri_analyze, INVALID_ARG for an
 * unwritable cache, CAPACITY when no candidate runs. */
hec_status_t tri_autotune(int32_t n, const int32_t *rowptr, const int32_t *col, const void *val,
                          hec_dtype_t dt, hec_uplo_t uplo, int32_t unit_diag, int32_t nrhs, int32_t nsys,
                          const int32_t *sys_ptr, const char *cache_path, double max_seconds,
                          hipStream_t stream, hec_tune_t *best, double *best_us);

#ifdef __cplusplus
}
#endif
#endif /* HEC_H */
