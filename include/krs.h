/*
 * krs.h — C ABI of the MI355X Krylov-reuse solver library (libkrs.so).
 *
 * The library solves sequences of sparse symmetric positive definite systems
 * A^(k) x^(k) = b^(k) with the augmented preconditioned conjugate gradient
 * method (APCG, Algorithm 1 of Gosselet, Rey & Pebrel, arXiv 1301.7530),
 * and carries an augmentation basis C from one system to the next:
 *   - total reuse (TRKS, Algorithm 2): every search direction is appended;
 *   - selective reuse (SRKS, Algorithm 3): only Ritz vectors whose Ritz
 *     values stagnated between the last two Lanczos steps are appended.
 *
 * Conventions shared by every call:
 *   - Every call returns a krs_status; nothing aborts or throws across the
 *     ABI.  krs_last_error() gives a thread-local message for the last
 *     failure of the calling thread.
 *   - Host inputs are copied before the call returns.  Device inputs are
 *     borrowed until the consuming call returns.  Outputs go to buffers
 *     owned by the caller.
 *   - Handles from *_create are owned by the caller and must be destroyed.
 *   - Indices are 0-based.  Dense blocks are column-major with an explicit
 *     leading dimension.  3x3 blocks are row-major.
 *   - A krs_seq is not thread-safe; distinct sequences may be used from
 *     distinct threads only if they belong to distinct contexts.
 *   - After any error a sequence stays valid and keeps its previous basis
 *     (the solution vector is then undefined).
 */
#ifndef KRS_H
#define KRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KRS_OK = 0,
    KRS_E_INVALID = 1,         /* bad argument or malformed input */
    KRS_E_OOM = 2,             /* device or host allocation failed */
    KRS_E_NOT_SPD = 3,         /* (w, A w) <= 0, (r, z) <= 0 or NaN: operator/preconditioner not SPD */
    KRS_E_COARSE_SINGULAR = 4, /* every basis column was rejected by the rank guard */
    KRS_E_MAXIT = 5,           /* max_iter reached; krs_solve_info is still filled */
    KRS_E_DEVICE = 6,          /* HIP runtime error */
    KRS_E_BUSY = 7,            /* resource temporarily unavailable (server queue full, sequence held by a server) */
    KRS_E_STATE = 8            /* call not valid in the object's current state */
} krs_status;

typedef enum { KRS_FP64 = 0, KRS_MIXED = 1, KRS_FP32 = 2, KRS_FP32_BASIS = 3 } krs_precision;
/* KRS_FP64: every vector, value and reduction in double precision.
 * KRS_MIXED: matrix values, preconditioner and basis (C, A C) stored and
 *   streamed in single precision; Krylov vectors, the iterate, every
 *   reduction, the coarse matrix C^T A C and its factorisation, the Ritz
 *   eigenproblem and periodic true-residual refinement (r = b - A x with the
 *   double-precision matrix, then a coarse re-projection) in double.
 * KRS_FP32: as KRS_MIXED but the Krylov vectors are single precision too
 *   (fewer bytes per iteration, more iterations on ill-conditioned systems).
 * KRS_FP32_BASIS: double-precision operator (matrix values) and vectors;
 *   the basis (C, A C) and the preconditioner stored and streamed in single
 *   precision, with the periodic refinement of KRS_MIXED (it re-projects the
 *   residual, whose C^T r recurrence runs on the rounded A C).  On
 *   ill-conditioned systems, where single-precision matrix values perturb
 *   the low end of the spectrum and cost iterations, this keeps the
 *   iteration count of KRS_FP64 with fewer bytes. */

typedef enum { KRS_REUSE_NONE = 0, KRS_REUSE_TOTAL = 1, KRS_REUSE_SELECTIVE = 2 } krs_reuse;
typedef enum { KRS_PC_JACOBI = 0, KRS_PC_BJACOBI3 = 1 } krs_precond;
/* KRS_PC_JACOBI: M = diag(A).  KRS_PC_BJACOBI3: M = the 3x3 diagonal blocks
 * (requires block == 3). */

typedef enum { KRS_CAP_RESTART = 0, KRS_CAP_FREEZE = 1, KRS_CAP_COST = 2 } krs_cap_policy;
/* With max_basis = n_c_lim > 0:
 * KRS_CAP_RESTART: once the basis reaches n_c_lim columns it is reset to the
 *   initial basis C0 (Algorithm 3, last step).
 * KRS_CAP_FREEZE: columns are appended only while the basis is below
 *   n_c_lim; SRKS appends the smallest selected Ritz values first, TRKS the
 *   first search directions.
 * KRS_CAP_COST: as KRS_CAP_FREEZE, and after each solve its modelled bytes
 *   (iterations x bytes per iteration, krs_solve_info.model_bytes) are
 *   compared with those of the latest solve made with the initial basis
 *   alone; when the recycled columns did not lower them, the basis is reset
 *   to C0 and nothing is appended for the next three systems, six after a
 *   second failed trial in a row, and so on up to 48.  An extension: it
 *   judges the basis after the fact from the measured iteration counts. */

/* max_basis = KRS_NC_LIM_AUTO (SRKS with KRS_CAP_RESTART or KRS_CAP_FREEZE):
 * n_c_lim is set by a complexity analysis (Section 4.4, the remark after
 * Algorithm 3) on the first solve of the sequence, whose iteration count
 * m_0 is taken for every non-augmented system.  Deflating the eigenvectors
 * of the k lowest eigenvalues is modelled as leaving the CG rate of the
 * reduced condition number theta_max / theta_(k+1) (Section 2.2, and the
 * rate of Section 4.3), i.e. m(k) = max(1, m_0 ln sigma_0 / ln sigma_k) with
 * sigma = (sqrt(kappa) - 1) / (sqrt(kappa) + 1) over the distinct Ritz values
 * of that solve, k running over the prefix of the ascending values that
 * passed the stagnation test (ritz_eps: only converged Ritz vectors
 * approximate eigenvectors; further columns are modelled as gaining nothing); each system with k columns is priced at m(k) times the
 * algorithmic bytes of an iteration with k columns plus the rebuild of k
 * columns (the library's byte model), and n_c_lim is the k <= 1024 of least
 * cost.  The value is reported in krs_solve_info.n_c_lim; krs_nc_limit
 * exposes the analysis itself. */
#define KRS_NC_LIM_AUTO (-1)

typedef struct krs_ctx krs_ctx;
typedef struct krs_seq krs_seq;

/* Optional device allocator (e.g. a framework's caching allocator).
 * alloc returns device memory of at least `bytes` usable on `stream` (or
 * NULL); free releases it.  NULL allocator: hipMalloc / hipFree. */
typedef struct {
    void* (*alloc)(void* user, size_t bytes, void* stream);
    void (*free)(void* user, void* ptr, void* stream);
    void* user;
} krs_allocator;

/* Sequence description.  The sparsity pattern is fixed for the whole
 * sequence (the systems differ in their values, Section 3).  block == 1:
 * scalar CSR with nb = n rows; block == 3: BSR with nb = n/3 block rows and
 * 3x3 row-major blocks.  row_ptr has nb+1 entries, col_idx nnzb entries
 * (block columns ascending within a row, diagonal block present).  Both
 * are host pointers, copied by krs_seq_create. */
typedef struct {
    int64_t n;
    int32_t block;
    int64_t nnzb;
    const int64_t* row_ptr;
    const int32_t* col_idx;
    krs_precision precision;
    krs_reuse reuse;
    krs_precond precond;
    krs_cap_policy cap_policy;
    double tol;            /* stop when ||r|| <= tol ||b|| (recursive, then confirmed with the true residual) */
    int32_t max_iter;      /* iterations per solve */
    double ritz_eps;       /* SRKS stagnation tolerance epsilon (Section 4.4), e.g. 1e-14 */
    int32_t max_basis;     /* n_c_lim; 0 = unlimited; KRS_NC_LIM_AUTO: from the complexity analysis */
    int32_t refine_every;  /* mixed: force a true-residual refinement at least every k iterations (0 = off) */
    int32_t history_cap;   /* Krylov vectors kept for SRKS (0 = max_iter); longer runs use the leading part */
    double rank_tol;       /* rank guard: drop a basis column whose Cholesky pivot <= rank_tol * max diag (0 = 1e-6) */
    double refine_drop;    /* mixed: refine when ||r|| fell by this factor since the last refinement
                              (0 = 0.1; negative: only when the recursion has converged).  A
                              replacement that more than doubles ||r|| restarts the direction. */
    int32_t exec_mode;     /* 0: iteration blocks replayed as captured HIP graphs; 1: eager kernel launches */
    int32_t update_rows;   /* block rows per workgroup of the update / projector kernel (0 = about one
                              range per compute unit); fixes the grouping of its partial sums */
    int32_t autotune;      /* 1: when the basis width changed by half, time several update_rows values on
                              the submitted system and keep the fastest (results then depend on the
                              choice in the last bits only) */
    int32_t kernel_flags;  /* bit 0: run the end-of-step reduction (coarse solve, beta, status) as a
                              kernel of its own instead of in the last workgroup of the update kernel;
                              same arithmetic, one more launch per iteration.
                              bit 1: form the next direction as Algorithm 1 writes it, w = z + beta w_old,
                              instead of the default w = z + beta P w_old, which applies the projector
                              P = I - C G^-1 (A C)^T to the old direction as well (the same vector in exact
                              arithmetic, Section 2.1; the default keeps rounding from moving the direction
                              out of the range of P, at no extra pass over memory).
                              bit 2: full reorthogonalisation (Section 2.1 remark, used in the experiments
                              of Section 5.1): each new direction is z made A-orthogonal to every kept
                              earlier direction, w = z - sum_i ((A w_i, z) / (w_i, A w_i)) w_i (classical
                              Gram-Schmidt in the A inner product); the first min(history_cap or max_iter,
                              8192) directions and their products with A are kept (2 n doubles each).
                              KRS_FP64 only; not in fused batches or the server (KRS_E_INVALID).
                              bits 3-6: load schedule of the double-precision block SpMV (same results up
                              to the grouping of the (w, A w) partial sums): bit 3 four blocks of a row in
                              flight instead of two, bit 4 non-temporal loads of the matrix, bits 5-6 the
                              cap on SpMV workgroups (0: 8192, 1: 2048, 2: 4096, 3: 8192).  With bits 3-6
                              all zero, a matrix larger than 256 MiB streams with non-temporal loads, and
                              the double-precision 3x3 SpMV reads the block columns as 16-bit differences
                              from the row when every one fits (same columns, same results).
                              bit 7 (KRS_FP64 only): the Krylov history of z_j kept in single precision,
                              half the memory of a long run; it only forms the Ritz vectors of the
                              recycle (combined in double precision, then A-orthonormalised with the
                              rest of the basis), so every solve still runs in double precision.
                              With non-temporal matrix loads (bit 4, or the default for a matrix larger
                              than 256 MiB) the vectors an iteration writes (A w; x, r, s; w and the
                              Krylov history) go out with non-temporal stores, so that no dirty cache
                              lines are left for the next kernel, which streams the matrix, to write back.
                              bit 8: plain stores instead (the same values). */
    int32_t reselect;      /* SRKS: 0 = keep every Ritz vector that passed the stagnation test;
                              1 = KRS_RESELECT_CLUSTER: drop the central cluster of those values
                              ("clust", Section 4.4), before the cap */
    double cluster_min_frac; /* minimum size of the central cluster as a fraction of the preselected
                                values (0 = 0.2, the paper's one fifth) */
} krs_seq_desc;
/* KRS_RESELECT_CLUSTER (Section 4.4): the values that passed the stagnation
 * test are sorted, the distances between neighbours taken on a log scale,
 * and those distances fitted in least squares by a three-level step
 * function whose middle step covers at least ceil(cluster_min_frac * s) of
 * the s values (the outer steps over the low and high ends, one of them
 * possibly empty); when the middle level is below the outer ones, its
 * values are the central cluster and are not recycled. */
#define KRS_RESELECT_CLUSTER 1

typedef struct {
    int32_t iters;          /* m: products A w performed in the last solve */
    int32_t n_c;            /* basis columns used by the last solve (after the rank guard) */
    int32_t refinements;    /* true-residual refinements performed */
    int32_t selected;       /* last recycle: Ritz values that passed the stagnation test (SRKS) */
    int32_t dropped;        /* last solve: basis columns dropped by the rank guard */
    int32_t added;          /* last recycle: columns appended */
    int32_t status;         /* krs_status of the last solve */
    int32_t update_rows;    /* block rows per update workgroup used by the last solve */
    double rel_res_true;    /* ||b - A x|| / ||b|| with double-precision A and x */
    double rel_res_recursive;
    double t_setup_ms;      /* value intake and preconditioner setup */
    double t_rebuild_ms;    /* A C, C^T A C, factorisation, initialisation */
    double t_iter_ms;       /* iterations (including refinements) */
    double t_recycle_ms;    /* Ritz extraction / selection / basis update */
    int64_t model_bytes;    /* algorithmic HBM bytes of the iterations of the last solve */
    int32_t n_c_lim;        /* cap in force: max_basis, the value set by KRS_NC_LIM_AUTO, 0 if none (-1: not yet set) */
    int32_t reserved;
} krs_solve_info;

/* ------------------------------------------------------------- context */
/* Bind to HIP device `device` and stream `hip_stream` (a hipStream_t; NULL
 * = a stream created and owned by the context).  `a` may be NULL. */
krs_status krs_ctx_create(int device, void* hip_stream, const krs_allocator* a, krs_ctx** out);
/* Fails with KRS_E_STATE while sequences created on it are alive. */
krs_status krs_ctx_destroy(krs_ctx* ctx);
const char* krs_status_str(krs_status s);
const char* krs_last_error(void);
const char* krs_version(void);

/* ------------------------------------------------------------ sequence */
/* Create a sequence.  C0 (host, n x m0, leading dimension ldc0 >= n, may be
 * NULL when m0 == 0) is the initial basis C^(0) of Algorithms 2 and 3. */
krs_status krs_seq_create(krs_ctx* ctx, const krs_seq_desc* desc, const double* C0, int32_t m0, int64_t ldc0,
                          krs_seq** out);
/* Load system k: `values` holds nnzb*block*block doubles in the order of
 * the pattern given at creation, `b` holds n doubles.  Host pointers,
 * copied.  Builds the preconditioner. */
krs_status krs_seq_submit(krs_seq* s, const double* values, const double* b);
/* Same with device pointers, borrowed until the call returns. */
krs_status krs_seq_submit_device(krs_seq* s, const double* d_values, const double* d_b);
/* Solve the submitted system with APCG(A, M, C, b) (Algorithm 1): rebuild
 * A C and C^T A C for the current basis, initialise x0 = C (C^T A C)^-1 C^T b,
 * iterate.  x (host, n doubles) receives the solution; info may be NULL.
 * Returns KRS_E_MAXIT (info filled) when max_iter is reached. */
krs_status krs_seq_solve(krs_seq* s, double* x, krs_solve_info* info);
/* Same, writing the solution to device memory d_x (n doubles). */
krs_status krs_seq_solve_device(krs_seq* s, double* d_x, krs_solve_info* info);
/* Update the basis from the last solve: TRKS concatenation (Algorithm 2)
 * or SRKS Ritz selection (Algorithm 3), then the cap policy.  n_added may
 * be NULL. */
krs_status krs_seq_recycle(krs_seq* s, int32_t* n_added);
/* Ritz values of the last SRKS extraction (Section 4.1: eigenvalues of the
 * Lanczos tridiagonal built from the CG coefficients; descending, m of them)
 * and the selection flags (1 = passed the stagnation test of Section 4.4,
 * Algorithm 3).  cap = array sizes; with a capped basis only the part of
 * the spectrum scanned to fill it is reported (m_out says how much). */
krs_status krs_seq_ritz(krs_seq* s, double* theta, uint8_t* selected, int32_t cap, int32_t* m_out);
/* CG coefficients of the last solve (Algorithm 1; the Lanczos tridiagonal
 * of Section 4.1 is built from them): alpha_j, rho_j = (r_j, z_j) and
 * gamma_j = (w_j, A w_j) for j < m.  Any pointer may be NULL. */
krs_status krs_seq_coeffs(krs_seq* s, double* alpha, double* rho, double* gamma, int32_t cap, int32_t* m_out);
/* Export the preconditioned projected residuals z_0 .. z_{m'-1} of the last
 * solve kept in the Krylov history (SRKS only; the vectors Algorithm 3
 * stores to build the Ritz vectors, Section 4.4), as doubles, n x m'
 * column-major with leading dimension ldz.  m' (m_out) is the number kept:
 * at most the iteration count, less when the history reservation was
 * shorter, 0 when no history was kept (TRKS, plain PCG, a full frozen
 * basis).  Z may be NULL to query m'.  Valid until the next solve. */
krs_status krs_seq_history(krs_seq* s, double* Z, int64_t ldz, int32_t cap, int32_t* m_out);
/* Export the current augmentation basis C^(k) of Algorithms 2 and 3 (n x
 * n_c, column-major, leading dim ldc) as doubles; C may be NULL to query n_c
 * only.  After a solve the columns are the A-orthonormalised ones (same
 * span as the carried basis). */
krs_status krs_seq_basis(krs_seq* s, double* C, int64_t ldc, int32_t cap, int32_t* n_c);
/* krs_seq_basis for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, result and errors, but the double-precision staging of
 * each column lives in a static 32 MiB device array (one per GPU, held until
 * the process ends) instead of a library allocation, so the call makes no
 * hipMalloc/hipFree or other allocating call.  n * 8 bytes must fit the
 * array (n <= 4,194,304), else KRS_E_INVALID with the limit in the message.
 * Every call on one GPU shares that array: calls that overlap in time on one
 * GPU (other threads, other contexts of the same device) race and must be
 * serialised by the caller.  Synchronous like krs_seq_basis. */
krs_status krs_seq_basis_noalloc(krs_seq* s, double* C, int64_t ldc, int32_t cap, int32_t* n_c);
krs_status krs_seq_info(krs_seq* s, krs_solve_info* info);
/* Live kernel timing.  When enabled, every 32nd iteration the SpMV + (w, A w)
 * kernel (0), the update / preconditioner / projector-reduction kernel (1)
 * and the coarse-correction / direction kernel (2) record the span from
 * their first workgroup's start to their last workgroup's end with the
 * device wall clock, during the normal (graph-replayed) iterations.
 * Enabling resets the sums.  krs_seq_kernel_time returns the number of
 * sampled launches of `kernel` and their total duration in milliseconds. */
krs_status krs_seq_set_timing(krs_seq* s, int32_t enable);
krs_status krs_seq_kernel_time(krs_seq* s, int32_t kernel, int64_t* launches, double* total_ms);
krs_status krs_seq_destroy(krs_seq* s);

/* --------------------------------------------------------------- batch */
/* Solve the submitted systems of `count` distinct sequences of ctx
 * together.  Sequences with the same precision and block size are fused:
 * each iteration is one launch per kernel covering the workgroups of every
 * member still iterating (members that finish drop out of the launches),
 * replayed as captured HIP graphs.  Every member keeps the launch geometry
 * of its own solve, so each result equals, bit for bit, the one
 * krs_seq_solve gives for that sequence alone.  x[i] (host, n_i doubles;
 * NULL or a NULL entry: not copied) and info[i] (may be NULL) receive the
 * results.  Returns the first non-OK member status (KRS_E_MAXIT only when
 * no member failed otherwise); every member's info is filled. */
krs_status krs_batch_solve(krs_ctx* ctx, krs_seq* const* seqs, int32_t count, double* const* x, krs_solve_info* info);
/* As krs_batch_solve with device output pointers d_x[i] (n_i doubles). */
krs_status krs_batch_solve_device(krs_ctx* ctx, krs_seq* const* seqs, int32_t count, double* const* d_x,
                                  krs_solve_info* info);
/* krs_seq_recycle for `count` distinct sequences of ctx, their host-side
 * Ritz analysis on parallel threads.  n_added[i] (may be NULL) receives
 * each count; returns the first non-OK status (every member is attempted). */
krs_status krs_batch_recycle(krs_ctx* ctx, krs_seq* const* seqs, int32_t count, int32_t* n_added);
/* krs_batch_solve_device followed by krs_batch_recycle, with the host-side
 * Ritz analysis of a member (Section 4.1; selection of Section 3 or 4.4)
 * started as soon as that member has finished, while the others still
 * iterate.  d_x[i] (device, n_i doubles; NULL or a NULL entry: not copied),
 * info[i] and n_added[i] (each may be NULL) receive the results; the same
 * results as the two calls in sequence.  Returns as krs_batch_solve. */
krs_status krs_batch_solve_recycle(krs_ctx* ctx, krs_seq* const* seqs, int32_t count, double* const* d_x,
                                   krs_solve_info* info, int32_t* n_added);

/* ------------------------------------------------------------- serving */
/* A server owns a worker thread that serves systems of many sequences of
 * one context with continuous batching: requests (one system each) are
 * admitted between blocks of iterations while fewer than max_slots are in
 * flight and their solve-time working sets (Krylov history, A C, staging)
 * fit in hbm_budget bytes (0 = no limit); admitted systems join the fused
 * launches of their type immediately, finished ones leave them, have their
 * solution copied to x_out and their basis recycled (TRKS / SRKS), and
 * release their working set; the basis itself stays resident with the
 * sequence.  Requests of one sequence are served in order, one at a time
 * (system k+1 needs the basis from system k); requests of different
 * sequences overlap on the device.  Each result equals the one of
 * krs_seq_submit + krs_seq_solve + krs_seq_recycle on the same sequence.
 * While a server exists its worker owns the context's stream: the caller
 * must not use that context's sequences directly.  A sequence with requests
 * in flight cannot be destroyed (KRS_E_STATE), and submit, solve, recycle,
 * basis export and the batch calls refuse it (KRS_E_BUSY). */
typedef struct krs_server krs_server;

typedef struct {
    uint64_t tag;          /* as given to krs_server_enqueue */
    krs_seq* seq;
    int32_t status;        /* krs_status of the solve (or of the admission) */
    int32_t batch_size;    /* members of the fused launches when it finished */
    double latency_ms;     /* completion - enqueue */
    double queue_ms;       /* admission - enqueue */
    krs_solve_info info;   /* info.added: columns appended by the recycle */
    char message[128];     /* error text when status != KRS_OK */
} krs_completion;

typedef struct {
    int64_t enqueued, completed, failed, queued;
    int64_t blocks;        /* blocks of iterations launched */
    double mean_batch;     /* members per block, averaged over blocks */
    double solves_per_s;   /* completed / (last completion - first enqueue) */
    double p50_ms, p99_ms, mean_ms;  /* request latency (completion - enqueue) */
    int64_t peak_bytes;    /* largest sum of admitted working sets */
} krs_server_report;

krs_status krs_server_create(krs_ctx* ctx, size_t hbm_budget, int32_t max_slots, krs_server** out);
/* Queue one system of `seq`: values (host, nnzb*block^2 doubles) and b
 * (host, n doubles) are copied; x_out (host, n doubles, or NULL) is written
 * before the completion is posted.  KRS_E_BUSY when the queue is full. */
krs_status krs_server_enqueue(krs_server* s, krs_seq* seq, const double* values, const double* b, double* x_out,
                              uint64_t tag);
/* Up to cap completions in completion order; waits up to timeout_ms
 * (0: no wait, negative: until one is available or the server stopped). */
krs_status krs_server_poll(krs_server* s, krs_completion* out, int32_t cap, int32_t* count, int32_t timeout_ms);
krs_status krs_server_stats(krs_server* s, krs_server_report* out);
/* Serves every queued request, then stops the worker and frees the server. */
krs_status krs_server_destroy(krs_server* s);

/* ------------------------------------------------ host-side Ritz logic */
/* Host only, no device: the complexity analysis of KRS_NC_LIM_AUTO on the
 * CG coefficients alpha[m], rho[m] of a non-augmented solve (Section 4.4
 * remark after Algorithm 3; model stated at KRS_NC_LIM_AUTO), with eps the
 * stagnation tolerance that marks a Ritz value converged, and the given byte
 * costs: bytes_iter0 per iteration without a basis, bytes_col_iter per
 * basis column per iteration, bytes_rebuild0 + k bytes_col_rebuild for the
 * rebuild of k > 0 columns.  *nc_lim receives the k in 0..kmax of least
 * modelled bytes per system (kmax is clipped to the number of distinct Ritz
 * values less one); cost (NULL, or kmax + 1 doubles) the modelled bytes for
 * each k; *k_out the clipped kmax. */
krs_status krs_nc_limit(const double* alpha, const double* rho, int32_t m, double bytes_iter0, double bytes_col_iter,
                        double bytes_rebuild0, double bytes_col_rebuild, int32_t kmax, double eps, double* cost,
                        int32_t* k_out, int32_t* nc_lim);
/* Host only, no device: the cluster reselection of KRS_RESELECT_CLUSTER
 * on Ritz values theta[m] (any order) and a preselection flags[m]
 * (1 = preselected); on return flags[i] = 1 only for the preselected values
 * outside the central cluster (Section 4.4). */
krs_status krs_cluster_reselect(const double* theta, int32_t m, double min_frac, uint8_t* flags);
/* Pure host computations exposed for testing the library's selection
 * logic; no device is touched.
 * krs_ritz_select: from alpha[m], rho[m] build the Lanczos tridiagonal H_m
 * (Section 4.1), compute the eigenvalues of H_m and H_{m-1} (descending,
 * theta[m], theta_prev[m-1]; either may be NULL) and flag the Ritz values
 * that passed the stagnation test with tolerance eps (selected[m]). */
krs_status krs_ritz_select(const double* alpha, const double* rho, int32_t m, double eps, double* theta,
                           double* theta_prev, uint8_t* selected);
/* Cholesky factorisation of the SPD coarse matrix G (nc x nc column-major)
 * with the rank guard, and the explicit inverse over the kept columns:
 * Ginv (nc x nc) gets zero rows/columns for dropped columns; kept[nc]. */
krs_status krs_coarse_factor(int32_t nc, const double* G, double rank_tol, double* Ginv, uint8_t* kept, int32_t* nk);

#ifdef __cplusplus
}
#endif

#endif /* KRS_H */
