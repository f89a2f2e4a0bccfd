// Internal declarations shared by the host runtime and the kernel launchers
// of libkrs.  Nothing here is part of the public ABI (include/krs.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "krs.h"

namespace krs {

// ELL slice height, in (block) rows: one lane per block row of a slice.
constexpr int kSlice = 64;
// Doubles reserved at the head of the reduction scratch for SpMV partials
// (>= the largest SpMV grid).
constexpr int64_t kPart1 = 8192;
// double-precision block matrices larger than this (the 256 MB Infinity
// Cache) stream through the SpMV with non-temporal loads by default
constexpr int64_t kNtBytes = int64_t(256) << 20;
// Byte offset of the fused update's ticket counters in the state allocation
// (one global counter, then one per group of kGroup update workgroups).
constexpr int kSyncOffset = 256;
constexpr int kGroup = 16;
constexpr int kSyncBytes = 4 * (1 + 2048 / kGroup) + 60;
// Threads of the update kernel (one block row each per step).
constexpr int kT3 = 512;
// Largest update grid (bounds the partial sums the finalize kernel reads).
constexpr int64_t kMaxUpdateGrid = 2048;
// Largest grid of a timed kernel (timing slots per kernel).
constexpr int64_t kMaxTimedGrid = 8192;

// Launch geometry of one system, fixed for a solve: the single-system and
// the fused batch launches use the same per-system workgroup counts, so a
// system's reductions (and results) are the same in both.
// Row length of the row-major A C: the next power of two of at least 4
// elements up to 32 columns (16-byte segments, whole rows per 128-byte
// chunk), else a multiple of the 128-byte chunk the projection reads
// (32 FP32 or 16 FP64 values).
inline int64_t ac_leading_dim(int64_t nc, int64_t elem_bytes) {
    const int64_t cw = 128 / elem_bytes;
    if (nc > 32) return (nc + cw - 1) / cw * cw;
    int64_t l = 4;
    while (l < nc) l *= 2;
    return l;
}

struct Geometry {
    int64_t cb3;  // block rows per update workgroup
    int32_t g1;   // SpMV / true-residual workgroups
    int32_t g3;   // update workgroups
    int32_t g5;   // direction-update workgroups
    int32_t gd;   // coarse-dot workgroups
    int32_t gcc;  // coarse-correction workgroups
    int32_t pad;
};

// Device-side solver status codes (DevState::status).
enum DevStatus : int32_t {
    ST_RUN = 0,        // iterating
    ST_DONE = 1,       // converged (true residual confirmed)
    ST_CHECK = 2,      // recursive residual converged; true residual pending
    ST_REFINE = 3,     // reliable update pending (mixed precision)
    ST_BREAKDOWN = 4,  // (w, A w) <= 0 or (r, z) <= 0 or NaN
    ST_MAXIT = 5,
};
constexpr uint32_t M_RUN = 1u << ST_RUN;
constexpr uint32_t M_CHECK = 1u << ST_CHECK;
constexpr uint32_t M_REFINE = 1u << ST_REFINE;

// Scalars of one solve, resident in device memory.  Written only by the
// single-workgroup finalize kernels, read by every workgroup of the next.
struct DevState {
    double rho;       // rho_j = (r_j, z_j)
    double alpha;     // alpha_j
    double beta;      // beta for the next direction update
    double bb;        // ||b||^2
    double rr;        // ||r||^2 of the recursion
    double rr_ref;    // ||r||^2 right after the last refinement
    double tol2;      // tol^2
    double drop2;     // refinement trigger (relative drop of ||r||^2)
    double rr_true;   // last true residual ||b - A x||^2
    int32_t iter;     // products A w performed
    int32_t status;   // DevStatus
    int32_t max_iter;
    int32_t hist_cap; // Z / W history slots available
    int32_t since_refine;
    int32_t refine_every;
    int32_t refinements;
    int32_t nc;       // basis columns active in this solve
    int32_t pending_dir;  // 1 between a residual replacement and its direction update
    int32_t first_restart;  // iteration of the first direction restart (Lanczos run ends there)
    int32_t restarts;
    // live kernel timing (device wall clock): summed spans of sampled
    // launches of the SpMV, update and direction kernels
    int32_t ktime_on;
    int32_t ktime_pad;
    unsigned long long ksum[3];
    unsigned long long kcnt[3];
};
static_assert(sizeof(DevState) % 8 == 0, "DevState is staged in 8-byte words");

// Per-launch view of one system, passed by value to the kernels.  V is the
// storage type of the matrix values, the preconditioner and the basis; W
// the type of the Krylov vectors; x, b and every reduction are double.
template <typename V, typename W>
struct SysView {
    // sliced-ELL matrix (block size B known at compile time)
    const int32_t* col;        // [slots*64] block column per entry
    const int16_t* col16;      // the same as (column - own block row) when every difference fits 16 bits, or null
    const int64_t* slice_ptr;  // [nslices+1] slot offsets
    const V* val;              // values in V precision (planar per slot)
    int32_t op64;              // 1: the SpMV streams val64 (double-precision operator)
    int32_t spmv_var;          // SpMV load schedule: bit 0 four blocks in flight, bit 1 non-temporal matrix loads
    const double* val64;       // values in double (for true residuals / A C)
    const V* minv;             // preconditioner inverse: n (Jacobi) or 9*nb (3x3 blocks)
    int64_t n;                 // scalar rows
    int64_t nb;                // block rows
    int64_t nslices;
    // vectors
    double* x;
    const double* b;
    W* r;
    W* s;
    W* w;
    W* q;
    // basis
    int32_t nc;      // columns of C in this solve
    int32_t nt_store;  // 1: the iteration's vector stores are non-temporal (set with the streaming schedule)
    const V* C;      // n x nc column-major, leading dim ldc (a multiple of 256 >= n)
    const V* AC;     // n x nc row-major, leading dim ldac = ac_leading_dim(nc, sizeof(V))
    int64_t ldc;
    int64_t ldac;
    const double* Ginv;  // nc x nc column-major
    double* mu;          // nc: G^-1 (AC)^T s of the current step
    double* u;           // nc: C^T r, tracked by recurrence (zero in exact arithmetic)
    double* mu2;         // nc: mu + beta G^-1 (AC)^T w_old, for the projected direction
    // histories
    V* zhist;        // z_j at column j (SRKS), or null
    float* zhist32;  // the same in single precision (kernel_flags bit 7, double bases), or null
    V* whist;        // w_j at column j (TRKS: columns of C past nc), or null
    int64_t ldh;
    double* alpha_h;  // [hist] alpha_j
    double* rho_h;    // rho_j
    double* gamma_h;  // (w_j, A w_j)
    int32_t coef_cap;
    // reductions
    double* part1;     // per-workgroup (w, A w) partials of the SpMV
    double* partials;  // per-workgroup partials of the other reductions
    DevState* st;
    unsigned* sync;              // ticket counter of the fused update (zero between launches)
    unsigned long long* kslots;  // per-workgroup start / end stamps of timed launches
    Geometry geo;
    int32_t fused;               // 1: the update kernel's last workgroup runs the finalize
    int32_t dir_literal;         // 1: w = z + beta w_old as written; 0: w = z + beta P w_old
    // full reorthogonalisation (null Wr: off): every direction and its
    // product with A kept row-major (n x ldr, columns j < rcap); the next
    // direction is z made A-orthogonal to all of them
    W* Wr;
    W* Qr;
    int64_t ldr;
    int32_t rcap;
    int32_t gr;       // row ranges (workgroups) of the coefficient partials
    double* rpart;    // gr x ldr partial sums (A w_i, z)
    double* rc;       // ldr coefficients (A w_i, z) / (w_i, A w_i)
    W* zr;            // z of the current step, written by the direction update
};
// largest number of directions a reorthogonalised solve keeps
constexpr int kReorthMax = 8192;

// Launch maps of a fused batch: map[k][i] = (system, workgroup) of launch
// k's workgroup i; count[k] = total workgroups.
enum BatchKernel {
    BK_SPMV = 0,  // SpMV and true residual (g1 per system)
    BK_UPD,       // update (g3)
    BK_ONE,       // one workgroup per system (F3, F11)
    BK_DIR,       // direction update (g5)
    BK_DOT,       // coarse dot (gd; systems with a basis)
    BK_ONEC,      // one workgroup per system with a basis
    BK_CC,        // coarse correction (gcc; systems with a basis)
    BK_DIR0,      // direction update of systems without a basis (kDirFewGroup K5 ranges each)
    BK_DIRF,      // direction update of systems with 1..kDirFewCols columns (kDirFewGroup K5 ranges each)
    BK_COUNT
};
// the direction update of systems with at most kDirFewCols basis columns:
// K5 workgroup ranges per workgroup
constexpr int kDirFewCols = 4;
constexpr int kDirFewGroup = 4;
struct BatchMaps {
    const int2* map[BK_COUNT];
    int64_t count[BK_COUNT];
    int32_t fused;  // every member uses the fused update
};

// ------------------------------------------------------------ launchers
// All launch on `stream`; the grid shapes come from the view's geometry.
// spmv_grid: cap on the SpMV workgroups (0: 2048)
Geometry make_geometry(int64_t n, int64_t nslices, int block, int64_t cb3_req, int spmv_grid = 0);
// doubles of reduction scratch (after kPart1) a solve with nc columns needs
int64_t partial_doubles(const Geometry& g, int nc);

template <typename V, typename W, int B> void launch_spmv_dot(const SysView<V, W>& v, hipStream_t stream);
template <typename V, typename W, int B>
void launch_update_reduce(const SysView<V, W>& v, int mode, hipStream_t stream);
// the update kernel alone (mode 1 only rewrites s and the partials: used to time tile choices)
template <typename V, typename W, int B>
void launch_update_only(const SysView<V, W>& v, int mode, hipStream_t stream);
template <typename V, typename W> void launch_correct_dir(const SysView<V, W>& v, int first, hipStream_t stream);
// full reorthogonalisation: the store after the SpMV; the coefficients and
// the update of w after the direction update
template <typename V, typename W> void launch_reorth_store(const SysView<V, W>& v, hipStream_t stream);
void launch_basis_combine_h32(const float* Z, int64_t ldz, int m, const double* F, int s, double* out, int64_t ldo,
                              int64_t n, hipStream_t stream);
template <typename V, typename W> void launch_reorth(const SysView<V, W>& v, hipStream_t stream);
template <typename V, typename W, int B>
void launch_true_resid(const SysView<V, W>& v, int final_only, hipStream_t stream);
template <typename V, typename W>
void launch_coarse_dot(const SysView<V, W>& v, int src_b, int with_bb, uint32_t mask, hipStream_t stream);
template <typename V, typename W>
void launch_coarse_correct(const SysView<V, W>& v, int from_b, uint32_t mask, hipStream_t stream);
template <typename V, typename W, int B>
void launch_spmm(const SysView<V, W>& v, const V* C, int64_t ldc, int nc, int64_t ldac, double* AC64, V* ACv,
                 hipStream_t stream);
template <typename V>
void launch_gram(const V* C, int64_t ldc, const double* AC64, int64_t ldac, int64_t n, int nc, double* G,
                 double* partials, int64_t partial_cap, hipStream_t stream);
template <typename V>
void launch_basis_combine(const V* Z, int64_t ldz, int m, const double* F, int s, V* out, int64_t ldo, int64_t n,
                          hipStream_t stream);
template <typename V>
void launch_scale_columns(V* C, int64_t ldc, int64_t n, const double* scale, int k, hipStream_t stream);
template <typename V>
void launch_copy_columns(const V* src, int64_t lds, V* dst, int64_t ldd, int64_t n, const int32_t* map, int k,
                         hipStream_t stream);
template <typename V, int B>
void launch_scatter_values(const double* in, const int64_t* map, int64_t nnzb, double* val64, V* valV,
                           hipStream_t stream);
template <typename V, int B>
void launch_precond_setup(const double* in, const int64_t* diag_idx, int64_t nb, V* minv, int32_t* bad,
                          hipStream_t stream);
template <typename V> void launch_d2v(const double* in, V* out, int64_t n, hipStream_t stream);
template <typename V> void launch_v2d(const V* in, double* out, int64_t n, hipStream_t stream);

// fused launches over the systems of a batch (views: device array)
template <typename V, typename W, int B>
void batch_spmv_dot(const SysView<V, W>* views, const BatchMaps& m, hipStream_t stream);
template <typename V, typename W, int B>
void batch_update_reduce(const SysView<V, W>* views, const BatchMaps& m, int mode, hipStream_t stream);
template <typename V, typename W, int B>
void batch_update_only(const SysView<V, W>* views, const BatchMaps& m, int mode, hipStream_t stream);
template <typename V, typename W>
void batch_correct_dir(const SysView<V, W>* views, const BatchMaps& m, int first, hipStream_t stream);
template <typename V, typename W, int B>
void batch_true_resid(const SysView<V, W>* views, const BatchMaps& m, int final_only, hipStream_t stream);
template <typename V, typename W>
void batch_coarse_dot(const SysView<V, W>* views, const BatchMaps& m, int src_b, int with_bb, uint32_t mask,
                      hipStream_t stream);
template <typename V, typename W>
void batch_coarse_correct(const SysView<V, W>* views, const BatchMaps& m, int from_b, uint32_t mask,
                          hipStream_t stream);
template <typename V, typename W>
void batch_status(const SysView<V, W>* views, int count, int32_t* out, hipStream_t stream);

// ----------------------------------------------------------- host logic
// qd array of the Lanczos tridiagonal H_m = R^T R of the CG coefficients
// (Section 4.1): q_j = R_jj^2 = 1/alpha_j, e_j = R_{j,j+1}^2 =
// (rho_{j+1}/rho_j)/alpha_j.  The leading (m-1) x (m-1) block H_{m-1} is
// the array cut to q[0..m-2], e[0..m-3] (ritz.cpp).
struct QdArray {
    std::vector<double> q, e;
};
QdArray qd_from_cg(const double* alpha, const double* rho, int m);
QdArray qd_leading(const QdArray& z, int m1);
// Number of eigenvalues below sigma (high relative accuracy).
int qd_count_below(const QdArray& z, double sigma);
// Whether the array has an eigenvalue in [lo, hi].
bool qd_has_eigenvalue_in(const QdArray& z, double lo, double hi);
// Eigenvalues of ascending ranks k0..k1-1 (0 = smallest) into out[k].
void qd_eigenvalues_asc(const QdArray& z, int k0, int k1, double* out, int threads);
// Every eigenvalue, descending.
void qd_eigenvalues_desc(const QdArray& z, std::vector<double>& theta, int threads);
// Eigenvector (unit 2-norm) of the explicit tridiagonal (diag, off) for eigenvalue theta.
void tridiag_eigvec(const std::vector<double>& diag, const std::vector<double>& off, double theta,
                    std::vector<double>& v);
// Byte costs of the complexity analysis behind n_c_lim (Section 4.4): one
// iteration without a basis, the extra bytes per basis column per
// iteration, the per-system rebuild of a non-empty basis and its extra
// bytes per column.
struct NcCostModel {
    double bytes_iter0 = 0.0, bytes_col_iter = 0.0, bytes_rebuild0 = 0.0, bytes_col_rebuild = 0.0;
    double eps = 1e-8;  // stagnation tolerance that marks a Ritz value converged
    int kmax = 0;
};
// n_c_lim from the CG coefficients of a solve taken as the non-augmented
// iteration count of every system; cost (optional) receives the modelled
// bytes per system for k = 0..kmax' (kmax' = kmax clipped to the spectrum).
int nc_limit(const double* alpha, const double* rho, int m, const NcCostModel& cm, int threads,
             std::vector<double>* cost);
// Cluster reselection (Section 4.4, "clust"): the preselected indices sel
// into theta without the central cluster, ascending.
std::vector<int> cluster_reselect(const std::vector<double>& theta, const std::vector<int>& sel, double min_frac);
// Stagnation selection (Section 4.4) on descending theta_m / theta_{m-1}.
std::vector<int> stagnation_select(const std::vector<double>& th_m, const std::vector<double>& th_m1, double eps);
// Cholesky with rank guard + explicit inverse (coarse.cpp). Returns kept count.
int coarse_factor(int nc, const double* G, double rank_tol, double* Ginv, uint8_t* kept);
// U (nc x nk) such that C U is the kept part of C made A-orthonormal.
int coarse_orthonormalizer(int nc, const double* G, double rank_tol, double* U, uint8_t* kept);

void set_error(const std::string& msg);

}  // namespace krs
