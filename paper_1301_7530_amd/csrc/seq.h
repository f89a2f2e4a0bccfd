// Host-side objects behind the opaque handles of include/krs.h.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"

struct krs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool has_alloc = false;
    krs_allocator alloc{};
    std::atomic<int> live_seqs{0};
    std::atomic<int> live_servers{0};
    std::atomic<int64_t> bytes_live{0};
    // bytes of the longest Krylov history that fit on this device after a
    // longer one did not (0: none failed); later sequences start there, so
    // that a request bound to fail does not make the allocator drop its
    // cached blocks
    std::atomic<int64_t> hist_fit_bytes{0};
};

namespace krs {

void* dev_alloc(krs_ctx* ctx, size_t bytes);
void dev_free(krs_ctx* ctx, void* p, size_t bytes);

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
    bool reserve(krs_ctx* ctx, size_t nbytes);                       // contents not kept
    bool grow_keep(krs_ctx* ctx, size_t nbytes, hipStream_t stream);  // contents kept
    void release(krs_ctx* ctx);
};

struct SeqBase {
    krs_ctx* ctx = nullptr;
    krs_seq_desc desc{};
    virtual ~SeqBase() {}
    virtual krs_status create(const krs_seq_desc& d, const double* C0, int32_t m0, int64_t ldc0) = 0;
    virtual krs_status submit(const double* values, const double* b, bool device) = 0;
    virtual krs_status solve(double* x, bool device_x, krs_solve_info* info) = 0;
    // solve() = begin_solve() + iterate() + end_solve(); a batch runs the
    // iterations of several begun systems in fused launches instead
    virtual krs_status begin_solve() = 0;
    // The coarse rebuild of begin_solve in stages, for a batch whose members
    // share one stream: stage 0 enqueues the first A C / Gram pass, stage 1
    // (after the caller's wait) orthonormalises and enqueues the second,
    // stage 2 factors and uploads G^-1 (or, if a column vanished, finishes
    // the rebuild on its own).  *more: whether the member needs the next
    // stage after a wait.  begin_solve then skips the rebuild.
    virtual krs_status rebuild_stage(int stage, bool* more) = 0;
    // iter_hint: the solve's final iteration count when the caller has read
    // it from the device status (lets the coefficient read-back start
    // before the wait), or -1
    virtual krs_status end_solve(double* x, bool device_x, krs_solve_info* info, int iter_hint = -1) = 0;
    virtual int type_key() const = 0;
    // device bytes a solve adds on top of the resident sequence (matrix,
    // vectors, basis): Krylov history, A C, staging and reduction scratch
    virtual int64_t working_bytes() const = 0;
    // release those solve-time buffers (they are re-created by the next solve)
    virtual void trim() = 0;
    std::atomic<int> in_server{0};  // requests of a server not yet completed
    int recycle_threads = 0;        // host threads of the Ritz bisection (0: automatic)
    virtual krs_status recycle(int32_t* n_added) = 0;
    // recycle() in two steps: host work only (may run on another thread
    // while the device is busy), then the device work on the stream
    virtual krs_status recycle_plan() = 0;
    virtual krs_status recycle_apply(int32_t* n_added) = 0;
    // message of the last failed recycle_plan (the error text is per thread,
    // and the plan may have run on a helper thread)
    char plan_msg[256] = {0};
    virtual krs_status basis(double* C, int64_t ld, int32_t cap, int32_t* n_c) = 0;
    // a begun solve's update tile (block rows per update workgroup), fixed
    // from here on for the sequence (the batch autotuner sets it)
    virtual krs_status set_update_rows(int64_t rows) = 0;
    bool batch_tuned = false;
    int batch_tuned_nc = 0;
    bool batch_tune_due() const {
        const int t = std::max(batch_tuned_nc, 1), c = std::max(nc, 1);
        return !batch_tuned || 2 * c > 3 * t || 3 * c < 2 * t;
    }
    // the export through caller-provided device staging of n doubles
    virtual krs_status basis_staged(double* C, int64_t ld, double* staging) = 0;
    virtual krs_status history(double* Z, int64_t ld, int32_t cap, int32_t* m_out) = 0;
    virtual void destroy() = 0;
    // live kernel timing (sampled iterations, device wall clock)
    bool timing = false;
    int64_t kt_count[3] = {0, 0, 0};
    double kt_ms[3] = {0.0, 0.0, 0.0};
    // last results (host mirrors)
    int m_last = 0;
    int nc = 0;
    int last_selected = 0;
    int restarts = 0;
    std::vector<double> coef_alpha, coef_rho, coef_gamma;
    std::vector<double> last_theta;
    std::vector<uint8_t> last_sel;
    krs_solve_info info_last{};
};

template <typename V, typename W>
struct SeqImpl : SeqBase {
    hipStream_t stream = nullptr;
    int B = 1;
    int64_t n = 0, nb = 0, nnzb = 0, nslices = 0, nslots = 0;
    int64_t ldc = 0;
    int64_t ldac = 32;
    int nc_cap = 0, nc0 = 0;
    int coef_cap = 0;
    int trks_slots = 0;
    bool submitted = false, solved = false;
    Buf d_col16;  // 16-bit relative block columns for the double-precision 3x3 SpMV, when they fit
    Buf d_col, d_slice_ptr, d_map, d_diag, d_val64, d_valV, d_minv, d_bad, d_in, d_b, d_x, d_r, d_s, d_w, d_q;
    Buf d_C, d_C0, d_AC64, d_ACv, d_G, d_Ginv, d_mu, d_Z, d_coef, d_partials, d_st, d_F, d_tmp, d_Ctmp, d_kslots;
    // full reorthogonalisation (kernel_flags bit 2): kept directions, their
    // A-products, partial sums, coefficients, the current z
    Buf d_Wr, d_Qr, d_rpart, d_rc, d_zr;
    int rcap = 0, rgr = 0;
    int64_t ldr = 0;
    bool reorth() const { return (desc.kernel_flags & 4) != 0; }
    // kernel_flags bit 7: the Krylov history of a double-precision basis
    // kept in single precision (it only forms the Ritz vectors)
    bool hist32() const { return (desc.kernel_flags & 128) != 0 && std::is_same<V, double>::value; }
    int64_t hist_elem() const { return hist32() ? (int64_t)sizeof(float) : (int64_t)sizeof(V); }
    // SpMV workgroup cap, kernel_flags bits 5-6: 0 the default (8192, the
    // size of the region of its partial sums, kPart1), 1: 2048, 2: 4096,
    // 3: 8192
    int spmv_grid_cap() const {
        const int code = (desc.kernel_flags >> 5) & 3;
        return code == 0 ? (int)kPart1 : (int)std::min<int64_t>(kPart1, (int64_t)1024 << code);
    }
    DevState* h_st = nullptr;
    double* h_coef = nullptr;  // pinned staging of the CG coefficients read back by end_solve
    size_t h_coef_cap = 0;     // doubles
    Geometry geo{};
    int tuned_nc = 0;
    int dropped_last = 0;
    int history_kept = 0;
    int history_fit = 0;  // history length that fit after a longer one did not (0: none failed)
    // the cost cap holds: the recycle after this solve appends nothing
    bool cost_held() const { return desc.cap_policy == KRS_CAP_COST && cost_hold > 0 && nc <= nc0; }
    // SRKS needs the run's directions unless nothing will be appended from
    // them: the basis is full and frozen, or the cost cap holds
    bool history_needed() const {
        if (has_cap() && (cap_value() == 0 || (desc.cap_policy == KRS_CAP_FREEZE && nc >= cap_value())))
            return false;
        return !cost_held();
    }
    // n_c_lim: given (max_basis > 0), or set by the complexity analysis on
    // the first solve (max_basis = KRS_NC_LIM_AUTO; -1 until then)
    int nc_lim_auto = -1;
    bool has_cap() const { return desc.max_basis > 0 || (desc.max_basis < 0 && nc_lim_auto >= 0); }
    int cap_value() const { return desc.max_basis > 0 ? desc.max_basis : std::max(0, nc_lim_auto); }
    std::vector<double> h_F;  // host source of the last basis-update upload
    struct RecyclePlan {
        bool ready = false;       // planned, not yet applied
        bool restore_c0 = false;  // cost cap: back to the initial basis
        int kind = 0;             // 0: nothing appended, 1: TRKS scaling, 2: SRKS combination
        int add = 0;              // columns appended
        int mu = 0;               // SRKS: length of the Lanczos pair combined
        double host_ms = 0.0;
    } plan;
    int64_t ref_cost = 0;   // modelled bytes of the latest solve with the initial basis (cost cap)
    int cost_hold = 0;      // systems left before the cost cap lets columns be appended again
    int cost_fails = 0;     // failed trials of recycled columns in a row
    static constexpr int kCostHold = 3;
    SysView<V, W> cur{};          // view of the solve in progress
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // rebuild / iteration timers
    // captured iteration blocks (16 and 64 iterations + refinement step)
    struct GraphSlot {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        SysView<V, W> view{};
        int block = 0;
    } gslot[2];
    krs_status graph_launch(const SysView<V, W>& v, int slot, int block);
    void graph_release();

    krs_status create(const krs_seq_desc& d, const double* C0, int32_t m0, int64_t ldc0) override;
    krs_status submit(const double* values, const double* b, bool device) override;
    krs_status solve(double* x, bool device_x, krs_solve_info* info) override;
    krs_status begin_solve() override;
    krs_status iterate();
    krs_status end_solve(double* x, bool device_x, krs_solve_info* info, int iter_hint = -1) override;
    void coef_readback(int mc);  // enqueue the copies of the first mc CG coefficients into h_coef
    int type_key() const override;
    krs_status tune_update();
    int64_t working_bytes() const override;
    void trim() override;
    krs_status recycle(int32_t* n_added) override;
    krs_status recycle_plan() override;
    krs_status recycle_apply(int32_t* n_added) override;
    krs_status basis(double* C, int64_t ld, int32_t cap, int32_t* n_c) override;
    krs_status set_update_rows(int64_t rows) override;
    krs_status basis_staged(double* C, int64_t ld, double* staging) override;
    krs_status history(double* Z, int64_t ld, int32_t cap, int32_t* m_out) override;
    void destroy() override;

    SysView<V, W> view();
    bool ensure_c_capacity(int cols);
    bool ensure_partials(int64_t extra);
    krs_status rebuild(int* dropped);
    krs_status rebuild_stage(int stage, bool* more) override;
    krs_status coarse_pass(std::vector<double>& G);
    krs_status coarse_pass_enqueue();
    void coarse_pass_read(std::vector<double>& G) const;
    bool rb_done = false;         // the staged rebuild has run for the submitted system
    int rb_dropped = 0;
    std::vector<double> rb_up;    // host source of the stage's upload (kept until the next wait)
    double* h_G = nullptr;        // pinned read-back of C^T A C
    size_t h_G_cap = 0;
    void k_spmv(const SysView<V, W>& v);
    void k_update(const SysView<V, W>& v, int mode);
    void k_resid(const SysView<V, W>& v, int final_only);
    void enqueue_iterations(const SysView<V, W>& v, int k);
    void enqueue_refine(const SysView<V, W>& v);
    int64_t model_bytes_per_iter(bool padded) const;
    int64_t cost_bytes_last = 0;  // streamed bytes of the last solve (cost cap)
    // double-precision operator with a single-precision basis / preconditioner
    bool op64() const { return desc.precision == KRS_FP32_BASIS; }
};

// Fused launches over a set of begun solves of one (V, W, B) type
// (type_key); members may change between blocks.
struct RunnerBase {
    virtual ~RunnerBase() {}
    virtual krs_status set_members(const std::vector<SeqBase*>& members) = 0;
    // enqueue one block of iterations (+ refinement step) for every member
    // and the read-back of their status words
    virtual krs_status launch(int block, bool graphs) = 0;
    // wait for the last launch; out[2 i] = status, out[2 i + 1] = iteration of member i
    virtual krs_status read_status(std::vector<int32_t>& out) = 0;
    virtual size_t size() const = 0;
    // time `reps` launches of the update kernel alone (initial mode: it
    // rewrites s and the partial sums, which the next step recomputes) over
    // every member; *ms receives the mean per launch
    virtual krs_status time_update(int reps, float* ms) = 0;
};
std::unique_ptr<RunnerBase> make_runner(krs_ctx* ctx, int type_key);
bool finished_status(int device_status);

// Recycle several sequences, their host work on parallel threads.
krs_status recycle_all(krs_ctx* ctx, SeqBase* const* seqs, int count, int32_t* added);
// The host step (recycle_plan) of several sequences on parallel threads;
// st[i] receives each status.  Makes no device calls.
void plan_all(SeqBase* const* seqs, int count, krs_status* st);

// Solve the submitted systems of several sequences in fused launches.
// With `added` (count entries) every member is also recycled (as by
// recycle_all), the host step of a member planned as soon as it finishes.
krs_status batch_solve(krs_ctx* ctx, SeqBase* const* seqs, int count, double* const* x, bool device_x,
                       krs_solve_info* info, int32_t* added = nullptr);

// The allocation-free entry point's static device scratch (noalloc.cpp):
// looked up once per device with that device current; the address kept
// per device (nullptr before noalloc_init succeeded on it).
krs_status noalloc_init(int device);
size_t noalloc_scratch_bytes();
void* noalloc_scratch(int device);

}  // namespace krs

struct krs_seq {
    std::unique_ptr<krs::SeqBase> impl;
};
