// C entry points of libkrs (include/krs.h): argument checks, error
// reporting and dispatch to the sequence runtime.  Nothing throws across
// this boundary.
#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <algorithm>
#include <string>
#include <thread>
#include <vector>

#include "seq.h"

namespace krs {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace krs

using krs::set_error;

#define KRS_GUARD_BEGIN try {
#define KRS_GUARD_END                                      \
    }                                                      \
    catch (const std::bad_alloc&) {                        \
        set_error("host allocation failed");               \
        return KRS_E_OOM;                                  \
    }                                                      \
    catch (const std::exception& e) {                      \
        set_error(std::string("internal error: ") + e.what()); \
        return KRS_E_INVALID;                              \
    }                                                      \
    catch (...) {                                          \
        set_error("internal error");                       \
        return KRS_E_INVALID;                              \
    }

extern "C" {

const char* krs_status_str(krs_status s) {
    switch (s) {
        case KRS_OK: return "ok";
        case KRS_E_INVALID: return "invalid argument";
        case KRS_E_OOM: return "out of memory";
        case KRS_E_NOT_SPD: return "operator or preconditioner not SPD (breakdown)";
        case KRS_E_COARSE_SINGULAR: return "coarse matrix singular";
        case KRS_E_MAXIT: return "maximum iterations reached";
        case KRS_E_DEVICE: return "device error";
        case KRS_E_BUSY: return "busy";
        case KRS_E_STATE: return "invalid state";
    }
    return "unknown status";
}

const char* krs_last_error(void) { return krs::g_last_error.c_str(); }

const char* krs_version(void) { return "krs 0.1 (gfx950)"; }

krs_status krs_ctx_create(int device, void* hip_stream, const krs_allocator* a, krs_ctx** out) {
    KRS_GUARD_BEGIN
    if (!out) {
        set_error("out is NULL");
        return KRS_E_INVALID;
    }
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        set_error("no such HIP device");
        return KRS_E_DEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) {
        set_error("hipSetDevice failed");
        return KRS_E_DEVICE;
    }
    {
        // the device address of the allocation-free entry point's scratch
        const krs_status st = krs::noalloc_init(device);
        if (st != KRS_OK) return st;
    }
    krs_ctx* c = new krs_ctx();
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            set_error("hipStreamCreate failed");
            return KRS_E_DEVICE;
        }
        c->own_stream = true;
    }
    if (a && a->alloc && a->free) {
        c->alloc = *a;
        c->has_alloc = true;
    }
    *out = c;
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_ctx_destroy(krs_ctx* ctx) {
    KRS_GUARD_BEGIN
    if (!ctx) return KRS_OK;
    if (ctx->live_seqs > 0 || ctx->live_servers > 0) {
        set_error("context still has live sequences or a server");
        return KRS_E_STATE;
    }
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_seq_create(krs_ctx* ctx, const krs_seq_desc* d, const double* C0, int32_t m0, int64_t ldc0,
                          krs_seq** out) {
    KRS_GUARD_BEGIN
    if (!ctx || !d || !out) {
        set_error("ctx, desc and out are required");
        return KRS_E_INVALID;
    }
    *out = nullptr;
    if (d->n <= 0 || (d->block != 1 && d->block != 3) || d->n % d->block != 0 || d->nnzb <= 0 || !d->row_ptr ||
        !d->col_idx || d->tol <= 0.0 || d->max_iter < 0 || m0 < 0 || d->max_basis < KRS_NC_LIM_AUTO ||
        d->history_cap < 0 ||
        d->refine_every < 0) {
        set_error("invalid sequence description");
        return KRS_E_INVALID;
    }
    if (d->precision != KRS_FP64 && d->precision != KRS_MIXED && d->precision != KRS_FP32 &&
        d->precision != KRS_FP32_BASIS) {
        set_error("unknown precision");
        return KRS_E_INVALID;
    }
    if ((d->kernel_flags & 128) && d->precision != KRS_FP64) {
        set_error("a single-precision history (kernel_flags bit 7) applies to the double-precision basis only");
        return KRS_E_INVALID;
    }
    if ((d->kernel_flags & 4) && d->precision != KRS_FP64) {
        set_error("full reorthogonalisation (kernel_flags bit 2) runs in double precision only");
        return KRS_E_INVALID;
    }
    if (d->reselect != 0 && (d->reselect != KRS_RESELECT_CLUSTER || d->reuse != KRS_REUSE_SELECTIVE ||
                             d->cluster_min_frac < 0.0 || d->cluster_min_frac > 1.0)) {
        set_error("cluster reselection needs selective reuse and 0 <= cluster_min_frac <= 1");
        return KRS_E_INVALID;
    }
    if (d->max_basis == KRS_NC_LIM_AUTO &&
        (d->reuse != KRS_REUSE_SELECTIVE || (d->cap_policy != KRS_CAP_RESTART && d->cap_policy != KRS_CAP_FREEZE))) {
        set_error("KRS_NC_LIM_AUTO needs selective reuse with the restart or freeze cap");
        return KRS_E_INVALID;
    }
    if (d->reuse != KRS_REUSE_NONE && d->reuse != KRS_REUSE_TOTAL && d->reuse != KRS_REUSE_SELECTIVE) {
        set_error("unknown reuse mode");
        return KRS_E_INVALID;
    }
    if ((d->precond == KRS_PC_BJACOBI3) != (d->block == 3) ||
        (d->precond != KRS_PC_JACOBI && d->precond != KRS_PC_BJACOBI3)) {
        set_error("KRS_PC_BJACOBI3 goes with block 3, KRS_PC_JACOBI with block 1");
        return KRS_E_INVALID;
    }
    if (d->cap_policy != KRS_CAP_RESTART && d->cap_policy != KRS_CAP_FREEZE && d->cap_policy != KRS_CAP_COST) {
        set_error("unknown cap policy");
        return KRS_E_INVALID;
    }
    if (m0 > 1024) {
        set_error("initial basis larger than 1024 columns");
        return KRS_E_INVALID;
    }
    const int64_t nb = d->n / d->block;
    if (d->row_ptr[0] != 0 || d->row_ptr[nb] != d->nnzb) {
        set_error("row_ptr must start at 0 and end at nnzb");
        return KRS_E_INVALID;
    }
    for (int64_t r = 0; r < nb; ++r) {
        if (d->row_ptr[r + 1] < d->row_ptr[r]) {
            set_error("row_ptr not monotone");
            return KRS_E_INVALID;
        }
        for (int64_t t = d->row_ptr[r]; t < d->row_ptr[r + 1]; ++t) {
            const int32_t c = d->col_idx[t];
            if (c < 0 || c >= nb || (t > d->row_ptr[r] && c <= d->col_idx[t - 1])) {
                set_error("column indices must be in range and strictly ascending per row");
                return KRS_E_INVALID;
            }
        }
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        set_error("hipSetDevice failed");
        return KRS_E_DEVICE;
    }
    std::unique_ptr<krs_seq> s(new krs_seq());
    if (d->precision == KRS_MIXED || d->precision == KRS_FP32_BASIS) s->impl.reset(new krs::SeqImpl<float, double>());
    else if (d->precision == KRS_FP32) s->impl.reset(new krs::SeqImpl<float, float>());
    else s->impl.reset(new krs::SeqImpl<double, double>());
    s->impl->ctx = ctx;
    krs_status st = KRS_OK;
    try {
        st = s->impl->create(*d, C0, m0, ldc0);
    } catch (...) {
        s->impl->destroy();  // device buffers of a creation that threw
        throw;
    }
    if (st != KRS_OK) {
        s->impl->destroy();
        return st;
    }
    s->impl->nc = m0;
    ctx->live_seqs += 1;
    *out = s.release();
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_seq_submit(krs_seq* s, const double* values, const double* b) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    if (s->impl->in_server.load() > 0) {
        set_error("the sequence has server requests in flight");
        return KRS_E_BUSY;
    }
    return s->impl->submit(values, b, false);
    KRS_GUARD_END
}

krs_status krs_seq_submit_device(krs_seq* s, const double* d_values, const double* d_b) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    if (s->impl->in_server.load() > 0) {
        set_error("the sequence has server requests in flight");
        return KRS_E_BUSY;
    }
    return s->impl->submit(d_values, d_b, true);
    KRS_GUARD_END
}

krs_status krs_seq_solve(krs_seq* s, double* x, krs_solve_info* info) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    if (s->impl->in_server.load() > 0) {
        set_error("the sequence has server requests in flight");
        return KRS_E_BUSY;
    }
    return s->impl->solve(x, false, info);
    KRS_GUARD_END
}

krs_status krs_seq_solve_device(krs_seq* s, double* d_x, krs_solve_info* info) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    if (s->impl->in_server.load() > 0) {
        set_error("the sequence has server requests in flight");
        return KRS_E_BUSY;
    }
    return s->impl->solve(d_x, true, info);
    KRS_GUARD_END
}

krs_status krs_seq_recycle(krs_seq* s, int32_t* n_added) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    if (s->impl->in_server.load() > 0) {
        set_error("the sequence has server requests in flight");
        return KRS_E_BUSY;
    }
    return s->impl->recycle(n_added);
    KRS_GUARD_END
}

krs_status krs_seq_ritz(krs_seq* s, double* theta, uint8_t* selected, int32_t cap, int32_t* m_out) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    const auto& th = s->impl->last_theta;
    const int m = (int)th.size();
    if (m_out) *m_out = m;
    if ((theta || selected) && cap < m) {
        set_error("output arrays too small");
        return KRS_E_INVALID;
    }
    for (int i = 0; i < m; ++i) {
        if (theta) theta[i] = th[i];
        if (selected) selected[i] = s->impl->last_sel[i];
    }
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_seq_coeffs(krs_seq* s, double* alpha, double* rho, double* gamma, int32_t cap, int32_t* m_out) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    const int m = s->impl->m_last;
    if (m_out) *m_out = m;
    if ((alpha || rho || gamma) && cap < m) {
        set_error("output arrays too small");
        return KRS_E_INVALID;
    }
    for (int i = 0; i < m && i < (int)s->impl->coef_alpha.size(); ++i) {
        if (alpha) alpha[i] = s->impl->coef_alpha[i];
        if (rho) rho[i] = s->impl->coef_rho[i];
        if (gamma) gamma[i] = s->impl->coef_gamma[i];
    }
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_seq_history(krs_seq* s, double* Z, int64_t ldz, int32_t cap, int32_t* m_out) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    if (s->impl->in_server.load() > 0) {
        set_error("the sequence has server requests in flight");
        return KRS_E_BUSY;
    }
    return s->impl->history(Z, ldz, cap, m_out);
    KRS_GUARD_END
}

krs_status krs_seq_basis(krs_seq* s, double* C, int64_t ldc, int32_t cap, int32_t* n_c) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    if (s->impl->in_server.load() > 0) {
        set_error("the sequence has server requests in flight");
        return KRS_E_BUSY;
    }
    return s->impl->basis(C, ldc, cap, n_c);
    KRS_GUARD_END
}

krs_status krs_seq_basis_noalloc(krs_seq* s, double* C, int64_t ldc, int32_t cap, int32_t* n_c) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    if (s->impl->in_server.load() > 0) {
        set_error("the sequence has server requests in flight");
        return KRS_E_BUSY;
    }
    krs::SeqBase* q = s->impl.get();
    int32_t nc = 0;
    krs_status st = q->basis(nullptr, ldc, 0, &nc);  // count only: no device work
    if (st != KRS_OK) return st;
    if (n_c) *n_c = nc;
    if (!C) return KRS_OK;
    const int64_t n = q->desc.n;
    if (ldc < n || cap < nc) {
        set_error("output basis too small");
        return KRS_E_INVALID;
    }
    if ((size_t)n * sizeof(double) > krs::noalloc_scratch_bytes()) {
        set_error("krs_seq_basis_noalloc: n = " + std::to_string(n) + " needs " +
                  std::to_string((size_t)n * sizeof(double)) + " bytes of staging, beyond the " +
                  std::to_string(krs::noalloc_scratch_bytes()) + "-byte scratch (n <= " +
                  std::to_string(krs::noalloc_scratch_bytes() / sizeof(double)) + ")");
        return KRS_E_INVALID;
    }
    void* staging = krs::noalloc_scratch(q->ctx->device);
    if (!staging) {
        set_error("krs_seq_basis_noalloc: scratch address unknown on this device");
        return KRS_E_DEVICE;
    }
    return q->basis_staged(C, ldc, (double*)staging);
    KRS_GUARD_END
}

krs_status krs_seq_info(krs_seq* s, krs_solve_info* info) {
    KRS_GUARD_BEGIN
    if (!s || !info) return KRS_E_INVALID;
    *info = s->impl->info_last;
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_seq_set_timing(krs_seq* s, int32_t enable) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_E_INVALID;
    s->impl->timing = enable != 0;
    for (int j = 0; j < 3; ++j) {
        s->impl->kt_count[j] = 0;
        s->impl->kt_ms[j] = 0.0;
    }
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_seq_kernel_time(krs_seq* s, int32_t kernel, int64_t* launches, double* total_ms) {
    KRS_GUARD_BEGIN
    if (!s || kernel < 0 || kernel > 2) return KRS_E_INVALID;
    if (launches) *launches = s->impl->kt_count[kernel];
    if (total_ms) *total_ms = s->impl->kt_ms[kernel];
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_seq_destroy(krs_seq* s) {
    KRS_GUARD_BEGIN
    if (!s) return KRS_OK;
    if (s->impl->in_server.load() > 0) {
        set_error("the sequence has server requests in flight");
        return KRS_E_STATE;
    }
    krs_ctx* ctx = s->impl->ctx;
    (void)hipStreamSynchronize(ctx->stream);
    s->impl->destroy();
    ctx->live_seqs -= 1;
    delete s;
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_nc_limit(const double* alpha, const double* rho, int32_t m, double bytes_iter0, double bytes_col_iter,
                        double bytes_rebuild0, double bytes_col_rebuild, int32_t kmax, double eps, double* cost,
                        int32_t* k_out, int32_t* nc_lim) {
    KRS_GUARD_BEGIN
    if (!nc_lim || m < 0 || kmax < 0 || (m > 0 && (!alpha || !rho))) {
        set_error("alpha, rho and nc_lim are required");
        return KRS_E_INVALID;
    }
    for (int j = 0; j < m; ++j)
        if (!(alpha[j] > 0.0) || !(rho[j] > 0.0)) {
            set_error("coefficients must be positive");
            return KRS_E_INVALID;
        }
    krs::NcCostModel cm;
    cm.bytes_iter0 = bytes_iter0;
    cm.bytes_col_iter = bytes_col_iter;
    cm.bytes_rebuild0 = bytes_rebuild0;
    cm.bytes_col_rebuild = bytes_col_rebuild;
    cm.kmax = kmax;
    cm.eps = eps;
    std::vector<double> c;
    const unsigned hc = std::thread::hardware_concurrency();
    *nc_lim = krs::nc_limit(alpha, rho, m, cm, (int)std::min(16u, std::max(1u, hc)), &c);
    if (k_out) *k_out = c.empty() ? 0 : (int32_t)c.size() - 1;
    if (cost)
        for (size_t k = 0; k < c.size(); ++k) cost[k] = c[k];
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_cluster_reselect(const double* theta, int32_t m, double min_frac, uint8_t* flags) {
    KRS_GUARD_BEGIN
    if (m < 0 || (m > 0 && (!theta || !flags)) || !(min_frac > 0.0) || min_frac > 1.0) {
        set_error("theta and flags are required, 0 < min_frac <= 1");
        return KRS_E_INVALID;
    }
    std::vector<double> th(theta, theta + m);
    std::vector<int> sel;
    for (int i = 0; i < m; ++i) {
        if (!flags[i]) continue;
        if (!(theta[i] > 0.0)) {
            set_error("preselected Ritz values must be positive");
            return KRS_E_INVALID;
        }
        sel.push_back(i);
    }
    const std::vector<int> keep = krs::cluster_reselect(th, sel, min_frac);
    for (int i = 0; i < m; ++i) flags[i] = 0;
    for (int i : keep) flags[i] = 1;
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_ritz_select(const double* alpha, const double* rho, int32_t m, double eps, double* theta,
                           double* theta_prev, uint8_t* selected) {
    KRS_GUARD_BEGIN
    if (m < 0 || (m > 0 && (!alpha || !rho))) {
        set_error("alpha and rho are required");
        return KRS_E_INVALID;
    }
    for (int j = 0; j < m; ++j) {
        if (!(alpha[j] > 0.0) || !(rho[j] > 0.0)) {
            set_error("alpha and rho must be positive");
            return KRS_E_INVALID;
        }
    }
    const krs::QdArray z = krs::qd_from_cg(alpha, rho, m);
    std::vector<double> th, th1;
    krs::qd_eigenvalues_desc(z, th, 8);
    if (m > 1) krs::qd_eigenvalues_desc(krs::qd_leading(z, m - 1), th1, 8);
    std::vector<int> sel = krs::stagnation_select(th, th1, eps);
    for (int i = 0; i < m; ++i) {
        if (theta) theta[i] = th[i];
        if (selected) selected[i] = 0;
    }
    for (int i = 0; i + 1 < m; ++i)
        if (theta_prev) theta_prev[i] = th1[i];
    if (selected)
        for (int i : sel) selected[i] = 1;
    return KRS_OK;
    KRS_GUARD_END
}

krs_status krs_coarse_factor(int32_t nc, const double* G, double rank_tol, double* Ginv, uint8_t* kept,
                             int32_t* nk) {
    KRS_GUARD_BEGIN
    if (nc < 0 || (nc > 0 && (!G || !Ginv || !kept))) {
        set_error("G, Ginv and kept are required");
        return KRS_E_INVALID;
    }
    const int k = krs::coarse_factor(nc, G, rank_tol > 0 ? rank_tol : 1e-6, Ginv, kept);
    if (nk) *nk = k;
    return (nc > 0 && k == 0) ? KRS_E_COARSE_SINGULAR : KRS_OK;
    KRS_GUARD_END
}

static krs_status batch_common(krs_ctx* ctx, krs_seq* const* seqs, int32_t count, double* const* x, bool device_x,
                               krs_solve_info* info, int32_t* n_added = nullptr, bool recycle = false) {
    if (!ctx || count < 0 || (count > 0 && !seqs)) {
        set_error("ctx and seqs are required");
        return KRS_E_INVALID;
    }
    std::vector<krs::SeqBase*> v(count);
    for (int i = 0; i < count; ++i) {
        if (!seqs[i] || seqs[i]->impl->ctx != ctx) {
            set_error("every sequence must belong to ctx");
            return KRS_E_INVALID;
        }
        if (seqs[i]->impl->in_server.load() > 0) {
            set_error("a sequence of the batch has server requests in flight");
            return KRS_E_BUSY;
        }
        if (seqs[i]->impl->desc.kernel_flags & 4) {
            set_error("full reorthogonalisation is not available in fused batches (solve the sequence alone)");
            return KRS_E_INVALID;
        }
        for (int j = 0; j < i; ++j)
            if (seqs[j] == seqs[i]) {
                set_error("a sequence appears twice in the batch");
                return KRS_E_INVALID;
            }
        v[i] = seqs[i]->impl.get();
    }
    if (!recycle) return krs::batch_solve(ctx, v.data(), count, x, device_x, info);
    std::vector<int32_t> added(count, 0);
    const krs_status st = krs::batch_solve(ctx, v.data(), count, x, device_x, info, added.data());
    if (n_added)
        for (int i = 0; i < count; ++i) n_added[i] = added[i];
    return st;
}

krs_status krs_batch_recycle(krs_ctx* ctx, krs_seq* const* seqs, int32_t count, int32_t* n_added) {
    KRS_GUARD_BEGIN
    if (!ctx || count < 0 || (count > 0 && !seqs)) {
        set_error("ctx and seqs are required");
        return KRS_E_INVALID;
    }
    std::vector<krs::SeqBase*> v(count);
    for (int i = 0; i < count; ++i) {
        if (!seqs[i] || seqs[i]->impl->ctx != ctx) {
            set_error("every sequence must belong to ctx");
            return KRS_E_INVALID;
        }
        if (seqs[i]->impl->in_server.load() > 0) {
            set_error("a sequence of the batch has server requests in flight");
            return KRS_E_BUSY;
        }
        if (seqs[i]->impl->desc.kernel_flags & 4) {
            set_error("full reorthogonalisation is not available in fused batches (solve the sequence alone)");
            return KRS_E_INVALID;
        }
        for (int j = 0; j < i; ++j)
            if (seqs[j] == seqs[i]) {
                set_error("a sequence appears twice in the batch");
                return KRS_E_INVALID;
            }
        v[i] = seqs[i]->impl.get();
    }
    return krs::recycle_all(ctx, v.data(), count, n_added);
    KRS_GUARD_END
}

krs_status krs_batch_solve(krs_ctx* ctx, krs_seq* const* seqs, int32_t count, double* const* x, krs_solve_info* info) {
    KRS_GUARD_BEGIN
    return batch_common(ctx, seqs, count, x, false, info);
    KRS_GUARD_END
}

krs_status krs_batch_solve_device(krs_ctx* ctx, krs_seq* const* seqs, int32_t count, double* const* d_x,
                                  krs_solve_info* info) {
    KRS_GUARD_BEGIN
    return batch_common(ctx, seqs, count, d_x, true, info);
    KRS_GUARD_END
}

krs_status krs_batch_solve_recycle(krs_ctx* ctx, krs_seq* const* seqs, int32_t count, double* const* d_x,
                                   krs_solve_info* info, int32_t* n_added) {
    KRS_GUARD_BEGIN
    return batch_common(ctx, seqs, count, d_x, true, info, n_added, true);
    KRS_GUARD_END
}

}  // extern "C"
