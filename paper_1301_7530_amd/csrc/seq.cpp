// Sequence runtime: system intake, coarse rebuild, the iteration driver and
// Krylov reuse (TRKS, Algorithm 2; SRKS, Algorithm 3) for one sequence of
// systems A^(k) x^(k) = b^(k) sharing a sparsity pattern.
#include "seq.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <stdexcept>
#include <thread>

namespace krs {

namespace {

inline int host_threads() {
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 4;
    return (int)std::min(16u, h);
}

}  // namespace

// ------------------------------------------------------------- memory

void* dev_alloc(krs_ctx* ctx, size_t bytes) {
    if (bytes == 0) bytes = 64;
    bytes = (bytes + 255) & ~(size_t)255;
    void* p = nullptr;
    if (ctx->has_alloc) {
        p = ctx->alloc.alloc(ctx->alloc.user, bytes, (void*)ctx->stream);
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    }
    if (p) ctx->bytes_live.fetch_add((int64_t)bytes);
    return p;
}

void dev_free(krs_ctx* ctx, void* p, size_t bytes) {
    if (!p) return;
    bytes = (bytes + 255) & ~(size_t)255;
    if (ctx->has_alloc) ctx->alloc.free(ctx->alloc.user, p, (void*)ctx->stream);
    else (void)hipFree(p);
    ctx->bytes_live.fetch_sub((int64_t)bytes);
}

bool Buf::reserve(krs_ctx* ctx, size_t nbytes) {
    if (nbytes <= bytes && p) return true;
    release(ctx);
    p = dev_alloc(ctx, nbytes);
    if (!p) return false;
    bytes = nbytes;
    return true;
}

bool Buf::grow_keep(krs_ctx* ctx, size_t nbytes, hipStream_t stream) {
    if (nbytes <= bytes && p) return true;
    void* q = dev_alloc(ctx, nbytes);
    if (!q) return false;
    if (p && bytes) {
        if (hipMemcpyAsync(q, p, bytes, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
            dev_free(ctx, q, nbytes);
            return false;
        }
        if (hipStreamSynchronize(stream) != hipSuccess) {
            dev_free(ctx, q, nbytes);
            return false;
        }
    }
    release(ctx);
    p = q;
    bytes = nbytes;
    return true;
}

void Buf::release(krs_ctx* ctx) {
    if (p) dev_free(ctx, p, bytes);
    p = nullptr;
    bytes = 0;
}

// ------------------------------------------------------------- helpers

#define KRS_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #call); \
            return KRS_E_DEVICE;                                                       \
        }                                                                              \
    } while (0)

#define KRS_CHECK_LAUNCH()                                                             \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess) {                                                        \
            set_error(std::string("kernel launch failed: ") + hipGetErrorString(e_));  \
            return KRS_E_DEVICE;                                                       \
        }                                                                              \
    } while (0)

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void start(hipStream_t s) { (void)hipEventRecord(a, s); }
    void stop(hipStream_t s) { (void)hipEventRecord(b, s); }
    double ms() {
        float t = 0.f;
        (void)hipEventSynchronize(b);
        (void)hipEventElapsedTime(&t, a, b);
        return (double)t;
    }
};

// ------------------------------------------------------------ creation

template <typename V, typename W>
krs_status SeqImpl<V, W>::create(const krs_seq_desc& d, const double* C0, int32_t m0, int64_t ldc0) {
    desc = d;
    desc.row_ptr = nullptr;
    desc.col_idx = nullptr;
    B = d.block;
    n = d.n;
    nb = n / B;
    nnzb = d.nnzb;
    stream = ctx->stream;
    if (desc.rank_tol <= 0.0) desc.rank_tol = 1e-6;
    if (desc.refine_drop == 0.0) desc.refine_drop = 0.1;
    if (desc.ritz_eps <= 0.0) desc.ritz_eps = 1e-14;
    if (desc.cluster_min_frac <= 0.0) desc.cluster_min_frac = 0.2;
    const int64_t* rp = d.row_ptr;
    const int32_t* ci = d.col_idx;
    // ---- sliced ELL layout
    nslices = (nb + kSlice - 1) / kSlice;
    std::vector<int64_t> slice_ptr(nslices + 1, 0);
    for (int64_t s = 0; s < nslices; ++s) {
        int64_t w = 0;
        for (int64_t r = s * kSlice; r < std::min(nb, (s + 1) * kSlice); ++r) w = std::max(w, rp[r + 1] - rp[r]);
        slice_ptr[s + 1] = slice_ptr[s] + w;
    }
    nslots = slice_ptr[nslices];
    std::vector<int32_t> col((size_t)nslots * kSlice, 0);
    std::vector<int64_t> map(nnzb, 0);
    std::vector<int64_t> diag(nb, -1);
    for (int64_t s = 0; s < nslices; ++s) {
        const int64_t w = slice_ptr[s + 1] - slice_ptr[s];
        for (int l = 0; l < kSlice; ++l) {
            const int64_t r = s * kSlice + l;
            const int64_t len = (r < nb) ? rp[r + 1] - rp[r] : 0;
            for (int64_t k = 0; k < w; ++k) {
                const int64_t E = (slice_ptr[s] + k) * kSlice + l;
                if (k < len) {
                    const int64_t t = rp[r] + k;
                    col[E] = ci[t];
                    map[t] = E;
                    if (ci[t] == r) diag[r] = t;
                } else {
                    col[E] = (int32_t)(r < nb ? r : 0);
                }
            }
        }
    }
    for (int64_t r = 0; r < nb; ++r)
        if (diag[r] < 0) {
            set_error("every (block) row needs its diagonal entry");
            return KRS_E_INVALID;
        }
    // The double-precision 3x3 SpMV streams the block columns as 16-bit
    // differences from the entry's own block row when every one fits (on a
    // mesh numbered plane by plane they stay within a few planes): 2 bytes
    // per 76-byte block instead of 4, the same columns, so the same sums.
    // Lanes past the last block row (in the last slice) read row nb - 1.
    std::vector<int16_t> col16;
    if (B == 3 && (std::is_same<V, double>::value || op64())) {
        bool fits = true;
        col16.assign(col.size(), 0);
        for (int64_t s = 0; s < nslices && fits; ++s)
            for (int64_t k = slice_ptr[s]; k < slice_ptr[s + 1] && fits; ++k)
                for (int l = 0; l < kSlice; ++l) {
                    const int64_t r = s * kSlice + l;
                    if (r >= nb) break;
                    const int64_t E = k * kSlice + l;
                    const int64_t d = (int64_t)col[E] - r;
                    if (d < INT16_MIN || d > INT16_MAX) {
                        fits = false;
                        break;
                    }
                    col16[E] = (int16_t)d;
                }
        if (!fits) col16.clear();
    }
    const size_t vb = (size_t)B * B;
    bool ok = true;
    ok = ok && d_col.reserve(ctx, col.size() * sizeof(int32_t));
    if (!col16.empty()) ok = ok && d_col16.reserve(ctx, col16.size() * sizeof(int16_t));
    else d_col16.release(ctx);
    ok = ok && d_slice_ptr.reserve(ctx, slice_ptr.size() * sizeof(int64_t));
    ok = ok && d_map.reserve(ctx, map.size() * sizeof(int64_t));
    ok = ok && d_diag.reserve(ctx, diag.size() * sizeof(int64_t));
    ok = ok && d_val64.reserve(ctx, (size_t)nslots * kSlice * vb * sizeof(double));
    if (!std::is_same<V, double>::value && !op64())
        ok = ok && d_valV.reserve(ctx, (size_t)nslots * kSlice * vb * sizeof(V));
    ok = ok && d_minv.reserve(ctx, (size_t)nb * vb * sizeof(V));
    ok = ok && d_bad.reserve(ctx, 64);
    ok = ok && d_b.reserve(ctx, n * sizeof(double));
    ok = ok && d_x.reserve(ctx, n * sizeof(double));
    ok = ok && d_r.reserve(ctx, n * sizeof(W));
    ok = ok && d_s.reserve(ctx, n * sizeof(W));
    ok = ok && d_w.reserve(ctx, n * sizeof(W));
    ok = ok && d_q.reserve(ctx, n * sizeof(W));
    ok = ok && d_st.reserve(ctx, kSyncOffset + kSyncBytes);
    ok = ok && d_mu.reserve(ctx, 3072 * sizeof(double));
    if (!ok) {
        set_error("device allocation failed while creating the sequence");
        return KRS_E_OOM;
    }
    // the uploads below read these host vectors: every way out of this
    // function waits for the stream before they are destroyed
    struct WaitOnExit {
        hipStream_t s;
        ~WaitOnExit() { (void)hipStreamSynchronize(s); }
    } wait_on_exit{stream};
    KRS_HIP(hipMemcpyAsync(d_col.p, col.data(), col.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    if (!col16.empty())
        KRS_HIP(hipMemcpyAsync(d_col16.p, col16.data(), col16.size() * sizeof(int16_t), hipMemcpyHostToDevice,
                               stream));
    KRS_HIP(hipMemcpyAsync(d_slice_ptr.p, slice_ptr.data(), slice_ptr.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                           stream));
    KRS_HIP(hipMemcpyAsync(d_map.p, map.data(), map.size() * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    KRS_HIP(hipMemcpyAsync(d_diag.p, diag.data(), diag.size() * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    KRS_HIP(hipMemsetAsync(d_val64.p, 0, d_val64.bytes, stream));
    if (d_valV.p) KRS_HIP(hipMemsetAsync(d_valV.p, 0, d_valV.bytes, stream));
    KRS_HIP(hipMemsetAsync(d_st.p, 0, kSyncOffset + kSyncBytes, stream));
    KRS_HIP(hipHostMalloc((void**)&h_st, sizeof(DevState), hipHostMallocDefault));
    std::memset(h_st, 0, sizeof(DevState));
    // ---- initial basis C0
    ldc = (n + 255) & ~(int64_t)255;
    geo = make_geometry(n, nslices, B, desc.update_rows, spmv_grid_cap());
    nc = 0;
    if (m0 > 0) {
        if (!C0 || ldc0 < n) {
            set_error("C0 must be n x m0 with ldc0 >= n");
            return KRS_E_INVALID;
        }
        if (!ensure_c_capacity(m0)) return KRS_E_OOM;
        if (!d_C0.reserve(ctx, (size_t)ldc * m0 * sizeof(V))) return KRS_E_OOM;
        Buf tmp;
        if (!tmp.reserve(ctx, (size_t)n * sizeof(double))) return KRS_E_OOM;
        for (int c = 0; c < m0; ++c) {
            KRS_HIP(hipMemcpyAsync(tmp.p, C0 + (size_t)c * ldc0, n * sizeof(double), hipMemcpyHostToDevice, stream));
            launch_d2v<V>((const double*)tmp.p, (V*)d_C.p + (size_t)c * ldc, n, stream);
            launch_d2v<V>((const double*)tmp.p, (V*)d_C0.p + (size_t)c * ldc, n, stream);
        }
        KRS_HIP(hipStreamSynchronize(stream));
        tmp.release(ctx);
        nc = m0;
    }
    nc0 = m0;
    KRS_HIP(hipStreamSynchronize(stream));
    return KRS_OK;
}

template <typename V, typename W>
bool SeqImpl<V, W>::ensure_c_capacity(int cols) {
    if (cols <= nc_cap && d_C.p) return true;
    int cap = std::max(cols, std::max(8, nc_cap + nc_cap / 2));
    if (cap > 1024 && cols <= 1024) cap = 1024;
    if (!d_C.grow_keep(ctx, (size_t)ldc * cap * sizeof(V), stream)) {
        set_error("device allocation failed for the basis");
        return false;
    }
    nc_cap = cap;
    return true;
}

template <typename V, typename W>
void SeqImpl<V, W>::destroy() {
    for (Buf* b : {&d_col16, &d_col, &d_slice_ptr, &d_map, &d_diag, &d_val64, &d_valV, &d_minv, &d_bad, &d_in, &d_b, &d_x,
                   &d_r, &d_s, &d_w, &d_q, &d_C, &d_C0, &d_AC64, &d_ACv, &d_G, &d_Ginv, &d_mu, &d_Z, &d_coef,
                   &d_partials, &d_st, &d_F, &d_tmp, &d_Ctmp, &d_kslots, &d_Wr, &d_Qr, &d_rpart, &d_rc, &d_zr})
        b->release(ctx);
    if (h_st) (void)hipHostFree(h_st);
    h_st = nullptr;
    if (h_coef) (void)hipHostFree(h_coef);
    h_coef = nullptr;
    h_coef_cap = 0;
    if (h_G) (void)hipHostFree(h_G);
    h_G = nullptr;
    h_G_cap = 0;
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    graph_release();
}

// ------------------------------------------------------------- submit

template <typename V, typename W>
krs_status SeqImpl<V, W>::submit(const double* values, const double* b, bool device) {
    rb_done = false;  // a new matrix needs its own rebuild
    if (!values || !b) {
        set_error("values and b are required");
        return KRS_E_INVALID;
    }
    Timer tm;
    tm.start(stream);
    const size_t vb = (size_t)B * B;
    const double* vin = values;
    if (!device) {
        if (!d_in.reserve(ctx, (size_t)nnzb * vb * sizeof(double))) {
            set_error("device allocation failed for the value staging buffer");
            return KRS_E_OOM;
        }
        KRS_HIP(hipMemcpyAsync(d_in.p, values, (size_t)nnzb * vb * sizeof(double), hipMemcpyHostToDevice, stream));
        KRS_HIP(hipMemcpyAsync(d_b.p, b, n * sizeof(double), hipMemcpyHostToDevice, stream));
        vin = (const double*)d_in.p;
    } else {
        KRS_HIP(hipMemcpyAsync(d_b.p, b, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
    }
    V* valV = (std::is_same<V, double>::value || op64()) ? nullptr : (V*)d_valV.p;
    KRS_HIP(hipMemsetAsync(d_bad.p, 0, 64, stream));
    if (B == 1) {
        launch_scatter_values<V, 1>(vin, (const int64_t*)d_map.p, nnzb, (double*)d_val64.p, valV, stream);
        launch_precond_setup<V, 1>(vin, (const int64_t*)d_diag.p, nb, (V*)d_minv.p, (int32_t*)d_bad.p, stream);
    } else {
        launch_scatter_values<V, 3>(vin, (const int64_t*)d_map.p, nnzb, (double*)d_val64.p, valV, stream);
        if (desc.precond == KRS_PC_BJACOBI3) {
            launch_precond_setup<V, 3>(vin, (const int64_t*)d_diag.p, nb, (V*)d_minv.p, (int32_t*)d_bad.p, stream);
        } else {
            set_error("block-3 systems use the 3x3 block-Jacobi preconditioner");
            return KRS_E_INVALID;
        }
    }
    KRS_CHECK_LAUNCH();
    int32_t bad = 0;
    KRS_HIP(hipMemcpyAsync(&bad, d_bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    tm.stop(stream);
    KRS_HIP(hipStreamSynchronize(stream));
    info_last.t_setup_ms = tm.ms();
    if (bad) {
        set_error("preconditioner pivot not positive: the diagonal (blocks) of A are not SPD");
        submitted = false;
        return KRS_E_NOT_SPD;
    }
    submitted = true;
    return KRS_OK;
}

// --------------------------------------------------------------- views

template <typename V, typename W>
SysView<V, W> SeqImpl<V, W>::view() {
    SysView<V, W> v;
    std::memset(&v, 0, sizeof v);
    v.col = (const int32_t*)d_col.p;
    // with the default load schedule (kernel_flags bits 3-6 zero)
    v.col16 = ((desc.kernel_flags >> 3) & 15) == 0 ? (const int16_t*)d_col16.p : nullptr;
    v.slice_ptr = (const int64_t*)d_slice_ptr.p;
    v.val = std::is_same<V, double>::value ? (const V*)d_val64.p : (const V*)d_valV.p;
    v.op64 = (std::is_same<V, double>::value || op64()) ? 1 : 0;
    v.val64 = (const double*)d_val64.p;
    v.minv = (const V*)d_minv.p;
    v.n = n;
    v.nb = nb;
    v.nslices = nslices;
    v.x = (double*)d_x.p;
    v.b = (const double*)d_b.p;
    v.r = (W*)d_r.p;
    v.s = (W*)d_s.p;
    v.w = (W*)d_w.p;
    v.q = (W*)d_q.p;
    v.C = (const V*)d_C.p;
    v.AC = std::is_same<V, double>::value ? (const V*)d_AC64.p : (const V*)d_ACv.p;
    v.nc = nc;
    v.geo = geo;
    v.ldc = ldc;
    v.ldac = ldac;
    v.Ginv = (const double*)d_Ginv.p;
    v.mu = (double*)d_mu.p;
    v.u = (double*)d_mu.p + 1024;
    v.mu2 = (double*)d_mu.p + 2048;
    v.zhist = nullptr;
    v.whist = nullptr;
    v.ldh = ldc;
    if (desc.reuse == KRS_REUSE_SELECTIVE) {
        if (hist32()) v.zhist32 = (float*)d_Z.p;
        else v.zhist = (V*)d_Z.p;
    }
    if (desc.reuse == KRS_REUSE_TOTAL && trks_slots > 0) v.whist = (V*)d_C.p + (size_t)nc * ldc;
    v.alpha_h = (double*)d_coef.p;
    v.rho_h = v.alpha_h + coef_cap;
    v.gamma_h = v.rho_h + coef_cap;
    v.coef_cap = coef_cap;
    v.part1 = (double*)d_partials.p;
    v.partials = (double*)d_partials.p + kPart1;
    v.st = (DevState*)d_st.p;
    v.sync = (unsigned*)((char*)d_st.p + kSyncOffset);
    v.kslots = (unsigned long long*)d_kslots.p;
    v.fused = (desc.kernel_flags & 1) ? 0 : 1;
    v.dir_literal = (desc.kernel_flags & 2) ? 1 : 0;
    v.spmv_var = (desc.kernel_flags >> 3) & 3;
    if (((desc.kernel_flags >> 3) & 15) == 0 && B == 3 && v.op64 && nslots * 64 * 9 * (int64_t)sizeof(double) > kNtBytes)
        v.spmv_var = 2;  // a matrix larger than the last-level cache streams with non-temporal loads
    // With the streaming schedule the vectors an iteration writes (q; x, r,
    // s; w and the history) go out with non-temporal stores: normal stores
    // leave dirty lines in the caches whose write-back then falls inside
    // the next kernel, which streams the matrix.
    v.nt_store = ((v.spmv_var & 2) && !(desc.kernel_flags & 256)) ? 1 : 0;
    if (reorth() && rcap > 0) {
        v.Wr = (W*)d_Wr.p;
        v.Qr = (W*)d_Qr.p;
        v.ldr = ldr;
        v.rcap = rcap;
        v.gr = rgr;
        v.rpart = (double*)d_rpart.p;
        v.rc = (double*)d_rc.p;
        v.zr = (W*)d_zr.p;
    }
    return v;
}

// ---------------------------------------------------- kernel dispatch

template <typename V, typename W>
void SeqImpl<V, W>::k_spmv(const SysView<V, W>& v) {
    if (B == 1) launch_spmv_dot<V, W, 1>(v, stream);
    else launch_spmv_dot<V, W, 3>(v, stream);
}
template <typename V, typename W>
void SeqImpl<V, W>::k_update(const SysView<V, W>& v, int mode) {
    if (B == 1) launch_update_reduce<V, W, 1>(v, mode, stream);
    else launch_update_reduce<V, W, 3>(v, mode, stream);
}
template <typename V, typename W>
void SeqImpl<V, W>::k_resid(const SysView<V, W>& v, int final_only) {
    if (B == 1) launch_true_resid<V, W, 1>(v, final_only, stream);
    else launch_true_resid<V, W, 3>(v, final_only, stream);
}

template <typename V, typename W>
void SeqImpl<V, W>::enqueue_iterations(const SysView<V, W>& v, int k) {
    for (int i = 0; i < k; ++i) {
        k_spmv(v);
        if (v.Wr) launch_reorth_store<V, W>(v, stream);
        k_update(v, 0);
        launch_correct_dir<V, W>(v, 0, stream);
        if (v.Wr) launch_reorth<V, W>(v, stream);
    }
}

template <typename V, typename W>
void SeqImpl<V, W>::enqueue_refine(const SysView<V, W>& v) {
    k_resid(v, 0);
    if (nc > 0) {
        launch_coarse_dot<V, W>(v, 0, 0, M_REFINE, stream);
        launch_coarse_correct<V, W>(v, 0, M_REFINE, stream);
    }
    k_update(v, 2);
    launch_correct_dir<V, W>(v, 2, stream);
}

// Replay a captured block of `block` iterations plus the refinement step.
// The capture is reused while the launch view (pointers, sizes, basis
// width) is unchanged; every kernel reads its scalars from device memory,
// so a replay needs no host-side arguments.
template <typename V, typename W>
krs_status SeqImpl<V, W>::graph_launch(const SysView<V, W>& v, int slot, int block) {
    GraphSlot& g = gslot[slot];
    if (!g.exec || g.block != block || std::memcmp(&g.view, &v, sizeof v) != 0) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        g.exec = nullptr;
        g.graph = nullptr;
        KRS_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        enqueue_iterations(v, block);
        enqueue_refine(v);
        hipError_t e = hipStreamEndCapture(stream, &g.graph);
        if (e != hipSuccess) {
            set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
            return KRS_E_DEVICE;
        }
        KRS_HIP(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
        g.view = v;
        g.block = block;
    }
    KRS_HIP(hipGraphLaunch(g.exec, stream));
    return KRS_OK;
}

template <typename V, typename W>
void SeqImpl<V, W>::graph_release() {
    for (auto& g : gslot) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        g.exec = nullptr;
        g.graph = nullptr;
    }
}

// ------------------------------------------------------------- rebuild

// A C (double) for the current basis, and G = C^T A C on the host.
template <typename V, typename W>
krs_status SeqImpl<V, W>::coarse_pass(std::vector<double>& G) {
    krs_status st = coarse_pass_enqueue();
    if (st != KRS_OK) return st;
    KRS_HIP(hipStreamSynchronize(stream));
    coarse_pass_read(G);
    return KRS_OK;
}

// The pass's kernels and the read-back of G into pinned memory, enqueued.
template <typename V, typename W>
krs_status SeqImpl<V, W>::coarse_pass_enqueue() {
    const size_t nn = (size_t)nc * nc;
    const bool need_v = !std::is_same<V, double>::value;
    ldac = ac_leading_dim(nc, sizeof(V));
    if (!d_AC64.reserve(ctx, (size_t)n * ldac * sizeof(double)) ||
        (need_v && !d_ACv.reserve(ctx, (size_t)n * ldac * sizeof(V))) || !d_G.reserve(ctx, nn * sizeof(double)) ||
        !d_Ginv.reserve(ctx, nn * sizeof(double)) || !d_mu.reserve(ctx, 3072 * sizeof(double))) {
        set_error("device allocation failed for A C / C^T A C");
        return KRS_E_OOM;
    }
    const int64_t gram_cap = (int64_t)std::min<size_t>(64 * nn, (size_t)16 << 20);
    if (!ensure_partials(gram_cap)) return KRS_E_OOM;
    SysView<V, W> v = view();
    V* ACv = std::is_same<V, double>::value ? (V*)d_AC64.p : (V*)d_ACv.p;
    if (B == 1) launch_spmm<V, W, 1>(v, (const V*)d_C.p, ldc, nc, ldac, (double*)d_AC64.p, ACv, stream);
    else launch_spmm<V, W, 3>(v, (const V*)d_C.p, ldc, nc, ldac, (double*)d_AC64.p, ACv, stream);
    launch_gram<V>((const V*)d_C.p, ldc, (const double*)d_AC64.p, ldac, n, nc, (double*)d_G.p,
                   (double*)d_partials.p + kPart1, (int64_t)(d_partials.bytes / sizeof(double)) - kPart1, stream);
    KRS_CHECK_LAUNCH();
    if (h_G_cap < nn) {
        if (h_G) (void)hipHostFree(h_G);
        h_G = nullptr;
        h_G_cap = 0;
        if (hipHostMalloc((void**)&h_G, nn * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            h_G = nullptr;
            set_error("pinned host allocation failed for C^T A C");
            return KRS_E_OOM;
        }
        h_G_cap = nn;
    }
    KRS_HIP(hipMemcpyAsync(h_G, d_G.p, nn * sizeof(double), hipMemcpyDeviceToHost, stream));
    return KRS_OK;
}

// G from the pinned read-back (after a wait), symmetrised.
template <typename V, typename W>
void SeqImpl<V, W>::coarse_pass_read(std::vector<double>& G) const {
    const size_t nn = (size_t)nc * nc;
    G.assign(h_G, h_G + nn);
    for (int a = 0; a < nc; ++a)
        for (int b = a + 1; b < nc; ++b) {
            const double s = 0.5 * (G[(size_t)a * nc + b] + G[(size_t)b * nc + a]);
            G[(size_t)a * nc + b] = s;
            G[(size_t)b * nc + a] = s;
        }
}

// Rebuild of the coarse space for A^(k) (Algorithm 1, first step):
//  1. A C, G = C^T A C; guarded Cholesky G = L L^T (drops dependent columns);
//  2. C <- C_k L_k^{-T}: the carried basis made A^(k)-orthonormal.  The
//     projector P and x0 depend on span(C) only, so the iteration is the
//     same; the coarse matrix becomes ~I, which keeps the single-precision
//     projector accurate;
//  3. A C and G again for the new basis, G^-1 for the iterations.
// The stages of rebuild_stage with a wait after each: a batch runs the same
// stages for all its members with one wait per stage.
template <typename V, typename W>
krs_status SeqImpl<V, W>::rebuild(int* dropped) {
    *dropped = 0;
    bool more = false;
    krs_status st = rebuild_stage(0, &more);
    for (int stage = 1; st == KRS_OK && more && stage <= 2; ++stage) {
        KRS_HIP(hipStreamSynchronize(stream));
        st = rebuild_stage(stage, &more);
    }
    rb_done = false;
    if (st != KRS_OK) return st;
    *dropped = rb_dropped;
    return KRS_OK;
}

// The rebuild split at its waits (stage 0: the first A C / Gram pass;
// stage 1, after a wait: the guarded orthonormalisation, the basis change
// and the second pass; stage 2, after a wait: the guarded factorisation and
// the upload of G^-1, or the remaining passes on this member alone when a
// column vanished after the change of basis).
template <typename V, typename W>
krs_status SeqImpl<V, W>::rebuild_stage(int stage, bool* more) {
    *more = false;
    if (stage == 0) {
        rb_done = false;
        rb_dropped = 0;
        if (!submitted || nc > 1024) return KRS_OK;  // begin_solve reports these
        // the start of the rebuild phase, which begin_solve leaves out when staged
        for (auto& e : ev)
            if (!e) KRS_HIP(hipEventCreate(&e));
        KRS_HIP(hipEventRecord(ev[0], stream));
        if (nc == 0) {
            rb_done = true;
            return KRS_OK;
        }
        krs_status st = coarse_pass_enqueue();
        *more = st == KRS_OK;
        return st;
    }
    std::vector<double> G;
    coarse_pass_read(G);
    if (stage == 1) {
        // the carried basis made A^(k)-orthonormal, then the second pass
        rb_up.assign((size_t)nc * nc, 0.0);
        std::vector<uint8_t> kept(nc, 1);
        const int nk = coarse_orthonormalizer(nc, G.data(), desc.rank_tol, rb_up.data(), kept.data());
        rb_dropped += nc - nk;
        if (nk == 0) {
            nc = 0;
            rb_done = true;
            return KRS_OK;
        }
        if (!d_F.reserve(ctx, (size_t)nc * nk * sizeof(double)) ||
            !d_Ctmp.reserve(ctx, (size_t)ldc * nk * sizeof(V))) {
            set_error("device allocation failed for the basis change");
            return KRS_E_OOM;
        }
        KRS_HIP(hipMemcpyAsync(d_F.p, rb_up.data(), (size_t)nc * nk * sizeof(double), hipMemcpyHostToDevice, stream));
        launch_basis_combine<V>((const V*)d_C.p, ldc, nc, (const double*)d_F.p, nk, (V*)d_Ctmp.p, ldc, n, stream);
        KRS_CHECK_LAUNCH();
        KRS_HIP(hipMemcpyAsync(d_C.p, d_Ctmp.p, (size_t)ldc * nk * sizeof(V), hipMemcpyDeviceToDevice, stream));
        nc = nk;
        krs_status st = coarse_pass_enqueue();
        *more = st == KRS_OK;
        return st;
    }
    // stage 2: G^-1, or (a column vanished after the change of basis) the
    // remaining passes of rebuild() on this member alone
    const size_t nn = (size_t)nc * nc;
    rb_up.assign(nn, 0.0);
    std::vector<uint8_t> kept(nc, 1);
    const int nk = coarse_factor(nc, G.data(), desc.rank_tol, rb_up.data(), kept.data());
    if (nk == nc) {
        KRS_HIP(hipMemcpyAsync(d_Ginv.p, rb_up.data(), nn * sizeof(double), hipMemcpyHostToDevice, stream));
        rb_done = true;
        return KRS_OK;
    }
    rb_dropped += nc - nk;
    if (nk == 0) {
        nc = 0;
        rb_done = true;
        return KRS_OK;
    }
    std::vector<int32_t> keep_map;
    for (int c = 0; c < nc; ++c)
        if (kept[c]) keep_map.push_back(c);
    if (!d_tmp.reserve(ctx, std::max<size_t>(keep_map.size() * sizeof(int32_t), 64))) return KRS_E_OOM;
    KRS_HIP(hipMemcpyAsync(d_tmp.p, keep_map.data(), keep_map.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           stream));
    launch_copy_columns<V>((const V*)d_C.p, ldc, (V*)d_C.p, ldc, n, (const int32_t*)d_tmp.p, nk, stream);
    KRS_CHECK_LAUNCH();
    KRS_HIP(hipStreamSynchronize(stream));
    nc = nk;
    for (int pass = 1; pass < 3; ++pass) {
        krs_status st = coarse_pass(G);
        if (st != KRS_OK) return st;
        const size_t m2 = (size_t)nc * nc;
        std::vector<double> Gi(m2);
        std::vector<uint8_t> kp(nc, 1);
        const int nk2 = coarse_factor(nc, G.data(), desc.rank_tol, Gi.data(), kp.data());
        if (nk2 == nc) {
            KRS_HIP(hipMemcpyAsync(d_Ginv.p, Gi.data(), m2 * sizeof(double), hipMemcpyHostToDevice, stream));
            KRS_HIP(hipStreamSynchronize(stream));
            rb_done = true;
            return KRS_OK;
        }
        rb_dropped += nc - nk2;
        if (nk2 == 0) {
            nc = 0;
            rb_done = true;
            return KRS_OK;
        }
        std::vector<int32_t> km;
        for (int c = 0; c < nc; ++c)
            if (kp[c]) km.push_back(c);
        if (!d_tmp.reserve(ctx, std::max<size_t>(km.size() * sizeof(int32_t), 64))) return KRS_E_OOM;
        KRS_HIP(hipMemcpyAsync(d_tmp.p, km.data(), km.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
        launch_copy_columns<V>((const V*)d_C.p, ldc, (V*)d_C.p, ldc, n, (const int32_t*)d_tmp.p, nk2, stream);
        KRS_CHECK_LAUNCH();
        KRS_HIP(hipStreamSynchronize(stream));
        nc = nk2;
    }
    set_error("coarse space did not stabilise under the rank guard");
    return KRS_E_COARSE_SINGULAR;
}

template <typename V, typename W>
bool SeqImpl<V, W>::ensure_partials(int64_t extra) {
    const int64_t need = kPart1 + std::max<int64_t>(partial_doubles(geo, nc), extra);
    if ((int64_t)(d_partials.bytes / sizeof(double)) >= need) return true;
    if (!d_partials.reserve(ctx, (size_t)need * sizeof(double))) {
        set_error("device allocation failed for reduction scratch");
        return false;
    }
    return true;
}

// --------------------------------------------------------------- solve

template <typename V, typename W>
int64_t SeqImpl<V, W>::working_bytes() const {
    const int max_iter = std::max(0, desc.max_iter);
    int64_t hist = 0;
    if (desc.reuse == KRS_REUSE_SELECTIVE && history_needed())
        hist = desc.history_cap > 0 ? std::min(desc.history_cap, max_iter + 1) : max_iter + 1;
    const int ncmax = std::max(nc, has_cap() ? cap_value() : nc);
    const int64_t ldm = ac_leading_dim(ncmax, sizeof(V));
    const int64_t vsz = std::is_same<V, double>::value ? 0 : (int64_t)sizeof(V);
    int64_t b = ldc * hist * hist_elem();                              // Z history
    b += n * ldm * (8 + vsz);                                          // A C (double and V)
    b += ldc * (int64_t)ncmax * (int64_t)sizeof(V);                    // basis change staging
    b += nnzb * B * B * 8;                                             // value staging
    b += (kPart1 + partial_doubles(make_geometry(n, nslices, B, desc.update_rows, spmv_grid_cap()), ncmax)) * 8;
    if (reorth()) {
        const int64_t rc = std::min<int64_t>(std::min<int64_t>(desc.max_iter + 1, kReorthMax), 1 << 30);
        b += 2 * n * ((rc + 15) / 16 * 16) * (int64_t)sizeof(W) + n * (int64_t)sizeof(W);
    }
    return b;
}

template <typename V, typename W>
void SeqImpl<V, W>::trim() {
    for (Buf* b : {&d_Z, &d_AC64, &d_ACv, &d_partials, &d_F, &d_Ctmp, &d_tmp, &d_in, &d_kslots, &d_Wr, &d_Qr, &d_rpart,
                   &d_rc, &d_zr})
        b->release(ctx);
    graph_release();
}

template <typename V, typename W>
int SeqImpl<V, W>::type_key() const {
    return (std::is_same<V, double>::value ? 0 : 1) + (std::is_same<W, double>::value ? 0 : 2) + (B == 3 ? 4 : 0) +
           ((desc.kernel_flags & 1) ? 8 : 0);
}

template <typename V, typename W>
krs_status SeqImpl<V, W>::solve(double* x, bool device_x, krs_solve_info* info) {
    krs_status st = begin_solve();
    if (st != KRS_OK) return st;
    st = iterate();
    if (st != KRS_OK) return st;
    return end_solve(x, device_x, info, h_st->iter);
}

// Update-kernel tile choice: time the update kernel alone (mode 1 rewrites
// only s = M^-1 r and the partial sums, which the initialisation that
// follows recomputes) for several block-row ranges per workgroup and keep
// the fastest.  Runs when the basis width changed by half since the last
// choice, with the device state already set to RUN.
template <typename V, typename W>
krs_status SeqImpl<V, W>::tune_update() {
    std::vector<int64_t> cand = {64, 128, 256, 512, 1024, 2048, (nb + 255) / 256, (nb + 511) / 512,
                                 (nb + 127) / 128};
    std::vector<Geometry> geos;
    for (int64_t c : cand) {
        const Geometry g = make_geometry(n, nslices, B, c, spmv_grid_cap());
        bool seen = false;
        for (const auto& h : geos) seen = seen || h.cb3 == g.cb3;
        if (!seen) geos.push_back(g);
    }
    int64_t need = 0;
    for (const auto& g : geos) need = std::max(need, partial_doubles(g, nc));
    if (!ensure_partials(need)) return KRS_E_OOM;
    for (auto& e : ev)
        if (!e) KRS_HIP(hipEventCreate(&e));
    SysView<V, W> v = view();
    double best = 1e300;
    Geometry bg = geo;
    for (const auto& g : geos) {
        v.geo = g;
        if (B == 1) launch_update_only<V, W, 1>(v, 1, stream);
        else launch_update_only<V, W, 3>(v, 1, stream);
        KRS_HIP(hipEventRecord(ev[2], stream));
        for (int r = 0; r < 5; ++r) {
            if (B == 1) launch_update_only<V, W, 1>(v, 1, stream);
            else launch_update_only<V, W, 3>(v, 1, stream);
        }
        KRS_HIP(hipEventRecord(ev[3], stream));
        KRS_CHECK_LAUNCH();
        KRS_HIP(hipEventSynchronize(ev[3]));
        float ms = 0.f;
        KRS_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
        if (ms < best) {
            best = ms;
            bg = g;
        }
    }
    geo = bg;
    tuned_nc = nc;
    return KRS_OK;
}

template <typename V, typename W>
krs_status SeqImpl<V, W>::set_update_rows(int64_t rows) {
    desc.update_rows = (int32_t)rows;
    geo = make_geometry(n, nslices, B, rows, spmv_grid_cap());
    if (!ensure_partials(0)) return KRS_E_OOM;
    cur = view();
    tuned_nc = std::max(nc, 1);
    batch_tuned = true;
    batch_tuned_nc = nc;
    return KRS_OK;
}

template <typename V, typename W>
krs_status SeqImpl<V, W>::begin_solve() {
    // a staged rebuild counts for this begin only
    const bool staged = rb_done;
    rb_done = false;
    if (!submitted) {
        set_error("krs_seq_solve needs a submitted system");
        return KRS_E_STATE;
    }
    if (nc > 1024) {
        set_error("basis larger than 1024 columns is not supported");
        return KRS_E_INVALID;
    }
    solved = false;
    for (auto& e : ev)
        if (!e) KRS_HIP(hipEventCreate(&e));
    int dropped = 0;
    krs_status st = KRS_OK;
    if (staged) {
        // rebuilt in stages by the batch (ev[0] recorded at its first stage)
        dropped = rb_dropped;
    } else {
        KRS_HIP(hipEventRecord(ev[0], stream));
        st = rebuild(&dropped);
        if (st != KRS_OK) return st;
    }
    dropped_last = dropped;
    // histories
    const int max_iter = std::max(0, desc.max_iter);
    if (coef_cap < max_iter + 2) {
        coef_cap = max_iter + 2;
        if (!d_coef.reserve(ctx, (size_t)3 * coef_cap * sizeof(double))) return KRS_E_OOM;
    }
    int hist = 0;
    trks_slots = 0;
    if (desc.reuse == KRS_REUSE_SELECTIVE && !history_needed()) {
        // nothing is appended from this run (a full frozen basis, or the
        // cost cap holds): no history
        d_Z.release(ctx);
        history_kept = 0;
    } else if (desc.reuse == KRS_REUSE_SELECTIVE) {
        hist = desc.history_cap > 0 ? std::min(desc.history_cap, max_iter + 1) : max_iter + 1;
        // keep as much of the run as memory allows: a shorter history only
        // shortens the Lanczos pair used for the Ritz analysis.  A length
        // that did not fit is not tried again by later solves (the attempt
        // would first release the reservation that does fit).
        if (history_fit > 0) hist = std::min(hist, history_fit);
        const int64_t per = ldc * hist_elem();
        const int64_t known = ctx->hist_fit_bytes.load();
        if (known > 0 && (int64_t)hist * per > known) hist = (int)std::max<int64_t>(64, known / per);
        bool failed = false;
        while (!d_Z.reserve(ctx, (size_t)ldc * hist * (size_t)hist_elem())) {
            if (hist <= 64) {
                set_error("device allocation failed for the Krylov history");
                return KRS_E_OOM;
            }
            hist /= 2;
            history_fit = hist;
            failed = true;
        }
        if (failed) ctx->hist_fit_bytes.store((int64_t)hist * per);
        history_kept = hist;
    } else if (desc.reuse == KRS_REUSE_TOTAL) {
        hist = max_iter + 1;
        if (desc.max_basis > 0) hist = std::min(hist, std::max(0, desc.max_basis - nc));
        if (desc.history_cap > 0) hist = std::min(hist, desc.history_cap);
        hist = std::min(hist, 1024 - nc);
        if (hist < 0 || cost_held()) hist = 0;
        if (!ensure_c_capacity(nc + hist)) return KRS_E_OOM;
        trks_slots = hist;
    }
    if (reorth()) {
        // every direction of the run up to kReorthMax (and the history cap)
        rcap = std::min(std::min(max_iter + 1, kReorthMax), desc.history_cap > 0 ? desc.history_cap : kReorthMax);
        rcap = std::min(rcap, coef_cap);
        ldr = ((int64_t)rcap + 15) / 16 * 16;
        // row ranges of about 1024 rows (at most 256): with the chunks of
        // kept directions they give the coefficient pass thousands of workgroups
        rgr = (int)std::max<int64_t>(1, std::min<int64_t>(256, (n + 1023) / 1024));
        if (!d_Wr.reserve(ctx, (size_t)n * ldr * sizeof(W)) || !d_Qr.reserve(ctx, (size_t)n * ldr * sizeof(W)) ||
            !d_rpart.reserve(ctx, (size_t)rgr * ldr * sizeof(double)) || !d_rc.reserve(ctx, (size_t)ldr * sizeof(double)) ||
            !d_zr.reserve(ctx, (size_t)n * sizeof(W))) {
            set_error("device allocation failed for the reorthogonalisation vectors");
            return KRS_E_OOM;
        }
    }
    if (!ensure_partials(0)) return KRS_E_OOM;
    // device state
    std::memset(h_st, 0, sizeof(DevState));
    h_st->tol2 = desc.tol * desc.tol;
    // reliable updates whenever single precision is involved
    // periodic re-projection and residual replacement whenever the basis
    // (and so the C^T r recurrence) is single precision
    const bool lowp = !std::is_same<V, double>::value;
    h_st->drop2 = (lowp && desc.refine_drop > 0.0) ? desc.refine_drop * desc.refine_drop : 0.0;
    h_st->refine_every = lowp ? desc.refine_every : 0;
    h_st->status = ST_RUN;
    h_st->first_restart = max_iter + 1;
    h_st->max_iter = max_iter;
    h_st->hist_cap = hist;
    h_st->nc = nc;
    h_st->ktime_on = timing ? 1 : 0;
    if (timing && !d_kslots.reserve(ctx, (size_t)3 * 2 * kMaxTimedGrid * sizeof(unsigned long long))) return KRS_E_OOM;
    KRS_HIP(hipMemcpyAsync(d_st.p, h_st, sizeof(DevState), hipMemcpyHostToDevice, stream));
    h_st->iter = 0;
    if (desc.autotune && !batch_tuned && nc > 0 &&
        (tuned_nc == 0 || 2 * nc > 3 * tuned_nc || 3 * nc < 2 * tuned_nc)) {
        st = tune_update();
        if (st != KRS_OK) return st;
        if (!ensure_partials(0)) return KRS_E_OOM;
    }
    SysView<V, W> v = view();
    cur = v;
    // initialisation: mu0 = Ginv C^T b, x0 = C mu0, r0 = b - AC mu0, s0, z0, w0
    launch_coarse_dot<V, W>(v, 1, 1, M_RUN, stream);
    launch_coarse_correct<V, W>(v, 1, M_RUN, stream);
    k_update(v, 1);
    launch_correct_dir<V, W>(v, 1, stream);
    KRS_CHECK_LAUNCH();
    KRS_HIP(hipEventRecord(ev[1], stream));
    return KRS_OK;
}

// Iteration blocks on the sequence's own stream; each block ends with the
// (gated) refinement step.
template <typename V, typename W>
krs_status SeqImpl<V, W>::iterate() {
    const SysView<V, W> v = cur;
    const bool graphs = desc.exec_mode == 0;
    int block = graphs ? 16 : 8;
    int last_iter = -1, stuck = 0;
    while (true) {
        if (graphs) {
            krs_status gs = graph_launch(v, block == 16 ? 0 : 1, block);
            if (gs != KRS_OK) return gs;
        } else {
            enqueue_iterations(v, block);
            enqueue_refine(v);
            KRS_CHECK_LAUNCH();
        }
        KRS_HIP(hipMemcpyAsync(h_st, d_st.p, sizeof(DevState), hipMemcpyDeviceToHost, stream));
        KRS_HIP(hipStreamSynchronize(stream));
        const int s = h_st->status;
        if (s == ST_DONE || s == ST_BREAKDOWN || s == ST_MAXIT) break;
        if (h_st->iter == last_iter) {
            if (++stuck > 4) {
                set_error("solver made no progress");
                return KRS_E_DEVICE;
            }
        } else {
            stuck = 0;
        }
        last_iter = h_st->iter;
        block = graphs ? 64 : std::min(block * 2, 64);
    }
    return KRS_OK;
}

// Pinned staging for the first mc coefficients of each of the three runs
// (alpha, rho, gamma), then their asynchronous copies on the stream.
template <typename V, typename W>
void SeqImpl<V, W>::coef_readback(int mc) {
    if (h_coef_cap < 3 * (size_t)mc) {
        if (h_coef) (void)hipHostFree(h_coef);
        h_coef = nullptr;
        h_coef_cap = 0;
        const size_t want = 3 * (size_t)std::min(coef_cap, 2 * mc);
        if (hipHostMalloc((void**)&h_coef, want * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            h_coef = nullptr;
            throw std::bad_alloc();
        }
        h_coef_cap = want;
    }
    const double* base = (const double*)d_coef.p;
    for (int a = 0; a < 3; ++a)
        if (hipMemcpyAsync(h_coef + (size_t)a * mc, base + (size_t)a * coef_cap, mc * sizeof(double),
                           hipMemcpyDeviceToHost, stream) != hipSuccess)
            throw std::runtime_error("coefficient read-back failed");
}

template <typename V, typename W>
krs_status SeqImpl<V, W>::end_solve(double* x, bool device_x, krs_solve_info* info, int iter_hint) {
    const SysView<V, W> v = cur;
    k_resid(v, 1);
    KRS_CHECK_LAUNCH();
    // with the final iteration count known, the coefficients come back with
    // the state (one wait); otherwise after it
    const int mc_pre = iter_hint >= 0 ? std::min(iter_hint + 1, coef_cap) : -1;
    if (mc_pre > 0) coef_readback(mc_pre);
    KRS_HIP(hipEventRecord(ev[2], stream));
    KRS_HIP(hipMemcpyAsync(h_st, d_st.p, sizeof(DevState), hipMemcpyDeviceToHost, stream));
    if (x) {
        if (device_x) KRS_HIP(hipMemcpyAsync(x, d_x.p, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
        else KRS_HIP(hipMemcpyAsync(x, d_x.p, n * sizeof(double), hipMemcpyDeviceToHost, stream));
    }
    KRS_HIP(hipStreamSynchronize(stream));
    if (timing) {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || khz <= 0)
            khz = 100000;
        for (int j = 0; j < 3; ++j) {
            kt_count[j] += (int64_t)h_st->kcnt[j];
            kt_ms[j] += (double)h_st->ksum[j] / (double)khz;
        }
    }
    const int m = h_st->iter;
    m_last = m;
    const int mc = std::min(m + 1, coef_cap);
    coef_alpha.assign(mc, 0.0);
    coef_rho.assign(mc, 0.0);
    coef_gamma.assign(mc, 0.0);
    if (mc > 0) {
        // the three coefficient runs come through pinned staging (a batch
        // ends hundreds of solves: no blocking copy each)
        if (mc != mc_pre) {
            coef_readback(mc);
            KRS_HIP(hipStreamSynchronize(stream));
        }
        std::memcpy(coef_alpha.data(), h_coef, mc * sizeof(double));
        std::memcpy(coef_rho.data(), h_coef + mc, mc * sizeof(double));
        std::memcpy(coef_gamma.data(), h_coef + 2 * (size_t)mc, mc * sizeof(double));
    }
    krs_solve_info inf = info_last;
    inf.iters = m;
    inf.n_c = nc;
    inf.refinements = h_st->refinements;
    inf.dropped = dropped_last;
    inf.selected = 0;
    inf.added = 0;
    inf.update_rows = (int32_t)geo.cb3;
    const double bb = h_st->bb > 0 ? h_st->bb : 1.0;
    inf.rel_res_true = std::sqrt(h_st->rr_true / bb);
    inf.rel_res_recursive = std::sqrt(h_st->rr / bb);
    float t0 = 0.f, t1 = 0.f;
    (void)hipEventElapsedTime(&t0, ev[0], ev[1]);
    (void)hipEventElapsedTime(&t1, ev[1], ev[2]);
    inf.t_rebuild_ms = t0;
    inf.t_iter_ms = t1;
    inf.t_recycle_ms = 0.0;
    inf.model_bytes = model_bytes_per_iter(false) * m;
    inf.n_c_lim = has_cap() ? cap_value() : (desc.max_basis < 0 ? -1 : 0);
    cost_bytes_last = model_bytes_per_iter(true) * m;
    krs_status rs = KRS_OK;
    if (h_st->status == ST_MAXIT) rs = KRS_E_MAXIT;
    else if (h_st->status == ST_BREAKDOWN) rs = KRS_E_NOT_SPD;
    inf.status = rs;
    info_last = inf;
    if (info) *info = inf;
    if (rs == KRS_E_NOT_SPD) {
        set_error("breakdown: (w, A w) or (r, z) not positive (operator or preconditioner not SPD)");
        return rs;
    }
    solved = true;
    if (rs == KRS_E_MAXIT) set_error("maximum number of iterations reached");
    return rs;
}

template <typename V, typename W>
int64_t SeqImpl<V, W>::model_bytes_per_iter(bool padded) const {
    // Algorithmic bytes of one iteration: B_A + B_M + 10 n p_w + 2 n p_x
    // (+ n p_z for the history column z_j when one is kept, p_z its storage
    // size) + 2 n n_c p;
    // p: matrix / basis storage, p_w: Krylov vectors, p_x = 8.
    // `padded`: the cost cap's figure instead, which counts the padded rows
    // of A C that the update kernel streams and a z column for every
    // selective-reuse iteration.
    const int64_t p = sizeof(V), pw = sizeof(W);
    const int64_t pa = op64() ? 8 : p;  // matrix value bytes
    const int64_t nnz = nnzb * B * B;
    const int64_t BA = (B == 1) ? nnz * (pa + 4) : nnz * pa + 4 * nnzb;
    const int64_t BM = (B == 1) ? n * p : 3 * n * p;
    if (padded) {
        const int64_t vec = 11 * n * pw + 2 * n * 8 - (desc.reuse == KRS_REUSE_SELECTIVE ? 0 : n * pw);
        const int64_t basis = nc > 0 ? n * (ac_leading_dim(nc, sizeof(V)) + nc) * p : 0;
        return BA + BM + vec + basis;
    }
    const bool z_kept = desc.reuse == KRS_REUSE_SELECTIVE && history_kept > 0;
    const int64_t vec = 10 * n * pw + 2 * n * 8 + (z_kept ? n * hist_elem() : 0);
    return BA + BM + vec + 2 * n * (int64_t)nc * p;
}

// ------------------------------------------------------------- recycle

// recycle() = recycle_plan() + recycle_apply().  The plan is host work only
// (the cost-cap decision, the Ritz analysis and selection, the combination
// matrix F) and touches no device state, so several sequences' plans can
// run on other threads while the device works; the apply step enqueues the
// basis update on the stream.
template <typename V, typename W>
krs_status SeqImpl<V, W>::recycle(int32_t* n_added) {
    krs_status st = recycle_plan();
    if (st != KRS_OK) return st;
    return recycle_apply(n_added);
}

template <typename V, typename W>
krs_status SeqImpl<V, W>::recycle_plan() {
    plan = RecyclePlan{};
    if (!solved) {
        set_error("krs_seq_recycle needs a completed solve");
        return KRS_E_STATE;
    }
    solved = false;
    plan.ready = true;
    const auto t_start = std::chrono::steady_clock::now();
    const int m = m_last;
    last_theta.clear();
    last_sel.clear();
    // Cost cap: the modelled bytes of the last solve (iterations times bytes
    // per iteration, which grow with the basis) against those of the latest
    // solve made with the initial basis alone.  Recycled columns that did
    // not pay for themselves are dropped (back to C0) and nothing is
    // appended for the next kCostHold systems (doubling with each failed
    // trial in a row).
    bool append_ok = true;
    if (desc.cap_policy == KRS_CAP_COST) {
        const int64_t cost = cost_bytes_last;
        if (info_last.n_c <= nc0) {
            ref_cost = cost;
            if (cost_hold > 0) {
                --cost_hold;
                append_ok = false;
            }
        } else if (ref_cost > 0 && cost >= ref_cost) {
            plan.restore_c0 = nc0 > 0;
            nc = nc0;
            restarts += 1;
            // every failed trial doubles the wait before the next one
            cost_hold = kCostHold << std::min(cost_fails, 4);
            cost_fails += 1;
            append_ok = false;
        } else {
            cost_fails = 0;
        }
    }
    if (desc.max_basis < 0 && nc_lim_auto < 0 && m > 0) {
        // n_c_lim by the complexity analysis of Section 4.4 on this first
        // solve, with the byte model of the iteration (basis columns in V)
        NcCostModel cm;
        const int64_t p = sizeof(V), pw = sizeof(W);
        const int64_t pa = op64() ? 8 : p;
        const int64_t nnz = nnzb * B * B;
        const int64_t BA = (B == 1) ? nnz * (pa + 4) : nnz * pa + 4 * nnzb;
        const int64_t BM = (B == 1) ? n * p : 3 * n * p;
        cm.bytes_iter0 = (double)(BA + BM + 10 * n * pw + 2 * n * 8);
        cm.bytes_col_iter = 2.0 * n * p;
        cm.bytes_rebuild0 = (double)BA;
        cm.bytes_col_rebuild = 7.0 * n * p;
        cm.kmax = std::min(1024, m - 1);
        cm.eps = desc.ritz_eps;
        const int nt = recycle_threads > 0 ? recycle_threads : host_threads();
        nc_lim_auto = nc_limit(coef_alpha.data(), coef_rho.data(), m, cm, nt, nullptr);
    }
    const bool capped = has_cap() && (desc.cap_policy == KRS_CAP_FREEZE || desc.cap_policy == KRS_CAP_COST);
    if (!append_ok) {
        // nothing appended
    } else if (desc.reuse == KRS_REUSE_TOTAL && m > 0) {
        // w_j / sqrt((w_j, A w_j)) for the captured directions (Algorithm 2)
        const int cnt = std::min(m, trks_slots);
        if (cnt > 0) {
            std::vector<double>& sc = h_F;  // kept alive: the copy in the apply step is asynchronous
            sc.assign(cnt, 0.0);
            for (int j = 0; j < cnt; ++j) sc[j] = 1.0 / std::sqrt(coef_gamma[j]);
            plan.kind = 1;
            plan.add = cnt;
        }
    } else if (desc.reuse == KRS_REUSE_SELECTIVE && m > 1 && !(capped && nc >= cap_value()) &&
               !(has_cap() && cap_value() == 0)) {
        // (with a full frozen basis nothing could be appended: no extraction)
        const int hist = h_st->hist_cap;
        // leading part of the Lanczos run: within the kept history and
        // before the first direction restart (after it H_m is block diagonal)
        const int mu = std::min(std::min(m, hist), h_st->first_restart);
        if (mu > 1) {
            // H_mu and its leading block H_{mu-1} as qd arrays (Section 4.1)
            const QdArray zm = qd_from_cg(coef_alpha.data(), coef_rho.data(), mu);
            const QdArray zm1 = qd_leading(zm, mu - 1);
            const int nt = recycle_threads > 0 ? recycle_threads : host_threads();
            // the frozen scan stops at the room; a reselection needs the
            // whole preselection first
            const bool frozen = capped && desc.reselect == 0;
            std::vector<double> th_m(mu, 0.0);  // descending (Algorithm 3 order)
            std::vector<int> sel;               // descending indices, ascending order
            if (!frozen) {
                std::vector<double> th_m1;
                qd_eigenvalues_desc(zm, th_m, nt);
                qd_eigenvalues_desc(zm1, th_m1, nt);
                sel = stagnation_select(th_m, th_m1, desc.ritz_eps);
                if (desc.reselect == KRS_RESELECT_CLUSTER) sel = cluster_reselect(th_m, sel, desc.cluster_min_frac);
                last_theta = th_m;
                last_sel.assign(mu, 0);
                for (int i : sel) last_sel[i] = 1;
                last_selected = (int)sel.size();
                if (capped) {
                    // fill the room smallest theta first, ties to the lower index
                    const int room = std::max(0, cap_value() - nc);
                    std::vector<int> cand(sel);
                    std::stable_sort(cand.begin(), cand.end(), [&](int i, int j) {
                        if (th_m[i] != th_m[j]) return th_m[i] < th_m[j];
                        return i < j;
                    });
                    if ((int)cand.size() > room) cand.resize(room);
                    std::sort(cand.begin(), cand.end());
                    sel = cand;
                }
            } else {
                // Smallest Ritz values first (the order in which a frozen
                // basis is filled): a_k, b_k are the k-th smallest
                // eigenvalues of H_m, H_{m-1}; a_k passed the stagnation test
                // iff it is within eps of one of its interlacing neighbours
                // b_{k-1} <= a_k <= b_k.  Stop once the room is filled (and
                // any exact ties of the last value are seen).
                // The interlacing neighbours of a_k are the only eigenvalues
                // of H_{m-1} that can lie within eps |a_k| of it, so the test
                // is whether H_{m-1} has an eigenvalue in that window: two
                // inertia counts instead of bisecting H_{m-1}'s spectrum.
                const int room = std::max(0, cap_value() - nc);
                std::vector<double> a(mu);
                std::vector<int> sel_asc;
                bool have_cut = false, stop = false;
                double cut = 0.0;
                int k = 0, done = 0;
                const int CH = 128;
                while (k < mu && !stop) {
                    const int k1 = std::min(mu, k + CH);
                    qd_eigenvalues_asc(zm, k, k1, a.data(), nt);
                    for (int kk = k; kk < k1; ++kk) {
                        if (have_cut && a[kk] > cut) {
                            stop = true;
                            break;
                        }
                        const double e = desc.ritz_eps * std::fabs(a[kk]);
                        if (qd_has_eigenvalue_in(zm1, a[kk] - e, a[kk] + e)) {
                            sel_asc.push_back(kk);
                            if (!have_cut && (int)sel_asc.size() >= room) {
                                have_cut = true;
                                cut = a[kk];
                            }
                        }
                        done = kk + 1;
                    }
                    k = k1;
                }
                // same order as the full rule: theta ascending, then the
                // descending index ascending
                std::vector<int> cand;
                for (int kk : sel_asc) cand.push_back(mu - 1 - kk);
                std::stable_sort(cand.begin(), cand.end(), [&](int i, int j) {
                    const double ti = a[mu - 1 - i], tj = a[mu - 1 - j];
                    if (ti != tj) return ti < tj;
                    return i < j;
                });
                if ((int)cand.size() > room) cand.resize(room);
                std::sort(cand.begin(), cand.end());
                sel = cand;
                last_selected = (int)sel_asc.size();
                // report the computed part, descending
                last_theta.assign(done, 0.0);
                last_sel.assign(done, 0);
                for (int kk = 0; kk < done; ++kk) last_theta[done - 1 - kk] = a[kk];
                for (int kk : sel_asc) last_sel[done - 1 - kk] = 1;
                for (int kk = 0; kk < done; ++kk) th_m[mu - 1 - kk] = a[kk];
            }
            sel.resize(std::min<size_t>(sel.size(), (size_t)std::max(0, 1024 - nc)));
            const int s = (int)sel.size();
            if (s > 0) {
                // F[j, t] = (-1)^j q_t[j] / (sqrt(rho_j) sqrt|theta_t|); the
                // explicit tridiagonal R^T R: diagonal q_j + e_{j-1},
                // off-diagonal sqrt(q_j e_j)
                std::vector<double> diag(mu), off(mu - 1);
                for (int j = 0; j < mu; ++j) diag[j] = zm.q[j] + (j > 0 ? zm.e[j - 1] : 0.0);
                for (int j = 0; j + 1 < mu; ++j) off[j] = std::sqrt(zm.q[j] * zm.e[j]);
                std::vector<double>& F = h_F;  // kept alive: the copy in the apply step is asynchronous
                F.assign((size_t)mu * s, 0.0);
                std::vector<double> q;
                for (int t = 0; t < s; ++t) {
                    const double th = th_m[sel[t]];
                    tridiag_eigvec(diag, off, th, q);
                    const double sc = 1.0 / std::sqrt(std::fabs(th));
                    for (int j = 0; j < mu; ++j)
                        F[(size_t)t * mu + j] = ((j & 1) ? -1.0 : 1.0) * q[j] * sc / std::sqrt(coef_rho[j]);
                }
                plan.kind = 2;
                plan.add = s;
                plan.mu = mu;
            }
        }
    }
    info_last.added = plan.add;
    info_last.selected = last_selected;
    info_last.n_c_lim = has_cap() ? cap_value() : (desc.max_basis < 0 ? -1 : 0);
    plan.host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return KRS_OK;
}

// Device side of a recycle: restore C0 (cost cap), scale the captured
// directions (TRKS) or combine the history into the new columns (SRKS),
// then the restart cap.  Only enqueues; stream-ordered before the next solve.
template <typename V, typename W>
krs_status SeqImpl<V, W>::recycle_apply(int32_t* n_added) {
    if (n_added) *n_added = 0;
    if (!plan.ready) {
        set_error("krs_seq_recycle needs a completed solve");
        return KRS_E_STATE;
    }
    plan.ready = false;
    const auto t_start = std::chrono::steady_clock::now();
    if (plan.restore_c0)
        KRS_HIP(hipMemcpyAsync(d_C.p, d_C0.p, (size_t)ldc * nc0 * sizeof(V), hipMemcpyDeviceToDevice, stream));
    if (plan.kind == 1) {
        const int cnt = plan.add;
        if (!d_F.reserve(ctx, cnt * sizeof(double))) return KRS_E_OOM;
        KRS_HIP(hipMemcpyAsync(d_F.p, h_F.data(), cnt * sizeof(double), hipMemcpyHostToDevice, stream));
        launch_scale_columns<V>((V*)d_C.p + (size_t)nc * ldc, ldc, n, (const double*)d_F.p, cnt, stream);
        KRS_CHECK_LAUNCH();
        nc += cnt;
    } else if (plan.kind == 2) {
        const int s = plan.add;
        if (!ensure_c_capacity(nc + s)) return KRS_E_OOM;
        if (!d_F.reserve(ctx, h_F.size() * sizeof(double))) return KRS_E_OOM;
        KRS_HIP(hipMemcpyAsync(d_F.p, h_F.data(), h_F.size() * sizeof(double), hipMemcpyHostToDevice, stream));
        if (hist32())
            launch_basis_combine_h32((const float*)d_Z.p, ldc, plan.mu, (const double*)d_F.p, s,
                                     reinterpret_cast<double*>((V*)d_C.p + (size_t)nc * ldc), ldc, n, stream);
        else
            launch_basis_combine<V>((const V*)d_Z.p, ldc, plan.mu, (const double*)d_F.p, s, (V*)d_C.p + (size_t)nc * ldc,
                                ldc, n, stream);
        KRS_CHECK_LAUNCH();
        nc += s;
    }
    // restart cap (Algorithm 3, last step)
    if (has_cap() && desc.cap_policy == KRS_CAP_RESTART && nc >= cap_value() && cap_value() > 0) {
        if (nc0 > 0) {
            KRS_HIP(hipMemcpyAsync(d_C.p, d_C0.p, (size_t)ldc * nc0 * sizeof(V), hipMemcpyDeviceToDevice, stream));
        }
        nc = nc0;
        restarts += 1;
    }
    KRS_CHECK_LAUNCH();
    // host wall time of plan and apply: neither waits for the device
    info_last.t_recycle_ms =
        plan.host_ms + std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (n_added) *n_added = plan.add;
    return KRS_OK;
}

template <typename V, typename W>
krs_status SeqImpl<V, W>::basis(double* C, int64_t ld, int32_t cap, int32_t* n_c) {
    if (n_c) *n_c = nc;
    if (!C) return KRS_OK;
    if (ld < n || cap < nc) {
        set_error("output basis too small");
        return KRS_E_INVALID;
    }
    if (!d_tmp.reserve(ctx, (size_t)n * sizeof(double))) return KRS_E_OOM;
    return basis_staged(C, ld, (double*)d_tmp.p);
}

template <typename V, typename W>
krs_status SeqImpl<V, W>::history(double* Z, int64_t ld, int32_t cap, int32_t* m_out) {
    // the directions z_0 .. z_{mh-1} of the last solve that the history kept
    const int mh = (desc.reuse == KRS_REUSE_SELECTIVE && d_Z.p) ? std::min(m_last, history_kept) : 0;
    if (m_out) *m_out = mh;
    if (!Z) return KRS_OK;
    if (ld < n || cap < mh) {
        set_error("output history too small");
        return KRS_E_INVALID;
    }
    if (!d_tmp.reserve(ctx, (size_t)n * sizeof(double))) return KRS_E_OOM;
    for (int c = 0; c < mh; ++c) {
        if (hist32()) launch_v2d<float>((const float*)d_Z.p + (size_t)c * ldc, (double*)d_tmp.p, n, stream);
        else launch_v2d<V>((const V*)d_Z.p + (size_t)c * ldc, (double*)d_tmp.p, n, stream);
        KRS_CHECK_LAUNCH();
        KRS_HIP(hipMemcpyAsync(Z + (size_t)c * ld, d_tmp.p, n * sizeof(double), hipMemcpyDeviceToHost, stream));
    }
    KRS_HIP(hipStreamSynchronize(stream));
    return KRS_OK;
}

// Each column converted to double in `staging` (n doubles of device memory)
// and copied out; the copies are stream-ordered behind the conversions, so
// one staging vector serves every column.
template <typename V, typename W>
krs_status SeqImpl<V, W>::basis_staged(double* C, int64_t ld, double* staging) {
    for (int c = 0; c < nc; ++c) {
        launch_v2d<V>((const V*)d_C.p + (size_t)c * ldc, staging, n, stream);
        KRS_CHECK_LAUNCH();
        KRS_HIP(hipMemcpyAsync(C + (size_t)c * ld, staging, n * sizeof(double), hipMemcpyDeviceToHost, stream));
    }
    KRS_HIP(hipStreamSynchronize(stream));
    return KRS_OK;
}

template struct SeqImpl<double, double>;
template struct SeqImpl<float, double>;
template struct SeqImpl<float, float>;

// ---------------------------------------------------------------- batch

namespace {

// Fused launches over a changing set of begun solves of one (V, W, B) type.
template <typename V, typename W>
struct BatchRunner : RunnerBase {
    krs_ctx* ctx;
    hipStream_t stream;
    int B;
    std::vector<SeqImpl<V, W>*> mem;
    Buf d_views, d_maps, d_stat;
    int32_t* h_stat = nullptr;
    size_t h_stat_cap = 0;
    BatchMaps maps{};
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int gblock[2] = {0, 0};

    BatchRunner(krs_ctx* c, int b) : ctx(c), stream(c->stream), B(b) {}
    ~BatchRunner() override {
        drop_graphs();
        d_views.release(ctx);
        d_maps.release(ctx);
        d_stat.release(ctx);
        if (h_stat) (void)hipHostFree(h_stat);
    }
    void drop_graphs() {
        for (int i = 0; i < 2; ++i) {
            if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
            exec[i] = nullptr;
            graph[i] = nullptr;
            gblock[i] = 0;
        }
    }
    size_t size() const override { return mem.size(); }
    const SysView<V, W>* views() const { return (const SysView<V, W>*)d_views.p; }

    // device copies of the members' views and the launch maps
    krs_status set_members(const std::vector<SeqBase*>& members) override {
        mem.clear();
        for (SeqBase* b : members) mem.push_back(static_cast<SeqImpl<V, W>*>(b));
        drop_graphs();
        const int cnt = (int)mem.size();
        if (cnt == 0) return KRS_OK;
        std::vector<SysView<V, W>> hv(cnt);
        std::vector<int2> lists[BK_COUNT];
        for (int i = 0; i < cnt; ++i) {
            const SysView<V, W>& v = mem[i]->cur;
            hv[i] = v;
            const bool basis = v.nc > 0;
            for (int b = 0; b < v.geo.g1; ++b) lists[BK_SPMV].push_back(make_int2(i, b));
            for (int b = 0; b < v.geo.g3; ++b) lists[BK_UPD].push_back(make_int2(i, b));
            lists[BK_ONE].push_back(make_int2(i, 0));
            if (v.nc > kDirFewCols) {
                for (int b = 0; b < v.geo.g5; ++b) lists[BK_DIR].push_back(make_int2(i, b));
            } else {
                const int k = v.nc == 0 ? BK_DIR0 : BK_DIRF;
                for (int b = 0; b < v.geo.g5; b += kDirFewGroup) lists[k].push_back(make_int2(i, b));
            }
            if (basis) {
                for (int b = 0; b < v.geo.gd; ++b) lists[BK_DOT].push_back(make_int2(i, b));
                lists[BK_ONEC].push_back(make_int2(i, 0));
                for (int b = 0; b < v.geo.gcc; ++b) lists[BK_CC].push_back(make_int2(i, b));
            }
        }
        size_t total = 0;
        for (auto& l : lists) total += l.size();
        if (!d_views.reserve(ctx, cnt * sizeof(SysView<V, W>)) || !d_maps.reserve(ctx, total * sizeof(int2)) ||
            !d_stat.reserve(ctx, 2 * (size_t)cnt * sizeof(int32_t))) {
            set_error("device allocation failed for the batch tables");
            return KRS_E_OOM;
        }
        if (h_stat_cap < 2 * (size_t)cnt) {
            if (h_stat) (void)hipHostFree(h_stat);
            h_stat = nullptr;
            h_stat_cap = 2 * (size_t)cnt;
            KRS_HIP(hipHostMalloc((void**)&h_stat, h_stat_cap * sizeof(int32_t), hipHostMallocDefault));
        }
        KRS_HIP(hipMemcpyAsync(d_views.p, hv.data(), cnt * sizeof(SysView<V, W>), hipMemcpyHostToDevice, stream));
        size_t off = 0;
        for (int k = 0; k < BK_COUNT; ++k) {
            maps.map[k] = (const int2*)d_maps.p + off;
            maps.count[k] = (int64_t)lists[k].size();
            if (!lists[k].empty())
                KRS_HIP(hipMemcpyAsync((int2*)d_maps.p + off, lists[k].data(), lists[k].size() * sizeof(int2),
                                       hipMemcpyHostToDevice, stream));
            off += lists[k].size();
        }
        maps.fused = mem[0]->cur.fused;
        KRS_HIP(hipStreamSynchronize(stream));
        return KRS_OK;
    }

    void spmv() {
        if (B == 1) batch_spmv_dot<V, W, 1>(views(), maps, stream);
        else batch_spmv_dot<V, W, 3>(views(), maps, stream);
    }
    krs_status time_update(int reps, float* ms) override {
        *ms = 0.f;
        if (mem.empty()) return KRS_OK;
        BatchMaps m = maps;
        m.fused = 0;  // the update kernel alone, no end-of-step reduction
        hipEvent_t e0 = nullptr, e1 = nullptr;
        KRS_HIP(hipEventCreate(&e0));
        KRS_HIP(hipEventCreate(&e1));
        krs_status st = KRS_OK;
        auto launch = [&] {
            if (m.count[BK_UPD] <= 0) return;
            if (B == 1) batch_update_only<V, W, 1>(views(), m, 1, stream);
            else batch_update_only<V, W, 3>(views(), m, 1, stream);
        };
        launch();
        if (hipEventRecord(e0, stream) != hipSuccess) st = KRS_E_DEVICE;
        for (int r = 0; r < reps && st == KRS_OK; ++r) launch();
        if (st == KRS_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(ms, e0, e1) != hipSuccess))
            st = KRS_E_DEVICE;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != KRS_OK) set_error("timing the fused update failed");
        *ms /= std::max(reps, 1);
        return st;
    }
    void update(int mode) {
        if (B == 1) batch_update_reduce<V, W, 1>(views(), maps, mode, stream);
        else batch_update_reduce<V, W, 3>(views(), maps, mode, stream);
    }
    void resid() {
        if (B == 1) batch_true_resid<V, W, 1>(views(), maps, 0, stream);
        else batch_true_resid<V, W, 3>(views(), maps, 0, stream);
    }
    // the same kernel sequence as a single system's iteration block
    void enqueue(int block) {
        for (int i = 0; i < block; ++i) {
            spmv();
            update(0);
            batch_correct_dir<V, W>(views(), maps, 0, stream);
        }
        resid();
        batch_coarse_dot<V, W>(views(), maps, 0, 0, M_REFINE, stream);
        batch_coarse_correct<V, W>(views(), maps, 0, M_REFINE, stream);
        update(2);
        batch_correct_dir<V, W>(views(), maps, 2, stream);
        batch_status<V, W>(views(), (int)mem.size(), (int32_t*)d_stat.p, stream);
    }

    krs_status launch(int block, bool graphs) override {
        if (mem.empty()) return KRS_OK;
        if (!graphs) {
            enqueue(block);
            KRS_CHECK_LAUNCH();
        } else {
            int slot = (gblock[0] == block || gblock[0] == 0) ? 0 : 1;
            if (gblock[slot] != block) {
                if (exec[slot]) (void)hipGraphExecDestroy(exec[slot]);
                if (graph[slot]) (void)hipGraphDestroy(graph[slot]);
                exec[slot] = nullptr;
                graph[slot] = nullptr;
            }
            if (!exec[slot]) {
                KRS_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
                enqueue(block);
                hipError_t e = hipStreamEndCapture(stream, &graph[slot]);
                if (e != hipSuccess) {
                    set_error(std::string("batch graph capture failed: ") + hipGetErrorString(e));
                    return KRS_E_DEVICE;
                }
                KRS_HIP(hipGraphInstantiate(&exec[slot], graph[slot], nullptr, nullptr, 0));
                gblock[slot] = block;
            }
            KRS_HIP(hipGraphLaunch(exec[slot], stream));
        }
        KRS_HIP(hipMemcpyAsync(h_stat, d_stat.p, 2 * mem.size() * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        return KRS_OK;
    }

    krs_status read_status(std::vector<int32_t>& out) override {
        KRS_HIP(hipStreamSynchronize(stream));
        out.assign(h_stat, h_stat + 2 * mem.size());
        return KRS_OK;
    }
};

}  // namespace

std::unique_ptr<RunnerBase> make_runner(krs_ctx* ctx, int key) {
    const int B = (key & 4) ? 3 : 1;  // bit 3 (separate finalize) only splits the groups
    switch (key & 3) {
        case 0: return std::unique_ptr<RunnerBase>(new BatchRunner<double, double>(ctx, B));
        case 1: return std::unique_ptr<RunnerBase>(new BatchRunner<float, double>(ctx, B));
        case 3: return std::unique_ptr<RunnerBase>(new BatchRunner<float, float>(ctx, B));
        default: return nullptr;
    }
}

bool finished_status(int s) { return s == ST_DONE || s == ST_BREAKDOWN || s == ST_MAXIT; }

krs_status batch_solve(krs_ctx* ctx, SeqBase* const* seqs, int count, double* const* x, bool device_x,
                       krs_solve_info* info, int32_t* added) {
    std::vector<krs_status> out(count, KRS_OK);
    // with `added`: every member is recycled too; a member that has finished
    // is completed (solution out) at once and its recycle planned on a helper
    // thread while the others iterate; the device steps follow in order
    const bool rec = added != nullptr;
    std::vector<char> ended(count, 0);
    std::vector<krs_status> pst(count, KRS_OK);
    std::vector<std::thread> helpers;
    struct Joiner {  // helpers are joined on every way out
        std::vector<std::thread>& t;
        ~Joiner() {
            for (auto& th : t)
                if (th.joinable()) th.join();
        }
    } joiner{helpers};
    std::vector<int> iter_of(count, -1);  // final iteration counts read from the status words
    auto end_member = [&](int i) {
        if (ended[i]) return;
        ended[i] = 1;
        out[i] = seqs[i]->end_solve(x ? x[i] : nullptr, device_x, info ? &info[i] : nullptr, iter_of[i]);
    };
    auto plan_members = [&](std::vector<int> idx) {
        std::vector<int> ok;
        for (int i : idx)
            if (out[i] == KRS_OK || out[i] == KRS_E_MAXIT) ok.push_back(i);
        if (ok.empty()) return;
        // everything the helper uses is allocated here: nothing on it can throw
        std::vector<SeqBase*> m;
        for (int i : ok) m.push_back(seqs[i]);
        std::vector<krs_status> st(ok.size(), KRS_OK);
        auto fn = [&pst, ok = std::move(ok), m = std::move(m), st = std::move(st)]() mutable {
            plan_all(m.data(), (int)m.size(), st.data());
            for (size_t j = 0; j < ok.size(); ++j) pst[ok[j]] = st[j];
        };
        try {
            helpers.emplace_back(fn);
        } catch (...) {
            fn();  // no helper thread: plan here
        }
    };
    // the members' coarse rebuilds in stages, one wait per stage for all
    {
        std::vector<char> more(count, 0);
        bool any = false;
        for (int i = 0; i < count; ++i) {
            bool m = false;
            out[i] = seqs[i]->rebuild_stage(0, &m);
            more[i] = m;
            any = any || m;
        }
        for (int stage = 1; stage <= 2 && any; ++stage) {
            if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
                set_error("device failure during the batched coarse rebuild");
                return KRS_E_DEVICE;
            }
            any = false;
            for (int i = 0; i < count; ++i) {
                if (!more[i] || out[i] != KRS_OK) continue;
                bool m = false;
                out[i] = seqs[i]->rebuild_stage(stage, &m);
                more[i] = m;
                any = any || m;
            }
        }
    }
    // begin every member; group the begun ones by type
    std::map<int, std::vector<int>> groups;
    for (int i = 0; i < count; ++i) {
        if (out[i] != KRS_OK) {
            ended[i] = 1;
            continue;
        }
        out[i] = seqs[i]->begin_solve();
        if (out[i] == KRS_OK) groups[seqs[i]->type_key()].push_back(i);
        else ended[i] = 1;
    }
    krs_status fatal = KRS_OK;
    for (auto& kv : groups) {
        std::unique_ptr<RunnerBase> r = make_runner(ctx, kv.first);
        std::vector<int> act = kv.second;
        bool graphs = true;
        for (int i : act) graphs = graphs && seqs[i]->desc.exec_mode == 0;
        auto members = [&](const std::vector<int>& idx) {
            std::vector<SeqBase*> m;
            for (int i : idx) m.push_back(seqs[i]);
            return m;
        };
        krs_status st = r->set_members(members(act));
        // Batch autotuner: members that ask for it and have not been tuned
        // in a batch (or whose basis width changed by half since) get the update tile (block rows per workgroup) whose
        // fused launch over the whole group is fastest; the tile then stays
        // with each sequence (it fixes the grouping of its partial sums).
        bool tune = false;
        for (int i : act) tune = tune || (seqs[i]->desc.autotune && seqs[i]->batch_tune_due());
        if (st == KRS_OK && tune) {
            const int64_t cand[] = {512, 1024, 2048, 4096, 8192, 16384};
            float best = 0.f;
            int64_t pick = 0;
            for (int64_t c : cand) {
                for (int i : act)
                    if (st == KRS_OK) st = seqs[i]->set_update_rows(c);
                if (st == KRS_OK) st = r->set_members(members(act));
                float ms = 0.f;
                if (st == KRS_OK) st = r->time_update(3, &ms);
                if (st != KRS_OK) break;
                if (pick == 0 || ms < best) {
                    best = ms;
                    pick = c;
                }
            }
            for (int i : act)
                if (st == KRS_OK) st = seqs[i]->set_update_rows(pick);
            if (st == KRS_OK) st = r->set_members(members(act));
        }
        // Short blocks: a member whose residual replacement is due waits
        // (gated) until the end of the block, and the gated workgroups of a
        // large batch still cost their dispatch.  The block length changes
        // when the gated steps run, not what any member computes.  Blocks of
        // 8 iterations measured fastest (256 diffusion sequences: 331 ms per
        // step against 378 ms with blocks of 64; 4 iterations: 333 ms).
        constexpr int kBatchBlock = 8;
        const int block = kBatchBlock;
        std::vector<int32_t> last(act.size(), -1), stat;
        int stuck = 0;
        while (st == KRS_OK && !act.empty()) {
            st = r->launch(block, graphs);
            if (st != KRS_OK) break;
            st = r->read_status(stat);
            if (st != KRS_OK) break;
            std::vector<int> keep, done_now;
            std::vector<int32_t> keep_last;
            bool progress = false;
            for (size_t i = 0; i < act.size(); ++i) {
                if (stat[2 * i + 1] != last[i]) progress = true;
                if (finished_status(stat[2 * i])) {
                    iter_of[act[i]] = stat[2 * i + 1];
                    if (rec && !ended[act[i]]) done_now.push_back(act[i]);
                    continue;
                }
                keep.push_back(act[i]);
                keep_last.push_back(stat[2 * i + 1]);
            }
            if (!progress && ++stuck > 4) {
                set_error("batch made no progress");
                st = KRS_E_DEVICE;
                break;
            }
            if (progress) stuck = 0;
            if (!keep.empty() && !done_now.empty()) {
                // finished while others still iterate: complete and plan now
                // (its launches are gated from here on)
                for (int i : done_now) end_member(i);
                plan_members(done_now);
            }
            if (keep.empty()) break;
            if (4 * keep.size() <= 3 * act.size()) {
                // finished members leave the launches once a quarter is done
                act = keep;
                last = keep_last;
                st = r->set_members(members(act));
            } else {
                for (size_t i = 0; i < act.size(); ++i) last[i] = stat[2 * i + 1];
            }
        }
        if (st != KRS_OK) {
            for (int i : kv.second) {
                out[i] = st;
                ended[i] = 1;
            }
            if (st == KRS_E_DEVICE) {
                fatal = st;
                break;
            }
            continue;
        }
        std::vector<int> rest;
        for (int i : kv.second)
            if (!ended[i]) {
                end_member(i);
                rest.push_back(i);
            }
        if (rec) plan_members(rest);
    }
    for (auto& th : helpers) th.join();
    helpers.clear();
    if (fatal != KRS_OK) return fatal;
    if (rec) {
        for (int i = 0; i < count; ++i) {
            int32_t a = 0;
            if ((out[i] == KRS_OK || out[i] == KRS_E_MAXIT) && ended[i]) {
                krs_status r2 = pst[i];
                if (r2 == KRS_OK) r2 = seqs[i]->recycle_apply(&a);
                else set_error(seqs[i]->plan_msg);
                if (r2 != KRS_OK) out[i] = r2;
                else if (info) info[i].added = a;
            }
            added[i] = a;
        }
    }
    krs_status worst = KRS_OK;
    for (krs_status st : out)
        if (st != KRS_OK && (worst == KRS_OK || worst == KRS_E_MAXIT)) worst = st;
    return worst;
}

void plan_all(SeqBase* const* seqs, int count, krs_status* st) {
    // Independent sequences: their host-side Ritz work runs on up to
    // host_threads() threads (this one included), one sequence per thread,
    // the threads left over shared out as bisection threads of each (all of
    // them when there is a single sequence).  Host work only: no device
    // calls.  Nothing escapes a thread: a plan that throws fails with a
    // status, and threads that cannot be started leave their sequences to
    // the ones that run.
    const int nt = std::max(1, std::min(count, host_threads()));
    const int per = std::max(1, host_threads() / nt);
    std::atomic<int> next{0};
    auto work = [&]() noexcept {
        for (int i = next.fetch_add(1); i < count; i = next.fetch_add(1)) {
            SeqBase* s = seqs[i];
            s->recycle_threads = per;
            krs_status r = KRS_OK;
            const char* msg = nullptr;
            try {
                r = s->recycle_plan();
                if (r != KRS_OK) msg = krs_last_error();
            } catch (const std::bad_alloc&) {
                r = KRS_E_OOM;
                msg = "host allocation failed in the Ritz analysis";
            } catch (...) {
                r = KRS_E_INVALID;
                msg = "internal error in the Ritz analysis";
            }
            if (msg) std::snprintf(s->plan_msg, sizeof s->plan_msg, "%s", msg);
            s->recycle_threads = 0;
            st[i] = r;
        }
    };
    std::vector<std::thread> pool;
    try {
        pool.reserve(nt - 1);
        for (int t = 1; t < nt; ++t) pool.emplace_back(work);
    } catch (...) {
        // fewer threads: the started ones and this one take every sequence
    }
    work();
    for (auto& th : pool) th.join();
}

krs_status recycle_all(krs_ctx* ctx, SeqBase* const* seqs, int count, int32_t* added) {
    (void)ctx;
    std::vector<krs_status> st(count, KRS_OK);
    plan_all(seqs, count, st.data());
    // the device work of the plans, in order, on the shared stream
    krs_status first = KRS_OK;
    for (int i = 0; i < count; ++i) {
        int32_t a = 0;
        if (st[i] == KRS_OK) st[i] = seqs[i]->recycle_apply(&a);
        else if (first == KRS_OK) set_error(seqs[i]->plan_msg);
        if (added) added[i] = a;
        if (st[i] != KRS_OK && first == KRS_OK) first = st[i];
    }
    return first;
}

}  // namespace krs
