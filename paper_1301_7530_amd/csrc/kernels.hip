// Device kernels of libkrs for gfx950 (CDNA4, wave64).
//
// One APCG iteration (Algorithm 1, standard Hestenes-Stiefel form) is four
// launches; cross-workgroup sums go through per-workgroup partials reduced
// in a fixed order (no floating-point atomics, so results are bitwise
// reproducible):
//   K1 spmv_dot         q = A w; partials of (w, q)
//   K3 update_reduce    alpha = rho / (w, q), x += alpha w, r -= alpha q,
//                       s = M^-1 r; partials of ||r||^2, (r, s), (AC)^T s,
//                       (AC)^T w
//   F3 finalize_update  one workgroup: gamma, alpha, mu = G^-1 (AC)^T s,
//                       rho = (r, z), beta, convergence / refinement status
//   K5 correct_dir      z = s - C mu, w = s - C mu2 + beta w
//
// Matrices are stored in sliced ELL: 64 (block) rows per slice, one lane
// per block row, slot k of every row of a slice stored contiguously so a
// wavefront reads 64 consecutive values per load.  3x3 blocks are stored as
// 9 planes of 64 values per slot: value (d, e) of the block in slot k of
// lane l sits at ((slot*9) + 3d + e)*64 + l.  In the SpMV a lane owns a
// whole block row (all nine planes stream in lane order; the block column
// and the three entries of x are loaded once per block); the A C product
// takes sub-row d in wave d of a 192-thread workgroup.
//
// Every iteration kernel is a device function of (system view, workgroup
// index); the single-system kernels call it with blockIdx.x, the fused
// multi-system kernels with the (system, workgroup) pair of a launch map.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cstdint>

#include "internal.h"

namespace krs {

namespace {

constexpr int kTpb = 256;  // threads per workgroup, scalar kernels
constexpr int kTF3 = 512;  // threads of the single-workgroup finalize of the update
static_assert(kTF3 == kT3, "the fused update runs the finalize in one of its workgroups");
// s_waitcnt operand: vector memory counter 0, the other counters unconstrained
constexpr int kWaitVm0 = 0x0F70;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup (fixed order); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) t += lds[i];
    }
    return t;
}

// Two sums over the workgroup at once (each in the order of block_sum);
// results valid in thread 0.  lds: 2 * (blockDim.x / 64) doubles.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* lds) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) {
        lds[wave] = a;
        lds[nw + wave] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < nw; ++i) ta += lds[i];
        for (int i = 0; i < nw; ++i) tb += lds[nw + i];
    }
    a = ta;
    b = tb;
}

// Reduce `nv` values over `np` partial rows (row stride `stride`) in a fixed
// order with all threads of the workgroup; out[k] for k < nv (LDS).
// Load of a value written by another workgroup of the same launch (agent-
// coherent: bypasses a possibly stale L2 of another XCD) or a plain load.
template <bool COH>
__device__ __forceinline__ double ld_part(const double* p) {
    if (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
}

// sum_r P[r * stride + k] over r = 0 .. rows-1 in ascending order (16
// loads in flight, also for a ragged last group: rows past the end load the
// last row and are not added).  The update's partial sums are reduced in two
// levels with it: each group of kGroup consecutive workgroups, then the
// groups.
template <bool COH>
__device__ __forceinline__ double col_sum(const double* P, int64_t rows, int64_t stride, int k) {
    double s = 0.0;
    for (int64_t r = 0; r < rows; r += 16) {
        double t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) t[u] = ld_part<COH>(P + min(r + u, rows - 1) * stride + k);
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (r + u < rows) s += t[u];
    }
    return s;
}

template <int UNR = 32, bool COH = false>
__device__ void reduce_partials(const double* partials, int64_t np, int nv, int stride, double* out, double* lds) {
    const int T = blockDim.x;
    int tpv = T / (nv > 0 ? nv : 1);
    if (tpv < 1) tpv = 1;
    if (tpv > 64) tpv = 64;
    // thread -> (value k, part p); values beyond T handled in rounds
    for (int base = 0; base < nv; base += T / tpv) {
        const int k = base + threadIdx.x / tpv;
        const int p = threadIdx.x % tpv;
        double acc = 0.0;
        if (k < nv && threadIdx.x / tpv < T / tpv) {
            // UNR independent loads in flight per thread
            int64_t i = p;
            for (; i + UNR * tpv <= np; i += UNR * tpv) {
                double t[UNR];
#pragma unroll
                for (int u = 0; u < UNR; ++u) t[u] = ld_part<COH>(partials + (i + u * tpv) * stride + k);
#pragma unroll
                for (int u = 0; u < UNR; ++u) acc += t[u];
            }
            for (; i < np; i += tpv) acc += ld_part<COH>(partials + i * stride + k);
        }
        __syncthreads();
        lds[threadIdx.x] = acc;
        __syncthreads();
        if (p == 0 && k < nv && threadIdx.x / tpv < T / tpv) {
            double t = 0.0;
            for (int j = 0; j < tpv; ++j) t += lds[threadIdx.x + j];
            out[k] = t;
        }
        __syncthreads();
    }
}

// Fixed-order per-thread sum of p[tid], p[tid + T], ... (T = blockDim.x)
// with the first UNR loads issued together (a loop would wait for each).
template <int UNR>
__device__ __forceinline__ double thread_sum(const double* p, int64_t np) {
    const int64_t T = blockDim.x;
    double t[UNR];
    // every load is issued (clamped into the array), then masked
    const int64_t last = np > 0 ? np - 1 : 0;
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
        const int64_t i = threadIdx.x + u * T;
        t[u] = np > 0 ? p[i < np ? i : last] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
        if (threadIdx.x + u * T >= np) t[u] = 0.0;
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < UNR; ++u) a += t[u];
    for (int64_t i = threadIdx.x + UNR * T; i < np; i += T) a += p[i];
    return a;
}

// Fixed-order sum of p[0..np), returned to every thread of the workgroup.
__device__ double sum_all(const double* p, int64_t np, double* lds) {
    double a = thread_sum<4>(p, np);
    a = wave_sum(a);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = a;
    __syncthreads();
    double t = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t += lds[i];
    __syncthreads();
    return t;
}

// mu = Ginv t for column-major Ginv (nc x nc) and t in LDS, with the whole
// workgroup: thread (row r, part p) sums columns p, p+P, ...; parts are
// combined in a fixed order.  lds needs blockDim.x doubles.
__device__ void ginv_matvec(const double* __restrict__ Ginv, int nc, const double* t, double* mu, double* lds) {
    const int T = blockDim.x;
    int P = T / nc;
    if (P < 1) P = 1;
    if (P > 64) P = 64;
    const int rows_per_round = T / P;
    for (int base = 0; base < nc; base += rows_per_round) {
        const int r = base + threadIdx.x / P;
        const int p = threadIdx.x % P;
        const bool act = (int)(threadIdx.x / P) < rows_per_round && r < nc;
        double m = 0.0;
        if (act) {
            // same order as a plain loop over c = p, p + P, ...; 8 loads in flight
            int c = p;
            for (; c + 7 * P < nc; c += 8 * P) {
                double g[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) g[u] = Ginv[(int64_t)(c + u * P) * nc + r];
#pragma unroll
                for (int u = 0; u < 8; ++u) m += g[u] * t[c + u * P];
            }
            for (; c < nc; c += P) m += Ginv[(int64_t)c * nc + r] * t[c];
        }
        __syncthreads();
        lds[threadIdx.x] = m;
        __syncthreads();
        if (act && p == 0) {
            double s = 0.0;
            for (int j = 0; j < P; ++j) s += lds[threadIdx.x + j];
            mu[r] = s;
        }
        __syncthreads();
    }
}

// mu = Ginv t and gv = Ginv tv with one pass over Ginv (each output in the
// order of ginv_matvec, so the results are those of two calls); lds needs
// blockDim.x doubles.
__device__ void ginv_matvec2(const double* __restrict__ Ginv, int nc, const double* t, const double* tv, double* mu,
                             double* gv, double* lds) {
    const int T = blockDim.x;
    int P = T / nc;
    if (P < 1) P = 1;
    if (P > 64) P = 64;
    const int rows_per_round = T / P;
    for (int base = 0; base < nc; base += rows_per_round) {
        const int r = base + threadIdx.x / P;
        const int p = threadIdx.x % P;
        const bool act = (int)(threadIdx.x / P) < rows_per_round && r < nc;
        double m = 0.0, mv = 0.0;
        if (act) {
            int c = p;
            for (; c + 7 * P < nc; c += 8 * P) {
                double g[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) g[u] = Ginv[(int64_t)(c + u * P) * nc + r];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    m += g[u] * t[c + u * P];
                    mv += g[u] * tv[c + u * P];
                }
            }
            for (; c < nc; c += P) {
                const double g = Ginv[(int64_t)c * nc + r];
                m += g * t[c];
                mv += g * tv[c];
            }
        }
        // the parts are combined through the one LDS buffer, mu then gv
        __syncthreads();
        lds[threadIdx.x] = m;
        __syncthreads();
        if (act && p == 0) {
            double s = 0.0;
            for (int j = 0; j < P; ++j) s += lds[threadIdx.x + j];
            mu[r] = s;
        }
        __syncthreads();
        lds[threadIdx.x] = mv;
        __syncthreads();
        if (act && p == 0) {
            double s = 0.0;
            for (int j = 0; j < P; ++j) s += lds[threadIdx.x + j];
            gv[r] = s;
        }
        __syncthreads();
    }
}

// Live kernel timing: iteration j is sampled when j % 32 == 1 (K1, K3) and
// its direction update (K5, which already sees j + 1) likewise.  Every
// workgroup of a sampled launch stores its start and end wall-clock stamps
// in its own slot (plain stores, no contention); the finalize kernel adds
// max(end) - min(start) to the running sums.
constexpr int kSlotStride = 2 * kMaxTimedGrid;
__device__ __forceinline__ bool ktime_sample(const DevState* st, int which) {
    return st->ktime_on && (st->iter & 31) == (which == 2 ? 2 : 1);
}
__device__ __forceinline__ void ktime_begin(unsigned long long* slots, int which, int64_t bid, bool on) {
    if (on && threadIdx.x == 0) slots[which * kSlotStride + 2 * bid] = (unsigned long long)wall_clock64();
}
__device__ __forceinline__ void ktime_end(unsigned long long* slots, int which, int64_t bid, bool on) {
    if (on) {
        __syncthreads();
        if (threadIdx.x == 0) slots[which * kSlotStride + 2 * bid + 1] = (unsigned long long)wall_clock64();
    }
}
// All threads: span of kernel `which` over np workgroup slots, added to
// the sums of st by thread 0.  lds: 2 * blockDim.x entries.
__device__ void ktime_collect(DevState* st, const unsigned long long* slots, int which, int64_t np,
                              unsigned long long* lds) {
    unsigned long long lo = ~0ull, hi = 0ull;
    for (int64_t i = threadIdx.x; i < np; i += blockDim.x) {
        const unsigned long long s0 = slots[which * kSlotStride + 2 * i], s1 = slots[which * kSlotStride + 2 * i + 1];
        lo = s0 < lo ? s0 : lo;
        hi = s1 > hi ? s1 : hi;
    }
    lds[threadIdx.x] = lo;
    lds[blockDim.x + threadIdx.x] = hi;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < (int)blockDim.x; ++t) {
            lo = lds[t] < lo ? lds[t] : lo;
            hi = lds[blockDim.x + t] > hi ? lds[blockDim.x + t] : hi;
        }
        if (hi > lo) {
            st->ksum[which] += hi - lo;
            st->kcnt[which] += 1;
        }
    }
    __syncthreads();
}

// Fixed-order sum of one value per thread, returned to every thread.
__device__ double sum_all_reg(double a, double* lds) {
    a = wave_sum(a);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = a;
    __syncthreads();
    double t = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t += lds[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ bool gate(const DevState* st, uint32_t mask) {
    return ((1u << st->status) & mask) != 0;
}

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v < 1.0e308; }

// One ELL row (lane) of a slice: sum_k val[k] * x[col[k]] over slots
// [k0, k1).  Slots are processed UNR at a time so that every load of the
// group is in flight before the first product needs it.
template <typename V, typename X>
__device__ __forceinline__ X ell_row1(const V* __restrict__ val, const int32_t* __restrict__ col,
                                      const X* __restrict__ x, int64_t k0, int64_t k1, int lane) {
    constexpr int UNR = 8;
    X acc = 0;
    int64_t k = k0;
    for (; k + UNR <= k1; k += UNR) {
        int32_t cc[UNR];
        V a[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t e = (k + u) * 64 + lane;
            cc[u] = col[e];
            a[u] = val[e];
        }
        X xs[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) xs[u] = x[cc[u]];
#pragma unroll
        for (int u = 0; u < UNR; ++u) acc += (X)a[u] * xs[u];
    }
    // the last (fewer than UNR) slots as one group: every load issued at a
    // clamped, valid slot before any is used, the sum in the same order
    const int64_t r = k1 - k;
    if (r > 0) {
        int32_t cc[UNR];
        V a[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t e = (k + (u < r ? u : r - 1)) * 64 + lane;
            cc[u] = col[e];
            a[u] = val[e];
        }
        X xs[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) xs[u] = x[cc[u]];
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (u < r) acc += (X)a[u] * xs[u];
    }
    return acc;
}

// A whole 3x3-block ELL row (one lane): the three sub-rows at once, so the
// block column index and the three entries of x are loaded once per block
// and all nine value planes stream in lane order.  UNR blocks in flight.
// UNR: blocks whose loads are issued together; NT: the matrix streams
// with non-temporal loads (read once per launch), leaving the caches to the
// gathered x.  Neither changes the order of the sums.
template <typename T, bool NT>
__device__ __forceinline__ T ld_stream(const T* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

// A store of an iteration vector: non-temporal with NT (written out at once
// instead of left dirty in the caches for the next kernel to write back).
// The value stored is the same either way.  NT is a compile-time choice: the
// two forms of one store behind a run-time test are merged into a plain one.
template <bool NT, typename T>
__device__ __forceinline__ void st_vec(T* p, T v) {
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// C16: the block columns come from col16 as differences from `base` (the
// lane's block row, clamped to the last one), two bytes each.  OWN (with
// C16): the lane's own three entries of x, gathered for the block whose
// column is `base` (the diagonal block, or a padding slot), are kept in
// own[] and *got is set, so that the caller need not load them again.
template <typename V, typename X, int UNR = 2, bool NT = false, bool C16 = false, bool OWN = false>
__device__ __forceinline__ void ell_row3all(const V* __restrict__ val, const int32_t* __restrict__ col,
                                            const X* __restrict__ x, int64_t k0, int64_t k1, int lane, X out[3],
                                            const int16_t* __restrict__ col16 = nullptr, int64_t base = 0,
                                            X* own = nullptr, bool* got = nullptr) {
    static_assert(!OWN || C16, "own entries are recognised by the relative block column");
    X a0 = 0, a1 = 0, a2 = 0;
    int64_t k = k0;
    for (; k + UNR <= k1; k += UNR) {
        int32_t cc[UNR];
        V a[UNR][9];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            if (C16) cc[u] = (int32_t)(base + ld_stream<int16_t, NT>(col16 + (k + u) * 64 + lane));
            else cc[u] = ld_stream<int32_t, NT>(col + (k + u) * 64 + lane);
            const V* vb = val + (k + u) * 9 * 64 + lane;
#pragma unroll
            for (int e = 0; e < 9; ++e) a[u][e] = ld_stream<V, NT>(vb + e * 64);
        }
        X xs[UNR][3];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t c = 3 * (int64_t)cc[u];
            xs[u][0] = x[c];
            xs[u][1] = x[c + 1];
            xs[u][2] = x[c + 2];
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            if (OWN && cc[u] == base) {
                own[0] = xs[u][0];
                own[1] = xs[u][1];
                own[2] = xs[u][2];
                *got = true;
            }
            a0 += (X)a[u][0] * xs[u][0] + (X)a[u][1] * xs[u][1] + (X)a[u][2] * xs[u][2];
            a1 += (X)a[u][3] * xs[u][0] + (X)a[u][4] * xs[u][1] + (X)a[u][5] * xs[u][2];
            a2 += (X)a[u][6] * xs[u][0] + (X)a[u][7] * xs[u][1] + (X)a[u][8] * xs[u][2];
        }
    }
    for (; k < k1; ++k) {
        const int64_t cb = C16 ? base + (int64_t)col16[k * 64 + lane] : (int64_t)col[k * 64 + lane];
        const int64_t c = 3 * cb;
        const V* vb = val + k * 9 * 64 + lane;
        const X x0 = x[c], x1 = x[c + 1], x2 = x[c + 2];
        if (OWN && cb == base) {
            own[0] = x0;
            own[1] = x1;
            own[2] = x2;
            *got = true;
        }
        a0 += (X)vb[0] * x0 + (X)vb[64] * x1 + (X)vb[128] * x2;
        a1 += (X)vb[192] * x0 + (X)vb[256] * x1 + (X)vb[320] * x2;
        a2 += (X)vb[384] * x0 + (X)vb[448] * x1 + (X)vb[512] * x2;
    }
    out[0] = a0;
    out[1] = a1;
    out[2] = a2;
}

// ------------------------------------------------------------------ K1
// q = A w over sliced ELL; per-workgroup partial sums of (w, q) go to
// part1[bid].  alpha = rho / (w, q) is formed from them by every workgroup
// of the next kernel (a fixed-order sum, so all agree).
// VAR: the load schedule fixed at compile time (the single-system kernel,
// one instantiation per schedule, so the registers are those of the one in
// use; 4 and 6 are schedules 0 and 2 with 16-bit relative block columns),
// or -1 to take v.spmv_var at run time (the batch kernel); bit 3 added to a
// schedule with non-temporal loads writes q with non-temporal stores.
template <typename V, typename W, int B, int VAR = -1>
__device__ __forceinline__ void spmv_dot_body(const SysView<V, W>& v, int64_t bid) {
    // VAR bit 3: q goes out with non-temporal stores
    constexpr bool NTS = VAR >= 0 && (VAR & 8) != 0;
    constexpr int VS = VAR >= 0 ? (VAR & 7) : VAR;
    if (!gate(v.st, M_RUN)) return;
    const bool tm = ktime_sample(v.st, 0);
    ktime_begin(v.kslots, 0, bid, tm);
    __shared__ double lds[8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nblk = v.geo.g1;
    double part = 0.0;
    if (B == 1) {
        // 4 slices per workgroup, one per wave
        for (int64_t sl = bid * 4 + wave; sl < v.nslices; sl += nblk * 4) {
            const int64_t k0 = v.slice_ptr[sl], k1 = v.slice_ptr[sl + 1];
            const W acc = v.op64 ? ell_row1<double, W>(v.val64, v.col, v.w, k0, k1, lane)
                                 : ell_row1<V, W>(v.val, v.col, v.w, k0, k1, lane);
            const int64_t row = sl * 64 + lane;
            if (row < v.n) {
                st_vec<NTS>(v.q + row, acc);
                part += (double)v.w[row] * (double)acc;
            }
        }
    } else {
        // two slices per workgroup step, one per wave; a lane owns a block row
        const int var = VAR >= 0 ? VAR : v.spmv_var;
        for (int64_t sl = bid * 2 + wave; sl < v.nslices; sl += nblk * 2) {
            const int64_t k0 = v.slice_ptr[sl], k1 = v.slice_ptr[sl + 1];
            W acc[3];
            W own[3] = {0, 0, 0};
            bool got = false;
            const int64_t prow = sl * 64 + lane;
            const int64_t base = prow < v.nb ? prow : v.nb - 1;
            if (VS == 4) {
                ell_row3all<double, W, 2, false, true, true>(v.val64, v.col, v.w, k0, k1, lane, acc, v.col16, base,
                                                             own, &got);
            } else if (VS == 6) {
                ell_row3all<double, W, 2, true, true, true>(v.val64, v.col, v.w, k0, k1, lane, acc, v.col16, base,
                                                            own, &got);
            } else if (std::is_same<V, double>::value || v.op64) {
                // (a double-precision basis always has the double-precision operator)
                if ((var & 3) == 0) ell_row3all<double, W, 2, false>(v.val64, v.col, v.w, k0, k1, lane, acc);
                else if ((var & 3) == 1) ell_row3all<double, W, 4, false>(v.val64, v.col, v.w, k0, k1, lane, acc);
                else if ((var & 3) == 2) ell_row3all<double, W, 2, true>(v.val64, v.col, v.w, k0, k1, lane, acc);
                else ell_row3all<double, W, 4, true>(v.val64, v.col, v.w, k0, k1, lane, acc);
            } else {
                ell_row3all<V, W>(v.val, v.col, v.w, k0, k1, lane, acc);
            }
            const int64_t p = sl * 64 + lane;
            if (p < v.nb) {
                // the row's own entries of w: from the gather where the row
                // stores its diagonal block (schedules 4 and 6), else loaded
                if (!got) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) own[d] = v.w[3 * p + d];
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    st_vec<NTS>(v.q + 3 * p + d, acc[d]);
                    part += (double)own[d] * (double)acc[d];
                }
            }
        }
    }
    const double bs = block_sum(part, lds);
    if (threadIdx.x == 0) v.part1[bid] = bs;
    ktime_end(v.kslots, 0, bid, tm);
}

// ------------------------------------------------------------------ K3
// Projector sums of one step: tacc[c] += sum_i AC[i, c] ss[i] and
// vacc[c] += sum_i AC[i, c] ws[i] over `rows` rows of a row-major AC tile
// (leading dimension ld: 4, 8, 16 or a multiple of 32 elements, so that a
// basis of a few columns costs few bytes).  Columns are taken in chunks of
// 128 bytes (or the whole row when it is shorter); a lane reads 16 bytes (QW
// columns) of one row, so LPR lanes cover a chunk of a row and a wave reads
// 64 / LPR rows per load.
// Each wave works on one (chunk, row phase) item: with fewer chunks than
// waves a chunk gets P waves that interleave its rows, so every chunk of the
// tile streams at once and each lane keeps UR loads in flight (the rows of a
// step take one or two rounds of loads instead of one per chunk).  Lanes of
// equal column are combined by shuffles, the waves of a chunk in a fixed
// order through LDS.
template <typename V>
struct alignas(16) Vec16 {
    V e[16 / sizeof(V)];
};

// Rows per load group of a lane: the single-system update kernel runs one
// workgroup per compute unit (up to 256 registers per lane), the fused batch
// kernel several (128).  The summation order does not depend on it.
constexpr int kUrOne = 12;
constexpr int kUrBatch = 4;

// Work split of the projection: wave `wave` takes item wave + k NW of the
// items (chunk it % nch, row phase it / nch), P waves per chunk.  A chunk
// is 128 bytes of a row, or the whole row when the leading dimension is
// shorter (a power of two from 16 bytes): LPR lanes read 16 bytes each of
// one row, a wave RPW rows per load.
template <typename V>
struct ProjSplit {
    static constexpr int QW = 16 / sizeof(V);
    static constexpr int CW = 128 / sizeof(V);
    static constexpr int NW = kT3 / 64;
    int cw, lpr, rpw, nch, P, items, step, q, rsub;
    __device__ ProjSplit(int nc, int64_t ld) {
        const int lane = threadIdx.x & 63;
        cw = ld < CW ? (int)ld : CW;
        lpr = cw / QW;
        rpw = 64 / lpr;
        q = lane % lpr;
        rsub = lane / lpr;
        nch = (nc + cw - 1) / cw;
        P = nch < NW ? NW / nch : 1;
        items = P * nch;
        step = rpw * P;
    }
};

// FULL: rows of at least one 128-byte chunk (the chunk geometry is then
// known at compile time).
//
// project_acc: item (chunk ch, row phase ph) of one wave over `rows` rows,
// added into the lane's sums at / av.
template <typename V, int UR, bool FULL>
__device__ __forceinline__ void project_acc(const V* __restrict__ ACt, int64_t ld, int rows, const double* ss,
                                            const double* ws, int ch, int ph, double* at, double* av,
                                            const ProjSplit<V>& g) {
    using G = ProjSplit<V>;
    constexpr int QW = G::QW;
    const int CW = FULL ? G::CW : g.cw, RPW = FULL ? 64 / (G::CW / QW) : g.rpw;
    const int q = g.q, rsub = g.rsub, step = g.step;
    const V* base = ACt + ch * CW + q * QW;
    for (int r0 = ph * RPW + rsub; r0 < rows; r0 += step * UR) {
        // rows past the step are clamped to its last row (weight 0)
        // so every load of the group is issued unconditionally
        Vec16<V> a[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const int rr = min(r0 + u * step, rows - 1);
            a[u] = *reinterpret_cast<const Vec16<V>*>(base + (int64_t)rr * ld);
        }
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const int rr = r0 + u * step;
            const bool ok = rr < rows;
            const double sv = ok ? ss[rr] : 0.0, wv = ok ? ws[rr] : 0.0;
#pragma unroll
            for (int e = 0; e < QW; ++e) {
                at[e] += (double)a[u].e[e] * sv;
                av[e] += (double)a[u].e[e] * wv;
            }
        }
    }
}

// project_flush: the lanes' sums of round k0 (items k0 .. k0 + NW - 1, one
// per wave) added into tacc / vacc: lanes of equal column by shuffles, the
// waves of a chunk in a fixed order through LDS.  Every thread of the
// workgroup calls it (two barriers).
template <typename V, bool FULL>
__device__ __forceinline__ void project_flush(double* at, double* av, int k0, int nc, double* tacc, double* vacc,
                                              double (*cred)[64], const ProjSplit<V>& g) {
    using G = ProjSplit<V>;
    constexpr int QW = G::QW, NW = G::NW;
    const int CW = FULL ? G::CW : g.cw, LPR = FULL ? G::CW / QW : g.lpr;
    const int wave = threadIdx.x >> 6;
    const int q = g.q, rsub = g.rsub, nch = g.nch, P = g.P;
    const bool act = k0 + wave < g.items;
#pragma unroll
    for (int e = 0; e < QW; ++e) {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            if (off >= LPR) {
                at[e] += __shfl_xor(at[e], off, 64);
                av[e] += __shfl_xor(av[e], off, 64);
            }
        }
    }
    if (rsub == 0 && act) {
#pragma unroll
        for (int e = 0; e < QW; ++e) {
            cred[wave][q * QW + e] = at[e];
            cred[wave][32 + q * QW + e] = av[e];
        }
    }
    __syncthreads();
    // chunks of this round: all of them when there are fewer than waves
    // (wave cl + p nch holds phase p of chunk cl), else NW of them
    const int nchr = nch <= NW ? nch : min(NW, nch - k0);
    const int t = threadIdx.x;
    if (t < nchr * CW) {
        const int cl = t / CW, e = t % CW;
        const int c = (nch <= NW ? cl : k0 + cl) * CW + e;
        if (c < nc) {
            double ts = 0.0, vs = 0.0;
            for (int p = 0; p < P; ++p) {
                const int w = cl + p * nch;
                ts += cred[w][e];
                vs += cred[w][32 + e];
            }
            tacc[c] += ts;
            vacc[c] += vs;
        }
    }
    __syncthreads();
}

template <typename V, int UR, bool FULL>
__device__ __forceinline__ void project_rows(const V* __restrict__ ACt, int64_t ld, int rows, int nc,
                                             const double* ss, const double* ws, double* tacc, double* vacc,
                                             double (*cred)[64], const ProjSplit<V>& g) {
    constexpr int QW = ProjSplit<V>::QW, NW = ProjSplit<V>::NW;
    const int wave = threadIdx.x >> 6;
    for (int k0 = 0; k0 < g.items; k0 += NW) {
        const int it = k0 + wave;
        double at[QW], av[QW];
#pragma unroll
        for (int e = 0; e < QW; ++e) {
            at[e] = 0.0;
            av[e] = 0.0;
        }
        if (it < g.items) project_acc<V, UR, FULL>(ACt, ld, rows, ss, ws, it % g.nch, it / g.nch, at, av, g);
        project_flush<V, FULL>(at, av, k0, nc, tacc, vacc, cred, g);
    }
}

// Loads of A C issued ahead.  When the items do not outnumber the waves and
// a step's rows take at most UF loads per lane, a wave's loads of the
// step's rows of A C are issued together with the step's vector loads, so
// that the two latencies overlap instead of following each other across
// the barrier; the products follow the barrier.
template <typename V, int UF>
__device__ __forceinline__ bool proj_ahead_fits(int rows, const ProjSplit<V>& g) {
    return g.items <= ProjSplit<V>::NW && rows <= g.step * UF;
}
template <typename V, int UF>
__device__ __forceinline__ void proj_ahead_issue(const V* __restrict__ ACt, int64_t ld, int rows,
                                                 const ProjSplit<V>& g, Vec16<V>* a) {
    const int wave = threadIdx.x >> 6;
    if (wave >= g.items) return;
    const V* base = ACt + (wave % g.nch) * g.cw + g.q * ProjSplit<V>::QW;
    const int r0 = (wave / g.nch) * g.rpw + g.rsub;
#pragma unroll
    for (int u = 0; u < UF; ++u) {
        const int rr = min(r0 + u * g.step, rows - 1);
        a[u] = *reinterpret_cast<const Vec16<V>*>(base + (int64_t)rr * ld);
    }
}
template <typename V, int UF>
__device__ __forceinline__ void proj_ahead_acc(const Vec16<V>* a, int rows, const double* ss, const double* ws,
                                               double* at, double* av, const ProjSplit<V>& g) {
    constexpr int QW = ProjSplit<V>::QW;
    const int wave = threadIdx.x >> 6;
    if (wave >= g.items) return;
    const int r0 = (wave / g.nch) * g.rpw + g.rsub;
#pragma unroll
    for (int u = 0; u < UF; ++u) {
        const int rr = r0 + u * g.step;
        const bool ok = rr < rows;
        const double sv = ok ? ss[rr] : 0.0, wv = ok ? ws[rr] : 0.0;
#pragma unroll
        for (int e = 0; e < QW; ++e) {
            at[e] += (double)a[u].e[e] * sv;
            av[e] += (double)a[u].e[e] * wv;
        }
    }
}

// mode 0: x += alpha w, r -= alpha q (the regular step)
// mode 1: initial step (r0 given), no update
// mode 2: after a true-residual replacement, no update
// then s = M^-1 r and per-workgroup partials, stride 2 nc + 2:
//   [ ||r||^2, (r, s), t = (AC)^T s (nc), v = (AC)^T w (nc, modes 0 and 2) ]
// v measures the A-component of w along C, which is zero in exact
// arithmetic; it drives the recurrence for u = C^T r used to form
// rho = (r, z) = (r, s) - (C^T r)^T mu exactly.  Workgroup bid owns the
// block rows [bid cb3, (bid + 1) cb3), one thread per block row, in steps
// of kT3 block rows; the step's s and w go through LDS to the projector.
// F3: one workgroup.  Reduces the partials of K1 (mode 0) and K3, records
// alpha_j, gamma_j, rho_{j+1}, decides convergence / refinement / breakdown
// and forms beta, mu = G^-1 t, mu2 and u = C^T r for the direction update.
// A single workgroup is latency bound, so every independent load (device
// state, K3 and K1 partials, G^-1, u) is issued before the first wait, and
// the state is worked on in LDS and written back once at the end.
// LDS (doubles) of the finalize body
constexpr int kStateWords = 32;
constexpr int fin_pool() { return kStateWords + kTF3 + 2056 + 3 * 1024 + 4096 + 8; }

// Inputs of the finalize that no workgroup of the launch writes before it
// runs (state words, u, G^-1): loaded into registers by fin_prefetch, which
// the fused update's group reducers issue before their last ticket.
struct FinPre {
    static constexpr int UU = 1024 / kTF3;
    static constexpr int GU = 4096 / kTF3;
    unsigned long long sw;
    double uv[UU];
    double gv[GU];
};
template <typename V, typename W>
__device__ __forceinline__ void fin_prefetch(const SysView<V, W>& v, int mode, FinPre& f) {
    constexpr int T = kTF3;
    constexpr int NWORD = (int)(sizeof(DevState) / 8);
    const int tid = threadIdx.x;
    const int nc = v.nc;
    f.sw = 0ull;
    if (tid < NWORD) f.sw = reinterpret_cast<const unsigned long long*>(v.st)[tid];
    if (mode == 0 && nc > 0) {
#pragma unroll
        for (int u = 0; u < FinPre::UU; ++u) f.uv[u] = v.u[min(tid + u * T, nc - 1)];
    }
    if (nc <= 64 && nc > 0) {
#pragma unroll
        for (int u = 0; u < FinPre::GU; ++u) f.gv[u] = v.Ginv[min(tid + u * T, nc * nc - 1)];
    }
}

// g_in: (w, q) of this step when the caller has already reduced the SpMV
// partials (the fused update, in the same order), else negative.  pre:
// fin_prefetch of this launch, or null.
template <typename V, typename W, bool COH>
__device__ __forceinline__ void finalize_update_body(const SysView<V, W>& v, int mode, double* pool,
                                                     double g_in = -1.0, const FinPre* pre = nullptr) {
    constexpr int T = kTF3;
    constexpr int NWORD = (int)(sizeof(DevState) / 8);
    static_assert(NWORD <= kStateWords, "state staging area too small");
    DevState& S = *reinterpret_cast<DevState*>(pool);
    double* red = pool + kStateWords;
    double* fin = red + T;
    double* muL = fin + 2056;
    double* gvL = muL + 1024;
    double* uL = gvL + 1024;
    double* Gl = uL + 1024;
    double& beta_s = Gl[4096];
    const int tid = threadIdx.x;
    const int nc = v.nc;
    const int nv = 2 * nc + 2;
    const int64_t np3 = v.geo.g3, np1 = v.geo.g1;
    const int64_t ng = (np3 + kGroup - 1) / kGroup;
    // ---- loads (state, SpMV partials, u, G^-1 and the update's sums): each
    // is issued at a clamped, valid address before any is used, so their
    // latencies overlap
    FinPre f;
    if (pre) f = *pre;
    else fin_prefetch(v, mode, f);
    const bool need_g = mode == 0 && !(g_in >= 0.0);
    double pt[4];
    if (need_g) {
#pragma unroll
        for (int u = 0; u < 4; ++u) pt[u] = v.part1[min((int64_t)tid + u * T, np1 - 1)];
    }
    constexpr int UU = FinPre::UU, GU = FinPre::GU;
    const bool have_u = mode == 0 && nc > 0;
    const bool gsmall = nc <= 64;
    // the groups' sums of this thread's column in one pass (the usual case)
    const double* gsum = v.partials + np3 * nv;
    const bool one = COH && nv <= T && ng <= 16;
    double gl[16];
    if (one) {
        const int kk = min(tid, nv - 1);
#pragma unroll
        for (int u = 0; u < 16; ++u) gl[u] = ld_part<true>(gsum + min((int64_t)u, ng - 1) * nv + kk);
    }
    // ---- use
    double p1 = 0.0;
    if (need_g) {
        // the order of thread_sum<4>
#pragma unroll
        for (int u = 0; u < 4; ++u) p1 += (tid + (int64_t)u * T < np1) ? pt[u] : 0.0;
        for (int64_t i = tid + 4 * (int64_t)T; i < np1; i += T) p1 += v.part1[i];
    }
#pragma unroll
    for (int u = 0; u < UU; ++u)
        if (tid + u * T < nc) uL[tid + u * T] = have_u ? f.uv[u] : 0.0;
    if (gsmall) {
#pragma unroll
        for (int u = 0; u < GU; ++u)
            if (tid + u * T < nc * nc) Gl[tid + u * T] = f.gv[u];
    }
    // fin[k]: the groups' sums (written by the group reducers, COH) in
    // ascending order, or both levels here
    if (one) {
        if (tid < nv) {
            double s2 = 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (u < ng) s2 += gl[u];
            fin[tid] = s2;
        }
    } else {
        for (int kk = tid; kk < nv; kk += T) {
            double s2 = 0.0;
            if (COH) {
                s2 = col_sum<true>(gsum, ng, nv, kk);
            } else {
                for (int64_t g = 0; g < ng; ++g) {
                    const int64_t r0 = g * kGroup;
                    const int64_t rn = (np3 - r0) < kGroup ? (np3 - r0) : kGroup;
                    s2 += col_sum<false>(v.partials + r0 * nv, rn, nv, kk);
                }
            }
            fin[kk] = s2;
        }
    }
    if (tid < NWORD) reinterpret_cast<unsigned long long*>(&S)[tid] = f.sw;
    __syncthreads();
    const uint32_t mask = (mode == 2) ? M_REFINE : M_RUN;
    if (((1u << S.status) & mask) == 0) return;
    const double g = need_g ? sum_all_reg(p1, red) : (mode == 0 ? g_in : 0.0);
    const double a = (mode == 0) ? S.rho / g : 0.0;
    double du = 0.0;
    if (nc > 0 && gsmall) {
        // G^-1 t, G^-1 (AC)^T w and the u recurrence with one barrier: row r
        // of G^-1 is taken by the 8 lanes 8 r .. 8 r + 7 of one wave (part p
        // sums the columns p, p + 8, ...; the parts are added by shuffles);
        // u^T mu is summed in row order by thread 0.
        static_assert(T == 512, "eight lanes per row of an up to 64-column G^-1");
        const int r = tid >> 3, p = tid & 7;
        double m = 0.0, mv = 0.0;
        if (r < nc) {
            for (int c = p; c < nc; c += 8) {
                const double g = Gl[c * nc + r];
                m += g * fin[2 + c];
                mv += g * fin[2 + nc + c];
            }
        }
#pragma unroll
        for (int off = 1; off < 8; off <<= 1) {
            m += __shfl_xor(m, off, 64);
            mv += __shfl_xor(mv, off, 64);
        }
        if (r < nc && p == 0) {
            muL[r] = m;
            gvL[r] = mv;
            // u = C^T r: recurrence u -= alpha (AC)^T w; zero after (re)projection
            const double uc = (mode == 0) ? uL[r] - a * fin[2 + nc + r] : 0.0;
            v.u[r] = uc;
            v.mu[r] = m;
            red[r] = uc * m;
        }
        __syncthreads();
        if (tid == 0)
            for (int i = 0; i < nc; ++i) du += red[i];
    } else if (nc > 0) {
        const double* Gi = gsmall ? Gl : v.Ginv;
        ginv_matvec2(Gi, nc, fin + 2, fin + 2 + nc, muL, gvL, red);
        // u = C^T r: recurrence u -= alpha (AC)^T w; zero after (re)projection
        double p = 0.0;
        for (int c = tid; c < nc; c += T) {
            const double uc = (mode == 0) ? uL[c] - a * fin[2 + nc + c] : 0.0;
            v.u[c] = uc;
            v.mu[c] = muL[c];
            p += uc * muL[c];
        }
        du = sum_all_reg(p, red);
    }
    const int j0 = S.iter;
    if (mode == 0 && S.ktime_on) {
        unsigned long long* tl = reinterpret_cast<unsigned long long*>(Gl);
        if ((j0 & 31) == 1) {
            ktime_collect(&S, v.kslots, 0, np1, tl);
            ktime_collect(&S, v.kslots, 1, np3, tl);
        } else if ((j0 & 31) == 2) {
            ktime_collect(&S, v.kslots, 2, v.geo.g5, tl);
        }
    }
    if (tid == 0) {
        const double rrn = fin[0];
        const double rho_new = fin[1] - du;  // (r, z) = (r, s) - (C^T r)^T mu
        const double rr_before = S.rr;
        const int j = j0;
        int stn = ST_RUN;
        if (mode == 0) {
            if (j < v.coef_cap) {
                v.gamma_h[j] = g;
                v.alpha_h[j] = a;
            }
            S.alpha = a;
            S.pending_dir = 0;
            const int it = j + 1;
            S.iter = it;
            S.since_refine += 1;
            S.rr = rrn;
            if (!finite_pos(g) || !(rrn == rrn)) {
                stn = ST_BREAKDOWN;
            } else if (rrn <= S.tol2 * S.bb) {
                stn = ST_CHECK;
            } else if (it >= S.max_iter) {
                stn = ST_MAXIT;
            } else if ((S.refine_every > 0 && S.since_refine >= S.refine_every) ||
                       (S.drop2 > 0.0 && rrn < S.drop2 * S.rr_ref)) {
                stn = ST_REFINE;
            }
        } else {
            S.rr = rrn;
            S.rr_ref = rrn;
            if (mode == 2) {
                S.since_refine = 0;
                S.pending_dir = 1;
            } else {
                if (rrn <= S.tol2 * S.bb) stn = ST_CHECK;
                if (S.max_iter <= 0 && stn == ST_RUN) stn = ST_MAXIT;
            }
        }
        if (stn == ST_RUN) {
            if (!finite_pos(rho_new)) {
                stn = ST_BREAKDOWN;
            } else {
                const int it = S.iter;
                double beta = (mode == 1) ? 0.0 : rho_new / S.rho;
                // A replacement that more than doubles the residual (the
                // single-precision operator's floor reached) voids the
                // conjugacy with the old direction: restart from z.
                if (mode == 2 && rrn > 4.0 * rr_before) {
                    beta = 0.0;
                    S.restarts += 1;
                    if (it < S.first_restart) S.first_restart = it;
                }
                S.beta = beta;
                S.rho = rho_new;
                if (it < v.coef_cap) v.rho_h[it] = rho_new;
            }
        }
        S.status = stn;
        beta_s = (stn == ST_RUN) ? S.beta : 0.0;
    }
    __syncthreads();
    if (tid < NWORD) reinterpret_cast<unsigned long long*>(v.st)[tid] = reinterpret_cast<const unsigned long long*>(&S)[tid];
    // the new direction is projected as a whole: w = P (z + beta w_old)
    // = s + beta w_old - C (mu + beta G^-1 (AC)^T w_old); with dir_literal
    // the old direction is taken as it is (w = z + beta w_old)
    const double bt = v.dir_literal ? 0.0 : beta_s;
    for (int c = tid; c < nc; c += T) v.mu2[c] = muL[c] + bt * gvL[c];
}

// LDS (doubles) of the update body for block size B
template <int B>
constexpr int upd_pool() {
    return 2 * kT3 * B + kT3 + 2048 + kT3;
}

// SINGLE: the single-system kernel, which also instantiates the projection
// with compile-time chunk geometry (same lanes and order as the general one).
// NTS: x, r and s go out with non-temporal stores.
template <typename V, typename W, int B, bool FUSE, int UR, bool SINGLE = false, bool NTS = false>
__device__ __forceinline__ void update_reduce_body(const SysView<V, W>& v, int64_t bid, int mode, double* pool) {
    DevState* st = v.st;
    const uint32_t mask = (mode == 2) ? M_REFINE : M_RUN;
    // the state words this body reads, loaded together up front (the
    // finalize that rewrites them runs after every workgroup has read them)
    const int32_t st_status = st->status, st_iter = st->iter, st_kt = st->ktime_on;
    const double st_rho = st->rho;
    constexpr int T = kT3;
    double* ss = pool;
    double* ws = ss + T * B;
    double* red = ws + T * B;
    double* tacc = red + T;
    double* vacc = tacc + 1024;
    double(*cred)[64] = reinterpret_cast<double(*)[64]>(vacc + 1024);
    const int tid = threadIdx.x;
    const int nc = v.nc;
    for (int c = tid; c < nc; c += T) {
        tacc[c] = 0.0;
        vacc[c] = 0.0;
    }
    const int64_t pb = bid * v.geo.cb3;
    const int64_t pe = (pb + v.geo.cb3) < v.nb ? (pb + v.geo.cb3) : v.nb;
    const ProjSplit<V> pg(nc, v.ldac);
    // With no more projection items than waves each wave keeps the running
    // sums of its item over all the steps of the range and they are reduced
    // across lanes and waves once, at the end; otherwise each step's sums
    // are reduced after that step.
    // This is done when, besides, a step's rows of A C take at most UF loads
    // per lane: those loads are then issued together with the step's vector
    // loads, so that the two latencies overlap instead of following each
    // other across the step's barrier (a 3x3-block step is 1008 rows: four
    // loads cover a basis of up to 4 double or 8 single columns; a scalar
    // step is 512 rows: two loads cover 2 double or 8 single columns).
    using PS = ProjSplit<V>;
    constexpr int UF = (B == 3) ? 4 : 2;
    constexpr int step_rows = (B == 3) ? 2 * 3 * 21 * (T / 64) : T * B;
    const bool persist = nc > 0 && proj_ahead_fits<V, UF>(step_rows, pg);
    double pat[PS::QW], pav[PS::QW];
#pragma unroll
    for (int e = 0; e < PS::QW; ++e) {
        pat[e] = 0.0;
        pav[e] = 0.0;
    }
    bool tm = false;
    double rr = 0.0, rs = 0.0;
    double a = 0.0, gam = -1.0;
    bool have_a = mode != 0;
    const bool run = ((1u << st_status) & mask) != 0;
    if (pb >= pe && !run) return;
    if constexpr (B == 3) {
        // One thread per unknown: in each of SUB sub-steps a wave takes 63
        // consecutive unknowns (21 block rows; lane 63 idles), so the loads
        // and stores of x, r, w, q and s are contiguous across the wave, and
        // so are the loads of the lane's row of the 3x3 block M^-1 (M^-1 is
        // stored as three planes of columns: entry c of unknown i at c n + i).
        // The residual entries of the other rows of the block come from the
        // neighbouring lanes.
        constexpr int NWV = T / 64, BPW = 21, SUB = 2;
        constexpr int SB = NWV * BPW * SUB;  // block rows per step
        static_assert(SB * 3 <= T * B, "a step's s and w fit the LDS rows of the projection");
        const int lane = tid & 63, wave = tid >> 6;
        const int l0 = lane - lane % 3;
        for (int64_t ps = pb; ps < pe; ps += SB) {
            const int64_t pn = (ps + SB) < pe ? (ps + SB) : pe;
            const int nloc = (int)((pn - ps) * 3);
            int loc[SUB];
            bool act[SUB];
            W rv[SUB], qv[SUB];
            double xv[SUB], wi[SUB];
            V mv[SUB][3];
#pragma unroll
            for (int k = 0; k < SUB; ++k) {
                loc[k] = k * (NWV * BPW * 3) + wave * (BPW * 3) + lane;
                act[k] = lane < 63 && loc[k] < nloc;
                wi[k] = 0.0;
                if (act[k]) {
                    const int64_t i = ps * 3 + loc[k];
                    rv[k] = v.r[i];
                    if (mode != 1) wi[k] = (double)v.w[i];
                    if (mode == 0) {
                        qv[k] = v.q[i];
                        xv[k] = v.x[i];
                    }
#pragma unroll
                    for (int e = 0; e < 3; ++e) mv[k][e] = v.minv[(int64_t)e * (3 * v.nb) + i];
                }
            }
            Vec16<V> ahead[UF];
            if (persist) proj_ahead_issue<V, UF>(v.AC + ps * 3 * v.ldac, v.ldac, nloc, pg, ahead);
            // the status is tested once the first step's loads are issued
            // (they are in bounds whatever it is), so the latencies overlap
            if (ps == pb) {
                if (!run) return;
                tm = mode == 0 && st_kt && (st_iter & 31) == 1;
                ktime_begin(v.kslots, 1, bid, tm);
            }
            if (!have_a) {
                gam = sum_all(v.part1, v.geo.g1, red);
                a = st_rho / gam;
                have_a = true;
            }
            double si[SUB];
#pragma unroll
            for (int k = 0; k < SUB; ++k) {
                W r2 = act[k] ? rv[k] : (W)0;
                double xn = 0.0;
                if (act[k] && mode == 0) {
                    xn = xv[k] + a * wi[k];
                    r2 = (W)((double)r2 - a * (double)qv[k]);
                }
                const double ri = (double)r2;
                // the block's three residual entries (every lane takes part in the shuffles)
                const double r0 = __shfl(ri, l0, 64), r1 = __shfl(ri, l0 + 1, 64), r2d = __shfl(ri, l0 + 2, 64);
                si[k] = 0.0;
                if (act[k]) {
                    si[k] = (double)(W)((double)mv[k][0] * r0 + (double)mv[k][1] * r1 + (double)mv[k][2] * r2d);
                    rr += ri * ri;
                    rs += ri * si[k];
                    const int64_t i = ps * 3 + loc[k];
                    if (mode == 0) {
                        st_vec<NTS>(v.x + i, xn);
                        st_vec<NTS>(v.r + i, (W)r2);
                    }
                    st_vec<NTS>(v.s + i, (W)si[k]);
                }
            }
            if (nc > 0) {
                // s and w of the step to LDS for the projection, once every
                // wave is done with the previous step's rows (a per-step
                // reduction ends with a barrier)
                if (persist && ps != pb) __syncthreads();
#pragma unroll
                for (int k = 0; k < SUB; ++k)
                    if (act[k]) {
                        ss[loc[k]] = si[k];
                        ws[loc[k]] = wi[k];
                    }
                __syncthreads();
                if (persist)
                    proj_ahead_acc<V, UF>(ahead, nloc, ss, ws, pat, pav, pg);
                else if (SINGLE && v.ldac >= ProjSplit<V>::CW)
                    project_rows<V, UR, true>(v.AC + ps * 3 * v.ldac, v.ldac, nloc, nc, ss, ws, tacc, vacc, cred,
                                              pg);
                else
                    project_rows<V, UR, false>(v.AC + ps * 3 * v.ldac, v.ldac, nloc, nc, ss, ws, tacc, vacc, cred,
                                               pg);
            }
        }
    } else {
        for (int64_t ps = pb; ps < pe; ps += T) {
            const int64_t p = ps + tid;
            double ri[B], wi[B], si[B];
#pragma unroll
            for (int d = 0; d < B; ++d) {
                ri[d] = 0.0;
                wi[d] = 0.0;
                si[d] = 0.0;
            }
            // the step's vector loads are issued before alpha is formed from
            // the SpMV partials, so the two latencies overlap
            W rv[B], qv[B];
            double xv[B];
            V mv[B * B];
            if (p < pe) {
#pragma unroll
                for (int d = 0; d < B; ++d) {
                    const int64_t i = p * B + d;
                    rv[d] = v.r[i];
                    if (mode != 1) wi[d] = (double)v.w[i];
                    if (mode == 0) {
                        qv[d] = v.q[i];
                        xv[d] = v.x[i];
                    }
                }
#pragma unroll
                for (int e = 0; e < B * B; ++e) mv[e] = v.minv[p * B * B + e];
            }
            const int64_t pn = (ps + T) < pe ? (ps + T) : pe;
            const int rows = (int)((pn - ps) * B);
            Vec16<V> ahead[UF];
            if (persist) proj_ahead_issue<V, UF>(v.AC + ps * B * v.ldac, v.ldac, rows, pg, ahead);
            // the status is tested once the first step's loads are issued (they
            // are in bounds whatever it is), so the latencies overlap
            if (ps == pb) {
                if (!run) return;
                tm = mode == 0 && st_kt && (st_iter & 31) == 1;
                ktime_begin(v.kslots, 1, bid, tm);
            }
            if (!have_a) {
                gam = sum_all(v.part1, v.geo.g1, red);
                a = st_rho / gam;
                have_a = true;
            }
            double xn[B];
            W rn[B];
            if (p < pe) {
#pragma unroll
                for (int d = 0; d < B; ++d) {
                    W r2 = rv[d];
                    if (mode == 0) {
                        xn[d] = xv[d] + a * wi[d];
                        r2 = (W)((double)r2 - a * (double)qv[d]);
                    }
                    rn[d] = r2;
                    ri[d] = (double)r2;
                }
                if (B == 1) {
                    si[0] = (double)(W)((double)mv[0] * ri[0]);
                } else {
#pragma unroll
                    for (int d = 0; d < B; ++d)
                        si[d] = (double)(W)((double)mv[3 * d] * ri[0] + (double)mv[3 * d + 1] * ri[1] +
                                            (double)mv[3 * d + 2] * ri[2]);
                }
#pragma unroll
                for (int d = 0; d < B; ++d) {
                    rr += ri[d] * ri[d];
                    rs += ri[d] * si[d];
                }
            }
            // s and w go to LDS before the stores are issued, so the barrier
            // does not wait for them (the previous step's projection ended with
            // a barrier, so the buffers are free)
            if (nc > 0) {
                if (persist && ps != pb) __syncthreads();
#pragma unroll
                for (int d = 0; d < B; ++d) {
                    ss[tid * B + d] = si[d];
                    ws[tid * B + d] = wi[d];
                }
                __syncthreads();
            }
            if (p < pe) {
#pragma unroll
                for (int d = 0; d < B; ++d) {
                    const int64_t i = p * B + d;
                    if (mode == 0) {
                        st_vec<NTS>(v.x + i, xn[d]);
                        st_vec<NTS>(v.r + i, (W)rn[d]);
                    }
                    st_vec<NTS>(v.s + i, (W)si[d]);
                }
            }
            if (nc > 0) {
                if (persist)
                    proj_ahead_acc<V, UF>(ahead, rows, ss, ws, pat, pav, pg);
                else if (SINGLE && v.ldac >= ProjSplit<V>::CW)
                    project_rows<V, UR, true>(v.AC + ps * B * v.ldac, v.ldac, rows, nc, ss, ws, tacc, vacc, cred, pg);
                else
                    project_rows<V, UR, false>(v.AC + ps * B * v.ldac, v.ldac, rows, nc, ss, ws, tacc, vacc, cred, pg);
            }
        }
    }
    if (persist) project_flush<V, false>(pat, pav, 0, nc, tacc, vacc, cred, pg);
    const int stride = 2 * nc + 2;
    double* myp = v.partials + bid * stride;
    double brr = rr, brs = rs;
    block_sum2(brr, brs, red);
    __syncthreads();
    if (!FUSE) {
        if (tid == 0) {
            myp[0] = brr;
            myp[1] = brs;
        }
        for (int c = tid; c < nc; c += T) {
            myp[2 + c] = tacc[c];
            myp[2 + nc + c] = vacc[c];
        }
        ktime_end(v.kslots, 1, bid, tm);
        return;
    }
    // Fused finalize: the partials are stored agent-coherent (written
    // through to where every XCD reads them), each thread waits for its
    // stores to complete, and the workgroup that takes the last ticket of
    // the counter reduces them with coherent loads.  Only that workgroup
    // continues; the ticket counter is reset for the next launch.
    if (tid == 0) {
        __hip_atomic_store(myp, brr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(myp + 1, brs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int c = tid; c < nc; c += T) {
        __hip_atomic_store(myp + 2 + c, tacc[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(myp + 2 + nc + c, vacc[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    ktime_end(v.kslots, 1, bid, tm);
    __syncthreads();
    unsigned* ticket = reinterpret_cast<unsigned*>(red);
    const int64_t g3 = v.geo.g3;
    const int64_t grp = bid / kGroup;
    const int64_t ng = (g3 + kGroup - 1) / kGroup;
    const int64_t gsz = (g3 - grp * kGroup) < kGroup ? (g3 - grp * kGroup) : kGroup;
    // level 1: the last workgroup of each group sums the group's rows
    if (tid == 0) *ticket = __hip_atomic_fetch_add(v.sync + 1 + grp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    unsigned mine = *ticket;
    __syncthreads();
    if (mine != (unsigned)(gsz - 1)) return;
    if (tid == 0) __hip_atomic_store(v.sync + 1 + grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double* gsum = v.partials + g3 * stride;
    for (int kk = tid; kk < stride; kk += T) {
        const double s = col_sum<true>(v.partials + grp * kGroup * stride, gsz, stride, kk);
        __hip_atomic_store(gsum + grp * stride + kk, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    // level 2: the last group reducer finishes the step.  The finalize's
    // read-only inputs are loaded while the ticket is in flight, in case
    // this reducer is the last.
    unsigned tk = 0;
    if (tid == 0) tk = __hip_atomic_fetch_add(v.sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    FinPre fpre;
    fin_prefetch(v, mode, fpre);
    if (tid == 0) *ticket = tk;
    __syncthreads();
    mine = *ticket;
    __syncthreads();
    if (mine != (unsigned)(ng - 1)) return;
    if (tid == 0) __hip_atomic_store(v.sync, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    finalize_update_body<V, W, true>(v, mode, pool, gam, &fpre);
}

// ------------------------------------------------------------------ K5
// z = s - C mu and w = s - C mu2 + beta w_old with mu2 = mu + beta G^-1
// (AC)^T w_old, i.e. w = P (z + beta w_old): the whole direction is kept
// A-orthogonal to C (in exact arithmetic (AC)^T w_old = 0 and mu2 = mu, so
// this is Algorithm 1's w = z + beta w_old; with dir_literal mu2 = mu).
// first = 1: initial direction w = z; first = 2: the update that follows a
// residual replacement (runs only when one is pending).  A workgroup owns
// 256 rows: lane l of every wave reads 4 consecutive rows of a column of C
// (16 or 32 bytes), wave k takes the columns k, k + 4, ... (U of them per
// load group; the order of the sums does not depend on U); the four
// partial sums per row are added in LDS in a fixed order.
template <typename V>
struct alignas(4 * sizeof(V)) Quad {
    V e[4];
};

template <typename V, typename W, int U, bool NTS = false>
__device__ __forceinline__ void correct_dir_body(const SysView<V, W>& v, int64_t bid, int first) {
    DevState* st = v.st;
    __shared__ double mu[1024];
    __shared__ double mu2[1024];
    __shared__ double part[4][2][256];
    const int nc = v.nc;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t nblk = (v.n + 255) / 256;
    // the first block's loads of C, s and w are issued before the status
    // test and the wait for the coefficients, so the latencies overlap
    Quad<V> cq[U];
    W sv = 0, wv0 = 0;
    auto load_c = [&](int64_t blk, int c0) {
        const V* Cb = v.C + blk * 256 + 4 * lane;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = c0 + 4 * u;
            cq[u] = (c < nc) ? *reinterpret_cast<const Quad<V>*>(Cb + (int64_t)c * v.ldc) : Quad<V>{{0, 0, 0, 0}};
        }
    };
    auto load_sw = [&](int64_t blk) {
        const int64_t i = blk * 256 + tid;
        if (i < v.n) {
            sv = v.s[i];
            if (first != 1) wv0 = v.w[i];
        }
    };
    if (bid < nblk) {
        if (wave < nc) load_c(bid, wave);
        load_sw(bid);
    }
    // the status is tested after those loads are issued (they are in bounds
    // whatever it is), so its latency overlaps theirs
    if (!gate(st, M_RUN)) return;
    if (first == 2 && st->pending_dir == 0) return;
    for (int c = tid; c < nc; c += 256) {
        mu[c] = v.mu[c];
        mu2[c] = (first == 1) ? v.mu[c] : v.mu2[c];
    }
    const double beta = (first == 1) ? 0.0 : st->beta;
    const int j = st->iter;
    const int hist_cap = st->hist_cap;
    const bool tm = first == 0 && ktime_sample(st, 2);
    ktime_begin(v.kslots, 2, bid, tm);
    __syncthreads();
    bool pre = true;
    for (int64_t blk = bid; blk < nblk; blk += v.geo.g5) {
        double az[4] = {0.0, 0.0, 0.0, 0.0}, aw[4] = {0.0, 0.0, 0.0, 0.0};
        if (!pre) load_sw(blk);
        for (int c0 = wave; c0 < nc; c0 += 4 * U) {
            if (!pre) load_c(blk, c0);
            pre = false;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = c0 + 4 * u;
                if (c < nc) {
                    const double m1 = mu[c], m2 = mu2[c];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        az[e] += (double)cq[u].e[e] * m1;
                        aw[e] += (double)cq[u].e[e] * m2;
                    }
                }
            }
        }
        pre = false;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            part[wave][0][4 * lane + e] = az[e];
            part[wave][1][4 * lane + e] = aw[e];
        }
        __syncthreads();
        const int64_t i = blk * 256 + tid;
        if (i < v.n) {
            const double cz = ((part[0][0][tid] + part[1][0][tid]) + part[2][0][tid]) + part[3][0][tid];
            const double cw = ((part[0][1][tid] + part[1][1][tid]) + part[2][1][tid]) + part[3][1][tid];
            const double s = (double)sv;
            const W zv = (W)(s - cz);
            const W wv = (first == 1) ? zv : (W)(s - cw + beta * (double)wv0);
            st_vec<NTS>(v.w + i, wv);
            if (v.zr) v.zr[i] = zv;
            if (j < hist_cap) {
                if (v.zhist) st_vec<NTS>(v.zhist + (int64_t)j * v.ldh + i, (V)zv);
                if (v.zhist32) st_vec<NTS>(v.zhist32 + (int64_t)j * v.ldh + i, (float)zv);
                if (v.whist) st_vec<NTS>(v.whist + (int64_t)j * v.ldh + i, (V)wv);
            }
        }
    }
    ktime_end(v.kslots, 2, bid, tm);
}

// ------------------------------------------------------- reorthogonalisation
// Full reorthogonalisation (Section 2.1 remark; the experiments of Section
// 5.1): after the direction update of step j, the new direction is
//   w = z - sum_{i < j'} ((A w_i, z) / (w_i, A w_i)) w_i,  j' = min(j, rcap),
// classical Gram-Schmidt in the A inner product over the kept directions
// (in exact arithmetic only the last term is nonzero and equals beta w_old).
// Four launches per step: the store of w_j and A w_j after the SpMV, then
// the partial sums (A w_i, z) per row range, their reduction to the
// coefficients, and the update of w.  The kept vectors are row-major so
// that a row's coefficients stream contiguously.

// after the SpMV of step j: row i of W_r and Q_r gets w_j[i] and (A w_j)[i]
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_reorth_store(SysView<V, W> v) {
    const DevState* st = v.st;
    if (!gate(st, M_RUN)) return;
    const int j = st->iter;
    if (j >= v.rcap) return;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < v.n; i += (int64_t)gridDim.x * 256) {
        v.Wr[i * v.ldr + j] = v.w[i];
        v.Qr[i * v.ldr + j] = v.q[i];
    }
}

// partial sums over the workgroup's row range of (A w_i, z), i < j'; thread
// t takes the columns t, t + 256, ...; rows in order
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_reorth_dot(SysView<V, W> v) {
    const DevState* st = v.st;
    if (!gate(st, M_RUN)) return;
    const int jn = st->iter < v.rcap ? st->iter : v.rcap;
    // workgroup = (row range g, chunk of 256 kept directions): chunks past
    // the directions kept so far have nothing to do
    const int nch = (v.rcap + 255) / 256;
    const int chunk = (int)(blockIdx.x % nch);
    const int64_t g = blockIdx.x / nch;
    if (chunk * 256 >= jn) return;
    __shared__ double zs[256];
    const int64_t per = (v.n + v.gr - 1) / v.gr;
    const int64_t r0 = g * per;
    const int64_t r1 = (r0 + per < v.n) ? r0 + per : v.n;
    const int i = chunk * 256 + (int)threadIdx.x;
    double acc = 0.0;
    for (int64_t rb = r0; rb < r1; rb += 256) {
        __syncthreads();
        if (rb + threadIdx.x < r1) zs[threadIdx.x] = (double)v.zr[rb + threadIdx.x];
        __syncthreads();
        const int cnt = (r1 - rb < 256) ? (int)(r1 - rb) : 256;
        if (i < jn) {
            // four independent chains of loads and products per thread
            const W* q = v.Qr + rb * v.ldr + i;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int t = 0;
            for (; t + 4 <= cnt; t += 4) {
                a0 += (double)q[(int64_t)t * v.ldr] * zs[t];
                a1 += (double)q[(int64_t)(t + 1) * v.ldr] * zs[t + 1];
                a2 += (double)q[(int64_t)(t + 2) * v.ldr] * zs[t + 2];
                a3 += (double)q[(int64_t)(t + 3) * v.ldr] * zs[t + 3];
            }
            for (; t < cnt; ++t) a0 += (double)q[(int64_t)t * v.ldr] * zs[t];
            acc += (a0 + a1) + (a2 + a3);
        }
    }
    if (i < jn) v.rpart[g * v.ldr + i] = acc;
}

// coefficients c_i = (sum over row ranges, in order) / (w_i, A w_i)
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_reorth_reduce(SysView<V, W> v) {
    const DevState* st = v.st;
    if (!gate(st, M_RUN)) return;
    const int jn = st->iter < v.rcap ? st->iter : v.rcap;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < jn; i += gridDim.x * 256) {
        double sum = 0.0;
        for (int g = 0; g < v.gr; ++g) sum += v.rpart[(int64_t)g * v.ldr + i];
        v.rc[i] = sum / v.gamma_h[i];
    }
}

// w = z - sum_i c_i w_i: a wave takes four rows at a time, lanes over i
// (each c_i read once from LDS serves the four rows: four independent
// chains of loads and products), then a fixed shuffle tree per row
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_reorth_apply(SysView<V, W> v) {
    const DevState* st = v.st;
    if (!gate(st, M_RUN)) return;
    const int jn = st->iter < v.rcap ? st->iter : v.rcap;
    __shared__ double cs[kReorthMax];
    for (int i = threadIdx.x; i < jn; i += 256) cs[i] = v.rc[i];
    __syncthreads();
    constexpr int R = 4;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * R; row0 < v.n; row0 += waves * R) {
        const W* wr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) wr[r] = v.Wr + ((row0 + r) < v.n ? (row0 + r) : (v.n - 1)) * v.ldr;
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        for (int i = lane; i < jn; i += 64) {
            const double c = cs[i];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += c * (double)wr[r][i];
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off);
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (row0 + r < v.n) v.w[row0 + r] = (W)((double)v.zr[row0 + r] - acc[r]);
        }
    }
}

// ----------------------------------------------------------------- K11
// r = b - A x with double-precision values and x.  final_only: only record
// ||r||^2 (for the report), leave r and the status alone.
template <typename V, typename W, int B>
__device__ __forceinline__ void true_resid_body(const SysView<V, W>& v, int64_t bid, int final_only) {
    DevState* st = v.st;
    if (!final_only && !gate(st, M_CHECK | M_REFINE)) return;
    __shared__ double lds[8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nblk = v.geo.g1;
    double part = 0.0;
    if (B == 1) {
        for (int64_t sl = bid * 4 + wave; sl < v.nslices; sl += nblk * 4) {
            const int64_t k0 = v.slice_ptr[sl], k1 = v.slice_ptr[sl + 1];
            const double acc = ell_row1<double, double>(v.val64, v.col, v.x, k0, k1, lane);
            const int64_t row = sl * 64 + lane;
            if (row < v.n) {
                const double ri = v.b[row] - acc;
                if (!final_only) v.r[row] = (W)ri;
                part += ri * ri;
            }
        }
    } else {
        for (int64_t sl = bid * 2 + wave; sl < v.nslices; sl += nblk * 2) {
            const int64_t k0 = v.slice_ptr[sl], k1 = v.slice_ptr[sl + 1];
            double acc[3];
            ell_row3all<double, double>(v.val64, v.col, v.x, k0, k1, lane, acc);
            const int64_t p = sl * 64 + lane;
            if (p < v.nb) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double ri = v.b[3 * p + d] - acc[d];
                    if (!final_only) v.r[3 * p + d] = (W)ri;
                    part += ri * ri;
                }
            }
        }
    }
    const double bs = block_sum(part, lds);
    if (threadIdx.x == 0) v.partials[bid] = bs;
}

// F11: one workgroup; ||b - A x||^2 and the decision after a true residual.
template <typename V, typename W>
__device__ __forceinline__ void finalize_resid_body(const SysView<V, W>& v, int final_only) {
    DevState* st = v.st;
    if (!final_only && !gate(st, M_CHECK | M_REFINE)) return;
    __shared__ double red[32];
    const double rt = sum_all(v.partials, v.geo.g1, red);
    if (threadIdx.x == 0) {
        st->rr_true = rt;
        if (!final_only) {
            if (rt <= st->tol2 * st->bb) {
                st->status = ST_DONE;
            } else if (!(rt == rt)) {
                st->status = ST_BREAKDOWN;
            } else {
                st->status = ST_REFINE;
                st->refinements += 1;
            }
        }
    }
}

// ------------------------------------------------------- coarse (rare)
// t = C^T u (u = b when src_b, else r), optionally bb = (u, u), as
// per-workgroup partials.  Used for x0 (u = b) and for the re-projection
// after a true-residual replacement (u = r).
template <typename V, typename W>
__device__ __forceinline__ void coarse_dot_body(const SysView<V, W>& v, int64_t bid, int src_b, uint32_t mask) {
    DevState* st = v.st;
    if (!gate(st, mask)) return;
    __shared__ double red[kTpb];
    __shared__ double wpart[4 * 1024];
    const int nc = v.nc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int stride = nc + 1;
    const int64_t nblk = v.geo.gd;
    double* myp = v.partials + bid * stride;
    // each thread accumulates over its rows, then waves reduce per column,
    // 16 columns per pass over the rows
    double bbp = 0.0;
    for (int c0 = 0; c0 < nc || c0 == 0; c0 += 16) {
        double acc[16];
        const int cn = (nc - c0) < 16 ? (nc - c0) : 16;
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = 0.0;
        for (int64_t i = bid * blockDim.x + threadIdx.x; i < v.n; i += nblk * blockDim.x) {
            const double u = src_b ? v.b[i] : (double)v.r[i];
            if (c0 == 0) bbp += u * u;
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k < cn) acc[k] += (double)v.C[(int64_t)(c0 + k) * v.ldc + i] * u;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k < cn) {
                const double t = wave_sum(acc[k]);
                if (lane == 0) wpart[wave * 1024 + c0 + k] = t;
            }
        }
        if (nc == 0) break;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wpart[w * 1024 + c];
        myp[1 + c] = t;
    }
    const double bsum = block_sum(bbp, red);
    if (threadIdx.x == 0) myp[0] = bsum;
}

// One workgroup: t and (u, u) from the partials of coarse_dot; mu = Ginv t.
template <typename V, typename W>
__device__ __forceinline__ void finalize_dot_body(const SysView<V, W>& v, int with_bb, uint32_t mask) {
    DevState* st = v.st;
    if (!gate(st, mask)) return;
    __shared__ double red[1024];
    __shared__ double fin[1024 + 4];
    const int nc = v.nc;
    const int stride = nc + 1;
    reduce_partials<8>(v.partials, v.geo.gd, stride, stride, fin, red);
    __syncthreads();
    if (threadIdx.x == 0 && with_bb) st->bb = fin[0];
    if (nc > 0) ginv_matvec(v.Ginv, nc, fin + 1, v.mu, red);
}

// x = (from_b ? 0 : x) + C mu;  r = (from_b ? b : r) - AC mu
template <typename V, typename W>
__device__ __forceinline__ void coarse_correct_body(const SysView<V, W>& v, int64_t bid, int from_b, uint32_t mask) {
    DevState* st = v.st;
    if (!gate(st, mask)) return;
    __shared__ double mu[1024];
    const int nc = v.nc;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) mu[c] = v.mu[c];
    __syncthreads();
    const int64_t i = bid * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    double xi = from_b ? 0.0 : v.x[i];
    double ri = from_b ? v.b[i] : (double)v.r[i];
    const V* ACi = v.AC + i * v.ldac;
    for (int c = 0; c < nc; ++c) {
        xi += (double)v.C[(int64_t)c * v.ldc + i] * mu[c];
        ri -= (double)ACi[c] * mu[c];
    }
    v.x[i] = xi;
    v.r[i] = (W)ri;
}

// ------------------------------------------- single-system entry points
template <typename V, typename W, int B, int VAR>
__global__ __launch_bounds__(256) void k_spmv_dot(SysView<V, W> v) {
    spmv_dot_body<V, W, B, VAR>(v, blockIdx.x);
}
template <typename V, typename W, int B>
__global__ __launch_bounds__(kT3, 2) void k_update_reduce(SysView<V, W> v, int mode) {
    __shared__ double pool[upd_pool<B>()];
    update_reduce_body<V, W, B, false, kUrOne, true>(v, blockIdx.x, mode, pool);
}
template <typename V, typename W, int B, bool NTS>
__global__ __launch_bounds__(kT3, 2) void k_update_fused(SysView<V, W> v, int mode) {
    __shared__ double pool[upd_pool<B>() > fin_pool() ? upd_pool<B>() : fin_pool()];
    update_reduce_body<V, W, B, true, kUrOne, true, NTS>(v, blockIdx.x, mode, pool);
}
template <typename V, typename W>
__global__ __launch_bounds__(kTF3) void k_finalize_update(SysView<V, W> v, int mode) {
    __shared__ double pool[fin_pool()];
    finalize_update_body<V, W, false>(v, mode, pool);
}
template <typename V, typename W, bool NTS>
__global__ __launch_bounds__(256) void k_correct_dir(SysView<V, W> v, int first) {
    correct_dir_body<V, W, 8, NTS>(v, blockIdx.x, first);
}
template <typename V, typename W, int B>
__global__ __launch_bounds__(256) void k_true_resid(SysView<V, W> v, int final_only) {
    true_resid_body<V, W, B>(v, blockIdx.x, final_only);
}
template <typename V, typename W>
__global__ __launch_bounds__(1024) void k_finalize_resid(SysView<V, W> v, int final_only) {
    finalize_resid_body<V, W>(v, final_only);
}
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_coarse_dot(SysView<V, W> v, int src_b, uint32_t mask) {
    coarse_dot_body<V, W>(v, blockIdx.x, src_b, mask);
}
template <typename V, typename W>
__global__ __launch_bounds__(1024) void k_finalize_dot(SysView<V, W> v, int with_bb, uint32_t mask) {
    finalize_dot_body<V, W>(v, with_bb, mask);
}
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_coarse_correct(SysView<V, W> v, int from_b, uint32_t mask) {
    coarse_correct_body<V, W>(v, blockIdx.x, from_b, mask);
}

// ----------------------------------------------- fused multi-system launches
// One launch covers the workgroups of every system of a batch: map[blockIdx.x]
// = (system, workgroup index within that system's own grid), so each
// system runs exactly the workgroups (and reductions) of its single launch.
template <typename V, typename W, int B>
__global__ __launch_bounds__(256) void kb_spmv_dot(const SysView<V, W>* __restrict__ views,
                                                   const int2* __restrict__ map) {
    const int2 e = map[blockIdx.x];
    spmv_dot_body<V, W, B>(views[e.x], e.y);
}
// (__launch_bounds__' second argument: waves per SIMD, 4 = two workgroups
// per compute unit within 128 registers; the 3x3-block body needs more and
// runs one workgroup per compute unit.)
template <typename V, typename W, int B>
__global__ __launch_bounds__(kT3, B == 3 ? 2 : 4) void kb_update_reduce(const SysView<V, W>* __restrict__ views,
                                                        const int2* __restrict__ map, int mode) {
    __shared__ double pool[upd_pool<B>()];
    const int2 e = map[blockIdx.x];
    update_reduce_body<V, W, B, false, kUrBatch>(views[e.x], e.y, mode, pool);
}
template <typename V, typename W, int B>
__global__ __launch_bounds__(kT3, B == 3 ? 2 : 4) void kb_update_fused(const SysView<V, W>* __restrict__ views,
                                                       const int2* __restrict__ map, int mode) {
    __shared__ double pool[upd_pool<B>() > fin_pool() ? upd_pool<B>() : fin_pool()];
    const int2 e = map[blockIdx.x];
    update_reduce_body<V, W, B, true, kUrBatch>(views[e.x], e.y, mode, pool);
}
template <typename V, typename W>
__global__ __launch_bounds__(kTF3) void kb_finalize_update(const SysView<V, W>* __restrict__ views,
                                                           const int2* __restrict__ map, int mode) {
    __shared__ double pool[fin_pool()];
    finalize_update_body<V, W, false>(views[map[blockIdx.x].x], mode, pool);
}
template <typename V, typename W>
__global__ __launch_bounds__(256) void kb_correct_dir(const SysView<V, W>* __restrict__ views,
                                                      const int2* __restrict__ map, int first) {
    const int2 e = map[blockIdx.x];
    correct_dir_body<V, W, 8>(views[e.x], e.y, first);
}
// The direction update of the members with at most kDirFewCols basis
// columns: z = s - C mu and w = s - C mu2 + beta w_old, without the general
// kernel's LDS stage.  With so few columns the general kernel gives each
// column to its own wave and adds the four waves' products in LDS in the
// order ((c0 + c1) + c2) + c3 (missing columns as zeros); the same products
// and the same order are formed here per row in registers, so the bits are
// the same.  NC = 0 serves the members without a basis (no column loads,
// fewer registers), NC = kDirFewCols the others.  A workgroup takes
// kDirFewGroup consecutive ranges b of that
// kernel's grid (blocks b, b + g5, ...) with every load of a round issued
// before any store: with thousands of small systems the per-workgroup
// latency, not the bytes, set the time of the general kernel.
template <typename V, typename W, int NC, bool NTS = false>
__device__ __forceinline__ void correct_dir_few_body(const SysView<V, W>& v, int64_t b0, int first) {
    constexpr int G = kDirFewGroup;
    static_assert(NC == 0 || NC == 4, "the general kernel's four waves hold one column each");
    constexpr int NA = NC > 0 ? NC : 1;
    const DevState* st = v.st;
    if (!gate(st, M_RUN)) return;
    if (first == 2 && st->pending_dir == 0) return;
    const int nc = v.nc;
    double m1[NA], m2[NA];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        m1[k] = (k < nc) ? v.mu[k] : 0.0;
        m2[k] = (k < nc) ? ((first == 1) ? v.mu[k] : v.mu2[k]) : 0.0;
    }
    const double beta = (first == 1) ? 0.0 : st->beta;
    const int j = st->iter;
    const int hist_cap = st->hist_cap;
    const bool tm = first == 0 && ktime_sample(st, 2);
    const int tid = threadIdx.x;
    const int64_t nblk = (v.n + 255) / 256;
    const int64_t g5 = v.geo.g5;
    const int nb = (int)((b0 + G) < g5 ? G : g5 - b0);
    for (int u = 0; u < nb; ++u) ktime_begin(v.kslots, 2, b0 + u, tm);
    for (int64_t r0 = 0; r0 + b0 < nblk; r0 += g5) {
        int64_t row[G];
        W sv[G], wv0[G];
        V cv[G][NA];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int64_t blk = r0 + b0 + u;
            row[u] = (u < nb && blk < nblk) ? blk * 256 + tid : v.n;
            sv[u] = 0;
            wv0[u] = 0;
#pragma unroll
            for (int k = 0; k < NA; ++k) cv[u][k] = 0;
            if (row[u] < v.n) {
                sv[u] = v.s[row[u]];
                if (first != 1) wv0[u] = v.w[row[u]];
#pragma unroll
                for (int k = 0; k < NC; ++k)
                    if (k < nc) cv[u][k] = v.C[(int64_t)k * v.ldc + row[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int64_t i = row[u];
            if (i < v.n) {
                double az[4] = {0.0, 0.0, 0.0, 0.0}, aw[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    if (k < nc) {
                        az[k] += (double)cv[u][k] * m1[k];
                        aw[k] += (double)cv[u][k] * m2[k];
                    }
                }
                const double cz = ((az[0] + az[1]) + az[2]) + az[3];
                const double cw = ((aw[0] + aw[1]) + aw[2]) + aw[3];
                const double s = (double)sv[u];
                const W zv = (W)(s - cz);
                const W wv = (first == 1) ? zv : (W)(s - cw + beta * (double)wv0[u]);
                st_vec<NTS>(v.w + i, wv);
                if (j < hist_cap) {
                    if (v.zhist) st_vec<NTS>(v.zhist + (int64_t)j * v.ldh + i, (V)zv);
                    if (v.zhist32) st_vec<NTS>(v.zhist32 + (int64_t)j * v.ldh + i, (float)zv);
                    if (v.whist) st_vec<NTS>(v.whist + (int64_t)j * v.ldh + i, (V)wv);
                }
            }
        }
    }
    for (int u = 0; u < nb; ++u) ktime_end(v.kslots, 2, b0 + u, tm);
}
template <typename V, typename W, int NC>
__global__ __launch_bounds__(256) void kb_correct_dir_few(const SysView<V, W>* __restrict__ views,
                                                          const int2* __restrict__ map, int first) {
    const int2 e = map[blockIdx.x];
    correct_dir_few_body<V, W, NC>(views[e.x], e.y, first);
}
// the same for one system (kDirFewGroup ranges per workgroup)
template <typename V, typename W, int NC, bool NTS>
__global__ __launch_bounds__(256) void k_correct_dir_few(SysView<V, W> v, int first) {
    correct_dir_few_body<V, W, NC, NTS>(v, (int64_t)blockIdx.x * kDirFewGroup, first);
}
template <typename V, typename W, int B>
__global__ __launch_bounds__(256) void kb_true_resid(const SysView<V, W>* __restrict__ views,
                                                     const int2* __restrict__ map, int final_only) {
    const int2 e = map[blockIdx.x];
    true_resid_body<V, W, B>(views[e.x], e.y, final_only);
}
template <typename V, typename W>
__global__ __launch_bounds__(1024) void kb_finalize_resid(const SysView<V, W>* __restrict__ views,
                                                          const int2* __restrict__ map, int final_only) {
    finalize_resid_body<V, W>(views[map[blockIdx.x].x], final_only);
}
template <typename V, typename W>
__global__ __launch_bounds__(256) void kb_coarse_dot(const SysView<V, W>* __restrict__ views,
                                                     const int2* __restrict__ map, int src_b, uint32_t mask) {
    const int2 e = map[blockIdx.x];
    coarse_dot_body<V, W>(views[e.x], e.y, src_b, mask);
}
template <typename V, typename W>
__global__ __launch_bounds__(1024) void kb_finalize_dot(const SysView<V, W>* __restrict__ views,
                                                        const int2* __restrict__ map, int with_bb, uint32_t mask) {
    finalize_dot_body<V, W>(views[map[blockIdx.x].x], with_bb, mask);
}
template <typename V, typename W>
__global__ __launch_bounds__(256) void kb_coarse_correct(const SysView<V, W>* __restrict__ views,
                                                         const int2* __restrict__ map, int from_b, uint32_t mask) {
    const int2 e = map[blockIdx.x];
    coarse_correct_body<V, W>(views[e.x], e.y, from_b, mask);
}
// status word and iteration count of every system of the batch
template <typename V, typename W>
__global__ void kb_status(const SysView<V, W>* __restrict__ views, int count, int32_t* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    out[2 * i] = views[i].st->status;
    out[2 * i + 1] = views[i].st->iter;
}

// ------------------------------------------------------------ rebuild
// AC64 = A C (double values), row-major n x nc with leading dimension
// ldac >= nc; ACv = AC64 in V.  blockIdx.y selects 8 columns; the pad
// columns nc..ldac-1 are written as zeros by the blockIdx.y == 0 workgroups.
template <typename V, typename W, int B>
__global__ __launch_bounds__(256) void k_spmm(SysView<V, W> v, const V* C, int64_t ldc, int nc, int64_t ldac,
                                              double* AC64, V* ACv) {
    constexpr int CW = 8;
    const int c0 = blockIdx.y * CW;
    const int cn = (nc - c0) < CW ? (nc - c0) : CW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int npad = (blockIdx.y == 0) ? (int)(ldac - nc) : 0;
    if (B == 1) {
        for (int64_t sl = (int64_t)blockIdx.x * 4 + wave; sl < v.nslices; sl += (int64_t)gridDim.x * 4) {
            const int64_t k0 = v.slice_ptr[sl], k1 = v.slice_ptr[sl + 1];
            double acc[CW];
#pragma unroll
            for (int j = 0; j < CW; ++j) acc[j] = 0.0;
            for (int64_t k = k0; k < k1; ++k) {
                const int64_t e = k * 64 + lane;
                const double a = v.val64[e];
                const int64_t col = v.col[e];
#pragma unroll
                for (int j = 0; j < CW; ++j)
                    if (j < cn) acc[j] += a * (double)C[(int64_t)(c0 + j) * ldc + col];
            }
            const int64_t row = sl * 64 + lane;
            if (row < v.n) {
#pragma unroll
                for (int j = 0; j < CW; ++j)
                    if (j < cn) {
                        AC64[row * ldac + c0 + j] = acc[j];
                        ACv[row * ldac + c0 + j] = (V)acc[j];
                    }
                for (int j = 0; j < npad; ++j) {
                    AC64[row * ldac + nc + j] = 0.0;
                    ACv[row * ldac + nc + j] = (V)0;
                }
            }
        }
    } else {
        const int d = wave;
        for (int64_t sl = blockIdx.x; sl < v.nslices; sl += gridDim.x) {
            const int64_t k0 = v.slice_ptr[sl], k1 = v.slice_ptr[sl + 1];
            double acc[CW];
#pragma unroll
            for (int j = 0; j < CW; ++j) acc[j] = 0.0;
            for (int64_t k = k0; k < k1; ++k) {
                const int64_t e = k * 64 + lane;
                const int64_t col = 3 * (int64_t)v.col[e];
                const double* vb = v.val64 + (k * 9 + 3 * d) * 64 + lane;
                const double a0 = vb[0], a1 = vb[64], a2 = vb[128];
#pragma unroll
                for (int j = 0; j < CW; ++j)
                    if (j < cn) {
                        const V* Cc = C + (int64_t)(c0 + j) * ldc + col;
                        acc[j] += a0 * (double)Cc[0] + a1 * (double)Cc[1] + a2 * (double)Cc[2];
                    }
            }
            const int64_t p = sl * 64 + lane;
            if (p < v.nb) {
                const int64_t row = 3 * p + d;
#pragma unroll
                for (int j = 0; j < CW; ++j)
                    if (j < cn) {
                        AC64[row * ldac + c0 + j] = acc[j];
                        ACv[row * ldac + c0 + j] = (V)acc[j];
                    }
                for (int j = 0; j < npad; ++j) {
                    AC64[row * ldac + nc + j] = 0.0;
                    ACv[row * ldac + nc + j] = (V)0;
                }
            }
        }
    }
}

// G = C^T AC64: 16x16 output tiles (blockIdx.y), row ranges (blockIdx.x)
// into partials[blockIdx.x][nc*nc]; k_gram_reduce sums them in order.
template <typename V>
__global__ __launch_bounds__(256) void k_gram_partial(const V* C, int64_t ldc, const double* AC64, int64_t ldac,
                                                      int64_t n, int nc, double* partials) {
    const int ntc = (nc + 15) / 16;
    const int ta = blockIdx.y / ntc, tb = blockIdx.y % ntc;
    const int a = threadIdx.x / 16, bcol = threadIdx.x % 16;
    __shared__ double sC[16][17];
    __shared__ double sA[16][17];
    const int64_t rows_per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per;
    const int64_t r1 = (r0 + rows_per) < n ? (r0 + rows_per) : n;
    double acc = 0.0;
    for (int64_t base = r0; base < r1; base += 16) {
        // load 16 rows x 16 columns of C (cols ta*16..) and AC (cols tb*16..)
        {
            const int rr = threadIdx.x / 16, cc = threadIdx.x % 16;
            const int64_t i = base + rr;
            const int ca = ta * 16 + cc, cb = tb * 16 + cc;
            sC[rr][cc] = (i < r1 && ca < nc) ? (double)C[(int64_t)ca * ldc + i] : 0.0;
            sA[rr][cc] = (i < r1 && cb < nc) ? AC64[i * ldac + cb] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) acc += sC[k][a] * sA[k][bcol];
        __syncthreads();
    }
    const int ga = ta * 16 + a, gb = tb * 16 + bcol;
    if (ga < nc && gb < nc) partials[(int64_t)blockIdx.x * nc * nc + (int64_t)gb * nc + ga] = acc;
}

__global__ void k_gram_reduce(const double* partials, int np, int nc, double* G) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nn = (int64_t)nc * nc;
    if (idx >= nn) return;
    double t = 0.0;
    for (int p = 0; p < np; ++p) t += partials[(int64_t)p * nn + idx];
    G[idx] = t;
}

// out[:, t] = sum_j Z[:, j] F[j, t]  (F column-major m x s, double)
template <typename V, typename ZT = V>
__global__ __launch_bounds__(256) void k_basis_combine(const ZT* Z, int64_t ldz, int m, const double* F, int s, V* out,
                                                       int64_t ldo, int64_t n) {
    constexpr int CW = 8;
    const int t0 = blockIdx.y * CW;
    const int tn = (s - t0) < CW ? (s - t0) : CW;
    __shared__ double sF[256][CW];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[CW];
#pragma unroll
    for (int k = 0; k < CW; ++k) acc[k] = 0.0;
    for (int j0 = 0; j0 < m; j0 += 256) {
        __syncthreads();
        const int jj = j0 + threadIdx.x;
#pragma unroll
        for (int k = 0; k < CW; ++k) sF[threadIdx.x][k] = (jj < m && k < tn) ? F[(int64_t)(t0 + k) * m + jj] : 0.0;
        __syncthreads();
        const int jn = (m - j0) < 256 ? (m - j0) : 256;
        if (i < n) {
            for (int j = 0; j < jn; ++j) {
                const double z = (double)Z[(int64_t)(j0 + j) * ldz + i];
#pragma unroll
                for (int k = 0; k < CW; ++k) acc[k] += z * sF[j][k];
            }
        }
    }
    if (i < n) {
#pragma unroll
        for (int k = 0; k < CW; ++k)
            if (k < tn) out[(int64_t)(t0 + k) * ldo + i] = (V)acc[k];
    }
}

// out[:, t] = sum_j Z[:, j] F[j, t] for single-precision Z and out, on the
// matrix cores (v_mfma_f32_32x32x2f32): a wave owns 32 rows and CT tiles of
// 32 columns, accumulating over j two at a time (ascending); a workgroup
// (4 waves) owns 128 rows.  Both operands go through LDS in chunks of KC
// values of j, double-buffered: while the waves multiply one chunk, the
// next one is loaded into registers (Z in 16-byte row segments, F as double
// and rounded to float) and stored to the other buffer.
// Operand layout of the instruction: lane l supplies A[l % 32][l / 32] and
// B[l / 32][l % 32]; accumulator register r of lane l holds
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
// Bounds: rows up to the next multiple of 128 lie within the leading
// dimension (a multiple of 256, at least n); indices of j past m are clamped
// to m - 1 and their F rows staged as zero.
typedef float mfma_f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int CT>
__global__ __launch_bounds__(256) void k_basis_combine_mfma(const float* __restrict__ Z, int64_t ldz, int m,
                                                            const double* __restrict__ F, int s,
                                                            float* __restrict__ out, int64_t ldo, int64_t n) {
    constexpr int KC = 32;
    constexpr int NC = CT * 32;
    constexpr int FPT = KC * NC / 256;  // F values staged per thread and chunk
    __shared__ float sZ[2][KC][128];
    __shared__ float sF[2][KC][NC];
    const int c0 = blockIdx.y * NC;
    const int ncol = (s - c0) < NC ? (s - c0) : NC;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t rowb = (int64_t)blockIdx.x * 128;
    const int khalf = lane >> 5;
    // staging roles: Z element (j = zj + 8 i, rows zr .. zr + 3); F element
    // (j = fj, column fc + 8 i)
    const int zj = tid >> 5, zr = (tid & 31) * 4;
    const int fj = tid & 31, fc = tid >> 5;
    f32x4 zreg[4];
    float freg[FPT];
    mfma_f32x16 acc[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
    const int nchunk = (m + KC - 1) / KC;
    for (int q = 0; q <= nchunk; ++q) {
        // load chunk q (into registers), multiply chunk q - 1 (from LDS),
        // store chunk q to the other buffer
        const int buf = q & 1;
        if (q < nchunk) {
            const int k0 = q * KC;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int kx = k0 + zj + 8 * i;
                kx = kx < m ? kx : m - 1;
                zreg[i] = *reinterpret_cast<const f32x4*>(Z + (int64_t)kx * ldz + rowb + zr);
            }
            const int kx = k0 + fj;
#pragma unroll
            for (int i = 0; i < FPT; ++i) {
                const int cc = fc + 8 * i;
                freg[i] = (kx < m && cc < ncol) ? (float)F[(int64_t)(c0 + cc) * m + kx] : 0.f;
            }
        }
        if (q > 0) {
            const int pb = buf ^ 1;
#pragma unroll
            for (int kk = 0; kk < KC; kk += 2) {
                const float a = sZ[pb][kk + khalf][wave * 32 + (lane & 31)];
#pragma unroll
                for (int t = 0; t < CT; ++t) {
                    const float b = sF[pb][kk + khalf][t * 32 + (lane & 31)];
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[t], 0, 0, 0);
                }
            }
        }
        if (q < nchunk) {
#pragma unroll
            for (int i = 0; i < 4; ++i) *reinterpret_cast<f32x4*>(&sZ[buf][zj + 8 * i][zr]) = zreg[i];
#pragma unroll
            for (int i = 0; i < FPT; ++i) sF[buf][fj][fc + 8 * i] = freg[i];
        }
        __syncthreads();
    }
    const int64_t row0 = rowb + wave * 32;
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        const int col = t * 32 + (lane & 31);
        if (col >= ncol) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t row = row0 + 8 * (r >> 2) + 4 * khalf + (r & 3);
            if (row < n) out[(int64_t)(c0 + col) * ldo + row] = acc[t][r];
        }
    }
}

template <typename V>
__global__ void k_scale_columns(V* C, int64_t ldc, int64_t n, const double* scale, int k) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n || c >= k) return;
    C[(int64_t)c * ldc + i] = (V)((double)C[(int64_t)c * ldc + i] * scale[c]);
}

// dst[:, t] = src[:, map[t]] (map ascending and map[t] >= t when src == dst)
template <typename V>
__global__ void k_copy_columns(const V* src, int64_t lds, V* dst, int64_t ldd, int64_t n, const int32_t* map, int k) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int t = 0; t < k; ++t) dst[(int64_t)t * ldd + i] = src[(int64_t)map[t] * lds + i];
}

// values in pattern order -> sliced ELL (double and V copies)
template <typename V, int B>
__global__ void k_scatter_values(const double* in, const int64_t* map, int64_t nnzb, double* val64, V* valV) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnzb) return;
    const int64_t E = map[t];
    if (B == 1) {
        const double a = in[t];
        val64[E] = a;
        if (valV) valV[E] = (V)a;
    } else {
        const int64_t slot = E >> 6, l = E & 63;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            const double a = in[t * 9 + e];
            const int64_t pos = (slot * 9 + e) * 64 + l;
            val64[pos] = a;
            if (valV) valV[pos] = (V)a;
        }
    }
}

// M^-1 from the diagonal (blocks) of the input values.  bad[0] != 0 when a
// pivot is not positive (M not SPD).
template <typename V, int B>
__global__ void k_precond_setup(const double* in, const int64_t* diag_idx, int64_t nb, V* minv, int32_t* bad) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nb) return;
    const int64_t t = diag_idx[p];
    if (B == 1) {
        const double a = in[t];
        if (!(a > 0.0)) atomicOr(bad, 1);
        minv[p] = (V)(1.0 / a);
    } else {
        const double* m = in + t * 9;
        const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5], g = m[6], h = m[7], k = m[8];
        const double A = e * k - f * h, Bc = -(d * k - f * g), Cc = d * h - e * g;
        const double det = a * A + b * Bc + c * Cc;
        const double m2 = a * e - b * d;
        if (!(a > 0.0) || !(m2 > 0.0) || !(det > 0.0)) atomicOr(bad, 1);
        const double id = 1.0 / det;
        // three planes of n = 3 nb entries: plane c holds column c of each
        // block row, so that entry (3 p + r, c) sits at c n + 3 p + r and a
        // lane per unknown reads its row with three contiguous loads
        const int64_t n = 3 * nb, o = 3 * p;
        minv[o] = (V)(A * id);
        minv[n + o] = (V)(-(b * k - c * h) * id);
        minv[2 * n + o] = (V)((b * f - c * e) * id);
        minv[o + 1] = (V)(Bc * id);
        minv[n + o + 1] = (V)((a * k - c * g) * id);
        minv[2 * n + o + 1] = (V)(-(a * f - c * d) * id);
        minv[o + 2] = (V)(Cc * id);
        minv[n + o + 2] = (V)(-(a * h - b * g) * id);
        minv[2 * n + o + 2] = (V)((a * e - b * d) * id);
    }
}

template <typename V>
__global__ void k_d2v(const double* in, V* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (V)in[i];
}

template <typename V>
__global__ void k_v2d(const V* in, double* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------ launchers

// ------------------------------------------------------------ geometry

Geometry make_geometry(int64_t n, int64_t nslices, int block, int64_t cb3_req, int spmv_grid) {
    Geometry g{};
    const int64_t nb = n / block;
    const int64_t per = (block == 1) ? 4 : 2;  // slices per workgroup step (one per wave)
    int64_t g1 = (nslices + per - 1) / per;
    // at most kPart1 workgroups: each writes its (w, A w) partial there
    const int64_t cap1 = spmv_grid > 0 ? std::min<int64_t>(spmv_grid, kPart1) : kPart1;
    g.g1 = (int32_t)std::min<int64_t>(std::max<int64_t>(g1, 1), cap1);
    // K3: contiguous ranges of cb3 block rows; by default one range per CU
    int64_t cb = cb3_req > 0 ? cb3_req : (nb + 255) / 256;
    if (cb < 64) cb = 64;
    if ((nb + cb - 1) / cb > kMaxUpdateGrid) cb = (nb + kMaxUpdateGrid - 1) / kMaxUpdateGrid;
    g.cb3 = cb;
    g.g3 = (int32_t)std::max<int64_t>((nb + cb - 1) / cb, 1);
    g.g5 = (int32_t)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), kMaxTimedGrid);
    g.gd = (int32_t)std::min<int64_t>(std::max<int64_t>((n + kTpb - 1) / kTpb, 1), 256);
    g.gcc = (int32_t)std::max<int64_t>((n + 255) / 256, 1);
    return g;
}

int64_t partial_doubles(const Geometry& g, int nc) {
    const int64_t c = std::max(nc, 1);
    const int64_t ng = (g.g3 + kGroup - 1) / kGroup;
    return std::max<int64_t>({(int64_t)(g.g3 + ng) * (2 * c + 2), (int64_t)g.g1 + 8, (int64_t)g.gd * (c + 1), 1024});
}

// ----------------------------------------------------- single-system launches

template <typename V, typename W, int B>
void launch_spmv_dot(const SysView<V, W>& v, hipStream_t stream) {
    const int threads = (B == 1) ? 256 : 128;
    const dim3 grid((unsigned)v.geo.g1);
    // 16-bit relative block columns (set with the default load schedule, 0 or 2);
    // non-temporal stores of q (bit 3) only with the non-temporal loads
    const int c16 = (B == 3 && v.op64 && v.col16 && (v.spmv_var & 1) == 0) ? 4 : 0;
    const int nts = (B == 3 && v.op64 && v.nt_store && (v.spmv_var & 2)) ? 8 : 0;
    switch ((B == 3 && v.op64) ? (v.spmv_var & 3) | c16 | nts : 0) {
        case 4: hipLaunchKernelGGL((k_spmv_dot<V, W, B, 4>), grid, dim3(threads), 0, stream, v); break;
        case 6: hipLaunchKernelGGL((k_spmv_dot<V, W, B, 6>), grid, dim3(threads), 0, stream, v); break;
        case 14: hipLaunchKernelGGL((k_spmv_dot<V, W, B, 14>), grid, dim3(threads), 0, stream, v); break;
        case 10: hipLaunchKernelGGL((k_spmv_dot<V, W, B, 10>), grid, dim3(threads), 0, stream, v); break;
        case 11: hipLaunchKernelGGL((k_spmv_dot<V, W, B, 11>), grid, dim3(threads), 0, stream, v); break;
        case 1: hipLaunchKernelGGL((k_spmv_dot<V, W, B, 1>), grid, dim3(threads), 0, stream, v); break;
        case 2: hipLaunchKernelGGL((k_spmv_dot<V, W, B, 2>), grid, dim3(threads), 0, stream, v); break;
        case 3: hipLaunchKernelGGL((k_spmv_dot<V, W, B, 3>), grid, dim3(threads), 0, stream, v); break;
        default: hipLaunchKernelGGL((k_spmv_dot<V, W, B, 0>), grid, dim3(threads), 0, stream, v); break;
    }
}

template <typename V, typename W, int B>
void launch_update_only(const SysView<V, W>& v, int mode, hipStream_t stream) {
    hipLaunchKernelGGL((k_update_reduce<V, W, B>), dim3((unsigned)v.geo.g3), dim3(kT3), 0, stream, v, mode);
}

template <typename V, typename W, int B>
void launch_update_reduce(const SysView<V, W>& v, int mode, hipStream_t stream) {
    if (v.fused) {
        if (v.nt_store)
            hipLaunchKernelGGL((k_update_fused<V, W, B, true>), dim3((unsigned)v.geo.g3), dim3(kT3), 0, stream, v, mode);
        else
            hipLaunchKernelGGL((k_update_fused<V, W, B, false>), dim3((unsigned)v.geo.g3), dim3(kT3), 0, stream, v,
                               mode);
        return;
    }
    hipLaunchKernelGGL((k_update_reduce<V, W, B>), dim3((unsigned)v.geo.g3), dim3(kT3), 0, stream, v, mode);
    hipLaunchKernelGGL((k_finalize_update<V, W>), dim3(1), dim3(kTF3), 0, stream, v, mode);
}

template <typename V, typename W>
void launch_correct_dir(const SysView<V, W>& v, int first, hipStream_t stream) {
    // up to kDirFewCols columns (and no copy of z for the reorthogonalisation):
    // the per-row kernel, same products in the same order
    if (!v.zr && v.nc <= kDirFewCols) {
        const dim3 grid((unsigned)((v.geo.g5 + kDirFewGroup - 1) / kDirFewGroup));
        const int k = (v.nc == 0 ? 0 : 1) | (v.nt_store ? 2 : 0);
        if (k == 0) hipLaunchKernelGGL((k_correct_dir_few<V, W, 0, false>), grid, dim3(256), 0, stream, v, first);
        if (k == 1)
            hipLaunchKernelGGL((k_correct_dir_few<V, W, kDirFewCols, false>), grid, dim3(256), 0, stream, v, first);
        if (k == 2) hipLaunchKernelGGL((k_correct_dir_few<V, W, 0, true>), grid, dim3(256), 0, stream, v, first);
        if (k == 3)
            hipLaunchKernelGGL((k_correct_dir_few<V, W, kDirFewCols, true>), grid, dim3(256), 0, stream, v, first);
        return;
    }
    const dim3 grid((unsigned)v.geo.g5);
    if (v.nt_store) hipLaunchKernelGGL((k_correct_dir<V, W, true>), grid, dim3(256), 0, stream, v, first);
    else hipLaunchKernelGGL((k_correct_dir<V, W, false>), grid, dim3(256), 0, stream, v, first);
}

template <typename V, typename W, int B>
void launch_true_resid(const SysView<V, W>& v, int final_only, hipStream_t stream) {
    const int threads = (B == 1) ? 256 : 128;
    hipLaunchKernelGGL((k_true_resid<V, W, B>), dim3((unsigned)v.geo.g1), dim3(threads), 0, stream, v, final_only);
    hipLaunchKernelGGL((k_finalize_resid<V, W>), dim3(1), dim3(1024), 0, stream, v, final_only);
}

template <typename V, typename W>
void launch_coarse_dot(const SysView<V, W>& v, int src_b, int with_bb, uint32_t mask, hipStream_t stream) {
    hipLaunchKernelGGL((k_coarse_dot<V, W>), dim3((unsigned)v.geo.gd), dim3(256), 0, stream, v, src_b, mask);
    hipLaunchKernelGGL((k_finalize_dot<V, W>), dim3(1), dim3(1024), 0, stream, v, with_bb, mask);
}

template <typename V, typename W>
void launch_coarse_correct(const SysView<V, W>& v, int from_b, uint32_t mask, hipStream_t stream) {
    hipLaunchKernelGGL((k_coarse_correct<V, W>), dim3((unsigned)v.geo.gcc), dim3(256), 0, stream, v, from_b, mask);
}

// ------------------------------------------------------ fused batch launches

template <typename V, typename W, int B>
void batch_spmv_dot(const SysView<V, W>* views, const BatchMaps& m, hipStream_t stream) {
    if (m.count[BK_SPMV] <= 0) return;
    const int threads = (B == 1) ? 256 : 128;
    hipLaunchKernelGGL((kb_spmv_dot<V, W, B>), dim3((unsigned)m.count[BK_SPMV]), dim3(threads), 0, stream, views,
                       m.map[BK_SPMV]);
}

template <typename V, typename W, int B>
void batch_update_reduce(const SysView<V, W>* views, const BatchMaps& m, int mode, hipStream_t stream) {
    if (m.fused) {
        if (m.count[BK_UPD] > 0)
            hipLaunchKernelGGL((kb_update_fused<V, W, B>), dim3((unsigned)m.count[BK_UPD]), dim3(kT3), 0, stream,
                               views, m.map[BK_UPD], mode);
        return;
    }
    if (m.count[BK_UPD] > 0)
        hipLaunchKernelGGL((kb_update_reduce<V, W, B>), dim3((unsigned)m.count[BK_UPD]), dim3(kT3), 0, stream, views,
                           m.map[BK_UPD], mode);
    if (m.count[BK_ONE] > 0)
        hipLaunchKernelGGL((kb_finalize_update<V, W>), dim3((unsigned)m.count[BK_ONE]), dim3(kTF3), 0, stream, views,
                           m.map[BK_ONE], mode);
}

// the update kernel of every member alone (no end-of-step reduction): the
// batch autotuner times it in the initial mode
template <typename V, typename W, int B>
void batch_update_only(const SysView<V, W>* views, const BatchMaps& m, int mode, hipStream_t stream) {
    if (m.count[BK_UPD] > 0)
        hipLaunchKernelGGL((kb_update_reduce<V, W, B>), dim3((unsigned)m.count[BK_UPD]), dim3(kT3), 0, stream, views,
                           m.map[BK_UPD], mode);
}

template <typename V, typename W>
void batch_correct_dir(const SysView<V, W>* views, const BatchMaps& m, int first, hipStream_t stream) {
    if (m.count[BK_DIR] > 0)
        hipLaunchKernelGGL((kb_correct_dir<V, W>), dim3((unsigned)m.count[BK_DIR]), dim3(256), 0, stream, views,
                           m.map[BK_DIR], first);
    if (m.count[BK_DIR0] > 0)
        hipLaunchKernelGGL((kb_correct_dir_few<V, W, 0>), dim3((unsigned)m.count[BK_DIR0]), dim3(256), 0, stream,
                           views, m.map[BK_DIR0], first);
    if (m.count[BK_DIRF] > 0)
        hipLaunchKernelGGL((kb_correct_dir_few<V, W, kDirFewCols>), dim3((unsigned)m.count[BK_DIRF]), dim3(256), 0,
                           stream, views, m.map[BK_DIRF], first);
}

template <typename V, typename W, int B>
void batch_true_resid(const SysView<V, W>* views, const BatchMaps& m, int final_only, hipStream_t stream) {
    const int threads = (B == 1) ? 256 : 128;
    if (m.count[BK_SPMV] > 0)
        hipLaunchKernelGGL((kb_true_resid<V, W, B>), dim3((unsigned)m.count[BK_SPMV]), dim3(threads), 0, stream,
                           views, m.map[BK_SPMV], final_only);
    if (m.count[BK_ONE] > 0)
        hipLaunchKernelGGL((kb_finalize_resid<V, W>), dim3((unsigned)m.count[BK_ONE]), dim3(1024), 0, stream, views,
                           m.map[BK_ONE], final_only);
}

template <typename V, typename W>
void batch_coarse_dot(const SysView<V, W>* views, const BatchMaps& m, int src_b, int with_bb, uint32_t mask,
                      hipStream_t stream) {
    if (m.count[BK_DOT] > 0)
        hipLaunchKernelGGL((kb_coarse_dot<V, W>), dim3((unsigned)m.count[BK_DOT]), dim3(256), 0, stream, views,
                           m.map[BK_DOT], src_b, mask);
    if (m.count[BK_ONEC] > 0)
        hipLaunchKernelGGL((kb_finalize_dot<V, W>), dim3((unsigned)m.count[BK_ONEC]), dim3(1024), 0, stream, views,
                           m.map[BK_ONEC], with_bb, mask);
}

template <typename V, typename W>
void batch_coarse_correct(const SysView<V, W>* views, const BatchMaps& m, int from_b, uint32_t mask,
                          hipStream_t stream) {
    if (m.count[BK_CC] <= 0) return;
    hipLaunchKernelGGL((kb_coarse_correct<V, W>), dim3((unsigned)m.count[BK_CC]), dim3(256), 0, stream, views,
                       m.map[BK_CC], from_b, mask);
}

template <typename V, typename W>
void batch_status(const SysView<V, W>* views, int count, int32_t* out, hipStream_t stream) {
    if (count <= 0) return;
    hipLaunchKernelGGL((kb_status<V, W>), dim3(cdiv(count, 256)), dim3(256), 0, stream, views, count, out);
}

template <typename V, typename W, int B>
void launch_spmm(const SysView<V, W>& v, const V* C, int64_t ldc, int nc, int64_t ldac, double* AC64, V* ACv,
                 hipStream_t stream) {
    if (nc <= 0) return;
    const int threads = (B == 1) ? 256 : 192;
    dim3 grid((unsigned)v.geo.g1, (unsigned)((nc + 7) / 8));
    hipLaunchKernelGGL((k_spmm<V, W, B>), grid, dim3(threads), 0, stream, v, C, ldc, nc, ldac, AC64, ACv);
}

template <typename V>
void launch_gram(const V* C, int64_t ldc, const double* AC64, int64_t ldac, int64_t n, int nc, double* G,
                 double* partials, int64_t partial_cap, hipStream_t stream) {
    if (nc <= 0) return;
    const int64_t nn = (int64_t)nc * nc;
    int np = (int)(partial_cap / nn);
    if (np > 64) np = 64;
    if (np < 1) np = 1;
    const int ntc = (nc + 15) / 16;
    hipLaunchKernelGGL((k_gram_partial<V>), dim3((unsigned)np, (unsigned)(ntc * ntc)), dim3(256), 0, stream, C, ldc,
                       AC64, ldac, n, nc, partials);
    hipLaunchKernelGGL(k_gram_reduce, dim3(cdiv(nn, 256)), dim3(256), 0, stream, partials, np, nc, G);
}

template <typename V>
void launch_basis_combine(const V* Z, int64_t ldz, int m, const double* F, int s, V* out, int64_t ldo, int64_t n,
                          hipStream_t stream) {
    if (s <= 0 || m <= 0) return;
    if (std::is_same<V, float>::value) {
        const float* Zf = reinterpret_cast<const float*>(Z);
        float* of = reinterpret_cast<float*>(out);
        if (s <= 32)
            hipLaunchKernelGGL((k_basis_combine_mfma<1>), dim3(cdiv(n, 128), 1), dim3(256), 0, stream, Zf, ldz, m, F,
                               s, of, ldo, n);
        else if (s <= 64)
            hipLaunchKernelGGL((k_basis_combine_mfma<2>), dim3(cdiv(n, 128), 1), dim3(256), 0, stream, Zf, ldz, m, F,
                               s, of, ldo, n);
        else
            hipLaunchKernelGGL((k_basis_combine_mfma<4>), dim3(cdiv(n, 128), (unsigned)((s + 127) / 128)), dim3(256),
                               0, stream, Zf, ldz, m, F, s, of, ldo, n);
        return;
    }
    dim3 grid(cdiv(n, 256), (unsigned)((s + 7) / 8));
    hipLaunchKernelGGL((k_basis_combine<V>), grid, dim3(256), 0, stream, Z, ldz, m, F, s, out, ldo, n);
}

// a double-precision basis combined from a single-precision history
void launch_basis_combine_h32(const float* Z, int64_t ldz, int m, const double* F, int s, double* out, int64_t ldo,
                              int64_t n, hipStream_t stream) {
    if (s <= 0 || m <= 0) return;
    dim3 grid(cdiv(n, 256), (unsigned)((s + 7) / 8));
    hipLaunchKernelGGL((k_basis_combine<double, float>), grid, dim3(256), 0, stream, Z, ldz, m, F, s, out, ldo, n);
}

template <typename V>
void launch_scale_columns(V* C, int64_t ldc, int64_t n, const double* scale, int k, hipStream_t stream) {
    if (k <= 0) return;
    hipLaunchKernelGGL((k_scale_columns<V>), dim3(cdiv(n, 256), (unsigned)k), dim3(256), 0, stream, C, ldc, n, scale,
                       k);
}

template <typename V>
void launch_copy_columns(const V* src, int64_t lds, V* dst, int64_t ldd, int64_t n, const int32_t* map, int k,
                         hipStream_t stream) {
    if (k <= 0) return;
    hipLaunchKernelGGL((k_copy_columns<V>), dim3(cdiv(n, 256)), dim3(256), 0, stream, src, lds, dst, ldd, n, map, k);
}

template <typename V, int B>
void launch_scatter_values(const double* in, const int64_t* map, int64_t nnzb, double* val64, V* valV,
                           hipStream_t stream) {
    hipLaunchKernelGGL((k_scatter_values<V, B>), dim3(cdiv(nnzb, 256)), dim3(256), 0, stream, in, map, nnzb, val64,
                       valV);
}

template <typename V, int B>
void launch_precond_setup(const double* in, const int64_t* diag_idx, int64_t nb, V* minv, int32_t* bad,
                          hipStream_t stream) {
    hipLaunchKernelGGL((k_precond_setup<V, B>), dim3(cdiv(nb, 256)), dim3(256), 0, stream, in, diag_idx, nb, minv,
                       bad);
}

template <typename V>
void launch_d2v(const double* in, V* out, int64_t n, hipStream_t stream) {
    hipLaunchKernelGGL((k_d2v<V>), dim3(cdiv(n, 256)), dim3(256), 0, stream, in, out, n);
}

template <typename V, typename W>
void launch_reorth_store(const SysView<V, W>& v, hipStream_t stream) {
    const int g = (int)std::min<int64_t>(cdiv(v.n, 256), 2048);
    hipLaunchKernelGGL((k_reorth_store<V, W>), dim3(g), dim3(256), 0, stream, v);
}

template <typename V, typename W>
void launch_reorth(const SysView<V, W>& v, hipStream_t stream) {
    // row ranges x chunks of 256 kept directions (the ones past the
    // current count exit at once)
    hipLaunchKernelGGL((k_reorth_dot<V, W>), dim3((unsigned)(v.gr * ((v.rcap + 255) / 256))), dim3(256), 0, stream,
                       v);
    hipLaunchKernelGGL((k_reorth_reduce<V, W>), dim3(cdiv(kReorthMax, 256)), dim3(256), 0, stream, v);
    const int g = (int)std::min<int64_t>(cdiv(v.n, 16), 8192);
    hipLaunchKernelGGL((k_reorth_apply<V, W>), dim3(g), dim3(256), 0, stream, v);
}

template <typename V>
void launch_v2d(const V* in, double* out, int64_t n, hipStream_t stream) {
    hipLaunchKernelGGL((k_v2d<V>), dim3(cdiv(n, 256)), dim3(256), 0, stream, in, out, n);
}

#define KRS_INST_VWB(V, W, B)                                                                                    \
    template void launch_spmv_dot<V, W, B>(const SysView<V, W>&, hipStream_t);                                    \
    template void launch_update_only<V, W, B>(const SysView<V, W>&, int, hipStream_t);                           \
    template void launch_update_reduce<V, W, B>(const SysView<V, W>&, int, hipStream_t);                         \
    template void launch_true_resid<V, W, B>(const SysView<V, W>&, int, hipStream_t);                            \
    template void launch_spmm<V, W, B>(const SysView<V, W>&, const V*, int64_t, int, int64_t, double*, V*,       \
                                       hipStream_t);                                                              \
    template void batch_spmv_dot<V, W, B>(const SysView<V, W>*, const BatchMaps&, hipStream_t);                  \
    template void batch_update_reduce<V, W, B>(const SysView<V, W>*, const BatchMaps&, int, hipStream_t);        \
    template void batch_update_only<V, W, B>(const SysView<V, W>*, const BatchMaps&, int, hipStream_t);          \
    template void batch_true_resid<V, W, B>(const SysView<V, W>*, const BatchMaps&, int, hipStream_t);

#define KRS_INST_VW(V, W)                                                                                         \
    template void launch_correct_dir<V, W>(const SysView<V, W>&, int, hipStream_t);                              \
    template void launch_reorth_store<V, W>(const SysView<V, W>&, hipStream_t);                                  \
    template void launch_reorth<V, W>(const SysView<V, W>&, hipStream_t);                                        \
    template void launch_coarse_dot<V, W>(const SysView<V, W>&, int, int, uint32_t, hipStream_t);                \
    template void launch_coarse_correct<V, W>(const SysView<V, W>&, int, uint32_t, hipStream_t);                 \
    template void batch_correct_dir<V, W>(const SysView<V, W>*, const BatchMaps&, int, hipStream_t);             \
    template void batch_coarse_dot<V, W>(const SysView<V, W>*, const BatchMaps&, int, int, uint32_t, hipStream_t); \
    template void batch_coarse_correct<V, W>(const SysView<V, W>*, const BatchMaps&, int, uint32_t, hipStream_t); \
    template void batch_status<V, W>(const SysView<V, W>*, int, int32_t*, hipStream_t);

#define KRS_INST_VB(V, B)                                                                                        \
    template void launch_scatter_values<V, B>(const double*, const int64_t*, int64_t, double*, V*, hipStream_t); \
    template void launch_precond_setup<V, B>(const double*, const int64_t*, int64_t, V*, int32_t*, hipStream_t);

#define KRS_INST_V(V)                                                                                             \
    template void launch_gram<V>(const V*, int64_t, const double*, int64_t, int64_t, int, double*, double*,      \
                                 int64_t, hipStream_t);                                                           \
    template void launch_basis_combine<V>(const V*, int64_t, int, const double*, int, V*, int64_t, int64_t,       \
                                          hipStream_t);                                                           \
    template void launch_scale_columns<V>(V*, int64_t, int64_t, const double*, int, hipStream_t);                \
    template void launch_copy_columns<V>(const V*, int64_t, V*, int64_t, int64_t, const int32_t*, int,            \
                                         hipStream_t);                                                            \
    template void launch_d2v<V>(const double*, V*, int64_t, hipStream_t);                                        \
    template void launch_v2d<V>(const V*, double*, int64_t, hipStream_t);

KRS_INST_VWB(double, double, 1)
KRS_INST_VWB(double, double, 3)
KRS_INST_VWB(float, double, 1)
KRS_INST_VWB(float, double, 3)
KRS_INST_VWB(float, float, 1)
KRS_INST_VWB(float, float, 3)
KRS_INST_VW(double, double)
KRS_INST_VW(float, double)
KRS_INST_VW(float, float)
KRS_INST_VB(float, 1)
KRS_INST_VB(float, 3)
KRS_INST_VB(double, 1)
KRS_INST_VB(double, 3)
KRS_INST_V(float)
KRS_INST_V(double)

}  // namespace krs
