// Device kernels of libkrs for gfx950 (CDNA4, wave64).
//
// One APCG iteration (Algorithm 1, standard Hestenes-Stiefel form) is three
// launches, each ending in a fixed-order grid reduction finished by the last
// workgroup to arrive (no floating-point atomics, so results are bitwise
// reproducible):
//   spmv_dot       q = A w, gamma = (w, q), alpha = rho / gamma
//   update_reduce  x += alpha w, r -= alpha q, s = M^-1 r,
//                  ||r||^2, (r, s), t = (AC)^T s;  last workgroup: beta, mu = G^-1 t
//   correct_dir    z = s - C mu, w = z + beta w   (z / w recorded for reuse)
// (r, s) equals (r, z) because C^T r = 0 (Section 2.2, constraint view).
//
// Matrices are stored in sliced ELL: 64 (block) rows per slice, one lane
// per block row, slot k of every row of a slice stored contiguously so a
// wavefront reads 64 consecutive values per load.  3x3 blocks are stored as
// 9 planes of 64 values per slot: value (d, e) of the block in slot k of
// lane l sits at ((slot*9) + 3d + e)*64 + l.  Sub-row d of a slice is
// handled by wave d of a 192-thread workgroup.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace krs {

namespace {

constexpr int kTpb = 256;          // threads per workgroup, scalar kernels
constexpr int kMaxGrid = 512;      // cap on the update grid (bounds the partial sums)
constexpr int kMaxChunks = 16;     // projector reduction: up to 16*64 = 1024 basis columns

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

// Reduce `nv` values over `np` partial rows (row stride `stride`) in a fixed
// order with all threads of the workgroup; out[k] for k < nv (LDS).
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
            // up to 32 independent loads in flight per thread
            int64_t i = p;
            for (; i + 32 * tpv <= np; i += 32 * tpv) {
                double t[32];
#pragma unroll
                for (int u = 0; u < 32; ++u) t[u] = partials[(i + u * tpv) * stride + k];
#pragma unroll
                for (int u = 0; u < 32; ++u) acc += t[u];
            }
            for (; i + 8 * tpv <= np; i += 8 * tpv) {
                double t[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) t[u] = partials[(i + u * tpv) * stride + k];
#pragma unroll
                for (int u = 0; u < 8; ++u) acc += t[u];
            }
            for (; i < np; i += tpv) acc += partials[i * stride + k];
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

// Fixed-order sum of p[0..np), returned to every thread of the workgroup.
__device__ double sum_all(const double* p, int64_t np, double* lds) {
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += blockDim.x) a += p[i];
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
        if (act)
            for (int c = p; c < nc; c += P) m += Ginv[(int64_t)c * nc + r] * t[c];
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

// Live kernel timing: iteration j is sampled when j % 32 == 1 (K1, K3) and
// its direction update (K5, which already sees j + 1) likewise.  Every
// workgroup of a sampled launch stores its start and end wall-clock stamps
// in its own slot (plain stores, no contention); the finalize kernel adds
// max(end) - min(start) to the running sums.
constexpr int kSlotStride = 2 * 4096;
__device__ __forceinline__ bool ktime_sample(const DevState* st, int which) {
    return st->ktime_on && (st->iter & 31) == (which == 2 ? 2 : 1);
}
__device__ __forceinline__ void ktime_begin(unsigned long long* slots, int which, bool on) {
    if (on && threadIdx.x == 0) slots[which * kSlotStride + 2 * blockIdx.x] = (unsigned long long)wall_clock64();
}
__device__ __forceinline__ void ktime_end(unsigned long long* slots, int which, bool on) {
    if (on) {
        __syncthreads();
        if (threadIdx.x == 0) slots[which * kSlotStride + 2 * blockIdx.x + 1] = (unsigned long long)wall_clock64();
    }
}
// All threads: span of kernel `which` over np workgroup slots, added to
// the sums by thread 0.  lds: 2 * blockDim.x entries.
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
    for (; k < k1; ++k) {
        const int64_t e = k * 64 + lane;
        acc += (X)val[e] * x[col[e]];
    }
    return acc;
}

// Sub-row d of one 3x3-block ELL row: the three entries (d, 0..2) of every
// block, times the three entries of x at its block column.
template <typename V, typename X>
__device__ __forceinline__ X ell_row3(const V* __restrict__ val, const int32_t* __restrict__ col,
                                      const X* __restrict__ x, int64_t k0, int64_t k1, int lane, int d) {
    constexpr int UNR = 4;
    X acc = 0;
    int64_t k = k0;
    for (; k + UNR <= k1; k += UNR) {
        int32_t cc[UNR];
        V a[UNR][3];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            cc[u] = col[(k + u) * 64 + lane];
            const V* vb = val + ((k + u) * 9 + 3 * d) * 64 + lane;
            a[u][0] = vb[0];
            a[u][1] = vb[64];
            a[u][2] = vb[128];
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
        for (int u = 0; u < UNR; ++u) acc += (X)a[u][0] * xs[u][0] + (X)a[u][1] * xs[u][1] + (X)a[u][2] * xs[u][2];
    }
    for (; k < k1; ++k) {
        const int64_t c = 3 * (int64_t)col[k * 64 + lane];
        const V* vb = val + (k * 9 + 3 * d) * 64 + lane;
        acc += (X)vb[0] * x[c] + (X)vb[64] * x[c + 1] + (X)vb[128] * x[c + 2];
    }
    return acc;
}

// ------------------------------------------------------------------ K1
// q = A w over sliced ELL; per-workgroup partial sums of (w, q) go to
// part1[blockIdx.x].  alpha = rho / (w, q) is formed from them by every
// workgroup of the next kernel (a fixed-order sum, so all agree).
template <typename V, typename W, int B>
__global__ __launch_bounds__(256) void k_spmv_dot(SysView<V, W> v) {
    if (!gate(v.st, M_RUN)) return;
    const bool tm = ktime_sample(v.st, 0);
    ktime_begin(v.kslots, 0, tm);
    __shared__ double lds[8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double part = 0.0;
    if (B == 1) {
        // 4 slices per workgroup, one per wave
        for (int64_t sl = (int64_t)blockIdx.x * 4 + wave; sl < v.nslices; sl += (int64_t)gridDim.x * 4) {
            const int64_t k0 = v.slice_ptr[sl], k1 = v.slice_ptr[sl + 1];
            const W acc = ell_row1<V, W>(v.val, v.col, v.w, k0, k1, lane);
            const int64_t row = sl * 64 + lane;
            if (row < v.n) {
                v.q[row] = acc;
                part += (double)v.w[row] * (double)acc;
            }
        }
    } else {
        // one slice per workgroup step; wave d = sub-row d of the 3x3 blocks
        const int d = wave;
        for (int64_t sl = blockIdx.x; sl < v.nslices; sl += gridDim.x) {
            const int64_t k0 = v.slice_ptr[sl], k1 = v.slice_ptr[sl + 1];
            const W acc = ell_row3<V, W>(v.val, v.col, v.w, k0, k1, lane, d);
            const int64_t p = sl * 64 + lane;
            if (p < v.nb) {
                v.q[3 * p + d] = acc;
                part += (double)v.w[3 * p + d] * (double)acc;
            }
        }
    }
    const double bs = block_sum(part, lds);
    if (threadIdx.x == 0) v.part1[blockIdx.x] = bs;
    ktime_end(v.kslots, 0, tm);
}

// ------------------------------------------------------------------ K3
// mode 0: x += alpha w, r -= alpha q (the regular step)
// mode 1: initial step (r0 given), no update
// mode 2: after a true-residual replacement, no update
// then s = M^-1 r and per-workgroup partials, stride 2 nc + 2:
//   [ ||r||^2, (r, s), t = (AC)^T s (nc), v = (AC)^T w (nc, modes 0 and 2) ]
// v measures the A-component of w along C, which is zero in exact
// arithmetic; it drives the recurrence for u = C^T r used to form
// rho = (r, z) = (r, s) - (C^T r)^T mu exactly.  Tiles of TR rows (block
// aligned); the projector part reads the tile's rows of AC (row-major) once
// with one lane per column (CW lanes, RW rows per wave step) and
// accumulates both sums per column in LDS.
template <typename V, typename W, int B>
__global__ __launch_bounds__(1024) void k_update_reduce(SysView<V, W> v, int mode, int np1) {
    DevState* st = v.st;
    const uint32_t mask = (mode == 2) ? M_REFINE : M_RUN;
    if (!gate(st, mask)) return;
    const bool tm = mode == 0 && ktime_sample(st, 1);
    ktime_begin(v.kslots, 1, tm);
    constexpr int TR = (B == 1) ? 1024 : 768;  // rows per tile == threads
    __shared__ double ss[TR];
    __shared__ double ws[TR];
    __shared__ double red[1024];
    __shared__ double red2[1024];
    __shared__ double tacc[1024];
    __shared__ double vacc[1024];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int nwaves = TR / 64;
    const int nc = st->nc;
    double a = 0.0;
    if (mode == 0) a = st->rho / sum_all(v.part1, np1, red);
    for (int c = tid; c < nc; c += TR) {
        tacc[c] = 0.0;
        vacc[c] = 0.0;
    }
    // projector reduction geometry
    int CW = 64;
    if (nc <= 32) CW = nc <= 1 ? 1 : (nc <= 2 ? 2 : (nc <= 4 ? 4 : (nc <= 8 ? 8 : (nc <= 16 ? 16 : 32))));
    const int RW = 64 / CW;
    const int nch = (nc + 63) / 64;
    const int c0 = lane % CW, rsub = lane / CW;
    const int G = nwaves * RW;
    const int g0 = wave * RW + rsub;
    double rr = 0.0, rs = 0.0;
    const int64_t ntiles = (v.n + TR - 1) / TR;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t i = tile * TR + tid;
        double ri = 0.0, wi = 0.0;
        if (i < v.n) {
            W rv = v.r[i];
            if (mode != 1) wi = (double)v.w[i];
            if (mode == 0) {
                v.x[i] += a * wi;
                rv = (W)((double)rv - a * (double)v.q[i]);
                v.r[i] = rv;
            }
            ri = (double)rv;
        }
        double si = 0.0;
        if (B == 1) {
            if (i < v.n) si = (double)(W)((double)v.minv[i] * ri);
        } else {
            __syncthreads();
            ss[tid] = ri;
            __syncthreads();
            if (i < v.n) {
                const int d = tid % 3;
                const int64_t p = i / 3;
                const V* mb = v.minv + p * 9 + d * 3;
                const int t0 = tid - d;
                si = (double)(W)((double)mb[0] * ss[t0] + (double)mb[1] * ss[t0 + 1] + (double)mb[2] * ss[t0 + 2]);
            }
        }
        if (i < v.n) {
            v.s[i] = (W)si;
            rr += ri * ri;
            rs += ri * si;
        }
        if (nc > 0) {
            __syncthreads();
            ss[tid] = (i < v.n) ? si : 0.0;
            ws[tid] = (i < v.n) ? wi : 0.0;
            __syncthreads();
            const int rows = (int)((v.n - tile * TR) < TR ? (v.n - tile * TR) : TR);
            const V* ACt = v.AC + tile * TR * v.ldac;
            constexpr int UR = 8;
            for (int ch = 0; ch < nch; ++ch) {
                const int c = ch * 64 + c0;
                double a2 = 0.0, b2 = 0.0;
                if (c < nc) {
                    for (int r = g0; r < rows; r += G * UR) {
                        // rows past the tile end are clamped (weight 0) so
                        // every load of the group is issued unconditionally
                        V av[UR];
#pragma unroll
                        for (int u = 0; u < UR; ++u) {
                            const int r2 = min(r + u * G, rows - 1);
                            av[u] = ACt[(int64_t)r2 * v.ldac + c];
                        }
#pragma unroll
                        for (int u = 0; u < UR; ++u) {
                            const int r2 = r + u * G;
                            const bool ok = r2 < rows;
                            a2 += (double)av[u] * (ok ? ss[r2] : 0.0);
                            b2 += (double)av[u] * (ok ? ws[r2] : 0.0);
                        }
                    }
                }
                // combine the G row groups of this chunk (fixed order)
                __syncthreads();
                red[g0 * CW + c0] = a2;
                red2[g0 * CW + c0] = b2;
                __syncthreads();
                if (tid < CW && ch * 64 + tid < nc) {
                    double t = 0.0, u2 = 0.0;
                    for (int gg = 0; gg < G; ++gg) {
                        t += red[gg * CW + tid];
                        u2 += red2[gg * CW + tid];
                    }
                    tacc[ch * 64 + tid] += t;
                    vacc[ch * 64 + tid] += u2;
                }
            }
        }
    }
    // workgroup partials
    const int stride = 2 * nc + 2;
    double* myp = v.partials + (int64_t)blockIdx.x * stride;
    {
        const double brr = block_sum(rr, red);
        if (tid == 0) myp[0] = brr;
        const double brs = block_sum(rs, red);
        if (tid == 0) myp[1] = brs;
    }
    __syncthreads();
    for (int c = tid; c < nc; c += TR) {
        myp[2 + c] = tacc[c];
        myp[2 + nc + c] = vacc[c];
    }
    ktime_end(v.kslots, 1, tm);
}

// F3: one workgroup.  Reduces the partials of K1 (mode 0) and K3, records
// alpha_j, gamma_j, rho_{j+1}, decides convergence / refinement / breakdown
// and forms beta, mu = G^-1 t, mu2 and u = C^T r for the direction update.
// Being a single workgroup it is latency bound: every independent load
// (K3 partials, K1 partials, G^-1, state) is issued before the first wait.
template <typename V, typename W>
__global__ __launch_bounds__(1024) void k_finalize_update(SysView<V, W> v, int mode, int np1, int np3, int np5) {
    DevState* st = v.st;
    const uint32_t mask = (mode == 2) ? M_REFINE : M_RUN;
    if (!gate(st, mask)) return;
    __shared__ double red[1024];
    __shared__ double fin[2048 + 4];
    __shared__ double muL[1024];
    __shared__ double gvL[1024];
    __shared__ double Gl[4096];
    __shared__ double beta_s;
    const int tid = threadIdx.x;
    const int T = blockDim.x;
    const int nc = st->nc;
    const int nv = 2 * nc + 2;
    const int stride = nv;
    // ---- issue loads: K3 partials (fast path: <= 32 per thread)
    int tpv = T / nv;
    if (tpv < 1) tpv = 1;
    if (tpv > 64) tpv = 64;
    const int per = (np3 + tpv - 1) / tpv;
    const bool fast = nv <= T && per <= 32;
    const int kv = tid / tpv, pv = tid % tpv;
    const bool act = fast && kv < nv && kv < T / tpv;
    double vals[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
        const int idx = pv + u * tpv;
        vals[u] = (act && idx < np3) ? v.partials[(int64_t)idx * stride + kv] : 0.0;
    }
    double p1 = 0.0;
    if (mode == 0)
        for (int64_t i = tid; i < np1; i += T) p1 += v.part1[i];
    const bool gsmall = nc <= 64;
    if (gsmall)
        for (int e = tid; e < nc * nc; e += T) Gl[e] = v.Ginv[e];
    // ---- combine
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 32; ++u) acc += vals[u];
    const double g = (mode == 0) ? sum_all_reg(p1, red) : 0.0;
    if (fast) {
        red[tid] = acc;
        __syncthreads();
        if (act && pv == 0) {
            double t = 0.0;
            for (int j = 0; j < tpv; ++j) t += red[tid + j];
            fin[kv] = t;
        }
        __syncthreads();
    } else {
        reduce_partials(v.partials, np3, nv, stride, fin, red);
        __syncthreads();
    }
    const double a = (mode == 0) ? st->rho / g : 0.0;
    double du = 0.0;
    if (nc > 0) {
        const double* Gi = gsmall ? Gl : v.Ginv;
        ginv_matvec(Gi, nc, fin + 2, muL, red);
        ginv_matvec(Gi, nc, fin + 2 + nc, gvL, red);
        __syncthreads();
        // u = C^T r: recurrence u -= alpha (AC)^T w; zero after (re)projection
        double p = 0.0;
        for (int c = tid; c < nc; c += T) {
            const double uc = (mode == 0) ? v.u[c] - a * fin[2 + nc + c] : 0.0;
            v.u[c] = uc;
            v.mu[c] = muL[c];
            p += uc * muL[c];
        }
        du = sum_all_reg(p, red);
    }
    const int j0 = st->iter;
    if (mode == 0 && st->ktime_on) {
        unsigned long long* tl = reinterpret_cast<unsigned long long*>(Gl);
        if ((j0 & 31) == 1) {
            ktime_collect(st, v.kslots, 0, np1, tl);
            ktime_collect(st, v.kslots, 1, np3, tl);
        } else if ((j0 & 31) == 2) {
            ktime_collect(st, v.kslots, 2, np5, tl);
        }
    }
    if (tid == 0) {
        const double rrn = fin[0];
        const double rho_new = fin[1] - du;  // (r, z) = (r, s) - (C^T r)^T mu
        const double rr_before = st->rr;
        const int j = j0;
        int stn = ST_RUN;
        if (mode == 0) {
            if (j < v.coef_cap) {
                v.gamma_h[j] = g;
                v.alpha_h[j] = a;
            }
            st->alpha = a;
            st->pending_dir = 0;
            const int it = j + 1;
            st->iter = it;
            st->since_refine += 1;
            st->rr = rrn;
            if (!finite_pos(g) || !(rrn == rrn)) {
                stn = ST_BREAKDOWN;
            } else if (rrn <= st->tol2 * st->bb) {
                stn = ST_CHECK;
            } else if (it >= st->max_iter) {
                stn = ST_MAXIT;
            } else if ((st->refine_every > 0 && st->since_refine >= st->refine_every) ||
                       (st->drop2 > 0.0 && rrn < st->drop2 * st->rr_ref)) {
                stn = ST_REFINE;
            }
        } else {
            st->rr = rrn;
            st->rr_ref = rrn;
            if (mode == 2) {
                st->since_refine = 0;
                st->pending_dir = 1;
            } else {
                if (rrn <= st->tol2 * st->bb) stn = ST_CHECK;
                if (st->max_iter <= 0 && stn == ST_RUN) stn = ST_MAXIT;
            }
        }
        if (stn == ST_RUN) {
            if (!finite_pos(rho_new)) {
                stn = ST_BREAKDOWN;
            } else {
                const int it = st->iter;
                double beta = (mode == 1) ? 0.0 : rho_new / st->rho;
                // A replacement that more than doubles the residual (the
                // single-precision operator's floor reached) voids the
                // conjugacy with the old direction: restart from z.
                if (mode == 2 && rrn > 4.0 * rr_before) {
                    beta = 0.0;
                    st->restarts += 1;
                    if (it < st->first_restart) st->first_restart = it;
                }
                st->beta = beta;
                st->rho = rho_new;
                if (it < v.coef_cap) v.rho_h[it] = rho_new;
            }
        }
        st->status = stn;
        beta_s = (stn == ST_RUN) ? st->beta : 0.0;
    }
    __syncthreads();
    // the new direction is projected as a whole: w = P (z + beta w_old)
    // = s + beta w_old - C (mu + beta G^-1 (AC)^T w_old)
    const double bt = beta_s;
    for (int c = tid; c < nc; c += T) v.mu2[c] = muL[c] + bt * gvL[c];
}

// ------------------------------------------------------------------ K5
// z = s - C mu (recorded for SRKS) and the new direction
// w = s - C mu2 + beta w_old with mu2 = mu + beta G^-1 (AC)^T w_old, i.e.
// w = P (z + beta w_old): the whole direction is kept A-orthogonal to C
// (in exact arithmetic (AC)^T w_old = 0 and mu2 = mu).  first = 1: initial
// direction w = z; first = 2: the update that follows a residual
// replacement (runs only when one is pending).
template <typename V, typename W>
__device__ __forceinline__ void correct_row(const SysView<V, W>& v, int64_t i, int nc, const double* mu,
                                            const double* mu2, double beta, int first, int j, int hist_cap) {
    const double s = (double)v.s[i];
    double cz = 0.0, cw = 0.0;
    const V* Ci = v.C + i;
    int c = 0;
    for (; c + 4 <= nc; c += 4) {
        const double c0 = (double)Ci[(int64_t)c * v.ldc], c1 = (double)Ci[(int64_t)(c + 1) * v.ldc];
        const double c2 = (double)Ci[(int64_t)(c + 2) * v.ldc], c3 = (double)Ci[(int64_t)(c + 3) * v.ldc];
        cz += c0 * mu[c] + c1 * mu[c + 1] + c2 * mu[c + 2] + c3 * mu[c + 3];
        cw += c0 * mu2[c] + c1 * mu2[c + 1] + c2 * mu2[c + 2] + c3 * mu2[c + 3];
    }
    for (; c < nc; ++c) {
        const double cc = (double)Ci[(int64_t)c * v.ldc];
        cz += cc * mu[c];
        cw += cc * mu2[c];
    }
    const W zv = (W)(s - cz);
    const W wv = (first == 1) ? zv : (W)(s - cw + beta * (double)v.w[i]);
    v.w[i] = wv;
    if (j < hist_cap) {
        if (v.zhist) v.zhist[(int64_t)j * v.ldh + i] = (V)zv;
        if (v.whist) v.whist[(int64_t)j * v.ldh + i] = (V)wv;
    }
}

template <typename V, typename W>
__global__ __launch_bounds__(256) void k_correct_dir(SysView<V, W> v, int first) {
    DevState* st = v.st;
    if (!gate(st, M_RUN)) return;
    if (first == 2 && st->pending_dir == 0) return;
    __shared__ double mu[1024];
    __shared__ double mu2[1024];
    const int nc = st->nc;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        mu[c] = v.mu[c];
        mu2[c] = (first == 1) ? v.mu[c] : v.mu2[c];
    }
    __syncthreads();
    const double beta = (first == 1) ? 0.0 : st->beta;
    const int j = st->iter;
    const bool tm = first == 0 && ktime_sample(st, 2);
    ktime_begin(v.kslots, 2, tm);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < v.n; i += (int64_t)gridDim.x * blockDim.x)
        correct_row(v, i, nc, mu, mu2, beta, first, j, st->hist_cap);
    ktime_end(v.kslots, 2, tm);
}

// ----------------------------------------------------------------- K11
// r = b - A x with double-precision values and x.  final_only: only record
// ||r||^2 (for the report), leave r and the status alone.
template <typename V, typename W, int B>
__global__ __launch_bounds__(256) void k_true_resid(SysView<V, W> v, int final_only) {
    DevState* st = v.st;
    if (!final_only && !gate(st, M_CHECK | M_REFINE)) return;
    __shared__ double lds[8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double part = 0.0;
    if (B == 1) {
        for (int64_t sl = (int64_t)blockIdx.x * 4 + wave; sl < v.nslices; sl += (int64_t)gridDim.x * 4) {
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
        const int d = wave;
        for (int64_t sl = blockIdx.x; sl < v.nslices; sl += gridDim.x) {
            const int64_t k0 = v.slice_ptr[sl], k1 = v.slice_ptr[sl + 1];
            const double acc = ell_row3<double, double>(v.val64, v.col, v.x, k0, k1, lane, d);
            const int64_t p = sl * 64 + lane;
            if (p < v.nb) {
                const double ri = v.b[3 * p + d] - acc;
                if (!final_only) v.r[3 * p + d] = (W)ri;
                part += ri * ri;
            }
        }
    }
    const double bs = block_sum(part, lds);
    if (threadIdx.x == 0) v.partials[blockIdx.x] = bs;
}

// F11: one workgroup; ||b - A x||^2 and the decision after a true residual.
template <typename V, typename W>
__global__ __launch_bounds__(1024) void k_finalize_resid(SysView<V, W> v, int final_only, int np) {
    DevState* st = v.st;
    if (!final_only && !gate(st, M_CHECK | M_REFINE)) return;
    __shared__ double red[32];
    const double rt = sum_all(v.partials, np, red);
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
// t = C^T u (u = src64 or srcV), optionally bb = (u, u); last workgroup:
// mu = Ginv t.  Used for x0 (u = b) and for the re-projection after a
// true-residual replacement (u = r).
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_coarse_dot(SysView<V, W> v, const double* src64, const W* srcV, int with_bb,
                                                    uint32_t mask) {
    DevState* st = v.st;
    if (!gate(st, mask)) return;
    __shared__ double red[kTpb];
    __shared__ double wpart[4 * 1024];
    const int nc = st->nc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int stride = nc + 1;
    double* myp = v.partials + (int64_t)blockIdx.x * stride;
    // each thread accumulates over its rows, then waves reduce per column,
    // 16 columns per pass over the rows
    double bbp = 0.0;
    for (int c0 = 0; c0 < nc || c0 == 0; c0 += 16) {
        double acc[16];
        const int cn = (nc - c0) < 16 ? (nc - c0) : 16;
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < v.n; i += (int64_t)gridDim.x * blockDim.x) {
            const double u = src64 ? src64[i] : (double)srcV[i];
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

// One workgroup: t and (u, u) from the partials of k_coarse_dot; mu = Ginv t.
template <typename V, typename W>
__global__ __launch_bounds__(1024) void k_finalize_dot(SysView<V, W> v, int with_bb, uint32_t mask, int np) {
    DevState* st = v.st;
    if (!gate(st, mask)) return;
    __shared__ double red[1024];
    __shared__ double fin[1024 + 4];
    const int nc = st->nc;
    const int stride = nc + 1;
    reduce_partials(v.partials, np, stride, stride, fin, red);
    __syncthreads();
    if (threadIdx.x == 0 && with_bb) st->bb = fin[0];
    if (nc > 0) ginv_matvec(v.Ginv, nc, fin + 1, v.mu, red);
}

// x = (from_b ? 0 : x) + C mu;  r = (from_b ? b : r) - AC mu
template <typename V, typename W>
__global__ __launch_bounds__(256) void k_coarse_correct(SysView<V, W> v, int from_b, uint32_t mask) {
    DevState* st = v.st;
    if (!gate(st, mask)) return;
    __shared__ double mu[1024];
    const int nc = st->nc;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) mu[c] = v.mu[c];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

// ------------------------------------------------------------ rebuild
// AC64 = A C (double values), row-major n x nc; ACv = AC64 in V.
// blockIdx.y selects 8 columns.
template <typename V, typename W, int B>
__global__ __launch_bounds__(256) void k_spmm(SysView<V, W> v, const V* C, int64_t ldc, int nc, double* AC64, V* ACv) {
    constexpr int CW = 8;
    const int c0 = blockIdx.y * CW;
    const int cn = (nc - c0) < CW ? (nc - c0) : CW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
                        AC64[row * nc + c0 + j] = acc[j];
                        ACv[row * nc + c0 + j] = (V)acc[j];
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
                        AC64[row * nc + c0 + j] = acc[j];
                        ACv[row * nc + c0 + j] = (V)acc[j];
                    }
            }
        }
    }
}

// G = C^T AC64: 16x16 output tiles (blockIdx.y), row ranges (blockIdx.x)
// into partials[blockIdx.x][nc*nc]; k_gram_reduce sums them in order.
template <typename V>
__global__ __launch_bounds__(256) void k_gram_partial(const V* C, int64_t ldc, const double* AC64, int64_t n, int nc,
                                                      double* partials) {
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
            sA[rr][cc] = (i < r1 && cb < nc) ? AC64[i * nc + cb] : 0.0;
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
template <typename V>
__global__ __launch_bounds__(256) void k_basis_combine(const V* Z, int64_t ldz, int m, const double* F, int s, V* out,
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
        V* o = minv + p * 9;
        o[0] = (V)(A * id);
        o[1] = (V)(-(b * k - c * h) * id);
        o[2] = (V)((b * f - c * e) * id);
        o[3] = (V)(Bc * id);
        o[4] = (V)((a * k - c * g) * id);
        o[5] = (V)(-(a * f - c * d) * id);
        o[6] = (V)(Cc * id);
        o[7] = (V)(-(a * h - b * g) * id);
        o[8] = (V)((a * e - b * d) * id);
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

int64_t spmv_grid(int64_t nslices, int block) {
    const int64_t per = (block == 1) ? 4 : 1;
    int64_t g = (nslices + per - 1) / per;
    if (g > 2048) g = 2048;
    return g < 1 ? 1 : g;
}

// Tiles are dealt round-robin; with at most kMaxGrid workgroups every
// workgroup gets ceil(ntiles / grid) or one fewer.
int64_t update_grid(int64_t n, int block) {
    const int64_t TR = (block == 1) ? 1024 : 768;
    const int64_t ntiles = (n + TR - 1) / TR;
    const int64_t per = (ntiles + kMaxGrid - 1) / kMaxGrid;
    const int64_t g = (ntiles + per - 1) / per;
    return g < 1 ? 1 : g;
}

int64_t correct_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    return g < 1 ? 1 : g;
}

int64_t dot_grid(int64_t n) {
    int64_t g = (n + kTpb - 1) / kTpb;
    if (g > 256) g = 256;
    return g < 1 ? 1 : g;
}

template <typename V, typename W, int B>
void launch_spmv_dot(const SysView<V, W>& v, hipStream_t stream) {
    const int threads = (B == 1) ? 256 : 192;
    hipLaunchKernelGGL((k_spmv_dot<V, W, B>), dim3((unsigned)spmv_grid(v.nslices, B)), dim3(threads), 0, stream, v);
}

template <typename V, typename W, int B>
void launch_update_reduce(const SysView<V, W>& v, int mode, hipStream_t stream) {
    const int threads = (B == 1) ? 1024 : 768;
    const int np1 = (int)spmv_grid(v.nslices, B);
    const int np3 = (int)update_grid(v.n, B);
    hipLaunchKernelGGL((k_update_reduce<V, W, B>), dim3((unsigned)np3), dim3(threads), 0, stream, v, mode, np1);
    hipLaunchKernelGGL((k_finalize_update<V, W>), dim3(1), dim3(1024), 0, stream, v, mode, np1, np3,
                       (int)correct_grid(v.n));
}

template <typename V, typename W>
void launch_correct_dir(const SysView<V, W>& v, int first, hipStream_t stream) {
    hipLaunchKernelGGL((k_correct_dir<V, W>), dim3((unsigned)correct_grid(v.n)), dim3(256), 0, stream, v, first);
}

template <typename V, typename W, int B>
void launch_true_resid(const SysView<V, W>& v, int final_only, hipStream_t stream) {
    const int threads = (B == 1) ? 256 : 192;
    const int np = (int)spmv_grid(v.nslices, B);
    hipLaunchKernelGGL((k_true_resid<V, W, B>), dim3((unsigned)np), dim3(threads), 0, stream, v, final_only);
    hipLaunchKernelGGL((k_finalize_resid<V, W>), dim3(1), dim3(1024), 0, stream, v, final_only, np);
}

template <typename V, typename W>
void launch_coarse_dot(const SysView<V, W>& v, const double* src64, const W* srcV, int with_bb, uint32_t mask,
                       hipStream_t stream) {
    const int np = (int)dot_grid(v.n);
    hipLaunchKernelGGL((k_coarse_dot<V, W>), dim3((unsigned)np), dim3(256), 0, stream, v, src64, srcV, with_bb, mask);
    hipLaunchKernelGGL((k_finalize_dot<V, W>), dim3(1), dim3(1024), 0, stream, v, with_bb, mask, np);
}

template <typename V, typename W>
void launch_coarse_correct(const SysView<V, W>& v, int from_b, uint32_t mask, hipStream_t stream) {
    hipLaunchKernelGGL((k_coarse_correct<V, W>), dim3(cdiv(v.n, 256)), dim3(256), 0, stream, v, from_b, mask);
}

template <typename V, typename W, int B>
void launch_spmm(const SysView<V, W>& v, const V* C, int64_t ldc, int nc, double* AC64, V* ACv, hipStream_t stream) {
    if (nc <= 0) return;
    const int threads = (B == 1) ? 256 : 192;
    dim3 grid((unsigned)spmv_grid(v.nslices, B), (unsigned)((nc + 7) / 8));
    hipLaunchKernelGGL((k_spmm<V, W, B>), grid, dim3(threads), 0, stream, v, C, ldc, nc, AC64, ACv);
}

template <typename V>
void launch_gram(const V* C, int64_t ldc, const double* AC64, int64_t n, int nc, double* G, double* partials,
                 int64_t partial_cap, hipStream_t stream) {
    if (nc <= 0) return;
    const int64_t nn = (int64_t)nc * nc;
    int np = (int)(partial_cap / nn);
    if (np > 64) np = 64;
    if (np < 1) np = 1;
    const int ntc = (nc + 15) / 16;
    hipLaunchKernelGGL((k_gram_partial<V>), dim3((unsigned)np, (unsigned)(ntc * ntc)), dim3(256), 0, stream, C, ldc,
                       AC64, n, nc, partials);
    hipLaunchKernelGGL(k_gram_reduce, dim3(cdiv(nn, 256)), dim3(256), 0, stream, partials, np, nc, G);
}

template <typename V>
void launch_basis_combine(const V* Z, int64_t ldz, int m, const double* F, int s, V* out, int64_t ldo, int64_t n,
                          hipStream_t stream) {
    if (s <= 0 || m <= 0) return;
    dim3 grid(cdiv(n, 256), (unsigned)((s + 7) / 8));
    hipLaunchKernelGGL((k_basis_combine<V>), grid, dim3(256), 0, stream, Z, ldz, m, F, s, out, ldo, n);
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

template <typename V>
void launch_v2d(const V* in, double* out, int64_t n, hipStream_t stream) {
    hipLaunchKernelGGL((k_v2d<V>), dim3(cdiv(n, 256)), dim3(256), 0, stream, in, out, n);
}

#define KRS_INST_VWB(V, W, B)                                                                                    \
    template void launch_spmv_dot<V, W, B>(const SysView<V, W>&, hipStream_t);                                    \
    template void launch_update_reduce<V, W, B>(const SysView<V, W>&, int, hipStream_t);                         \
    template void launch_true_resid<V, W, B>(const SysView<V, W>&, int, hipStream_t);                            \
    template void launch_spmm<V, W, B>(const SysView<V, W>&, const V*, int64_t, int, double*, V*, hipStream_t);

#define KRS_INST_VW(V, W)                                                                                         \
    template void launch_correct_dir<V, W>(const SysView<V, W>&, int, hipStream_t);                              \
    template void launch_coarse_dot<V, W>(const SysView<V, W>&, const double*, const W*, int, uint32_t,          \
                                          hipStream_t);                                                           \
    template void launch_coarse_correct<V, W>(const SysView<V, W>&, int, uint32_t, hipStream_t);

#define KRS_INST_VB(V, B)                                                                                        \
    template void launch_scatter_values<V, B>(const double*, const int64_t*, int64_t, double*, V*, hipStream_t); \
    template void launch_precond_setup<V, B>(const double*, const int64_t*, int64_t, V*, int32_t*, hipStream_t);

#define KRS_INST_V(V)                                                                                             \
    template void launch_gram<V>(const V*, int64_t, const double*, int64_t, int, double*, double*, int64_t,       \
                                 hipStream_t);                                                                    \
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
