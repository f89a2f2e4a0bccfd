// Host-side Ritz analysis for selective reuse (Section 4.1 and 4.4).
//
// The Lanczos tridiagonal recovered from the CG coefficients is factored as
// H_m = L D L^T with d_j = 1/alpha_j and l_j^2 = beta_{j+1} = rho_{j+1}/rho_j
// (expanding L D L^T gives delta_j = d_j + l_{j-1}^2 d_{j-1} and
// eta_j = l_j d_j, the entries of Section 4.1).  Eigenvalues are obtained by
// bisection on the inertia of L D L^T - sigma I computed with the stationary
// qd transform, which keeps high relative accuracy for the small Ritz values
// that the 1e-14 stagnation test must resolve.  Eigenvectors of the few
// selected values come from a twisted factorisation of T - theta I.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <thread>
#include <vector>

#include "internal.h"

namespace krs {

namespace {

// number of eigenvalues of L D L^T strictly below sigma
inline int inertia_below(int m, const double* d, const double* l2d, double sigma) {
    int neg = 0;
    double t = -sigma;
    for (int i = 0; i < m; ++i) {
        double piv = d[i] + t;
        if (piv == 0.0) piv = -DBL_EPSILON * (std::fabs(d[i]) + std::fabs(t)) - DBL_MIN;
        neg += piv < 0.0;
        if (i + 1 < m) t = (l2d[i] / piv) * t - sigma;
    }
    return neg;
}

void bisect_range(int m, const double* d, const double* l2d, double lo, double hi, int k0, int k1, double* out) {
    for (int k = k0; k < k1; ++k) {
        double a = lo, b = hi;
        while (true) {
            const double mid = 0.5 * (a + b);
            if (!(mid > a && mid < b)) break;
            if (inertia_below(m, d, l2d, mid) <= k) a = mid;
            else b = mid;
        }
        out[k] = 0.5 * (a + b);
    }
}

}  // namespace

// Gershgorin interval of the explicit tridiagonal of L D L^T.
static void ldl_bounds(const std::vector<double>& d, const std::vector<double>& l2, const std::vector<double>& l2d,
                       double& lo, double& hi) {
    const int m = (int)d.size();
    lo = 0.0;
    hi = 0.0;
    for (int i = 0; i < m; ++i) {
        const double diag = d[i] + (i > 0 ? l2d[i - 1] : 0.0);
        double off = 0.0;
        if (i > 0) off += std::sqrt(l2[i - 1]) * std::fabs(d[i - 1]);
        if (i + 1 < m) off += std::sqrt(l2[i]) * std::fabs(d[i]);
        if (i == 0 || diag - off < lo) lo = diag - off;
        if (i == 0 || diag + off > hi) hi = diag + off;
    }
    lo = std::min(lo, 0.0);
    hi = hi * (1.0 + 4.0 * DBL_EPSILON) + DBL_MIN;
}

void ldl_eigenvalues_range(const std::vector<double>& d, const std::vector<double>& l2, int k0, int k1,
                           double* asc, int threads) {
    const int m = (int)d.size();
    if (k1 > m) k1 = m;
    if (k0 >= k1) return;
    std::vector<double> l2d(m, 0.0);
    for (int i = 0; i + 1 < m; ++i) l2d[i] = l2[i] * d[i];
    double lo, hi;
    ldl_bounds(d, l2, l2d, lo, hi);
    const int cnt = k1 - k0;
    const int nt = std::max(1, std::min(threads, cnt / 4 + 1));
    if (nt == 1) {
        bisect_range(m, d.data(), l2d.data(), lo, hi, k0, k1, asc);
        return;
    }
    // ranges whose thread cannot be started are bisected on this thread
    std::vector<std::thread> pool;
    try {
        pool.reserve(nt);
    } catch (...) {
    }
    for (int t = 0; t < nt; ++t) {
        const int a = k0 + (int)((int64_t)cnt * t / nt), b = k0 + (int)((int64_t)cnt * (t + 1) / nt);
        bool started = false;
        try {
            pool.emplace_back(bisect_range, m, d.data(), l2d.data(), lo, hi, a, b, asc);
            started = true;
        } catch (...) {
        }
        if (!started) bisect_range(m, d.data(), l2d.data(), lo, hi, a, b, asc);
    }
    for (auto& th : pool) th.join();
}

int ldl_count_below(const std::vector<double>& d, const std::vector<double>& l2, double sigma) {
    const int m = (int)d.size();
    if (m == 0) return 0;
    std::vector<double> l2d(m, 0.0);
    for (int i = 0; i + 1 < m; ++i) l2d[i] = l2[i] * d[i];
    return inertia_below(m, d.data(), l2d.data(), sigma);
}

bool ldl_has_eigenvalue_in(const std::vector<double>& d, const std::vector<double>& l2d, double lo, double hi) {
    const int m = (int)d.size();
    if (m == 0) return false;
    // eigenvalues in [lo, hi]: count below the next double above hi, minus count below lo
    return inertia_below(m, d.data(), l2d.data(), std::nextafter(hi, INFINITY)) >
           inertia_below(m, d.data(), l2d.data(), lo);
}

void ldl_eigenvalues(const std::vector<double>& d, const std::vector<double>& l2, std::vector<double>& theta,
                     int threads) {
    const int m = (int)d.size();
    theta.assign(m, 0.0);
    if (m == 0) return;
    std::vector<double> asc(m);
    ldl_eigenvalues_range(d, l2, 0, m, asc.data(), threads);
    for (int k = 0; k < m; ++k) theta[m - 1 - k] = asc[k];
}

// Twisted factorisation of T - theta I = N_r Delta_r N_r^T: the top-down
// and bottom-up triangular factorisations meet at the index r where the
// twist element |gamma_r| is smallest; the eigenvector solves
// N_r^T z = e_r, i.e. a two-sided product recurrence from z_r = 1.
void tridiag_eigvec(const std::vector<double>& diag, const std::vector<double>& off, double theta,
                    std::vector<double>& v) {
    const int m = (int)diag.size();
    v.assign(m, 0.0);
    if (m == 0) return;
    if (m == 1) {
        v[0] = 1.0;
        return;
    }
    double tn = 0.0;
    for (int i = 0; i < m; ++i)
        tn = std::max(tn, std::fabs(diag[i]) + (i ? std::fabs(off[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(off[i]) : 0.0));
    const double tiny = DBL_EPSILON * (tn > 0 ? tn : 1.0) * 1e-3;
    auto safe = [&](double p) { return p == 0.0 ? tiny : p; };
    std::vector<double> dp(m), dm(m), lf(m), ub(m);
    dp[0] = safe(diag[0] - theta);
    for (int i = 0; i + 1 < m; ++i) {
        lf[i] = off[i] / dp[i];
        dp[i + 1] = safe(diag[i + 1] - theta - lf[i] * off[i]);
    }
    dm[m - 1] = safe(diag[m - 1] - theta);
    for (int i = m - 1; i >= 1; --i) {
        ub[i] = off[i - 1] / dm[i];
        dm[i - 1] = safe(diag[i - 1] - theta - ub[i] * off[i - 1]);
    }
    int r = 0;
    double best = INFINITY;
    for (int i = 0; i < m; ++i) {
        const double g = dp[i] + dm[i] - (diag[i] - theta);
        if (std::fabs(g) < best) {
            best = std::fabs(g);
            r = i;
        }
    }
    v[r] = 1.0;
    for (int i = r - 1; i >= 0; --i) v[i] = -lf[i] * v[i + 1];
    for (int i = r; i + 1 < m; ++i) v[i + 1] = -ub[i + 1] * v[i];
    double nrm = 0.0;
    for (double x : v) nrm += x * x;
    nrm = std::sqrt(nrm);
    int im = 0;
    for (int i = 1; i < m; ++i)
        if (std::fabs(v[i]) > std::fabs(v[im])) im = i;
    const double sc = (v[im] < 0 ? -1.0 : 1.0) / nrm;
    for (double& x : v) x *= sc;
}

std::vector<int> stagnation_select(const std::vector<double>& th_m, const std::vector<double>& th_m1, double eps) {
    const int m1 = (int)th_m1.size();
    std::vector<uint8_t> flag(th_m.size(), 0);
    for (int j = 0; j < m1; ++j) {
        if (std::fabs(th_m[j] - th_m1[j]) <= eps * std::fabs(th_m[j])) flag[j] = 1;
        if (std::fabs(th_m[j + 1] - th_m1[j]) <= eps * std::fabs(th_m[j + 1])) flag[j + 1] = 1;
    }
    std::vector<int> out;
    for (int i = 0; i < (int)flag.size(); ++i)
        if (flag[i]) out.push_back(i);
    return out;
}

}  // namespace krs
