// Host-side Ritz analysis for selective reuse (Section 4.1 and 4.4).
//
// The Lanczos tridiagonal recovered from the CG coefficients is positive
// definite and factors as H_m = R^T R with R upper bidiagonal,
//   R_jj^2 = q_j = 1/alpha_j,   R_{j,j+1}^2 = e_j = beta_{j+1}/alpha_j,
// beta_{j+1} = rho_{j+1}/rho_j (expanding R^T R gives the diagonal
// q_j + e_{j-1} and the off-diagonal sqrt(q_j e_j) of Section 4.1).  The
// pair (q, e) is the qd array of H_m; it determines the eigenvalues to high
// relative accuracy, which the stagnation test needs for the small Ritz
// values.  Eigenvalues are counted with the progressive differential qd
// transform of R R^T - sigma I (same spectrum as R^T R): its pivots are the
// LDL^T pivots of R R^T - sigma I, so by Sylvester's law of inertia the
// number of negative pivots is the number of eigenvalues below sigma.
// Ranks are isolated by splitting intervals whose end counts are known
// (geometric midpoints once an interval is away from zero, so small values
// converge in relative terms) and refined to adjacent doubles.  Eigenvectors
// of the few selected values come from a twisted factorisation of
// T - theta I.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <limits>
#include <thread>
#include <vector>

#include "internal.h"

namespace krs {

namespace {

// Eigenvalues of the qd array (q[0..m-1], e[0..m-2]) strictly below sigma.
int pqd_negatives(const double* q, const double* e, int m, double sigma) {
    if (m <= 0) return 0;
    int neg = 0;
    double d = q[0] - sigma;
    for (int i = 0; i + 1 < m; ++i) {
        double piv = d + e[i];
        // a pivot that is exactly zero is taken as the smallest negative
        // number (the count of a sigma perturbed by less than an ulp); the
        // next pivot then overflows to +inf, whose limit is handled below
        if (piv == 0.0) piv = -std::numeric_limits<double>::denorm_min();
        neg += piv < 0.0;
        d = std::isinf(piv) ? q[i + 1] - sigma : d * (q[i + 1] / piv) - sigma;
    }
    neg += d < 0.0;
    return neg;
}

// Upper bound of the spectrum: Gershgorin discs of R R^T, whose diagonal is
// q_i + e_i and off-diagonal sqrt(e_i q_{i+1}); widened until every
// eigenvalue counts below it.
double qd_upper(const double* q, const double* e, int m) {
    double hi = 0.0;
    for (int i = 0; i < m; ++i) {
        const double ei = (i + 1 < m) ? e[i] : 0.0;
        double r = q[i] + ei;
        if (i > 0) r += std::sqrt(e[i - 1] * q[i]);
        if (i + 1 < m) r += std::sqrt(ei * q[i + 1]);
        hi = std::max(hi, r);
    }
    hi = hi * (1.0 + 16.0 * DBL_EPSILON) + DBL_MIN;
    for (int t = 0; t < 64 && pqd_negatives(q, e, m, hi) < m; ++t) hi *= 2.0;
    return hi;
}

inline double split_point(double a, double b) {
    // geometric midpoint while the interval spans more than a factor 2 away
    // from zero (relative convergence of small values), arithmetic otherwise
    if (a > 0.0 && b > 2.0 * a) return std::sqrt(a) * std::sqrt(b);
    return a + 0.5 * (b - a);
}

// Eigenvalues of ascending ranks k0..k1-1 into out[k] (absolute index).
void rank_range(const double* q, const double* e, int m, double hi, int k0, int k1, double* out) {
    struct Interval {
        double a, b;
        int below_a, below_b;  // eigenvalues below a, below b: ranks [below_a, below_b) lie in [a, b)
    };
    std::vector<Interval> work;
    work.push_back({0.0, hi, 0, m});
    while (!work.empty()) {
        const Interval iv = work.back();
        work.pop_back();
        if (iv.below_b <= k0 || iv.below_a >= k1 || iv.below_b == iv.below_a) continue;
        const double mid = split_point(iv.a, iv.b);
        if (!(mid > iv.a && mid < iv.b)) {
            // adjacent doubles: every rank inside takes the interval's centre
            const double v = iv.a + 0.5 * (iv.b - iv.a);
            for (int k = std::max(iv.below_a, k0); k < std::min(iv.below_b, k1); ++k) out[k] = v;
            continue;
        }
        const int c = std::min(std::max(pqd_negatives(q, e, m, mid), iv.below_a), iv.below_b);
        work.push_back({mid, iv.b, c, iv.below_b});
        work.push_back({iv.a, mid, iv.below_a, c});
    }
}

}  // namespace

QdArray qd_from_cg(const double* alpha, const double* rho, int m) {
    QdArray z;
    z.q.resize(std::max(m, 0));
    z.e.resize(std::max(m - 1, 0));
    for (int j = 0; j < m; ++j) z.q[j] = 1.0 / alpha[j];
    for (int j = 0; j + 1 < m; ++j) z.e[j] = (rho[j + 1] / rho[j]) * z.q[j];
    return z;
}

QdArray qd_leading(const QdArray& z, int m1) {
    QdArray t;
    m1 = std::max(0, std::min(m1, (int)z.q.size()));
    t.q.assign(z.q.begin(), z.q.begin() + m1);
    t.e.assign(z.e.begin(), z.e.begin() + std::max(m1 - 1, 0));
    return t;
}

int qd_count_below(const QdArray& z, double sigma) {
    return pqd_negatives(z.q.data(), z.e.data(), (int)z.q.size(), sigma);
}

bool qd_has_eigenvalue_in(const QdArray& z, double lo, double hi) {
    const int m = (int)z.q.size();
    if (m == 0) return false;
    return pqd_negatives(z.q.data(), z.e.data(), m, std::nextafter(hi, INFINITY)) >
           pqd_negatives(z.q.data(), z.e.data(), m, lo);
}

void qd_eigenvalues_asc(const QdArray& z, int k0, int k1, double* out, int threads) {
    const int m = (int)z.q.size();
    k1 = std::min(k1, m);
    k0 = std::max(k0, 0);
    if (k0 >= k1) return;
    const double* q = z.q.data();
    const double* e = z.e.data();
    const double hi = qd_upper(q, e, m);
    const int cnt = k1 - k0;
    const int nt = std::max(1, std::min(threads, cnt / 8 + 1));
    if (nt == 1) {
        rank_range(q, e, m, hi, k0, k1, out);
        return;
    }
    // rank chunks on threads; a chunk whose thread cannot start runs here
    std::vector<std::thread> pool;
    try {
        pool.reserve(nt);
    } catch (...) {
    }
    for (int t = 0; t < nt; ++t) {
        const int a = k0 + (int)((int64_t)cnt * t / nt), b = k0 + (int)((int64_t)cnt * (t + 1) / nt);
        bool started = false;
        try {
            pool.emplace_back(rank_range, q, e, m, hi, a, b, out);
            started = true;
        } catch (...) {
        }
        if (!started) rank_range(q, e, m, hi, a, b, out);
    }
    for (auto& th : pool) th.join();
}

void qd_eigenvalues_desc(const QdArray& z, std::vector<double>& theta, int threads) {
    const int m = (int)z.q.size();
    theta.assign(m, 0.0);
    if (m == 0) return;
    std::vector<double> asc(m);
    qd_eigenvalues_asc(z, 0, m, asc.data(), threads);
    for (int k = 0; k < m; ++k) theta[m - 1 - k] = asc[k];
}

// n_c_lim by a complexity analysis (Section 4.4, after Algorithm 3).  The
// m_0 iterations of the given solve stand for every non-augmented system.
// Deflating the eigenvectors of the k lowest eigenvalues leaves the CG rate
// of the reduced condition number theta_max / theta_(k+1) (Section 2.2 and
// the rate of Section 4.3), so an augmented solve is modelled at
//   m(k) = max(1, m_0 ln(sigma_0) / ln(sigma_k)),  sigma = (sqrt(kappa)-1)/(sqrt(kappa)+1),
// iterations over the distinct Ritz values (finite-precision Lanczos
// repeats converged values: a value within a relative 1e-10 of the last
// kept one is a copy); only converged Ritz vectors approximate
// eigenvectors (the stagnation test at eps), so k deflates the converged
// prefix of the ascending values and columns past it gain nothing.  It moves
//   T(k) = m(k) (bytes_iter0 + k bytes_col_iter) + [k > 0] (bytes_rebuild0 + k bytes_col_rebuild)
// bytes per system.  n_c_lim minimises T over k = 0..kmax (the smaller k on
// a tie).  Only the low end of the spectrum and its top are computed.
int nc_limit(const double* alpha, const double* rho, int m, const NcCostModel& cm, int threads,
             std::vector<double>* cost) {
    if (cost) cost->clear();
    if (m <= 0) return 0;
    const QdArray z = qd_from_cg(alpha, rho, m);
    const QdArray z1 = qd_leading(z, std::max(m - 1, 0));
    std::vector<double> asc(m, 0.0);  // out[k] at the absolute rank k
    qd_eigenvalues_asc(z, m - 1, m, asc.data(), 1);
    const double top = asc[m - 1];
    // distinct values ascending (a value within a relative 1e-10 of the
    // last kept one is a Lanczos copy), each marked converged if it or a
    // copy passes the stagnation test: H_{m-1} has an eigenvalue within
    // eps |theta| (one of its interlacing neighbours)
    std::vector<double> distinct;
    std::vector<uint8_t> conv;
    const int want = std::max(0, cm.kmax) + 1;
    const int CH = 256;
    for (int k = 0; k < m && (int)distinct.size() < want; k += CH) {
        const int k1 = std::min(m, k + CH);
        qd_eigenvalues_asc(z, k, k1, asc.data(), threads);
        for (int t = k; t < k1; ++t) {
            const double a = asc[t];
            const double e = cm.eps * std::fabs(a);
            const bool c = m > 1 && qd_has_eigenvalue_in(z1, a - e, a + e);
            if (!distinct.empty() && std::fabs(a - distinct.back()) <= 1e-10 * std::fabs(a)) {
                conv.back() = conv.back() || c;
                continue;
            }
            if ((int)distinct.size() >= want) break;
            distinct.push_back(a);
            conv.push_back(c);
        }
    }
    int kconv = 0;
    while (kconv < (int)conv.size() && conv[kconv]) ++kconv;
    const int kmax = std::min(std::max(0, cm.kmax), (int)distinct.size() - 1);
    auto log_rate = [](double kappa) {
        if (!(kappa > 1.0)) return -std::numeric_limits<double>::infinity();
        const double r = std::sqrt(kappa);
        return std::log((r - 1.0) / (r + 1.0));
    };
    const double l0 = log_rate(top / distinct[0]);
    int best = 0;
    double best_t = 0.0;
    for (int k = 0; k <= kmax; ++k) {
        // columns past the converged prefix deflate nothing more
        const double lk = log_rate(top / distinct[std::min(k, kconv)]);
        const double mk = std::isfinite(lk) ? std::max(1.0, (double)m * (l0 / lk)) : 1.0;
        const double t = mk * (cm.bytes_iter0 + k * cm.bytes_col_iter) +
                         (k > 0 ? cm.bytes_rebuild0 + k * cm.bytes_col_rebuild : 0.0);
        if (cost) cost->push_back(t);
        if (k == 0 || t < best_t) {
            best = k;
            best_t = t;
        }
    }
    return best;
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

// Reselection by cluster identification (Section 4.4, "clust"): of the
// preselected Ritz values, drop the central cluster.  The sorted values'
// neighbour distances on a log scale are fitted, in least squares, by a
// three-level step function (outer levels over the low and high ends, which
// may be empty but not both, and a middle level over at least
// ceil(min_frac * s) values); when the middle level lies below the outer
// ones its values are the cluster.  Exhaustive over the two breakpoints
// with running sums (s is at most a few hundred).
std::vector<int> cluster_reselect(const std::vector<double>& theta, const std::vector<int>& sel, double min_frac) {
    const int s = (int)sel.size();
    if (s < 3) {
        std::vector<int> out(sel);
        std::sort(out.begin(), out.end());
        return out;
    }
    std::vector<int> ord(sel);
    std::sort(ord.begin(), ord.end(), [&](int i, int j) {
        if (theta[i] != theta[j]) return theta[i] < theta[j];
        return i < j;
    });
    const int G = s - 1;
    std::vector<long double> S1(G + 1, 0.0L), S2(G + 1, 0.0L);
    for (int i = 0; i < G; ++i) {
        const double d = std::log(theta[ord[i + 1]] / theta[ord[i]]);
        S1[i + 1] = S1[i] + d;
        S2[i + 1] = S2[i] + (long double)d * d;
    }
    auto piece = [&](int i, int j) -> long double {  // squared deviation of g[i..j)
        if (j <= i) return 0.0L;
        const long double t = S1[j] - S1[i];
        return (S2[j] - S2[i]) - t * t / (j - i);
    };
    const int L = std::max(1, (int)std::ceil(min_frac * s - 1e-9));
    int ba = -1, bb = -1;
    long double best = 0.0L;
    for (int a = 0; a <= G; ++a)
        for (int b = std::max(a + 1, a + L - 1); b <= G; ++b) {
            if (a == 0 && b == G) continue;
            const long double c = piece(0, a) + piece(a, b) + piece(b, G);
            if (ba < 0 || c < best) {
                best = c;
                ba = a;
                bb = b;
            }
        }
    std::vector<int> out;
    bool drop_mid = ba >= 0;
    if (drop_mid) {
        const long double mid = (S1[bb] - S1[ba]) / (bb - ba);
        if (ba > 0 && !(mid < S1[ba] / ba)) drop_mid = false;
        if (bb < G && !(mid < (S1[G] - S1[bb]) / (G - bb))) drop_mid = false;
    }
    std::vector<uint8_t> dropped(theta.size(), 0);
    if (drop_mid)
        for (int t = ba; t <= bb; ++t) dropped[ord[t]] = 1;
    for (int i : sel)
        if (!dropped[i]) out.push_back(i);
    std::sort(out.begin(), out.end());
    return out;
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
