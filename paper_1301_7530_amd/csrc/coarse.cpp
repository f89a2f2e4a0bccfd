// Coarse matrix G = C^T A C: Cholesky factorisation with a rank guard, the
// A-orthonormalising change of basis and the explicit inverse used by the
// per-iteration projector.  (Section 2.3: the coarse matrix is built and
// factored once per system; each iteration applies one coarse solve, here a
// dense matrix-vector product with the explicit inverse.)
//
// Rank guard (the paper leaves the full-rank check open, Section 2.3):
// columns are processed in order; a column whose Cholesky pivot, after
// elimination against the kept columns, is <= rank_tol * max_i G_ii is
// declared dependent and dropped.
#include <cmath>
#include <vector>

#include "internal.h"

namespace krs {

namespace {

// Guarded left-looking Cholesky.  On return idx lists the kept columns and
// Li (nk x nk, row-major, lower) holds the inverse of their factor L_k.
void guarded_factor(int nc, const double* G, double rank_tol, uint8_t* kept, std::vector<int>& idx,
                    std::vector<double>& Li) {
    double dmax = 0.0;
    for (int i = 0; i < nc; ++i) dmax = std::max(dmax, G[(size_t)i * nc + i]);
    idx.clear();
    // L[i*nc + t]: factor entry of row i in kept column t
    std::vector<double> L((size_t)nc * nc, 0.0);
    for (int j = 0; j < nc; ++j) {
        const int nk = (int)idx.size();
        double piv = G[(size_t)j * nc + j];
        for (int t = 0; t < nk; ++t) piv -= L[(size_t)j * nc + t] * L[(size_t)j * nc + t];
        if (!(piv > rank_tol * dmax)) {
            kept[j] = 0;
            continue;
        }
        kept[j] = 1;
        const double ljj = std::sqrt(piv);
        L[(size_t)j * nc + nk] = ljj;
        for (int i = j + 1; i < nc; ++i) {
            double s = G[(size_t)j * nc + i];
            for (int t = 0; t < nk; ++t) s -= L[(size_t)i * nc + t] * L[(size_t)j * nc + t];
            L[(size_t)i * nc + nk] = s / ljj;
        }
        idx.push_back(j);
    }
    const int nk = (int)idx.size();
    Li.assign((size_t)nk * nk, 0.0);
    for (int col = 0; col < nk; ++col) {
        for (int a = col; a < nk; ++a) {
            double s = (a == col) ? 1.0 : 0.0;
            const double* La = &L[(size_t)idx[a] * nc];
            for (int t = col; t < a; ++t) s -= La[t] * Li[(size_t)t * nk + col];
            Li[(size_t)a * nk + col] = s / La[a];
        }
    }
}

}  // namespace

int coarse_factor(int nc, const double* G, double rank_tol, double* Ginv, uint8_t* kept) {
    if (nc <= 0) return 0;
    std::vector<int> idx;
    std::vector<double> Li;
    guarded_factor(nc, G, rank_tol, kept, idx, Li);
    const int nk = (int)idx.size();
    for (size_t i = 0; i < (size_t)nc * nc; ++i) Ginv[i] = 0.0;
    // Ginv_k = Li^T Li
    for (int a = 0; a < nk; ++a)
        for (int b = 0; b <= a; ++b) {
            double s = 0.0;
            for (int t = a; t < nk; ++t) s += Li[(size_t)t * nk + a] * Li[(size_t)t * nk + b];
            Ginv[(size_t)idx[b] * nc + idx[a]] = s;
            Ginv[(size_t)idx[a] * nc + idx[b]] = s;
        }
    return nk;
}

// U (nc x nk, column-major) with C U = C_k L_k^{-T}: the kept columns made
// A-orthonormal (U^T G U = I up to rounding).
int coarse_orthonormalizer(int nc, const double* G, double rank_tol, double* U, uint8_t* kept) {
    if (nc <= 0) return 0;
    std::vector<int> idx;
    std::vector<double> Li;
    guarded_factor(nc, G, rank_tol, kept, idx, Li);
    const int nk = (int)idx.size();
    for (size_t i = 0; i < (size_t)nc * nk; ++i) U[i] = 0.0;
    for (int a = 0; a < nk; ++a)
        for (int t = 0; t <= a; ++t) U[(size_t)a * nc + idx[t]] = Li[(size_t)a * nk + t];
    return nk;
}

}  // namespace krs
