"""Pins of the oracle's Ritz analysis and reuse logic (Sections 3 and 4):
the Lanczos tridiagonal recovered from the CG coefficients, Ritz values in
closed form, interlacing, relative accuracy of the eigenvalue routine, the
stagnation selection and its edge cases, the Ritz-vector normalisation and
the TRKS independence relation.
"""
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

import gen
import oracle as O


def _csr(A):
    S = sp.csr_matrix(A)
    S.sort_indices()
    return S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.float64)


def _lap3(N):
    rp, ci, v = gen.diffusion_matrix(np.ones((N, N, N)))
    return rp, ci, v


def _lanczos_V(r):
    m = r["m"]
    sgn = np.where(np.arange(m) % 2 == 0, 1.0, -1.0)
    return r["Z"][:, :m] * (sgn / np.sqrt(r["rho"][:m]))[None, :]


def test_lanczos_matrix_from_cg_coefficients():
    """V^T A V = H_m and V^T M V = I (Section 4.1, C = 0)."""
    seq = gen.config_diffusion_20(N=6)
    rp, ci, v, b = seq.csr(0)
    A = sp.csr_matrix((v, ci, rp)).toarray()
    r = O.apcg(rp, ci, v, b, "jacobi", tol=1e-300, max_iter=15, record_z=True)
    V = _lanczos_V(r)
    delta, eta = O.lanczos_tridiag(r["alpha"], r["rho"])
    H = np.diag(delta) + np.diag(eta, 1) + np.diag(eta, -1)
    assert np.abs(V.T @ A @ V - H).max() <= 1e-10 * np.abs(H).max()
    M = np.diag(np.diag(A))
    assert np.abs(V.T @ M @ V - np.eye(r["m"])).max() <= 1e-10
    assert np.all(eta > 0)


def test_ritz_vectors_with_augmentation():
    """Y^T A Y = Theta also holds with C != 0; Y^T M Y = I holds only for C = 0."""
    seq = gen.config_diffusion_20(N=6)
    rp, ci, v, b = seq.csr(0)
    A = sp.csr_matrix((v, ci, rp)).toarray()
    C = np.random.default_rng(1).standard_normal((seq.n, 4))
    r = O.apcg(rp, ci, v, b, "jacobi", C=C, tol=1e-300, max_iter=12, record_z=True)
    V = _lanczos_V(r)
    delta, eta = O.lanczos_tridiag(r["alpha"], r["rho"])
    th, Q = np.linalg.eigh(np.diag(delta) + np.diag(eta, 1) + np.diag(eta, -1))
    Y = V @ Q
    assert np.abs(Y.T @ A @ Y - np.diag(th)).max() <= 1e-9 * th.max()
    assert np.abs(C.T @ A @ Y).max() <= 1e-9 * np.linalg.norm(C) * np.linalg.norm(A @ Y)


def test_ritz_values_closed_form_1d_laplacian():
    n = 32
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    b = np.random.default_rng(2).standard_normal(n)
    r = O.apcg(*_csr(A), b, "none", tol=1e-300, max_iter=n)
    th, _ = O.ritz_values(r["alpha"], r["rho"])
    exact = 2 - 2 * np.cos(np.arange(n, 0, -1) * np.pi / (n + 1))
    assert np.abs(th - exact).max() <= 1e-12


def test_ritz_extremes_3d_laplacian_jacobi():
    """7-point Laplacian N = 10 with Jacobi (M = 6I): extreme eigenvalues
    3(2 -+ 2cos(pi/11))/6 are captured by the Ritz values."""
    N = 10
    rp, ci, v = _lap3(N)
    b = np.random.default_rng(3).standard_normal(N ** 3)
    r = O.apcg(rp, ci, v, b, "jacobi", tol=1e-10, max_iter=500)
    th, _ = O.ritz_values(r["alpha"], r["rho"])
    lo = 3 * (2 - 2 * np.cos(np.pi / 11)) / 6
    hi = 3 * (2 + 2 * np.cos(np.pi / 11)) / 6
    assert lo == pytest.approx(0.0405070, abs=1e-7)
    assert th[-1] == pytest.approx(lo, rel=1e-10)
    assert th[0] == pytest.approx(hi, rel=1e-10)


def test_interlacing():
    seq = gen.config_diffusion_20(N=8)
    rp, ci, v, b = seq.csr(0)
    r = O.apcg(rp, ci, v, b, "jacobi", tol=1e-8, max_iter=400)
    th_m, th_m1 = O.ritz_values(r["alpha"], r["rho"])
    m = len(th_m)
    assert len(th_m1) == m - 1 and np.all(np.diff(th_m) <= 0)
    for j in range(m - 1):
        assert th_m[j] >= th_m1[j] * (1 - 1e-15) and th_m1[j] >= th_m[j + 1] * (1 - 1e-15)


def test_ldl_eigenvalues_match_explicit_tridiagonal():
    seq = gen.config_diffusion_20(N=8)
    rp, ci, v, b = seq.csr(1)
    r = O.apcg(rp, ci, v, b, "jacobi", tol=1e-8, max_iter=400)
    th, _ = O.ritz_values(r["alpha"], r["rho"])
    delta, eta = O.lanczos_tridiag(r["alpha"], r["rho"])
    ref = sl.eigh_tridiagonal(delta, eta, eigvals_only=True)[::-1]
    assert np.abs(th - ref).max() <= 1e-13 * th[0]
    # the oracle's own dense Jacobi-rotation solver agrees too
    H = np.diag(delta) + np.diag(eta, 1) + np.diag(eta, -1)
    jac = O.jacobi_eigvals(H[:40, :40])[::-1]
    ref40 = sl.eigh_tridiagonal(delta[:40], eta[:39], eigvals_only=True)[::-1]
    assert np.abs(jac - ref40).max() <= 1e-13 * ref40[0]


def test_ldl_eigenvalues_high_relative_accuracy():
    """With d spanning 12 orders of magnitude the smallest eigenvalue is
    recovered to ~1e-13 relative; the reference is 1/lambda_max(T^-1) with
    T^-1 = L^-T D^-1 L^-1 formed from positive products only."""
    rng = np.random.default_rng(4)
    m = 40
    d = np.geomspace(1e-12, 1.0, m)[rng.permutation(m)]
    l2 = rng.uniform(0.1, 2.0, m - 1)
    th = O.ldl_eigvals(d, l2)
    # L with sub-diagonal -sqrt(l2) (same eigenvalues) has an entrywise positive inverse
    Linv = np.eye(m)
    for i in range(1, m):
        Linv[i, :i] = np.sqrt(l2[i - 1]) * Linv[i - 1, :i]
    Tinv = Linv.T @ np.diag(1.0 / d) @ Linv
    assert np.all(Tinv > 0)
    lam_max_inv = np.linalg.eigvalsh(Tinv)[-1]
    assert th[-1] == pytest.approx(1.0 / lam_max_inv, rel=1e-12)
    # counts are consistent with the returned values
    for k in (0, 5, m - 1):
        assert O.lib().orc_ldl_count(m, O._p(np.ascontiguousarray(d)), O._p(np.ascontiguousarray(l2)),
                                     th[m - 1 - k] * (1 + 1e-12)) == k + 1


def test_tridiagonal_eigenvector():
    rng = np.random.default_rng(5)
    m = 30
    dg = rng.uniform(1, 3, m)
    of = rng.uniform(0.1, 0.5, m - 1)
    th, Q = sl.eigh_tridiagonal(dg, of)
    for i in (0, 7, m - 1):
        v = O.tridiag_eigvec(dg, of, th[i])
        assert abs(abs(v @ Q[:, i]) - 1.0) <= 1e-12


def test_selection_edge_cases():
    assert O.srks_select(np.array([]), np.array([]), 1e-14) == []
    assert O.srks_select(np.array([2.0]), np.array([]), 1e-14) == []
    # m = 2: j = 0 tests theta_m[0] vs theta_{m-1}[0] and theta_m[1] vs theta_{m-1}[0]
    assert O.srks_select(np.array([3.0, 1.0]), np.array([3.0]), 1e-14) == [0]
    assert O.srks_select(np.array([3.0, 1.0]), np.array([1.0]), 1e-14) == [1]
    # inclusive boundary, relative to |theta_m|
    eps = 0.25
    assert O.srks_select(np.array([4.0, 1.0]), np.array([3.0]), eps) == [0]
    assert O.srks_select(np.array([4.0, 1.0]), np.array([2.999]), eps) == []
    # an index found twice (as j+1 at step j and as j at step j+1) is taken once
    th_m = np.array([5.0, 3.0, 1.0])
    th_m1 = np.array([3.0, 3.0])
    assert O.srks_select(th_m, th_m1, 1e-14) == [1]


def test_selection_matches_dense_bruteforce():
    seq = gen.config_diffusion_20(N=8)
    rp, ci, v, b = seq.csr(0)
    r = O.apcg(rp, ci, v, b, "jacobi", tol=1e-10, max_iter=400)
    delta, eta = O.lanczos_tridiag(r["alpha"], r["rho"])
    m = len(delta)
    H = np.diag(delta) + np.diag(eta, 1) + np.diag(eta, -1)
    ref_m = np.linalg.eigvalsh(H)[::-1]
    ref_m1 = np.linalg.eigvalsh(H[: m - 1, : m - 1])[::-1]
    th_m, th_m1 = O.ritz_values(r["alpha"], r["rho"])
    for eps in (1e-4, 1e-6, 1e-8):
        brute = O.srks_select(ref_m, ref_m1, eps)
        mine = O.srks_select(th_m, th_m1, eps)
        assert mine == brute and len(mine) > 0


def test_srks_block_normalisation_constant_operator():
    """With A unchanged, the new coarse block Y^T A Y / |theta| is ~ I for
    converged Ritz vectors (Section 4.4, normalisation by sqrt(|theta|))."""
    seq = gen.config_diffusion_20(N=8)
    rp, ci, v, b = seq.csr(0)
    A = sp.csr_matrix((v, ci, rp))
    r = O.apcg(rp, ci, v, b, "jacobi", tol=1e-10, max_iter=400, record_z=True)
    th_m, th_m1 = O.ritz_values(r["alpha"], r["rho"])
    sel = O.srks_select(th_m, th_m1, 1e-8)
    assert len(sel) >= 2
    Cn = O.ritz_block(r["Z"], r["alpha"], r["rho"], sel, th_m)
    G = Cn.T @ (A @ Cn)
    assert np.abs(np.diag(G) - 1).max() <= 1e-6
    assert np.abs(G - np.diag(np.diag(G))).max() <= 1e-6


def test_trks_independence_relation():
    """C^(k)T A^(k) W^(k) = 0 (Section 3) and TRKS columns are A-normalised."""
    seq = gen.config_diffusion_20(N=6)
    recs, C = O.solve_sequence(seq, 2, reuse="trks")
    rp, ci, v, b = seq.csr(1)
    A1 = sp.csr_matrix((v, ci, rp))
    C1 = C[:, : recs[1]["nc"]]
    r = O.apcg(rp, ci, v, b, "jacobi", C=C1, tol=1e-8, max_iter=400, record_w=True)
    W = r["W"]
    rel = np.abs(C1.T @ (A1 @ W)) / np.outer(np.sqrt(np.einsum("ij,ij->j", C1, A1 @ C1)), np.sqrt(r["gamma"]))
    assert rel.max() <= 1e-8
    Wn = O.trks_block(W, r["gamma"])
    assert np.allclose(np.einsum("ij,ij->j", Wn, A1 @ Wn), 1.0, rtol=1e-12)


def test_trks_multiple_rhs_iterations_non_increasing():
    N = 6
    rp, ci, v = _lap3(N)

    class Fixed:
        n = N ** 3
        block = 1
        n_systems = 4

        def csr(self, k):
            return rp, ci, v, np.random.default_rng(100 + k).standard_normal(N ** 3)

    recs, _ = O.solve_sequence(Fixed(), reuse="trks")
    ms = [r["m"] for r in recs]
    assert all(b <= a for a, b in zip(ms, ms[1:])) and ms[-1] < ms[0]
    assert all(r["relres_true"] <= 1e-8 * 1.01 for r in recs)


def test_cap_policies():
    seq = gen.config_diffusion_20(N=6)
    recs, C = O.solve_sequence(seq, 3, reuse="trks", cap=30, cap_policy="freeze")
    assert recs[0]["nc_next"] == 30 and recs[1]["added"] == 0 and C.shape[1] == 30
    recs, C = O.solve_sequence(seq, 3, reuse="trks", cap=30, cap_policy="restart")
    assert recs[0].get("restarted") and recs[1]["nc"] == 0
    # freeze keeps the smallest Ritz values first
    th = np.array([5.0, 4.0, 3.0, 2.0, 1.0])
    assert O.freeze_pick([0, 1, 3, 4], th, 2) == [3, 4]
    assert O.freeze_pick([0, 1], th, 0) == []
