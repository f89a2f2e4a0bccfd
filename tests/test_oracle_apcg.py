"""Pins of the oracle's APCG solve (Algorithm 1, Section 2) against what the
paper and the mathematics fix: dense solves, exact termination, the basic
orthogonality relations, the projector identities, Propositions 1 and 3,
Corollary 2, the printed Gram-Schmidt form, and the CG bound of Section 4.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle as O


def _csr(A):
    S = sp.csr_matrix(A)
    S.sort_indices()
    return S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.float64)


def _rand_spd(n, kappa, rng):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, kappa, n)
    return (Q * ev) @ Q.T


def _proj(A, C):
    G = C.T @ A @ C
    return np.eye(A.shape[0]) - C @ np.linalg.solve(G, C.T @ A)


def test_dense_cholesky_solve_matches_numpy():
    rng = np.random.default_rng(1)
    A = _rand_spd(20, 1e3, rng)
    b = rng.standard_normal(20)
    x = O.dense_cholesky_solve(A, b)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    with pytest.raises(ValueError):
        O.dense_cholesky_solve(-A, b)


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_pcg_solution_matches_dense_solve(precond):
    rng = np.random.default_rng(2)
    n, kappa = 48, 1e4
    A = _rand_spd(n, kappa, rng)
    A += np.diag(rng.uniform(0.5, 2.0, n))  # distinct diagonal for Jacobi
    b = rng.standard_normal(n)
    r = O.apcg(*_csr(A), b, precond, tol=1e-12, max_iter=4 * n)
    xs = np.linalg.solve(A, b)
    assert r["status"] == O.ORC_OK
    assert np.linalg.norm(r["x"] - xs) / np.linalg.norm(xs) <= 1e-8 * kappa
    assert r["relres_true"] <= 1e-11


def test_exact_termination_distinct_eigenvalues():
    # diagonal matrix with d distinct eigenvalues: CG terminates in d steps
    d = 7
    vals = np.repeat(np.linspace(1.0, 10.0, d), 5)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((len(vals), len(vals))))
    A = (Q * vals) @ Q.T
    b = rng.standard_normal(len(vals))
    r = O.apcg(*_csr(A), b, "none", tol=1e-12, max_iter=50)
    assert r["m"] == d
    assert r["resnorm"][d - 1] > 1e-6 * r["resnorm"][0]


def test_augmented_exact_termination():
    # kappa = 10 keeps the loss of orthogonality of finite-precision CG
    # below what would delay termination past n - n_c steps
    rng = np.random.default_rng(4)
    n, nc = 32, 5
    A = _rand_spd(n, 10.0, rng)
    C = rng.standard_normal((n, nc))
    b = rng.standard_normal(n)
    r = O.apcg(*_csr(A), b, "none", C=C, tol=1e-12, max_iter=n)
    assert r["status"] == O.ORC_OK and r["m"] <= n - nc
    assert r["relres_true"] <= 1e-11


def test_orthogonality_relations_and_projector():
    """(r_i, z_j) = 0, (w_i, A w_j) = 0 for i != j; C^T A w_j = 0, C^T r = 0."""
    rng = np.random.default_rng(5)
    n, nc = 40, 4
    A = _rand_spd(n, 50.0, rng)
    A += np.diag(rng.uniform(0.5, 1.5, n))
    C = rng.standard_normal((n, nc))
    b = rng.standard_normal(n)
    r = O.apcg(*_csr(A), b, "jacobi", C=C, tol=1e-300, max_iter=12, record_z=True, record_w=True)
    W, Z = r["W"], r["Z"]
    G = W.T @ A @ W
    dn = np.sqrt(np.diag(G))
    off = G / np.outer(dn, dn) - np.eye(W.shape[1])
    assert np.abs(off).max() <= 1e-10
    # C^T A w_j = 0 and C^T A z_j = 0 (C^T A P = 0)
    for M in (W, Z):
        assert np.abs(C.T @ A @ M).max() <= 1e-10 * np.linalg.norm(C) * np.linalg.norm(A @ M)
    # residuals rebuilt from the recursion: r_j = b - A x_j; C^T r_final = 0
    res_final = b - A @ r["x"]
    assert np.abs(C.T @ res_final).max() <= 1e-12 * np.linalg.norm(C) * max(np.linalg.norm(b), 1.0)
    # (r_i, z_j) = 0 for i != j, with r_j = b - A x_j rebuilt from
    # x_j = x_0 + sum_{k<j} alpha_k w_k
    G0 = C.T @ A @ C
    x = C @ np.linalg.solve(G0, C.T @ b)
    R = []
    for j in range(W.shape[1]):
        R.append(b - A @ x)
        x = x + r["alpha"][j] * W[:, j]
    R = np.array(R).T
    RZ = R.T @ Z
    rd = np.sqrt(np.abs(np.diag(RZ)))
    assert np.abs(RZ / np.outer(rd, rd) - np.diag(np.sign(np.diag(RZ)))).max() <= 1e-9
    assert np.allclose(np.diag(RZ), r["rho"], rtol=1e-10)
    assert np.abs(C.T @ R).max() <= 1e-10 * np.linalg.norm(C) * np.linalg.norm(b)


def test_dense_projector_identities():
    """P C = 0, P^2 = P, A P = P^T A P = P^T A (Section 2.1)."""
    rng = np.random.default_rng(6)
    n, nc = 12, 3
    A = _rand_spd(n, 20.0, rng)
    C = rng.standard_normal((n, nc))
    P = _proj(A, C)
    assert np.abs(P @ C).max() < 1e-12
    assert np.abs(P @ P - P).max() < 1e-12
    assert np.abs(A @ P - P.T @ A @ P).max() < 1e-12
    assert np.abs(A @ P - P.T @ A).max() < 1e-12
    assert np.abs(C.T @ A @ P).max() < 1e-12


def test_proposition1_equivalence_with_projected_cg():
    """APCG(A, I, C, b) and CG(P^T A P, P^T b) produce the same residuals."""
    rng = np.random.default_rng(7)
    n, nc = 30, 4
    A = _rand_spd(n, 200.0, rng)
    C = rng.standard_normal((n, nc))
    b = rng.standard_normal(n)
    P = _proj(A, C)
    k = 10
    ra = O.apcg(*_csr(A), b, "none", C=C, tol=1e-300, max_iter=k)
    B = P.T @ A @ P
    B = 0.5 * (B + B.T)
    rb = O.apcg(*_csr(B), P.T @ b, "none", tol=1e-300, max_iter=k)
    assert np.allclose(ra["resnorm"], rb["resnorm"], rtol=1e-8)
    assert np.allclose(ra["alpha"], rb["alpha"], rtol=1e-8)


def test_corollary2_nested_augmentation():
    """APCG(A, I, [C, D], b) == APCG(P^T A P, I, D, P^T b) (same residuals)."""
    rng = np.random.default_rng(8)
    n = 30
    A = _rand_spd(n, 200.0, rng)
    C = rng.standard_normal((n, 3))
    Dm = rng.standard_normal((n, 2))
    b = rng.standard_normal(n)
    P = _proj(A, C)
    k = 8
    ra = O.apcg(*_csr(A), b, "none", C=np.hstack([C, Dm]), tol=1e-300, max_iter=k)
    B = P.T @ A @ P
    # P^T A P is singular on range(C); Dm restricted to range(P) gives the same augmentation
    B = 0.5 * (B + B.T)
    rb = O.apcg(*_csr(B + 0.0), P.T @ b, "none", C=P @ Dm, tol=1e-300, max_iter=k)
    assert np.allclose(ra["resnorm"][1:], rb["resnorm"][1:], rtol=1e-7)


def test_proposition3_preconditioned_equivalence():
    """APCG(A, M, C, b) == APCG(L^-1 A L^-T, I, L^T C, L^-1 b): same alpha, beta."""
    rng = np.random.default_rng(9)
    n, nc = 36, 3
    A = _rand_spd(n, 100.0, rng) + np.diag(rng.uniform(1, 5, n))
    C = rng.standard_normal((n, nc))
    b = rng.standard_normal(n)
    L = np.sqrt(np.diag(A))  # M = diag(A) = L L^T
    k = 12
    ra = O.apcg(*_csr(A), b, "jacobi", C=C, tol=1e-300, max_iter=k)
    Ah = A / np.outer(L, L)
    rb = O.apcg(*_csr(Ah), b / L, "none", C=C * L[:, None], tol=1e-300, max_iter=k)
    assert np.allclose(ra["alpha"], rb["alpha"], rtol=1e-9)
    beta_a = ra["rho"][1:] / ra["rho"][:-1]
    beta_b = rb["rho"][1:] / rb["rho"][:-1]
    assert np.allclose(beta_a, beta_b, rtol=1e-9)


def test_block_jacobi_preconditioner_first_direction():
    """z_0 = M^-1 b with M the 3x3 diagonal blocks (no augmentation)."""
    rng = np.random.default_rng(10)
    n = 18
    A = _rand_spd(n, 30.0, rng) + np.eye(n) * 3
    b = rng.standard_normal(n)
    r = O.apcg(*_csr(A), b, "block3", tol=1e-300, max_iter=1, record_z=True)
    z0 = np.concatenate([np.linalg.solve(A[3 * p:3 * p + 3, 3 * p:3 * p + 3], b[3 * p:3 * p + 3]) for p in range(n // 3)])
    assert np.allclose(r["Z"][:, 0], z0, rtol=1e-12)


def test_printed_gram_schmidt_form_agrees():
    """Algorithm 1's Gram-Schmidt beta is minus the standard beta; alphas agree."""
    rng = np.random.default_rng(11)
    n, nc = 40, 3
    A = _rand_spd(n, 100.0, rng) + np.diag(rng.uniform(1, 3, n))
    C = rng.standard_normal((n, nc))
    b = rng.standard_normal(n)
    k = 10
    rs = O.apcg(*_csr(A), b, "jacobi", C=C, tol=1e-300, max_iter=k)
    x1, a1, bgs = O.apcg_alg1(*_csr(A), b, k, "jacobi", C=C)
    assert np.allclose(a1, rs["alpha"], rtol=1e-10)
    beta_std = rs["rho"][1:] / rs["rho"][:-1]
    assert np.allclose(bgs[1:k], -beta_std[: k - 1], rtol=1e-9)
    assert np.allclose(x1, rs["x"], rtol=1e-10, atol=1e-12)


def test_deflation_with_exact_eigenvectors():
    """C = n_c lowest eigenvectors: the effective spectrum is [lambda_{nc+1}, lambda_n]
    (reading of Section 2.2: kappa = lambda_n / lambda_{n_c+1})."""
    n, nc = 60, 6
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    lam = 2 - 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    V = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(np.arange(1, n + 1), np.arange(1, n + 1)) * np.pi / (n + 1))
    C = V[:, :nc]
    b = np.random.default_rng(12).standard_normal(n)
    r = O.apcg(*_csr(A), b, "none", C=C, tol=1e-300, max_iter=n - nc)
    th, _ = O.ritz_values(r["alpha"], r["rho"])
    assert th[-1] == pytest.approx(lam[nc], rel=1e-9)
    assert th[0] == pytest.approx(lam[-1], rel=1e-9)
    # and the error reduction obeys the CG bound with kappa = lam_n / lam_{nc+1}
    kappa = lam[-1] / lam[nc]
    xs = np.linalg.solve(A, b)
    x0 = C @ np.linalg.solve(C.T @ A @ C, C.T @ b)
    e0 = xs - x0
    eA0 = np.sqrt(e0 @ A @ e0)
    for i in (5, 10, 15):
        ri = O.apcg(*_csr(A), b, "none", C=C, tol=1e-300, max_iter=i)
        e = xs - ri["x"]
        sigma = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
        assert np.sqrt(e @ A @ e) / eA0 <= 2 * sigma ** i * (1 + 1e-9)


def test_cg_iteration_bound_on_laplacian():
    """Section 4 bound: A-norm error reduced by eps within n_eps iterations."""
    N = 8
    I = np.eye(N)
    T = 2 * I - np.eye(N, k=1) - np.eye(N, k=-1)
    A = np.kron(np.kron(T, I), I) + np.kron(np.kron(I, T), I) + np.kron(np.kron(I, I), T)
    lam = 2 - 2 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    kappa = lam[-1] / lam[0]
    eps = 1e-6
    nbound = O.cg_iteration_bound(kappa, eps)
    b = np.random.default_rng(13).standard_normal(N ** 3)
    xs = np.linalg.solve(A, b)
    k = int(np.ceil(nbound))
    r = O.apcg(*_csr(A), b, "none", tol=1e-300, max_iter=k)
    e = xs - r["x"]
    assert np.sqrt(e @ A @ e) / np.sqrt(xs @ A @ xs) <= eps


def test_rank_guard_drops_duplicate_column():
    rng = np.random.default_rng(14)
    n = 30
    A = _rand_spd(n, 50.0, rng)
    c = rng.standard_normal((n, 2))
    C = np.hstack([c, c[:, :1] * 2.0, rng.standard_normal((n, 1))])
    b = rng.standard_normal(n)
    r = O.apcg(*_csr(A), b, "none", C=C, tol=1e-10, max_iter=3 * n)
    assert list(r["kept"]) == [True, True, False, True]
    assert r["status"] == O.ORC_OK and r["relres_true"] <= 1e-9


def test_breakdown_on_indefinite_matrix():
    A = np.diag([1.0, 2.0, -3.0, 4.0])
    b = np.ones(4)
    r = O.apcg(*_csr(A), b, "none", tol=1e-12, max_iter=10)
    assert r["status"] == O.ORC_BREAKDOWN


def test_maxit_and_zero_rhs():
    rng = np.random.default_rng(15)
    A = _rand_spd(20, 1e3, rng)
    r = O.apcg(*_csr(A), rng.standard_normal(20), "none", tol=1e-14, max_iter=2)
    assert r["status"] == O.ORC_MAXIT and r["m"] == 2
    r = O.apcg(*_csr(A), np.zeros(20), "none", tol=1e-8, max_iter=5)
    assert r["m"] == 0 and np.all(r["x"] == 0)


def test_direction_forms_agree_on_recycled_bases():
    """w = z + beta w_old (Algorithm 1) and w = z + beta P w_old (the
    library's default: the projector applied to the old direction as well)
    are one iteration in exact arithmetic (P w_old = w_old, Section 2.1).
    In double precision their iteration counts agree within +-2 and both
    solutions meet the tolerance, with a basis of recycled Ritz vectors
    (elasticity 6^3, SRKS after system 0) and with a random basis."""
    import gen

    seq = gen.config_elasticity(6, 3)
    recs, C = O.solve_sequence(seq, 1, reuse="srks", eps=1e-10, cap=24, cap_policy="freeze", tol=1e-8,
                               max_iter=4000)
    rng = np.random.default_rng(11)
    bases = [C, rng.standard_normal((seq.n, 12))]
    for k in (1, 2):
        rp, ci, v, b = seq.csr(k)
        for Cb in bases:
            a = O.apcg(rp, ci, v, b, "block3", C=Cb, tol=1e-8, max_iter=4000, direction="literal")
            p = O.apcg(rp, ci, v, b, "block3", C=Cb, tol=1e-8, max_iter=4000, direction="project_old")
            assert a["status"] == O.ORC_OK and p["status"] == O.ORC_OK
            assert abs(a["m"] - p["m"]) <= 2, (k, a["m"], p["m"])
            assert a["relres_true"] <= 1e-8 and p["relres_true"] <= 1e-8
            # the first coefficients agree to rounding
            assert np.allclose(a["alpha"][:20], p["alpha"][:20], rtol=1e-9, atol=0)


def test_reorth_exact_termination_and_solution():
    """Full reorthogonalisation on tiny SPD inputs (kappa up to 1e4): exact
    termination within n - n_c steps, the dense solution, and the same
    coefficients as the plain iteration over the first steps."""
    rng = np.random.default_rng(12)
    for n, nc, kappa in ((24, 0, 1e2), (32, 5, 1e4)):
        A = _rand_spd(n, kappa, rng)
        C = rng.standard_normal((n, nc)) if nc else None
        b = rng.standard_normal(n)
        r = O.apcg(*_csr(A), b, "none", C=C, tol=1e-12, max_iter=n, reorth=True)
        assert r["status"] == O.ORC_OK and r["m"] <= n - nc, (n, r["m"])
        xs = np.linalg.solve(A, b)
        assert np.linalg.norm(r["x"] - xs) / np.linalg.norm(xs) <= 1e-10 * kappa
        p = O.apcg(*_csr(A), b, "none", C=C, tol=1e-12, max_iter=n)
        k = min(5, r["m"], p["m"])
        assert np.allclose(r["alpha"][:k], p["alpha"][:k], rtol=1e-8)


def test_reorth_keeps_directions_conjugate_and_ritz_values_simple():
    """At n = 6,084 and about 10^3 steps (elasticity 12^3, tol 1e-10):
    with full reorthogonalisation every pair of directions is A-conjugate to
    1e-12 (normalised), and no two Ritz values coincide to 1e-8 (no ghost
    copies, so the 1e-14 stagnation test selects each eigenvalue once);
    without it conjugacy is lost and ghost pairs appear (Section 5.1)."""
    import gen

    seq = gen.config_elasticity(12, 1)
    rp, ci, v, b = seq.csr(0)
    A = sp.csr_matrix((v, ci, rp), shape=(seq.n, seq.n))
    out = {}
    for reorth in (False, True):
        r = O.apcg(rp, ci, v, b, "block3", tol=1e-10, max_iter=3000, record_w=True, reorth=reorth)
        assert r["status"] == O.ORC_OK and r["relres_true"] <= 1e-9
        W = r["W"]
        G = W.T @ (A @ W)
        d = np.sqrt(np.diag(G))
        Gn = G / d[:, None] / d[None, :]
        np.fill_diagonal(Gn, 0.0)
        th, th1 = O.ritz_values(r["alpha"], r["rho"])
        close = int(np.sum(np.abs(np.diff(th)) / th[1:] < 1e-8))
        sel = O.srks_select(th, th1, 1e-14)
        out[reorth] = (r["m"], np.abs(Gn).max(), close, th[sel])
    m0, cos0, close0, _ = out[False]
    m1, cos1, close1, sel1 = out[True]
    assert m1 > 500
    assert cos1 <= 1e-12, cos1
    assert close1 == 0
    assert np.all(np.abs(np.diff(sel1)) / sel1[1:] > 1e-8)
    # the pin discriminates: the plain run has lost conjugacy and has ghosts
    assert cos0 > 1e-3 and close0 > 10
    assert m1 <= m0


def test_extended_accumulation_is_a_faithful_evaluation():
    """Accumulating the products in extended precision is the same solve up
    to rounding: the same iteration count within one step and the same
    solution to the solve tolerance on a well-conditioned case, and the
    first coefficients to 1e-12."""
    seq = gen.config_diffusion_20(0, 1, N=8)
    rp, ci, v, b = seq.csr(0)
    a = O.apcg(rp, ci, v, b, "jacobi", tol=1e-10, max_iter=500)
    e = O.apcg(rp, ci, v, b, "jacobi", tol=1e-10, max_iter=500, extended=True)
    assert abs(a["m"] - e["m"]) <= 1
    assert np.linalg.norm(a["x"] - e["x"]) <= 1e-9 * np.linalg.norm(a["x"])
    assert np.allclose(a["alpha"][:20], e["alpha"][:20], rtol=1e-12, atol=0)
    assert e["relres_true"] <= 1e-10 * 1.01
