"""Synthetic workload generators: structure, SPD-ness, closed forms, seeds."""
import numpy as np
import pytest
import scipy.sparse as sp

import gen
from gen.diffusion import diffusion_matrix
from gen.elasticity import bsr_to_csr, elasticity_matrix, q1_reference_stiffness


def _dense(rp, ci, v):
    n = len(rp) - 1
    return sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()


def test_unit_diffusion_is_textbook_laplacian():
    N = 5
    rp, ci, v = diffusion_matrix(np.ones((N, N, N)))
    A = _dense(rp, ci, v)
    I = np.eye(N)
    T = 2 * I - np.eye(N, k=1) - np.eye(N, k=-1)
    L3 = np.kron(np.kron(T, I), I) + np.kron(np.kron(I, T), I) + np.kron(np.kron(I, I), T)
    assert np.array_equal(A, L3)


def test_diffusion_pattern_counts_and_symmetry():
    seq = gen.config_diffusion_20()
    assert seq.n == 8000 and seq.nnz == 53600
    rp, ci, v, b = seq.csr(3)
    assert np.all(np.diff(rp) >= 4) and np.all(np.diff(rp) <= 7)
    for i in (0, 17, 4000):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
    A = sp.csr_matrix((v, ci, rp))
    assert abs(A - A.T).max() == 0.0
    # harmonic transmissibility between two cells
    k = seq.coefficients(3).ravel()
    t01 = 2 * k[0] * k[1] / (k[0] + k[1])
    assert A[0, 1] == pytest.approx(-t01, rel=1e-15)


def test_diffusion_damage_is_cumulative_and_seeded():
    s1 = gen.config_diffusion_20(seq_id=2)
    s2 = gen.config_diffusion_20(seq_id=2)
    k0, k1, k2 = (s1.coefficients(i).ravel() for i in range(3))
    changed = k1 != k0
    assert changed.sum() == 400
    assert np.all(k1[changed] / k0[changed] >= 0.5) and np.all(k1 <= k0)
    assert np.all(k2 <= k1)
    v1, b1 = s1.system(2)
    v2, b2 = s2.system(2)
    assert np.array_equal(v1, v2) and np.array_equal(b1, b2)
    s3 = gen.config_diffusion_20(seq_id=3)
    assert not np.array_equal(s3.rhs(0), s1.rhs(0))


def test_q1_reference_stiffness_rigid_modes():
    h = 0.25
    K = q1_reference_stiffness(h)
    assert np.abs(K - K.T).max() < 1e-15
    xyz = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], float) * h
    modes = []
    for d in range(3):
        t = np.zeros((8, 3)); t[:, d] = 1.0; modes.append(t.ravel())
    for (i, j) in ((0, 1), (1, 2), (0, 2)):
        r = np.zeros((8, 3)); r[:, i] = -xyz[:, j]; r[:, j] = xyz[:, i]; modes.append(r.ravel())
    for m in modes:
        assert np.abs(K @ m).max() < 1e-14
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev > 1e-10) == 18  # 24 dofs - 6 rigid modes
    # uniaxial strain energy: u_x = eps*x on a unit-modulus cube of side h
    eps = 1e-3
    u = np.zeros((8, 3)); u[:, 0] = eps * xyz[:, 0]
    nu = 0.3
    lam = nu / ((1 + nu) * (1 - 2 * nu)); mu = 1 / (2 * (1 + nu))
    energy = 0.5 * u.ravel() @ K @ u.ravel()
    assert energy == pytest.approx(0.5 * (lam + 2 * mu) * eps ** 2 * h ** 3, rel=1e-12)


def test_elasticity_counts_match_mesh():
    for E, n, nnzb in ((40, 201720, 1727638),):
        rp, ci, valid = gen.elasticity._pattern(E)
        assert 3 * (len(rp) - 1) == n and rp[-1] == nnzb
    for E in (2, 3):
        rp, ci, bl = elasticity_matrix(np.ones((E, E, E)))
        r, c, v = bsr_to_csr(rp, ci, bl)
        A = _dense(r, c, v)
        assert A.shape == (3 * E * (E + 1) ** 2,) * 2
        assert np.abs(A - A.T).max() == 0.0
        np.linalg.cholesky(A)  # SPD once the x = 0 face is clamped


def test_elasticity_sequence_structure():
    seq = gen.config_elasticity(6, 3)
    blocks0, b0 = seq.system(0)
    blocks1, _ = seq.system(1)
    assert blocks0.shape == (9 * seq.nnzb,) and b0.shape == (seq.n,)
    m0, m1 = seq.moduli(0), seq.moduli(1)
    assert set(np.unique(m0)) <= {1.0, 1e3}
    frac = (m1 != m0).mean()
    assert abs(frac - 0.05) < 0.01 and np.all(m1 <= m0)
    rp, ci, v, b = seq.csr(1)
    A = _dense(rp, ci, v)
    np.linalg.cholesky(A)
    # the BSR blocks are the diagonal 3x3 blocks of the scalar matrix
    p = 5
    k = seq.row_ptr[p] + np.searchsorted(seq.col_idx[seq.row_ptr[p]:seq.row_ptr[p + 1]], p)
    assert np.array_equal(blocks1.reshape(-1, 3, 3)[k], A[3 * p:3 * p + 3, 3 * p:3 * p + 3])


def test_batched_and_serving_sizes():
    shapes = gen.batched_diffusion_sizes()
    assert len(shapes) == 256
    ns = np.array([a * b * c for a, b, c in shapes])
    assert ns.min() > 3e3 and ns.max() < 2.3e5
    Es = gen.serving_elasticity_sizes()
    dofs = np.array([3 * E * (E + 1) ** 2 for E in Es])
    assert len(Es) == 64 and dofs.min() > 5e3 and dofs.max() < 6e5


def test_elasticity_c_assembly_matches_numpy_bitwise():
    """The C assembly helper and the vectorised numpy assembly produce the
    same blocks bit for bit (same sums in the same order)."""
    from gen.elasticity import elasticity_blocks, elasticity_matrix

    for E in (2, 5, 9):
        sq = gen.config_elasticity(E, 2)
        for k in range(2):
            _, _, ref = elasticity_matrix(sq.moduli(k), sq.nu, sq._kref)
            got = elasticity_blocks(sq.moduli(k), sq._kref, sq.nnzb)
            assert np.array_equal(ref, got), (E, k)
