"""The solution-driven workload (gen.NewtonSequence): its strain measure on
displacements with known strains, its softening law, and that its matrices
stay symmetric positive definite while they soften.  CPU only."""
import numpy as np
import pytest

import gen
import oracle as O


def _nodes(E):
    """Free-node coordinates (x, y, z) in the dof order of the cube."""
    n1 = E + 1
    iz, iy, ix = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(1, n1), indexing="ij")
    return np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1) / E


def test_strain_of_known_fields():
    E = 5
    X = _nodes(E)
    # uniform stretch along x (the clamped face x = 0 stays fixed): e_xx = 0.3
    u = np.zeros_like(X)
    u[:, 0] = 0.3 * X[:, 0]
    assert np.allclose(gen.centre_strain(E, u.ravel()), 0.3)
    # simple shear u_y = 0.2 x: gamma_xy = 0.2, equivalent strain 0.2 / sqrt(2)
    u = np.zeros_like(X)
    u[:, 1] = 0.2 * X[:, 0]
    assert np.allclose(gen.centre_strain(E, u.ravel()), 0.2 / np.sqrt(2.0))
    # a rigid rotation about the x axis has no (linearised) strain, away from
    # the first layer of elements, whose clamped face does not rotate
    u = np.zeros_like(X)
    u[:, 1], u[:, 2] = -1e-3 * X[:, 2], 1e-3 * X[:, 1]
    eps = gen.centre_strain(E, u.ravel())
    assert np.allclose(eps[:, :, 1:], 0.0, atol=1e-12) and np.all(eps[:, :, 0] >= 0)


def test_softening_law():
    t = np.linspace(0.0, 10.0, 201)
    g = gen.softening(t)
    assert np.all(g[t <= 1.0] == 1.0)
    assert np.all(np.diff(g) <= 0.0) and g.min() >= 0.05 and g[-1] < 0.1


def test_matrices_soften_and_stay_spd():
    seq = gen.NewtonSequence(3, 4, (gen.SEED_ROOT, 6, 0))
    prev = None
    for k in range(4):
        rp, ci, v, b = seq.csr(k)
        A = np.zeros((seq.n, seq.n))
        for i in range(seq.n):
            A[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
        assert np.allclose(A, A.T)
        assert np.linalg.eigvalsh(A).min() > 0
        if prev is not None:
            assert np.all(seq.moduli(k) <= seq.moduli(0) + 0)
        x = np.linalg.solve(A, b)
        seq.advance(x)
        prev = A
    # the load grows and damage appears (some elements softened)
    assert np.any(seq.moduli(3) < seq.moduli(0))
    assert np.all(seq.moduli(3) > 0)


def test_solution_requires_advance():
    seq = gen.NewtonSequence(3, 3, (gen.SEED_ROOT, 6, 1))
    seq.system(0)
    with pytest.raises(ValueError):
        seq.system(1)


def test_oracle_sequence_on_newton_workload():
    seq = gen.NewtonSequence(5, 4, (gen.SEED_ROOT, 6, 2))
    recs, C = O.solve_sequence(seq, 4, reuse="srks", eps=1e-10, tol=1e-8, max_iter=4000)
    assert all(r["relres_true"] <= 1e-8 for r in recs)
    # the recycled basis pays on the later (solution-driven) systems
    assert recs[-1]["m"] < recs[0]["m"]
