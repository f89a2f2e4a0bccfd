"""GPU edge cases through the C ABI: degenerate right-hand sides and bases,
iteration caps, invalid operators, and the recycle of an empty run."""
import numpy as np
import pytest

import gen
import oracle as O

pytestmark = pytest.mark.gpu


def _K():
    import paper_1301_7530_amd as K

    return K


def _relres(csr, x):
    rp, ci, v, b = csr
    return np.linalg.norm(b - O.spmv(rp, ci, v, x)) / np.linalg.norm(b)


@pytest.mark.parametrize("precision", ["fp64", "fp32basis", "mixed"])
def test_zero_rhs(gpu, precision):
    """b = 0: nothing to iterate, x = 0 (the recursion starts converged)."""
    K = _K()
    seq = gen.DiffusionSequence((9, 8, 7), 1, (gen.SEED_ROOT, 97, 0))
    vals, b = seq.system(0)
    s = K.sequence_for(gpu, seq, precision=precision, reuse="selective", tol=1e-8, max_iter=500)
    try:
        s.submit(vals, np.zeros_like(b))
        x, info = s.solve()
        assert info["status"] == 0 and info["iters"] == 0
        assert np.all(x == 0.0)
        assert s.recycle() == 0  # m = 0: nothing to extract
    finally:
        s.close()


def test_basis_containing_the_solution(gpu):
    """C0 = [x*]: the coarse initialisation x0 = C G^-1 C^T b is already the
    solution, so at most one iteration is needed (Section 2.1, x0)."""
    K = _K()
    seq = gen.DiffusionSequence((10, 9, 8), 1, (gen.SEED_ROOT, 97, 1))
    rp, ci, v, b = seq.csr(0)
    xs = O.apcg(rp, ci, v, b, "jacobi", tol=1e-13, max_iter=5000)["x"]
    C0 = np.column_stack([xs, np.random.default_rng(0).standard_normal(seq.n)])
    s = K.sequence_for(gpu, seq, precision="fp64", reuse="none", tol=1e-8, max_iter=500, C0=C0)
    try:
        s.submit(*seq.system(0))
        x, info = s.solve()
        assert info["status"] == 0 and info["iters"] <= 1, info["iters"]
        assert _relres(seq.csr(0), x) <= 1e-8
    finally:
        s.close()


def test_dependent_basis_columns_are_dropped(gpu):
    """Duplicated and zero columns in C0 are removed by the rank guard and
    reported; the solve is unaffected."""
    K = _K()
    seq = gen.DiffusionSequence((10, 10, 10), 1, (gen.SEED_ROOT, 97, 2))
    rng = np.random.default_rng(1)
    c = rng.standard_normal((seq.n, 3))
    C0 = np.column_stack([c, c[:, :1] * 2.0, np.zeros(seq.n), c[:, 1:2] - c[:, 2:3] + c[:, 2:3]])
    s = K.sequence_for(gpu, seq, precision="fp64", reuse="none", tol=1e-8, max_iter=2000, C0=C0)
    try:
        s.submit(*seq.system(0))
        x, info = s.solve()
        assert info["status"] == 0
        assert info["n_c"] == 3 and info["dropped"] == 3
        assert _relres(seq.csr(0), x) <= 1e-8
        rp, ci, v, b = seq.csr(0)
        ref = O.apcg(rp, ci, v, b, "jacobi", C=C0, tol=1e-8, max_iter=2000)
        assert abs(info["iters"] - ref["m"]) <= 2
    finally:
        s.close()


def test_max_iter_reports_and_keeps_state(gpu):
    K = _K()
    seq = gen.DiffusionSequence((12, 12, 12), 2, (gen.SEED_ROOT, 97, 3))
    s = K.sequence_for(gpu, seq, precision="fp64", reuse="selective", tol=1e-8, max_iter=7, ritz_eps=1e-8)
    try:
        s.submit(*seq.system(0))
        with pytest.raises(K.KrsError) as e:
            s.solve(allow_maxit=False)
        assert e.value.status == 5  # KRS_E_MAXIT
        info = s.info()
        assert info["iters"] == 7 and info["rel_res_true"] > 1e-8
        s.recycle()  # a capped run still yields a Lanczos pair
        s.submit(*seq.system(1))
        x, info = s.solve()  # and the sequence goes on
        assert info["iters"] == 7
    finally:
        s.close()


def test_not_spd_operator_is_rejected(gpu):
    K = _K()
    seq = gen.DiffusionSequence((6, 6, 6), 1, (gen.SEED_ROOT, 97, 4))
    vals, b = seq.system(0)
    rp, ci = seq.row_ptr, seq.col_idx
    bad = vals.copy()
    diag = [k for i in range(seq.n) for k in range(rp[i], rp[i + 1]) if ci[k] == i]
    bad[diag[5]] = -abs(bad[diag[5]])
    s = K.sequence_for(gpu, seq, precision="fp64", reuse="none", tol=1e-8, max_iter=100)
    try:
        with pytest.raises(K.KrsError) as e:
            s.submit(bad, b)
        assert e.value.status == 3  # KRS_E_NOT_SPD
        s.submit(vals, b)  # the sequence stays usable
        x, info = s.solve()
        assert info["status"] == 0
    finally:
        s.close()


def test_single_row_slice_and_tiny_system(gpu):
    """n below one slice and below one update step (n = 8)."""
    K = _K()
    seq = gen.DiffusionSequence((2, 2, 2), 2, (gen.SEED_ROOT, 97, 5))
    rp, ci, v, b = seq.csr(0)
    ref = O.apcg(rp, ci, v, b, "jacobi", tol=1e-8, max_iter=100)
    s = K.sequence_for(gpu, seq, precision="fp64", reuse="total", tol=1e-8, max_iter=100)
    try:
        s.submit(*seq.system(0))
        x, info = s.solve()
        assert info["status"] == 0 and abs(info["iters"] - ref["m"]) <= 1
        assert _relres(seq.csr(0), x) <= 1e-8
        s.recycle()
        s.submit(*seq.system(1))
        x, info = s.solve()
        assert info["status"] == 0 and _relres(seq.csr(1), x) <= 1e-8
    finally:
        s.close()


def test_cost_cap_drops_columns_that_do_not_pay(gpu):
    """Cost cap: after every solve the basis holds recycled columns only if
    the last solve with them cost fewer modelled bytes than the latest solve
    with the initial (empty) basis; every solve meets the tolerance."""
    K = _K()
    seq = gen.DiffusionSequence((14, 13, 12), 8, (gen.SEED_ROOT, 97, 6))
    s = K.sequence_for(gpu, seq, precision="fp64", reuse="selective", tol=1e-8, max_iter=2000, ritz_eps=1e-8,
                       max_basis=60, cap_policy="cost")
    ref = None
    try:
        for k in range(8):
            s.submit(*seq.system(k))
            x, info = s.solve()
            assert info["status"] == 0 and _relres(seq.csr(k), x) <= 1e-8
            s.recycle()
            if info["n_c"] == 0:
                ref = info["model_bytes"]
            elif info["model_bytes"] >= ref:
                assert s.n_c == 0, (k, info["model_bytes"], ref)
    finally:
        s.close()


def test_cost_cap_keeps_paying_columns(gpu):
    """The other branch of the cost cap: columns whose solve cost fewer
    modelled bytes than the reference are kept."""
    K = _K()
    seq = gen.config_elasticity(12, 3)
    s = K.sequence_for(gpu, seq, precision="fp64", reuse="selective", tol=1e-8, max_iter=8000, ritz_eps=1e-8,
                       max_basis=24, cap_policy="cost")
    ref = None
    try:
        for k in range(3):
            s.submit(*seq.system(k))
            x, info = s.solve()
            assert info["status"] == 0 and _relres(seq.csr(k), x) <= 1e-8
            n_before = info["n_c"]
            s.recycle()
            if n_before == 0:
                ref = info["model_bytes"]
                assert s.n_c > 0  # columns appended after the reference solve
            elif info["model_bytes"] < ref:
                assert s.n_c >= n_before, (k, info["model_bytes"], ref)
            else:
                assert s.n_c == 0
    finally:
        s.close()
