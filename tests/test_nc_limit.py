"""n_c_lim from the complexity analysis of Section 4.4 (the remark after
Algorithm 3): the oracle's ``nc_limit`` pinned by properties of the model
that do not depend on how it is written, and the library's host routine
(``krs_nc_limit``, its own eigenvalue method) against the oracle on the same
CG coefficients.  CPU only."""
import numpy as np
import pytest

import gen
import oracle as O


def _cg_on_spectrum(eigs, seed=3):
    """CG coefficients of a run on diag(eigs) to a relative residual of
    1e-12, with full reorthogonalisation so that the converged Ritz values
    are eigenvalues to rounding (Jacobi would flatten the spectrum: no
    preconditioner)."""
    n = len(eigs)
    rp = np.arange(n + 1, dtype=np.int64)
    ci = np.arange(n, dtype=np.int32)
    b = np.random.default_rng(seed).standard_normal(n)
    r = O.apcg(rp, ci, np.asarray(eigs, dtype=np.float64), b, "none", tol=1e-12, max_iter=n, reorth=True)
    return r["alpha"], r["rho"]


def _two_clusters(n_low=5, n_mid=35):
    low = 1e-4 * np.arange(1, n_low + 1)
    mid = np.linspace(0.5, 1.0, n_mid)
    return np.concatenate([low, mid])


def test_ritz_spectrum_recovers_the_isolated_values_and_the_top():
    eigs = _two_clusters()
    a, r = _cg_on_spectrum(eigs)
    th = O.distinct_ritz_ascending(a, r)
    assert len(th) >= len(eigs) - 2
    assert np.allclose(th[:5], eigs[:5], rtol=1e-8)
    assert th[-1] == pytest.approx(1.0, rel=1e-8)


def test_free_columns_deflate_everything():
    # columns that cost nothing: more deflation never costs iterations, and
    # the limit is the first k at the least cost
    a, r = _cg_on_spectrum(_two_clusters(8, 60))
    k, T = O.nc_limit(a, r, 1.0, 0.0, 0.0, 0.0, kmax=30)
    assert np.all(np.diff(T) <= 0)
    assert T[k] == T.min() and (k == 0 or T[k - 1] > T[k])
    assert k >= 8


def test_costly_columns_are_never_worth_it():
    a, r = _cg_on_spectrum(_two_clusters())
    k, T = O.nc_limit(a, r, 1.0, 1e6, 0.0, 0.0, kmax=30)
    assert k == 0
    assert T[0] == pytest.approx(len(a) * 1.0)  # m_0 iterations of bytes_iter0


def test_isolated_low_eigenvalues_are_the_ones_worth_deflating():
    # five isolated values far below a dense cluster: deflating them drops
    # the condition number from 1e4 to 2 and the iterations to the floor of
    # one; every further column only adds its rebuild (half an iteration)
    a, r = _cg_on_spectrum(_two_clusters())
    k, T = O.nc_limit(a, r, 1.0, 0.01, 0.0, 0.5, kmax=30)
    assert k == 5
    assert T[5] < T[4] and T[5] < T[6]


def test_limit_never_grows_with_the_column_cost():
    a, r = _cg_on_spectrum(_two_clusters(8, 60))
    ks = [O.nc_limit(a, r, 1.0, c, 5.0, 0.1, kmax=60)[0] for c in (0.0, 1e-4, 1e-3, 1e-2, 0.1, 1.0, 10.0)]
    assert all(x >= y for x, y in zip(ks, ks[1:])), ks
    assert ks[0] > ks[-1] == 0


def _elasticity_coeffs():
    seq = gen.config_elasticity(6, 1)
    rp, ci, v, b = seq.csr(0)
    r = O.apcg(rp, ci, v, b, "block3", tol=1e-10, max_iter=3000)
    return r["alpha"], r["rho"], seq.n


@pytest.mark.parametrize("case", ["diag", "elasticity"])
def test_library_nc_limit_matches_oracle(case):
    import paper_1301_7530_amd as K

    if case == "diag":
        a, r = _cg_on_spectrum(_two_clusters(8, 60))
        n = 68
    else:
        a, r, n = _elasticity_coeffs()
    for col in (0.0, 2.0 * n * 8 / 1e6, 16.0 * n / 1e5, 1e-3, 0.05):
        args = (1.0, col, 3.0, 7.0 * col, 200)
        k_o, T_o = O.nc_limit(a, r, *args)
        k_l, T_l = K.nc_limit(a, r, *args)
        assert len(T_l) == len(T_o)
        assert np.allclose(T_l, T_o, rtol=1e-9, atol=0)
        # the same choice, or one whose modelled cost ties within the tolerance
        assert k_l == k_o or abs(T_o[k_l] - T_o[k_o]) <= 1e-9 * T_o[k_o], (col, k_l, k_o)
