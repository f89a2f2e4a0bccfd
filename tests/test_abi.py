"""The C ABI library loads on a machine without a GPU, exports every entry
point that include/krs.h declares, and its host-side logic (Ritz analysis,
guarded coarse factorisation) agrees with the oracle.  No device calls."""
import os
import re

import numpy as np
import pytest

import gen
import oracle as O
from ritz_compare import assert_ritz_close, selection_flips

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "krs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(krs_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    import paper_1301_7530_amd as K

    names = _declared()
    assert len(names) >= 20
    lib = K.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    bound = {s[0] for s in K.SIGNATURES}
    assert set(names) == bound


def test_status_strings_and_version():
    import paper_1301_7530_amd as K

    assert b"ok" == K.lib().krs_status_str(0)
    assert K.version().startswith("krs")


def test_library_ritz_selection_matches_oracle():
    import paper_1301_7530_amd as K

    seq = gen.config_elasticity(6, 1)
    rp, ci, v, b = seq.csr(0)
    r = O.apcg(rp, ci, v, b, "block3", tol=1e-10, max_iter=3000)
    oth, oth1 = O.ritz_values(r["alpha"], r["rho"])
    for eps in (1e-14, 1e-10, 1e-6):
        th, th1, sel = K.ritz_select(r["alpha"], r["rho"], eps)
        assert_ritz_close(th, oth)
        assert_ritz_close(th1, oth1)
        flips = selection_flips(np.nonzero(sel)[0], O.srks_select(oth, oth1, eps), oth, oth1, eps)
        assert len(flips) <= 2, flips


def test_library_ritz_values_closed_form():
    """The library's eigenvalue routine alone against the 1D Laplacian's
    closed form: CG on tridiag(-1, 2, -1), n = 48, run n steps, recovers
    every eigenvalue 2 - 2 cos(k pi / (n + 1)) (Section 4.1)."""
    import paper_1301_7530_amd as K
    import scipy.sparse as sp

    n = 48
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    b = np.random.default_rng(5).standard_normal(n)
    r = O.apcg(A.indptr, A.indices, A.data, b, "none", tol=1e-300, max_iter=n)
    assert r["m"] == n
    th, _, _ = K.ritz_select(r["alpha"], r["rho"], 1e-14)
    exact = np.sort(2 - 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))[::-1]
    assert np.abs(th - exact).max() < 1e-8


def test_library_coarse_factor_guard():
    import paper_1301_7530_amd as K

    rng = np.random.default_rng(3)
    X = rng.standard_normal((40, 7))
    X[:, 4] = X[:, 1] + 1e-9 * rng.standard_normal(40)  # dependent up to 1e-9
    G = X.T @ X
    Ginv, kept, nk = K.coarse_factor(G, 1e-6)
    assert list(kept) == [True, True, True, True, False, True, True] and nk == 6
    keep = np.nonzero(kept)[0]
    Gk = G[np.ix_(keep, keep)]
    assert np.abs(Ginv[np.ix_(keep, keep)] @ Gk - np.eye(6)).max() < 1e-10
    assert np.all(Ginv[4, :] == 0) and np.all(Ginv[:, 4] == 0)
    # the oracle's guard keeps the same columns
    A = np.eye(40)
    bvec = rng.standard_normal(40)
    import scipy.sparse as sp
    S = sp.csr_matrix(A)
    res = O.apcg(S.indptr, S.indices, S.data, bvec, "none", C=X, tol=1e-10, max_iter=80)
    assert list(res["kept"]) == list(kept)


def test_invalid_arguments_rejected_without_device():
    import ctypes

    import paper_1301_7530_amd as K

    lib = K.lib()
    assert lib.krs_ritz_select(None, None, -1, 1e-8, None, None, None) == K.KRS_E_INVALID
    h = ctypes.c_void_p()
    d = K.SeqDesc()
    assert lib.krs_seq_create(None, ctypes.byref(d), None, 0, 0, ctypes.byref(h)) == K.KRS_E_INVALID
