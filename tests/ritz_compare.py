"""Tolerances for comparing the library's Ritz analysis with the oracle's.

The two sides compute the eigenvalues of the Lanczos tridiagonal (Section
4.1) with different methods: the oracle by bisection on the stationary qd
(LDL^T) inertia of H_m itself, the library by bisection on the progressive
differential qd inertia of R R^T.  Both keep high relative accuracy, so each
Ritz value is compared to a relative tolerance (with an absolute floor at
the top of the spectrum).  The stagnation test of Section 4.4 compares two
such values at a relative distance eps; an index may be selected on one
side and not on the other only when its stagnation ratio lies within the
eigenvalue tolerance of eps.
"""
import numpy as np

# Relative tolerance of one Ritz value: both methods are accurate to a few
# units in the last place times a modest growth factor (measured: <= 2e-15
# on elasticity runs of 433 and 1113 steps).
RITZ_RTOL = 1e-13
RITZ_ATOL_FRAC = 1e-13  # absolute floor, as a fraction of the largest Ritz value


def assert_ritz_close(th_lib, th_orc):
    th_lib = np.asarray(th_lib, dtype=np.float64)
    th_orc = np.asarray(th_orc, dtype=np.float64)
    assert th_lib.shape == th_orc.shape, (th_lib.shape, th_orc.shape)
    if th_orc.size == 0:
        return
    tol = np.maximum(RITZ_RTOL * np.abs(th_orc), RITZ_ATOL_FRAC * np.abs(th_orc).max())
    bad = np.nonzero(np.abs(th_lib - th_orc) > tol)[0]
    assert bad.size == 0, (bad[:5], th_lib[bad[:5]], th_orc[bad[:5]])


def stagnation_ratios(th_m, th_m1):
    """Per index of theta_m (descending): the smaller relative distance to
    its two interlacing neighbours in theta_{m-1} (Algorithm 3's two tests)."""
    m = len(th_m)
    r = np.full(m, np.inf)
    for j in range(len(th_m1)):
        r[j] = min(r[j], abs(th_m[j] - th_m1[j]) / abs(th_m[j]))
        r[j + 1] = min(r[j + 1], abs(th_m[j + 1] - th_m1[j]) / abs(th_m[j + 1]))
    return r


def selection_flips(sel_lib, sel_orc, th_m, th_m1, eps):
    """Indices selected on one side only; raises if any of them is not at
    the threshold (its ratio farther than the eigenvalue tolerance from eps)."""
    a = set(int(i) for i in sel_lib)
    b = set(int(i) for i in sel_orc)
    flips = sorted(a ^ b)
    if flips:
        r = stagnation_ratios(th_m, th_m1)
        band = 4.0 * RITZ_RTOL
        far = [i for i in flips if abs(r[i] - eps) > band]
        assert not far, ("selection differs away from the threshold", far, [r[i] for i in far], eps)
    return flips
