"""Cluster reselection of Section 4.4 ("clust"): the oracle's
``cluster_reselect`` pinned on spectra whose central cluster is known by
construction and by exhaustive optimality on tiny inputs, and the library's
host routine (``krs_cluster_reselect``) against it.  CPU only."""
import itertools
import math

import numpy as np
import pytest

import gen
import oracle as O


def _three_zone_spectrum(n_low=8, n_mid=30, n_high=8):
    low = 1e-8 * 10.0 ** np.arange(n_low)                   # isolated, a decade apart
    mid = low[-1] * 10.0 * np.exp(1e-3 * np.arange(n_mid))   # dense central zone
    high = mid[-1] * 2.0 ** np.arange(1, n_high + 1)        # isolated, an octave apart
    return np.concatenate([low, mid, high])


def test_known_central_cluster_is_dropped():
    th = _three_zone_spectrum()
    rng = np.random.default_rng(5)
    perm = rng.permutation(len(th))  # any order of theta; indices refer to it
    th_p = th[perm]
    keep = O.cluster_reselect(th_p, range(len(th_p)))
    kept_vals = np.sort(th_p[keep])
    assert np.array_equal(kept_vals, np.concatenate([th[:8], th[38:]]))


def test_subset_preselection_only_touches_preselected():
    th = _three_zone_spectrum()
    pre = [i for i in range(len(th)) if i % 3 != 1]
    keep = O.cluster_reselect(th, pre)
    assert set(keep) <= set(pre)
    assert all(i in keep for i in pre if i < 8)


def test_no_cluster_in_an_even_spectrum():
    th = np.exp(0.1 * np.arange(40))
    assert O.cluster_reselect(th, range(40)) == list(range(40))


@pytest.mark.parametrize("s", [0, 1, 2])
def test_too_few_values_are_kept(s):
    assert O.cluster_reselect(np.arange(1.0, s + 1.0), range(s)) == list(range(s))


def _split_cost(g, a, b):
    return sum(float(np.var(p)) * len(p) for p in (g[:a], g[a:b], g[b:]) if len(p))


@pytest.mark.parametrize("seed", range(12))
def test_chosen_split_is_least_squares_optimal(seed):
    rng = np.random.default_rng(seed)
    s = int(rng.integers(5, 13))
    th = np.cumprod(np.exp(rng.uniform(0.001, 2.0, size=s)))
    keep = O.cluster_reselect(th, range(s))
    g = np.log(th[1:] / th[:-1])
    G = s - 1
    L = math.ceil(0.2 * s - 1e-9)
    valid = [(a, b) for a, b in itertools.combinations(range(G + 1), 2) if b - a + 1 >= L and not (a == 0 and b == G)]
    costs = {ab: _split_cost(g, *ab) for ab in valid}
    best = min(costs.values())
    if len(keep) < s:
        dropped = sorted(set(range(s)) - set(keep))
        a, b = dropped[0], dropped[-1]
        assert dropped == list(range(a, b + 1))           # one contiguous run of sorted values
        assert costs[(a, b)] <= best + 1e-12 * max(1.0, best)
        mid = g[a:b].mean()
        assert all(mid < p.mean() for p in (g[:a], g[b:]) if len(p))


def _elasticity_ritz(eps):
    seq = gen.config_elasticity(6, 1)
    rp, ci, v, b = seq.csr(0)
    r = O.apcg(rp, ci, v, b, "block3", tol=1e-10, max_iter=3000)
    th, th1 = O.ritz_values(r["alpha"], r["rho"])
    return th, O.srks_select(th, th1, eps)


@pytest.mark.parametrize("case", ["three_zone", "random", "elasticity14", "elasticity8"])
def test_library_matches_oracle(case):
    import paper_1301_7530_amd as K

    if case == "three_zone":
        th = _three_zone_spectrum()
        pre = list(range(len(th)))
    elif case == "random":
        rng = np.random.default_rng(11)
        th = np.sort(np.exp(rng.normal(0.0, 3.0, size=150)))[::-1]
        pre = sorted(rng.choice(150, size=90, replace=False).tolist())
    else:
        th, pre = _elasticity_ritz(1e-14 if case == "elasticity14" else 1e-8)
        assert len(pre) >= 3
    flags = np.zeros(len(th), dtype=bool)
    flags[pre] = True
    for frac in (0.2, 0.1, 0.5):
        want = O.cluster_reselect(th, pre, frac)
        got = np.nonzero(K.cluster_reselect(th, flags, frac))[0].tolist()
        assert got == want, (case, frac, len(got), len(want))
