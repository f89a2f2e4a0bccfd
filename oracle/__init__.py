"""FP64 CPU oracle for APCG with total (TRKS) and selective (SRKS) Krylov reuse.

TEST INFRASTRUCTURE ONLY.  Nothing in the library package imports this
module; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` use it.  The inner solver is plain C (``oracle.c``, built
with gcc); the sequence logic below (Lanczos tridiagonal, Ritz selection,
basis update) is plain numpy following the paper step by step.

Paper: Gosselet, Rey, Pebrel, arXiv 1301.7530.
  * Algorithm 1 / Section 2.1: APCG with the pair (x0, P).
  * Algorithm 2 / Section 3: TRKS, concatenation of all search directions.
  * Section 4.1: Ritz values/vectors from the CG coefficients.
  * Section 4.4 / Algorithm 3: SRKS stagnation test and concatenation.
"""

from __future__ import annotations

import ctypes
import math

import numpy as np

from .build import ensure_built

ORC_OK, ORC_MAXIT, ORC_BREAKDOWN, ORC_INVALID, ORC_NOMEM = range(5)
PRECOND = {"none": 0, "jacobi": 1, "block3": 3}

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_INT = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(ensure_built())
        L.orc_apcg.restype = ctypes.c_int
        L.orc_apcg.argtypes = [ctypes.c_int64, _I64, _I32, _D, ctypes.c_int, _D, ctypes.c_int, ctypes.c_int64,
                               _D, ctypes.c_double, ctypes.c_int, ctypes.c_double, _D, _D, _D, _D, _D,
                               _D, ctypes.c_int64, _D, ctypes.c_int64, _INT, _INT, _D, ctypes.c_int]
        L.orc_apcg_alg1.restype = ctypes.c_int
        L.orc_apcg_alg1.argtypes = [ctypes.c_int64, _I64, _I32, _D, ctypes.c_int, _D, ctypes.c_int, ctypes.c_int64,
                                    _D, ctypes.c_int, ctypes.c_double, _D, _D, _D]
        L.orc_spmv.restype = None
        L.orc_spmv.argtypes = [ctypes.c_int64, _I64, _I32, _D, _D, _D]
        L.orc_ldl_count.restype = ctypes.c_int
        L.orc_ldl_count.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double]
        L.orc_ldl_eigvals.restype = None
        L.orc_ldl_eigvals.argtypes = [ctypes.c_int, _D, _D, _D]
        L.orc_tridiag_eigvec.restype = None
        L.orc_tridiag_eigvec.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double, _D]
        L.orc_jacobi_eigvals.restype = None
        L.orc_jacobi_eigvals.argtypes = [ctypes.c_int, _D, _D]
        L.orc_dense_cholesky_solve.restype = ctypes.c_int
        L.orc_dense_cholesky_solve.argtypes = [ctypes.c_int, _D, _D, _D]
        _lib = L
    return _lib


def _p(a, t=_D):
    return None if a is None else a.ctypes.data_as(t)


def _csr(row_ptr, col_idx, values):
    return (np.ascontiguousarray(row_ptr, dtype=np.int64), np.ascontiguousarray(col_idx, dtype=np.int32),
            np.ascontiguousarray(values, dtype=np.float64))


# ----------------------------------------------------------------- kernels

def spmv(row_ptr, col_idx, values, x):
    rp, ci, v = _csr(row_ptr, col_idx, values)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(len(rp) - 1)
    lib().orc_spmv(len(y), _p(rp, _I64), _p(ci, _I32), _p(v), _p(x), _p(y))
    return y


DIRECTION = {"literal": 0, "project_old": 1}


def apcg(row_ptr, col_idx, values, b, precond="jacobi", C=None, tol=1e-8, max_iter=None, guard=1e-6,
         record_z=False, record_w=False, direction="literal", reorth=False, orthonormal=False, extended=False):
    """One APCG(A, M, C, b) solve (Algorithm 1, standard form; see oracle.c).

    ``direction``: 'literal' (w = z + beta w_old, Algorithm 1) or
    'project_old' (w = z + beta P w_old, the same in exact arithmetic).
    ``reorth``: full reorthogonalisation of every new direction against all
    earlier ones (Section 2.1 remark; used in the experiments of Section 5.1).
    ``orthonormal``: work with the A-orthonormal basis C L^{-T} of the kept
    columns (G = L L^T) instead of C and the Cholesky factor: the same
    projector in exact arithmetic, without the condition number of G in its
    rounding.
    ``extended``: accumulate the matrix-vector and dot products in extended
    precision (both evaluations are faithful; their difference over a long
    run is what rounding alone moves).

    Returns a dict with x, m, status, alpha[m], gamma[m], rho[m] (rho_0..rho_{m-1}),
    resnorm[m+1], relres_true, kept (bool per column of C), and Z / W
    (n x m, when requested).
    """
    rp, ci, v = _csr(row_ptr, col_idx, values)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = len(b)
    if max_iter is None:
        max_iter = max(10, 4 * n)
    if C is None or C.shape[1] == 0:
        Cf, nc, ldc = None, 0, n
    else:
        Cf = np.asfortranarray(C, dtype=np.float64)
        nc, ldc = Cf.shape[1], n
    x = np.zeros(n)
    alpha = np.zeros(max_iter + 1)
    rho = np.zeros(max_iter + 1)
    gamma = np.zeros(max_iter + 1)
    resn = np.zeros(max_iter + 2)
    Z = np.empty((n, max_iter), order="F") if record_z else None
    W = np.empty((n, max_iter), order="F") if record_w else None
    kept = np.ones(max(nc, 1), dtype=np.intc)
    m = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = lib().orc_apcg(n, _p(rp, _I64), _p(ci, _I32), _p(v), PRECOND[precond], _p(Cf), nc, ldc, _p(b), tol,
                        max_iter, guard, _p(x), _p(alpha), _p(rho), _p(gamma), _p(resn), _p(Z), n, _p(W), n,
                        _p(kept, _INT), ctypes.byref(m), ctypes.byref(rel),
                        DIRECTION[direction] | (2 if reorth else 0) | (4 if orthonormal else 0)
                        | (8 if extended else 0))
    if st in (ORC_INVALID, ORC_NOMEM):
        raise ValueError(f"oracle apcg failed with status {st}")
    m = m.value
    out = dict(x=x, m=m, status=st, alpha=alpha[:m].copy(), gamma=gamma[:m].copy(), rho=rho[:m].copy(),
               resnorm=resn[: m + 1].copy(), relres_true=rel.value, kept=kept[:nc].astype(bool))
    if record_z:
        out["Z"] = Z[:, :m]
    if record_w:
        out["W"] = W[:, :m]
    return out


def apcg_alg1(row_ptr, col_idx, values, b, iters, precond="jacobi", C=None, guard=1e-6):
    """APCG from its conjugacy conditions (the Gram-Schmidt form Algorithm 1
    prints); returns (x, alpha, bgs) with bgs the Gram-Schmidt coefficients."""
    rp, ci, v = _csr(row_ptr, col_idx, values)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = len(b)
    if C is None or C.shape[1] == 0:
        Cf, nc = None, 0
    else:
        Cf = np.asfortranarray(C, dtype=np.float64)
        nc = Cf.shape[1]
    x = np.zeros(n)
    alpha = np.zeros(iters)
    bgs = np.zeros(max(iters, 1))
    st = lib().orc_apcg_alg1(n, _p(rp, _I64), _p(ci, _I32), _p(v), PRECOND[precond], _p(Cf), nc, n, _p(b),
                             iters, guard, _p(x), _p(alpha), _p(bgs))
    if st != ORC_OK:
        raise ValueError(f"oracle apcg_alg1 failed with status {st}")
    return x, alpha, bgs


# ------------------------------------------------------ Ritz (Section 4.1)

def lanczos_factors(alpha, rho):
    """H_m = L D L^T: d_j = 1/alpha_j, l_j^2 = beta_{j+1} = rho_{j+1}/rho_j."""
    alpha = np.asarray(alpha, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    m = len(alpha)
    d = 1.0 / alpha
    l2 = rho[1:m] / rho[: m - 1] if m > 1 else np.zeros(0)
    return d, l2


def lanczos_tridiag(alpha, rho):
    """Explicit H_m of Section 4.1: diagonal delta_j and off-diagonal eta_j.

    delta_0 = 1/alpha_0, delta_j = 1/alpha_j + beta_j/alpha_{j-1},
    eta_j = sqrt(beta_{j+1})/alpha_j, with beta_j = rho_j/rho_{j-1}.
    """
    alpha = np.asarray(alpha, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    m = len(alpha)
    beta = np.zeros(m)
    beta[1:] = rho[1:m] / rho[: m - 1]
    delta = 1.0 / alpha
    delta[1:] += beta[1:] / alpha[:-1]
    eta = np.sqrt(beta[1:]) / alpha[:-1]
    return delta, eta


def ldl_eigvals(d, l2):
    """Eigenvalues of L D L^T, descending, by bisection (oracle.c)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    l2 = np.ascontiguousarray(l2 if len(l2) else np.zeros(1), dtype=np.float64)
    m = len(d)
    th = np.zeros(m)
    if m:
        lib().orc_ldl_eigvals(m, _p(d), _p(l2), _p(th))
    return th


def ritz_values(alpha, rho):
    """(Theta_m, Theta_{m-1}) in descending order (Algorithm 3)."""
    d, l2 = lanczos_factors(alpha, rho)
    m = len(d)
    th_m = ldl_eigvals(d, l2)
    th_m1 = ldl_eigvals(d[: m - 1], l2[: max(m - 2, 0)]) if m > 1 else np.zeros(0)
    return th_m, th_m1


def tridiag_eigvec(delta, eta, theta):
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    eta = np.ascontiguousarray(eta if len(eta) else np.zeros(1), dtype=np.float64)
    v = np.zeros(len(delta))
    lib().orc_tridiag_eigvec(len(delta), _p(delta), _p(eta), float(theta), _p(v))
    return v


def jacobi_eigvals(A):
    a = np.asfortranarray(A, dtype=np.float64).copy(order="F")
    ev = np.zeros(a.shape[0])
    lib().orc_jacobi_eigvals(a.shape[0], _p(a), _p(ev))
    return ev


def dense_cholesky_solve(A, b):
    a = np.asfortranarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    st = lib().orc_dense_cholesky_solve(a.shape[0], _p(a), _p(b), _p(x))
    if st != ORC_OK:
        raise ValueError("matrix not SPD")
    return x


def srks_select(th_m, th_m1, eps):
    """Indices (0-based, ascending) of converged Ritz values (Section 4.4).

    For j = 0..m-2 (the paper's 1..m-1): theta_m[j] has converged if
    |theta_m[j] - theta_{m-1}[j]| <= eps |theta_m[j]|, and theta_m[j+1] if
    |theta_m[j+1] - theta_{m-1}[j]| <= eps |theta_m[j+1]|.  An index found
    twice is taken once.
    """
    sel = set()
    for j in range(len(th_m1)):
        if abs(th_m[j] - th_m1[j]) <= eps * abs(th_m[j]):
            sel.add(j)
        if abs(th_m[j + 1] - th_m1[j]) <= eps * abs(th_m[j + 1]):
            sel.add(j + 1)
    return sorted(sel)


def ritz_block(Z, alpha, rho, idx, th_m):
    """Columns y^i / sqrt(|theta^i|) for i in idx (Algorithm 3).

    y^i = V_m q^i with V_m = [(-1)^j z_j / sqrt(rho_j)] and q^i the unit
    eigenvector of H_m for theta^i.
    """
    m = len(alpha)
    if not len(idx):
        return np.zeros((Z.shape[0], 0))
    delta, eta = lanczos_tridiag(alpha, rho)
    Q = np.stack([tridiag_eigvec(delta, eta, th_m[i]) for i in idx], axis=1)
    sgn = np.where(np.arange(m) % 2 == 0, 1.0, -1.0)
    F = (sgn / np.sqrt(rho[:m]))[:, None] * Q / np.sqrt(np.abs(th_m[idx]))[None, :]
    return Z[:, :m] @ F


def trks_block(W, gamma):
    """All search directions w_j, scaled by 1/sqrt((w_j, A w_j)) (Algorithm 2)."""
    return W / np.sqrt(gamma)[None, :]


def freeze_pick(idx, th_m, room):
    """Cap policy 'freeze': keep at most `room` indices, smallest Ritz values first."""
    if room <= 0:
        return []
    if len(idx) <= room:
        return list(idx)
    order = sorted(idx, key=lambda i: (th_m[i], i))
    return sorted(order[:room])


def cluster_reselect(th_m, idx, min_frac=0.2):
    """Drop the central cluster from a preselection (Section 4.4, the
    reselection behind "clust14").

    The preselected Ritz values (indices ``idx`` into ``th_m``) are sorted
    ascending, v_1 < ... < v_s, and the distances between neighbours taken on
    a log scale, g_i = ln(v_{i+1} / v_i).  The sequence g is approximated in
    the least-squares sense by a piecewise-constant function of three pieces
    g[0:a], g[a:b], g[b:] (each level the mean of its piece; outer pieces may
    be empty, not both) whose middle piece covers at least
    L = ceil(min_frac * s) values (b - a + 1 >= L; one fifth of the preselection
    for the default, as the paper sets it); ties go to the smaller a,
    then the smaller b.  When the middle level is below every non-empty
    outer level, the values v_{a+1}..v_{b+1} (1-based) form the central
    cluster and are dropped.  Returns the kept indices, ascending.
    """
    idx = [int(i) for i in idx]
    s = len(idx)
    if s < 3:
        return sorted(idx)
    order = sorted(idx, key=lambda i: (th_m[i], i))
    v = np.array([th_m[i] for i in order], dtype=np.float64)
    g = np.log(v[1:] / v[:-1])
    G = len(g)
    L = max(1, int(math.ceil(min_frac * s - 1e-9)))
    c1 = np.concatenate([[0.0], np.cumsum(g)])
    c2 = np.concatenate([[0.0], np.cumsum(g * g)])

    def sse(i, j):  # pieces g[i:j]
        if j <= i:
            return 0.0
        t = c1[j] - c1[i]
        return (c2[j] - c2[i]) - t * t / (j - i)

    best = None
    for a in range(0, G + 1):
        for b in range(a + 1, G + 1):
            if b - a + 1 < L or (a == 0 and b == G):
                continue
            cost = sse(0, a) + sse(a, b) + sse(b, G)
            if best is None or cost < best[0]:
                best = (cost, a, b)
    if best is None:
        return sorted(idx)
    _, a, b = best
    mid = (c1[b] - c1[a]) / (b - a)
    outer = [(c1[a] - c1[0]) / a] if a > 0 else []
    if b < G:
        outer.append((c1[G] - c1[b]) / (G - b))
    if not all(mid < o for o in outer):
        return sorted(idx)
    drop = set(order[a : b + 1])
    return sorted(i for i in idx if i not in drop)


def distinct_ritz_ascending(alpha, rho, merge=1e-10):
    """Ritz values of H_m ascending, with copies (values within a relative
    ``merge`` of the previous kept one, as finite-precision Lanczos repeats
    converged values) counted once."""
    th = np.sort(ritz_values(alpha, rho)[0])
    out = []
    for t in th:
        if out and abs(t - out[-1]) <= merge * abs(t):
            continue
        out.append(float(t))
    return np.array(out)


def nc_limit(alpha, rho, bytes_iter0, bytes_col_iter, bytes_rebuild0, bytes_col_rebuild, kmax, eps=1e-8,
             merge=1e-10):
    """n_c_lim from a complexity analysis (Section 4.4, remark after Algorithm 3).

    Under the assumption that every non-augmented system takes the m_0
    iterations of the solve that produced (alpha, rho), a system augmented
    by the eigenvectors of its k lowest eigenvalues converges at the rate of
    the reduced condition number theta_max / theta_(k+1) (Section 2.2
    deflation; the CG rate of Section 4.3), so it takes
        m(k) = max(1, m_0 ln(sigma(kappa_0)) / ln(sigma(kappa_k))),
        sigma(kappa) = (sqrt(kappa) - 1) / (sqrt(kappa) + 1),
    iterations, the spectrum taken from the distinct Ritz values.  Only
    converged Ritz vectors approximate eigenvectors (Section 4.4: those whose
    values pass the stagnation test at ``eps``), so k runs over the
    converged prefix of the ascending Ritz values: past the first value
    that has not converged, more columns are modelled as gaining nothing.
    A solve with k columns moves
        T(k) = m(k) (bytes_iter0 + k bytes_col_iter) + [k > 0] (bytes_rebuild0 + k bytes_col_rebuild)
    bytes; n_c_lim is the k in 0..kmax that minimises T (the smaller k on a
    tie).  Returns (n_c_lim, T as an array over k).
    """
    th_m, th_m1 = ritz_values(alpha, rho)
    conv = set(srks_select(th_m, th_m1, eps)) if len(alpha) > 1 else set()
    order = sorted(range(len(th_m)), key=lambda i: (th_m[i], i))
    th, ok = [], []
    for i in order:  # distinct values ascending; a value converged if any copy passed
        t = float(th_m[i])
        if th and abs(t - th[-1]) <= merge * abs(t):
            ok[-1] = ok[-1] or (i in conv)
            continue
        th.append(t)
        ok.append(i in conv)
    th = np.array(th)
    kconv = 0
    while kconv < len(ok) and ok[kconv]:
        kconv += 1
    m0 = len(alpha)
    kmax = int(max(0, min(kmax, len(th) - 1)))
    tmax = th[-1]

    def lnsig(kappa):
        if kappa <= 1.0:
            return -np.inf  # one distinct eigenvalue left: converges at once
        r = math.sqrt(kappa)
        return math.log((r - 1.0) / (r + 1.0))

    l0 = lnsig(tmax / th[0])
    T = np.empty(kmax + 1)
    for k in range(kmax + 1):
        kd = min(k, kconv)  # columns past the converged prefix deflate nothing more
        lk = lnsig(tmax / th[kd])
        mk = max(1.0, m0 * (l0 / lk)) if np.isfinite(lk) else 1.0
        T[k] = mk * (bytes_iter0 + k * bytes_col_iter) + ((bytes_rebuild0 + k * bytes_col_rebuild) if k else 0.0)
    best = int(np.argmin(T))
    return best, T


def solve_sequence(seq, n_systems=None, reuse="srks", precond=None, tol=1e-8, eps=1e-14, cap=0,
                   cap_policy="freeze", C0=None, max_iter=None, guard=1e-6, keep_x=False, cost_model=None,
                   reselect=None, cluster_min_frac=0.2, direction="literal", reorth=False):
    """Run TRKS / SRKS / plain PCG over systems 0..n_systems-1 of ``seq``.

    ``reuse``: 'none' (PCG), 'trks' (Algorithm 2) or 'srks' (Algorithm 3).
    ``cap`` (n_c_lim, 0 = none) with ``cap_policy`` 'restart' (reset the
    basis to C0 once its size reaches the cap, Algorithm 3) or 'freeze'
    (append only while below the cap, smallest Ritz values first).
    A sequence with an ``advance(x)`` method (gen.NewtonSequence) receives
    each solution before its next system is built.  ``direction``, ``reorth``:
    the direction-update form and full reorthogonalisation of ``apcg``.
    ``reselect='cluster'``: the SRKS preselection is reduced by
    ``cluster_reselect`` before the cap ("clust", Section 4.4).
    ``cap='auto'``: n_c_lim from ``nc_limit`` on the first solve's
    coefficients, with ``cost_model`` = dict(bytes_iter0, bytes_col_iter,
    bytes_rebuild0, bytes_col_rebuild, kmax).
    Returns one record per system.
    """
    auto = cap == "auto"
    if auto:
        cap = 0
    n_systems = seq.n_systems if n_systems is None else n_systems
    if precond is None:
        precond = "block3" if getattr(seq, "block", 1) == 3 else "jacobi"
    n = seq.n
    C_init = np.zeros((n, 0)) if C0 is None else np.asarray(C0, dtype=np.float64)
    C = C_init.copy()
    recs = []
    for k in range(n_systems):
        rp, ci, v, b = seq.csr(k)
        res = apcg(rp, ci, v, b, precond, C, tol, max_iter, guard, record_z=(reuse == "srks"),
                   record_w=(reuse == "trks"), direction=direction, reorth=reorth)
        if hasattr(seq, "advance"):
            seq.advance(res["x"])  # a sequence whose next matrix depends on this solution
        nc_in = C.shape[1]
        if nc_in:
            C = C[:, res["kept"]]
        rec = dict(k=k, m=res["m"], nc=C.shape[1], nc_in=nc_in, dropped=nc_in - C.shape[1], status=res["status"],
                   relres_true=res["relres_true"], alpha=res["alpha"], rho=res["rho"], gamma=res["gamma"],
                   resnorm=res["resnorm"])
        if keep_x:
            rec["x"] = res["x"]
        m = res["m"]
        if auto and k == 0:
            cap, _ = nc_limit(res["alpha"], res["rho"], eps=eps, **cost_model)
            rec["nc_lim"] = cap
            if cap == 0:
                cap = -1  # nothing may be appended
        new = np.zeros((n, 0))
        if reuse == "trks" and m > 0:
            cols = list(range(m))
            if cap and cap_policy == "freeze":
                cols = cols[: max(cap - C.shape[1], 0)]
            elif cap < 0:
                cols = []
            new = trks_block(res["W"][:, cols], res["gamma"][cols])
        elif reuse == "srks" and m > 1:
            th_m, th_m1 = ritz_values(res["alpha"], res["rho"])
            sel = srks_select(th_m, th_m1, eps)
            rec["theta"] = th_m
            rec["preselected"] = list(sel)
            if reselect == "cluster":
                sel = cluster_reselect(th_m, sel, cluster_min_frac)
            rec["selected_all"] = list(sel)
            if cap and cap_policy == "freeze":
                sel = freeze_pick(sel, th_m, cap - C.shape[1])
            elif cap < 0:
                sel = []
            rec["selected"] = list(sel)
            new = ritz_block(res["Z"], res["alpha"], res["rho"], sel, th_m)
        rec["added"] = new.shape[1]
        C = np.concatenate([C, new], axis=1) if new.shape[1] else C
        if cap > 0 and cap_policy == "restart" and C.shape[1] >= cap:
            C = C_init.copy()
            rec["restarted"] = True
        rec["nc_next"] = C.shape[1]
        recs.append(rec)
    return recs, C


def cg_iteration_bound(kappa, eps):
    """n_eps = ln(eps/2)/ln(sigma), sigma = (sqrt(kappa)-1)/(sqrt(kappa)+1) (Section 4, CG bound)."""
    s = (math.sqrt(kappa) - 1.0) / (math.sqrt(kappa) + 1.0)
    return math.log(eps / 2.0) / math.log(s)
