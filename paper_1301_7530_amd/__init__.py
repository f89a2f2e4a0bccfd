"""Python binding of libkrs, the MI355X Krylov-reuse APCG library.

Argument marshalling only: every step of a solve runs in the HIP kernels
and host runtime of ``libkrs.so`` (see ``include/krs.h``).  PyTorch, when
present, supplies the device allocator (its caching allocator) and the
stream; numpy arrays are accepted for host data.

Importing this package fails loudly if ``libkrs.so`` has not been built
(``python paper_1301_7530_amd/build.py``).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkrs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library with `python paper_1301_7530_amd/build.py`"
    )

_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------ ABI mirror
KRS_OK, KRS_E_INVALID, KRS_E_OOM, KRS_E_NOT_SPD, KRS_E_COARSE_SINGULAR, KRS_E_MAXIT, KRS_E_DEVICE, KRS_E_BUSY, \
    KRS_E_STATE = range(9)
PRECISION = {"fp64": 0, "mixed": 1, "fp32": 2, "fp32basis": 3}
REUSE = {"none": 0, "total": 1, "trks": 1, "selective": 2, "srks": 2}
PRECOND = {"jacobi": 0, "bjacobi3": 1, "block3": 1}
CAP_POLICY = {"restart": 0, "freeze": 1, "cost": 2}
NC_LIM_AUTO = -1  # max_basis: n_c_lim from the complexity analysis on the first solve

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U8 = ctypes.POINTER(ctypes.c_uint8)


class SeqDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("block", ctypes.c_int32),
        ("nnzb", ctypes.c_int64),
        ("row_ptr", _I64),
        ("col_idx", _I32),
        ("precision", ctypes.c_int),
        ("reuse", ctypes.c_int),
        ("precond", ctypes.c_int),
        ("cap_policy", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("ritz_eps", ctypes.c_double),
        ("max_basis", ctypes.c_int32),
        ("refine_every", ctypes.c_int32),
        ("history_cap", ctypes.c_int32),
        ("rank_tol", ctypes.c_double),
        ("refine_drop", ctypes.c_double),
        ("exec_mode", ctypes.c_int32),
        ("update_rows", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("kernel_flags", ctypes.c_int32),
        ("reselect", ctypes.c_int32),
        ("cluster_min_frac", ctypes.c_double),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("n_c", ctypes.c_int32),
        ("refinements", ctypes.c_int32),
        ("selected", ctypes.c_int32),
        ("dropped", ctypes.c_int32),
        ("added", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("update_rows", ctypes.c_int32),
        ("rel_res_true", ctypes.c_double),
        ("rel_res_recursive", ctypes.c_double),
        ("t_setup_ms", ctypes.c_double),
        ("t_rebuild_ms", ctypes.c_double),
        ("t_iter_ms", ctypes.c_double),
        ("t_recycle_ms", ctypes.c_double),
        ("model_bytes", ctypes.c_int64),
        ("n_c_lim", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Completion(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_uint64),
        ("seq", ctypes.c_void_p),
        ("status", ctypes.c_int32),
        ("batch_size", ctypes.c_int32),
        ("latency_ms", ctypes.c_double),
        ("queue_ms", ctypes.c_double),
        ("info", SolveInfo),
        ("message", ctypes.c_char * 128),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("enqueued", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("queued", ctypes.c_int64),
        ("blocks", ctypes.c_int64),
        ("mean_batch", ctypes.c_double),
        ("solves_per_s", ctypes.c_double),
        ("p50_ms", ctypes.c_double),
        ("p99_ms", ctypes.c_double),
        ("mean_ms", ctypes.c_double),
        ("peak_bytes", ctypes.c_int64),
    ]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_S = ctypes.c_int

# (name, restype, argtypes): every entry point declared in include/krs.h
SIGNATURES = [
    ("krs_ctx_create", _S, [ctypes.c_int, _P, ctypes.POINTER(Allocator), _PP]),
    ("krs_ctx_destroy", _S, [_P]),
    ("krs_status_str", ctypes.c_char_p, [_S]),
    ("krs_last_error", ctypes.c_char_p, []),
    ("krs_version", ctypes.c_char_p, []),
    ("krs_seq_create", _S, [_P, ctypes.POINTER(SeqDesc), _D, ctypes.c_int32, ctypes.c_int64, _PP]),
    ("krs_seq_submit", _S, [_P, _D, _D]),
    ("krs_seq_submit_device", _S, [_P, _P, _P]),
    ("krs_seq_solve", _S, [_P, _D, ctypes.POINTER(SolveInfo)]),
    ("krs_seq_solve_device", _S, [_P, _P, ctypes.POINTER(SolveInfo)]),
    ("krs_seq_recycle", _S, [_P, _I32]),
    ("krs_seq_ritz", _S, [_P, _D, _U8, ctypes.c_int32, _I32]),
    ("krs_seq_coeffs", _S, [_P, _D, _D, _D, ctypes.c_int32, _I32]),
    ("krs_seq_basis", _S, [_P, _D, ctypes.c_int64, ctypes.c_int32, _I32]),
    ("krs_seq_history", _S, [_P, _D, ctypes.c_int64, ctypes.c_int32, _I32]),
    ("krs_seq_basis_noalloc", _S, [_P, _D, ctypes.c_int64, ctypes.c_int32, _I32]),
    ("krs_seq_info", _S, [_P, ctypes.POINTER(SolveInfo)]),
    ("krs_seq_set_timing", _S, [_P, ctypes.c_int32]),
    ("krs_seq_kernel_time", _S, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), _D]),
    ("krs_seq_destroy", _S, [_P]),
    ("krs_batch_solve", _S, [_P, _PP, ctypes.c_int32, ctypes.POINTER(_D), ctypes.POINTER(SolveInfo)]),
    ("krs_batch_solve_device", _S, [_P, _PP, ctypes.c_int32, _PP, ctypes.POINTER(SolveInfo)]),
    ("krs_batch_recycle", _S, [_P, _PP, ctypes.c_int32, _I32]),
    ("krs_batch_solve_recycle", _S, [_P, _PP, ctypes.c_int32, _PP, ctypes.POINTER(SolveInfo), _I32]),
    ("krs_server_create", _S, [_P, ctypes.c_size_t, ctypes.c_int32, _PP]),
    ("krs_server_enqueue", _S, [_P, _P, _D, _D, _D, ctypes.c_uint64]),
    ("krs_server_poll", _S, [_P, ctypes.POINTER(Completion), ctypes.c_int32, _I32, ctypes.c_int32]),
    ("krs_server_stats", _S, [_P, ctypes.POINTER(ServerStats)]),
    ("krs_server_destroy", _S, [_P]),
    ("krs_nc_limit", _S, [_D, _D, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, ctypes.c_int32, ctypes.c_double, _D, _I32, _I32]),
    ("krs_cluster_reselect", _S, [_D, ctypes.c_int32, ctypes.c_double, _U8]),
    ("krs_ritz_select", _S, [_D, _D, ctypes.c_int32, ctypes.c_double, _D, _D, _U8]),
    ("krs_coarse_factor", _S, [ctypes.c_int32, _D, ctypes.c_double, _D, _U8, _I32]),
]

for _name, _res, _args in SIGNATURES:
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class KrsError(RuntimeError):
    def __init__(self, status, where):
        msg = _lib.krs_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.krs_status_str(status).decode()} ({status}): {msg}")
        self.status = status


def _check(status, where, allow=()):
    if status != KRS_OK and status not in allow:
        raise KrsError(status, where)
    return status


def _dptr(a):
    return a.ctypes.data_as(_D)


def lib():
    return _lib


def version():
    return _lib.krs_version().decode()


# ------------------------------------------------------- host-side logic

def ritz_select(alpha, rho, eps):
    """Library's Ritz analysis on given CG coefficients (no device used).

    Returns (theta_m descending, theta_{m-1} descending, selected bool[m]).
    """
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    m = len(alpha)
    th = np.zeros(max(m, 1))
    th1 = np.zeros(max(m - 1, 1))
    sel = np.zeros(max(m, 1), dtype=np.uint8)
    _check(_lib.krs_ritz_select(_dptr(alpha), _dptr(rho), m, float(eps), _dptr(th), _dptr(th1),
                                sel.ctypes.data_as(_U8)), "krs_ritz_select")
    return th[:m], th1[: max(m - 1, 0)], sel[:m].astype(bool)


def nc_limit(alpha, rho, bytes_iter0, bytes_col_iter, bytes_rebuild0, bytes_col_rebuild, kmax, eps=1e-8):
    """Library's complexity analysis for n_c_lim (no device used).

    Returns (n_c_lim, modelled bytes per system for k = 0..kmax')."""
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    cost = np.zeros(int(kmax) + 1)
    k = ctypes.c_int32(0)
    nl = ctypes.c_int32(0)
    _check(_lib.krs_nc_limit(_dptr(alpha), _dptr(rho), len(alpha), float(bytes_iter0), float(bytes_col_iter),
                             float(bytes_rebuild0), float(bytes_col_rebuild), int(kmax), float(eps), _dptr(cost),
                             ctypes.byref(k), ctypes.byref(nl)), "krs_nc_limit")
    return nl.value, cost[: k.value + 1]


def cluster_reselect(theta, selected, min_frac=0.2):
    """Library's cluster reselection (no device used): theta (any order) and
    a bool preselection; returns the bool flags kept."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    fl = np.ascontiguousarray(np.asarray(selected, dtype=bool).astype(np.uint8))
    _check(_lib.krs_cluster_reselect(_dptr(th), len(th), float(min_frac), fl.ctypes.data_as(_U8)),
           "krs_cluster_reselect")
    return fl.astype(bool)


def coarse_factor(G, rank_tol=1e-6):
    """Library's guarded Cholesky + inverse of a coarse matrix (no device used)."""
    G = np.asfortranarray(G, dtype=np.float64)
    nc = G.shape[0]
    Ginv = np.zeros((nc, nc), order="F")
    kept = np.zeros(max(nc, 1), dtype=np.uint8)
    nk = ctypes.c_int32(0)
    st = _lib.krs_coarse_factor(nc, _dptr(G), float(rank_tol), _dptr(Ginv), kept.ctypes.data_as(_U8),
                                ctypes.byref(nk))
    _check(st, "krs_coarse_factor", allow=(KRS_E_COARSE_SINGULAR,))
    return Ginv, kept[:nc].astype(bool), nk.value


# ---------------------------------------------------------------- device

class Context:
    """A libkrs context on one HIP device, bound to torch's current stream
    and caching allocator."""

    def __init__(self, device: int = 0, use_torch: bool = True):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible")
        torch.cuda.set_device(device)
        self.device = device
        self._torch = torch
        self._keep = []
        alloc = None
        if use_torch:
            def _alloc(user, nbytes, stream):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
                except Exception:
                    return None

            def _free(user, ptr, stream):
                torch.cuda.caching_allocator_delete(ptr)

            a_fn, f_fn = _ALLOC_FN(_alloc), _FREE_FN(_free)
            self._keep += [a_fn, f_fn]
            alloc = Allocator(a_fn, f_fn, None)
        stream = torch.cuda.current_stream(device).cuda_stream
        self._stream = stream
        h = ctypes.c_void_p()
        _check(_lib.krs_ctx_create(device, ctypes.c_void_p(stream), ctypes.byref(alloc) if alloc else None,
                                   ctypes.byref(h)), "krs_ctx_create")
        self._alloc_struct = alloc
        self.handle = h
        self._seqs = []

    def close(self):
        if self.handle:
            for s in list(self._seqs):
                s.close()
            _check(_lib.krs_ctx_destroy(self.handle), "krs_ctx_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def batch_solve(self, seqs, xs=None):
        """Solve the submitted systems of several sequences in fused launches.

        ``xs``: optional list of float64 device tensors (one per sequence)
        that receive the solutions; otherwise host numpy arrays are returned.
        Returns (xs, [info dict per sequence])."""
        cnt = len(seqs)
        arr_h = (ctypes.c_void_p * cnt)(*[s.handle.value for s in seqs])
        infos = (SolveInfo * cnt)()
        if xs is None:
            xs = [np.zeros(s.n) for s in seqs]
            arr_x = (_D * cnt)(*[_dptr(x) for x in xs])
            st = _lib.krs_batch_solve(self.handle, ctypes.cast(arr_h, _PP), cnt, arr_x, infos)
            _check(st, "krs_batch_solve", allow=(KRS_E_MAXIT,))
        else:
            arr_x = (ctypes.c_void_p * cnt)(*[x.data_ptr() for x in xs])
            st = _lib.krs_batch_solve_device(self.handle, ctypes.cast(arr_h, _PP), cnt, ctypes.cast(arr_x, _PP),
                                             infos)
            _check(st, "krs_batch_solve_device", allow=(KRS_E_MAXIT,))
        return xs, [infos[i].as_dict() for i in range(cnt)]

    def batch_solve_recycle(self, seqs, xs):
        """batch_solve into the device tensors ``xs`` followed by
        batch_recycle, each member's recycle planned as soon as it finishes.
        Returns ([info dict per sequence], [columns appended per sequence])."""
        cnt = len(seqs)
        arr_h = (ctypes.c_void_p * cnt)(*[s.handle.value for s in seqs])
        infos = (SolveInfo * cnt)()
        added = (ctypes.c_int32 * max(cnt, 1))()
        arr_x = (ctypes.c_void_p * cnt)(*[x.data_ptr() for x in xs])
        st = _lib.krs_batch_solve_recycle(self.handle, ctypes.cast(arr_h, _PP), cnt, ctypes.cast(arr_x, _PP), infos,
                                          ctypes.cast(added, _I32))
        _check(st, "krs_batch_solve_recycle", allow=(KRS_E_MAXIT,))
        return [infos[i].as_dict() for i in range(cnt)], [int(added[i]) for i in range(cnt)]

    def batch_recycle(self, seqs):
        """krs_seq_recycle for several sequences (host work in parallel);
        returns the number of columns appended to each."""
        cnt = len(seqs)
        arr_h = (ctypes.c_void_p * cnt)(*[s.handle.value for s in seqs])
        added = (ctypes.c_int32 * max(cnt, 1))()
        _check(_lib.krs_batch_recycle(self.handle, ctypes.cast(arr_h, _PP), cnt,
                                      ctypes.cast(added, _I32)), "krs_batch_recycle")
        return [int(added[i]) for i in range(cnt)]


class Sequence:
    """One sequence of systems on a fixed sparsity pattern.

    ``row_ptr``/``col_idx``: (block) CSR pattern; ``block``: 1 or 3.
    """

    def __init__(self, ctx: Context, row_ptr, col_idx, n, block=1, precision="fp64", reuse="selective",
                 precond=None, cap_policy="freeze", tol=1e-8, max_iter=10000, ritz_eps=1e-14, max_basis=0,
                 refine_every=0, history_cap=0, rank_tol=0.0, refine_drop=0.0, C0=None, eager=False,
                 update_rows=0, autotune=False, separate_finalize=False, literal_direction=False, reorth=False,
                 spmv_variant=0, history_fp32=False, reselect=None,
                 cluster_min_frac=0.0, plain_stores=False):
        self.ctx = ctx
        self.n = int(n)
        self.block = int(block)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.nnzb = len(ci)
        if precond is None:
            precond = "bjacobi3" if block == 3 else "jacobi"
        d = SeqDesc()
        d.n = self.n
        d.block = self.block
        d.nnzb = self.nnzb
        d.row_ptr = rp.ctypes.data_as(_I64)
        d.col_idx = ci.ctypes.data_as(_I32)
        d.precision = PRECISION[precision]
        d.reuse = REUSE[reuse]
        d.precond = PRECOND[precond]
        d.cap_policy = CAP_POLICY[cap_policy]
        d.tol = tol
        d.max_iter = max_iter
        d.ritz_eps = ritz_eps
        d.max_basis = max_basis
        d.refine_every = refine_every
        d.history_cap = history_cap
        d.rank_tol = rank_tol
        d.refine_drop = refine_drop
        d.exec_mode = 1 if eager else 0
        d.update_rows = update_rows
        d.autotune = 1 if autotune else 0
        d.kernel_flags = ((1 if separate_finalize else 0) | (2 if literal_direction else 0) | (4 if reorth else 0)
                          | ((int(spmv_variant) & 15) << 3) | (128 if history_fp32 else 0)
                          | (256 if plain_stores else 0))
        d.reselect = {None: 0, "none": 0, "cluster": 1}[reselect]
        d.cluster_min_frac = cluster_min_frac
        self.desc = d
        h = ctypes.c_void_p()
        if C0 is not None and C0.shape[1] > 0:
            C0 = np.asfortranarray(C0, dtype=np.float64)
            _check(_lib.krs_seq_create(ctx.handle, ctypes.byref(d), _dptr(C0), C0.shape[1], C0.shape[0],
                                       ctypes.byref(h)), "krs_seq_create")
        else:
            _check(_lib.krs_seq_create(ctx.handle, ctypes.byref(d), None, 0, self.n, ctypes.byref(h)),
                   "krs_seq_create")
        self.handle = h
        ctx._seqs.append(self)

    # -- data
    def submit(self, values, b):
        """Load a system: numpy arrays (host, copied) or torch device tensors (borrowed)."""
        torch = self.ctx._torch
        if isinstance(values, torch.Tensor):
            assert values.is_cuda and b.is_cuda and values.dtype == torch.float64 and b.dtype == torch.float64
            values = values.contiguous()
            b = b.contiguous()
            _check(_lib.krs_seq_submit_device(self.handle, ctypes.c_void_p(values.data_ptr()),
                                              ctypes.c_void_p(b.data_ptr())), "krs_seq_submit_device")
            return
        v = np.ascontiguousarray(values, dtype=np.float64)
        bb = np.ascontiguousarray(b, dtype=np.float64)
        if v.size != self.nnzb * self.block * self.block or bb.size != self.n:
            raise ValueError("values / b have the wrong size")
        _check(_lib.krs_seq_submit(self.handle, _dptr(v), _dptr(bb)), "krs_seq_submit")

    def solve(self, allow_maxit=True):
        """Solve the submitted system; returns (x numpy float64[n], info dict)."""
        x = np.zeros(self.n)
        info = SolveInfo()
        allow = (KRS_E_MAXIT,) if allow_maxit else ()
        _check(_lib.krs_seq_solve(self.handle, _dptr(x), ctypes.byref(info)), "krs_seq_solve", allow=allow)
        return x, info.as_dict()

    def solve_device(self, x_tensor, allow_maxit=True):
        info = SolveInfo()
        allow = (KRS_E_MAXIT,) if allow_maxit else ()
        _check(_lib.krs_seq_solve_device(self.handle, ctypes.c_void_p(x_tensor.data_ptr()), ctypes.byref(info)),
               "krs_seq_solve_device", allow=allow)
        return info.as_dict()

    def recycle(self):
        k = ctypes.c_int32(0)
        _check(_lib.krs_seq_recycle(self.handle, ctypes.byref(k)), "krs_seq_recycle")
        return k.value

    def ritz(self):
        m = ctypes.c_int32(0)
        _check(_lib.krs_seq_ritz(self.handle, None, None, 0, ctypes.byref(m)), "krs_seq_ritz")
        th = np.zeros(max(m.value, 1))
        sel = np.zeros(max(m.value, 1), dtype=np.uint8)
        _check(_lib.krs_seq_ritz(self.handle, _dptr(th), sel.ctypes.data_as(_U8), len(th), ctypes.byref(m)),
               "krs_seq_ritz")
        return th[: m.value], sel[: m.value].astype(bool)

    def coeffs(self):
        m = ctypes.c_int32(0)
        _check(_lib.krs_seq_coeffs(self.handle, None, None, None, 0, ctypes.byref(m)), "krs_seq_coeffs")
        k = max(m.value, 1)
        a, r, g = np.zeros(k), np.zeros(k), np.zeros(k)
        _check(_lib.krs_seq_coeffs(self.handle, _dptr(a), _dptr(r), _dptr(g), k, ctypes.byref(m)), "krs_seq_coeffs")
        mm = m.value
        return a[:mm], r[:mm], g[:mm]

    @property
    def n_c(self):
        k = ctypes.c_int32(0)
        _check(_lib.krs_seq_basis(self.handle, None, self.n, 0, ctypes.byref(k)), "krs_seq_basis")
        return k.value

    def basis(self):
        nc = self.n_c
        C = np.zeros((self.n, max(nc, 1)), order="F")
        k = ctypes.c_int32(0)
        _check(_lib.krs_seq_basis(self.handle, _dptr(C), self.n, C.shape[1], ctypes.byref(k)), "krs_seq_basis")
        return C[:, :nc]

    def history(self):
        """z_j kept in the Krylov history by the last solve (n x m', float64)."""
        m = ctypes.c_int32(0)
        _check(_lib.krs_seq_history(self.handle, None, self.n, 0, ctypes.byref(m)), "krs_seq_history")
        Z = np.zeros((self.n, max(m.value, 1)), order="F")
        _check(_lib.krs_seq_history(self.handle, _dptr(Z), self.n, Z.shape[1], ctypes.byref(m)), "krs_seq_history")
        return Z[:, : m.value]

    def basis_noalloc(self):
        """The basis through krs_seq_basis_noalloc (no device allocation)."""
        nc = self.n_c
        C = np.zeros((self.n, max(nc, 1)), order="F")
        k = ctypes.c_int32(0)
        _check(_lib.krs_seq_basis_noalloc(self.handle, _dptr(C), self.n, C.shape[1], ctypes.byref(k)),
               "krs_seq_basis_noalloc")
        return C[:, :nc]

    def set_timing(self, enable=True):
        _check(_lib.krs_seq_set_timing(self.handle, 1 if enable else 0), "krs_seq_set_timing")

    def kernel_time(self, kernel):
        """(sampled launches, mean duration ms) of kernel 0 (SpMV), 1 (update), 2 (direction)."""
        cnt = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        _check(_lib.krs_seq_kernel_time(self.handle, kernel, ctypes.byref(cnt), ctypes.byref(ms)),
               "krs_seq_kernel_time")
        return cnt.value, (ms.value / cnt.value if cnt.value else float("nan"))

    def info(self):
        info = SolveInfo()
        _check(_lib.krs_seq_info(self.handle, ctypes.byref(info)), "krs_seq_info")
        return info.as_dict()

    def close(self):
        if self.handle:
            _check(_lib.krs_seq_destroy(self.handle), "krs_seq_destroy")
            self.handle = None
            if self in self.ctx._seqs:
                self.ctx._seqs.remove(self)


class Server:
    """Continuous-batching server over the sequences of one context.

    ``hbm_budget``: bytes of solve-time working sets admitted at once (0: no
    limit); ``max_slots``: systems in flight at once.  While it exists the
    server's worker owns the context's stream."""

    def __init__(self, ctx: Context, hbm_budget=0, max_slots=64):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(_lib.krs_server_create(ctx.handle, int(hbm_budget), int(max_slots), ctypes.byref(h)),
               "krs_server_create")
        self.handle = h
        self._pending = {}  # tag -> (sequence, x, values, b) kept alive until completion

    def enqueue(self, seq, values, b, tag):
        """Queue one system of ``seq`` (host arrays, copied); the solution
        arrives with the completion of ``tag``."""
        v = np.ascontiguousarray(values, dtype=np.float64)
        bb = np.ascontiguousarray(b, dtype=np.float64)
        if v.size != seq.nnzb * seq.block * seq.block or bb.size != seq.n:
            raise ValueError("values / b have the wrong size")
        x = np.zeros(seq.n)
        if int(tag) in self._pending:
            raise ValueError(f"tag {tag} is already in flight")
        self._pending[int(tag)] = (seq, x)  # before the call: the completion may arrive at once
        st = _lib.krs_server_enqueue(self.handle, seq.handle, _dptr(v), _dptr(bb), _dptr(x), int(tag))
        if st != KRS_OK:
            self._pending.pop(int(tag), None)
        _check(st, "krs_server_enqueue")

    def poll(self, timeout_ms=-1, cap=256):
        """Completed requests: list of dicts with tag, status, latency_ms,
        queue_ms, batch_size, info and x."""
        buf = (Completion * cap)()
        cnt = ctypes.c_int32(0)
        _check(_lib.krs_server_poll(self.handle, buf, cap, ctypes.byref(cnt), int(timeout_ms)), "krs_server_poll")
        out = []
        for i in range(cnt.value):
            c = buf[i]
            seq, x = self._pending.pop(int(c.tag))
            out.append(dict(tag=int(c.tag), status=int(c.status), latency_ms=c.latency_ms, queue_ms=c.queue_ms,
                            batch_size=int(c.batch_size), info=c.info.as_dict(), x=x, seq=seq,
                            message=c.message.decode(errors="replace")))
        return out

    def stats(self):
        st = ServerStats()
        _check(_lib.krs_server_stats(self.handle, ctypes.byref(st)), "krs_server_stats")
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self):
        if self.handle:
            _check(_lib.krs_server_destroy(self.handle), "krs_server_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def sequence_for(ctx, seq, **kw):
    """Sequence handle for a ``gen`` workload object (pattern taken from it)."""
    return Sequence(ctx, seq.row_ptr, seq.col_idx, seq.n, block=getattr(seq, "block", 1), **kw)


__all__ = ["Context", "Sequence", "Server", "KrsError", "ritz_select", "nc_limit", "cluster_reselect", "coarse_factor", "sequence_for", "version", "lib",
           "SIGNATURES", "LIB_PATH"]
