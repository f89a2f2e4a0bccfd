"""Write the FP64 oracle fixtures used by the full-size GPU parity tests.

Calls only ``oracle`` (and the input generators of ``gen``); nothing here
comes from the HIP library.  Run from the repository root:

    python tests/golden/make_fixtures.py [name ...]
    python tests/golden/make_fixtures.py --draws name [n_perturbed [workers]]

Each fixture is a JSON file with, per system of an SRKS sequence (Algorithm
3, 3x3 block-Jacobi, FP64, tol 1e-8, with or without full
reorthogonalisation as the fixture states; the direction update in the form
w = z + beta P w_old, which equals Algorithm 1's w = z + beta w_old in exact
arithmetic and is the library's default): the iteration count, the
basis width before the solve and after the recycle, the selected Ritz
indices, the first CG coefficients, the true relative residual, and a
fingerprint of the span of the recycled basis: with R a seeded n x 8 probe,
F = (Q^T R)^T (Q^T R) for Q an orthonormal basis of span(C), which depends on
the span only (any basis of it, A-orthonormalised or not, gives the same F).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle as O  # noqa: E402

FIXTURES = {
    # the 40^3 elasticity workload, first three systems, cap 60 (freeze)
    "elasticity40_srks_fp64": dict(E=40, workload_id=2, systems=3, cap=60, eps=1e-8, max_iter=30000),
    # the 100^3 workload's setup at 30^3, its first eight systems, cap 200
    # (freeze), the paper's eps = 1e-14 (at 1e-8 the first system's 200
    # smallest stagnated values include copies whose vectors stall the next
    # solve near 4e-7 on the oracle)
    "elasticity30_srks_fp64": dict(E=30, workload_id=3, systems=8, cap=200, eps=1e-14, max_iter=30000),
    # the 40^3 workload with n_c_lim from the complexity analysis of the
    # first solve (byte model of the library's FP64 iteration), freeze cap
    "elasticity40_auto_fp64": dict(E=40, workload_id=2, systems=4, cap="auto", eps=1e-8, max_iter=30000),
    # the 40^3 workload's setup at 24^3 with full reorthogonalisation (the
    # remark of Section 2.1, the setting of Section 5.1) at eps = 1e-14
    "elasticity24_reorth_fp64": dict(E=24, workload_id=2, systems=3, cap=60, eps=1e-14, max_iter=4096,
                                     reorth=True),
    # the 40^3 workload's first system with full reorthogonalisation at
    # eps = 1e-14; the reruns under other roundings are skipped (with
    # reorthogonalisation they agree to the iteration at 24^3)
    "elasticity40_reorth_fp64": dict(E=40, workload_id=2, systems=1, cap=60, eps=1e-14, max_iter=8192,
                                     reorth=True, faithful=False),
}


def cost_model_fp64(seq, kmax):
    """Algorithmic bytes of the FP64 iteration and rebuild (3x3 blocks):
    matrix values and block columns, the block preconditioner, ten vector
    passes plus x read and written; two passes over a basis column per
    iteration; the rebuild streams A once and seven passes per column."""
    nnz = 9 * seq.nnzb
    BA = nnz * 8 + 4 * seq.nnzb
    BM = 3 * seq.n * 8
    return dict(bytes_iter0=BA + BM + 10 * seq.n * 8 + 2 * seq.n * 8, bytes_col_iter=2 * seq.n * 8,
                bytes_rebuild0=BA, bytes_col_rebuild=7 * seq.n * 8, kmax=kmax)
N_COEF = 40


def probe(n: int) -> np.ndarray:
    return np.random.default_rng(np.random.SeedSequence([13017530, 99, n])).standard_normal((n, 8))


def span_fingerprint(C: np.ndarray, R: np.ndarray) -> np.ndarray:
    if C.shape[1] == 0:
        return np.zeros((R.shape[1], R.shape[1]))
    U, s, _ = np.linalg.svd(C, full_matrices=False)
    Q = U[:, s > s[0] * 1e-10]
    P = Q.T @ R
    return P.T @ P


def make(name: str) -> None:
    cfg = FIXTURES[name]
    seq = gen.config_elasticity(cfg["E"], cfg["systems"], cfg["workload_id"])
    R = probe(seq.n)
    t = time.perf_counter()
    recs = []
    C = np.zeros((seq.n, 0))
    cap = cfg["cap"]
    nc_lim = None
    for k in range(cfg["systems"]):
        rp, ci, v, b = seq.csr(k)
        ro = cfg.get("reorth", False)
        res = O.apcg(rp, ci, v, b, "block3", C=C, tol=1e-8, max_iter=cfg["max_iter"], record_z=True,
                     direction="project_old", reorth=ro)
        nc_in = C.shape[1]
        if nc_in:
            C = C[:, res["kept"]]
        C_solve = C  # the basis this solve used (after the guard), for the perturbed solves
        rec = dict(k=k, m=int(res["m"]), nc_in=int(nc_in), nc_solve=int(C.shape[1]),
                   status=int(res["status"]), relres_true=float(res["relres_true"]),
                   alpha=res["alpha"][:N_COEF].tolist(), rho=res["rho"][:N_COEF].tolist(),
                   gamma=res["gamma"][:N_COEF].tolist())
        if cap == "auto":
            nc_lim, _ = O.nc_limit(res["alpha"], res["rho"], eps=cfg["eps"],
                                   **cost_model_fp64(seq, min(1024, res["m"] - 1)))
            cap = nc_lim
            rec["nc_lim"] = int(nc_lim)
        room = cap - C.shape[1]
        sel = []
        if res["m"] > 1 and room > 0:
            th_m, th_m1 = O.ritz_values(res["alpha"], res["rho"])
            allsel = O.srks_select(th_m, th_m1, cfg["eps"])
            sel = O.freeze_pick(allsel, th_m, room)
            rec["selected_all_count"] = len(allsel)
            new = O.ritz_block(res["Z"], res["alpha"], res["rho"], sel, th_m)
            C = np.concatenate([C, new], axis=1)
        # the oracle's own sensitivity: the same solve with b perturbed at
        # the rounding level (relative 1e-15, one draw); the spread of
        # these iteration counts is what rounding alone moves
        prng = np.random.default_rng(np.random.SeedSequence([13017530, 98, k]))
        pm = []
        for _ in range(1 if cfg.get("faithful", True) else 0):
            bp = b * (1.0 + 1e-15 * prng.standard_normal(b.shape))
            pm.append(int(O.apcg(rp, ci, v, bp, "block3", C=C_solve, tol=1e-8, max_iter=cfg["max_iter"],
                                 direction="project_old", reorth=ro)["m"]))
        rec["m_perturbed"] = pm
        # and with the products accumulated in extended precision: another
        # faithful rounding of the same arithmetic
        rec["m_extended"] = (int(O.apcg(rp, ci, v, b, "block3", C=C_solve, tol=1e-8, max_iter=cfg["max_iter"],
                                        direction="project_old", extended=True, reorth=ro)["m"])
                             if cfg.get("faithful", True) else rec["m"])
        rec["selected"] = [int(i) for i in sel]
        rec["nc_next"] = int(C.shape[1])
        rec["fingerprint"] = span_fingerprint(C, R).tolist()
        recs.append(rec)
        del res
        print(f"{name} system {k}: m={rec['m']} (perturbed {pm}, extended {rec['m_extended']}) n_c {rec['nc_in']}->{rec['nc_solve']} (+{len(sel)}) "
              f"rel res {rec['relres_true']:.2e}  [{time.perf_counter() - t:.0f} s]", flush=True)
    out = dict(name=name, config=cfg, n=seq.n, n_coef=N_COEF, generator="tests/golden/make_fixtures.py",
               systems=recs)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=0)


def draw(name: str, kind: str, seed: int = 0) -> dict:
    """The whole sequence again under another faithful rounding of the same
    arithmetic: every right-hand side perturbed at the rounding level
    (relative 1e-15, seeded per system) or every product accumulated in
    extended precision.  Per system: iterations, basis width at the solve,
    columns appended and the span fingerprint.  Without reorthogonalisation
    rounding moves long runs by about 1 %, and a different run selects a
    slightly different set of Ritz vectors, which moves the later systems of
    the sequence further: the spread over such draws is the oracle's own."""
    cfg = FIXTURES[name]
    seq = gen.config_elasticity(cfg["E"], cfg["systems"], cfg["workload_id"])
    R = probe(seq.n)
    ro = cfg.get("reorth", False)
    C = np.zeros((seq.n, 0))
    cap = cfg["cap"]
    out = []
    t = time.perf_counter()
    for k in range(cfg["systems"]):
        rp, ci, v, b = seq.csr(k)
        if kind == "perturbed":
            prng = np.random.default_rng(np.random.SeedSequence([13017530, 97, k, seed]))
            b = b * (1.0 + 1e-15 * prng.standard_normal(b.shape))
        res = O.apcg(rp, ci, v, b, "block3", C=C, tol=1e-8, max_iter=cfg["max_iter"], record_z=True,
                     direction="project_old", reorth=ro, extended=(kind == "extended"))
        if C.shape[1]:
            C = C[:, res["kept"]]
        nc_solve = C.shape[1]
        if cap == "auto":
            cap, _ = O.nc_limit(res["alpha"], res["rho"], eps=cfg["eps"],
                                **cost_model_fp64(seq, min(1024, res["m"] - 1)))
        room = cap - C.shape[1]
        sel = []
        if res["m"] > 1 and room > 0:
            th_m, th_m1 = O.ritz_values(res["alpha"], res["rho"])
            sel = O.freeze_pick(O.srks_select(th_m, th_m1, cfg["eps"]), th_m, room)
            C = np.concatenate([C, O.ritz_block(res["Z"], res["alpha"], res["rho"], sel, th_m)], axis=1)
        out.append(dict(k=k, m=int(res["m"]), nc_solve=int(nc_solve), added=len(sel),
                        fingerprint=span_fingerprint(C, R).tolist()))
        del res
        print(f"{name} draw {kind} system {k}: m={out[-1]['m']} n_c {nc_solve} (+{len(sel)})  "
              f"[{time.perf_counter() - t:.0f} s]", flush=True)
    return dict(kind=kind, seed=seed, systems=out)


def _draw_task(task):
    return draw(*task)


def add_draws(name: str, n_perturbed: int = 1, workers: int = 1) -> None:
    """Reruns of the whole sequence: n_perturbed seeds of the perturbed
    right-hand sides and one with extended-precision accumulation."""
    tasks = [(name, "perturbed", i) for i in range(n_perturbed)] + [(name, "extended", 0)]
    if workers > 1:
        import multiprocessing as mp

        with mp.get_context("fork").Pool(workers) as pool:
            draws = pool.map(_draw_task, tasks)
    else:
        draws = [_draw_task(t) for t in tasks]
    path = os.path.join(HERE, name + ".json")
    with open(path) as f:
        fx = json.load(f)
    fx["sequence_draws"] = draws
    with open(path, "w") as f:
        json.dump(fx, f, indent=0)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--draws":
        # --draws NAME [N_PERTURBED [WORKERS]]
        add_draws(args[1], int(args[2]) if len(args) > 2 else 1, int(args[3]) if len(args) > 3 else 1)
    else:
        for nm in args or list(FIXTURES):
            make(nm)
