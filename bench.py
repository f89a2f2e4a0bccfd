#!/usr/bin/env python3
"""Throughput benchmark of the Krylov-reuse APCG library on one GPU.

A step is one system of the sequence taken through the whole hot path:
intake of the new matrix values and right-hand side (already resident in
HBM), rebuild of A C and C^T A C for the carried basis, the APCG iterations
to a true relative residual of 1e-8, and the Ritz extraction / selection /
basis update (SRKS).  The same systems are then solved with plain PCG
(no basis) on the same GPU for comparison.

Default workload: Q1 elasticity on a 40^3 mesh (n = 201,720 dofs,
15,548,742 nonzeros in 3x3 blocks), 64 stiff cubic inclusions, cumulative
damage between systems, 3x3 block-Jacobi, SRKS with eps = 1e-8 and a basis
of at most 60 vectors (frozen once full); double-precision operator and
vectors with the basis and preconditioner streamed in single precision
(--precision fp32basis; "mixed" also rounds the matrix values, which on this
stiff-inclusion problem costs about half again as many iterations).

Other workloads: --workload batched (many diffusion sequences in fused
launches), --workload serving (Poisson arrivals into the continuous-batching
server), elasticity100, diffusion20.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32basis|mixed|fp64|fp32]

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s

# Bytes per launch of k_spmv_dot read from the hardware counters
# (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000 KiB, the factors from a 1 GiB
# device copy), by (workload, precision); kept only while the kernel is the
# one the counters were taken on.
TRAFFIC_K1 = {("elasticity40", "fp32basis"): 146268827}

WORKLOADS = {
    "elasticity40": dict(kind="elasticity", size=40, n_systems=20, workload_id=2, max_basis=60, eps=1e-8),
    # the whole Krylov run is kept (16000 x 3.06 M single-precision vectors,
    # 196 GB): with a shorter history only the top of the spectrum stagnates
    "elasticity100": dict(kind="elasticity", size=100, n_systems=30, workload_id=3, max_basis=200, eps=1e-8,
                          history_cap=16000),
    "diffusion20": dict(kind="diffusion", size=(20, 20, 20), n_systems=8, workload_id=1, max_basis=0, eps=1e-14),
    # many independent diffusion sequences (n ~ U[5e3, 2e5]) solved in fused launches
    # fused launches use wide update tiles (fewer, longer workgroups per
    # system); the one-at-a-time comparison keeps the default tile
    "batched": dict(kind="batched", size=None, n_systems=10, workload_id=4, max_basis=60, eps=1e-8, cap_policy="cost",
                    update_rows=4096),
    # clients with elasticity sequences (1e4..5e5 dofs) served with continuous batching
    "serving": dict(kind="serving", size=None, n_systems=50, workload_id=5, max_basis=200, eps=1e-8),
    # calibration for hardware byte counters: device-to-device copies of a known size
    "copy": dict(kind="copy", size=None, n_systems=0, workload_id=0, max_basis=0, eps=0.0),
}


def _log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def spmv_bytes(seq, p, pw):
    """Algorithmic bytes of one SpMV launch: matrix values (p bytes) + block
    column indices + the vector read once + the product written once (pw)."""
    nnz = seq.nnzb * seq.block * seq.block
    if seq.block == 1:
        return nnz * (p + 4) + 2 * seq.n * pw
    return nnz * p + 4 * seq.nnzb + 2 * seq.n * pw


def run_phase(K, ctx, seq, dev_sys, reuse, args, wl, order, timing=False):
    import torch

    s = K.sequence_for(ctx, seq, precision=args.precision, reuse=reuse, tol=1e-8, max_iter=args.max_iter,
                       history_cap=wl.get("history_cap", 0),
                       ritz_eps=args.eps if args.eps else wl["eps"], max_basis=args.max_basis or wl["max_basis"],
                       cap_policy="freeze",
                       refine_drop=args.refine_drop, autotune=args.autotune, update_rows=args.update_rows,
                       eager=args.eager, separate_finalize=args.separate_finalize)
    x = torch.empty(seq.n, dtype=torch.float64, device="cuda")
    infos = []
    lat = []
    C_before = None
    try:
        for i, k in enumerate(order[: args.warmup]):
            s.submit(*dev_sys[k])
            s.solve_device(x)
            s.recycle()
        if reuse != "none":
            C_before = s.basis() if args.cpu_baseline else None
        if timing:
            s.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in order[args.warmup:]:
            ts = time.perf_counter()
            s.submit(*dev_sys[k])
            info = s.solve_device(x)
            s.recycle()
            info["added"] = s.info()["added"]
            info["t_recycle_ms"] = s.info()["t_recycle_ms"]
            infos.append(info)
            lat.append(time.perf_counter() - ts)
            _log(f"  system {k}: {info['iters']} iterations, n_c {info['n_c']}, {1e3 * lat[-1]:.1f} ms")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ktimes = [s.kernel_time(j) for j in range(3)] if timing else None
        coeffs = s.coeffs()
    finally:
        s.close()
    return dict(time=t1 - t0, infos=infos, lat=lat, ktimes=ktimes, C_before=C_before, coeffs=coeffs)


def cpu_baseline(seq, k, C, m_avg, sample_iters, coeffs):
    """Time the oracle on a bounded sample of the same workload."""
    import oracle as O

    rp, ci, v, b = seq.csr(k)
    pc = "block3" if seq.block == 3 else "jacobi"
    t = time.perf_counter()
    O.apcg(rp, ci, v, b, pc, C=C, tol=1e-8, max_iter=1)
    t_first = time.perf_counter() - t
    t = time.perf_counter()
    O.apcg(rp, ci, v, b, pc, C=C, tol=1e-8, max_iter=1 + sample_iters)
    t_long = time.perf_counter() - t
    t_iter = max(t_long - t_first, 1e-9) / sample_iters
    # Ritz analysis of an m-step run: the oracle bisects every eigenvalue of
    # H_m and H_{m-1} (about 70 Sturm counts of length m each); time a few
    # counts on the GPU run's own coefficients and scale
    alpha, rho = coeffs
    m = max(len(alpha), 2)
    d, l2 = O.lanczos_factors(alpha, rho)
    dd = np.ascontiguousarray(d)
    ll = np.ascontiguousarray(l2 if len(l2) else np.zeros(1))
    lib = O.lib()
    pre = 64
    t = time.perf_counter()
    for j in range(pre):
        lib.orc_ldl_count(len(dd), O._p(dd), O._p(ll), float(j) / pre)
    t_count = (time.perf_counter() - t) / pre
    t_ritz = 2 * m * 70 * t_count
    solve_s = t_first + (m_avg - 1) * t_iter + t_ritz
    return dict(value=1.0 / solve_s, unit="solves/s", cores=1, kind="oracle",
                sample=(f"oracle (C, fp64, 1 thread) on system {k} of the same sequence with the GPU's basis "
                        f"(n_c={0 if C is None else C.shape[1]}): build + {sample_iters} APCG iterations timed "
                        f"({t_first:.2f}s first iteration incl. coarse build, {t_iter*1e3:.1f} ms/iteration), "
                        f"Ritz bisection timed on {pre} Sturm counts of length {m} (the GPU run's coefficients); "
                        f"scaled to the GPU's mean "
                        f"{m_avg:.0f} iterations per solve"),
                seconds_per_solve=solve_s)


def _gen_system(task):
    shape, seq_id, k, n_systems = task
    import gen

    sq = gen.make_sequence("diffusion", shape, n_systems, 4, seq_id)
    vals, b = sq.system(k)
    return seq_id, k, vals, b


def gen_batched(args):
    """Host data of the batched workload, generated by worker processes
    before this process touches the GPU."""
    import concurrent.futures as cf

    import gen

    wl = WORKLOADS["batched"]
    shapes = gen.batched_diffusion_sizes(args.sequences)
    nsys = wl["n_systems"]
    ks = [k % nsys for k in range(args.warmup + args.steps)]
    seqs = [gen.make_sequence("diffusion", sh, nsys, 4, i) for i, sh in enumerate(shapes)]
    _log(f"batched: {len(seqs)} sequences, sum n = {sum(sq.n for sq in seqs)}, "
         f"generating {len(set(ks))} systems each")
    tasks = [(sh, i, k, nsys) for i, sh in enumerate(shapes) for k in sorted(set(ks))]
    host = {}
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        for i, k, vals, b in ex.map(_gen_system, tasks, chunksize=4):
            host[(i, k)] = (vals, b)
    return seqs, ks, host


def _gen_client(task):
    E, cid, systems, n_systems = task
    import gen

    sq = gen.make_sequence("elasticity", E, n_systems, 5, cid)
    return cid, [sq.system(k) for k in range(systems)]


def gen_serving(args):
    """Host data of the serving workload (worker processes, before the GPU is touched)."""
    import concurrent.futures as cf

    import gen

    wl = WORKLOADS["serving"]
    Es = gen.serving_elasticity_sizes(64)[: args.clients]
    seqs = [gen.make_sequence("elasticity", E, wl["n_systems"], 5, c) for c, E in enumerate(Es)]
    _log(f"serving: {len(seqs)} clients, dofs {min(s.n for s in seqs)}..{max(s.n for s in seqs)}, "
         f"{args.systems} systems each")
    host = {}
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        for cid, systems in ex.map(_gen_client, [(E, c, args.systems, wl["n_systems"]) for c, E in enumerate(Es)]):
            host[cid] = systems
    return seqs, host


def run_serving(args, K, torch, data):
    """Open-loop Poisson arrivals per client into the continuous-batching
    server; the same requests served one at a time for comparison."""
    import threading

    wl = WORKLOADS["serving"]
    seqs, host = data
    ctx = K.Context(0)
    kw = dict(precision=args.precision, reuse="selective", tol=1e-8, max_iter=args.max_iter,
              ritz_eps=args.eps or wl["eps"], max_basis=wl["max_basis"], cap_policy="freeze",
              history_cap=args.history_cap, refine_drop=args.refine_drop)
    rng = np.random.default_rng(np.random.SeedSequence((13017530, 5, 1 << 21)))
    arrivals = []
    for c in range(len(seqs)):
        t = np.cumsum(rng.exponential(1.0 / args.rate, size=args.systems))
        arrivals += [(float(t[k]), c, k) for k in range(args.systems)]
    arrivals.sort()

    def serve(max_slots):
        hs = [K.sequence_for(ctx, sq, **kw) for sq in seqs]
        srv = K.Server(ctx, hbm_budget=int(args.hbm_budget * (1 << 30)), max_slots=max_slots)
        done = []
        try:
            def producer():
                t0 = time.perf_counter()
                for t, c, k in arrivals:
                    dt = t - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                    srv.enqueue(hs[c], *host[c][k], tag=c * 1000 + k)

            th = threading.Thread(target=producer)
            t_start = time.perf_counter()
            th.start()
            while len(done) < len(arrivals):
                got = srv.poll(timeout_ms=60000)
                if not got:
                    raise RuntimeError("server made no progress for 60 s")
                done += got
                _log(f"served {len(done)}/{len(arrivals)}")
            th.join()
            wall = time.perf_counter() - t_start
            st = srv.stats()
        finally:
            srv.close()
            for h in hs:
                h.close()
        bad = [c for c in done if c["status"] != 0 or c["info"]["rel_res_true"] > 1e-8]
        if bad:
            raise RuntimeError(f"{len(bad)} requests missed the tolerance: {bad[0]['message']}")
        st["wall_s"] = wall
        st["iters_mean"] = float(np.mean([c["info"]["iters"] for c in done]))
        return st

    _log("continuous batching")
    cb = serve(args.clients)
    seq_st = None
    if args.plain:
        _log("one request at a time")
        seq_st = serve(1)
    ctx.close()
    n_tot = sum(sq.n for sq in seqs)
    out = {
        "metric": "solves/s at 1e-8 resid vs plain PCG same GPU; %HBM peak; p50/p99 latency",
        "value": round(cb["solves_per_s"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(arrivals),
        "warmup": 0,
        "ms_per_step": round(1e3 / cb["solves_per_s"], 3) if cb["solves_per_s"] else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f32+f64", "fp64": "f64", "fp32": "f32", "fp32basis": "f64+f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"serving: {len(seqs)} clients, Q1 elasticity "
                               f"{min(s.n for s in seqs)}..{max(s.n for s in seqs)} dofs, {args.systems} systems "
                               f"each, Poisson arrivals {args.rate}/s per client, SRKS cap {wl['max_basis']}",
                   "clients": len(seqs), "sum_n": n_tot, "rate_per_client": args.rate,
                   "hbm_budget_gib": args.hbm_budget, "precision": args.precision},
        "latency_ms": {"p50": cb["p50_ms"], "p99": cb["p99_ms"], "mean": cb["mean_ms"]},
        "mean_batch": cb["mean_batch"],
        "peak_working_set_gib": cb["peak_bytes"] / (1 << 30),
        "iters_mean": cb["iters_mean"],
    }
    if seq_st:
        out["one_at_a_time"] = {"value": round(seq_st["solves_per_s"], 4),
                                "latency_ms": {"p50": seq_st["p50_ms"], "p99": seq_st["p99_ms"]}}
        out["speedup_vs_one_at_a_time"] = cb["solves_per_s"] / seq_st["solves_per_s"]
    print(json.dumps(out), flush=True)


def run_batched(args, K, torch, data):
    """Fused multi-sequence solves (one batch_solve per step over every
    sequence) against the same sequences solved one after the other, and
    plain PCG in fused launches."""
    wl = WORKLOADS["batched"]
    seqs, ks, host = data
    n_tot = sum(sq.n for sq in seqs)
    dev = {key: (torch.from_numpy(v).to("cuda"), torch.from_numpy(b).to("cuda")) for key, (v, b) in host.items()}
    torch.cuda.synchronize()
    ctx = K.Context(0)
    kw = dict(precision=args.precision, tol=1e-8, max_iter=args.max_iter, ritz_eps=args.eps or wl["eps"],
              max_basis=wl["max_basis"], cap_policy=wl.get("cap_policy", "freeze"), history_cap=args.history_cap,
              refine_drop=args.refine_drop, separate_finalize=args.separate_finalize)
    fused_rows = args.update_rows or wl["update_rows"]

    def phase(reuse, fused):
        hs = [K.sequence_for(ctx, sq, reuse=reuse, update_rows=fused_rows if fused else 0, **kw) for sq in seqs]
        xs = [torch.empty(sq.n, dtype=torch.float64, device="cuda") for sq in seqs]
        iters, t_steps, t_rec, ncs = [], [], [], []
        try:
            for step, k in enumerate(ks):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for i, h in enumerate(hs):
                    h.submit(*dev[(i, k)])
                if fused and reuse != "none":
                    # each member's recycle planned as soon as it finishes
                    infos, _ = ctx.batch_solve_recycle(hs, xs)
                elif fused:
                    _, infos = ctx.batch_solve(hs, xs=xs)
                else:
                    infos = [h.solve_device(x) for h, x in zip(hs, xs)]
                t1 = time.perf_counter()
                if reuse != "none" and not fused:
                    for h in hs:
                        h.recycle()
                torch.cuda.synchronize()
                if step >= args.warmup:
                    t_steps.append(time.perf_counter() - t0)
                    t_rec.append(time.perf_counter() - t1)
                    iters.append([inf["iters"] for inf in infos])
                    ncs.append(float(np.mean([inf["n_c"] for inf in infos])))
                    bad = [inf for inf in infos if inf["rel_res_true"] > 1e-8 or inf["status"] != 0]
                    if bad:
                        raise RuntimeError(f"{len(bad)} systems missed the tolerance: {bad[0]}")
        finally:
            for h in hs:
                h.close()
        t = sum(t_steps)
        return dict(value=len(hs) * len(t_steps) / t, time=t, iters_mean=float(np.mean(iters)),
                    step_ms=[round(1e3 * x, 2) for x in t_steps], recycle_ms=[round(1e3 * x, 2) for x in t_rec],
                    n_c_mean=[round(x, 2) for x in ncs])

    _log("fused SRKS")
    fused = phase("selective", True)
    _log("sequential SRKS")
    alone = phase("selective", False) if args.plain else None
    _log("fused plain PCG")
    plain = phase("none", True) if args.plain else None
    ctx.close()
    out = {
        "metric": "solves/s at 1e-8 resid vs plain PCG same GPU; %HBM peak; p50/p99 latency",
        "value": round(fused["value"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * fused["time"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f32+f64", "fp64": "f64", "fp32": "f32", "fp32basis": "f64+f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"batched: {len(seqs)} diffusion sequences, n ~ U[5e3, 2e5] (sum {n_tot}), "
                               f"SRKS eps={kw['ritz_eps']:.0e} cap {wl['max_basis']} ({kw['cap_policy']}), "
                               f"fused launches",
                   "sequences": len(seqs), "sum_n": n_tot, "precision": args.precision,
                   "history_cap": args.history_cap, "update_rows_fused": fused_rows},
        "iters_mean": fused["iters_mean"],
        "step_ms": fused["step_ms"],
        "recycle_ms": fused["recycle_ms"],
        "n_c_mean_per_step": fused["n_c_mean"],
        "recycle_mode": "host Ritz work of each member started when it finishes, during the fused launches "
                        "(krs_batch_solve_recycle); recycle_ms is the part left after that call returns",
    }
    if alone:
        out["sequential"] = {"value": round(alone["value"], 4), "iters_mean": alone["iters_mean"]}
        out["speedup_vs_sequential"] = fused["value"] / alone["value"]
    if plain:
        out["plain_pcg"] = {"value": round(plain["value"], 4), "iters_mean": plain["iters_mean"]}
        out["speedup_vs_plain_pcg"] = fused["value"] / plain["value"]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="elasticity40", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["mixed", "fp64", "fp32", "fp32basis"],
                    help="default: fp32basis (elasticity, serving), mixed (batched diffusion), fp64 (diffusion20)")
    ap.add_argument("--max-iter", type=int, default=30000)
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--no-plain", dest="plain", action="store_false")
    ap.add_argument("--cpu-iters", type=int, default=100)
    ap.add_argument("--eps", type=float, default=0.0, help="SRKS stagnation tolerance (default: per workload)")
    ap.add_argument("--refine-drop", type=float, default=0.0, help="mixed: refinement trigger (0 = library default)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default update-kernel tile instead of timing candidates")
    ap.add_argument("--update-rows", type=int, default=0, help="fixed update-kernel block rows per workgroup")
    ap.add_argument("--max-basis", type=int, default=0, help="basis cap (0: the workload's)")
    ap.add_argument("--sequences", type=int, default=256, help="batched workload: number of sequences")
    ap.add_argument("--history-cap", type=int, default=256, help="batched workload: Krylov vectors kept per solve")
    ap.add_argument("--eager", action="store_true", help="launch kernels one by one instead of graph replay")
    ap.add_argument("--separate-finalize", action="store_true",
                    help="run the end-of-step reduction as its own kernel")
    ap.add_argument("--clients", type=int, default=64, help="serving workload: clients (sequences)")
    ap.add_argument("--systems", type=int, default=3, help="serving workload: systems per client")
    ap.add_argument("--rate", type=float, default=1.0, help="serving workload: arrivals per second per client")
    ap.add_argument("--hbm-budget", type=float, default=64.0, help="serving workload: working-set budget (GiB)")
    args = ap.parse_args()
    if args.precision is None:
        args.precision = {"batched": "mixed", "diffusion20": "fp64"}.get(args.workload, "fp32basis")
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one process / one GPU only", file=sys.stderr)
        sys.exit(2)

    batched_data = gen_batched(args) if args.workload == "batched" else None
    serving_data = gen_serving(args) if args.workload == "serving" else None

    import torch

    import gen
    import paper_1301_7530_amd as K

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload == "copy":
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                          "copies": args.steps}), flush=True)
        return
    if args.workload == "batched":
        run_batched(args, K, torch, batched_data)
        return
    if args.workload == "serving":
        if args.history_cap == 256:
            args.history_cap = 1000
        run_serving(args, K, torch, serving_data)
        return
    wl = WORKLOADS[args.workload]
    seq = gen.make_sequence(wl["kind"], wl["size"], wl["n_systems"], wl["workload_id"])
    total = args.warmup + args.steps
    order = [k % wl["n_systems"] for k in range(total)]
    _log(f"workload {args.workload}: n={seq.n} nnzb={seq.nnzb} block={seq.block}; generating {min(total, wl['n_systems'])} systems")
    dev_sys = {}
    for k in sorted(set(order)):
        vals, b = seq.system(k)
        dev_sys[k] = (torch.from_numpy(vals).to("cuda"), torch.from_numpy(b).to("cuda"))
    torch.cuda.synchronize()
    ctx = K.Context(0)
    _log("SRKS phase")
    srks = run_phase(K, ctx, seq, dev_sys, "selective" if wl["max_basis"] else "total", args, wl, order, timing=True)
    plain = None
    if args.plain:
        _log("plain PCG phase")
        plain = run_phase(K, ctx, seq, dev_sys, "none", args, wl, order)
    ctx.close()

    p = 8 if args.precision in ("fp64", "fp32basis") else 4       # matrix value bytes
    pw = 4 if args.precision == "fp32" else 8      # Krylov vector bytes
    value = args.steps / srks["time"]
    infos = srks["infos"]
    iters = [i["iters"] for i in infos]
    lat_ms = np.array(srks["lat"]) * 1e3
    model_bytes = sum(i["model_bytes"] for i in infos)
    k_cnt, k_ms = srks["ktimes"][0]
    kb = spmv_bytes(seq, p, pw)
    achieved = kb / (k_ms * 1e-3) if k_cnt else float("nan")
    out = {
        "metric": "solves/s at 1e-8 resid vs plain PCG same GPU; %HBM peak; p50/p99 latency",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * srks["time"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f32+f64", "fp64": "f64", "fp32": "f32", "fp32basis": "f64+f32"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: Q1 elasticity {wl['size']}^3" if wl["kind"] == "elasticity"
            else f"{args.workload}: 7-point diffusion {wl['size']}",
            "n": seq.n,
            "nnz": seq.nnzb * seq.block * seq.block,
            "systems_timed": args.steps,
            "reuse": f"SRKS eps={args.eps if args.eps else wl['eps']:.0e}" if wl["max_basis"] else "TRKS",
            "max_basis": args.max_basis or wl["max_basis"],
            "cap_policy": "freeze",
            "precond": "3x3 block-Jacobi" if seq.block == 3 else "Jacobi",
            "tol": 1e-8,
            "precision": args.precision,
            "precision_detail": {"mixed": "fp32 matrix/preconditioner/basis, fp64 vectors and reductions", "fp64": "fp64 throughout", "fp32": "fp32 matrix, basis and vectors, fp64 reductions", "fp32basis": "fp64 matrix and vectors, fp32 basis (C, AC) and preconditioner, fp64 reductions"}[args.precision],
        },
        "iters_mean": float(np.mean(iters)),
        "update_rows": sorted({i["update_rows"] for i in infos}),
        "n_c_mean": float(np.mean([i["n_c"] for i in infos])),
        "rel_res_true_max": float(max(i["rel_res_true"] for i in infos)),
        "refinements_mean": float(np.mean([i["refinements"] for i in infos])),
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "phase_ms_mean": {k: float(np.mean([i[k] for i in infos])) for k in
                          ("t_setup_ms", "t_rebuild_ms", "t_iter_ms", "t_recycle_ms")},
        "hbm_frac_model": model_bytes / srks["time"] / HBM_PEAK,
        "kernel_ms_mean": {name: srks["ktimes"][j][1] for j, name in enumerate(("spmv_dot", "update_reduce", "correct_dir"))},
        "roofline": {
            "kernel": "k_spmv_dot",
            "bound": "hbm",
            "achieved": achieved / 1e9,
            "peak": HBM_PEAK / 1e9,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK,
            "traffic": TRAFFIC_K1.get((args.workload, args.precision)),
            "algorithmic_bytes_per_launch": kb,
            "launches_sampled": k_cnt,
        },
    }
    if plain is not None:
        pv = args.steps / plain["time"]
        out["plain_pcg"] = {
            "value": round(pv, 4),
            "iters_mean": float(np.mean([i["iters"] for i in plain["infos"]])),
            "rel_res_true_max": float(max(i["rel_res_true"] for i in plain["infos"])),
        }
        out["speedup_vs_plain_pcg"] = value / pv
    if args.cpu_baseline:
        _log("CPU baseline (oracle sample)")
        k = order[args.warmup]
        a, r, _ = srks["coeffs"]
        out["cpu_baseline"] = cpu_baseline(seq, k, srks["C_before"], float(np.mean(iters)), args.cpu_iters, (a, r))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
