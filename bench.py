"""Benchmark: time to a 1e-9 solve on the d=3 level (7,6,5) grid, one MI355X.

Workload (synthetic, seeded): N = 127*63*31 = 248,031 unknowns, 7-point FD
Laplacian, f iid U[-1,1) from splitmix64 seed 2, Hilbert curve (the curve of
the paper's experiments; the Z-order run is reported beside it), P = 256
subdomains, gamma = 1/2 (100% overlap), q = 32 (N0 = 8192), omega-weighted
balanced two-level Schwarz preconditioner, outer PCG (flexible CG with FP32
factors) in FP64 to a relative residual of 1e-9.

One step = the whole hot path on a fresh right-hand side: setup (curve order,
partition, neighbour table, local assembly, batched Cholesky of the 256 local
matrices, coarse matrix and its inverse) + the outer solve.  The headline is
the FP32-factor path; the all-FP64 path is timed beside it.  Inputs are
resident in HBM before the timed region; the workspace is allocated once.

Prints one JSON line (see the design notes for the field definitions).
"""
from __future__ import annotations

import argparse
import dataclasses
import gc
import json
import os
import sys
import time
from fractions import Fraction

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
FP64_MFMA_PEAK_TFLOPS = 78.6
# (d, L) of the combination-technique runs (Sec. 4.3 setting, L <= 17 - d)
CT_RUNS = [(2, 14), (4, 12), (6, 10)]
# relative residual that brings the headline solve's error against the exact
# solution below 1e-9 (error / residual is about 1.9 on that grid)
RTOL_ERROR_1E9 = 5e-10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--local", default="cholesky", choices=["cholesky", "inverse"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2, help="PCG iterations in the CPU oracle sample")
    ap.add_argument("--cpu-full", action="store_true",
                    help="run the CPU oracle's PCG to the tolerance instead of a sample of iterations")
    ap.add_argument("--cpu-only", action="store_true",
                    help="run only the CPU oracle leg (needs no GPU) and print its JSON")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--profile-workload", default="c2", choices=["c2", "c5"],
                    help="with --profile-only: the workload (c2: the headline grid; c5: the 8.26 M-unknown grid)")
    ap.add_argument("--profile-coarse", default="dense", choices=["dense", "iterative"],
                    help="with --profile-only: the coarse solver")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + steps of the headline path only (for rocprofv3)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="with --profile-only: also copy a buffer of this many MiB three times "
                         "(the reference kernel that scales the HBM byte counters)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 84-grid layer")
    ap.add_argument("--no-sweep", action="store_true", help="skip the overlap (gamma) sweep")
    ap.add_argument("--no-large", action="store_true", help="skip the large single grid (8.26 M unknowns)")
    ap.add_argument("--no-tune", action="store_true", help="use the default launch shapes (no autotuning)")
    return ap.parse_args()


def run_path(w, f_dev, fdtype, local, steps, warmup, ws_cache, prof_steps=0, curve="hilbert",
             coarse_precision="auto", rtol=None, max_iter=500, coarse_solver="dense", tune=None):
    """Times `steps` full setup+solve passes (after `warmup` untimed ones);
    then, when prof_steps > 0, that many more passes with the library's
    per-kernel HIP events on (they add about 3% to a solve, so the step times
    above are taken without them).  Returns a dict of measurements."""
    import torch
    import paper_2110_11211_amd as m
    kw = dict(levels=list(w.levels[0]), P=w.P, gamma=w.gamma, factor_dtype=fdtype, local_solver=local,
              curve=curve, coarse_precision=coarse_precision, coarse_solver=coarse_solver)
    rtol = w.rtol if rtol is None else rtol
    nbytes = m.workspace_size(**kw)
    key = (fdtype, local)
    if key not in ws_cache or ws_cache[key].numel() < nbytes + 256:
        ws_cache.clear()
        torch.cuda.empty_cache()
        ws_cache[key] = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:0")
    ws = ws_cache[key]
    method = "fcg" if fdtype == "fp32" else "pcg"
    times, setups, solves, iters = [], [], [], []
    x = None
    ktimes = None
    piters = []
    csteps = []
    tuning = None
    S = None
    for k in range(warmup + steps + prof_steps):
        timed = warmup <= k < warmup + steps
        prof = k >= warmup + steps
        if S is not None:
            S.close()
            S = None
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record()
        S = m.SFCSchwarz(device="cuda:0", workspace=ws, **kw)
        e1.record()
        if tune is not None and k == 0:
            # autotune the launch shapes on the first (untimed) pass; later
            # setups of this shape start from the recorded choice
            torch.cuda.synchronize()
            tuning = S.tune("all", tune)
            torch.cuda.synchronize()
            e0.record()
            e1.record()
        if prof:
            S.set_profiling(True)
        x, info = S.solve(f_dev, rtol=rtol, max_iter=max_iter, method=method)
        e2.record()
        torch.cuda.synchronize()
        if timed:
            times.append(e0.elapsed_time(e2))
            setups.append(e0.elapsed_time(e1))
            solves.append(e1.elapsed_time(e2))
            iters.append(info["iterations"])
        if timed:
            csteps.append(info["coarse_steps"])
        if prof:
            piters.append(info["iterations"] + info["restarts"])
            kt = {kk: S.kernel_time(kk) for kk in ("local_solve", "scatter", "spmv", "spmv_b", "coarse")}
            ktimes = kt if ktimes is None else {kk: (ktimes[kk][0] + kt[kk][0], ktimes[kk][1] + kt[kk][1])
                                               for kk in kt}
            S.set_profiling(False)
    sinfo = S.info()
    S.close()
    return {"ms": sorted(times)[len(times) // 2], "ms_min": min(times), "setup_ms": sorted(setups)[len(setups) // 2],
            "solve_ms": sorted(solves)[len(solves) // 2], "iterations": iters[-1], "info": sinfo,
            "kernels": ktimes, "prof_steps": prof_steps, "prof_full_launches": sum(piters), "x": x,
            "rel_residual": info["rel_residual"], "restarts": info["restarts"],
            "coarse_steps": max(csteps) if csteps else 0, "tuning": tuning}


def kernel_rates(res, w, local):
    """Average launch time and algorithmic GB/s of the substitution kernel and
    of the SpMV from a run with the library's per-kernel events on."""
    info = res["info"]
    d = len(w.levels[0])
    if local == "cholesky":
        local_bytes = 2 * info["factor_algo_bytes"] + 16 * info["sum_Ni"]   # two sweeps over the triangle
    else:
        local_bytes = info["factor_algo_bytes"] + 16 * info["sum_Ni"]       # one pass over the inverse
    ms_local, n_local = res["kernels"]["local_solve"]
    # launches that did work: one per iteration (the application enqueued
    # after the converging step skips every subdomain and its few
    # microseconds stay in the numerator)
    avg_local = ms_local / max(min(n_local, res["prof_full_launches"]), 1)
    # y = A x reads x and 2d int32 neighbour indices and writes y; y = b - A x
    # also reads b
    ms_ax, n_ax = res["kernels"]["spmv"]
    ms_bx, n_bx = res["kernels"]["spmv_b"]
    bytes_ax = (16 + 8 * d) * info["N"]
    bytes_bx = (24 + 8 * d) * info["N"]
    ms_spmv, n_spmv = ms_ax + ms_bx, n_ax + n_bx
    avg_spmv = ms_spmv / max(n_spmv, 1)
    spmv_bytes = (n_ax * bytes_ax + n_bx * bytes_bx) / max(n_spmv, 1)   # per launch, averaged
    rate = lambda b, ms, n: b / (ms / max(n, 1) * 1e-3) / 1e9 if n else None
    return {"local_bytes": local_bytes, "avg_local_ms": avg_local,
            "local_gbps": local_bytes / (avg_local * 1e-3) / 1e9,
            "spmv_bytes": spmv_bytes, "avg_spmv_ms": avg_spmv,
            "spmv_gbps": spmv_bytes / (avg_spmv * 1e-3) / 1e9,
            "spmv_modes": {"ax": {"launches": n_ax, "avg_ms": ms_ax / max(n_ax, 1), "bytes": bytes_ax,
                                  "gbps": rate(bytes_ax, ms_ax, n_ax)},
                           "b_minus_ax": {"launches": n_bx, "avg_ms": ms_bx / max(n_bx, 1), "bytes": bytes_bx,
                                          "gbps": rate(bytes_bx, ms_bx, n_bx)}}}


def dtype_label(info):
    """The arithmetic of a run, from the context's precision choices."""
    if info["coarse_inv_fp32"]:
        coarse = "f32 coarse factor and inverse" if info["coarse_fp32"] else \
            "f64 coarse factor rounded to f32, f32 coarse inverse"
    else:
        coarse = "f64 coarse factor and inverse"
    return (f"f32 subdomain factors and solves (MFMA, f32 accumulate), {coarse} (f64 coarse matrix "
            f"and sums), f64 outer flexible CG, dots and residuals")


def hbm_read_probe():
    """Streaming-read rate of this GPU (GB/s): the library's 16-byte-per-lane
    read kernel over 4 GiB, best of 5."""
    import torch
    import paper_2110_11211_amd as m
    a = torch.zeros(1 << 30, dtype=torch.float32, device="cuda:0")
    ms = m.read_probe(a, repeats=5)
    del a
    torch.cuda.empty_cache()
    return 4.0 * (1 << 30) / (ms * 1e-3) / 1e9


def source_digest(files=("trsv.hip",)):
    """Digest of the given kernel sources: a stored HBM byte count is only
    valid for the code it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2110_11211_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def factor_digest():
    """Digest of the sources of the batched factorisation (its stored counter
    summary is only valid for the code it was measured on)."""
    return source_digest(("factor.hip", "common.h"))


def _profile_fields(kernel_file):
    path = os.path.join(ROOT, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    return vals


def stored_mfma(kernel_file):
    """MFMA-busy fraction and rates from the committed counter summary, or None
    when it is missing or was taken on other factorisation sources."""
    vals = _profile_fields(kernel_file)
    if vals is None or vals.get("source_digest") != factor_digest():
        return None
    try:
        return {"mfma_busy": float(vals["mfma_busy"]), "executed_tflops": float(vals["executed_tflops"]),
                "useful_tflops": float(vals["useful_tflops"]),
                "lds_conflict_fraction": float(vals["lds_conflict_fraction"]), "source": kernel_file}
    except (KeyError, ValueError):
        return None


LARGE_TRAFFIC = "k_spmv_trsv_fp32_d3_l8x8x7_P4096_traffic.txt"


def stored_traffic(kernel_file, key="traffic_bytes_per_launch", digest_key="source_digest",
                   sources=("trsv.hip",)):
    """HBM bytes per launch from the committed counter summary, or None when
    the summary is missing or was taken on other kernel sources."""
    vals = _profile_fields(kernel_file)
    if vals is None or vals.get(digest_key) != source_digest(sources):
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def run_batch(w, fdtype, steps, warmup, sequential=False):
    """The 84-grid combination-technique layer: setup (+ substitution-kernel
    autotuning) + solve of every grid, either as one batched context or grid
    after grid.  Returns (median ms, max iterations, solutions, waves)."""
    import numpy as np
    import torch
    import paper_2110_11211_amd as m
    grids = [dict(levels=list(lv), P=w.P, gamma=w.gamma) for lv in w.levels]
    f = np.concatenate([w.rhs(g) for g in range(len(w.levels))])
    f_dev = torch.tensor(f, dtype=torch.float64, device="cuda:0")
    offs = np.concatenate([[0], np.cumsum([w.N(g) for g in range(len(w.levels))])])
    method = "fcg" if fdtype == "fp32" else "pcg"
    ws = None
    times, iters, x, waves = [], 0, None, None
    for k in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        if not sequential:
            S = m.SFCSchwarzBatch(grids, factor_dtype=fdtype, workspace=ws)
            ws = S.ws
            tuning = S.tune("all", 2)
            x, _ = S.solve(f_dev, rtol=w.rtol, method=method, max_iter=500)
            its, _ = S.batch_stats()
            waves = tuning
            S.close()
            iters = max(its)
        else:
            x = torch.empty_like(f_dev)
            iters = 0
            for g, gk in enumerate(grids):
                Sg = m.SFCSchwarz(levels=gk["levels"], P=gk["P"], gamma=gk["gamma"], factor_dtype=fdtype)
                xg, ig = Sg.solve(f_dev[offs[g]:offs[g + 1]], rtol=w.rtol, method=method, max_iter=500)
                x[offs[g]:offs[g + 1]].copy_(xg)
                iters = max(iters, ig["iterations"])
                Sg.close()
        t1.record()
        torch.cuda.synchronize()
        if k >= warmup:
            times.append(t0.elapsed_time(t1))
    return sorted(times)[len(times) // 2], iters, x.cpu().numpy(), waves, offs


def ct_batch_report(steps, warmup):
    """The 84-grid layer batched (FP32 and FP64 factors) and grid after grid.
    Returns the report and the solutions, which the oracle leg checks."""
    from seeded_inputs import workloads
    w = workloads()["c4"]
    b32, it32, x32, waves, offs = run_batch(w, "fp32", steps, warmup)
    b64, it64, x64, _, _ = run_batch(w, "fp64", steps, warmup)
    s32, _, _, _, _ = run_batch(w, "fp32", 1, 1, sequential=True)
    rep = {"workload": w.name, "grids": len(w.levels), "N_total": int(offs[-1]),
           "batched_fp32_ms": round(b32, 3), "batched_fp64_ms": round(b64, 3),
           "sequential_fp32_ms": round(s32, 3),
           "speedup_batched_vs_sequential": round(s32 / b32, 3),
           "speedup_fp32_vs_fp64": round(b64 / b32, 3),
           "max_iterations_fp32": it32, "max_iterations_fp64": it64, "tuning_fp32": waves,
           "max_rel_error_vs_exact_fp32": None, "max_rel_error_vs_exact_fp64": None,
           "note": "setup + autotune + solve of all 84 grids to 1e-9 per step (the tuner times the launch "
                   "shapes on the warm-up pass; later setups of the same shapes start from its choice and "
                   "the call returns at once)"}
    return rep, {"w": w, "offs": offs, "x32": x32, "x64": x64}


def ct_solve_report(d, L, steps, warmup, npts=20000):
    """The combination-technique experiment of Sec. 4.3 on one GPU: every grid
    of the level-L combination in d dimensions (Phat = 2^(L-8), so about 2^8
    points per subdomain; gamma = 1/4; FP32 factors; flexible CG to a relative
    residual of 1e-8) set up and solved as one batch, then the combined
    solution evaluated at npts seeded uniform points.  One step = setup +
    solve + combination; the error is the maximum absolute error against the
    manufactured solution at the points."""
    from fractions import Fraction
    import numpy as np
    import torch
    import paper_2110_11211_amd as m
    from seeded_inputs import manufactured, uniform01
    phat = 1 << max(0, L - 8)
    CT = m.CombinationTechnique(d, L, phat=phat, gamma=Fraction(1, 4), factor_dtype="fp32")
    f = np.concatenate([manufactured(CT.grid_points(g))[1] for g in range(CT.ngrids)])
    f_dev = torch.tensor(f, dtype=torch.float64, device="cuda:0")
    X = uniform01(8000 + 10 * d + L, npts * d).reshape(npts, d)
    x_dev = torch.tensor(X, dtype=torch.float64, device="cuda:0")
    ws = CT.batch.ws
    subdomains = sum(CT.batch._arr[g].P for g in range(CT.ngrids))
    CT.close()
    times, tcomb, iters = [], [], 0
    for k in range(warmup + steps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record()
        CT = m.CombinationTechnique(d, L, phat=phat, gamma=Fraction(1, 4), factor_dtype="fp32", workspace=ws)
        u, _ = CT.solve(f_dev, rtol=1e-8, max_iter=500)
        e1.record()
        val = CT.evaluate(u, x_dev)
        e2.record()
        torch.cuda.synchronize()
        its, _ = CT.batch.batch_stats()
        iters = max(its)
        CT.close()
        if k >= warmup:
            times.append(e0.elapsed_time(e2))
            tcomb.append(e1.elapsed_time(e2))
    err = float(np.abs(val.cpu().numpy() - manufactured(X)[0]).max())
    return {"d": d, "L": L, "phat": phat, "grids": CT.ngrids, "subdomains": subdomains,
            "N_total": int(f.size), "ms": round(sorted(times)[len(times) // 2], 3),
            "combine_ms": round(sorted(tcomb)[len(tcomb) // 2], 3),
            "max_iterations": iters, "max_abs_error_vs_manufactured": err, "points": npts}


def adjoint_report(steps, warmup):
    """The d=6 anisotropic workload as a differentiable solve: forward solve,
    J = 1/2 ||u||^2, adjoint backward (second solve with the same factors and
    the coefficient-gradient kernel), FP32 factors, rtol of the workload."""
    import torch
    import paper_2110_11211_amd as m
    from seeded_inputs import workloads
    w = workloads()["c3"]
    f0 = w.rhs()
    times = []
    for k in range(warmup + steps):
        f = torch.tensor(f0, dtype=torch.float64, device="cuda:0").requires_grad_(True)
        a = torch.tensor(w.coeff, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        u = m.solve_poisson(f, a, w.levels[0], P=w.P, gamma=w.gamma, factor_dtype="fp32", rtol=w.rtol)
        J = 0.5 * (u * u).sum()
        J.backward()
        e1.record()
        torch.cuda.synchronize()
        if k >= warmup:
            times.append(e0.elapsed_time(e1))
    rep = {"workload": w.name, "N": w.N(), "P": w.P, "ms": round(sorted(times)[len(times) // 2], 3),
           "rel_error_grad_f": None, "max_rel_error_grad_a": None,
           "note": "setup + forward solve + adjoint solve + coefficient gradient, FP32 factors, rtol 1e-9"}
    return rep, {"w": w, "f0": f0, "gf": f.grad.detach().cpu().numpy(), "ga": a.grad.detach().numpy()}


def cpu_model():
    """CPU model name of this host (first /proc/cpuinfo entry), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, gpu_iterations, sample_iters, full=False):
    """The oracle as it stands (plain FP64 NumPy/SciPy, untuned) on the headline
    workload, in two legs: BLAS/LAPACK on every thread the library uses here,
    and on one thread (threadpoolctl).  Each leg times the oracle's whole setup
    (curve order, partition, A and A_0, all P local Cholesky factorisations and
    the coarse one) and its balanced PCG from the balancing start.  By default
    the PCG runs `sample_iters` iterations (the bounded sample) and the leg's
    value is setup + start + gpu_iterations x the measured time per iteration;
    with full=True it runs to the workload's tolerance and the value is the
    measured total."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.grid import Grid
    from oracle.schwarz import OracleSchwarz
    from oracle import solvers
    g = Grid(levels=w.levels[0])
    f = w.rhs()
    legs = {}
    for name, limit in (("all_threads", None), ("one_thread", 1)):
        with threadpool_limits(limits=limit):
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
            t = time.perf_counter()
            O = OracleSchwarz(g, w.P, w.gamma, curve="hilbert")
            t_setup = time.perf_counter() - t
            print(f"bench: CPU oracle {name}: setup {t_setup:.1f} s", file=sys.stderr, flush=True)
            t = time.perf_counter()
            x0 = O.balancing_start(f)
            t_start = time.perf_counter() - t
            t = time.perf_counter()
            x, its, pinfo = solvers.pcg(O.A_nat, f, O.apply, x0=x0, rtol=w.rtol,
                                        maxit=1000 if full else sample_iters)
            t_iter = time.perf_counter() - t
        per_iter = t_iter / max(its, 1)
        converged = not pinfo.get("not_converged", False)
        if full:
            total = t_setup + t_start + t_iter
        else:
            total = t_setup + t_start + gpu_iterations * per_iter
        legs[name] = {"value": round(1e3 * total, 1), "unit": "ms", "threads": int(threads),
                      "setup_s": round(t_setup, 3), "start_s": round(t_start, 4),
                      "per_iteration_s": round(per_iter, 4), "iterations_run": int(its),
                      "converged": bool(converged and full),
                      "rel_residual": float(np.linalg.norm(f - O.A_nat @ x) / np.linalg.norm(f)) if full else None}
        del O
    allt = legs["all_threads"]
    if full:
        sample = (f"full run: the oracle's setup and its balanced PCG to rtol {w.rtol:g} "
                  f"({allt['iterations_run']} iterations; GPU {gpu_iterations})")
    else:
        sample = (f"the oracle's full setup (all {w.P} local factorisations, coarse matrix and factor) timed "
                  f"in full, then {sample_iters} iterations of its balanced PCG timed and scaled to the "
                  f"GPU's {gpu_iterations} iterations")
    return {"value": allt["value"], "unit": "ms", "cores": allt["threads"], "kind": "oracle",
            "sample": sample, "os_cpu_count": os.cpu_count(), "cpu_model": cpu_model(), "legs": legs}


def oracle_checks(w, x_head, ct_raw, adj_raw, extra=None, big=None):
    """Part of the CPU-baseline leg: errors of the GPU results against the
    oracle's exact DST-I solutions and adjoint gradients."""
    import numpy as np
    from oracle.grid import Grid
    from oracle import exact, grad as ograd
    out = {}
    xs = exact.solve(Grid(levels=w.levels[0]), w.rhs())
    out["headline_rel_error_vs_exact"] = float(np.linalg.norm(x_head - xs) / np.linalg.norm(xs))
    for k, xv in (extra or {}).items():
        out[k + "_rel_error_vs_exact"] = float(np.linalg.norm(xv - xs) / np.linalg.norm(xs))
    if big is not None:
        wl, xl, xli = big
        xe = exact.solve(Grid(levels=wl.levels[0]), wl.rhs())
        out["large_grid_rel_error_vs_exact"] = float(np.linalg.norm(xl - xe) / np.linalg.norm(xe))
        out["large_grid_iterative_rel_error_vs_exact"] = float(np.linalg.norm(xli - xe) / np.linalg.norm(xe))
    if ct_raw is not None:
        wc, offs = ct_raw["w"], ct_raw["offs"]
        e32 = e64 = 0.0
        for g in range(len(wc.levels)):
            ref = exact.solve(Grid(levels=wc.levels[g]), wc.rhs(g))
            nr = np.linalg.norm(ref)
            e32 = max(e32, float(np.linalg.norm(ct_raw["x32"][offs[g]:offs[g + 1]] - ref) / nr))
            e64 = max(e64, float(np.linalg.norm(ct_raw["x64"][offs[g]:offs[g + 1]] - ref) / nr))
        out["ct_batch_max_rel_error_fp32"] = e32
        out["ct_batch_max_rel_error_fp64"] = e64
    if adj_raw is not None:
        wa = adj_raw["w"]
        g = Grid(levels=wa.levels[0], coeff=wa.coeff)
        u_ref = exact.solve(g, adj_raw["f0"])
        gf_ref, ga_ref = ograd.adjoint_gradient(g, u_ref, u_ref)
        out["adjoint_rel_error_grad_f"] = float(np.linalg.norm(adj_raw["gf"] - gf_ref) / np.linalg.norm(gf_ref))
        out["adjoint_max_rel_error_grad_a"] = float(np.max(np.abs(adj_raw["ga"] - ga_ref) / np.abs(ga_ref)))
    return out


def progress(what):
    """Progress line after a section; also collects cyclic garbage there,
    between the timed regions (automatic collection is paused)."""
    print(f"bench: {what} done", file=sys.stderr, flush=True)
    gc.collect()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} was asked for): the solver has no "
              f"multi-GPU path; its sharding across GPUs is described, not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.cpu_only:
        from seeded_inputs import workloads
        w = workloads()["c2"]
        print(json.dumps({"cpu_baseline": cpu_baseline(w, 30, args.cpu_sample, full=args.cpu_full)}), flush=True)
        return
    import numpy as np
    import torch
    import paper_2110_11211_amd as m
    from seeded_inputs import workloads
    m.lib()
    # Python's cyclic garbage collector is paused while the GPU paths are
    # timed: a full collection (tens of milliseconds with torch loaded) would
    # otherwise land inside some steps.  Reference counting still frees
    # everything the steps drop; the collector runs again for the CPU leg.
    gc.collect()
    gc.freeze()
    gc.disable()
    w = workloads()["c5" if args.profile_only and args.profile_workload == "c5" else "c2"]
    f_dev = torch.tensor(w.rhs(), dtype=torch.float64, device="cuda:0")
    ws_cache = {}
    head = run_path(w, f_dev, "fp32", args.local, args.steps, max(1, args.warmup), ws_cache, prof_steps=args.steps,
                    coarse_solver=args.profile_coarse if args.profile_only else "dense",
                    tune=None if args.no_tune else 3)
    psteps = head["prof_steps"]
    progress("headline")
    if args.profile_only:
        ms_l, n_l = head["kernels"]["local_solve"]
        n_full = head["prof_full_launches"]
        kr = kernel_rates(head, w, args.local)
        out = {"profile_only": True, "workload": w.name, "ms": head["ms"], "local_solve_launches": n_l,
               "local_solve_full_launches": min(n_l, n_full),
               "local_solve_avg_ms": ms_l / max(min(n_l, n_full), 1),
               "local_solve_gbps": kr["local_gbps"],
               "spmv_launches": head["kernels"]["spmv"][1] + head["kernels"]["spmv_b"][1],
               "spmv_avg_ms": kr["avg_spmv_ms"], "spmv_gbps": kr["spmv_gbps"],
               "spmv_algorithmic_bytes": kr["spmv_bytes"], "iterations": head["iterations"],
               "coarse_ms": head["kernels"]["coarse"][0] / max(psteps, 1), "coarse_steps": head["coarse_steps"],
               "setup_ms": head["setup_ms"], "solve_ms": head["solve_ms"], "q": head["info"]["q"]}
        if args.copy_probe > 0:
            ws_cache.clear()
            n = args.copy_probe * (1 << 20) // 4
            a = torch.ones(n, dtype=torch.float32, device="cuda:0")
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            torch.cuda.synchronize()
            out["copy_probe_bytes_read"] = 4 * n
            out["copy_probe_bytes_written"] = 4 * n
        print(json.dumps(out), flush=True)
        return
    zo = run_path(w, f_dev, "fp32", args.local, max(2, args.steps // 2), args.warmup, ws_cache, curve="zorder")
    progress("Z-order path")
    # the overlap axis of Sec. 4.1 on the same grid: gamma = 1/4, 1 and 3/2
    # beside the headline's 1/2 (more overlap: fewer iterations, larger
    # subdomain factors)
    sweep = []
    if not args.no_sweep:
        for gam in (Fraction(1, 4), Fraction(1), Fraction(3, 2)):
            r = run_path(dataclasses.replace(w, gamma=gam), f_dev, "fp32", args.local, max(2, args.steps // 2),
                         args.warmup, ws_cache)
            sweep.append((gam, r))
        progress("overlap sweep")
    f64 = None
    if not args.skip_fp64:
        f64 = run_path(w, f_dev, "fp64", args.local, max(2, args.steps // 2), args.warmup, ws_cache, prof_steps=1)
        progress("FP64 path")
    # FP32 subdomain factors beside an all-FP64 coarse operator
    c64 = run_path(w, f_dev, "fp32", args.local, max(2, args.steps // 2), args.warmup, ws_cache,
                   coarse_precision="fp64")
    progress("FP64-coarse path")
    # the headline run to an error of 1e-9 against the exact solution rather
    # than a residual of 1e-9 (on this grid the error is about twice the
    # relative residual)
    e9 = run_path(w, f_dev, "fp32", args.local, max(2, args.steps // 2), args.warmup, ws_cache,
                  rtol=RTOL_ERROR_1E9)
    progress("error-1e-9 path")
    ws_cache.clear()
    # the large single grid: 8.26 M unknowns, 4096 subdomains of ~2521 points
    big = None
    if not args.no_large:
        wl = workloads()["c5"]
        fl_dev = torch.tensor(wl.rhs(), dtype=torch.float64, device="cuda:0")
        big = run_path(wl, fl_dev, "fp32", args.local, 2, 1, ws_cache, prof_steps=1,
                       tune=None if args.no_tune else 2)
        big["x"] = big["x"].cpu().numpy()
        ws_cache.clear()
        torch.cuda.empty_cache()
        # the same grid at the paper's q = 64 (N0 = 262,144) with the iterative coarse solve
        bigi = run_path(wl, fl_dev, "fp32", args.local, 2, 1, ws_cache, prof_steps=1, coarse_solver="iterative",
                        tune=None if args.no_tune else 2)
        bigi["x"] = bigi["x"].cpu().numpy()
        del fl_dev
        ws_cache.clear()
        torch.cuda.empty_cache()
        progress("large grid")

    xh = head["x"].cpu().numpy()

    info = head["info"]
    sumN = info["sum_Ni"]
    N = info["N"]
    kr = kernel_rates(head, w, args.local)
    local_bytes, avg_local, gbs_local = kr["local_bytes"], kr["avg_local_ms"], kr["local_gbps"]
    avg_spmv, gbs_spmv = kr["avg_spmv_ms"], kr["spmv_gbps"]
    ms_local = head["kernels"]["local_solve"][0]
    # the dominant kernel class over a whole step
    solve_local_ms = ms_local / psteps
    factor_ms = info["setup_ms"][3]
    nt = [(n + 63) // 64 for n in [info["max_Ni"]]]
    read_peak = hbm_read_probe()
    traffic = stored_traffic("k_schwarz_trsv_fp32_d3_l7x6x5_P256_traffic.txt") \
        if args.local == "cholesky" else None
    roofline = {"kernel": "k_schwarz_trsv (FP32 factors)" if args.local == "cholesky" else "k_symv_tiles (FP32 inverse)",
                "bound": "hbm", "achieved": round(gbs_local, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs_local / HBM_PEAK_GBS, 4), "traffic": traffic,
                "avg_launch_ms": avg_local, "algorithmic_bytes_per_launch": local_bytes,
                "measured_read_GBps": round(read_peak, 1), "frac_of_measured_read": round(gbs_local / read_peak, 4),
                "local_solve_ms_per_step": solve_local_ms, "factor_ms_per_step": factor_ms}
    out = {
        "metric": "time-to-1e-9 solve & GB/s of SpMV+Schwarz: FP32-precond vs FP64, 1 GPU",
        "value": round(head["ms"], 3), "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype_label(info), "data": "synthetic",
        "config": {"workload": w.name, "levels": list(w.levels[0]), "N": N, "P": w.P, "curve": "hilbert",
                   "gamma": str(w.gamma), "q": info["q"], "N0": info["N0"], "rtol": w.rtol,
                   "variant": "balanced", "weighting": "omega", "local_solver": args.local,
                   "outer": "flexible CG (fp32) / PCG (fp64)"},
        "headline": {"setup_ms": round(head["setup_ms"], 3), "solve_ms": round(head["solve_ms"], 3),
                     "ms_min": round(head["ms_min"], 3), "iterations": head["iterations"],
                     "restarts": head["restarts"], "rel_residual": head["rel_residual"],
                     "rel_error_vs_exact": None, "setup_phases_ms": info["setup_ms"]},
        "gbps": {"schwarz_local_solve": round(gbs_local, 1), "spmv": round(gbs_spmv, 1),
                 "local_solve_avg_ms": avg_local, "spmv_avg_ms": avg_spmv,
                 "spmv_note": "the SpMV's 9.9 MB working set stays in the caches at this size and a launch "
                              "lasts a few microseconds (latency-bound); its HBM roofline is measured on the "
                              "large grid (large_grid.roofline_spmv)"},
        "kernel_ms_per_step": {k: round(v[0] / psteps, 3) for k, v in head["kernels"].items()},
        "kernel_launches_per_step": {k: v[1] // psteps for k, v in head["kernels"].items()},
        "roofline": roofline,
        "tuning": head["tuning"],
    }
    if f64 is not None:
        i64 = f64["info"]
        ms64, n64 = f64["kernels"]["local_solve"]
        b64 = (2 * i64["factor_algo_bytes"] if args.local == "cholesky" else i64["factor_algo_bytes"]) + 16 * sumN
        out["fp64"] = {"ms": round(f64["ms"], 3), "setup_ms": round(f64["setup_ms"], 3),
                       "solve_ms": round(f64["solve_ms"], 3), "iterations": f64["iterations"],
                       "local_solve_gbps": round(b64 / (ms64 / max(n64, 1) * 1e-3) / 1e9, 1),
                       "setup_phases_ms": i64["setup_ms"]}
        out["speedup_fp32_vs_fp64"] = round(f64["ms"] / head["ms"], 3)
    out["fp64_coarse"] = {"ms": round(c64["ms"], 3), "setup_ms": round(c64["setup_ms"], 3),
                          "solve_ms": round(c64["solve_ms"], 3), "iterations": c64["iterations"],
                          "dtype": dtype_label(c64["info"]), "rel_error_vs_exact": None,
                          "note": "headline workload with the coarse factor, inverse and solves in FP64"}
    out["to_error_1e-9"] = {"ms": round(e9["ms"], 3), "setup_ms": round(e9["setup_ms"], 3),
                            "solve_ms": round(e9["solve_ms"], 3), "iterations": e9["iterations"],
                            "rtol": RTOL_ERROR_1E9, "rel_residual": e9["rel_residual"], "rel_error_vs_exact": None,
                            "note": "headline run to a relative residual of 5e-10, which brings the error "
                                    "against the exact solution below 1e-9"}
    if big is not None:
        bi = big["info"]
        krl = kernel_rates(big, wl, args.local)
        out["large_grid"] = {
            "workload": wl.name, "levels": list(wl.levels[0]), "N": bi["N"], "P": wl.P, "gamma": str(wl.gamma),
            "q": bi["q"], "N0": bi["N0"], "curve": "hilbert", "dtype": dtype_label(bi),
            "ms": round(big["ms"], 3), "setup_ms": round(big["setup_ms"], 3), "solve_ms": round(big["solve_ms"], 3),
            "iterations": big["iterations"], "rel_residual": big["rel_residual"], "rel_error_vs_exact": None,
            "factor_bytes": bi["factor_algo_bytes"], "tuning": big["tuning"],
            "kernel_ms_per_step": {k: round(v[0], 3) for k, v in big["kernels"].items()},
            "roofline_spmv": {"kernel": "k_spmv", "bound": "hbm", "achieved": round(krl["spmv_gbps"], 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(krl["spmv_gbps"] / HBM_PEAK_GBS, 4), "target_frac": 0.6,
                              "avg_launch_ms": krl["avg_spmv_ms"], "algorithmic_bytes_per_launch": krl["spmv_bytes"],
                              "modes": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                                        for k, v in krl["spmv_modes"].items()},
                              "note": "both forms of the solve's SpMV, y = A x with the x . y partials and "
                                      "y = b - A x (which also reads b), launch-weighted; traffic: the "
                                      "counters of y = A x",
                              "traffic": stored_traffic(LARGE_TRAFFIC, sources=("apply.hip",))},
            "roofline_local_solve": {"kernel": "k_schwarz_trsv (FP32 factors)", "bound": "hbm",
                                     "achieved": round(krl["local_gbps"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": round(krl["local_gbps"] / HBM_PEAK_GBS, 4), "target_frac": 0.6,
                                     "avg_launch_ms": krl["avg_local_ms"],
                                     "algorithmic_bytes_per_launch": krl["local_bytes"],
                                     "traffic": stored_traffic(LARGE_TRAFFIC, key="trsv_traffic_bytes_per_launch",
                                                               digest_key="trsv_source_digest")},
            "note": "q = 4 under the dense coarse-size cap N0 <= 16384 (the four-levels-coarser rule gives 64)"}
        ii = bigi["info"]
        out["large_grid"]["iterative_coarse"] = {
            "q": ii["q"], "N0": ii["N0"], "N0d": ii["N0d"], "ell_width": ii["ell_width"],
            "ms": round(bigi["ms"], 3), "setup_ms": round(bigi["setup_ms"], 3),
            "solve_ms": round(bigi["solve_ms"], 3), "iterations": bigi["iterations"],
            "inner_steps_max": bigi["coarse_steps"], "inner_budget": ii["coarse_steps"],
            "rel_residual": bigi["rel_residual"], "rel_error_vs_exact": None,
            "kernel_ms_per_step": {k: round(v[0], 3) for k, v in bigi["kernels"].items()},
            "tuning": bigi["tuning"],
            "note": "q by the four-levels-coarser rule (64); A_0 kept sparse and solved by an inner FP64 CG "
                    "to a relative residual of 1e-6 at every coarse solve"}
    if sweep:
        rows = sorted([(w.gamma, head)] + sweep, key=lambda t: t[0])
        out["overlap_sweep"] = [{"gamma": str(gm), "ms": round(r["ms"], 3), "setup_ms": round(r["setup_ms"], 3),
                                 "solve_ms": round(r["solve_ms"], 3), "iterations": r["iterations"],
                                 "max_Ni": r["info"]["max_Ni"], "factor_bytes": r["info"]["factor_algo_bytes"]}
                                for gm, r in rows]
    out["zorder"] = {"ms": round(zo["ms"], 3), "setup_ms": round(zo["setup_ms"], 3),
                     "solve_ms": round(zo["solve_ms"], 3), "iterations": zo["iterations"],
                     "iterations_hilbert": head["iterations"],
                     "note": "same workload with the Z-order (Morton) curve instead of the Hilbert curve"}
    # MFMA rate of the batched subdomain factorisation over the tile envelopes
    # (the library's count: 2 TS^3 per tile product, 2 TS^3 / 3 per diagonal tile)
    fflops = float(head["info"]["factor_flops"])
    out["factor"] = {"flops": fflops, "ms": round(factor_ms, 3),
                     "tflops": round(fflops / (factor_ms * 1e-3) / 1e12, 2), "peak_tflops": FP32_MFMA_PEAK_TFLOPS,
                     "frac": round(fflops / (factor_ms * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS, 4),
                     "note": "FP32 MFMA over the tile envelopes; one chain of dependent diagonal tiles per "
                             "subdomain, concurrent with the coarse setup",
                     "counters": stored_mfma("k_potrf_full_fp32_d3_l7x6x5_P256_mfma.txt")}
    ct_raw = adj_raw = None
    if not args.no_batch:
        out["ct_batch"], ct_raw = ct_batch_report(max(2, args.steps // 2), 1)
        progress("84-grid layer")
        out["adjoint"], adj_raw = adjoint_report(max(2, args.steps // 2), 1)
        progress("adjoint")
        out["combination"] = []
        for d, L in CT_RUNS:
            out["combination"].append(ct_solve_report(d, L, max(2, args.steps // 2), 1))
            progress(f"combination d={d} L={L}")
    gc.enable()
    if not args.no_cpu_baseline:
        # the oracle leg: CPU timing of the oracle, then the accuracy checks
        iters = f64["iterations"] if f64 is not None else head["iterations"]
        out["cpu_baseline"] = cpu_baseline(w, iters, args.cpu_sample, full=args.cpu_full)
        progress("CPU oracle baseline")
        chk = oracle_checks(w, xh, ct_raw, adj_raw,
                            extra={"fp64_coarse": c64["x"].cpu().numpy(), "to_error_1e-9": e9["x"].cpu().numpy()},
                            big=(wl, big["x"], bigi["x"]) if big is not None else None)
        for k in ("fp64_coarse", "to_error_1e-9"):
            out[k]["rel_error_vs_exact"] = chk[k + "_rel_error_vs_exact"]
        if big is not None:
            out["large_grid"]["rel_error_vs_exact"] = chk["large_grid_rel_error_vs_exact"]
            out["large_grid"]["iterative_coarse"]["rel_error_vs_exact"] = chk["large_grid_iterative_rel_error_vs_exact"]
        out["cpu_baseline"]["accuracy_vs_oracle"] = chk
        out["headline"]["rel_error_vs_exact"] = chk["headline_rel_error_vs_exact"]
        if ct_raw is not None:
            out["ct_batch"]["max_rel_error_vs_exact_fp32"] = chk["ct_batch_max_rel_error_fp32"]
            out["ct_batch"]["max_rel_error_vs_exact_fp64"] = chk["ct_batch_max_rel_error_fp64"]
        if adj_raw is not None:
            out["adjoint"]["rel_error_grad_f"] = chk["adjoint_rel_error_grad_f"]
            out["adjoint"]["max_rel_error_grad_a"] = chk["adjoint_max_rel_error_grad_a"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
