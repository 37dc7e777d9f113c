#!/usr/bin/env python3
"""Pressure-projection benchmark on one MI355X.

Workload: the 256^3 layer-plus-droplets density field (periodic in x and y,
walls in z; liquid rho=1000 below a sinusoidal surface, gas rho=1.2 above with
200 liquid droplets, seed 2), u* uniform[-1, 1], dt = 1e-3, solved to a
relative residual of 1e-8.

One step = one complete projection for a new density field, every row of the
hot path on the GPU, inputs resident in HBM:
    face coefficients beta = 1/rho_f from rho and the
    hierarchy rebuild (coarse beta, FP32 copies, A^+)  (pp_update_density)
    b = D u* / dt                                     (pp_divergence)
    A p = b - mean(b) to 1e-8                          (pp_solve)
    u = u* - dt beta G p                               (pp_project)
The adjoint solve (pp_solve_adjoint, the backward pass) is timed in a loop of
its own and reported beside the forward figure.

Prints one JSON line: the headline `value` is mixed-precision (FP32 V-cycle,
FP64 outer) solves/s; FP64 and FP16-storage runs of the same steps are
reported under "modes", each with its max relative error of p, div(u) and u
against the FP64 CPU oracle's solution of the same system (solved to 1e-13),
computed after the timed region.  The same line carries, under "configs",
the 128^3 bubbles at density ratio 1000 (walls; FP64 and mixed FP32:
solves/s, iterations, errors against the oracle) and the 512^3 jet (walls;
mixed FP32 forward and backward: ms, iterations, device memory).  The CPU
baseline is the oracle's full projection step (face coefficients,
divergence, MG-PCG to the same tolerance, projection) on the same 256^3
system, median of 3 runs on all host threads, plus one run on one thread at
128^3.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="cells per direction (default 256)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--modes", default="fp32,fp64,fp16",
                    help="comma list; the first is the headline mode")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the error metrics against the oracle")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 128^3 bubbles and 512^3 jet blocks")
    ap.add_argument("--quick", action="store_true",
                    help="timed steps only (no CPU baseline, errors, configs or adjoint): "
                         "for profiling runs")
    ap.add_argument("--cpu-repeats", type=int, default=3,
                    help="oracle projection steps timed on all threads (median reported)")
    ap.add_argument("--cpu-1thread-n", type=int, default=128,
                    help="grid of the one-thread oracle run (same geometry; 0 = skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="time the plain copy kernel on 2 x 1 GiB buffers and exit (reference "
                         "for achievable HBM bandwidth and for scaling FETCH/WRITE counters)")
    ap.add_argument("--workload", default="layer256", choices=["layer256", "jet512"],
                    help="layer256: the headline metric; jet512: forward + backward projection "
                         "at 512^3 (time and memory per solve), printed as its own JSON line")
    ap.add_argument("--summarize-db", metavar="RESULTS_DB",
                    help="print a per-kernel, per-grid summary of a rocprofv3 kernel trace "
                         "(the *_results.db it writes) and exit")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def summarize_db(path):
    """Per-kernel and per-launch-grid duration table of a rocprofv3 trace."""
    import sqlite3
    con = sqlite3.connect(path)
    rows = con.execute(
        "select name, grid_x, grid_y, grid_z, count(*), sum(duration), avg(duration), "
        "min(duration), max(duration) from kernels group by name, grid_x, grid_y, grid_z "
        "order by sum(duration) desc").fetchall()
    total = sum(r[5] for r in rows)
    print(f"total kernel time {total / 1e6:.3f} ms over {sum(r[4] for r in rows)} dispatches\n")
    print("| kernel | grid (threads) | calls | total ms | avg us | min us | max us | % |")
    print("|---|---|---|---|---|---|---|---|")
    for name, gx, gy, gz, n, tot, avg, mn, mx in rows:
        short = name.split("(")[0].replace("void ", "")
        print(f"| {short} | {gx}x{gy}x{gz} | {n} | {tot / 1e6:.3f} | {avg / 1e3:.2f} | "
              f"{mn / 1e3:.2f} | {mx / 1e3:.2f} | {100 * tot / total:.1f} |")


COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "fused2_rbgs_layer256.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2012_11744_amd", "csrc", "pp_fused.hip")


def counter_traffic():
    """HBM bytes per launch of the roofline kernel from the committed counter
    summary (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, scaled by the copy-kernel
    calibration), or None when the kernel source changed since then."""
    import hashlib
    import re
    try:
        text = open(COUNTER_SUMMARY).read()
        src = open(KERNEL_SOURCE, "rb").read()
    except OSError:
        return None, "no counter summary"
    m = re.search(r"kernel_source_sha256_16: (\w+)", text)
    t = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not m or not t:
        return None, "no counter summary"
    if m.group(1) != hashlib.sha256(src).hexdigest()[:16]:
        return None, "kernel source changed since the counters were taken"
    return int(t.group(1)), os.path.relpath(COUNTER_SUMMARY, ROOT)


def copy_bandwidth(reps=10, nbytes=1 << 30):
    """Plain device copy through the library's copy kernel: GB/s counting the
    bytes read plus the bytes written."""
    import torch
    from paper_2012_11744_amd import solver as S
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    S.k_copy(src, dst)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        S.k_copy(src, dst)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del src, dst
    return {"bytes_per_launch": 2 * n * 8, "avg_ms": ms, "GBps": 2 * n * 8 / (ms * 1e-3) / 1e9}


def main():
    args = parse()
    if args.summarize_db:
        summarize_db(args.summarize_db)
        return
    if args.calibrate_copy:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"copy_kernel": copy_bandwidth()}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "a single solve is one globally coupled system and is not sharded here.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2012_11744_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.quick:
        args.no_cpu_baseline = args.no_adjoint = args.no_errors = args.no_configs = True
    if args.workload == "jet512":
        print(json.dumps(bench_jet512(args)), flush=True)
        return
    N = args.n
    t0 = time.time()
    w = W.config3(N)
    log(f"[bench] workload {w.name} {N}^3 generated in {time.time() - t0:.1f}s")
    modes = args.modes.split(",")
    results, roof, fields = run_modes(w, modes, args, keep=not args.no_errors)

    copy = copy_bandwidth()
    log(f"[bench] copy kernel: {copy['GBps']:.0f} GB/s")
    if roof is not None:
        roof["copy_kernel_GBps"] = round(copy["GBps"], 1)
        roof["frac_of_copy"] = round(roof["achieved"] / copy["GBps"], 4)

    configs = {}
    if not args.no_configs:
        configs["bubbles128"] = bench_bubbles128(args)
        configs["jet512"] = bench_jet512(args)

    # host-side work from here on: nothing below is timed on the GPU
    cpu, ref = None, None
    if not args.no_cpu_baseline:
        cpu, ref = cpu_baseline(w, args)
    if not args.no_errors:
        errs = oracle_errors(w, fields, ref, args.tol)
        for m, e in errs.items():
            results[m].update(e)
        del fields

    head = results[modes[0]]
    line = {
        "metric": "Poisson solves/s at 256^3 to 1e-8 rel residual, mixed vs FP64; achieved HBM GB/s",
        "value": round(head["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16": "f16"}[modes[0]] + "+f64",
        "data": "synthetic",
        "config": {"workload": f"layer+200 droplets, rho 1000/1.2, {N}^3, periodic x,y walls z, "
                               f"tol {args.tol:g}", "cells": w.cells, "parallelism": "single GPU"},
        "dof_per_s": round(head["dof_per_s"], 1),
        "modes": {m: {k: _fmt(v) for k, v in r.items() if k != "kernels"}
                  for m, r in results.items()},
        "kernels": {m: r["kernels"] for m, r in results.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if "fp64" in results and modes[0] != "fp64":
        line["mixed_over_fp64"] = round(head["solves_per_s"] / results["fp64"]["solves_per_s"], 3)
    if configs:
        line["configs"] = configs
    print(json.dumps(line), flush=True)


def _fmt(v):
    if isinstance(v, float):
        return float(f"{v:.6g}")
    if isinstance(v, dict):
        return {k: _fmt(x) for k, x in v.items()}
    return v


def _dev(a):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _step_fn(sol, rho, us, b, p, u, w, tol):
    """One projection step for the density field rho in one call (pp_step):
    coefficients and hierarchy, right-hand side, solve, projection."""
    def step():
        sol.step(rho, us, w.dt, tol=tol, p=p, rhs=b, out=u)
    return step


def run_modes(w, modes, args, keep):
    """Times `steps` projection steps per V-cycle precision on the workload;
    returns per-mode results, the roofline object of the first mode and (when
    keep) host copies of p and u of each mode's last step."""
    import numpy as np
    import torch

    from paper_2012_11744_amd import _lib as L
    from paper_2012_11744_amd import solver as S

    rho = _dev(w.rho)
    us = [_dev(u) for u in w.us]
    beta = tuple(torch.empty_like(rho) for _ in range(3))
    b = torch.empty_like(rho)
    p = torch.empty_like(rho)
    u = tuple(torch.empty_like(rho) for _ in range(3))
    S.face_coeffs(rho, w.h, w.bc, out=beta)
    results, fields = {}, {}
    roof = None
    for mi, mode in enumerate(modes):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        sol = S.Solver(beta, w.h, w.bc, precision=mode)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - ts) * 1e3
        step = _step_fn(sol, rho, us, b, p, u, w, args.tol)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        iters = []
        # timed region: exactly `steps` steps.  HIP events stamped by the
        # dispatches of the roofline kernel (fine-level smoother) time its
        # launches in the first quarter of them (at least two steps): each
        # timed launch carries a few microseconds of dispatch overhead, which
        # the other steps do not pay
        timed_steps = min(args.steps, max(2, (args.steps + 3) // 4))
        sol.timing(True, kinds=[L.PP_KT_SMOOTH])
        sol.timing_reset()
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for s_i in range(args.steps):
            step()
            iters.append(sol.last_stats["outer_iters"])
            if s_i + 1 == timed_steps:
                sol.timing(False)
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        sol.timing(False)
        kt = {L.PP_KT_SMOOTH: sol.timing_get(L.PP_KT_SMOOTH)}
        ms = (t_end - t_start) * 1e3 / args.steps
        st = sol.last_stats
        if keep:
            fields[mode] = (p.cpu().numpy(), [c.cpu().numpy() for c in u], st["rel_res"])
        # diagnostic passes (not the headline): the same steps without any
        # timer; every fine-level kernel kind timed; the parts of a step
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - t1) * 1e3 / args.steps
        sol.timing(True)
        sol.timing_reset()
        for _ in range(max(2, args.steps // 4)):
            step()
        torch.cuda.synchronize()
        for k in range(L.PP_KT_COUNT):
            if k != L.PP_KT_SMOOTH:
                kt[k] = sol.timing_get(k)
        sol.timing(False)
        parts = step_parts(sol, rho, us, b, p, u, w, args.tol, reps=max(2, args.steps // 4))
        r = {
            "solves_per_s": 1e3 / ms,
            "ms_per_step": ms,
            "ms_per_step_no_timers": ms_plain,
            "dof_per_s": w.cells * 1e3 / ms,
            "outer_iters": int(np.median(iters)),
            "rel_res": st["rel_res"],
            "fell_back": st["fell_back"],
            "memory_bytes": sol.memory_bytes,
            "setup_ms": setup_ms,
            "step_parts_ms": parts,
        }
        r["kernels"] = kernel_rates(mode, kt, r["outer_iters"], w.cells)
        kern = r["kernels"]
        if mi == 0 and "smoother_sweep" in kern:
            k = kern["smoother_sweep"]
            traffic, source = (counter_traffic() if mode == "fp32" and w.n[0] == 256
                               else (None, "other shape"))
            roof = {"kernel": "fused red-black Gauss-Seidel pass (fine level, %s, %s)"
                              % (mode, "one sweep per launch" if mode == "fp64" else
                                 "two sweeps per launch"),
                    "bound": "hbm", "achieved": round(k["GBps"], 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(k["GBps"] / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "traffic_source": source,
                    "alg_bytes_per_launch": k["alg_bytes"], "avg_launch_ms": k["avg_ms"],
                    "timed_launches": k["launches"], "timed_steps": timed_steps}
        if not args.no_adjoint and mi == 0:
            g_p = _dev(w.us[0])
            for _ in range(2):
                sol.adjoint(p, g_p, tol=args.tol)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            na = max(3, args.steps // 4)
            for _ in range(na):
                sol.adjoint(p, g_p, tol=args.tol)
            torch.cuda.synchronize()
            r["adjoint_ms"] = (time.perf_counter() - ta) * 1e3 / na
            r["adjoint_iters"] = sol.last_stats["outer_iters"]
            del g_p
        results[mode] = r
        log(f"[bench] {mode}: {r['solves_per_s']:.1f} solves/s, {ms:.3f} ms/step "
            f"(no timers {ms_plain:.3f}), iters={r['outer_iters']}, setup {setup_ms:.1f} ms, "
            f"parts {parts}, kernels="
            + ", ".join(f"{k}={v['GBps']:.0f}GB/s" for k, v in kern.items()))
        sol.close()
    del rho, us, beta, b, p, u
    torch.cuda.empty_cache()
    return results, roof, fields


def step_parts(sol, rho, us, b, p, u, w, tol, reps):
    """Mean device time of each part of a step (HIP events on the stream),
    measured in a loop of its own after the timed region."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    acc = [0.0] * 4
    for _ in range(reps):
        ev[0].record()
        sol.update_density(rho)
        ev[1].record()
        sol.divergence(us, 1.0 / w.dt, out=b)
        ev[2].record()
        sol.solve(b, tol=tol, p=p)
        ev[3].record()
        sol.project(us, p, w.dt, out=u)
        ev[4].record()
        torch.cuda.synchronize()
        for i in range(4):
            acc[i] += ev[i].elapsed_time(ev[i + 1])
    names = ("update_density", "divergence", "solve", "project")
    return {n: round(a / reps, 4) for n, a in zip(names, acc)}


def kernel_rates(mode, kt, n_it, cells):
    """Algorithmic GB/s of the fine-level kernel kinds timed by the library."""
    from paper_2012_11744_amd import _lib as L
    # fine-level smoother: each launch reads e_in, r and the three face
    # coefficients once and writes e_out: 6 words per cell; the first
    # launch of each cycle starts from zero and skips e_in (5 words).  FP32
    # and FP16 storage run two sweeps per launch (one launch in two starts
    # from zero with nu_pre = nu_post = 2), FP64 one sweep per launch (one
    # in four).  In FP32 the post-smoothing launch also forms r . z, from
    # values it holds already (no bytes of its own).
    word = {"fp64": 8, "fp32": 4, "fp16": 2}[mode]
    dword = 8 if mode == "fp64" else 4          # outer search direction
    zero_share = 0.25 if mode == "fp64" else 0.5
    n_sm, ms_sm = kt[L.PP_KT_SMOOTH]
    n_rr, ms_rr = kt[L.PP_KT_RESTRICT]
    n_oa, ms_oa = kt[L.PP_KT_OUTER_APPLY]
    n_ou, ms_ou = kt[L.PP_KT_OUTER_UPDATE]
    kern = {}

    def put(name, n, ms, byt):
        avg = ms / n
        kern[name] = {"launches": n, "avg_ms": avg, "alg_bytes": byt,
                      "GBps": byt / (avg * 1e-3) / 1e9}

    if n_sm:
        put("smoother_sweep", n_sm, ms_sm, (6.0 - zero_share) * word * cells)
    if n_rr:
        put("resid_restrict", n_rr, ms_rr, (5 * word + word / 8) * cells)  # e, r, 3 beta; r_H
    if n_oa:
        # new direction + operator: z (V-cycle word) and rho in (the step
        # loads the coefficients from the densities, so the kernel forms
        # beta from them), D_new and q out; from the second iteration D_old
        # in; the iterate takes two directions at a time, in the passes of
        # even iterations from the second: x in and out and D_{k-2} in
        n_it = max(1, n_it)
        n_hold = n_it // 2
        n_two = n_it - 1 - n_hold
        put("outer_apply", n_oa, ms_oa,
            ((16 + word + dword) + n_hold * (16 + word + 2 * dword)
             + n_two * (32 + word + 3 * dword)) / n_it * cells)
    if n_ou:
        put("outer_update", n_ou, ms_ou, (24 + word) * cells)   # q, r in; r, r_T out
    return kern


def errors_vs(w, beta, p_ref, p, u):
    """Max relative errors of a GPU answer against the oracle's: p, D u (at
    the scale of D u*) and u (at the scale of u*); plus the oracle's FP64
    relative residual of the GPU p."""
    import numpy as np

    import oracle
    u_ref = oracle.project(beta, w.bc, w.h, w.dt, w.us, p_ref)
    du = oracle.divergence(u, w.bc, w.h)
    du_ref = oracle.divergence(u_ref, w.bc, w.h)
    dus = np.abs(oracle.divergence(w.us, w.bc, w.h)).max()
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    bm = rhs - rhs.mean()
    res = np.linalg.norm(bm - oracle.apply(beta, w.bc, w.h, p)) / np.linalg.norm(bm)
    return {
        "err_p": float(np.abs(p - p_ref).max() / np.abs(p_ref).max()),
        "err_div": float(np.abs(du - du_ref).max() / dus),
        "err_u": float(max(np.abs(u[m] - u_ref[m]).max() for m in range(3))
                       / max(np.abs(c).max() for c in w.us)),
        "rel_res_oracle": float(res),
    }


def oracle_reference(w, p0=None):
    """The oracle's solution of the workload's system to 1e-13 (warm-started
    from p0 when given)."""
    import oracle
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    t0 = time.perf_counter()
    p_ref, it, rel = oracle.solve(beta, w.bc, w.h, rhs, tol=1e-13, p0=p0)
    log(f"[bench] oracle reference {w.name} {w.n}: {it} iterations to rel {rel:.2e} "
        f"in {time.perf_counter() - t0:.1f}s")
    return beta, p_ref


def oracle_errors(w, fields, ref, tol):
    """Errors of each mode's last step against the oracle (solved to 1e-13)."""
    _beta, p_ref = oracle_reference(w, p0=None if ref is None else ref)
    out = {}
    for mode, (p, u, _rel) in fields.items():
        out[mode] = errors_vs(w, _beta, p_ref, p, u)
        log(f"[bench] {mode} vs oracle: " + ", ".join(f"{k}={v:.2e}" for k, v in out[mode].items()))
    return out


def bench_bubbles128(args):
    """128^3, walls, 20 gas bubbles in liquid at density ratio 1000 (seed 1),
    gravity term in u*: FP64 and mixed FP32 projection steps to args.tol
    with the V-cycle and with the W-cycle (solves/s, iterations), with errors
    against the oracle."""
    import numpy as np
    import torch

    from paper_2012_11744_amd import solver as S
    from paper_2012_11744_amd import workloads as W
    w = W.config2(128)
    rho = _dev(w.rho)
    us = [_dev(u) for u in w.us]
    beta = S.face_coeffs(rho, w.h, w.bc)
    b, p = torch.empty_like(rho), torch.empty_like(rho)
    u = tuple(torch.empty_like(rho) for _ in range(3))
    out, fields = {}, {}
    steps = max(5, args.steps // 2)
    for mode, cycle in (("fp64", "v"), ("fp32", "v"), ("fp64", "w"), ("fp32", "w"), ("fp64", "f"),
                        ("fp32", "f")):
        key = mode if cycle == "v" else f"{mode}_{cycle}_cycle"
        with S.Solver(beta, w.h, w.bc, precision=mode, cycle=cycle) as sol:
            step = _step_fn(sol, rho, us, b, p, u, w, args.tol)
            for _ in range(2):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            iters = []
            for _ in range(steps):
                step()
                iters.append(sol.last_stats["outer_iters"])
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            st = sol.last_stats
            out[key] = {"solves_per_s": 1e3 / ms, "ms_per_step": ms,
                        "outer_iters": int(np.median(iters)), "rel_res": st["rel_res"],
                        "fell_back": st["fell_back"]}
            fields[key] = (p.cpu().numpy(), [c.cpu().numpy() for c in u])
        log(f"[bench] bubbles 128^3 {key}: {1e3 / ms:.1f} solves/s, {ms:.3f} ms/step, "
            f"iters={out[key]['outer_iters']}")
    del rho, us, beta, b, p, u
    torch.cuda.empty_cache()
    if not args.no_errors:
        beta_o, p_ref = oracle_reference(w)
        for mode, (ph, uh) in fields.items():
            out[mode].update(errors_vs(w, beta_o, p_ref, ph, uh))
    res = {"workload": "20 gas bubbles in liquid, rho 1000/1, 128^3, walls, gravity in u*, "
                       f"tol {args.tol:g}", "steps": steps}
    res.update({m: _fmt(v) for m, v in out.items()})
    if "fp64" in out and "fp32" in out:
        res["mixed_over_fp64"] = round(out["fp32"]["solves_per_s"] / out["fp64"]["solves_per_s"], 3)
    return res


def bench_jet512(args):
    """Forward (coefficients and hierarchy from rho, divergence, mixed solve
    to tol, projection) and backward (adjoint solve re-running the V-cycles,
    face products) at 512^3 with walls on all sides: ms and iterations per
    solve, device memory, and the oracle's FP64 residuals of the answers."""
    import numpy as np
    import torch

    import oracle
    from paper_2012_11744_amd import solver as S
    from paper_2012_11744_amd import workloads as W
    t0 = time.time()
    w = W.config5(512)
    log(f"[bench] jet 512^3 generated in {time.time() - t0:.1f}s")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, total = torch.cuda.mem_get_info()
    rho = _dev(w.rho)
    us = [_dev(u) for u in w.us]
    wt = _dev(w.w)
    beta = S.face_coeffs(rho, w.h, w.bc)
    b, p = torch.empty_like(rho), torch.empty_like(rho)
    u = tuple(torch.empty_like(rho) for _ in range(3))
    sol = S.Solver(beta, w.h, w.bc, precision="fp32")
    fwd = _step_fn(sol, rho, us, b, p, u, w, args.tol)
    reps = 3
    fwd()
    torch.cuda.synchronize()
    tf = []
    for _ in range(reps):
        t1 = time.perf_counter()
        fwd()
        torch.cuda.synchronize()
        tf.append((time.perf_counter() - t1) * 1e3)
    fwd_it = sol.last_stats["outer_iters"]
    g = sol.adjoint(p, wt, tol=args.tol)
    torch.cuda.synchronize()
    tb = []
    for _ in range(reps):
        del g
        t2 = time.perf_counter()
        g = sol.adjoint(p, wt, tol=args.tol)
        torch.cuda.synchronize()
        tb.append((time.perf_counter() - t2) * 1e3)
    bwd_it = sol.last_stats["outer_iters"]
    free1, _ = torch.cuda.mem_get_info()
    res = {
        "workload": "jet along x, rho 800/1, 512^3, walls, mixed FP32 V-cycle in FP64 PCG, "
                    f"tol {args.tol:g}",
        "forward_ms": round(float(np.median(tf)), 3), "forward_iters": fwd_it,
        "backward_ms": round(float(np.median(tb)), 3), "backward_iters": bwd_it,
        "solver_context_bytes": sol.memory_bytes,
        "device_bytes_in_use": int(free0 - free1),
        "device_bytes_note": "fields (rho, u*, w, beta, b, p, u), solver context and adjoint "
                             "outputs (lambda, 3 face products), all resident at once",
        "cells": w.cells, "reps": reps,
    }
    if not args.no_errors:
        ph, lh = p.cpu().numpy(), g[0].cpu().numpy()
        uh = [c.cpu().numpy() for c in u]
        betah = [x.cpu().numpy() for x in beta]
        rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
        bm = rhs - rhs.mean()
        res["rel_res_oracle"] = float(np.linalg.norm(bm - oracle.apply(betah, w.bc, w.h, ph))
                                      / np.linalg.norm(bm))
        du = oracle.divergence(uh, w.bc, w.h)
        res["rel_div_u"] = float(np.linalg.norm(du) / np.linalg.norm(
            oracle.divergence(w.us, w.bc, w.h)))
        wm = w.w - w.w.mean()
        res["adjoint_rel_res_oracle"] = float(
            np.linalg.norm(wm - oracle.apply(betah, w.bc, w.h, lh)) / np.linalg.norm(wm))
    sol.close()
    del rho, us, wt, beta, b, p, u, g
    torch.cuda.empty_cache()
    log(f"[bench] jet 512^3: forward {res['forward_ms']} ms ({fwd_it} iterations), backward "
        f"{res['backward_ms']} ms ({bwd_it} iterations), device bytes {res['device_bytes_in_use']}")
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_projection_step(w, tol):
    """The oracle's projection step (face coefficients, divergence, solve to
    tol, projection); returns (seconds, p, iterations, rel_res)."""
    import oracle
    t0 = time.perf_counter()
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    p, it, rel = oracle.solve(beta, w.bc, w.h, rhs, tol=tol)
    oracle.project(beta, w.bc, w.h, w.dt, w.us, p)
    return time.perf_counter() - t0, p, it, rel


def cpu_baseline(w, args):
    """The FP64 CPU oracle's full projection step on the same system and
    tolerance, timed: median of args.cpu_repeats runs on all host threads,
    then one run on one thread of the same geometry at args.cpu_1thread_n^3.
    Returns the baseline object and the last p (a warm start for the error
    reference)."""
    import numpy as np

    import oracle
    from paper_2012_11744_amd import workloads as W
    threads = oracle.threads()
    runs = []
    p = None
    for _ in range(max(1, args.cpu_repeats)):
        t, p, it, rel = cpu_projection_step(w, args.tol)
        runs.append(t)
        log(f"[bench] cpu oracle step: {t:.2f}s ({it} iterations, rel {rel:.2e}, "
            f"{threads} threads)")
    med = float(np.median(runs))
    one = None
    if args.cpu_1thread_n > 0:
        w1 = W.config3(args.cpu_1thread_n)
        oracle.set_threads(1)
        try:
            t1, _, it1, rel1 = cpu_projection_step(w1, args.tol)
        finally:
            oracle.set_threads(threads)
        one = {"value": round(1.0 / t1, 6), "unit": "solves/s", "cores": 1,
               "workload": f"the same geometry at {args.cpu_1thread_n}^3", "seconds": round(t1, 3),
               "iterations": it1, "rel_res": rel1}
        log(f"[bench] cpu oracle step, 1 thread, {args.cpu_1thread_n}^3: {t1:.2f}s "
            f"({it1} iterations)")
    out = {"value": round(1.0 / med, 6), "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"measured: the oracle's full projection step (face coefficients, "
                     f"divergence, FP64 MG-PCG to rel. residual {args.tol:g}, projection) on "
                     f"the same {w.n[0]}^3 system, {it} iterations (rel {rel:.2e}), median of "
                     f"{len(runs)} runs on {threads} threads",
           "runs_s": [round(x, 3) for x in runs], "iterations": it, "cpu_model": cpu_model(),
           "one_thread": one}
    return out, p


if __name__ == "__main__":
    main()
