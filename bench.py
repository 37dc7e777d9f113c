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
reported under "modes".
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
    ap.add_argument("--cpu-sample-iters", type=int, default=12,
                    help="oracle PCG iterations in the CPU-baseline sample")
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

    from paper_2012_11744_amd import _lib as L
    from paper_2012_11744_amd import solver as S
    from paper_2012_11744_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "jet512":
        jet512(args)
        return
    N = args.n
    t0 = time.time()
    w = W.config3(N)
    log(f"[bench] workload {w.name} {N}^3 generated in {time.time() - t0:.1f}s")

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    rho = dev(w.rho)
    us = [dev(u) for u in w.us]
    beta = tuple(torch.empty_like(rho) for _ in range(3))
    b = torch.empty_like(rho)
    p = torch.empty_like(rho)
    u = tuple(torch.empty_like(rho) for _ in range(3))
    S.face_coeffs(rho, w.h, w.bc, out=beta)

    modes = args.modes.split(",")
    results = {}
    roof = None
    for mi, mode in enumerate(modes):
        sol = S.Solver(beta, w.h, w.bc, precision=mode)

        def step():
            sol.update_density(rho)
            sol.divergence(us, 1.0 / w.dt, out=b)
            sol.solve(b, tol=args.tol, p=p)
            sol.project(us, p, w.dt, out=u)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        iters = []
        # timed region: exactly `steps` steps; HIP-event timers bracket the
        # launches of the roofline kernel (fine-level smoother) only
        sol.timing(True, kinds=[L.PP_KT_SMOOTH])
        sol.timing_reset()
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            step()
            iters.append(sol.last_stats["outer_iters"])
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        kt = {L.PP_KT_SMOOTH: sol.timing_get(L.PP_KT_SMOOTH)}
        sol.timing(False)
        ms = (t_end - t_start) * 1e3 / args.steps
        # diagnostic pass (not the headline): the same steps without any timer,
        # then with every fine-level kernel kind timed
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
        st = sol.last_stats
        r = {
            "solves_per_s": 1e3 / ms,
            "ms_per_step": ms,
            "ms_per_step_no_timers": ms_plain,
            "dof_per_s": w.cells * 1e3 / ms,
            "outer_iters": int(np.median(iters)),
            "rel_res": st["rel_res"],
            "fell_back": st["fell_back"],
            "memory_bytes": sol.memory_bytes,
        }
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
        if n_sm:
            avg = ms_sm / n_sm
            byt = (6.0 - zero_share) * word * w.cells
            kern["smoother_sweep"] = {"launches": n_sm, "avg_ms": avg, "alg_bytes": byt,
                                      "GBps": byt / (avg * 1e-3) / 1e9}
        if n_rr:
            avg = ms_rr / n_rr
            byt = (5 * word + word / 8) * w.cells   # e, r, 3 beta in; r_H out
            kern["resid_restrict"] = {"launches": n_rr, "avg_ms": avg, "alg_bytes": byt,
                                      "GBps": byt / (avg * 1e-3) / 1e9}
        if n_oa:
            avg = ms_oa / n_oa
            # new direction + operator: z (V-cycle word) and rho in (the step
            # loads the coefficients from the densities, so the kernel forms
            # beta from them), D_new and q out; from the second iteration D_old
            # in; the iterate takes two directions at a time, in the passes of
            # even iterations from the second: x in and out and D_{k-2} in
            n_it = max(1, r["outer_iters"])
            n_hold = n_it // 2
            n_two = n_it - 1 - n_hold
            byt = ((16 + word + dword) + n_hold * (16 + word + 2 * dword)
                   + n_two * (32 + word + 3 * dword)) / n_it * w.cells
            kern["outer_apply"] = {"launches": n_oa, "avg_ms": avg, "alg_bytes": byt,
                                   "GBps": byt / (avg * 1e-3) / 1e9}
        if n_ou:
            avg = ms_ou / n_ou
            byt = (24 + word) * w.cells             # q, r in; r out; r_T out
            kern["outer_update"] = {"launches": n_ou, "avg_ms": avg, "alg_bytes": byt,
                                    "GBps": byt / (avg * 1e-3) / 1e9}
        r["kernels"] = kern
        if mi == 0 and "smoother_sweep" in kern:
            k = kern["smoother_sweep"]
            traffic, source = counter_traffic() if mode == "fp32" and N == 256 else (None, "other shape")
            roof = {"kernel": "fused red-black Gauss-Seidel pass (fine level, %s, %s)"
                              % (mode, "one sweep per launch" if mode == "fp64" else
                                 "two sweeps per launch"),
                    "bound": "hbm", "achieved": round(k["GBps"], 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(k["GBps"] / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "traffic_source": source,
                    "alg_bytes_per_launch": k["alg_bytes"], "avg_launch_ms": k["avg_ms"]}
        if not args.no_adjoint and mi == 0:
            g_p = dev(w.us[0])
            gr = torch.empty_like(rho)
            for _ in range(2):
                sol.adjoint(p, g_p, tol=args.tol)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for _ in range(max(3, args.steps // 4)):
                sol.adjoint(p, g_p, tol=args.tol)
            torch.cuda.synchronize()
            r["adjoint_ms"] = (time.perf_counter() - ta) * 1e3 / max(3, args.steps // 4)
            r["adjoint_iters"] = sol.last_stats["outer_iters"]
            del gr
        results[mode] = r
        log(f"[bench] {mode}: {r['solves_per_s']:.1f} solves/s, {ms:.3f} ms/step "
            f"(no timers {ms_plain:.3f}), iters={r['outer_iters']}, kernels="
            + ", ".join(f"{k}={v['GBps']:.0f}GB/s" for k, v in kern.items()))
        sol.close()

    copy = copy_bandwidth()
    log(f"[bench] copy kernel: {copy['GBps']:.0f} GB/s")
    if roof is not None:
        roof["copy_kernel_GBps"] = round(copy["GBps"], 1)
        roof["frac_of_copy"] = round(roof["achieved"] / copy["GBps"], 4)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args)

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
        "modes": {m: {k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in r.items()
                      if k != "kernels"} for m, r in results.items()},
        "kernels": {m: r["kernels"] for m, r in results.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if "fp64" in results and modes[0] != "fp64":
        line["mixed_over_fp64"] = round(head["solves_per_s"] / results["fp64"]["solves_per_s"], 3)
    print(json.dumps(line), flush=True)


def jet512(args):
    """Forward (setup + divergence + mixed solve to 1e-8 + projection) and
    backward (adjoint solve re-running the V-cycles + face products) at 512^3
    with walls on all sides: ms and device memory per solve."""
    import numpy as np
    import torch

    from paper_2012_11744_amd import solver as S
    from paper_2012_11744_amd import workloads as W
    t0 = time.time()
    w = W.config5(512)
    log(f"[bench] jet 512^3 generated in {time.time() - t0:.1f}s")

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    rho = dev(w.rho)
    us = [dev(u) for u in w.us]
    wt = dev(w.w)
    beta = tuple(torch.empty_like(rho) for _ in range(3))
    b = torch.empty_like(rho)
    p = torch.empty_like(rho)
    u = tuple(torch.empty_like(rho) for _ in range(3))
    S.face_coeffs(rho, w.h, w.bc, out=beta)
    torch.cuda.synchronize()
    fields = torch.cuda.memory_allocated()
    sol = S.Solver(beta, w.h, w.bc, precision="fp32")

    def forward():
        sol.update_density(rho)
        sol.divergence(us, 1.0 / w.dt, out=b)
        sol.solve(b, tol=args.tol, p=p)
        sol.project(us, p, w.dt, out=u)

    reps = max(2, args.steps // 4)
    forward()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        forward()
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t1) * 1e3 / reps
    fwd_it = sol.last_stats["outer_iters"]
    sol.adjoint(p, wt, tol=args.tol)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(reps):
        g = sol.adjoint(p, wt, tol=args.tol)
        del g
    torch.cuda.synchronize()
    bwd_ms = (time.perf_counter() - t2) * 1e3 / reps
    bwd_it = sol.last_stats["outer_iters"]
    peak = torch.cuda.max_memory_allocated()
    line = {
        "metric": "pressure projection forward + backward at 512^3, ms and device memory per solve",
        "workload": "jet along x, rho 800 / 1, 512^3, walls, mixed FP32 V-cycle in FP64 PCG, tol %g"
                    % args.tol,
        "forward_ms": round(fwd_ms, 3), "forward_iters": fwd_it,
        "backward_ms": round(bwd_ms, 3), "backward_iters": bwd_it,
        "solver_context_bytes": sol.memory_bytes,
        "torch_fields_bytes": int(fields),
        "torch_peak_bytes_with_backward_outputs": int(peak),
        "cells": w.cells, "reps": reps,
    }
    sol.close()
    print(json.dumps(line), flush=True)


def cpu_baseline(w, args):
    """The FP64 CPU oracle on a bounded sample of the same solve: its MG-PCG
    on the full-size system, capped at a few iterations; solves/s is scaled
    by the iteration count needed for tol, extrapolated from the observed
    residual reduction per iteration."""
    import numpy as np

    import oracle
    t0 = time.perf_counter()
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    t_setup = time.perf_counter() - t0
    k = args.cpu_sample_iters
    t1 = time.perf_counter()
    _, it, rel = oracle.solve(beta, w.bc, w.h, rhs, tol=args.tol, maxit=k, check=False)
    t_solve = time.perf_counter() - t1
    if rel <= args.tol:
        need = it
    else:
        rate = rel ** (1.0 / max(it, 1))
        need = it * math.log(args.tol) / math.log(rel) if rate < 1 else float("inf")
    per_iter = t_solve / max(it, 1)
    est = t_setup + per_iter * need
    log(f"[bench] cpu oracle: {it} iterations in {t_solve:.1f}s (rel {rel:.2e}), "
        f"~{need:.1f} needed -> {est:.1f}s per solve on {oracle.threads()} threads")
    return {"value": round(1.0 / est, 6), "unit": "solves/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"oracle FP64 MG-PCG on the same {w.n[0]}^3 system, {it} iterations "
                      f"({t_solve:.1f}s, rel res {rel:.2e}); per-solve time = setup + "
                      f"per-iteration time x {need:.1f} iterations extrapolated to tol {args.tol:g}"}


if __name__ == "__main__":
    main()
