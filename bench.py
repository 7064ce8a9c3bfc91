"""Benchmark of the two-site DMRG hot path on one MI355X.

Workload: pf shell, 40 m-scheme sites, 8 protons + 8 neutrons, M = 0
(the 56Ni valence space; m-scheme dimension 1,087,455,228), random
eps / Vbar of the seeded generator, natural orbital ordering.  The sweep
schedule ramps the bond dimension 512, 512, 1024, 1024 (warm-up sweeps)
and the timed sweeps run at D = 2048.  One "step" is one full sweep
(left-to-right and back), i.e. every stage of the hot path at every bond:
blocking, H_eff diagonal, Davidson with H_eff.psi products, density-matrix
truncation, renormalisation and prediction.

The same schedule runs twice from scratch: FP64 products, then mixed FP32
products with FP64 residual correction.  The reported value is the mixed
run's H_eff.psi throughput (algorithmic flops of the sector GEMMs divided by
their device time, HIP events on the library stream); the FP64 run gives the
reference energy and sweep time.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precisions fp64,fp32]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # dense MFMA TFLOP/s, MI355X
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
SWEEP_CRIT_MEV = 1e-4   # the paper sweeps until the energy changes by less than this between sweeps
HBM_PEAK = 8000.0   # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_schedule(workload, prec: str, warmup: int, steps: int, D_main: int, seed: int, tol: float,
                 check: bool = False):
    """The benchmark schedule in one precision: `warmup` sweeps of the ramp
    (then D_main), `steps` timed sweeps at D_main; with `check`, one more
    (untimed) sweep in which every mixed solve is repeated in FP64 from the
    same guess on the same H_eff (dmrg_check_fp64)."""
    import torch
    import paper_1507_00161_amd as pk
    h = workload.hamiltonian()
    sp = h.space
    ctx = pk.Context(precision=PREC[prec], davidson_tol=tol, noise=1e-4, noise_sweeps=2, seed=seed)
    ctx.load_hamiltonian(sp.species, sp.two_m, h.eps, h.V.ravel(), h.n_p, h.n_n, h.two_M)
    ramp = list(workload.D_schedule)
    energies = []      # every sweep of the schedule, warm-up included
    for w in range(warmup):
        D = ramp[w] if w < len(ramp) else D_main
        t = time.perf_counter()
        r = ctx.sweep(D)
        energies.append(r["energy"])
        log(f"[{prec}] warmup sweep {w} D={D}: E={r['energy']:.9f} {time.perf_counter() - t:.1f}s "
            f"products lo/64={r['products_low']}/{r['products_fp64']} not converged {r['not_converged']}")
    torch.cuda.synchronize()
    tot = {}
    walls = []
    deltas = []        # energy change against the previous sweep, per timed sweep (MeV)
    energy = None
    # host clock readings around the timed sweeps, so that a profiler's trace
    # (whose timestamps come from one of these clocks) can pick out their launches
    win = {"boottime": [time.clock_gettime_ns(time.CLOCK_BOOTTIME)], "monotonic": [time.monotonic_ns()]}
    for k in range(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = ctx.sweep(D_main)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t)
        energy = r["energy"]
        energies.append(energy)
        deltas.append(r["delta_energy"])
        for key, v in r.items():
            if isinstance(v, (int, float)) and key not in ("energy", "last_theta", "code", "status",
                                                           "delta_energy"):
                tot[key] = tot.get(key, 0) + v
        log(f"[{prec}] timed sweep {k} D={D_main}: E={r['energy']:.9f} dE={r['delta_energy']:.2e} {walls[-1]:.2f}s "
            f"products lo/64={r['products_low']}/{r['products_fp64']} not converged {r['not_converged']} "
            f"heff {r['heff_flops'] / max(r['heff_seconds'], 1e-12) / 1e12:.2f} TF/s; "
            f"time in products {r['heff_seconds']:.2f}s, truncation+renorm+prediction "
            f"{r['renorm_seconds']:.2f}s (density {r['density_seconds']:.2f}, eig {r['eig_seconds']:.2f}, "
            f"renormalize {r['renormalize_seconds']:.2f}, predict {r['predict_seconds']:.2f}), "
            f"blocking+plans {r['blocking_seconds']:.2f}s")
    torch.cuda.synchronize()
    win["boottime"].append(time.clock_gettime_ns(time.CLOCK_BOOTTIME))
    win["monotonic"].append(time.monotonic_ns())
    chk = None
    if check and prec != "fp64":
        ctx.check_fp64(True)
        t = time.perf_counter()
        r = ctx.sweep(D_main)
        chk = {"solves": int(r["check_solves"]), "max_rel": r["check_max_rel"], "energy": r["energy"]}
        log(f"[{prec}] check sweep D={D_main}: every solve repeated in FP64 from the same guess, "
            f"{chk['solves']} pairs, max |theta - theta_fp64| / |theta_fp64| = {chk['max_rel']:.3e} "
            f"({time.perf_counter() - t:.1f}s)")
    ctx.close()
    return dict(energy=energy, walls=walls, tot=tot, energies=energies, deltas=deltas, check=chk, window=win)


def plateaus(name: str, prec: str, Ds, per: int, tol: float, trunc_eps: float = 0.0, d_min: int = 0,
             n_states: int = 1):
    """Energy against discarded weight along a D schedule of plateaus (`per`
    sweeps at each D), with the sweep time and the H_eff GEMM throughput of the
    last sweep of each plateau; one JSON line per plateau."""
    import torch
    import paper_1507_00161_amd as pk
    from workloads import WORKLOADS
    h = WORKLOADS[name].hamiltonian()
    sp = h.space
    ctx = pk.Context(precision=PREC[prec], davidson_tol=tol, noise=1e-4, noise_sweeps=2, seed=1507,
                     trunc_eps=trunc_eps, d_min=d_min, n_states=n_states)
    ctx.load_hamiltonian(sp.species, sp.two_m, h.eps, h.V.ravel(), h.n_p, h.n_n, h.two_M)
    peak = PEAK[prec]
    for D in Ds:
        for k in range(per):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = ctx.sweep(D)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
            log(f"[{name} {prec}] D={D} sweep {k}: E={r['energy']:.9f} discarded max {r['discarded_max']:.2e} "
                f"kept max {r['kept_max']} {wall:.1f}s products lo/64={r['products_low']}/{r['products_fp64']} "
                f"not converged {r['not_converged']}"
                + (f" E1={r['energy_excited']:.9f}" if n_states == 2 else ""))
        free, total = torch.cuda.mem_get_info()
        g = {}
        for ph, kn in (("gemm1", "k_heff_z"), ("gemm2", "k_heff_y")):
            if r[f"{ph}_seconds"] > 0:
                tf = r[f"{ph}_flops"] / r[f"{ph}_seconds"] / 1e12
                g[kn] = {"tflops": tf, "frac_of_peak": tf / peak}
        print(json.dumps({"workload": name, "precision": prec, "D": D, "energy": r["energy"],
                          "trunc_eps": trunc_eps, "d_min": d_min, "kept_max": r["kept_max"],
                          "n_states": n_states, "energy_excited": r["energy_excited"] if n_states == 2 else None,
                          "discarded_max": r["discarded_max"], "discarded_sum": r["discarded_sum"],
                          "sweep_s": wall, "heff_tflops": r["heff_flops"] / max(r["heff_seconds"], 1e-12) / 1e12,
                          "products_low": r["products_low"], "products_fp64": r["products_fp64"],
                          "not_converged": r["not_converged"], "gemm_phases": g,
                          "device_mem_used_gb": (total - free) / 1e9}), flush=True)
    ctx.close()


def converge(name: str, prec: str, Ds, max_sweeps: int, budget_s: float, tol: float):
    """The paper's stopping rule along a D schedule: at each D, sweep until the
    energy changes by less than 1e-4 MeV between two sweeps (at most
    `max_sweeps` sweeps or `budget_s` seconds per D).  One JSON line per D,
    then the paper's extrapolation E(M) = E_inf + X1 M^X2 over the D values
    whose sweeps met the rule.  Returns {D: energy}."""
    import torch
    import paper_1507_00161_amd as pk
    from workloads import WORKLOADS
    h = WORKLOADS[name].hamiltonian()
    sp = h.space
    ctx = pk.Context(precision=PREC[prec], davidson_tol=tol, noise=1e-4, noise_sweeps=2, seed=1507)
    ctx.load_hamiltonian(sp.species, sp.two_m, h.eps, h.V.ravel(), h.n_p, h.n_n, h.two_M)
    out = {}
    for D in Ds:
        t_plateau = time.perf_counter()
        energies, deltas, walls = [], [], []
        met = False
        for k in range(max_sweeps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = ctx.sweep(D)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t)
            energies.append(r["energy"])
            # the first sweep at a new D is compared with the last one at the previous D;
            # the rule is applied from the second sweep of the plateau on
            d = r["delta_energy"]
            deltas.append(d)
            log(f"[{name} {prec}] D={D} sweep {k}: E={r['energy']:.9f} dE={d:.3e} {walls[-1]:.2f}s "
                f"not converged {r['not_converged']}")
            if k >= 1 and abs(d) < SWEEP_CRIT_MEV:
                met = True
                break
            if time.perf_counter() - t_plateau > budget_s:
                break
        out[D] = {"energy": energies[-1], "met": met}
        print(json.dumps({"mode": "converge", "workload": name, "precision": prec, "D": D,
                          "criterion_MeV": SWEEP_CRIT_MEV, "met": met, "sweeps": len(energies),
                          "energy": energies[-1],
                          "delta_E_MeV_last": None if math.isnan(deltas[-1]) else deltas[-1],
                          "delta_E_MeV": [None if math.isnan(x) else x for x in deltas],
                          "s_per_sweep_mean": sum(walls) / len(walls),
                          "plateau_s": time.perf_counter() - t_plateau}), flush=True)
    ctx.close()
    pts = sorted((D, v["energy"]) for D, v in out.items() if v["met"])
    fit = extrapolate(pts)
    print(json.dumps({"mode": "extrapolation", "workload": name, "precision": prec,
                      "points": pts, "fit": fit}), flush=True)
    return out


def extrapolate(pts):
    """E(M) = E_inf + X1 M^X2 through (M, E) points (least squares; exact
    through three points).  None when fewer than three points or no fit."""
    if len(pts) < 3:
        return None
    import numpy as np
    from scipy.optimize import least_squares
    M = np.array([p[0] for p in pts], float)
    E = np.array([p[1] for p in pts], float)

    def lin(x2):   # for fixed X2 the model is linear in (E_inf, X1)
        A = np.stack([np.ones_like(M), M ** x2], 1)
        c, *_ = np.linalg.lstsq(A, E, rcond=None)
        return c, A @ c - E
    try:
        r = least_squares(lambda x: lin(x[0])[1], x0=[-0.5], bounds=([-6.0], [-1e-3]), jac="3-point",
                          xtol=1e-15, ftol=1e-15, gtol=1e-15)
        x2 = float(r.x[0])
        c, res = lin(x2)
    except Exception:
        return None
    return {"E_inf": float(c[0]), "X1": float(c[1]), "X2": x2, "max_residual_MeV": float(np.abs(res).max())}


def preprocess(name: str, prec: str, D_pre: int, sweeps_pre: int, Ds, per: int, tol: float):
    """The preprocessing phase of the entropy paragraph and what it buys:
    measuring sweeps at a small D give the one-orbital entropies and the
    mutual information; the Fiedler-vector ordering of the latter is then run
    against the natural order on the same D schedule (fresh contexts, the same
    options).  One JSON line for the measurement, one per plateau and order."""
    import numpy as np
    import torch
    import paper_1507_00161_amd as pk
    from workloads import WORKLOADS
    h = WORKLOADS[name].hamiltonian()
    sp = h.space
    n = sp.n_sites
    common = dict(precision=PREC[prec], davidson_tol=tol, noise=1e-4, noise_sweeps=2, seed=1507)
    ctx = pk.Context(measure=1, **common)
    ctx.load_hamiltonian(sp.species, sp.two_m, h.eps, h.V.ravel(), h.n_p, h.n_n, h.two_M)
    for k in range(sweeps_pre):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = ctx.sweep(D_pre)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        log(f"[{name} {prec}] measuring sweep {k} D={D_pre}: E={r['energy']:.9f} {wall:.1f}s "
            f"(measurement {r['measure_seconds']:.2f}s)")
    m = ctx.orbital_entropies()
    ctx.close()
    order, fval = pk.fiedler_ordering(m["mutual"])
    I = m["mutual"]

    def dist(o):
        pos = np.empty(n, np.int64)
        pos[np.asarray(o)] = np.arange(n)
        return float(np.sum(np.triu(I * (pos[:, None] - pos[None, :]) ** 2.0, 1)))

    iu = np.triu_indices(n, 1)
    top = np.argsort(I[iu])[::-1][:8]
    print(json.dumps({"workload": name, "precision": prec, "phase": "measure", "D": D_pre,
                      "sweeps": sweeps_pre, "energy": r["energy"], "sweep_s": wall,
                      "measure_s": r["measure_seconds"],
                      "s1": {"min": float(m["s1"].min()), "max": float(m["s1"].max()),
                             "mean": float(m["s1"].mean())},
                      "mutual_max": float(I.max()),
                      "top_pairs": [[int(iu[0][x]), int(iu[1][x]), float(I[iu][x])] for x in top],
                      "fiedler_value": fval, "ordering": order.tolist(),
                      "I_dist_natural": dist(np.arange(n)), "I_dist_fiedler": dist(order)}), flush=True)
    # natural and Fiedler orders from the hash start; natural order from the
    # CI-DEAS start built with the measured entropies and occupations
    for label, ordering in (("natural", None), ("fiedler", order), ("natural_cideas", None)):
        c = pk.Context(**common)
        c.load_hamiltonian(sp.species, sp.two_m, h.eps, h.V.ravel(), h.n_p, h.n_n, h.two_M)
        if label.endswith("cideas"):
            c.set_cideas(m["s1"], m["n1"])
        for D in Ds:
            for k in range(per):
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = c.sweep(D, ordering)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t
                log(f"[{name} {prec} {label}] D={D} sweep {k}: E={r['energy']:.9f} "
                    f"discarded max {r['discarded_max']:.2e} {wall:.1f}s")
                print(json.dumps({"workload": name, "precision": prec, "phase": "sweep", "order": label,
                                  "D": D, "sweep": k, "energy": r["energy"], "sweep_s": wall}), flush=True)
            print(json.dumps({"workload": name, "precision": prec, "phase": "production", "order": label,
                              "D": D, "energy": r["energy"], "discarded_max": r["discarded_max"],
                              "discarded_sum": r["discarded_sum"], "sweep_s": wall,
                              "not_converged": r["not_converged"]}), flush=True)
        c.close()


def cpu_baseline(budget_s: float = 25.0, D: int = 256):
    """The oracle's H_eff.psi throughput beside the GPU's on one bounded
    sample of the benchmark workload: the first sweep at D (same options as
    the benchmark) is run step by step by the NumPy oracle until `budget_s`
    seconds have passed, then the same steps by the library in FP64 and mixed
    FP32.  Both rates are algorithmic flops (the library's count for the
    products of each step, cheaper contraction order) per second of product
    time, so they are in one unit; the oracle's products per step are its own."""
    import torch
    from threadpoolctl import threadpool_info
    import paper_1507_00161_amd as pk
    from oracle import dmrg
    from workloads import WORKLOADS

    class _Stop(Exception):
        pass

    h = WORKLOADS["pf_8p8n"].hamiltonian()
    sp = h.space
    opts = dict(davidson_tol=1e-7, noise=1e-4, noise_sweeps=2, seed=1507)
    o = dmrg.DMRG(h.eps, h.V, sp.species, sp.two_m, h.n_p, h.n_n, h.two_M, opts=dmrg.Options(**opts))
    steps = []     # per step: oracle products, oracle seconds in products
    last = [0.0, 0]
    t0 = time.perf_counter()

    def hook(oo, bond, direction, setup):
        steps.append((oo.nprod_total - last[1], oo.heff_seconds - last[0]))
        last[0], last[1] = oo.heff_seconds, oo.nprod_total
        if time.perf_counter() - t0 > budget_s:
            raise _Stop

    try:
        o.sweep(D, on_step=hook)
    except _Stop:
        pass
    threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    k = len(steps)
    gpu = {}
    alg_per_product = None
    for prec in ("fp64", "fp32"):
        c = pk.Context(precision=PREC[prec], **opts)
        c.load_hamiltonian(sp.species, sp.two_m, h.eps, h.V.ravel(), h.n_p, h.n_n, h.two_M)
        prev = {"heff_flops": 0.0, "heff_seconds": 0.0, "products_low": 0, "products_fp64": 0}
        rows = []
        for _ in range(k):
            r = c.sweep_steps(D, 1)
            d = {key: r[key] - prev[key] for key in prev}
            prev = {key: r[key] for key in prev}
            rows.append(d)
        torch.cuda.synchronize()
        c.close()
        fl = sum(d["heff_flops"] for d in rows)
        sec = sum(d["heff_seconds"] for d in rows)
        gpu[prec] = {"tflops": fl / max(sec, 1e-12) / 1e12,
                     "products": int(sum(d["products_low"] + d["products_fp64"] for d in rows)),
                     "product_seconds": sec}
        if prec == "fp64":
            alg_per_product = [d["heff_flops"] / max(d["products_low"] + d["products_fp64"], 1) for d in rows]
    cpu_flops = sum(a * n for a, (n, _) in zip(alg_per_product, steps))
    cpu_sec = sum(t for _, t in steps)
    return {"value": cpu_flops / max(cpu_sec, 1e-12) / 1e12, "unit": "TFLOP/s", "cores": int(threads),
            "host_cpus": os.cpu_count(), "kind": "oracle",
            "products": int(sum(n for n, _ in steps)), "product_seconds": cpu_sec,
            "gpu_same_sample": gpu,
            "sample": f"pf 8p+8n, first sweep at D={D} from the hash start, its first {k} two-site steps "
                      f"(the oracle's {budget_s:.0f} s budget), run by the NumPy oracle (BLAS threads = cores) "
                      f"and by the library (gpu_same_sample); algorithmic H_eff flops per second of product time"}


# the kernels and the engine that builds their task lists: counters taken for
# other sources do not describe the current launches
KERNEL_SRCS = [os.path.join(ROOT, "paper_1507_00161_amd", "csrc", f) for f in ("device.hip", "engine.cpp")]
# HBM traffic summaries of the two H_eff GEMM phases (FP32, benchmark workload)
TRAFFIC_FILES = {"k_heff_y<float, float, 32>": os.path.join(ROOT, "profiles", "k_heff_y_f32_pf_8p8n_D2048_traffic.txt"),
                 "k_heff_z<float, float, 32>": os.path.join(ROOT, "profiles", "k_heff_z_f32_pf_8p8n_D2048_traffic.txt")}


def source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, alg_bytes_per_launch):
    """HBM bytes per launch of `kernel` from its committed counter summary, or
    None when there is none, the kernel source changed since it was taken, or
    it was taken over other launches (its algorithmic bytes per launch differ
    from this run's by more than 0.1%: another schedule of sweeps)."""
    try:
        lines = open(TRAFFIC_FILES[kernel]).read().splitlines()
    except (OSError, KeyError):
        return None
    kv = dict(l.strip().split("=", 1) for l in lines if "=" in l and not l.startswith("#"))
    if kv.get("sources_sha256") != source_sha():
        return None
    alg = [float(l.split()[-1]) for l in lines if l.startswith("# algorithmic bytes per launch")]
    if not alg or abs(alg[0] - alg_bytes_per_launch) > 1e-3 * alg_bytes_per_launch:
        return None
    return float(kv["hbm_bytes_per_launch"])


def _csv_rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _find(d, suffix):
    import glob
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def _short(name):
    return name.split("(")[0].replace("void ", "").replace("dmrgdev::", "")


def summarize_trace(d, bench_json, kernel):
    """Markdown summary of a `rocprofv3 --kernel-trace --stats` run of this
    benchmark: the kernel table, and the average duration of `kernel` over the
    timed sweeps (its last N dispatches, N from the benchmark's own line)."""
    b = json.loads([l for l in open(bench_json) if l.startswith("{")][-1])
    kernel = kernel or b["roofline"]["kernel"]
    n = int(b["roofline"]["launches"])
    stats = _csv_rows(_find(d, "kernel_stats.csv"))
    trace = _csv_rows(_find(d, "kernel_trace.csv"))
    sel = [r for r in trace if _short(r["Kernel_Name"]) == kernel]
    sel.sort(key=lambda r: int(r["Start_Timestamp"]))
    # the dispatches inside the timed sweeps' window, on whichever host clock
    # the trace's timestamps follow (the one whose window holds the launch count)
    best = None
    for clock, (w0, w1) in b["roofline"].get("timed_window_ns", {}).items():
        inside = [r for r in sel if int(r["Start_Timestamp"]) >= w0 and int(r["End_Timestamp"]) <= w1]
        if best is None or abs(len(inside) - n) < abs(len(best[1]) - n):
            best = (clock, inside)
    if best is None or not best[1]:
        raise SystemExit("no dispatch of the kernel inside the timed window")
    clock, last = best
    avg = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in last) / len(last)
    # device busy time in the window: the union of all kernels' intervals
    w0, w1 = b["roofline"]["timed_window_ns"][clock]
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in trace
                if int(r["Start_Timestamp"]) >= w0 and int(r["End_Timestamp"]) <= w1)
    busy, cs, ce = 0, None, None
    for s0, s1 in iv:
        if ce is None or s0 > ce:
            busy += (ce - cs) if ce is not None else 0
            cs, ce = s0, s1
        else:
            ce = max(ce, s1)
    busy += (ce - cs) if ce is not None else 0
    out = [f"- benchmark line: value {b['value']:.2f} {b['unit']}, ms_per_step {b['ms_per_step']:.0f}, "
           f"roofline.launch_ms {b['roofline']['launch_ms']:.4f} over {n} launches",
           f"- `{kernel}`: {len(sel)} dispatches in the run; {len(last)} inside the timed sweeps "
           f"(host {clock} clock window); their mean duration = {avg / 1e6:.4f} ms",
           f"- device busy inside the timed window (union of all kernel intervals): {busy / 1e9:.2f} s of "
           f"{(w1 - w0) / 1e9:.2f} s",
           "", "| kernel | calls | total s | avg us | % |", "|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:15]:
        out.append(f"| `{_short(r['Name'])[:70]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e9:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    print("\n".join(out))


def summarize_counters(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, bench_json, kernel, copy_mib):
    """HBM traffic per launch of `kernel` over the timed sweeps from two PMC
    runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by what the
    same counter reads for a plain copy of known size."""
    b = json.loads([l for l in open(bench_json) if l.startswith("{")][-1])
    n = int(b["roofline"]["launches"])   # both H_eff phases launch once per product and group
    kernel = kernel or b["roofline"]["kernel"]

    def per_dispatch(d, counter, match):
        rows = [r for r in _csv_rows(_find(d, "counter_collection.csv"))
                if r["Counter_Name"] == counter and match(_short(r["Kernel_Name"]))]
        by = {}
        for r in rows:
            k = int(r["Dispatch_Id"])
            by.setdefault(k, [int(r["Start_Timestamp"]), int(r["End_Timestamp"]), 0.0])
            by[k][2] += float(r["Counter_Value"])
        return sorted(by.values())

    def timed(disp):
        """the dispatches inside the timed sweeps (host clock window of the run's own line)"""
        best = None
        for w0, w1 in b["roofline"].get("timed_window_ns", {}).values():
            inside = [v for s0, s1, v in disp if s0 >= w0 and s1 <= w1]
            if best is None or abs(len(inside) - n) < abs(len(best) - n):
                best = inside
        if not best:
            # counter collection stamps dispatches on another clock: the run has
            # no check sweep and no CPU baseline (--no-check --no-cpu-baseline),
            # so the timed sweeps' launches are the kernel's last n
            return [v for _, _, v in disp[-n:]]
        return best

    fk = timed(per_dispatch(fetch_dir, "FETCH_SIZE", lambda s: s == kernel))
    wk = timed(per_dispatch(write_dir, "WRITE_SIZE", lambda s: s == kernel))
    cf = max(v for _, _, v in per_dispatch(copy_fetch_dir, "FETCH_SIZE",
                                           lambda s: "copy" in s.lower() or "elementwise" in s))
    cw = max(v for _, _, v in per_dispatch(copy_write_dir, "WRITE_SIZE",
                                           lambda s: "copy" in s.lower() or "elementwise" in s))
    kib = copy_mib * 1024.0
    sf, sw = kib / cf, kib / cw
    fetch = sum(fk) / len(fk) * 1024 * sf
    write = sum(wk) / len(wk) * 1024 * sw
    print(f"# {kernel}: HBM traffic per launch over the timed sweeps ({len(fk)} launches)")
    print(f"# copy reference: {copy_mib} MiB copy reads FETCH_SIZE {cf:.0f} KiB (scale {sf:.3f}), "
          f"WRITE_SIZE {cw:.0f} KiB (scale {sw:.3f})")
    rl = b["roofline"]
    ph = rl if kernel == rl["kernel"] else rl.get("other_phase", {})
    if ph.get("kernel", rl["kernel"]) == kernel:
        print(f"# algorithmic bytes per launch {ph['algorithmic_gb_per_launch'] * 1e9:.7g}")
    print(f"fetch_bytes_per_launch={fetch:.6g}")
    print(f"write_bytes_per_launch={write:.6g}")
    print(f"hbm_bytes_per_launch={fetch + write:.6g}")
    print(f"sources_sha256={source_sha()}")


def copy_reference(mib):
    import torch
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copied_bytes": a.numel() * 4}))


def hbm_check(mib: int, reps: int = 20):
    """The roofline denominators checked on the device: the CU count and
    clock the runtime reports, and the rate of a plain device-to-device copy
    of `mib` MiB (read + write bytes over the event-timed copy)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    clk = getattr(p, "clock_rate", None)
    print(json.dumps({"device": p.name, "gcn_arch": getattr(p, "gcnArchName", None),
                      "compute_units": p.multi_processor_count, "clock_khz": clk,
                      "copy_mib": mib, "copy_s": s, "copy_read_write_gb_s": 2 * a.numel() * 4 / s / 1e9}))


def batched(k: int, precision: str = "fp32"):
    """Independent small solves: the first k seeded instances (p / sd / pf
    spaces, 2..8 particles per species, D from 64..512), one sweep each at
    their D, first one at a time, then all together with dmrg_sweep_many
    (fresh contexts, same inputs)."""
    import paper_1507_00161_amd as pk
    import torch
    from workloads import batched_instances
    ws = batched_instances(k)

    def make(w, group=1):
        h = w.hamiltonian()
        sp = h.space
        c = pk.Context(precision=PREC[precision], davidson_tol=1e-7, noise=1e-4, noise_sweeps=1, seed=1507,
                       group_products=group)
        c.load_hamiltonian(sp.species, sp.two_m, h.eps, h.V.ravel(), h.n_p, h.n_n, h.two_M)
        return c

    ctxs = [make(w) for w in ws]
    torch.cuda.synchronize()
    t = time.perf_counter()
    e_seq = [c.sweep(w.D_schedule[0])["energy"] for c, w in zip(ctxs, ws)]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    for c in ctxs:
        c.close()
    ctxs = [make(w) for w in ws]
    torch.cuda.synchronize()
    t = time.perf_counter()
    st, out = pk.sweep_many(ctxs, [w.D_schedule[0] for w in ws])
    torch.cuda.synchronize()
    t_con = time.perf_counter() - t
    for c in ctxs:
        c.close()
    # the same call with every context launching its own products on its own stream
    ctxs = [make(w, 0) for w in ws]
    torch.cuda.synchronize()
    t = time.perf_counter()
    st_ind, out_ind = pk.sweep_many(ctxs, [w.D_schedule[0] for w in ws])
    torch.cuda.synchronize()
    t_ind = time.perf_counter() - t
    for c in ctxs:
        c.close()
    diff_ind = max(abs(o["energy"] - e) / abs(e) for o, e in zip(out_ind, e_seq))
    diff = max(abs(o["energy"] - e) / abs(e) for o, e in zip(out, e_seq))
    flops = sum(o["heff_flops"] for o in out)
    # against the oracle's first-sweep energies of the instances it has
    vo = None
    try:
        g = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_batched.json")))
        if g["options"] == {"davidson_tol": 1e-7, "noise": 1e-4, "noise_sweeps": 1, "seed": 1507}:
            rel = [abs(out[int(i)]["energy"] - v["energy"]) / abs(v["energy"])
                   for i, v in g["instances"].items() if int(i) < k]
            vo = {"instances": len(rel), "rel_max": max(rel) if rel else None}
    except OSError:
        pass
    res = {"batched": {"instances": k, "precision": precision, "status": st,
                       "sequential_s": t_seq, "concurrent_s": t_con, "speedup": t_seq / t_con,
                       "independent_streams_s": t_ind, "independent_max_rel_energy_diff": diff_ind,
                       "heff_gflop_total": flops / 1e9, "heff_tflops_over_wall": flops / t_con / 1e12,
                       "max_rel_energy_diff": diff, "vs_oracle": vo,
                       "spaces": [w.space for w in ws], "D": [w.D_schedule[0] for w in ws]}}
    print(json.dumps(res))


ORACLE_SCHEDULE = os.path.join(ROOT, "tests", "golden", "oracle_bench_schedule.json")


def vs_oracle(res, wl, args):
    """Sweep energies of the GPU runs against the oracle's on the same
    schedule and options (tests/golden/oracle_bench_schedule.json, written by
    the oracle alone), for the sweeps the oracle has."""
    try:
        g = json.load(open(ORACLE_SCHEDULE))
    except OSError:
        return None
    ramp = list(wl.D_schedule)
    sched = [ramp[w] if w < len(ramp) else args.D for w in range(args.warmup)] + [args.D] * args.steps
    o = g["options"]
    if (o["davidson_tol"] != args.tol or o["seed"] != 1507 or o["noise"] != 1e-4 or o["noise_sweeps"] != 2
            or g["workload"] != "pf_8p8n"):
        return None
    n = 0
    while n < min(len(sched), len(g["D"])) and sched[n] == g["D"][n]:
        n += 1
    if n == 0:
        return None
    out = {"sweeps": n, "D": sched[:n], "oracle_energies": g["energies"][:n]}
    for p, r in res.items():
        rel = [abs(a - b) / abs(b) for a, b in zip(r["energies"][:n], g["energies"][:n])]
        out[p] = {"rel": rel, "rel_max": max(rel)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed sweeps at D=2048")
    ap.add_argument("--warmup", type=int, default=4, help="warm-up sweeps of the D ramp")
    ap.add_argument("--precisions", default="fp64,fp32")
    ap.add_argument("--D", type=int, default=2048)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the FP64 re-solve sweep of the mixed run")
    ap.add_argument("--summarize-trace", metavar="DIR", help="summarise a rocprofv3 kernel-trace run")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="HBM traffic from rocprofv3 --pmc runs of this benchmark and of --copy-reference")
    ap.add_argument("--bench-json", help="the benchmark line of the profiled run")
    ap.add_argument("--kernel", help="kernel to summarise (default: the benchmark line's roofline kernel)")
    ap.add_argument("--copy-reference", type=int, metavar="MIB", help="one plain device copy of MIB MiB")
    ap.add_argument("--hbm-check", type=int, metavar="MIB",
                    help="CU count, clock and the rate of a timed device copy of MIB MiB")
    ap.add_argument("--plateaus", metavar="WORKLOAD",
                    help="energy vs discarded weight along --D-list plateaus (--per sweeps each)")
    ap.add_argument("--D-list", default="512,1024,2048")
    ap.add_argument("--per", type=int, default=2)
    ap.add_argument("--trunc-eps", type=float, default=0.0, help="plateaus: DBSS truncation error (0 = fixed D)")
    ap.add_argument("--d-min", type=int, default=0, help="plateaus: DBSS minimum block states")
    ap.add_argument("--n-states", type=int, default=1, help="plateaus: 2 = the two lowest states at once")
    ap.add_argument("--preprocess", metavar="WORKLOAD",
                    help="measuring sweeps at --D-pre, Fiedler ordering, then --D-list plateaus in both orders")
    ap.add_argument("--D-pre", type=int, default=256)
    ap.add_argument("--sweeps-pre", type=int, default=2)
    ap.add_argument("--converge", metavar="WORKLOAD",
                    help="at each --D-list value, sweep until |dE| < 1e-4 MeV between sweeps; then E(M) fit")
    ap.add_argument("--max-sweeps", type=int, default=60, help="converge: most sweeps per D")
    ap.add_argument("--budget-s", type=float, default=300.0, help="converge: most seconds per D")
    ap.add_argument("--batched", type=int, metavar="K",
                    help="independent small solves: K instances one at a time vs dmrg_sweep_many")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.bench_json, args.kernel)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.bench_json, args.kernel, args.copy_reference or 256)
        return
    if args.copy_reference:
        copy_reference(args.copy_reference)
        return
    if args.hbm_check:
        hbm_check(args.hbm_check)
        return
    if args.batched:
        batched(args.batched)
        return
    if args.preprocess:
        for p in args.precisions.split(","):
            preprocess(args.preprocess, p, args.D_pre, args.sweeps_pre, [int(x) for x in args.D_list.split(",")],
                       args.per, args.tol)
        return
    if args.converge:
        got = {}
        for p in [x.strip() for x in args.precisions.split(",") if x.strip()]:
            got[p] = converge(args.converge, p, [int(x) for x in args.D_list.split(",")], args.max_sweeps,
                              args.budget_s, args.tol)
        if "fp64" in got:
            for p, g in got.items():
                if p == "fp64":
                    continue
                cmp = {D: abs(v["energy"] - got["fp64"][D]["energy"]) / abs(got["fp64"][D]["energy"])
                       for D, v in g.items() if v["met"] and got["fp64"][D]["met"]}
                print(json.dumps({"mode": "converged_vs_fp64", "precision": p, "rel": cmp}), flush=True)
        return
    if args.plateaus:
        for p in [x.strip() for x in args.precisions.split(",") if x.strip()]:
            plateaus(args.plateaus, p, [int(x) for x in args.D_list.split(",")], args.per, args.tol,
                     args.trunc_eps, args.d_min, args.n_states)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU; the multi-GPU path (term-sharded H_eff with an "
              "all-reduce of H_eff.psi) is designed but not built, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from workloads import WORKLOADS
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    wl = WORKLOADS["pf_8p8n"]
    precs = [p.strip() for p in args.precisions.split(",") if p.strip()]
    res = {}
    for p in precs:
        res[p] = run_schedule(wl, p, args.warmup, args.steps, args.D, seed=1507, tol=args.tol,
                              check=not args.no_check)
    main_p = "fp32" if "fp32" in res else precs[-1]
    R = res[main_p]
    t = R["tot"]
    value = t["heff_flops"] / max(t["heff_seconds"], 1e-12) / 1e12
    # dominant kernel: the GEMM phase with the larger device time
    k = "gemm2" if t["gemm2_seconds"] >= t["gemm1_seconds"] else "gemm1"
    nl = max(t[f"{k}_launches"], 1)
    kdt = t[f"{k}_seconds"] / nl
    kfl = t[f"{k}_flops"] / nl
    achieved = kfl / max(kdt, 1e-12) / 1e12
    kiss = t[f"{k}_issued_flops"] / nl
    ctype = {"fp64": "double, double, 16", "fp32": "float, float, 32"}.get(main_p, "")
    kname = f"{'k_heff_y' if k == 'gemm2' else 'k_heff_z'}<{ctype}>" if ctype else "k_gemm_bf16"
    traffic = measured_traffic(kname, t[f"{k}_bytes"] / nl)
    ko = "gemm1" if k == "gemm2" else "gemm2"   # the other H_eff phase, for reference
    nlo = max(t[f"{ko}_launches"], 1)
    oname = f"{'k_heff_y' if ko == 'gemm2' else 'k_heff_z'}<{ctype}>" if ctype else "k_gemm_bf16"
    out = {
        "metric": "Davidson H_eff·psi TFLOP/s + sweep time at D=2048, mixed vs FP64, |dE|<1e-6",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sum(R["walls"]) / len(R["walls"]),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[main_p],
        "data": "synthetic",
        "config": {"workload": "pf_8p8n: pf shell, 40 sites, 8p+8n, 2M=0, random eps/Vbar seed 150703, "
                               f"natural order, D ramp 512,512,1024,1024 then D={args.D}",
                   "D": args.D, "precision": main_p, "davidson_tol": args.tol},
        "roofline": {"bound": "mfma", "kernel": kname,
                     "achieved": achieved, "peak": PEAK[main_p], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[main_p], "traffic": traffic,
                     "launch_ms": 1e3 * kdt, "launches": int(t[f"{k}_launches"]),
                     "algorithmic_gflop_per_launch": kfl / 1e9,
                     "issued_gflop_per_launch": kiss / 1e9,
                     "algorithmic_gb_per_launch": t[f"{k}_bytes"] / nl / 1e9,
                     "split_k_reduce_ms_per_launch": 1e3 * t.get("reduce_seconds", 0.0) / nl,
                     "other_phase": {"kernel": oname, "launch_ms": 1e3 * t[f"{ko}_seconds"] / nlo,
                                     "algorithmic_gflop_per_launch": t[f"{ko}_flops"] / nlo / 1e9,
                                     "issued_gflop_per_launch": t[f"{ko}_issued_flops"] / nlo / 1e9,
                                     "algorithmic_gb_per_launch": t[f"{ko}_bytes"] / nlo / 1e9},
                     "timed_window_ns": R["window"]},
        "flop_counts": {"value_counts": "algorithmic: per term and psi block the cheaper of the two "
                                        "contraction orders, nonzero sub-blocks, intermediates formed once",
                        "algorithmic_gflop": t["heff_flops"] / 1e9,
                        "executed_gflop": t["heff_flops_executed"] / 1e9,
                        "executed_tflops": t["heff_flops_executed"] / max(t["heff_seconds"], 1e-12) / 1e12},
    }
    for p, r in res.items():
        tt = r["tot"]
        out[f"{p}_run"] = {"energy": r["energy"], "ms_per_sweep": 1e3 * sum(r["walls"]) / len(r["walls"]),
                           "heff_tflops": tt["heff_flops"] / max(tt["heff_seconds"], 1e-12) / 1e12,
                           "products_low": int(tt["products_low"]), "products_fp64": int(tt["products_fp64"]),
                           "heff_seconds": tt["heff_seconds"],
                           "delta_E_MeV_timed": [None if math.isnan(x) else x for x in r["deltas"]],
                           "paper_sweep_criterion_met": bool(r["deltas"]) and abs(r["deltas"][-1]) < SWEEP_CRIT_MEV}
        # (a NaN delta, the first sweep after the blocks were set up, compares False)
    if "fp64" in res and main_p != "fp64":
        e64, em = res["fp64"]["energy"], R["energy"]
        # sweep by sweep along the two trajectories (same schedule, same start)
        rel = [abs(a - b) / abs(b) for a, b in zip(R["energies"], res["fp64"]["energies"])]
        nt = args.steps
        par = {"trajectory_rel_last": abs(em - e64) / abs(e64),
               "trajectory_rel_max_timed": max(rel[-nt:]),
               "trajectory_rel_max_all": max(rel),
               "trajectory_MeV_last": em - e64,
               "note": "trajectory_*: the mixed and the FP64 GPU runs of the same schedule, sweep by sweep "
                       "(both truncated and unconverged, so they keep slightly different states)"}
        if R["check"]:
            par["fixed_heff_rel_max"] = R["check"]["max_rel"]
            par["fixed_heff_solves"] = R["check"]["solves"]
            par["fixed_heff_note"] = ("one extra sweep after the timed ones: at every bond the mixed solve "
                                      "and an FP64 solve from the same guess on the same H_eff")
        out["parity"] = par
        out["sweep_speedup_vs_fp64"] = out["fp64_run"]["ms_per_sweep"] / out[f"{main_p}_run"]["ms_per_sweep"]
    vo = vs_oracle(res, wl, args)
    if vo:
        out.setdefault("parity", {})["vs_oracle"] = vo
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
