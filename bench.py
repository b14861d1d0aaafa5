"""Benchmark of the elastic Helmholtz hot path on one MI355X.

One step = one pass of the whole path on one batch of synthetic input that is
already resident in HBM: operator setup (coefficients, Galerkin hierarchy,
coarsest inverse) + the preconditioned FGMRES solve of every right-hand side to
relative residual 1e-6 + release.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E


def rhs_tensor(S, w):
    import torch
    nrhs = len(w.sources())
    B = np.zeros((nrhs, 2 * S.N))
    # unknown index of a face/cell in the library layout (x fastest per component)
    n = list(w.n) + [1] * (3 - len(w.n))
    offs = np.concatenate([[0], np.cumsum(S.counts)])
    for r, (comp, pos, amp) in enumerate(w.sources()):
        dims = [n[a] - (1 if a == comp else 0) for a in range(3)]
        c = [pos[a] - (1 if a == comp else 0) for a in range(len(pos))] + [0] * (3 - len(pos))
        idx = offs[comp] + c[0] + dims[0] * (c[1] + dims[1] * c[2])
        B[r, idx] += amp.real
        B[r, S.N + idx] += amp.imag
    return torch.as_tensor(B, device="cuda")


def run_gpu(w, steps, warmup, tol, tune=True):
    import torch
    from paper_1806_11277_amd import ehh, tuning
    m = w.media()
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    lam, mu, rho = dev(m["lam"]), dev(m["mu"]), dev(m["rho"])
    opts = dict(levels=w.levels, cycle=w.cycle, cycle_level=w.cycle_level, nu1=w.nu1, nu2=w.nu2, vanka=w.vanka,
                precond_bits=w.precond_bits, restart=w.restart, dd_parts=w.dd_parts,
                dd_overlap=w.dd_overlap, dd_pad=w.dd_pad, dd_colors=w.dd_colors, damping=w.damping,
                abl_max=w.abl_max, atten0=w.atten0, coarse_bits=w.coarse_bits,
                coarse_dd_parts=w.coarse_dd_parts, coarse_dd_overlap=w.coarse_dd_overlap,
                coarse_dd_colors=w.coarse_dd_colors, damping_p=w.damping_p)

    def make():
        return ehh.Solver(w.dim, w.n, w.h, w.omega, w.shift, w.abl_cells, lam, mu, rho, **opts)

    S0 = make()
    B = rhs_tensor(S0, w)
    X = torch.zeros_like(B)
    # launch shapes: the autotuner's table for this configuration (untimed; from
    # the cache when an earlier run stored it), installed in every step's solver
    table, how = tuning.tune(S0, B.shape[0]) if tune else (None, "heuristic")
    S0.close()
    torch.cuda.synchronize()
    results = []

    def step():
        t0 = time.perf_counter()
        S = make()
        if table is not None:
            S.set_tuning(table)
        t1 = time.perf_counter()
        st, stats = S.solve(B, X, tol=tol, maxit=w.maxit)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        S.close()
        results.append((t1 - t0, t2 - t1, st, stats))
        print(f"[bench] step: setup {1e3 * (t1 - t0):.1f} ms, solve {1e3 * (t2 - t1):.1f} ms, "
              f"iters {[s_['iters'] for s_ in stats][:4]}", file=sys.stderr, flush=True)

    for _ in range(warmup):
        step()
    results.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return total, results, B, X, {"source": how, "table": table}


KERNEL_SOURCES = ["paper_1806_11277_amd/csrc/levels.hip", "paper_1806_11277_amd/csrc/ops.hpp",
                  "paper_1806_11277_amd/csrc/common.hpp", "paper_1806_11277_amd/csrc/setup.hip",
                  "paper_1806_11277_amd/csrc/dd.hip", "paper_1806_11277_amd/csrc/launchlog.hpp"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(workload, kernel):
    """HBM bytes per launch of a kernel from the committed counter summaries
    (FETCH_SIZE and WRITE_SIZE runs scaled by a plain copy's reading), or None
    when there is none or the kernel sources changed since it was taken."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    for f in sorted(os.listdir(d)):
        if not f.endswith(".md"):
            continue
        for line in open(os.path.join(d, f)):
            if line.startswith("traffic-record: "):
                rec = json.loads(line[len("traffic-record: "):])
                if rec.get("workload") == workload and rec.get("kernel") == kernel:
                    if rec.get("source_hash") != kernel_source_hash():
                        return None
                    return rec
    return None


def cycle_profile(w, reps=5, table=None):
    """Every kernel of one preconditioner application, timed live on this
    stream: the library records the launches of a real application
    (ehh_profile_precondition) and replays them with their arguments.  The
    primary figure (avg_us_seq) replays the whole application in order, each
    launch timed by start / stop events its own dispatch records
    (hipExtLaunchKernel): no launch gaps, and every kernel finds the caches as
    the preceding kernels left them, as inside a solve.  Two bounds come with
    it: each kernel's launches from a HIP graph after a 512 MiB write that
    evicts the L2s and the MALL (its own time subtracted; cold), and back to
    back (warm, which includes launch gaps).  The dominant kernel is the one
    with the largest time per application."""
    import torch
    from paper_1806_11277_amd import ehh
    S = ehh.solver_for_workload(w)
    if table is not None:
        S.set_tuning(table)
    nrhs = len(w.sources())
    g = torch.Generator(device="cuda").manual_seed(5)
    v = torch.randn((nrhs, S.stride), dtype=torch.float64, device="cuda", generator=g)
    v /= v.norm(dim=1, keepdim=True)
    z = torch.zeros_like(v)
    evict = torch.empty(64 * 2 ** 20, dtype=torch.float64, device="cuda")   # 512 MiB
    rows = S.profile_precondition(v, z, reps=reps, evict=evict)
    torch.cuda.synchronize()
    del evict, v, z
    S.close()
    for r in rows:
        r["avg_us_cold"] = r.pop("avg_us")
        t = r["avg_us_seq"]
        r["us_per_application"] = r["launches"] * t
        r["gbs"] = r["bytes"] / t / 1e3 if t > 0 else None
        r["gbs_model"] = r["bytes_model"] / t / 1e3 if t > 0 else None
    rows.sort(key=lambda r: -r["us_per_application"])
    tot_t = sum(r["us_per_application"] for r in rows)
    tot_b = sum(r["launches"] * r["bytes"] for r in rows)
    tot_bm = sum(r["launches"] * r["bytes_model"] for r in rows)
    return dict(kernels=rows, us_per_application=tot_t, gbs=tot_b / tot_t / 1e3,
                gbs_model=tot_bm / tot_t / 1e3)


def roofline(w, prof, copy_gbs):
    """The roofline object of the dominant kernel of a cycle profile."""
    dom = prof["kernels"][0]
    rec = traffic_record(w.name, dom["kernel"])
    return {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["gbs"], "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": dom["gbs"] / PEAK_HBM_GBS,
            "traffic": (rec["hbm_bytes_per_launch"] if rec else None),
            "traffic_unit": "HBM bytes per launch (counters scaled by a plain copy)",
            "bytes_per_launch": dom["bytes"], "avg_launch_us": dom["avg_us_seq"],
            "timing": "in-order replay of one application, each launch between its own dispatch's start and "
                      "stop events (hipExtLaunchKernel); cold: after a 512 MiB cache-evicting write; warm: "
                      "graph replay back to back (includes launch gaps)",
            "avg_launch_us_cold": dom["avg_us_cold"], "avg_launch_us_warm": dom["avg_us_warm"],
            "achieved_cold": dom["bytes"] / dom["avg_us_cold"] / 1e3 if dom["avg_us_cold"] > 0 else None,
            "achieved_warm": dom["bytes"] / dom["avg_us_warm"] / 1e3 if dom["avg_us_warm"] > 0 else None,
            "launches_per_application": dom["launches"],
            "share_of_application": dom["us_per_application"] / prof["us_per_application"],
            "achieved_model_bytes": dom["gbs_model"], "frac_model_bytes": dom["gbs_model"] / PEAK_HBM_GBS,
            "bytes_model_per_launch": dom["bytes_model"],
            "copy_gbs": copy_gbs, "frac_of_copy": dom["gbs"] / copy_gbs,
            "application": {"us": prof["us_per_application"], "gbs": prof["gbs"], "gbs_model": prof["gbs_model"],
                            "frac": prof["gbs"] / PEAK_HBM_GBS},
            "kernels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                        for r in prof["kernels"]]}


def copy_bandwidth(mib=1024, reps=10):
    """Achievable device bandwidth for context: a plain 1 GiB device-to-device
    copy (read + write bytes over the best of `reps` timed copies)."""
    import torch
    src = torch.ones(mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    del src, dst
    return 2 * mib * 2 ** 20 / best / 1e9


def cpu_baseline(w):
    """The oracle on this host: its direct solve (sparse LU of the assembled
    operator of eq. (14) on the nested-dissection order, then one forward and
    back substitution per source) of the workload's sources, the factorisation
    and per-source times reported apart.  SuperLU runs on one core.  Returns
    the baseline record and the factorisation (reused for the errors)."""
    from oracle import direct
    from oracle import discretisation as disc
    try:
        from threadpoolctl import threadpool_info
        blas = sum(i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas")
    except Exception:  # pragma: no cover
        blas = None
    m = w.media()
    t0 = time.perf_counter()
    pb = disc.Problem(w.n, w.h, w.omega, m["lam"], m["mu"], m["rho"], w.abl_cells, w.abl_max,
                      w.atten0, shift=w.shift)
    lu = direct.factorize(pb)
    t1 = time.perf_counter()
    srcs = w.sources()
    sol = [lu.solve(disc.point_source_vector(w.n, [s_])) for s_ in srcs]
    t2 = time.perf_counter()
    per_source = (t2 - t1) / len(srcs)
    total = t2 - t0
    rec = dict(value=len(srcs) / total, unit="solves/s", cores=1, kind="oracle",
               sample=f"oracle direct solve of {w.name}: assembly + sparse LU ({t1 - t0:.1f} s, "
                      f"{lu.nnz:.2e} nonzeros in L+U) + {len(srcs)} substitution(s) ({per_source:.2f} s each), "
                      f"whole, not extrapolated",
               factor_s=t1 - t0, per_source_s=per_source,
               host_cores=len(os.sched_getaffinity(0)), blas_threads=blas,
               threads_used="1 (SuperLU is sequential)")
    return rec, lu, sol


def errors_vs_oracle(w, X, lu):
    """Relative 2-norm error of every source's solution against the oracle's
    direct solution of the same operator (the operator of c2 and c3 is the
    same: the factorisation is shared)."""
    from oracle import discretisation as disc
    x = X.double().cpu().numpy()
    N = x.shape[1] // 2
    out = []
    for r, s_ in enumerate(w.sources()):
        ref = lu.solve(disc.point_source_vector(w.n, [s_]))
        got = x[r, :N] + 1j * x[r, N:]
        out.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    return out


def poisson_sweep_report():
    """Preconditioning cycles to 1e-6 for constant mu = rho = 1 and lambda from 0.5
    to 16 (section 6, Fig. 5), full and economic Vanka, on 256x128, 512x256 and
    1024x512 (its coarsest level solved by DD), and Table 2's rows (lambda = 16,
    constant against component damping)."""
    import torch
    from paper_1806_11277_amd import ehh
    from workloads.configs import poisson_sweep, SWEEP_LAMBDAS, SWEEP_GRIDS, SWEEP_COARSE_DD

    def iters(w):
        S = ehh.solver_for_workload(w)
        b = rhs_tensor(S, w)
        x = torch.zeros_like(b)
        st, stats = S.solve(b, x, tol=1e-6, maxit=600)
        torch.cuda.synchronize()
        S.close()
        print(f"[sweep] {w.name}: {stats[0]['iters'] if st == 0 else None}", file=sys.stderr, flush=True)
        return stats[0]["iters"] if st == 0 else None

    out = {"experiment": "Poisson-ratio sweep, constant mu = rho = 1", "lambda": list(SWEEP_LAMBDAS), "grids": [],
           "table2": []}
    for nx in (256, 512, 1024):
        row = {"cells": [nx, nx // 2], "omega_over_pi": 3 * nx // 256, "levels": SWEEP_GRIDS[nx][0],
               "shift": SWEEP_GRIDS[nx][1], "coarse_dd_parts": list(SWEEP_COARSE_DD.get(nx, ((1, 1, 1), 0))[0][:2]),
               "coarse_dd_overlap": SWEEP_COARSE_DD.get(nx, ((1, 1, 1), 0))[1]}
        for vanka, key in ((1, "full_vanka"), (0, "economic_vanka")):
            row[key] = [iters(poisson_sweep(nx, lam, vanka)) for lam in SWEEP_LAMBDAS]
        out["grids"].append(row)
        out["table2"].append({"cells": [nx, nx // 2], "red_black_constant_0.75": iters(poisson_sweep(nx, 16.0, 1)),
                              "red_black_component_0.85_0.65": iters(poisson_sweep(nx, 16.0, 1, "component"))})
    return out


def accuracy_solve(w, tol, table=None):
    """One more (untimed) solve of the workload's sources to a tighter relative
    residual, for the errors against the oracle at that residual."""
    import torch
    from paper_1806_11277_amd import ehh
    S = ehh.solver_for_workload(w)
    if table is not None:
        S.set_tuning(table)
    B = rhs_tensor(S, w)
    X = torch.zeros_like(B)
    st, stats = S.solve(B, X, tol=tol, maxit=4 * w.maxit)
    torch.cuda.synchronize()
    S.close()
    return X, max(s_["rel_res_true"] for s_ in stats), [s_["iters"] for s_ in stats]


def workload_entry(w, steps, warmup, tol, copy_gbs, with_profile, tune=True):
    """Time `steps` steps of a workload (after `warmup`), with its cycle profile."""
    total, res, B, X, tuned = run_gpu(w, steps, warmup, tol, tune)
    stats = res[-1][3]
    iters = [s_["iters"] for s_ in stats]
    out = {"workload": w.name, "nrhs": len(stats), "value": len(stats) * steps / total, "unit": "solves/s",
           "ms_per_step": 1e3 * total / steps, "steps": steps,
           "setup_ms": 1e3 * float(np.mean([r[0] for r in res])),
           "solve_ms": 1e3 * float(np.mean([r[1] for r in res])),
           "iters": iters if len(iters) <= 4 else [min(iters), max(iters)],
           "rel_res_true_max": max(s_["rel_res_true"] for s_ in stats), "status": res[-1][2],
           "dtype": "f64" if w.precond_bits == 64 else "f32 cycle + f64 Krylov/coarsest",
           "launch_shapes": tuned}
    if with_profile:
        print(f"[bench] cycle profile {w.name}", file=sys.stderr, flush=True)
        out["roofline"] = roofline(w, cycle_profile(w, table=tuned["table"]), copy_gbs)
    return out, X


def profile_solves(w, solves, tune=True):
    """Solves alone, for kernel traces: the solver is set up and tuned, solves
    once (warm-up), then a short spin kernel (torch.cuda._sleep) marks the start
    of `solves` solves of the workload's sources and another their end; the
    dispatches between the two markers in a trace are the solves' only.  The
    cycle profile (HIP events around replays, the figures of the bench line)
    follows the second marker."""
    import torch
    from paper_1806_11277_amd import ehh, tuning
    S = ehh.solver_for_workload(w)
    B = rhs_tensor(S, w)
    table, how = tuning.tune(S, B.shape[0]) if tune else (None, "heuristic")
    X = torch.zeros_like(B)
    S.solve(B, X, tol=1e-6, maxit=w.maxit)
    torch.cuda.synchronize()
    torch.cuda._sleep(1000)
    torch.cuda.synchronize()
    per = []
    for _ in range(solves):
        X.zero_()
        t0 = time.perf_counter()
        st, stats = S.solve(B, X, tol=1e-6, maxit=w.maxit)
        torch.cuda.synchronize()
        per.append(1e3 * (time.perf_counter() - t0))
    torch.cuda._sleep(1000)
    torch.cuda.synchronize()
    S.close()
    prof = cycle_profile(w, table=table)
    dom = prof["kernels"][0]
    return {"workload": w.name, "solves": solves, "solve_ms": per, "iters": [s_["iters"] for s_ in stats],
            "launch_shapes": {"source": how, "table": table},
            "cycle_us": prof["us_per_application"],
            "cycle_kernels": [{k: r[k] for k in ("kernel", "launches", "avg_us_seq", "avg_us_cold", "avg_us_warm",
                                                 "bytes", "bytes_model")}
                              for r in prof["kernels"]],
            "dominant": dom["kernel"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2_hetero512_fp64")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (its direct solve is also the reference of the errors)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--companions", default="c3_hetero512_batch32_fp32,c4_layered128_dd8_batch16_fp32",
                    help="comma-separated workloads reported in the same line ('' for none)")
    ap.add_argument("--companion-steps", type=int, default=2)
    ap.add_argument("--accuracy-tol", type=float, default=1e-8,
                    help="relative residual of an extra untimed solve per workload whose error against "
                         "the oracle is reported beside the error at --tol (0: none)")
    ap.add_argument("--poisson-sweep", action="store_true",
                    help="print the Poisson-ratio sweep (constant media, lambda 0.5..16) as one JSON line and exit")
    ap.add_argument("--coarse-bits", type=int, default=None, choices=(16, 32),
                    help="storage of the 3D Galerkin levels' stored rows in the complex64 cycle "
                         "(16: FP16 with a power-of-two scale per level)")
    ap.add_argument("--profile-solves", type=int, default=0,
                    help="for kernel traces: set up once, then time this many solves of --config between two "
                         "marker kernels and print their record as one JSON line (no bench line)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the heuristic launch shapes instead of the autotuner's (cached) table")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for traffic counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver runs all subdomains and right-hand sides "
              "on a single device; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import dataclasses
    import torch
    from workloads import get_config
    if a.poisson_sweep:
        print(json.dumps(poisson_sweep_report()), flush=True)
        return
    if a.calibrate_copy:
        src = torch.ones(256 * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = get_config(a.config)
    if a.coarse_bits is not None:
        w = dataclasses.replace(w, coarse_bits=a.coarse_bits)
    if a.profile_solves > 0:
        print(json.dumps(profile_solves(w, a.profile_solves, not a.no_tune)), flush=True)
        return
    copy_gbs = None if a.no_roofline else copy_bandwidth()
    print(f"[bench] {w.name}: n={w.n} nrhs={len(w.sources())} levels={w.levels} cycle={w.cycle} "
          f"bits={w.precond_bits}", file=sys.stderr, flush=True)
    main_e, X = workload_entry(w, a.steps, a.warmup, a.tol, copy_gbs, False, not a.no_tune)
    table = main_e["launch_shapes"]["table"]
    out = {
        "metric": "preconditioned solves/sec at rel. residual 1e-6; V-cycle HBM GB/s vs peak",
        "value": main_e["value"],
        "unit": "solves/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": main_e["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w.precond_bits == 64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.n), "unknowns": int(X.shape[1] // 2),
                   "nrhs": main_e["nrhs"], "levels": w.levels, "cycle": "V" if w.cycle == 1 else "W",
                   "cycle_level": w.cycle_level,
                   "nu": [w.nu1, w.nu2], "vanka": "full" if w.vanka else "economic",
                   "shift": w.shift, "precond_bits": w.precond_bits, "restart": w.restart,
                   "dd_parts": list(w.dd_parts[:w.dim]), "coarse_bits": w.coarse_bits, "tol": a.tol},
        "setup_ms": main_e["setup_ms"], "solve_ms": main_e["solve_ms"],
        "iters": main_e["iters"], "rel_res_true_max": main_e["rel_res_true_max"], "status": main_e["status"],
        "launch_shapes": main_e["launch_shapes"],
    }
    results = {w.name: (w, X, None)}
    if a.accuracy_tol > 0 and not a.no_cpu_baseline:
        results[w.name] = (w, X, accuracy_solve(w, a.accuracy_tol, table))
    if not a.no_roofline:
        print(f"[bench] cycle profile {w.name}", file=sys.stderr, flush=True)
        rl = roofline(w, cycle_profile(w, table=table), copy_gbs)
        out["roofline"] = {k: v for k, v in rl.items() if k != "kernels"}
        out["cycle_kernels"] = rl["kernels"]
    comps = [c for c in a.companions.split(",") if c]
    out["companions"] = []
    for name in comps:
        wc = get_config(name)
        if a.coarse_bits is not None:
            wc = dataclasses.replace(wc, coarse_bits=a.coarse_bits)
        print(f"[bench] companion {wc.name}", file=sys.stderr, flush=True)
        e, Xc = workload_entry(wc, a.companion_steps, 1, a.tol, copy_gbs, not a.no_roofline, not a.no_tune)
        e["speedup_vs_plain_fp64_single_source"] = e["value"] / out["value"]
        out["companions"].append(e)
        acc = accuracy_solve(wc, a.accuracy_tol, e["launch_shapes"]["table"]) if (a.accuracy_tol > 0 and not a.no_cpu_baseline and
                                                    wc.dim == 2) else None
        results[wc.name] = (wc, Xc, acc)
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline: the oracle's direct solve", file=sys.stderr, flush=True)
        base, lu, _ = cpu_baseline(w)
        out["cpu_baseline"] = base
        # errors against the oracle's direct solution, for every workload on this operator
        out["err_vs_oracle"] = {}
        for name, (wk, Xk, acc) in results.items():
            same = wk.dim == w.dim and tuple(wk.n) == tuple(w.n) and wk.media_fn is not None and \
                wk.h == w.h and abs(wk.omega - w.omega) < 1e-12 * w.omega and wk.abl_cells == w.abl_cells and \
                wk.atten0 == w.atten0 and np.array_equal(wk.media()["mu"], w.media()["mu"]) and \
                np.array_equal(wk.media()["lam"], w.media()["lam"]) and np.array_equal(wk.media()["rho"], w.media()["rho"])
            if same:
                errs = errors_vs_oracle(wk, Xk, lu)
                rec = {"tol": a.tol, "per_source": errs, "max": max(errs),
                       "reference": "oracle direct solve (sparse LU)"}
                if acc is not None:
                    ea = errors_vs_oracle(wk, acc[0], lu)
                    rec["at_accuracy_tol"] = {"tol": a.accuracy_tol, "per_source": ea, "max": max(ea),
                                              "rel_res_true_max": acc[1], "iters": [min(acc[2]), max(acc[2])]}
                out["err_vs_oracle"][name] = rec
            else:
                out["err_vs_oracle"][name] = {"per_source": None, "max": None,
                                              "reference": "parity unpinned at this size: no direct solve of "
                                                           "this operator fits the host; the configuration is "
                                                           "compared with the oracle at 32^3 and 16^3 and a "
                                                           "full-size subdomain cycle in the tests"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
