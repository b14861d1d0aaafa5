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


def level_bytes(info, bits, nrhs, fine, dim, with_e=True, coef_bytes=None):
    """Algorithmic HBM bytes of one half-sweep launch on a level: b and e_in read,
    e_out written (every unknown, complex, per right-hand side; without e_in when
    the sweep starts from zero) plus the level's operator coefficients read once
    (finest: mu, 1/(lambda+mu), rho, gamma per cell; coarser: the stored
    Galerkin stencil, at coef_bytes per real when the level keeps its
    coefficients in another precision than the cycle's)."""
    es = 4 if bits == 32 else 8
    ncell_ = int(np.prod(info["n"][:dim]))
    nu = info["N"] - ncell_          # displacement unknowns
    # b: the rows of the colour's cells (every face, half the pressures);
    # e_in: every unknown the rows touch; e_out: every unknown
    vec = ((nu + ncell_ / 2) + (info["N"] if with_e else 0) + info["N"]) * 2 * es * nrhs
    ncell = int(np.prod(info["n"][:dim]))
    if fine:
        coef = 4 * ncell * es
    else:
        nuu, nup = (8, 6) if dim == 2 else (38, 18)
        coef = (sum(info["counts"][:dim]) * (2 * nuu + nup) + ncell) * (coef_bytes or es)
    return vec + coef


def run_gpu(w, steps, warmup, tol):
    import torch
    from paper_1806_11277_amd import ehh
    m = w.media()
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    lam, mu, rho = dev(m["lam"]), dev(m["mu"]), dev(m["rho"])
    opts = dict(levels=w.levels, cycle=w.cycle, cycle_level=w.cycle_level, nu1=w.nu1, nu2=w.nu2, vanka=w.vanka,
                precond_bits=w.precond_bits, restart=w.restart, dd_parts=w.dd_parts,
                dd_overlap=w.dd_overlap, dd_pad=w.dd_pad, dd_colors=w.dd_colors, damping=w.damping,
                abl_max=w.abl_max, atten0=w.atten0, coarse_bits=w.coarse_bits)

    def make():
        return ehh.Solver(w.dim, w.n, w.h, w.omega, w.shift, w.abl_cells, lam, mu, rho, **opts)

    S0 = make()
    B = rhs_tensor(S0, w)
    X = torch.zeros_like(B)
    S0.close()
    torch.cuda.synchronize()
    results = []

    def step():
        t0 = time.perf_counter()
        S = make()
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
    return total, results, B, X


def visits_per_cycle(w):
    """Visits of each non-coarsest level in one cycle: a level makes `cycle`
    recursive calls from cycle_level on (one call above it and into the
    coarsest level, whose exact solve a second call would only repeat)."""
    v = [1]
    for l in range(w.levels - 2):
        calls = 1 if (l + 1 == w.levels - 1 or l < w.cycle_level) else w.cycle
        v.append(v[-1] * calls)
    return v


def relax_kernel_name(w, level, ncell):
    """The half-sweep kernel the library launches on a level (same routing as
    its launcher): one thread per cell on the finest level, LDS-staged tiles on
    2D Galerkin levels of at least 256^2 cells with more than 8 sources, eight
    lanes per cell with row coefficients stored at setup on the other Galerkin
    levels (3D: blocks of 8 (FP32) or 2 (FP64) sources per coefficient load; the
    smallest FP64 2D levels split each row over two wavefronts for the sweeps
    that start from e_in)."""
    t = "float" if w.precond_bits == 32 else "double"
    if w.dim == 2:
        if level == 0:
            return f"k_relax_cell2d<{t}, {t}>"
        if ncell >= 65536 and len(w.sources()) > 8:
            return f"k_relax_lds2d<{t}, StOp<2, {t}>>"
        if t == "double" and -(-(ncell // 2) * 8 // 256) * 4 <= 256:
            return "k_relax_st2d_split<double>"   # three of the visit's four half-sweeps
        return f"k_relax_st2d<{t}, {'true' if t == 'float' else 'false'}, false>"
    if level == 0:
        return f"k_relax_cell3d<{t}>"
    if t == "double":
        return "k_relax_st3d<double, 2, 4, double>"
    return f"k_relax_st3d<float, 8, 8, {'_Float16' if w.coarse_bits == 16 else 'float'}>"


KERNEL_SOURCES = ["paper_1806_11277_amd/csrc/levels.hip", "paper_1806_11277_amd/csrc/ops.hpp",
                  "paper_1806_11277_amd/csrc/common.hpp"]


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


def kernel_roofline(w, reps=30):
    """HBM roofline of the dominant kernel, the red-black Vanka half-sweep.
    Every level's half-sweep is timed with HIP events around the replay of a
    graph of its launches (captured from the library's launches on the
    caller's stream), each visit preceded by a 512 MiB write that evicts the
    caches as the rest of a solve does, whose own time is subtracted.  Launches are weighted by their
    count in one cycle (2 (nu1 + nu2) half-sweeps per visit) and grouped by the
    kernel each level uses; the dominant kernel is the one with the largest
    time per cycle.  achieved = its algorithmic bytes per launch / its average
    launch duration."""
    import torch
    from paper_1806_11277_amd import ehh
    S = ehh.solver_for_workload(w)
    nrhs = len(w.sources())
    dt = torch.float32 if w.precond_bits == 32 else torch.float64
    stream = torch.cuda.current_stream()
    visits = visits_per_cycle(w)
    rows = []
    groups = {}
    scrub = torch.empty(64 * 2 ** 20, dtype=torch.float64, device="cuda")   # 512 MiB
    for l in range(w.levels - 1):
        info = S.level_info(0, l)
        # several vector sets in turn, so that a visit does not find the previous
        # visit's vectors in L2 (inside a solve the level's vectors were last
        # touched by other kernels)
        nset = 4
        sets = []
        for _ in range(nset):
            b = torch.randn((nrhs, 2 * info["N"]), dtype=dt, device="cuda")
            sets.append((b, torch.randn_like(b), torch.zeros_like(b)))
        # one visit's sweeps as the cycle launches them: the first pre-smoothing
        # half-sweep starts from zero (no e_in), the others read e_in
        nsw = 2 * (w.nu1 + w.nu2)
        nzero = 1 if w.nu1 > 0 else 0

        def visit(v=0):
            b, e_in, e_out = sets[v % nset]
            for k in range(nsw):
                S.level_relax(0, l, k % 2, b, None if k < nzero else e_in, e_out)
        visit()
        torch.cuda.synchronize()
        # The sweeps are replayed from a captured graph, as the solver replays its
        # Arnoldi steps, so that host launch gaps do not enter the timing.  Each
        # visit is preceded by a write of 512 MiB that evicts the L2s and the
        # MALL, as the other kernels of a solve do between two visits of a level:
        # t = (time of scrub + visit - time of scrub alone) per half-sweep.
        def timed(with_visit):
            graph = torch.cuda.CUDAGraph()
            cap = torch.cuda.Stream()
            with torch.cuda.graph(graph, stream=cap):
                for r in range(reps):
                    scrub.zero_()
                    if with_visit:
                        visit(r)
            graph.replay()
            best = float("inf")
            for _ in range(3):
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                ev0.record(stream)
                graph.replay()
                ev1.record(stream)
                torch.cuda.synchronize()
                best = min(best, ev0.elapsed_time(ev1) / 1e3)
            del graph
            return best
        t = max(timed(True) - timed(False), 0.0) / (reps * nsw)
        cb = 2 if (w.coarse_bits == 16 and w.dim == 3) else None
        nb = (nzero * level_bytes(info, w.precond_bits, nrhs, l == 0, w.dim, with_e=False, coef_bytes=cb) +
              (nsw - nzero) * level_bytes(info, w.precond_bits, nrhs, l == 0, w.dim, coef_bytes=cb)) / nsw
        launches = 2 * (w.nu1 + w.nu2) * visits[l]
        ncell = int(np.prod(info["n"][:w.dim]))
        name = relax_kernel_name(w, l, ncell)
        rows.append(dict(level=l, n=info["n"][:w.dim], kernel=name, bytes=nb, us=t * 1e6, gbs=nb / t / 1e9,
                         launches_per_cycle=launches))
        g = groups.setdefault(name, dict(kernel=name, launches_per_cycle=0, bytes_per_cycle=0.0,
                                         us_per_cycle=0.0))
        g["launches_per_cycle"] += launches
        g["bytes_per_cycle"] += launches * nb
        g["us_per_cycle"] += launches * t * 1e6
        del sets
    del scrub
    S.close()
    for g in groups.values():
        g["avg_launch_us"] = g["us_per_cycle"] / g["launches_per_cycle"]
        g["bytes_per_launch"] = g["bytes_per_cycle"] / g["launches_per_cycle"]
        g["gbs"] = g["bytes_per_cycle"] / g["us_per_cycle"] / 1e3
    dom = max(groups.values(), key=lambda g: g["us_per_cycle"])
    achieved = dom["gbs"]
    rec = traffic_record(w.name, dom["kernel"])
    tot_b = sum(g["bytes_per_cycle"] for g in groups.values())
    tot_t = sum(g["us_per_cycle"] for g in groups.values())
    return dict(bound="hbm", kernel=dom["kernel"], achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s",
                frac=achieved / PEAK_HBM_GBS,
                traffic=(rec["hbm_bytes_per_launch"] if rec else None),
                traffic_unit="HBM bytes per launch (counters scaled by a plain copy)",
                bytes_per_launch=dom["bytes_per_launch"], avg_launch_us=dom["avg_launch_us"],
                launches_per_cycle=dom["launches_per_cycle"],
                all_levels={"gbs": tot_b / tot_t / 1e3, "us_per_cycle": tot_t, "bytes_per_cycle": tot_b},
                kernels=sorted(groups.values(), key=lambda g: -g["us_per_cycle"]), levels=rows)


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


def cpu_baseline(w, gpu_iters, budget_s=20.0):
    """The oracle as it stands (numpy/scipy, FP64) on this host: hierarchy setup
    plus as many FGMRES iterations as fit in the budget, scaled to a full solve
    with the GPU's iteration count."""
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:  # pragma: no cover
        limiter = None
    from oracle import discretisation as disc, multigrid as mg
    m = w.media()
    t0 = time.perf_counter()
    pb = disc.Problem(w.n, w.h, w.omega, m["lam"], m["mu"], m["rho"], w.abl_cells, w.abl_max,
                      w.atten0, shift=w.shift)
    A = pb.matrix()
    H = mg.build_hierarchy(pb, w.levels, list(w.damping), economic=(w.vanka == 0), cycle=w.cycle,
                           nu1=w.nu1, nu2=w.nu2, cycle_level=w.cycle_level)
    t_setup = time.perf_counter() - t0
    b = disc.point_source_vector(w.n, w.sources()[:1])
    v = b / np.linalg.norm(b)
    k = 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < budget_s:
        z = H.cycle(v)
        wv = A @ z
        v = wv / np.linalg.norm(wv)
        k += 1
    t_iter = (time.perf_counter() - t1) / k
    t_solve = t_setup + gpu_iters * t_iter
    if limiter is not None:
        limiter.unregister()
    return dict(value=1.0 / t_solve, unit="solves/s", cores=1, kind="oracle",
                sample=f"oracle setup ({t_setup:.1f} s) + {k} preconditioned FGMRES iterations "
                       f"({t_iter:.2f} s each) of {w.name}, one right-hand side, scaled to "
                       f"{gpu_iters} iterations")


def poisson_sweep_report():
    """Preconditioning cycles to 1e-6 for constant mu = rho = 1 and lambda from 0.5
    to 16 (section 6, Fig. 5), full and economic Vanka, on the grids whose
    exact coarsest level fits a dense inverse."""
    import torch
    from paper_1806_11277_amd import ehh
    from workloads.configs import poisson_sweep, SWEEP_LAMBDAS, SWEEP_GRIDS
    out = {"experiment": "Poisson-ratio sweep, constant mu = rho = 1", "lambda": list(SWEEP_LAMBDAS), "grids": []}
    for nx in (256, 512):
        row = {"cells": [nx, nx // 2], "omega_over_pi": 3 * nx // 256, "levels": SWEEP_GRIDS[nx][0],
               "shift": SWEEP_GRIDS[nx][1]}
        for vanka, key in ((1, "full_vanka"), (0, "economic_vanka")):
            its = []
            for lam in SWEEP_LAMBDAS:
                w = poisson_sweep(nx, lam, vanka)
                S = ehh.solver_for_workload(w)
                b = rhs_tensor(S, w)
                x = torch.zeros_like(b)
                st, stats = S.solve(b, x, tol=1e-6, maxit=600)
                torch.cuda.synchronize()
                S.close()
                its.append(stats[0]["iters"] if st == 0 else None)
                print(f"[sweep] {w.name}: {its[-1]}", file=sys.stderr, flush=True)
            row[key] = its
        out["grids"].append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2_hetero512_fp64")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--batched", default="c3_hetero512_batch32_fp32",
                    help="batched companion workload reported in the same line ('' to skip)")
    ap.add_argument("--batched-steps", type=int, default=2)
    ap.add_argument("--poisson-sweep", action="store_true",
                    help="print the Poisson-ratio sweep (constant media, lambda 0.5..16) as one JSON line and exit")
    ap.add_argument("--coarse-bits", type=int, default=None, choices=(16, 32),
                    help="storage of the 3D Galerkin levels' stored rows in the complex64 cycle "
                         "(16: FP16 with a power-of-two scale per level)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for traffic counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver runs all subdomains and right-hand sides "
              "on a single device; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
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
        import dataclasses
        w = dataclasses.replace(w, coarse_bits=a.coarse_bits)
    print(f"[bench] {w.name}: n={w.n} nrhs={len(w.sources())} levels={w.levels} cycle={w.cycle} "
          f"bits={w.precond_bits}", file=sys.stderr, flush=True)
    total, res, B, X = run_gpu(w, a.steps, a.warmup, a.tol)
    setup_ms = 1e3 * float(np.mean([r[0] for r in res]))
    solve_ms = 1e3 * float(np.mean([r[1] for r in res]))
    stats = res[-1][3]
    iters = [s["iters"] for s in stats]
    nrhs = len(stats)
    ms_per_step = 1e3 * total / a.steps
    out = {
        "metric": "preconditioned solves/sec at rel. residual 1e-6; V-cycle HBM GB/s vs peak",
        "value": nrhs * a.steps / total,
        "unit": "solves/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w.precond_bits == 64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.n), "unknowns": int(B.shape[1] // 2),
                   "nrhs": nrhs, "levels": w.levels, "cycle": "V" if w.cycle == 1 else "W",
                   "cycle_level": w.cycle_level,
                   "nu": [w.nu1, w.nu2], "vanka": "full" if w.vanka else "economic",
                   "shift": w.shift, "precond_bits": w.precond_bits, "restart": w.restart,
                   "dd_parts": list(w.dd_parts[:w.dim]), "coarse_bits": w.coarse_bits, "tol": a.tol},
        "setup_ms": setup_ms, "solve_ms": solve_ms,
        "iters": iters if nrhs <= 4 else [min(iters), max(iters)],
        "rel_res_true_max": max(s["rel_res_true"] for s in stats),
        "status": res[-1][2],
    }
    if not a.no_roofline:
        print("[bench] roofline of the dominant kernel", file=sys.stderr, flush=True)
        out["roofline"] = kernel_roofline(w)
        cg = copy_bandwidth()
        out["roofline"]["copy_gbs"] = cg          # achievable plain-copy bandwidth on this GPU (context)
        out["roofline"]["frac_of_copy"] = out["roofline"]["achieved"] / cg
    if a.batched:
        wb = get_config(a.batched)
        print(f"[bench] batched companion {wb.name}", file=sys.stderr, flush=True)
        tb, rb, Bb, _ = run_gpu(wb, a.batched_steps, 1, a.tol)
        sb = rb[-1][3]
        itb = [s_["iters"] for s_ in sb]
        vb = len(sb) * a.batched_steps / tb
        out["batched"] = {"workload": wb.name, "nrhs": len(sb), "value": vb, "unit": "solves/s",
                          "ms_per_step": 1e3 * tb / a.batched_steps,
                          "dtype": "f32 cycle + f64 Krylov/coarsest",
                          "iters_min_max": [min(itb), max(itb)],
                          "rel_res_true_max": max(s_["rel_res_true"] for s_ in sb),
                          "speedup_vs_plain_fp64_single_source": vb / out["value"]}
        if not a.no_roofline:
            out["batched"]["roofline"] = kernel_roofline(wb)
            cg = out["roofline"]["copy_gbs"]
            out["batched"]["roofline"]["copy_gbs"] = cg
            out["batched"]["roofline"]["frac_of_copy"] = out["batched"]["roofline"]["achieved"] / cg
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, int(np.median(iters)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
