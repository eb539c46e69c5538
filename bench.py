#!/usr/bin/env python3
"""Benchmark: Robin-Schwarz solves per second to a 1e-8 relative residual on
one MI355X, batched FP32-inner form vs the plain FP64 stepwise form.

Default workload: 128^3 Q2 elements on the unit cube, 8x8x8 subdomains (17.98 M
local unknowns, an HBM-resident working set), Robin p = 8/h, layered
crater-like density anomaly with 10 Gaussian blobs (seeded, synthetic).

A step is one slice of k outer iterations of the hot path (local right-hand
side and residual, the fused subdomain-CG kernel, the Robin exchange, and a
global residual check every 10 outer iterations), replayed as HIP graphs with
the inputs already in HBM. Solves run back to back from a zero start: each
solve takes N outer iterations, N measured by a reference solve of the same
workload first, and k is chosen so that the K timed steps cover at least one
whole solve. value = (K k / N) / (timed seconds) solves/s; every solve that
completes inside the timed region is checked to have reached the tolerance.

Prints one JSON line. The roofline entry comes from the reference solve,
launched eagerly with HIP events around every fused CG launch on the
library's stream: algorithmic bytes per launch (12 words per CG iteration and
local unknown, counted by the kernel) over the average launch duration. The
plain form is timed on a bounded sample of outer iterations. The CPU
baseline times the oracle (exact subdomain solves) on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PMC_GLOB = os.path.join(ROOT, "profiles", "fused_cg_*_pmc.json")
GOLDEN_COUNTS = os.path.join(ROOT, "tests", "golden", "oracle_outer_counts.json")
CSRC = os.path.join(ROOT, "paper_2112_03851_amd", "csrc")
KERNEL_SRCS = [os.path.join(CSRC, n) for n in ("sos_device.h", "sos_kernels.h", "sos_internal.h", "sos_kernels.hip",
                                               "sos_fused.hip")]


def kernel_sha():
    """Hash of every source file the kernels are compiled from."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


# The headline metric: whole solves per second to a 1e-8 relative residual,
# reported with the fused CG kernel's bandwidth against HBM peak and the plain
# FP64 form beside it.
METRIC = "Schwarz solves/s to 1e-8 rel residual + SpMV HBM GB/s (% peak), batched vs plain"


def measured_traffic(launch_bytes, st, workload_name):
    """HBM bytes per fused-kernel launch from committed rocprofv3 counters
    (FETCH_SIZE + WRITE_SIZE, each scaled by its reading for a plain copy),
    if some counter file was taken on this workload and the current kernel
    source with the same block shape, team size and residency level;
    per launch of this run (the counters' ratio to the algorithmic bytes)."""
    shape = (st["block"], st["cols_per_thread"], st["team"], st["wave_rows"], st["resident"])
    for path in sorted(glob.glob(PMC_GLOB)):
        try:
            pmc = json.load(open(path))
        except Exception:
            continue
        if pmc.get("workload_name") != workload_name or pmc.get("kernel_sha") != kernel_sha():
            continue
        if (pmc.get("block"), pmc.get("cols_per_thread"), pmc.get("team"), pmc.get("wave_rows", 0),
                pmc.get("resident")) != shape:
            continue
        return pmc["traffic_over_algorithmic"] * launch_bytes
    return None


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def host_info():
    """Host CPUs of this machine: logical CPUs, the ones this process may use,
    and the model name."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except Exception:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def cpu_baseline(wl, budget_s, phi_gpu, n_outer_solve, n_outer_basis):
    """The oracle (exact FDM subdomain solves, Jacobi exchange, global residual
    after every outer iteration) on a bounded number of outer iterations of the
    same workload, with the BLAS threads it gets by default and again limited
    to one thread; scaled to solves/s with n_outer_solve outer iterations per
    solve. cores = process CPU time over wall time of the sample (the threads
    it actually kept busy)."""
    import numpy as np
    from oracle import assemble as A
    from oracle import direct as D
    from oracle import mesh as M
    from oracle import partition as P
    from oracle import schwarz as S
    from oracle import subdomain as SD
    m = M.BoxMesh(wl.ne, wl.lengths, wl.bc)
    part = P.BoxPartition(m, wl.cuts)
    drho = wl.drho()
    f = A.load_from_density(m, drho, wl.G)
    fs = [SD.density_load(part, s, drho, wl.G) for s in part.subs]
    t0 = time.perf_counter()
    orc = S.SchwarzOracle(part, wl.p, "fdm")
    setup_s = time.perf_counter() - t0

    def sample(budget):
        lam = orc.zero_data()
        n = 0
        c0, t0 = time.process_time(), time.perf_counter()
        while n < 2 or time.perf_counter() - t0 < budget:
            u = orc.subdomain_solves(fs, lam)
            lam = orc.exchange(u, lam)
            A.residual_norm(m, orc.glue(u), f)
            n += 1
        el = time.perf_counter() - t0
        return n, el, (time.process_time() - c0) / el

    log(f"cpu baseline: oracle set up in {setup_s:.1f} s")
    n, el, busy = sample(budget_s)
    log(f"cpu baseline: {n} outer iterations in {el:.1f} s")
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            n1, el1, busy1 = sample(budget_s / 2)
        one = {"value": (n1 / el1) / n_outer_solve, "outer_iters_per_s": n1 / el1, "sample": f"{n1} outer iterations "
               f"in {el1:.1f} s", "cores": round(busy1, 2)}
    except Exception as e:  # threadpoolctl missing: no one-thread figure
        one = {"error": str(e)}
    out = {"value": (n / el) / n_outer_solve, "unit": "solves/s", "cores": round(busy, 2), "kind": "oracle",
           "sample": f"{n} outer iterations of the oracle's Schwarz solve of this workload (exact FDM subdomain "
                     f"solves, exchange, global residual) in {el:.1f} s (setup {setup_s:.1f} s excluded), "
                     f"scaled by {n_outer_solve} outer iterations per solve ({n_outer_basis})",
           "outer_iters_per_s": n / el, "one_thread": one, **host_info()}
    if phi_gpu is not None:
        log("cpu baseline: the oracle's direct solve for the error of the GPU result")
        t0 = time.perf_counter()
        ud = D.solve_direct(m, f, "fdm")
        out["direct_solve_s"] = time.perf_counter() - t0
        out["gpu_max_rel_err_vs_oracle_direct"] = float(np.abs(phi_gpu - ud).max() / np.abs(ud).max())
        out["gpu_rel_residual_by_oracle"] = A.residual_norm(m, phi_gpu, f)
    return out


def reference_copy(torch, mib):
    """A plain device-to-device copy of known size (profiling runs only): what
    the memory counters read for it scales their reading of the solver's kernels."""
    if mib <= 0:
        return
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {n * 4} bytes device to device (one read and one write of each byte)", flush=True)


def robin_of(wl):
    """(p, q, description) of a workload's transmission condition: the stated
    p, or for the slab workloads the symmetric second-order condition that
    minimises the two-subdomain Fourier factor over the interface's
    frequency range (CMA-ES in the library, host)."""
    kind = wl.extra.get("robin_kind")
    if kind is None:
        return wl.p, 0.0, f"zeroth order p = {wl.p:g}"
    from paper_2112_03851_amd.sos import optimize_robin
    pq, rho, _ = optimize_robin(kind, wl.extra["kmin"], wl.extra["kmax"])
    return pq[0], pq[1], (f"second order p = {pq[0]:.6g}, q = {pq[1]:.6g} (CMA-ES over k in "
                          f"[{wl.extra['kmin']:.4g}, {wl.extra['kmax']:.4g}], rho_max = {rho:.4f})")


def candidate_pipeline(args, torch, Problem, workload):
    """Stochastic transmission-condition search at scale: seeded candidates
    (p log-uniform on [h^-3/2, 10/h], q uniform on [0, h], h of the copy)
    scored by their convergence rate between outer iterations 10 and 20 on the
    32^3 copy, all candidates in one context; the best moves to the 128^3 mesh
    with p h and q / h kept (both meshes have 16^3-element subdomains) and is
    solved to 1e-8, next to the prescribed zeroth-order p = 8/h."""
    from synth.generators import robin_candidates
    small, big = workload("c5copy", seed=args.seed), workload("c5", seed=args.seed)
    h, H = small.lengths[0] / small.ne[0], big.lengths[0] / big.ne[0]
    p, q = robin_candidates(args.candidates, h, seed=args.seed)
    d_small = torch.tensor(small.drho(), device="cuda")
    prob = Problem(small.ne, small.lengths, small.bc, cuts=small.cuts, p=p, q=q, G=small.G, precision="fp32",
                   mode="batched", check_every=10, inner_tol=args.inner_tol, copies=args.candidates)
    prob.batch_rates(d_small, 10, 20)  # first call tunes the block shape
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rates, r1, r2, best, st = prob.batch_rates(d_small, 10, 20)
    torch.cuda.synchronize()
    t_score = time.perf_counter() - t0
    prob.close()
    pb, qb = p[best] * h / H, q[best] * H / h
    d_big = torch.tensor(big.drho(), device="cuda")
    out = {}
    for name, pp, qq in (("transferred_best", pb, qb), ("prescribed_p_8_over_h", big.p, 0.0)):
        pr = Problem(big.ne, big.lengths, big.bc, cuts=big.cuts, p=pp, q=qq, G=big.G, precision="fp32",
                     mode="batched", check_every=args.check_every, inner_tol=args.inner_tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, s = pr.solve(d_big, big.tol)
        torch.cuda.synchronize()
        out[name] = {"p": pp, "q": qq, "seconds": time.perf_counter() - t0, "outer_iters": s["outer_iters"],
                     "inner_iters": s["inner_iters"], "rel_residual": s["rel_residual"], "converged": s["converged"],
                     "block": s["block"], "cols_per_thread": s["cols_per_thread"], "team": s["team"]}
        pr.close()
    line = {"metric": "candidate scoring on the 32^3 copy + 128^3 solve to 1e-8 with the best condition",
            "value": t_score, "unit": "s (scoring all candidates)", "n_gpus": 1, "higher_is_better": False,
            "data": "synthetic", "dtype": "f32+f64",
            "config": {"workload": f"{args.candidates} candidates x 8 subdomains of the 32^3 copy (one context, "
                                   f"{args.candidates * 8} subdomains per launch), 20 outer iterations; then 128^3, "
                                   f"8x8x8 subdomains, crater-like anomaly seed {args.seed}"},
            "scoring": {"outer_iters": st["outer_iters"], "inner_iters": st["inner_iters"], "best": best,
                        "best_rate": float(rates[best]), "p_best": float(p[best]), "q_best": float(q[best]),
                        "rate_range": [float(np.nanmin(rates)), float(np.nanmax(rates))],
                        "block": st["block"], "team": st["team"]},
            "solves": out}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--inner-tol", type=float, default=0.1)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--team", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--plain-outer", type=int, default=20,
                    help="outer iterations of the plain FP64 form's bounded sample")
    ap.add_argument("--profile-outer", type=int, default=0,
                    help="profiling only: run one batched solve of this many outer iterations "
                         "(no convergence, no JSON line) for rocprofv3 counter collection")
    ap.add_argument("--candidates", type=int, default=0,
                    help="instead of the default line: score this many seeded (p, q) candidates on the 32^3 copy "
                         "(all copies in every launch), transfer the best to the 128^3 workload and solve it")
    ap.add_argument("--profile-copy-mib", type=int, default=0,
                    help="profiling only: finally copy a buffer of this many MiB device to device, "
                         "the reference for scaling the memory counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_03851_amd.sos import Problem
    from synth import workload

    if args.candidates:
        candidate_pipeline(args, torch, Problem, workload)
        return
    wl = workload(args.workload, seed=args.seed)
    drho = torch.tensor(wl.drho(), device="cuda")
    rp, rq, rdesc = robin_of(wl)
    if args.profile_outer:
        if not (args.block and args.team):
            raise SystemExit("--profile-outer needs --block and --team (no autotuner launches in a counter run)")
        prob = Problem(wl.ne, wl.lengths, wl.bc, cuts=wl.cuts, p=rp, q=rq, G=wl.G, precision="fp32", mode="batched",
                       check_every=args.check_every, inner_tol=args.inner_tol, block=args.block,
                       team=args.team, max_outer=args.profile_outer, timing=1)
        phi, st = prob.solve(drho, wl.tol)
        print(f"profiled {st['outer_iters']} outer iterations, {st['kernel_launches']} fused launches, "
              f"{st['kernel_bytes'] / st['kernel_launches']:.0f} algorithmic bytes per launch, "
              f"{st['kernel_ms'] / st['kernel_launches']:.4f} ms per launch", flush=True)
        print("shape " + json.dumps({k: st[k] for k in ("block", "cols_per_thread", "team", "wave_rows", "resident")}),
              flush=True)
        reference_copy(torch, args.profile_copy_mib)
        return
    every = args.check_every
    prob = Problem(wl.ne, wl.lengths, wl.bc, cuts=wl.cuts, p=rp, q=rq, G=wl.G, precision="fp32", mode="batched",
                   check_every=every, inner_tol=args.inner_tol, timing=1, block=args.block, team=args.team)
    # reference solve (the first solve also tunes the fused kernel's block
    # shape): outer iterations per solve, and the roofline from HIP events
    # around every fused launch (eager launches)
    log(f"workload {wl.name}: reference solve (eager, HIP events; the first solve tunes the block shape)")
    phi, ref = prob.solve(drho, wl.tol)
    log(f"reference solve: {ref['outer_iters']} outer iterations, {ref['seconds']:.2f} s, block {ref['block']} x "
        f"{ref['cols_per_thread']}, team {ref['team']}, resident {ref['resident']}")
    if not ref["converged"]:
        raise RuntimeError(f"batched reference solve did not converge: {ref}")
    phi_np = phi.cpu().numpy()
    n_solve = ref["outer_iters"]
    launch_bytes = ref["kernel_bytes"] / ref["kernel_launches"]
    launch_s = ref["kernel_ms"] * 1e-3 / ref["kernel_launches"]
    achieved = launch_bytes / launch_s / 1e9
    traffic = measured_traffic(launch_bytes, ref, args.workload)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_fused_cg<float>", "avg_launch_ms": launch_s * 1e3,
                "algorithmic_bytes_per_launch": launch_bytes, "launches": ref["kernel_launches"],
                "basis": "algorithmic bytes (12 FP32 words per CG iteration and local unknown + the FP64 update "
                         "of u, counted by the kernel) / average launch duration from HIP events on the "
                         "library's stream over the eager reference solve",
                "measured_dram_gbs": traffic / launch_s / 1e9 if traffic else None,
                "measured_dram_frac": traffic / launch_s / 1e9 / HBM_PEAK_GBS if traffic else None}

    # timed steps: graph replays of k outer iterations, solves back to back
    prob.set_opts(timing=0)
    k = every * max(1, -(-n_solve // (args.steps * every)))
    lay = prob.layout()
    zu = torch.zeros(int(lay["offsets"][-1]), dtype=torch.float64, device="cuda")
    zl = torch.zeros(max(1, int(lay["face_off"][-1])), dtype=torch.float64, device="cuda")
    state = {"pos": 0, "solves": 0, "res": []}

    def restart():
        prob.set_state(zu, zl)
        state["pos"] = 0

    def step():
        left = k
        while left > 0:
            n = min(left, n_solve - state["pos"])
            st_ = prob.iterate(n)
            state["pos"] += n
            left -= n
            if state["pos"] == n_solve:
                state["res"].append(st_["rel_residual"])
                state["solves"] += 1
                restart()

    log(f"{args.warmup} warm-up and {args.steps} timed steps of {k} outer iterations")
    restart()
    for _ in range(args.warmup):
        step()
    restart()
    state["solves"], state["res"] = 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log(f"timed: {args.steps * k} outer iterations in {el:.2f} s, {state['solves']} solves completed")
    if not state["res"] or max(state["res"]) > wl.tol:
        raise RuntimeError(f"a timed solve missed the tolerance: {state['res']}")
    outer_timed = args.steps * k
    solves = outer_timed / n_solve
    batched = {"outer_iters_per_solve": n_solve, "inner_iters_per_solve": ref["inner_iters"],
               "rel_residual": ref["rel_residual"], "block": ref["block"],
               "cols_per_thread": ref["cols_per_thread"], "team": ref["team"], "wave_rows": ref["wave_rows"],
               "resident": ref["resident"], "seconds_per_solve": el / solves,
               "timed_outer_iters": outer_timed, "timed_solves_completed": state["solves"],
               "timed_solve_residuals": state["res"], "outer_iters_per_step": k,
               "reference_solve_eager_s": ref["seconds"],
               "inner_tol": args.inner_tol, "check_every": every}
    prob.close()

    plain = None
    if not args.no_plain:
        # bounded sample: the plain FP64 form (one launch per CG step over all
        # subdomains, inner stop 1e-12 ||b_s||) over the first outer iterations
        p64 = Problem(wl.ne, wl.lengths, wl.bc, cuts=wl.cuts, p=rp, q=rq, G=wl.G, precision="fp64", mode="stepwise",
                      check_every=1, inner_tol=0.0, inner_abs=1e-12, max_inner=2000, timing=1)
        log(f"plain FP64 form: {args.plain_outer} outer iterations")
        p64.set_density(drho)
        p64.set_state(zu, zl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s64 = p64.iterate(args.plain_outer)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        p64.close()
        s_outer = t_plain / args.plain_outer
        plain = {"form": "FP64 Jacobi-PCG per subdomain, one launch per CG step (apply + p'q, update + r'z, r'r) "
                         "over all subdomains, inner stop 1e-12 ||b_s||, global residual every outer iteration",
                 "sample": f"the first {args.plain_outer} outer iterations of the solve from zero",
                 "seconds_per_outer_iter": s_outer,
                 "inner_iters_per_outer_iter": s64["inner_iters"] / args.plain_outer,
                 "cg_kernel_gbs": s64["kernel_bytes"] / (s64["kernel_ms"] * 1e-3) / 1e9,
                 "cg_kernel_frac_of_hbm_peak": s64["kernel_bytes"] / (s64["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "cg_kernel_bytes_basis": "10 FP64 vectors read or written per CG iteration and local unknown, "
                                          "over the summed duration of the CG step kernels (HIP events)",
                 "estimated_seconds_per_solve": s_outer * n_solve,
                 "estimate_basis": f"seconds per outer iteration x the batched form's {n_solve} outer iterations "
                                   f"per solve (with near-exact inner solves the plain form needs about 7 % fewer "
                                   f"on 64^3)"}

    cpu = None
    if not args.no_cpu:
        n_or, basis = n_solve, "the GPU batched form's count for this workload"
        try:
            n_or = json.load(open(GOLDEN_COUNTS))[f"{wl.name}_seed{wl.seed}"]["outer_iters"]
            basis = "the oracle's own count for this workload"
        except Exception:
            pass
        cpu = cpu_baseline(wl, args.cpu_seconds, phi_np, n_or, basis)
    line = {
        "metric": METRIC, "value": solves / el, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{wl.name}: box {wl.lengths[0]:g}x{wl.lengths[1]:g}x{wl.lengths[2]:g}, "
                               f"{wl.ne[0]}x{wl.ne[1]}x{wl.ne[2]} Q2 elements, "
                               f"{wl.nparts[0]}x{wl.nparts[1]}x{wl.nparts[2]} subdomains, {rdesc}"
                               f"{' (8/h)' if not wl.extra.get('robin_kind') else ''}, crater-like anomaly "
                               f"(seed {wl.seed}), tol {wl.tol:g}",
                   "form": "batched: fused FP32 CG kernel per outer iteration, FP64 outer residual, "
                           "exchange and refinement, outer iterations replayed as HIP graphs",
                   "step": f"{k} outer iterations (graph replays of {every} iterations + a global residual "
                           f"check); solves of {n_solve} outer iterations run back to back from zero; "
                           f"value = timed outer iterations / {n_solve} / timed seconds",
                   "parallelism": "single GPU"},
        "roofline": roofline, "batched": batched, "plain": plain,
        "batched_vs_plain_speedup": (plain["estimated_seconds_per_solve"] / (el / solves)) if plain else None,
        "cpu_baseline": cpu, "kernel_sha": kernel_sha(),
    }
    print(json.dumps(line), flush=True)
    reference_copy(torch, args.profile_copy_mib)


if __name__ == "__main__":
    main()
