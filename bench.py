"""Benchmark: F-lambda applies/s and Newton-step time of the TFETI path on one GPU.

A step is one load step of the elastoplastic time stepping (Algorithm 4):
Newton iterations until convergence, each with the return map and tangent
assembly at every Gauss point, fixing-node regularization, batched band
Cholesky of the subdomains whose tangent changed, panel packing and the whole
PCGP (Algorithm 3) with its F-applies, projections and lumped preconditioner;
then the commit.  The default times load steps 2..30 of the 10x10x10
benchmark after one untimed load step.

value = F-applies executed inside the K timed load steps / their wall time.
newton_step_ms = wall time / Newton iterations with a linear solve.
roofline: the subdomain-solve kernel of the F-apply, algorithmic bytes = two
passes over the skyline (envelope) of every subdomain factor, divided by the
kernel's mean duration from HIP events on the library's stream.
cpu_baseline: the FP64 oracle's F-apply on a sample of the same subdomains.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "F·λ applies/s (HBM GB/s) + Newton-step time at 1e-6 rel. error vs FP64 oracle"
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(seconds: float = 12.0):
    """Time the oracle's F-apply on 8 subdomains of 8^3 Q1 elements (the
    per-subdomain shape of the 10x10x10 benchmark mesh) and scale to the
    1000 subdomains of one full F-apply."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import assembly
    from oracle.mesh import Mesh
    from oracle.tfeti import TFETI

    w = W.small_cube(S=(2, 2, 2), n=(8, 8, 8), amp=400.0)
    mesh = Mesh(w)
    ed = assembly.element_dofs_torn(mesh)
    a = assembly.assemble(mesh, ed, mesh.n_torn, np.zeros(mesh.n_torn), np.zeros((mesh.n_elems, 8, 6)),
                          np.zeros((mesh.n_elems, 8)))
    tf = TFETI(mesh)
    tf.set_matrix(a["K"])
    lam = np.random.default_rng(0).standard_normal(mesh.m)
    with threadpool_limits(limits=1):
        tf.F(lam)
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            tf.F(lam)
            n += 1
        dt = (time.perf_counter() - t0) / n
    scale = 1000 / len(mesh.subs)
    return {"value": 1.0 / (dt * scale), "unit": "F-applies/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle F-apply (scipy banded Cholesky solves) on 8 subdomains of 8^3 Q1 elements, "
                      f"{n} applies in {n * dt:.1f} s, scaled x{scale:.0f} to the 1000-subdomain mesh; "
                      f"BLAS limited to 1 thread"}


def describe(w, sz) -> str:
    """The workload in words: mesh, decomposition, sizes and load."""
    sub = ("8^3" if set(w.nx) | set(w.ny) | set(w.nz) == {8}
           else f"{min(w.nx + w.ny + w.nz)}..{max(w.nx + w.ny + w.nz)} elements per axis")
    top = w.traction[5]
    load = " + ".join(t for t, v in (("x shear", top[0]), ("y shear", top[1]), ("z traction", top[2])) if v)
    return (f"{w.name}: unit cube of Q1 hexahedra, {sz['n_sub']} box subdomains of {sub}, {sz['n_torn']} torn DOF, "
            f"{sz['m']} multipliers, clamped bottom, top face {load}, load ramp over {w.steps} steps")


def measured_traffic(workload: str, precision: str, tile: int, threads: int):
    """HBM bytes per launch of the F-apply solve kernel from the committed
    FETCH_SIZE/WRITE_SIZE summary, or None if that summary was taken on
    another workload, kernel source, tile or workgroup size."""
    import hashlib
    if workload != "cube10x10x10_sub8":
        return None
    path = os.path.join(ROOT, "profiles", "ksolve_traffic_cube10x10x10_sub8.md")
    src = os.path.join(ROOT, "paper_1205_1926_amd", "csrc", "ksolve.hip")
    try:
        line = [l for l in open(path) if l.startswith("traffic: ")][0]
        rec = json.loads(line[len("traffic: "):])
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, IndexError, ValueError):
        return None
    ent = rec.get(precision, {}).get(f"{tile}/{threads}")
    if rec.get("ksolve_sha256") != sha or not ent:
        return None
    return ent["traffic_bytes"]


def counter_probe(g, reps: int) -> int:
    """Kernels of known traffic for FETCH_SIZE / WRITE_SIZE runs: the F-apply
    on the factors of the first Newton iteration, then a plain device copy of
    1 GiB (reads 1 GiB, writes 1 GiB) that calibrates the counters."""
    import torch
    g.begin_load_step()
    du = g.zeros(g.sizes["n_torn"])
    g.assemble(du)
    g.factorize()
    sz = g.refresh_sizes()
    lam = torch.randn(sz["m"], dtype=torch.float64, device=g.device)
    q = torch.empty_like(lam)
    for _ in range(reps):
        g.fapply(lam, q)
    torch.cuda.synchronize()
    src = torch.ones(1 << 27, dtype=torch.float64, device=g.device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    fb = 8 if sz["precision"] == 0 else 4
    print(json.dumps({"probe": "counters", "fapply_reps": reps, "tile": sz["tile"], "schedule": sz["schedule"],
                      "skyline_bytes_per_apply": 2 * sz["skyline_entries"] * fb,
                      "stored_panel_bytes_per_apply": 2 * sz["factor_entries"] * fb,
                      "copy_bytes_each_way": src.numel() * 8}), flush=True)
    g.close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=29, help="timed load steps")
    ap.add_argument("--warmup", type=int, default=1, help="untimed load steps before them")
    ap.add_argument("--learned", default=None, help="safetensors weights of the warm-start network")
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--graph", type=int, default=1, help="replay the PCGP iteration from a HIP graph")
    ap.add_argument("--refine-eps", type=float, default=0.0, help="FP32 mode: inner PCGP tolerance")
    ap.add_argument("--fapply-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--counter-probe", action="store_true",
                    help="for hardware-counter runs: factorize once, run --fapply-reps F-applies and one "
                         "device copy of 1 GiB (the scale reference of the byte counters), print sizes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU decomposition is a design only)"}))
        return 2

    import torch

    import workloads as W
    from paper_1205_1926_amd import GpuSolver, _capi

    w = W.config(args.config, load_seed=0)
    log(f"setup {w.name} precision={args.precision}")
    t0 = time.perf_counter()
    g = GpuSolver(w, precision=args.precision, tile=args.tile, use_graph=args.graph, refine_eps=args.refine_eps)
    torch.cuda.synchronize()
    sz = g.sizes
    log(f"setup done in {time.perf_counter() - t0:.1f} s: {sz['n_sub']} subdomains, n={sz['n_torn']}, "
        f"m={sz['m']}, tile={sz['tile']}")

    if args.counter_probe:
        return counter_probe(g, args.fapply_reps)

    net = None
    if args.learned:
        from paper_1205_1926_amd.warmstart import WarmNet
        net = WarmNet.load(args.learned, device="cuda:0")

    def load_step():
        """Newton iterations to convergence and the commit; returns the
        reports of the iterations that solved."""
        from paper_1205_1926_amd.warmstart import run_step
        hist, _ = run_step(g, net=net)
        return hist

    for i in range(args.warmup):
        hist = load_step()
        log(f"warmup load step {g.k}: {len(hist)} Newton solves, pcg {[r['pcg_iters'] for r in hist]}")

    g.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for i in range(args.steps):
        hist = load_step()
        reps.extend(hist)
        log(f"load step {g.k}: " + ", ".join(
            f"it {r['iteration']}: pcg {r['pcg_iters']} ({r['warm_choice']}), refac {r['refactored']}, "
            f"pl {r['plastic_gp']}, {r['ms_total']:.1f} ms" for r in hist))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_ms, k_cnt = g.timing()
    graph_state = g.graph_active()
    g.set_timing(False)
    fapplies = sum(r["fapplies"] for r in reps)
    pcg_iters = sum(r["pcg_iters"] for r in reps)
    value = fapplies / elapsed
    sz = g.refresh_sizes()  # tile and schedule chosen by the autotuner

    # isolated F-apply throughput on the factors of the next load step's
    # first tangent (the committed state stays as it is)
    g.begin_load_step()
    g.assemble(g.zeros(sz["n_torn"]))
    g.factorize()
    lam = torch.randn(sz["m"], dtype=torch.float64, device="cuda:0")
    q = torch.empty_like(lam)
    g.fapply(lam, q)
    g.set_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.fapply_reps):
        g.fapply(lam, q)
    torch.cuda.synchronize()
    iso = (time.perf_counter() - t1) / args.fapply_reps
    iso_ms, iso_cnt = g.timing()
    g.set_timing(False)

    fbytes = 8 if args.precision == "fp64" else 4
    alg_bytes = 2 * sz["skyline_entries"] * fbytes
    if k_cnt == 0:
        raise SystemExit("no F-apply kernel was timed inside the timed region")
    mean_kernel_s = (k_ms / k_cnt) / 1e3
    achieved = alg_bytes / mean_kernel_s / 1e9
    iso_kernel_s = (iso_ms / max(iso_cnt, 1)) / 1e3
    log(f"timed: {fapplies} F-applies in {elapsed:.3f} s; solve kernel mean {mean_kernel_s * 1e3:.3f} ms "
        f"over {k_cnt}; isolated F-apply {iso * 1e3:.3f} ms (kernel {iso_kernel_s * 1e3:.3f} ms)")

    traffic = measured_traffic(w.name, args.precision, sz["tile"], sz["threads"])
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline()
        log(f"cpu baseline {cpu['value']:.3f} F-applies/s")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "F-applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / max(args.steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-factors/f64",
        "data": "synthetic",
        "config": {"workload": describe(w, sz),
                   "precision": args.precision, "tile": sz["tile"], "schedule": sz["schedule"],
                   "threads_per_subdomain": sz["threads"], "autotuned": sz["autotuned"], "preconditioner": "lumped",
                   "graph": bool(args.graph), "graph_active": graph_state,
                   "eps_pcg": w.eps_pcg, "eps_newton": w.eps_newton},
        "newton_step_ms": elapsed / max(len(reps), 1) * 1e3,
        "newton_solves": len(reps),
        "pcg_iters_total": pcg_iters,
        "pcg_iters_per_s": pcg_iters / elapsed,
        "fapplies_total": fapplies,
        "learned_warm_start": args.learned,
        "steps_detail": [{k: r[k] for k in ("iteration", "pcg_iters", "fapplies", "refactored", "restored", "warm_choice",
                                             "plastic_gp", "ms_assembly", "ms_factor", "ms_pcg", "ms_total")}
                         for r in reps],
        "fapply_isolated": {"ms": iso * 1e3, "kernel_ms": iso_kernel_s * 1e3,
                            "applies_per_s": 1.0 / iso,
                            "GB_s_algorithmic": alg_bytes / iso_kernel_s / 1e9},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_GBs": (traffic / mean_kernel_s / 1e9) if traffic else None,
                     "kernel": "ksolve_kernel (fused B^T scatter + forward/backward substitution)",
                     "bytes_per_launch": alg_bytes, "mean_kernel_ms": mean_kernel_s * 1e3,
                     "kernels_timed": k_cnt},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    g.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
