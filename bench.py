"""Benchmark: F-lambda applies/s and Newton-step time of the TFETI path on one GPU.

A step is one Newton iteration of the elastoplastic time stepping with a
linear solve: return map + tangent assembly at every Gauss point, fixing-node
regularization, batched band Cholesky, panel packing, and the whole PCGP
(Algorithm 3) with its F-applies, projections and lumped preconditioner.
When a load step converges (residual test, no solve) it is committed and the
next load step starts, so every timed step contains exactly one linear solve.

value = F-applies executed inside the K timed steps / wall time of the steps.
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--graph", type=int, default=1, help="replay the PCGP iteration from a HIP graph")
    ap.add_argument("--refine-eps", type=float, default=0.0, help="FP32 mode: inner PCGP tolerance")
    ap.add_argument("--fapply-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    state = {"active": False}

    def solve_step():
        """One Newton iteration with a linear solve; returns its report."""
        while True:
            if not state["active"]:
                g.begin_load_step()
                state["active"] = True
            rc, rep = g.newton_step()
            if rc == _capi.TFETI_CONVERGED or rc == _capi.TFETI_W_NEWTON_MAXIT:
                g.commit()
                state["active"] = False
                log(f"load step {g.k} converged")
                continue
            return rep

    for i in range(args.warmup):
        rep = solve_step()
        log(f"warmup step {i}: pcg {rep['pcg_iters']} it, {rep['ms_total']:.1f} ms")

    g.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for i in range(args.steps):
        rep = solve_step()
        reps.append(rep)
        log(f"step {i}: newton it {rep['iteration']}, pcg {rep['pcg_iters']} it, fapplies {rep['fapplies']}, "
            f"relres {rep['relres']:.2e}, plastic gp {rep['plastic_gp']}, {rep['ms_total']:.1f} ms "
            f"(assembly {rep['ms_assembly']:.1f}, factor {rep['ms_factor']:.1f}, pcg {rep['ms_pcg']:.1f})")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_ms, k_cnt = g.timing()
    g.set_timing(False)
    fapplies = sum(r["fapplies"] for r in reps)
    value = fapplies / elapsed

    # isolated F-apply throughput on the last factors
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
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-factors/f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: unit cube, {sz['n_sub']} box subdomains of 8^3 Q1 hexahedra, "
                               f"{sz['n_torn']} torn DOF, {sz['m']} multipliers, clamped bottom, top traction "
                               f"(compression + shear), load ramp over {w.steps} steps",
                   "precision": args.precision, "tile": sz["tile"], "preconditioner": "lumped",
                   "graph": bool(args.graph), "graph_active": g.graph_active(),
                   "eps_pcg": w.eps_pcg, "eps_newton": w.eps_newton},
        "newton_step_ms": elapsed / args.steps * 1e3,
        "pcg_iters": [r["pcg_iters"] for r in reps],
        "fapply_isolated": {"ms": iso * 1e3, "kernel_ms": iso_kernel_s * 1e3,
                            "applies_per_s": 1.0 / iso,
                            "GB_s_algorithmic": alg_bytes / iso_kernel_s / 1e9},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
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
