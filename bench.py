"""Benchmark: F-lambda applies/s and Newton-step time of the TFETI path on one GPU.

A step is one load step of the elastoplastic time stepping (Algorithm 4):
Newton iterations until convergence, each with the return map and tangent
assembly at every Gauss point, fixing-node regularization, batched band
Cholesky of the subdomains whose tangent changed, panel packing and the whole
PCGP (Algorithm 3) with its F-applies, projections and lumped preconditioner;
then the commit.  Default workload: the 10x10x10 cube of 8^3-element
subdomains; W untimed load steps, then K timed ones.

The same load steps run in several forms (legs), each on a fresh handle
(default: fp32_hybrid, fp32_all, fp64_plain, fp64_graph_warm,
fp64_dirichlet, fp32_learned, fp64_explicit):
  fp32_hybrid     the headline line: FP32 inner PCGP with FP64 outer dual
                  refinement, warm start, PCGP iteration replayed from a HIP
                  graph; each F-apply in one launch applies the explicit
                  local operator of every subdomain that keeps its elastic
                  factor and the FP32 factor sweeps to the others;
  fp32_all        the same with the factor sweeps for every subdomain
                  (--learned adds the learned warm-start candidate);
  fp32_learned    fp32_all with the learned warm-start candidate of the
                  network in the package (trained on the uneven 8x8x8 mesh);
  fp64_plain      FP64 factors, cold start, eager launches (plain GPU TFETI);
  fp64_graph_warm FP64 factors with the warm start and the graph;
  fp64_dirichlet, fp32_dirichlet  the same with the Dirichlet preconditioner
                  Bbar Sbar Bbar^T instead of the lumped one (Section 4.2);
  fp64_explicit, fp32_explicit, fp64_hybrid  the explicit operators for
                  every subdomain (formed at each factorization), or the
                  hybrid launch, in FP64 or FP32.

value = F-applies inside the timed load steps of the headline leg / their
wall time; newton_step_ms = wall time / Newton iterations with a solve.
roofline: the headline leg's subdomain-solve kernel of the F-apply;
algorithmic bytes per launch = two passes over the envelope of each factor
it solves with plus the stored tiles of each explicit operator it applies
(as the library counts them for the timed launches), divided by the
kernel's mean duration from HIP events on the library's stream over the
timed region; traffic (FETCH_SIZE + WRITE_SIZE) only for the factor sweeps'
kernel, as measured.
rel_error_vs_oracle: displacements and multipliers of load step 1 of every
leg against the FP64 oracle at full size (computed in a child process that
runs beside the GPU legs), and the headline leg's displacements after the
timed steps against the plain FP64 leg's.
cpu_baseline: the oracle's F-apply on a sample of 8 subdomains of the same
shape, run by one process per host core at once and scaled to the whole
mesh; plus the oracle's full-size single-core timings of load step 1.

One compact JSON line goes to stdout; the full record, progress and
per-iteration detail go to stderr (and, with --detail PATH, the detail to a
JSON file).

--plate LEVEL runs the notched-plate benchmark instead (the box stand-in for
the paper's Section 5 plate with a hole): time discretizations (a) one step
and (b) eight steps to t = 1/4, one stderr row per Newton iteration (PCGP
iterations, plastic elements, increment criterion, relative residual, time)
and one JSON line with the totals and the two discretizations' final plastic
element counts.
"""

from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "F·λ applies/s (HBM GB/s) + Newton-step time at 1e-6 rel. error vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
LEGS = {
    "fp32_all": dict(precision="fp32", use_graph=1, warm_start=1),
    "fp64_plain": dict(precision="fp64", use_graph=0, warm_start=0),
    "fp64_graph_warm": dict(precision="fp64", use_graph=1, warm_start=1),
    "fp64_dirichlet": dict(precision="fp64", use_graph=1, warm_start=1, preconditioner=2),
    "fp32_dirichlet": dict(precision="fp32", use_graph=1, warm_start=1, preconditioner=2),
    "fp32_learned": dict(precision="fp32", use_graph=1, warm_start=1),
    # explicit local dual operators in place of the factor sweeps (formed at
    # every factorization of a subdomain)
    "fp64_explicit": dict(precision="fp64", use_graph=1, warm_start=1, fapply_format="explicit"),
    "fp32_explicit": dict(precision="fp32", use_graph=1, warm_start=1, fapply_format="explicit"),
    # in one launch: operators for the subdomains that keep their elastic
    # factor, factor sweeps for the others
    "fp32_hybrid": dict(precision="fp32", use_graph=1, warm_start=1, fapply_format="hybrid"),
    "fp64_hybrid": dict(precision="fp64", use_graph=1, warm_start=1, fapply_format="hybrid"),
}
# the learned candidate of the fp32_learned leg (and of fp32_all with --learned)
DEFAULT_WEIGHTS = os.path.join(ROOT, "paper_1205_1926_amd", "weights", "warmstart_cube8x8x8_uneven.safetensors")
SAMPLE_S, SAMPLE_N = (2, 2, 2), (8, 8, 8)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cores() -> int:
    """Host cores this run may use: the box's share of 16 per GPU, or fewer."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def single_thread_env() -> dict:
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        env[k] = "1"
    return env


# ---------------------------------------------------------------------- CPU legs (oracle)
def cpu_worker(seconds: float) -> int:
    """One baseline process: the oracle's F-apply, PCGP and factorization on
    the 2x2x2 sample of 8^3-element subdomains with the benchmark's element
    size, single-threaded.  Prints one JSON line."""
    import numpy as np

    import workloads as W
    from oracle import reference
    from oracle.tfeti import TFETI
    from oracle.mesh import Mesh

    w = W.small_cube(S=SAMPLE_S, n=SAMPLE_N, amp=400.0)
    w.extent = tuple(0.1 * s for s in SAMPLE_S)   # 1/80 elements, as in the 10^3 x 8^3 cube
    mesh = Mesh(w)
    K = reference.elastic_tangent_blocks(mesh)
    tf = TFETI(mesh)
    t0 = time.perf_counter()
    tf.set_matrix(K)
    t_fact = time.perf_counter() - t0
    lam = np.random.default_rng(0).standard_normal(mesh.m)
    tf.F(lam)
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        tf.F(lam)
        n += 1
    t_f = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = tf.solve(mesh.torn_load(1.0 / 30.0), eps=w.eps_pcg)
    t_s = time.perf_counter() - t0
    print(json.dumps({"applies": n, "seconds": t_f, "nsub": len(mesh.subs), "fact_s": t_fact,
                      "solve_s": t_s, "iters": res["iters"]}), flush=True)
    return 0


def oracle_reference(config: int, out: str) -> int:
    """Child process: load step 1 of the workload on the FP64 oracle at full
    size; writes du (untorn), lambda, the untorn index and timings."""
    import numpy as np

    import workloads as W
    from oracle import reference

    t0 = time.perf_counter()
    r = reference.elastic_first_step(W.config(config), fapply_seed=0,
                                     log=lambda m: print(f"[oracle-ref] {m}", file=sys.stderr, flush=True))
    idx = r["untorn"]
    t = r["times"]
    np.savez(out, du=r["du"][idx], lam=r["lam"], untorn=idx, iters=r["iters"], relres=r["relres"],
             times=json.dumps(t), wall=time.perf_counter() - t0)
    return 0


def cpu_baseline_start(workers: int, seconds: float):
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", str(seconds)]
    return [subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, env=single_thread_env(),
                             cwd=ROOT, text=True) for _ in range(workers)]


def cpu_baseline_finish(procs, ncells: int):
    rows = []
    for p in procs:
        outp, _ = p.communicate()
        if p.returncode == 0 and outp.strip():
            rows.append(json.loads(outp.strip().splitlines()[-1]))
    if not rows:
        return None
    rate = sum(r["applies"] * r["nsub"] / r["seconds"] for r in rows) / ncells
    per_core = rate / len(rows)
    r0 = rows[0]
    return {"value": rate, "unit": "F-applies/s", "cores": len(rows), "kind": "oracle",
            "sample": f"oracle F-apply (scipy banded Cholesky solves, 1 BLAS thread) on 2x2x2 subdomains of 8^3 "
                      f"Q1 elements in each of {len(rows)} processes at once for {r0['seconds']:.0f} s, "
                      f"subdomain solves per second summed and divided by the {ncells} subdomains of the mesh",
            "per_core_fapplies_s": per_core,
            "sample_pcg_iter_s": r0["solve_s"] / max(r0["iters"], 1),
            "sample_factor_s_per_subdomain": r0["fact_s"] / r0["nsub"],
            "cpu": cpu_model(), "nproc": os.cpu_count()}


# ---------------------------------------------------------------------- GPU legs
def describe(w, sz) -> str:
    """The workload in words: mesh, decomposition, sizes and load."""
    sub = ("8^3" if set(w.nx) | set(w.ny) | set(w.nz) == {8}
           else f"{min(w.nx + w.ny + w.nz)}..{max(w.nx + w.ny + w.nz)} elements per axis")
    top = w.traction[5]
    load = " + ".join(t for t, v in (("x shear", top[0]), ("y shear", top[1]), ("z traction", top[2])) if v)
    return (f"{w.name}: unit cube of Q1 hexahedra, {sz['n_sub']} box subdomains of {sub}, {sz['n_torn']} torn DOF, "
            f"{sz['m']} multipliers, clamped bottom, top face {load}, load ramp over {w.steps} steps")


def compact(line: dict, head: str, sz: dict, w) -> dict:
    """The stdout record: the full one's headline fields, short."""
    out = {k: line[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                                "higher_is_better", "scaling", "vs_baseline", "dtype", "data")}
    cfg = dict(line["config"])
    cfg["workload"] = (f"{w.name}: {sz['n_sub']} box subdomains, {sz['n_torn']} torn DOF, {sz['m']} multipliers, "
                       f"load ramp over {w.steps} steps")
    out["config"] = cfg
    for k in ("newton_step_ms", "pcg_iters_per_s", "fapply_isolated_ms"):
        out[k] = line[k]
    rf = line["roofline"]
    out["roofline"] = {k: rf[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
    out["legs"] = {n: [r["value"], r["newton_step_ms"]] for n, r in line["legs"].items()}
    acc = line["rel_error_vs_oracle"]
    if acc:
        err = {"load_step": acc.get("load_step")}
        for k in ("u", "lam"):
            if isinstance(acc.get(k), dict) and acc[k]:
                err[k] = acc[k].get(head)
                err[k + "_max_legs"] = max(v for v in acc[k].values() if v is not None)
        after = acc.get("u_after_timed_vs_fp64_plain")
        if after:
            err["u_after_timed_vs_fp64_plain"] = max(after.values())
        out["rel_error_vs_oracle"] = err
    cpu = line["cpu_baseline"]
    if cpu:
        c = {k: cpu[k] for k in ("value", "unit", "cores", "kind", "cpu", "nproc") if k in cpu}
        c["sample"] = "oracle F-apply of 2x2x2 subdomains of 8^3 in each process, scaled to 1000 subdomains"
        full = cpu.get("oracle_full_size_1core")
        if full:
            c["full_size_1core_s"] = {k: full[k] for k in ("fapply_s", "pcg_iter_s", "newton_step_s")}
        out["cpu_baseline"] = c
    if "newton_step_speedup_vs_fp64_plain" in line:
        out["newton_step_speedup_vs_fp64_plain"] = line["newton_step_speedup_vs_fp64_plain"]
    return out


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
                      "threads": sz["threads"], "skyline_bytes_per_apply": 2 * sz["skyline_entries"] * fb,
                      "stored_panel_bytes_per_apply": 2 * sz["factor_entries"] * fb,
                      "explicit_bytes_per_apply": sz["explicit_bytes"],
                      "copy_bytes_each_way": src.numel() * 8}), flush=True)
    g.close()
    return 0


def run_leg(name, w, args, net, detail):
    """Warmup and timed load steps of one form on a fresh handle."""
    import torch

    from paper_1205_1926_amd import GpuSolver
    from paper_1205_1926_amd.warmstart import run_step

    opts = LEGS[name]
    t0 = time.perf_counter()
    g = GpuSolver(w, tile=args.tile, refine_eps=args.refine_eps, **opts)
    torch.cuda.synchronize()
    sz = g.sizes
    log(f"{name}: setup in {time.perf_counter() - t0:.1f} s ({sz['n_sub']} subdomains, n={sz['n_torn']}, "
        f"m={sz['m']})")
    leg_net = net if name in ("fp32_all", "fp32_learned") else None
    first = None

    def step():
        hist, _ = run_step(g, net=leg_net)
        detail.setdefault(name, []).append([{k: r[k] for k in ("iteration", "pcg_iters", "fapplies", "refactored",
                                                                "restored", "warm_choice", "plastic_gp",
                                                                "ms_assembly", "ms_factor", "ms_pcg",
                                                                "ms_total")} for r in hist])
        return hist

    for i in range(args.warmup):
        hist = step()
        if g.k == 1:
            st = g.state()
            first = dict(u=st["u"].cpu().numpy(), lam=g.lam().cpu().numpy(), solves=len(hist),
                         plastic=sum(r["plastic_gp"] for r in hist))
        log(f"{name}: warmup load step {g.k}: pcg {[r['pcg_iters'] for r in hist]}")
    g.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for i in range(args.steps):
        hist = step()
        reps.extend(hist)
        log(f"{name}: load step {g.k}: " + ", ".join(
            f"pcg {r['pcg_iters']} ({r['warm_choice']}) {r['ms_total']:.0f} ms" for r in hist))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_ms, k_cnt = g.timing()
    k_bytes = g.timing_bytes()
    graph_state = g.graph_active()
    g.set_timing(False)
    u_final = g.state()["u"].cpu().numpy()
    sz = g.refresh_sizes()
    # isolated F-apply throughput on the factors of the next load step's
    # first tangent (the committed state stays as it is)
    g.begin_load_step()
    g.assemble(g.zeros(sz["n_torn"]))
    g.factorize()
    lam = torch.randn(sz["m"], dtype=torch.float64, device=g.device)
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
    iso_bytes = g.timing_bytes()
    g.set_timing(False)
    g.close()
    # algorithmic bytes of one F-apply: both sweeps over the factor envelope,
    # or the stored lower triangles of the explicit operators
    # algorithmic bytes per F-apply launch, as the library counts them for
    # the timed launches: both sweeps over the factor envelopes, or the
    # stored operator tiles, or (hybrid) the mix of each factorization
    alg = k_bytes / k_cnt if k_cnt > 0 else iso_bytes / max(iso_cnt, 1)
    iso_kernel_s = iso_ms / max(iso_cnt, 1) / 1e3
    if k_cnt > 0:
        kernel_s, src = k_ms / k_cnt / 1e3, "timed load steps"
    else:
        # no PCGP iteration in the timed window: the isolated F-applies
        kernel_s, src, k_cnt = iso_kernel_s, "isolated F-applies (no PCGP iteration was timed)", iso_cnt
    fapplies = sum(r["fapplies"] for r in reps)
    pcg = sum(r["pcg_iters"] for r in reps)
    res = dict(name=name, sizes=sz, elapsed=elapsed, fapplies=fapplies, pcg=pcg, solves=len(reps),
               kernel_s=kernel_s, kernel_src=src, kernels_timed=k_cnt, alg_bytes=alg, iso=iso,
               iso_kernel_s=iso_kernel_s, graph=graph_state, first=first, u_final=u_final,
               precision=opts["precision"])
    log(f"{name}: {fapplies} F-applies, {pcg} PCGP iterations, {len(reps)} Newton solves in {elapsed:.3f} s; "
        f"solve kernel {kernel_s * 1e3:.3f} ms ({alg / kernel_s / 1e12:.2f} TB/s algorithmic) over {k_cnt}; "
        f"isolated F-apply {iso * 1e3:.3f} ms")
    return res


def plate_run(args) -> int:
    """The notched-plate benchmark (the box stand-in for the paper's Section 5
    plate, Tables 2 and 3): both time discretizations, (a) one step and (b)
    eight steps to t = 1/4, on the GPU.  One row per Newton iteration on
    stderr (load step, iteration, PCGP iterations, plastic elements, the
    increment criterion, relative residual, time) and one JSON line with the
    totals; the two discretizations' final plastic zones are compared (the
    paper finds them almost equal)."""
    import torch

    import workloads as W
    from paper_1205_1926_amd import GpuSolver
    from paper_1205_1926_amd import _capi as A

    opts = LEGS[args.plate_form]
    out = {"metric": "notched plate: Newton iterations, PCGP iterations, plastic elements and wall time per "
                     "time discretization", "form": args.plate_form, "level": args.plate,
           "eps_newton": args.plate_eps[0], "eps_pcg": args.plate_eps[1]}
    for disc, steps in (("a", 1), ("b", 8)):
        w = W.plate_notch(args.plate, steps=steps, eps_newton=args.plate_eps[0], eps_pcg=args.plate_eps[1])
        g = GpuSolver(w, tile=args.tile, **opts)
        torch.cuda.synchronize()
        sz = g.sizes
        if disc == "a":
            out["workload"] = (f"{w.name.rsplit('_n', 1)[0]}: {sz['n_sub']} box subdomains, {sz['n_elem']} "
                               f"elements, {sz['n_torn']} torn DOF, {sz['m']} multipliers")
        log(f"plate ({disc}): {steps} load steps; step  it  pcg  plastic_el  crit  relres  ms")
        t0 = time.perf_counter()
        newton = pcg = 0
        for k in range(steps):
            # Newton iterations one call at a time, each reported as it ends
            g.begin_load_step()
            while True:
                rc, r = g.newton_step()
                if rc == A.TFETI_CONVERGED:
                    break
                newton += 1
                pcg += r["pcg_iters"]
                log(f"plate ({disc}) {k + 1:2d} {r['iteration']:2d} {r['pcg_iters']:4d} {r['plastic_elements']:7d} "
                    f"{r['crit']:.2e} {r['relres']:.2e} {r['ms_total']:.1f}")
                if rc == A.TFETI_W_NEWTON_MAXIT:
                    log(f"plate ({disc}): load step {k + 1} stopped at the Newton iteration limit")
                    break
            g.commit()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        kappa = g.state()["kappa"].reshape(-1, 8)
        plastic = int((kappa > 0).any(dim=1).sum().item())
        umax = float(g.state()["u"].abs().max().item())
        g.close()
        out[disc] = {"steps": steps, "newton": newton, "pcg": pcg, "plastic_el": plastic, "u_max": rounded(umax),
                     "seconds": rounded(elapsed)}
    out["plastic_spread"] = rounded(abs(out["a"]["plastic_el"] - out["b"]["plastic_el"]) /
                                    max(out["b"]["plastic_el"], 1))
    print(json.dumps(out, separators=(",", ":")), flush=True)
    return 0


def rel(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rounded(x, digits=5):
    """Floats to `digits` significant digits (keeps the JSON line short)."""
    if isinstance(x, float):
        return float(f"{x:.{digits}g}")
    if isinstance(x, dict):
        return {k: rounded(v, digits) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [rounded(v, digits) for v in x]
    return x


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed load steps")
    ap.add_argument("--warmup", type=int, default=1, help="untimed load steps before them (at least 1)")
    ap.add_argument("--learned", default=None, help="safetensors weights of the warm-start network (fp32_all leg)")
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--legs", default="fp32_hybrid,fp32_all,fp64_plain,fp64_graph_warm,fp64_dirichlet,fp32_learned,"
                                      "fp64_explicit",
                    help="comma-separated forms; the first is the headline line")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--refine-eps", type=float, default=0.0, help="FP32 mode: inner PCGP tolerance")
    ap.add_argument("--fapply-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle", action="store_true", help="skip the full-size oracle accuracy leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--detail", default=None, help="write per-iteration reports of every leg to this JSON file")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32"],
                    help="with --counter-probe: the factor precision")
    ap.add_argument("--fapply-format", default="factors", choices=["factors", "explicit", "hybrid"],
                    help="with --counter-probe: the F-apply format")
    ap.add_argument("--counter-probe", action="store_true",
                    help="for hardware-counter runs: factorize once, run --fapply-reps F-applies and one "
                         "device copy of 1 GiB (the scale reference of the byte counters), print sizes")
    ap.add_argument("--plate", type=int, default=None,
                    help="run the notched-plate benchmark at this mesh level instead (both discretizations)")
    ap.add_argument("--plate-form", default="fp64_graph_warm", help="leg options used by --plate")
    ap.add_argument("--plate-eps", default="1e-9,1e-12", help="--plate: Newton and PCGP tolerances")
    ap.add_argument("--cpu-worker", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--oracle-ref", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker is not None:
        return cpu_worker(args.cpu_worker)
    if args.oracle_ref is not None:
        return oracle_reference(args.config, args.oracle_ref)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(the multi-GPU decomposition is a design only)"}), flush=True)
        return 2
    legs = [l for l in args.legs.split(",") if l]
    if not legs or any(l not in LEGS for l in legs):
        raise SystemExit(f"--legs: choose from {sorted(LEGS)}")
    args.warmup = max(1, args.warmup)
    if args.plate is not None:
        if args.plate_form not in LEGS or args.plate_form == "fp32_learned":
            raise SystemExit(f"--plate-form: choose from {sorted(set(LEGS) - {'fp32_learned'})}")
        args.plate_eps = [float(x) for x in args.plate_eps.split(",")]
        return plate_run(args)

    import workloads as W
    w = W.config(args.config, load_seed=0)
    if args.counter_probe:
        from paper_1205_1926_amd import GpuSolver
        g = GpuSolver(w, precision=args.precision or "fp64", tile=args.tile, use_graph=1,
                      fapply_format=args.fapply_format)
        return counter_probe(g, args.fapply_reps)

    # child processes start before anything touches the GPU
    tmp = tempfile.mkdtemp(prefix="bench_")
    ref_path = os.path.join(tmp, "oracle_ref.npz")
    ref_proc = None
    if not args.no_oracle:
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = "2"
        ref_proc = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-ref", ref_path,
                                     "--config", str(args.config)], env=env, cwd=ROOT)
        log(f"oracle reference of load step 1 started (pid {ref_proc.pid})")
    cpu = None
    ncells = w.S[0] * w.S[1] * w.S[2]
    if not args.no_cpu_baseline:
        workers = max(1, host_cores() - (1 if ref_proc else 0))
        log(f"cpu baseline: {workers} oracle processes for {args.cpu_seconds:.0f} s ...")
        cpu = cpu_baseline_finish(cpu_baseline_start(workers, args.cpu_seconds), ncells)
        if cpu:
            log(f"cpu baseline: {cpu['value']:.3f} F-applies/s of the whole mesh on {cpu['cores']} cores "
                f"({cpu['cpu']})")

    import numpy as np
    import torch

    nets = {}
    if args.learned or "fp32_learned" in legs:
        from paper_1205_1926_amd.warmstart import WarmNet
        if args.learned:
            nets["fp32_all"] = WarmNet.load(args.learned, device="cuda:0")
        if "fp32_learned" in legs:
            nets["fp32_learned"] = WarmNet.load(args.learned or DEFAULT_WEIGHTS, device="cuda:0")
    detail = {}
    results = {}
    for name in legs:
        results[name] = run_leg(name, w, args, nets.get(name), detail)
    if args.detail:
        with open(args.detail, "w") as fh:
            json.dump(detail, fh)

    # accuracy: load step 1 against the oracle, the headline leg against plain FP64 after the timed steps
    acc = {"load_step": 1}
    full_1core = None
    if ref_proc is not None:
        log("waiting for the oracle reference ...")
        rc = ref_proc.wait()
        if rc == 0 and os.path.exists(ref_path):
            ref = np.load(ref_path)
            idx = ref["untorn"]
            acc["u"] = {n: rel(r["first"]["u"][idx], ref["du"]) for n, r in results.items() if r["first"]}
            acc["lam"] = {n: rel(r["first"]["lam"], ref["lam"]) for n, r in results.items()
                          if r["first"] and r["first"]["solves"] == 1}
            acc["oracle_pcg_iters"] = int(ref["iters"])
            t = json.loads(str(ref["times"]))
            full_1core = {"fapply_s": t.get("fapply"), "pcg_iter_s": t["solve"] / max(int(ref["iters"]), 1),
                          "newton_step_s": t["assembly"] + t["factorization"] + t["solve"] + t["return_map"],
                          "factorization_s": t["factorization"], "cores": 1}
            log(f"oracle reference: {json.dumps(acc)}")
        else:
            log(f"oracle reference failed (exit {rc})")
    head = results[legs[0]]
    if "fp64_plain" in results:
        acc["u_after_timed_vs_fp64_plain"] = {n: rel(r["u_final"], results["fp64_plain"]["u_final"])
                                              for n, r in results.items() if n != "fp64_plain"}
    if cpu is not None and full_1core is not None:
        cpu["oracle_full_size_1core"] = full_1core

    sz = head["sizes"]
    kernel_s = head["kernel_s"]
    achieved = head["alg_bytes"] / kernel_s / 1e9
    # (measured for the factor sweeps' kernel; none for the other formats)
    traffic = (measured_traffic(w.name, head["precision"], sz["tile"], sz["threads"])
               if LEGS[legs[0]].get("fapply_format", "factors") == "factors" else None)
    newton_ms = {n: r["elapsed"] / max(r["solves"], 1) * 1e3 for n, r in results.items()}
    line = {
        "metric": METRIC,
        "value": head["fapplies"] / head["elapsed"],
        "unit": "F-applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["elapsed"] / max(args.steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head["precision"] == "fp64" else "f32/f64",
        "data": "synthetic",
        "config": {"workload": describe(w, sz), "form": legs[0], "tile": sz["tile"], "threads": sz["threads"],
                   "graph_active": head["graph"], "learned": bool(args.learned and legs[0] == "fp32_all")},
        "newton_step_ms": newton_ms[legs[0]],
        "pcg_iters_per_s": head["pcg"] / head["elapsed"],
        "fapply_isolated_ms": head["iso"] * 1e3,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "ksolve_kernel", "mean_kernel_ms": kernel_s * 1e3,
                     "kernels_timed": head["kernels_timed"]},
        "legs": {n: {"value": r["fapplies"] / r["elapsed"], "ms_per_step": r["elapsed"] / max(args.steps, 1) * 1e3,
                     "newton_step_ms": newton_ms[n], "pcg_iters": r["pcg"], "solves": r["solves"],
                     "kernel_ms": r["kernel_s"] * 1e3, "frac": r["alg_bytes"] / r["kernel_s"] / 1e9 / HBM_PEAK_GBS}
                 for n, r in results.items()},
        "rel_error_vs_oracle": acc,
        "cpu_baseline": cpu,
    }
    if "fp64_plain" in results and legs[0] != "fp64_plain":
        line["newton_step_speedup_vs_fp64_plain"] = newton_ms["fp64_plain"] / newton_ms[legs[0]]
    # everything on stderr; on stdout one short line with the same headline
    # fields, the legs as [F-applies/s, Newton-step ms] and the errors as
    # the headline leg's and the largest over the legs
    log("full result: " + json.dumps(rounded(line), separators=(",", ":"), ensure_ascii=False))
    print(json.dumps(rounded(compact(line, legs[0], sz, w)), separators=(",", ":"), ensure_ascii=False), flush=True)
    try:
        os.remove(ref_path)
        os.rmdir(tmp)
    except OSError:
        pass
    return 0


if __name__ == "__main__":
    sys.exit(main())
