"""The benchmark's stdout record: one short JSON line with the contract's
fields (value, ms_per_step, steps, dtype, config.workload, roofline,
cpu_baseline, Newton-step time, errors against the oracle), built from the
full record bench.py writes to stderr."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


class _W:
    name = "cube10x10x10_sub8"
    steps = 30


def _full():
    legs = {n: {"value": 800.0 - i, "ms_per_step": 290.0, "newton_step_ms": 49.0 + i, "pcg_iters": 4300,
                "solves": 119, "kernel_ms": 0.69, "frac": 0.77}
            for i, n in enumerate(("fp32_all", "fp64_plain", "fp64_graph_warm", "fp64_dirichlet", "fp32_learned"))}
    return {
        "metric": bench.METRIC, "value": 803.72, "unit": "F-applies/s", "n_gpus": 1, "steps": 20, "warmup": 1,
        "ms_per_step": 290.77, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": "long text " * 30, "form": "fp32_all", "tile": 32, "threads": 256,
                   "graph_active": 1, "learned": False},
        "newton_step_ms": 48.87, "pcg_iters_per_s": 738.4, "fapply_isolated_ms": 0.699,
        "roofline": {"bound": "hbm", "achieved": 6178.6, "peak": 8000.0, "unit": "GB/s", "frac": 0.772,
                     "traffic": 4.5675e9, "kernel": "ksolve_kernel", "mean_kernel_ms": 0.693,
                     "kernels_timed": 1070},
        "legs": legs,
        "rel_error_vs_oracle": {"load_step": 1, "u": {n: 1e-10 * (i + 1) for i, n in enumerate(legs)},
                                "lam": {n: 1e-9 * (i + 1) for i, n in enumerate(legs)}, "oracle_pcg_iters": 25,
                                "u_after_timed_vs_fp64_plain": {"fp32_all": 2e-10, "fp64_dirichlet": 3e-10}},
        "cpu_baseline": {"value": 39.4, "unit": "F-applies/s", "cores": 15, "kind": "oracle", "sample": "x" * 300,
                         "cpu": "AMD EPYC", "nproc": 16, "per_core_fapplies_s": 2.6,
                         "oracle_full_size_1core": {"fapply_s": 0.27, "pcg_iter_s": 0.42, "newton_step_s": 24.1,
                                                    "factorization_s": 11.1, "cores": 1}},
        "newton_step_speedup_vs_fp64_plain": 2.13,
    }


def test_compact_record_is_short_and_complete():
    full = _full()
    rec = bench.compact(full, "fp32_all", {"n_sub": 1000, "n_torn": 2187000, "m": 612360}, _W)
    text = json.dumps(bench.rounded(rec), separators=(",", ":"), ensure_ascii=False)
    assert "\n" not in text and len(text.encode()) < 1400, len(text.encode())
    back = json.loads(text)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "newton_step_ms", "pcg_iters_per_s"):
        assert back[k] == bench.rounded(full)[k], k
    assert back["config"]["workload"].startswith("cube10x10x10_sub8: 1000 box subdomains")
    rf = back["roofline"]
    assert set(rf) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    cpu = back["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["cores"] == 15 and cpu["sample"]
    assert cpu["full_size_1core_s"]["newton_step_s"] == 24.1
    err = back["rel_error_vs_oracle"]
    assert err["u"] == 1e-10 and err["u_max_legs"] == 5e-10 and err["lam_max_legs"] == 5e-9
    assert err["u_after_timed_vs_fp64_plain"] == 3e-10
    assert back["legs"]["fp64_plain"] == [799.0, 50.0]
