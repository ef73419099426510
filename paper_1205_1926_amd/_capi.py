"""ctypes declarations of the C ABI in include/tfeti.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtfeti.so")

TFETI_OK = 0
TFETI_CONVERGED = 1
TFETI_W_PCG_MAXIT = 2
TFETI_W_NEWTON_MAXIT = 3
TFETI_W_WARMSTART_REJECTED = 4
TFETI_E_INVALID = -1
TFETI_E_HIP = -2
TFETI_E_OOM = -3
TFETI_E_NOT_SPD = -4
PREC_FP64 = 0
PREC_FP32 = 1
FAPPLY_FACTORS = 0
FAPPLY_EXPLICIT = 1
FAPPLY_HYBRID = 2


class Material(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("sigma_y", C.c_double), ("H", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("S", C.c_int32 * 3), ("n_host", C.POINTER(C.c_int32) * 3), ("extent", C.c_double * 3),
                ("mat", Material), ("dirichlet", (C.c_int32 * 3) * 6), ("traction", (C.c_double * 3) * 6),
                ("absent_host", C.POINTER(C.c_uint8))]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("preconditioner", C.c_int32), ("eps_pcg", C.c_double),
                ("eps_newton", C.c_double), ("max_pcg", C.c_int32), ("max_newton", C.c_int32),
                ("warm_start", C.c_int32), ("use_graph", C.c_int32), ("tile", C.c_int32),
                ("refine_eps", C.c_double), ("check_every", C.c_int32), ("refactor_all", C.c_int32),
                ("fapply_format", C.c_int32), ("pad", C.c_int32)]


class PcgReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("fapplies", C.c_int32), ("converged", C.c_int32), ("outer", C.c_int32),
                ("r_ref", C.c_double), ("r_final", C.c_double), ("ms", C.c_double),
                ("warm_choice", C.c_int32), ("pad", C.c_int32)]


class NewtonReport(C.Structure):
    _fields_ = [("iteration", C.c_int32), ("pcg_iters", C.c_int32), ("fapplies", C.c_int32),
                ("plastic_gp", C.c_int32), ("plastic_elements", C.c_int32), ("relres", C.c_double),
                ("crit", C.c_double), ("ms_assembly", C.c_double), ("ms_factor", C.c_double),
                ("ms_pcg", C.c_double), ("ms_total", C.c_double), ("warm_choice", C.c_int32),
                ("refactored", C.c_int32), ("restored", C.c_int32), ("pad", C.c_int32)]


class Sizes(C.Structure):
    _fields_ = [("n_sub", C.c_int64), ("n_torn", C.c_int64), ("m", C.c_int64), ("m_G", C.c_int64),
                ("m_U", C.c_int64), ("l", C.c_int64), ("n_elem", C.c_int64), ("n_gp", C.c_int64),
                ("n_gdof", C.c_int64), ("skyline_entries", C.c_int64), ("factor_entries", C.c_int64),
                ("factor_bytes", C.c_int64), ("tile", C.c_int32), ("precision", C.c_int32),
                ("schedule", C.c_int32), ("autotuned", C.c_int32), ("threads", C.c_int32), ("pad", C.c_int32),
                ("explicit_bytes", C.c_int64)]


class Mlp(C.Structure):
    _fields_ = [("d_in", C.c_int32), ("d_h", C.c_int32), ("d_out", C.c_int32)] + [
        (name, C.c_void_p * 3) for name in ("W", "b", "Wb", "gW", "gb", "mW", "vW", "mb", "vb")]


def struct_dict(s) -> dict:
    return {k: getattr(s, k) for k, _ in s._fields_}


P = C.c_void_p
I32, I64, D = C.c_int32, C.c_int64, C.c_double

# name -> (restype, argtypes); every symbol declared in include/tfeti.h
SIGNATURES = {
    "tfeti_setup": (I32, [C.POINTER(Problem), C.POINTER(Options), P, C.POINTER(P)]),
    "tfeti_destroy": (None, [P]),
    "tfeti_last_error": (C.c_char_p, [P]),
    "tfeti_get_sizes": (I32, [P, C.POINTER(Sizes)]),
    "tfeti_get_B_host": (I32, [P, C.POINTER(I64), P, P, P]),
    "tfeti_begin_load_step": (I32, [P, D]),
    "tfeti_newton_step": (I32, [P, C.POINTER(NewtonReport)]),
    "tfeti_commit_load_step": (I32, [P]),
    "tfeti_dual_pcg": (I32, [P, P, P, P, P, C.POINTER(PcgReport)]),
    "tfeti_assemble": (I32, [P, P, P, C.POINTER(I64)]),
    "tfeti_factorize": (I32, [P]),
    "tfeti_fapply": (I32, [P, P, P]),
    "tfeti_kplus": (I32, [P, P, P]),
    "tfeti_project": (I32, [P, P, P]),
    "tfeti_precondition": (I32, [P, P, P]),
    "tfeti_get_state": (I32, [P, P, P, P, P, P, P, P]),
    "tfeti_set_state": (I32, [P, P, P, P, P]),
    "tfeti_get_lambda": (I32, [P, P]),
    "tfeti_set_timing": (I32, [P, I32]),
    "tfeti_get_timing": (I32, [P, C.POINTER(D), C.POINTER(I64)]),
    "tfeti_get_timing_bytes": (I32, [P, C.POINTER(D)]),
    "tfeti_graph_status": (I32, [P]),
    "tfeti_model_host": (I32, [C.POINTER(Problem), I32, C.POINTER(Sizes), C.POINTER(I64), P, P, P]),
    "return_map": (I32, [C.POINTER(Material), I64, P, P, P, P, P, P, P, P]),
    "tfeti_warm_nodes": (I32, [P, C.POINTER(I64)]),
    "tfeti_warm_features": (I32, [P, P, D, P, P]),
    "tfeti_warm_targets": (I32, [P, P, P, D, P]),
    "tfeti_warm_candidate": (I32, [P, P, P, D, P]),
    "tfeti_set_learned_guess": (I32, [P, P]),
    "tfeti_get_converged_lambda": (I32, [P, P, C.POINTER(I32)]),
    "tfeti_mlp_work_size": (I32, [C.POINTER(Mlp), I64, C.POINTER(I64)]),
    "tfeti_mlp_sync_bf16": (I32, [C.POINTER(Mlp), P]),
    "tfeti_mlp_forward": (I32, [C.POINTER(Mlp), I64, P, P, P, P]),
    "tfeti_mlp_forward_noalloc": (I32, [C.POINTER(Mlp), I64, P, P, P]),
    "tfeti_mlp_loss_grad": (I32, [C.POINTER(Mlp), I64, P, P, P, P, P, P, P]),
    "tfeti_mlp_adam": (I32, [C.POINTER(Mlp), I32, C.c_float, C.c_float, C.c_float, C.c_float, P]),
}

_lib = None


class TfetiError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load libtfeti.so and declare its signatures.  Raises if it is missing:
    there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise TfetiError(f"{path} is missing: build it with paper_1205_1926_amd.build.build()")
    # torch brings its own HIP runtime; load it first so that the library
    # binds to the same one instead of starting a second runtime
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def make_problem(w):
    """tfeti_problem from a workloads.Workload; returns (problem, keepalive)."""
    prob = Problem()
    keep = []
    for a, arr in enumerate((w.nx, w.ny, w.nz)):
        prob.S[a] = len(arr)
        buf = (C.c_int32 * len(arr))(*arr)
        keep.append(buf)
        prob.n_host[a] = C.cast(buf, C.POINTER(C.c_int32))
        prob.extent[a] = w.extent[a]
    m = w.material
    prob.mat = Material(m.E, m.nu, m.sigma_y, m.H)
    for f in range(6):
        for c in range(3):
            prob.dirichlet[f][c] = int(w.dirichlet[f][c])
            prob.traction[f][c] = float(w.traction[f][c])
    absent = getattr(w, "absent", None)
    if absent:
        S = [len(w.nx), len(w.ny), len(w.nz)]
        flags = (C.c_uint8 * (S[0] * S[1] * S[2]))()
        for (I, J, K) in absent:
            if not (0 <= I < S[0] and 0 <= J < S[1] and 0 <= K < S[2]):
                raise ValueError(f"absent box {(I, J, K)} outside the {S[0]} x {S[1]} x {S[2]} decomposition")
            flags[I + S[0] * (J + S[1] * K)] = 1
        keep.append(flags)
        prob.absent_host = C.cast(flags, C.POINTER(C.c_uint8))
    return prob, keep


def make_options(w=None, precision=None, eps_pcg=None, eps_newton=None, preconditioner=1, max_pcg=5000,
                 max_newton=50, warm_start=1, use_graph=0, tile=0, refine_eps=0.0, check_every=8,
                 refactor_all=0, fapply_format=0):
    o = Options()
    prec = precision if precision is not None else (w.precision if w is not None else "fp64")
    o.precision = PREC_FP32 if prec in ("fp32", PREC_FP32) else PREC_FP64
    o.preconditioner = preconditioner
    o.eps_pcg = eps_pcg if eps_pcg is not None else (w.eps_pcg if w is not None else 1e-8)
    o.eps_newton = eps_newton if eps_newton is not None else (w.eps_newton if w is not None else 1e-10)
    o.max_pcg = max_pcg
    o.max_newton = max_newton
    o.warm_start = warm_start
    o.use_graph = use_graph
    o.tile = tile
    o.refine_eps = refine_eps
    o.check_every = check_every
    o.refactor_all = refactor_all
    o.fapply_format = {"factors": FAPPLY_FACTORS, "explicit": FAPPLY_EXPLICIT, "hybrid": FAPPLY_HYBRID}.get(
        fapply_format, fapply_format)
    return o
