"""Thin Python binding over the C ABI: torch tensors provide device memory and
the stream; every step of the method runs in the HIP library."""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as A


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class GpuSolver:
    """Handle-owning wrapper.  ``workload`` is a ``workloads.Workload``."""

    def __init__(self, workload, device: str = "cuda:0", stream=None, **opts):
        torch = _torch()
        self.lib = A.load()
        self.w = workload
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise A.TfetiError("the TFETI library runs on a GPU device only")
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        prob, self._keep = A.make_problem(workload)
        opt = A.make_options(workload, **opts)
        self.options = opt
        h = C.c_void_p()
        rc = self.lib.tfeti_setup(C.byref(prob), C.byref(opt), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self.h = h
        if rc < 0:
            msg = self.lib.tfeti_last_error(h).decode() if h.value else "setup failed"
            if h.value:
                self.lib.tfeti_destroy(h)
            self.h = None
            raise A.TfetiError(f"tfeti_setup: {rc}: {msg}")
        self.refresh_sizes()
        self.k = 0

    # ------------------------------------------------------------------ plumbing
    def _check(self, rc, what):
        if rc < 0:
            raise A.TfetiError(f"{what}: {rc}: {self.lib.tfeti_last_error(self.h).decode()}")
        return rc

    def refresh_sizes(self):
        """Re-read the sizes (tile and schedule change when the autotuner runs
        at the first factorization)."""
        s = A.Sizes()
        self._check(self.lib.tfeti_get_sizes(self.h, C.byref(s)), "get_sizes")
        self.sizes = A.struct_dict(s)
        return self.sizes

    def zeros(self, n, dtype=None):
        torch = _torch()
        return torch.zeros(int(n), dtype=dtype or torch.float64, device=self.device)

    def close(self):
        if getattr(self, "h", None):
            self.lib.tfeti_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ maps
    def B_host(self):
        nnz = C.c_int64()
        self._check(self.lib.tfeti_get_B_host(self.h, C.byref(nnz), None, None, None), "get_B")
        m = self.sizes["m"]
        rp = np.zeros(m + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int64)
        val = np.zeros(nnz.value, dtype=np.float64)
        self._check(self.lib.tfeti_get_B_host(self.h, C.byref(nnz), rp.ctypes.data_as(C.c_void_p),
                                              col.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p)),
                    "get_B")
        return rp, col, val

    # ------------------------------------------------------------------ building blocks
    def assemble(self, du):
        fint = self.zeros(self.sizes["n_torn"])
        cnt = C.c_int64()
        self._check(self.lib.tfeti_assemble(self.h, _ptr(du), _ptr(fint), C.byref(cnt)), "assemble")
        return fint, cnt.value

    def factorize(self):
        self._check(self.lib.tfeti_factorize(self.h), "factorize")

    def fapply(self, lam, out=None):
        q = out if out is not None else self.zeros(self.sizes["m"])
        self._check(self.lib.tfeti_fapply(self.h, _ptr(lam), _ptr(q)), "fapply")
        return q

    def kplus(self, x):
        y = self.zeros(self.sizes["n_torn"])
        self._check(self.lib.tfeti_kplus(self.h, _ptr(x), _ptr(y)), "kplus")
        return y

    def project(self, w):
        out = self.zeros(self.sizes["m"])
        self._check(self.lib.tfeti_project(self.h, _ptr(w), _ptr(out)), "project")
        return out

    def precondition(self, w):
        out = self.zeros(self.sizes["m"])
        self._check(self.lib.tfeti_precondition(self.h, _ptr(w), _ptr(out)), "precondition")
        return out

    def dual_pcg(self, f, guess=None):
        lam = self.zeros(self.sizes["m"])
        u = self.zeros(self.sizes["n_torn"])
        rep = A.PcgReport()
        rc = self._check(self.lib.tfeti_dual_pcg(self.h, _ptr(f), _ptr(guess), _ptr(lam), _ptr(u), C.byref(rep)),
                         "dual_pcg")
        return lam, u, A.struct_dict(rep), rc

    def lam(self):
        out = self.zeros(self.sizes["m"])
        self._check(self.lib.tfeti_get_lambda(self.h, _ptr(out)), "get_lambda")
        return out

    # ------------------------------------------------------------------ state
    def state(self):
        torch = _torch()
        n_gp, n = self.sizes["n_gp"], self.sizes["n_torn"]
        out = dict(sigma=self.zeros(6 * n_gp), kappa=self.zeros(n_gp), u=self.zeros(n), du=self.zeros(n),
                   dsigma=self.zeros(6 * n_gp), dkappa=self.zeros(n_gp),
                   plastic=self.zeros(n_gp, dtype=torch.uint8))
        self._check(self.lib.tfeti_get_state(self.h, *[_ptr(out[k]) for k in
                                                       ("sigma", "kappa", "u", "du", "dsigma", "dkappa", "plastic")]),
                    "get_state")
        return out

    def set_state(self, sigma=None, kappa=None, u=None, du=None):
        self._check(self.lib.tfeti_set_state(self.h, _ptr(sigma), _ptr(kappa), _ptr(u), _ptr(du)), "set_state")

    # ------------------------------------------------------------------ time stepping
    def begin_load_step(self, dlf=None):
        if dlf is None:
            dlf = self.w.load_factor(self.k + 1) - self.w.load_factor(self.k)
        self._check(self.lib.tfeti_begin_load_step(self.h, C.c_double(dlf)), "begin_load_step")

    def newton_step(self):
        rep = A.NewtonReport()
        rc = self._check(self.lib.tfeti_newton_step(self.h, C.byref(rep)), "newton_step")
        return rc, A.struct_dict(rep)

    def commit(self):
        self._check(self.lib.tfeti_commit_load_step(self.h), "commit")
        self.k += 1

    def load_step(self):
        """Newton iterations until convergence, then commit.  Returns the
        reports of the iterations that solved."""
        self.begin_load_step()
        hist = []
        while True:
            rc, rep = self.newton_step()
            if rc == A.TFETI_CONVERGED:
                break
            hist.append(rep)
            if rc == A.TFETI_W_NEWTON_MAXIT:
                break
        self.commit()
        return hist

    def run(self, steps=None):
        n = self.w.steps if steps is None else steps
        return [self.load_step() for _ in range(n)]

    # ------------------------------------------------------------------ learned warm start
    def warm_nodes(self) -> int:
        n = C.c_int64()
        self._check(self.lib.tfeti_warm_nodes(self.h, C.byref(n)), "warm_nodes")
        return n.value

    def warm_features(self, lam_prev, dload, X=None, M=None, want_mask=True):
        """Features (n x 31, FP32) of every interface node; mask (n x 21) if wanted."""
        torch = _torch()
        n = self.warm_nodes()
        if X is None:
            X = torch.empty((n, 31), dtype=torch.float32, device=self.device)
        if want_mask and M is None:
            M = torch.empty((n, 21), dtype=torch.float32, device=self.device)
        self._check(self.lib.tfeti_warm_features(self.h, _ptr(lam_prev), C.c_double(dload), _ptr(X),
                                                 _ptr(M) if want_mask else None), "warm_features")
        return X, M

    def warm_targets(self, lam_prev, lam_next, dload, T=None):
        torch = _torch()
        if T is None:
            T = torch.empty((self.warm_nodes(), 21), dtype=torch.float32, device=self.device)
        self._check(self.lib.tfeti_warm_targets(self.h, _ptr(lam_prev), _ptr(lam_next), C.c_double(dload),
                                                _ptr(T)), "warm_targets")
        return T

    def warm_candidate(self, lam_prev, Y, dload, out=None):
        if out is None:
            out = self.zeros(self.sizes["m"])
        self._check(self.lib.tfeti_warm_candidate(self.h, _ptr(lam_prev), _ptr(Y), C.c_double(dload), _ptr(out)),
                    "warm_candidate")
        return out

    def set_learned_guess(self, lam):
        self._check(self.lib.tfeti_set_learned_guess(self.h, _ptr(lam)), "set_learned_guess")

    def converged_lambda(self):
        lam = self.zeros(self.sizes["m"])
        ok = C.c_int32()
        self._check(self.lib.tfeti_get_converged_lambda(self.h, _ptr(lam), C.byref(ok)), "get_converged_lambda")
        return lam, bool(ok.value)

    def load_increment(self, k=None):
        k = self.k if k is None else k
        return self.w.load_factor(k + 1) - self.w.load_factor(k)

    # ------------------------------------------------------------------ timing
    def set_timing(self, on: bool):
        self._check(self.lib.tfeti_set_timing(self.h, 1 if on else 0), "set_timing")

    def graph_active(self) -> int:
        """0 not captured, 1 replaying a HIP graph, 2 capture failed (eager)."""
        return int(self.lib.tfeti_graph_status(self.h))

    def timing(self):
        ms = C.c_double()
        cnt = C.c_int64()
        self._check(self.lib.tfeti_get_timing(self.h, C.byref(ms), C.byref(cnt)), "get_timing")
        return ms.value, cnt.value

    def timing_bytes(self) -> float:
        """Algorithmic bytes of the F-apply kernels that timing() counts."""
        b = C.c_double()
        self._check(self.lib.tfeti_get_timing_bytes(self.h, C.byref(b)), "get_timing_bytes")
        return b.value


def model_host(workload, tile: int = 0):
    """Host-only model build (no GPU): sizes and B in CSR."""
    lib = A.load()
    prob, keep = A.make_problem(workload)
    s = A.Sizes()
    nnz = C.c_int64()
    rc = lib.tfeti_model_host(C.byref(prob), tile, C.byref(s), C.byref(nnz), None, None, None)
    if rc < 0:
        raise A.TfetiError(f"tfeti_model_host: {rc}: {lib.tfeti_last_error(None).decode()}")
    sizes = A.struct_dict(s)
    rp = np.zeros(sizes["m"] + 1, dtype=np.int64)
    col = np.zeros(nnz.value, dtype=np.int64)
    val = np.zeros(nnz.value, dtype=np.float64)
    rc = lib.tfeti_model_host(C.byref(prob), tile, C.byref(s), C.byref(nnz), rp.ctypes.data_as(C.c_void_p),
                              col.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p))
    if rc < 0:
        raise A.TfetiError(f"tfeti_model_host: {rc}: {lib.tfeti_last_error(None).decode()}")
    return sizes, rp, col, val


def return_map(material, sigma_k, kappa_k, deps, want_tangent=True, stream=None):
    """Stateless return map on device tensors (FP64)."""
    torch = _torch()
    lib = A.load()
    n = kappa_k.numel()
    dev = sigma_k.device
    ds = torch.empty(6 * n, dtype=torch.float64, device=dev)
    dk = torch.empty(n, dtype=torch.float64, device=dev)
    D = torch.empty(36 * n, dtype=torch.float64, device=dev) if want_tangent else None
    pl = torch.empty(n, dtype=torch.uint8, device=dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    mat = A.Material(material.E, material.nu, material.sigma_y, material.H)
    rc = lib.return_map(C.byref(mat), n, _ptr(sigma_k), _ptr(kappa_k), _ptr(deps), _ptr(ds), _ptr(dk), _ptr(D),
                        _ptr(pl), C.c_void_p(st.cuda_stream))
    if rc < 0:
        raise A.TfetiError(f"return_map: {rc}")
    return ds, dk, D, pl
