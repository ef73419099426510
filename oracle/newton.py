"""Semismooth Newton (Algorithms 2 and 4) and time stepping (Algorithm 1).

Oracle (test infrastructure), float64.

Two linear solvers are available for the Newton systems:
* "tfeti": the torn system solved by Algorithm 3 (``oracle.tfeti``);
* "mono":  the plain definition the TFETI solution must reproduce: the
  global stiffness with the Dirichlet rows and columns removed
  (Section 3.1, the restricted system), solved by banded Cholesky.

Newton stopping.  The paper's test (Algorithm 2 / Algorithm 4) is the
relative increment ||du_i - du_{i-1}|| / (||du_i|| + ||du_{i-1}||).  With a
dual solver stopped at a relative tolerance eps_PCG, the increments never fall
much below eps_PCG times the size of the torn interface forces (the solver's
error appears as a jump of du across interfaces, not as a residual), so an
increment tolerance below eps_PCG cannot be met.  The reading used here stops
on the relative residual of the assembled system on free DOFs,
||r(du_{i-1})|| / ||df|| <= eps_Newton, tested at the start of iteration i >= 2
(before any solve); the paper's increment criterion is recorded alongside,
with norms over untorn global DOFs (each DOF once, its lowest-numbered
subdomain copy).  The paper's test is available as criterion="increment".

Commit (Algorithm 1 / Problem 2): the stress and hardening increments added
to sigma_k, kappa_k are those evaluated at the converged displacement
increment.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import assembly
from .mesh import Mesh
from .tfeti import TFETI, lower_band


class Solver:
    def __init__(self, workload, linear: str = "tfeti", eps_pcg: float | None = None,
                 eps_newton: float | None = None, max_newton: int = 50, max_pcg: int = 5000):
        self.w = workload
        self.mesh = Mesh(workload)
        self.linear = linear
        self.eps_pcg = workload.eps_pcg if eps_pcg is None else eps_pcg
        self.eps_newton = workload.eps_newton if eps_newton is None else eps_newton
        self.max_newton = max_newton
        self.max_pcg = max_pcg
        m = self.mesh
        self.ne = m.n_elems
        self.sigma = np.zeros((self.ne, 8, 6))
        self.kappa = np.zeros((self.ne, 8))
        self.edofs_t = assembly.element_dofs_torn(m)
        self.edofs_g = assembly.element_dofs_global(m)
        self.untorn = m.untorn_index()
        self.f1_torn = m.torn_load(1.0)
        self.n_global = 3 * m.n_gnodes
        # free global DOFs: not fixed, and of a node in some subdomain
        self.free = ~m.dir_mask.ravel() & np.repeat(m.used, 3)
        if linear == "tfeti":
            self.tf = TFETI(m)
            self.u = np.zeros(m.n_torn)
        else:
            self.tf = None
            self.u = np.zeros(self.n_global)
            self.f1_global = self._assemble_global_load()
        self.k = 0
        self.lam_prev = None

    # ------------------------------------------------------------------ helpers
    def _assemble_global_load(self) -> np.ndarray:
        fg = np.zeros(self.n_global)
        for s in self.mesh.subs:
            fs = self.f1_torn[s.off:s.off + s.n_dofs].reshape(-1, 3)
            np.add.at(fg.reshape(-1, 3), s.l2g, fs)
        return fg

    def untorn_of(self, v: np.ndarray) -> np.ndarray:
        return v[self.untorn] if self.linear == "tfeti" else v

    def global_displacement(self) -> np.ndarray:
        return self.untorn_of(self.u)

    def plastic_elements(self, plastic_gp: np.ndarray) -> int:
        return int(np.count_nonzero(plastic_gp.any(axis=1)))

    # ------------------------------------------------------------------ one load step
    def load_step(self, record: bool = False, criterion: str = "residual"):
        """Solve load step k -> k+1 (Algorithm 4 / Algorithm 2).

        Each iteration i assembles at the current increment du_{i-1}
        (return map, internal force, tangent), then solves for the correction
        and updates du.  Stopping:
        * "residual" (default): before solving at iteration i >= 2, stop if
          ||assembled residual on free DOFs|| / ||df on free DOFs|| <= eps_Newton.
          The commit then uses the increments of that final assembly, which
          are exactly the increments at the converged du (Algorithm 1).
        * "increment": the paper's relative increment test after the update;
          the commit re-evaluates the increments at the converged du.
        The paper's increment criterion is recorded in both modes.
        Returns a history list with one dict per iteration that solved.
        """
        k = self.k
        dlf = self.w.load_factor(k + 1) - self.w.load_factor(k)
        df = dlf * (self.f1_torn if self.linear == "tfeti" else self.f1_global)
        du = np.zeros_like(self.u)
        hist = []
        dfn = self._assembled_norm(df)
        lam_guess = None
        final = None
        for i in range(1, self.max_newton + 1):
            a = self._assemble(du)
            f = df - a["fint"]
            relres = self._assembled_norm(f) / dfn if dfn > 0 else 0.0
            if criterion == "residual" and i >= 2 and relres <= self.eps_newton:
                final = a
                break
            delta, info = self._solve(a, f, lam_guess)
            du_new = du + delta
            a_ = self.untorn_of(du_new)
            b_ = self.untorn_of(du)
            crit = np.linalg.norm(a_ - b_) / (np.linalg.norm(a_) + np.linalg.norm(b_))
            h = dict(i=i, crit=crit, relres=relres, pcg_iters=info["pcg_iters"],
                     plastic_gp=int(np.count_nonzero(a["plastic"])),
                     plastic_el=self.plastic_elements(a["plastic"]))
            if record:
                h["info"] = info
                h["assembly"] = a
                h["du_before"] = du.copy()
            hist.append(h)
            du = du_new
            if criterion == "increment" and crit <= self.eps_newton:
                break
        if final is None:
            final = self._assemble(du, want_K=False)
        self.sigma = self.sigma + final["dsigma"]
        self.kappa = self.kappa + final["dkappa"]
        self.u = self.u + du
        self.last_du = du
        self.k += 1
        return hist

    def _assemble(self, du, want_K: bool = True):
        if self.linear == "tfeti":
            return assembly.assemble(self.mesh, self.edofs_t, self.mesh.n_torn, du,
                                     self.sigma, self.kappa, want_K=want_K)
        return assembly.assemble(self.mesh, self.edofs_g, self.n_global, du,
                                 self.sigma, self.kappa, want_K=want_K)

    def _assembled_norm(self, v: np.ndarray) -> float:
        """Norm of a force vector summed over subdomain copies, free DOFs only."""
        if self.linear != "tfeti":
            return float(np.linalg.norm(v[self.free]))
        rg = np.zeros(self.n_global)
        for s in self.mesh.subs:
            np.add.at(rg.reshape(-1, 3), s.l2g, v[s.off:s.off + s.n_dofs].reshape(-1, 3))
        return float(np.linalg.norm(rg[self.free]))

    def _solve(self, a, f, lam_guess=None):
        if self.linear == "tfeti":
            self.tf.set_matrix(a["K"])
            res = self.tf.solve(f, eps=self.eps_pcg, maxit=self.max_pcg, lam_guess=lam_guess)
            return res["u"], dict(pcg_iters=res["iters"], pcg=res, f=f)
        free = self.free
        Kr = a["K"][free][:, free]
        ab, _ = lower_band(Kr)
        c = sla.cholesky_banded(ab, lower=True)
        x = np.zeros(self.n_global)
        x[free] = sla.cho_solve_banded((c, True), f[free])
        return x, dict(pcg_iters=0, f=f)

    def run(self, steps: int | None = None, record: bool = False):
        n = self.w.steps if steps is None else steps
        return [self.load_step(record=record) for _ in range(n)]
