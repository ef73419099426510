"""TFETI dual solver: rigid modes, generalized inverse, projector, lumped and
Dirichlet preconditioners and the projected preconditioned CG (Algorithm 3).

Oracle (test infrastructure), float64, plain numpy/scipy.

Notation.  The paper sets N = -R^T B^T, e = -R^T f, H = (N N^T)^{-1}
(Algorithm 3).  Here G = R^T B^T = -N is used; the projector
P = I - N^T (N N^T)^{-1} N = I - G^T (G G^T)^{-1} G is the same matrix, and

    lambda_Im = N^T H e = G^T (G G^T)^{-1} R^T f,
    alpha     = H N (d - F lambda) = -(G G^T)^{-1} G (d - F lambda).

Generalized inverse (Remark 1: kernel basis and fixing nodes, no extra
fill-in).  The paper defers the construction to its references; the reading
used here: the fixing nodes of a box subdomain are three non-collinear corner
nodes of its last node layer, (0,0,nz), (nx,0,nz), (0,ny,nz); with R_S the
9 x 6 rows of R_p at their DOFs and Q an orthonormal basis of Im R_S,
K_reg = K_p + rho Q Q^T with rho = max_j K_p[j, j].  Since Q^T R_p is
nonsingular, K K_reg^{-1} K = K, i.e. K_reg^{-1} is a generalized inverse in
the sense of Section 4.2.  Its action is a banded Cholesky solve (the factor
keeps the band of K_p: the fixing nodes lie within one node layer).

Stopping test (Algorithm 3).  Read literally, the test sits after the update
and compares ||w^{j-1}|| with ||r^0||.  The reading used here tests right
after the projection, ||w^j|| <= eps * ||P(d - F lambda_Im)||: the reference
is the cold-start projected residual, which does not depend on the choice of
generalized inverse nor on a warm start.  Iterations are counted as F-applies
inside the loop.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def rigid_modes(sub) -> np.ndarray:
    """Orthonormal basis of the rigid body modes of a subdomain (n_p, 6).

    Columns: translations x, y, z, then rotations (-Y, X, 0), (0, -Z, Y),
    (Z, 0, -X) about the centroid of the subdomain nodes; each column is
    normalised and one modified Gram-Schmidt pass is applied."""
    X = sub.coords - sub.coords.mean(axis=0)
    n = sub.n_nodes
    R = np.zeros((n, 3, 6))
    R[:, 0, 0] = 1.0
    R[:, 1, 1] = 1.0
    R[:, 2, 2] = 1.0
    R[:, 0, 3], R[:, 1, 3] = -X[:, 1], X[:, 0]
    R[:, 1, 4], R[:, 2, 4] = -X[:, 2], X[:, 1]
    R[:, 0, 5], R[:, 2, 5] = X[:, 2], -X[:, 0]
    R = R.reshape(3 * n, 6)
    R /= np.linalg.norm(R, axis=0)[None, :]
    for j in range(6):
        for i in range(j):
            R[:, j] -= (R[:, i] @ R[:, j]) * R[:, i]
        R[:, j] /= np.linalg.norm(R[:, j])
    return R


def fixing_dofs(sub) -> np.ndarray:
    nx, ny, nz = sub.n
    ni, nj = nx + 1, ny + 1
    nodes = [0 + ni * (0 + nj * nz), nx + ni * (0 + nj * nz), 0 + ni * (ny + nj * nz)]
    return np.array([3 * a + c for a in nodes for c in range(3)], dtype=np.int64)


def regularize(Kp: sp.csr_matrix, Rp: np.ndarray, fix: np.ndarray) -> sp.csr_matrix:
    Rs = Rp[fix, :]                                   # (9, 6)
    Q, _ = np.linalg.qr(Rs)                           # (9, 6) orthonormal, Im Q = Im R_S
    rho = Kp.diagonal().max()
    blk = rho * (Q @ Q.T)
    rr = np.repeat(fix, 9)
    cc = np.tile(fix, 9)
    reg = sp.csr_matrix((blk.ravel(), (rr, cc)), shape=Kp.shape)
    return (Kp + reg).tocsr()


def lower_band(A: sp.spmatrix):
    """Lower banded storage ab[k, j] = A[j + k, j] (scipy's convention)."""
    C = sp.tril(A).tocoo()
    b = int((C.row - C.col).max()) if C.nnz else 0
    ab = np.zeros((b + 1, A.shape[0]))
    ab[C.row - C.col, C.col] = C.data
    return ab, b


class TFETI:
    def __init__(self, mesh):
        self.mesh = mesh
        self.B = mesh.B
        self.Bt = mesh.B.T.tocsr()
        self.R = [rigid_modes(s) for s in mesh.subs]
        self.fix = [fixing_dofs(s) for s in mesh.subs]
        s_cnt = len(mesh.subs)
        self.l = 6 * s_cnt
        blocks = [sp.csr_matrix(Rp) for Rp in self.R]
        self.Rmat = sp.block_diag(blocks, format="csr")          # (n, l)
        self.Gt = (self.B @ self.Rmat).tocsc()                   # G^T = B R  (m, l)
        self.G = self.Gt.T.tocsr()                               # (l, m)
        GGt = (self.G @ self.Gt).toarray()
        self.GGt = GGt
        self.GGt_fac = sla.cho_factor(GGt, lower=True)
        self.K = None

    # ------------------------------------------------------------- operators
    def set_matrix(self, K: sp.csr_matrix):
        """K: torn block-diagonal tangent (n, n).  Regularizes and factors."""
        self.K = K.tocsr()
        self.fac = []
        self.Kreg = []
        for s, Rp, fx in zip(self.mesh.subs, self.R, self.fix):
            sl = slice(s.off, s.off + s.n_dofs)
            Kp = self.K[sl, sl]
            Kr = regularize(Kp, Rp, fx)
            ab, b = lower_band(Kr)
            self.Kreg.append(Kr)
            self.fac.append(sla.cholesky_banded(ab, lower=True))

    def kplus(self, x: np.ndarray) -> np.ndarray:
        y = np.empty_like(x)
        for s, c in zip(self.mesh.subs, self.fac):
            sl = slice(s.off, s.off + s.n_dofs)
            y[sl] = sla.cho_solve_banded((c, True), x[sl])
        return y

    def F(self, lam: np.ndarray) -> np.ndarray:
        return self.B @ self.kplus(self.Bt @ lam)

    def coarse(self, v: np.ndarray) -> np.ndarray:
        return sla.cho_solve(self.GGt_fac, v)

    def project(self, w: np.ndarray) -> np.ndarray:
        return w - self.Gt @ self.coarse(self.G @ w)

    def precondition(self, w: np.ndarray) -> np.ndarray:
        """Lumped preconditioner B K B^T w (Section 4.2) with the unregularized K."""
        return self.B @ (self.K @ (self.Bt @ w))

    # ---------------------------------------------------- Dirichlet preconditioner
    def boundary_dofs(self, p: int) -> np.ndarray:
        """Local DOFs of subdomain p's boundary nodes: every DOF of a node that
        carries a gluing or Dirichlet row of B (Section 4.2: the nodes with
        imposed Dirichlet and gluing conditions).  The others are interior."""
        sub = self.mesh.subs[p]
        cols = self.B.indices[(self.B.indices >= sub.off) & (self.B.indices < sub.off + sub.n_dofs)] - sub.off
        nodes = np.unique(cols // 3)
        return (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()

    def schur_complements(self):
        """Dense Schur complements S_p = K_bb - K_bi K_ii^{-1} K_ib of the
        unregularized subdomain tangents onto their boundary DOFs."""
        out = []
        for p, sub in enumerate(self.mesh.subs):
            sl = slice(sub.off, sub.off + sub.n_dofs)
            Kp = self.K[sl, sl].toarray()
            b = self.boundary_dofs(p)
            i = np.setdiff1d(np.arange(sub.n_dofs), b)
            S = Kp[np.ix_(b, b)]
            if len(i):
                S = S - Kp[np.ix_(b, i)] @ np.linalg.solve(Kp[np.ix_(i, i)], Kp[np.ix_(i, b)])
            out.append((b, S))
        return out

    def precondition_dirichlet(self, w: np.ndarray) -> np.ndarray:
        """Dirichlet preconditioner Bbar Sbar Bbar^T w (Section 4.2): B^T w
        restricted to the boundary DOFs of each subdomain, multiplied by that
        subdomain's Schur complement, and gathered by B."""
        if getattr(self, "_schur_of", None) is not self.K:
            self._schur = self.schur_complements()
            self._schur_of = self.K
        x = self.Bt @ w
        y = np.zeros_like(x)
        for sub, (b, S) in zip(self.mesh.subs, self._schur):
            y[sub.off + b] = S @ x[sub.off + b]
        return self.B @ y

    # ------------------------------------------------------------- Algorithm 3
    def solve(self, f: np.ndarray, eps: float = 1e-8, maxit: int = 5000,
              lam_guess: np.ndarray | None = None, precond=True,
              record: bool = False):
        """Algorithm 3.  precond: True or "lumped" (B K B^T), "dirichlet"
        (Bbar Sbar Bbar^T), False or None (no preconditioner)."""
        if precond is True or precond == "lumped":
            apply_prec = self.precondition
        elif precond == "dirichlet":
            apply_prec = self.precondition_dirichlet
        else:
            apply_prec = None
        Rtf = self.Rmat.T @ f                                   # = -e
        lam_im = self.Gt @ self.coarse(Rtf)                     # N^T H e
        d = self.B @ self.kplus(f)
        d_tilde = d - self.F(lam_im)
        r_ref = np.linalg.norm(self.project(d_tilde))
        lam_ker = np.zeros(self.B.shape[0])
        r = d_tilde.copy()
        if lam_guess is not None:
            lam_ker = self.project(lam_guess)
            r = d_tilde - self.F(lam_ker)
        hist = []
        it = 0
        p = None
        yw_prev = None
        converged = False
        while True:
            w = self.project(r)
            nw = np.linalg.norm(w)
            if record:
                hist.append(nw)
            if nw <= eps * r_ref or r_ref == 0.0:
                converged = True
                break
            if it >= maxit:
                break
            z = apply_prec(w) if apply_prec else w
            y = self.project(z)
            yw = y @ w
            if p is None:
                p = y.copy()
            else:
                p = y + (yw / yw_prev) * p
            q = self.F(p)
            gamma = yw / (p @ q)
            lam_ker = lam_ker + gamma * p
            r = r - gamma * q
            yw_prev = yw
            it += 1
        lam = lam_im + lam_ker
        alpha = -self.coarse(self.G @ r)                        # H N (d - F lambda)
        u = self.kplus(f - self.Bt @ lam) + self.Rmat @ alpha
        return dict(lam=lam, alpha=alpha, u=u, iters=it, converged=converged,
                    r_ref=r_ref, hist=hist, lam_im=lam_im, d=d)
