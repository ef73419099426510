"""Pins of the oracle's TFETI solver (Section 4.2, Algorithm 3) against the
saddle-point system it must solve (dense brute force), the monolithic
Dirichlet-eliminated system, and the algebraic identities of the method:
orthonormal kernel basis, generalized inverse, projector, symmetry and
definiteness of F on Ker G, feasibility and equilibrium of the result, and
invariance to the choice of generalized inverse."""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import assembly
from oracle.mesh import Mesh
from oracle.tfeti import TFETI, regularize
import workloads as W


def elastic_problem(w):
    mesh = Mesh(w)
    ed = assembly.element_dofs_torn(mesh)
    ne = mesh.n_elems
    a = assembly.assemble(mesh, ed, mesh.n_torn, np.zeros(mesh.n_torn),
                          np.zeros((ne, 8, 6)), np.zeros((ne, 8)))
    tf = TFETI(mesh)
    tf.set_matrix(a["K"])
    return mesh, tf, a["K"], mesh.torn_load(1.0)


@pytest.fixture(scope="module")
def small():
    return elastic_problem(W.small_cube(S=(2, 2, 2), n=(2, 3, 2), amp=400.0, shear=100.0))


def test_rigid_modes_orthonormal_and_in_kernel(small):
    mesh, tf, K, f = small
    for s, R in zip(mesh.subs, tf.R):
        assert np.allclose(R.T @ R, np.eye(6), atol=1e-14)
        Kp = K[s.off:s.off + s.n_dofs, s.off:s.off + s.n_dofs]
        assert np.abs(Kp @ R).max() <= 1e-10 * abs(Kp).max()


def test_generalized_inverse_identity(small):
    mesh, tf, K, f = small
    s = mesh.subs[3]
    Kp = K[s.off:s.off + s.n_dofs, s.off:s.off + s.n_dofs].toarray()
    Kr = tf.Kreg[3].toarray()
    X = np.linalg.solve(Kr, Kp)
    assert np.abs(Kp @ X - Kp).max() <= 1e-9 * np.abs(Kp).max()
    # regularization adds only inside the existing band
    diff = (tf.Kreg[3] - sp.csr_matrix(Kp)).tocoo()
    bw = max(abs(i - j) for i, j in zip(*sp.csr_matrix(Kp).nonzero()))
    assert np.abs(diff.row - diff.col).max() <= bw


def test_projector_properties(small):
    mesh, tf, K, f = small
    rng = np.random.default_rng(1)
    x = rng.standard_normal(mesh.m)
    y = rng.standard_normal(mesh.m)
    Px = tf.project(x)
    assert np.allclose(tf.project(Px), Px, atol=1e-12)
    assert abs(Px @ y - x @ tf.project(y)) < 1e-10
    assert np.abs(tf.G @ Px).max() < 1e-12


def test_F_symmetric_positive_on_kerG(small):
    mesh, tf, K, f = small
    rng = np.random.default_rng(2)
    xs = [tf.project(rng.standard_normal(mesh.m)) for _ in range(4)]
    Fx = [tf.F(x) for x in xs]
    for i in range(4):
        assert xs[i] @ Fx[i] > 0
        for j in range(4):
            a, b = xs[i] @ Fx[j], xs[j] @ Fx[i]
            assert abs(a - b) <= 1e-10 * abs(a)


def test_tfeti_equals_dense_kkt(small):
    """The pair (u, lambda) must solve the saddle-point system of Section 4.2."""
    mesh, tf, K, f = small
    res = tf.solve(f, eps=1e-13)
    n, m = mesh.n_torn, mesh.m
    A = np.zeros((n + m, n + m))
    A[:n, :n] = K.toarray()
    A[:n, n:] = mesh.B.T.toarray()
    A[n:, :n] = mesh.B.toarray()
    rhs = np.concatenate([f, np.zeros(m)])
    x = np.linalg.solve(A, rhs)
    u, lam = x[:n], x[n:]
    assert np.linalg.norm(res["u"] - u) <= 1e-9 * np.linalg.norm(u)
    assert np.linalg.norm(res["lam"] - lam) <= 1e-8 * np.linalg.norm(lam)


def test_tfeti_invariants(small):
    mesh, tf, K, f = small
    res = tf.solve(f, eps=1e-12)
    u, lam = res["u"], res["lam"]
    assert np.linalg.norm(mesh.B @ u) <= 1e-10 * np.linalg.norm(u)
    g = tf.Rmat.T @ (f - mesh.B.T @ lam)
    assert np.abs(g).max() <= 1e-11 * np.abs(f).max()
    resid = K @ u - (f - mesh.B.T @ lam)
    assert np.linalg.norm(resid) <= 1e-8 * np.linalg.norm(f)
    assert res["converged"] and res["iters"] > 3


def test_tfeti_equals_monolithic():
    w = W.config(0)
    mesh, tf, K, f = elastic_problem(w)
    res = tf.solve(f, eps=1e-12)
    # monolithic: assemble the global stiffness, drop Dirichlet rows/columns
    eg = assembly.element_dofs_global(mesh)
    ne = mesh.n_elems
    ng = 3 * mesh.n_gnodes
    a = assembly.assemble(mesh, eg, ng, np.zeros(ng), np.zeros((ne, 8, 6)), np.zeros((ne, 8)))
    fg = np.zeros(ng)
    for s in mesh.subs:
        np.add.at(fg.reshape(-1, 3), s.l2g, f[s.off:s.off + s.n_dofs].reshape(-1, 3))
    free = ~mesh.dir_mask.ravel()
    Kf = a["K"][free][:, free].toarray()
    ug = np.zeros(ng)
    ug[free] = sla.solve(Kf, fg[free], assume_a="pos")
    ut = res["u"][mesh.untorn_index()]
    assert np.linalg.norm(ut - ug) <= 1e-9 * np.linalg.norm(ug)


def test_generalized_inverse_choice_invariance(small):
    """Fixing-node K_reg^{-1}, (K + rho R R^T)^{-1} and the Moore-Penrose
    pseudoinverse give the same lambda, u and PCGP iteration count."""
    mesh, tf, K, f = small
    ref = tf.solve(f, eps=1e-10)

    class Alt(TFETI):
        def __init__(self, base, mode):
            self.__dict__.update(base.__dict__)
            self.mode = mode
            self.inv = []
            for s, R in zip(mesh.subs, base.R):
                Kp = K[s.off:s.off + s.n_dofs, s.off:s.off + s.n_dofs].toarray()
                if mode == "pinv":
                    self.inv.append(np.linalg.pinv(Kp, rcond=1e-12))
                else:
                    rho = Kp.diagonal().max()
                    self.inv.append(np.linalg.inv(Kp + rho * R @ R.T))

        def kplus(self, x):
            y = np.empty_like(x)
            for s, Ai in zip(mesh.subs, self.inv):
                y[s.off:s.off + s.n_dofs] = Ai @ x[s.off:s.off + s.n_dofs]
            return y

    for mode in ("pinv", "rrT"):
        alt = Alt(tf, mode).solve(f, eps=1e-10)
        assert abs(alt["iters"] - ref["iters"]) <= 1
        assert np.linalg.norm(alt["lam"] - ref["lam"]) <= 1e-8 * np.linalg.norm(ref["lam"])
        assert np.linalg.norm(alt["u"] - ref["u"]) <= 1e-8 * np.linalg.norm(ref["u"])


def test_warm_start_reaches_same_solution(small):
    mesh, tf, K, f = small
    ref = tf.solve(f, eps=1e-10)
    rng = np.random.default_rng(3)
    guess = ref["lam"] + 1e-3 * np.linalg.norm(ref["lam"]) / np.sqrt(mesh.m) * rng.standard_normal(mesh.m)
    ws = tf.solve(f, eps=1e-10, lam_guess=guess)
    assert ws["iters"] < ref["iters"]
    assert np.linalg.norm(ws["u"] - ref["u"]) <= 1e-8 * np.linalg.norm(ref["u"])


def _strain_energy(mesh, u):
    """Sum over elements and Gauss points of w_g (B_g u_e)^T C (B_g u_e) for a
    torn displacement u: twice the elastic strain energy of u, formed per
    element from the Q1 strain matrices and the Hooke matrix alone (no
    assembled matrix)."""
    from oracle import constitutive, q1
    m = mesh.w.material
    Bg, wg = q1.strain_matrices(mesh.h)
    C = constitutive.hooke_matrix(m.E, m.nu)
    total = 0.0
    for s in mesh.subs:
        us = u[s.off:s.off + s.n_dofs].reshape(-1, 3)
        for el in s.elems:
            ue = us[el].ravel()
            for g in range(8):
                e = Bg[g] @ ue
                total += wg[g] * (e @ C @ e)
    return total


def _lumped_pin(mesh, apply_fn, seed=5):
    """v^T M w against the polarized interface strain energy
    1/2 (E(v + w) - E(v) - E(w)) of the torn fields B^T v, B^T w, and
    w^T M w against E(w), for the operator M = apply_fn."""
    rng = np.random.default_rng(seed)
    errs = []
    for _ in range(3):
        v = rng.standard_normal(mesh.m)
        w = rng.standard_normal(mesh.m)
        Ev, Ew, Evw = (_strain_energy(mesh, mesh.B.T @ x) for x in (v, w, v + w))
        errs.append(abs(w @ apply_fn(w) - Ew) / Ew)
        errs.append(abs(v @ apply_fn(w) - 0.5 * (Evw - Ev - Ew)) / Ew)
    return max(errs)


def test_lumped_preconditioner_is_interface_strain_energy():
    """Lumped preconditioner B K B^T (Section 4.2) with the unregularized
    elastic K: its quadratic and bilinear forms equal the strain energy of
    the torn fields B^T w summed element by element.  A variant that applies
    the regularized K_reg instead of K (the fixing-node term rho Q Q^T) fails
    the same pin."""
    w = W.small_cube(S=(2, 2, 1), n=(2, 2, 2), amp=400.0, shear=100.0)
    mesh, tf, K, f = elastic_problem(w)
    assert _lumped_pin(mesh, tf.precondition) <= 1e-12
    import scipy.sparse as sp
    Kreg = sp.block_diag(tf.Kreg, format="csr")
    wrong = lambda x: mesh.B @ (Kreg @ (mesh.B.T @ x))
    assert _lumped_pin(mesh, wrong) > 1e-3


# ---------------------------------------------------------------- Dirichlet preconditioner
def test_dirichlet_boundary_nodes_are_the_glued_and_clamped_faces():
    """Boundary nodes of a box subdomain (Section 4.2: nodes with gluing or
    Dirichlet conditions) are the nodes on faces shared with a neighbour or
    lying on the clamped face, read off the decomposition geometry."""
    w = W.small_cube(S=(3, 2, 2), n=(2, 3, 2), amp=400.0)
    mesh = Mesh(w)
    tf = TFETI(mesh)
    for p, sub in enumerate(mesh.subs):
        I, J, K = sub.IJK
        S = mesh.S
        ni, nj, nk = sub.n
        a = np.arange(sub.n_nodes)
        i, j, k = a % (ni + 1), (a // (ni + 1)) % (nj + 1), a // ((ni + 1) * (nj + 1))
        on = ((i == 0) & (I > 0)) | ((i == ni) & (I < S[0] - 1)) | ((j == 0) & (J > 0)) | \
             ((j == nj) & (J < S[1] - 1)) | ((k == 0) & (K > 0)) | ((k == nk) & (K < S[2] - 1)) | \
             ((k == 0) & (K == 0))                                   # clamped bottom face
        expect = (3 * a[on][:, None] + np.arange(3)[None, :]).ravel()
        assert np.array_equal(tf.boundary_dofs(p), expect), p


def test_dirichlet_schur_complement_is_harmonic_extension(small):
    """S x_b = (K x)_b for the harmonic extension x = (x_b, x_i) of x_b,
    with x_i found by CG on K_ii x_i = -K_ib x_b (a different route than the
    oracle's dense solve), and x_b^T S x_b is the least energy x^T K x over
    all extensions of x_b."""
    import scipy.sparse.linalg as spla
    mesh, tf, K, f = small
    rng = np.random.default_rng(8)
    for p, (b, S) in enumerate(tf.schur_complements()):
        sub = mesh.subs[p]
        Kp = K[sub.off:sub.off + sub.n_dofs, sub.off:sub.off + sub.n_dofs].tocsr()
        i = np.setdiff1d(np.arange(sub.n_dofs), b)
        xb = rng.standard_normal(len(b))
        x = np.zeros(sub.n_dofs)
        x[b] = xb
        xi, info = spla.cg(Kp[i][:, i], -(Kp[i][:, b] @ xb), rtol=1e-14, maxiter=5000)
        assert info == 0
        x[i] = xi
        Kx = Kp @ x
        assert np.abs(S @ xb - Kx[b]).max() <= 1e-9 * np.abs(Kx[b]).max()
        e0 = xb @ S @ xb
        for _ in range(3):
            y = x.copy()
            y[i] += 1e-3 * np.abs(xi).max() * rng.standard_normal(len(i))
            assert y @ (Kp @ y) > e0
        assert S.shape == (len(b), len(b)) and np.allclose(S, S.T, atol=1e-9 * np.abs(S).max())


def test_dirichlet_equals_lumped_when_every_node_is_on_the_boundary():
    """Subdomains of one element inside a box clamped on all faces: every
    node carries a row of B, no DOF is interior, S = K and the two
    preconditioners coincide."""
    w = W.small_cube(S=(2, 2, 2), n=(1, 1, 1), amp=400.0)
    w.dirichlet = [[1, 1, 1] for _ in range(6)]
    mesh, tf, K, f = elastic_problem(w)
    rng = np.random.default_rng(9)
    x = rng.standard_normal(mesh.m)
    assert np.abs(tf.precondition_dirichlet(x) - tf.precondition(x)).max() <= 1e-12 * np.abs(tf.precondition(x)).max()


def test_dirichlet_pcgp_fewer_iterations_same_solution():
    """With the Dirichlet preconditioner PCGP reaches the lumped solution in
    fewer iterations (the paper's Table 1 reports fewer iterations for it)."""
    w = W.config(0)
    mesh, tf, K, f = elastic_problem(w)
    lum = tf.solve(f, eps=1e-10, precond="lumped")
    dir_ = tf.solve(f, eps=1e-10, precond="dirichlet")
    assert dir_["converged"] and dir_["iters"] < lum["iters"]
    assert np.linalg.norm(dir_["u"] - lum["u"]) <= 1e-8 * np.linalg.norm(lum["u"])
    assert np.linalg.norm(dir_["lam"] - lum["lam"]) <= 1e-7 * np.linalg.norm(lum["lam"])
