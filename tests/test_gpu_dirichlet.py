"""GPU parity of the Dirichlet preconditioner Bbar Sbar Bbar^T (Section 4.2,
options.preconditioner = 2) against the oracle's dense Schur complements.

The library never forms Sbar: it applies K_tt x - K_ti K_ii^{-1} K_it x with
banded Cholesky factors of the interior blocks, so single applications are
compared entry by entry (FP64 rounding amplified by the condition numbers of
K_ii, 1e3-1e4 here: tested at 1e-9 of the largest entry), and whole solves
at the displacement bar 1e-6 and 1e-5 for the multipliers.
"""

import numpy as np
import pytest

import workloads as W
from oracle import assembly
from oracle.mesh import Mesh
from oracle.newton import Solver as OracleSolver
from oracle.tfeti import TFETI

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1205_1926_amd import load
    load()
    return torch.device("cuda:0")


def T(x, dev):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def N(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def emax(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def uneven():
    w = W.Workload("uneven", (2, 3, 2), [3, 5], [2, 4, 3], [6, 2],
                   dirichlet=[[0, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0], [1, 1, 1], [0, 0, 0]])
    w.traction[5] = [50.0, 0.0, -300.0]
    return w


CASES = {
    "cube2x2x2_sub4": lambda: (W.config(0), False),
    "plastic": lambda: (W.small_cube(S=(2, 2, 2), n=(3, 3, 3), amp=700.0, shear=150.0, steps=2), True),
    "uneven": lambda: (uneven(), False),
    "rollers": lambda: (W.patch_test(S=(2, 1, 2), n=(2, 3, 2), q=300.0), False),
}


class DPair:
    """A Dirichlet-preconditioned handle and the oracle on the same tangent."""

    def __init__(self, name, dev, precision="fp64", tile=32):
        from paper_1205_1926_amd import GpuSolver
        w, plastic = CASES[name]()
        self.w = w
        self.mesh = Mesh(w)
        self.tf = TFETI(self.mesh)
        ne = self.mesh.n_elems
        sig, kap = np.zeros((ne, 8, 6)), np.zeros((ne, 8))
        if plastic:
            o = OracleSolver(w, "tfeti")
            o.load_step()
            sig, kap = o.sigma, o.kappa
        self.g = GpuSolver(w, precision=precision, tile=tile, preconditioner=2)
        self.g.set_state(sigma=T(sig.ravel(), dev), kappa=T(kap.ravel(), dev))
        self.du = np.random.default_rng(11).standard_normal(self.mesh.n_torn) * 1e-4
        self.a = assembly.assemble(self.mesh, assembly.element_dofs_torn(self.mesh), self.mesh.n_torn, self.du,
                                   sig, kap)
        self.tf.set_matrix(self.a["K"])
        self.g.assemble(T(self.du, dev))
        self.g.factorize()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dirichlet_apply_matches_oracle(name, precision, dev):
    """FP64 mode to 1e-9 of the largest entry; FP32 mode (FP32 coupling
    values and interior panels of the FP64 interior factor) to 1e-5."""
    P = DPair(name, dev, precision=precision)
    tol = 1e-9 if precision == "fp64" else 1e-5
    rng = np.random.default_rng(4)
    for _ in range(2):
        w = rng.standard_normal(P.mesh.m)
        assert emax(N(P.g.precondition(T(w, dev))), P.tf.precondition_dirichlet(w)) <= tol
    P.g.close()


@pytest.mark.parametrize("name", ["cube2x2x2_sub4", "plastic", "uneven"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dirichlet_dual_pcg_matches_oracle(name, precision, dev):
    P = DPair(name, dev, precision=precision)
    f = P.mesh.torn_load(1.0) - P.a["fint"]
    ref = P.tf.solve(f, eps=1e-8, precond="dirichlet")
    lum = P.tf.solve(f, eps=1e-8, precond="lumped")
    lam, u, rep, rc = P.g.dual_pcg(T(f, dev))
    assert rep["converged"] == 1
    if precision == "fp64":
        assert abs(rep["iters"] - ref["iters"]) <= 1
    assert ref["iters"] <= lum["iters"]
    assert rel(N(u), ref["u"]) <= 1e-6
    assert rel(N(lam), ref["lam"]) <= 1e-5
    P.g.close()


@pytest.mark.parametrize("tile", [0, 16, 64])
def test_dirichlet_other_tiles(tile, dev):
    """Fixed tiles 16 and 64, and tile 0: the autotuner also picks the
    interior solves' own tile and workgroup size."""
    P = DPair("uneven", dev, tile=tile)
    w = np.random.default_rng(5).standard_normal(P.mesh.m)
    assert emax(N(P.g.precondition(T(w, dev))), P.tf.precondition_dirichlet(w)) <= 1e-9
    P.g.close()


def test_dirichlet_without_interior_equals_lumped(dev):
    """One-element subdomains in a box clamped on every face: no node is
    interior, and the Dirichlet preconditioner is the lumped one."""
    from paper_1205_1926_amd import GpuSolver
    w = W.small_cube(S=(2, 2, 2), n=(1, 1, 1), amp=400.0)
    w.dirichlet = [[1, 1, 1] for _ in range(6)]
    gd = GpuSolver(w, tile=16, preconditioner=2)
    gl = GpuSolver(w, tile=16, preconditioner=1)
    for g in (gd, gl):
        g.assemble(g.zeros(g.sizes["n_torn"]))
        g.factorize()
    x = T(np.random.default_rng(6).standard_normal(gd.sizes["m"]), dev)
    assert torch.equal(gd.precondition(x), gl.precondition(x))
    gd.close()
    gl.close()


def test_dirichlet_newton_graph_matches_oracle(dev):
    """Plastic load steps with the Dirichlet preconditioner, graph replay and
    warm start (factor reuse and copied-back elastic interior factors on the
    path): displacements match the oracle load step by load step, and the
    graph replay is bitwise the eager result."""
    from paper_1205_1926_amd import GpuSolver
    w = W.small_cube(S=(3, 2, 2), n=(3, 3, 3), amp=650.0, shear=150.0, steps=3)
    o = OracleSolver(w, "tfeti")
    ge = GpuSolver(w, preconditioner=2, use_graph=0, tile=32)
    gg = GpuSolver(w, preconditioner=2, use_graph=1, tile=32)
    restored = 0
    for k in range(w.steps):
        o.load_step()
        he = ge.load_step()
        hg = gg.load_step()
        restored += sum(r["restored"] for r in hg)
        assert [r["pcg_iters"] for r in he] == [r["pcg_iters"] for r in hg]
        ue, ug = N(ge.state()["u"]), N(gg.state()["u"])
        assert np.array_equal(ue, ug)
        assert rel(ug[o.untorn], o.u[o.untorn]) <= 1e-6, k
    assert restored > 0 and gg.graph_active() == 1
    ge.close()
    gg.close()
