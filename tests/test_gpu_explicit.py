"""GPU parity of the explicit local dual operators (options.fapply_format =
TFETI_FAPPLY_EXPLICIT): per subdomain the block of K_reg^{-1} on the DOFs
that carry rows of B, formed from the FP64 factor and applied as one
symmetric product (F = B K^+ B^T, Section 4.2; K^+ from the regularized
Cholesky factor, Remark 1).

The operator is the same F as the factor path's, so the tolerances are the
factor path's: F entry by entry to 1e-9 of the largest entry in FP64 (the
explicit block carries the rounding of two triangular solves with the
same factor, as a solve does) and to 1e-5 with FP32 storage; PCGP and Newton
results to the 1e-6 displacement bar.  Explicit and factor F-applies on one
tangent agree to 1e-10 in FP64.
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
    """Largest entry difference relative to the largest entry of b."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


class Pair:
    """GPU handles (explicit and factor F-applies) and the oracle on one
    tangent."""

    def __init__(self, w, dev, precision="fp64", plastic_step=False, tile=32):
        from paper_1205_1926_amd import GpuSolver
        self.w = w
        self.mesh = Mesh(w)
        self.tf = TFETI(self.mesh)
        ne = self.mesh.n_elems
        sigma = np.zeros((ne, 8, 6))
        kappa = np.zeros((ne, 8))
        if plastic_step:
            o = OracleSolver(w, "tfeti")
            o.load_step()
            sigma, kappa = o.sigma, o.kappa
        ed = assembly.element_dofs_torn(self.mesh)
        rng = np.random.default_rng(11)
        self.du = rng.standard_normal(self.mesh.n_torn) * 1e-4
        self.a = assembly.assemble(self.mesh, ed, self.mesh.n_torn, self.du, sigma, kappa)
        self.tf.set_matrix(self.a["K"])
        self.g = {}
        for fmt in ("explicit", "hybrid", "factors"):
            g = GpuSolver(w, precision=precision, tile=tile, fapply_format=fmt)
            g.set_state(sigma=T(sigma.ravel(), dev), kappa=T(kappa.ravel(), dev))
            g.assemble(T(self.du, dev))
            g.factorize()
            self.g[fmt] = g

    def close(self):
        for g in self.g.values():
            g.close()


def _uneven():
    w = W.Workload("uneven", (2, 3, 2), [3, 5], [2, 4, 3], [6, 2],
                   dirichlet=[[0, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0], [1, 1, 1], [0, 0, 0]])
    w.traction[5] = [50.0, 0.0, -300.0]
    return w


CASES = {
    "cube_elastic": lambda: (W.config(0), False),
    "cube_plastic": lambda: (W.small_cube(S=(2, 2, 2), n=(3, 3, 3), amp=700.0, shear=150.0, steps=2), True),
    "uneven": lambda: (_uneven(), False),
}


@pytest.fixture(scope="module", params=list(CASES))
def pair(request, dev):
    w, plastic = CASES[request.param]()
    P = Pair(w, dev, plastic_step=plastic)
    P.name = request.param
    yield P
    P.close()


def test_explicit_fapply_matches_oracle(pair, dev):
    """Cubes: the library's fixing nodes are the oracle's, so F agrees entry
    by entry; the uneven mesh's other fixing nodes leave P F on Ker G
    (Section 4.2).  The explicit and factor applies of one tangent agree."""
    P = pair
    rng = np.random.default_rng(3)
    lam = rng.standard_normal(P.mesh.m)
    qf = N(P.g["factors"].fapply(T(lam, dev)))
    lk = P.tf.project(lam)
    for fmt in ("explicit", "hybrid"):
        qe = N(P.g[fmt].fapply(T(lam, dev)))
        assert emax(qe, qf) <= 1e-10, fmt
        if P.name != "uneven":
            assert emax(qe, P.tf.F(lam)) <= 1e-9, fmt
        assert emax(P.tf.project(N(P.g[fmt].fapply(T(lk, dev)))), P.tf.project(P.tf.F(lk))) <= 1e-9, fmt


def test_explicit_fapply_deterministic(pair, dev):
    rng = np.random.default_rng(8)
    lam = T(rng.standard_normal(pair.mesh.m), dev)
    for fmt in ("explicit", "hybrid"):
        a = N(pair.g[fmt].fapply(lam))
        b = N(pair.g[fmt].fapply(lam))
        assert np.array_equal(a, b), fmt


def test_explicit_dual_pcg(pair, dev):
    P = pair
    f = P.mesh.torn_load(1.0) - P.a["fint"]
    ref = P.tf.solve(f, eps=1e-8)
    for fmt in ("explicit", "hybrid"):
        lam, u, rep, rc = P.g[fmt].dual_pcg(T(f, dev))
        assert rep["converged"] == 1, fmt
        assert abs(rep["iters"] - ref["iters"]) <= 1, fmt
        assert rel(N(u), ref["u"]) <= 1e-6, fmt
        assert rel(N(lam), ref["lam"]) <= 1e-5, fmt


@pytest.mark.parametrize("name", list(CASES))
def test_explicit_fp32(name, dev):
    """FP32 storage of the FP64-formed block: F-applies within 1e-5 of the
    oracle's (cubes) or on Ker G (uneven), and the FP32 inner PCGP with FP64
    outer refinement reaches the oracle's solution."""
    w, plastic = CASES[name]()
    P = Pair(w, dev, precision="fp32", plastic_step=plastic)
    rng = np.random.default_rng(5)
    lam = rng.standard_normal(P.mesh.m)
    lk = P.tf.project(lam)
    f = P.mesh.torn_load(1.0) - P.a["fint"]
    ref = P.tf.solve(f, eps=1e-8)
    for fmt in ("explicit", "hybrid"):
        if name != "uneven":
            assert emax(N(P.g[fmt].fapply(T(lam, dev))), P.tf.F(lam)) <= 1e-5, fmt
        assert emax(P.tf.project(N(P.g[fmt].fapply(T(lk, dev)))), P.tf.project(P.tf.F(lk))) <= 1e-5, fmt
        lam_g, u, rep, rc = P.g[fmt].dual_pcg(T(f, dev))
        assert rep["converged"] == 1 and 1 <= rep["outer"] <= 4, fmt
        assert rel(N(u), ref["u"]) <= 1e-6, fmt
        assert rel(N(lam_g), ref["lam"]) <= 1e-5, fmt
    P.close()


@pytest.mark.parametrize("S,n", [((1, 1, 1), (3, 3, 3)), ((3, 1, 2), (1, 1, 1)), ((2, 1, 1), (4, 2, 3))],
                         ids=["single_subdomain", "one_element_subdomains", "flat_subdomains"])
def test_explicit_degenerate_decompositions(S, n, dev):
    """One subdomain (B holds only Dirichlet rows), one-element subdomains
    (24 DOFs, every DOF touched, factors padded to 64 rows) and flat boxes:
    the explicit solve matches the oracle's."""
    w = W.small_cube(S=S, n=n, amp=500.0, shear=100.0)
    P = Pair(w, dev, tile=16)
    rng = np.random.default_rng(2)
    lam = rng.standard_normal(P.mesh.m)
    f = P.mesh.torn_load(1.0) - P.a["fint"]
    ref = P.tf.solve(f, eps=1e-8)
    for fmt in ("explicit", "hybrid"):
        assert emax(N(P.g[fmt].fapply(T(lam, dev))), N(P.g["factors"].fapply(T(lam, dev)))) <= 1e-10, fmt
        lam_g, u, rep, rc = P.g[fmt].dual_pcg(T(f, dev))
        assert rep["converged"] == 1, fmt
        assert rel(N(u), ref["u"]) <= 1e-6, fmt
    P.close()


@pytest.mark.parametrize("fmt,precision", [("explicit", "fp64"), ("explicit", "fp32"), ("hybrid", "fp64"),
                                            ("hybrid", "fp32")])
def test_explicit_newton_plastic_matches_oracle(fmt, precision, dev):
    """Load steps with plastic subdomains refactorized, elastic ones kept and
    elastic-again ones copied back, graph replay on.  Explicit: every
    factorized or copied-back subdomain's block formed again.  Hybrid: the
    subdomains with kept elastic factors use their blocks (formed with the
    factor, copied back with it), the others their factor sweeps, in one
    launch.  The oracle's displacements and hardening."""
    from paper_1205_1926_amd import GpuSolver
    w = W.small_cube(S=(3, 2, 2), n=(3, 3, 3), amp=650.0, shear=150.0, steps=3)
    o = OracleSolver(w, "tfeti")
    g = GpuSolver(w, use_graph=1, fapply_format=fmt, precision=precision)
    hist = []
    for k in range(w.steps):
        o.load_step()
        hist += g.load_step()
        ug = N(g.state()["u"])
        assert rel(ug[o.untorn], o.u[o.untorn]) <= 1e-6, k
    st = g.state()
    assert np.abs(N(st["kappa"]) - o.kappa.ravel()).max() <= 1e-6 * np.abs(o.kappa).max()
    assert any(0 < r["refactored"] < 12 for r in hist)
    assert sum(r["restored"] for r in hist) > 0
    g.close()


def test_explicit_factor_reuse_is_exact(dev):
    """With explicit blocks, keeping elastic factors (and copying back the
    kept elastic factor of subdomains elastic again, whose block is formed
    from it) gives bit-identical results to factorizing every subdomain each
    iteration."""
    from paper_1205_1926_amd import GpuSolver
    w = W.small_cube(S=(3, 2, 2), n=(3, 3, 3), amp=650.0, shear=150.0, steps=3)
    runs = {}
    for flag in (0, 1):
        g = GpuSolver(w, refactor_all=flag, tile=32, fapply_format="explicit")
        hist = g.run()
        runs[flag] = (hist, N(g.state()["u"]), N(g.lam()))
        g.close()
    assert np.array_equal(runs[0][1], runs[1][1])
    assert np.array_equal(runs[0][2], runs[1][2])
    assert sum(r["restored"] for h in runs[0][0] for r in h) > 0


def test_explicit_sizes_report_bytes(dev):
    """explicit_bytes counts the stored lower-triangle tiles: per subdomain
    of m_p touched DOFs (columns of B with an entry in it) ceil(m_p / 16)
    (ceil(m_p / 16) + 1) / 2 tiles of 16 x 16 entries, 8 bytes each in FP64
    and 4 in FP32; 0 on the factor path."""
    from paper_1205_1926_amd import GpuSolver
    w = W.config(0)
    mesh = Mesh(w)
    cols = np.unique(mesh.B.tocoo().col)
    tiles = 0
    for s in mesh.subs:
        m_p = int(((cols >= s.off) & (cols < s.off + s.n_dofs)).sum())
        mt = (m_p + 15) // 16
        tiles += mt * (mt + 1) // 2
    for prec, esz in (("fp64", 8), ("fp32", 4)):
        g = GpuSolver(w, precision=prec, fapply_format="explicit")
        assert g.sizes["explicit_bytes"] == tiles * 256 * esz
        g.close()
        g = GpuSolver(w, precision=prec)
        assert g.sizes["explicit_bytes"] == 0
        g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["cube_plastic", "uneven"])
def test_hybrid_wide_tiles(name, precision, dev):
    """64-row tiles: the solve kernel's wide-tile instances walk an
    operator's tiles with half of the workgroup's wavefronts.  The hybrid
    F-apply equals the factor path's (FP64) or the oracle's F within 1e-5
    (FP32, on Ker G for the uneven mesh), and its dual solve reaches the
    oracle's solution."""
    w, plastic = CASES[name]()
    P = Pair(w, dev, precision=precision, plastic_step=plastic, tile=64)
    rng = np.random.default_rng(13)
    lam = rng.standard_normal(P.mesh.m)
    lk = P.tf.project(lam)
    qh = N(P.g["hybrid"].fapply(T(lam, dev)))
    if precision == "fp64":
        assert emax(qh, N(P.g["factors"].fapply(T(lam, dev)))) <= 1e-10
    elif name != "uneven":
        assert emax(qh, P.tf.F(lam)) <= 1e-5
    assert emax(P.tf.project(N(P.g["hybrid"].fapply(T(lk, dev)))), P.tf.project(P.tf.F(lk))) <= 1e-5
    f = P.mesh.torn_load(1.0) - P.a["fint"]
    ref = P.tf.solve(f, eps=1e-8)
    lam_g, u, rep, rc = P.g["hybrid"].dual_pcg(T(f, dev))
    assert rep["converged"] == 1
    assert rel(N(u), ref["u"]) <= 1e-6
    assert rel(N(lam_g), ref["lam"]) <= 1e-5
    assert P.g["hybrid"].sizes["tile"] == 64
    P.close()
