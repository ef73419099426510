"""GPU parity: every stage of the HIP path, called through the C ABI, against
the FP64 oracle on the same seeded inputs.

Tolerances follow from FP64 rounding (unit roundoff 1.1e-16) amplified by the
conditioning of each stage: the return map and assembly are well conditioned
(1e-12); the regularized subdomain matrices have condition numbers of 1e4-1e5
on these meshes, so K^+ and F agree to ~1e-11 and are tested at 1e-9; PCGP
results agree to the solver tolerance and are tested at the 1e-6 displacement
bar.  Operators (K^+, F, P, the preconditioner) are compared entry by entry:
the largest entry difference relative to the largest entry of the oracle's
result.  FP32 panels of the FP64 factor (unit roundoff 6e-8 per entry,
amplified by the subdomain condition numbers) give F-applies within about
1e-6 of FP64; they are tested at 1e-5.
"""

import numpy as np
import pytest

import workloads as W
from oracle import assembly, constitutive
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


# ---------------------------------------------------------------- return map
def test_return_map_matches_oracle(dev):
    from paper_1205_1926_amd import return_map
    rng = np.random.default_rng(7)
    n = 5000
    sig = rng.standard_normal((n, 6)) * 150.0
    kap = np.abs(rng.standard_normal(n)) * 1e-3
    de = rng.standard_normal((n, 6)) * 2e-3
    mat = W.Material()
    ds, dk, D, pl = return_map(mat, T(sig, dev), T(kap, dev), T(de, dev))
    ods, odk, oD, opl, ophi = constitutive.return_map(sig, kap, de, mat.E, mat.nu, mat.sigma_y, mat.H)
    away = np.abs(ophi) > 1e-10 * mat.sigma_y
    assert np.array_equal(N(pl).astype(bool)[away], opl[away])
    assert np.abs(N(ds).reshape(n, 6) - ods).max() <= 1e-13 * np.abs(ods).max()
    assert np.abs(N(dk) - odk).max() <= 1e-13 * max(np.abs(odk).max(), 1e-30)
    assert np.abs(N(D).reshape(n, 6, 6) - oD).max() <= 1e-12 * np.abs(oD).max()


def test_return_map_empty(dev):
    from paper_1205_1926_amd import return_map
    e = torch.zeros(0, dtype=torch.float64, device=dev)
    ds, dk, D, pl = return_map(W.Material(), e, e, e)
    assert ds.numel() == 0


# ---------------------------------------------------------------- one linear system
class Pair:
    """GPU handle and oracle objects for the same workload and state."""

    def __init__(self, w, dev, precision="fp64", tile=0, plastic_step=False):
        from paper_1205_1926_amd import GpuSolver
        self.w = w
        self.mesh = Mesh(w)
        self.tf = TFETI(self.mesh)
        ne = self.mesh.n_elems
        self.sigma = np.zeros((ne, 8, 6))
        self.kappa = np.zeros((ne, 8))
        if plastic_step:
            o = OracleSolver(w, "tfeti")
            o.load_step()
            self.sigma, self.kappa = o.sigma, o.kappa
        self.g = GpuSolver(w, precision=precision, tile=tile)
        self.g.set_state(sigma=T(self.sigma.ravel(), dev), kappa=T(self.kappa.ravel(), dev))
        self.ed = assembly.element_dofs_torn(self.mesh)
        rng = np.random.default_rng(11)
        self.du = rng.standard_normal(self.mesh.n_torn) * 1e-4
        self.a = assembly.assemble(self.mesh, self.ed, self.mesh.n_torn, self.du, self.sigma, self.kappa)
        self.tf.set_matrix(self.a["K"])
        self.fint_g, self.npl = self.g.assemble(T(self.du, dev))
        self.g.factorize()


@pytest.fixture(scope="module")
def pair0(dev):
    return Pair(W.config(0), dev, plastic_step=False)


@pytest.fixture(scope="module")
def pair_plastic(dev):
    w = W.small_cube(S=(2, 2, 2), n=(3, 3, 3), amp=700.0, shear=150.0, steps=2)
    return Pair(w, dev, plastic_step=True)


@pytest.fixture(scope="module")
def pair_uneven(dev):
    w = W.Workload("uneven", (2, 3, 2), [3, 5], [2, 4, 3], [6, 2],
                   dirichlet=[[0, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0], [1, 1, 1], [0, 0, 0]])
    w.traction[5] = [50.0, 0.0, -300.0]
    return Pair(w, dev)


@pytest.mark.parametrize("name", ["pair0", "pair_plastic", "pair_uneven"])
def test_assembly_internal_force(name, request, dev):
    P = request.getfixturevalue(name)
    assert emax(N(P.fint_g), P.a["fint"]) <= 1e-12
    st = P.g.state()
    pl_g = N(st["plastic"]).astype(bool)
    away = np.abs(P.a["phi"].ravel()) > 1e-10 * P.w.material.sigma_y
    assert np.array_equal(pl_g[away], P.a["plastic"].ravel()[away])
    assert np.abs(N(st["dsigma"]) - P.a["dsigma"].ravel()).max() <= 1e-12 * np.abs(P.a["dsigma"]).max()


@pytest.mark.parametrize("name", ["pair0", "pair_plastic"])
def test_kplus_and_fapply(name, request, dev):
    """Cubes: the library's factor ordering is the natural one, so its fixing
    nodes and K_reg are the oracle's and K^+ and F agree entry by entry."""
    P = request.getfixturevalue(name)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(P.mesh.n_torn)
    assert emax(N(P.g.kplus(T(x, dev))), P.tf.kplus(x)) <= 1e-9
    lam = rng.standard_normal(P.mesh.m)
    assert emax(N(P.g.fapply(T(lam, dev))), P.tf.F(lam)) <= 1e-9


@pytest.mark.parametrize("name", ["pair0", "pair_plastic", "pair_uneven"])
def test_kplus_and_fapply_invariant_parts(name, request, dev):
    """Any mesh: generalized inverses built on different fixing nodes differ
    by rigid body modes on Im K, so K^+ x agrees off Ker K for x in Im K, and
    P F agrees on Ker G (Section 4.2)."""
    P = request.getfixturevalue(name)
    rng = np.random.default_rng(3)
    x = P.tf.K @ rng.standard_normal(P.mesh.n_torn)
    R = P.tf.Rmat
    off = lambda v: v - R @ (R.T @ v)
    zg = N(P.g.kplus(T(x, dev)))
    assert emax(off(zg), off(P.tf.kplus(x))) <= 1e-9
    assert emax(P.tf.K @ zg, x) <= 1e-9
    lam = P.tf.project(rng.standard_normal(P.mesh.m))
    assert emax(P.tf.project(N(P.g.fapply(T(lam, dev)))), P.tf.project(P.tf.F(lam))) <= 1e-9


@pytest.mark.parametrize("name", ["pair0", "pair_plastic", "pair_uneven"])
def test_projector_and_preconditioner(name, request, dev):
    P = request.getfixturevalue(name)
    rng = np.random.default_rng(4)
    w = rng.standard_normal(P.mesh.m)
    assert emax(N(P.g.project(T(w, dev))), P.tf.project(w)) <= 1e-12
    assert emax(N(P.g.precondition(T(w, dev))), P.tf.precondition(w)) <= 1e-12


@pytest.mark.parametrize("name", ["pair0", "pair_plastic", "pair_uneven"])
def test_dual_pcg(name, request, dev):
    P = request.getfixturevalue(name)
    f = P.mesh.torn_load(1.0) - P.a["fint"]
    ref = P.tf.solve(f, eps=1e-8)
    lam, u, rep, rc = P.g.dual_pcg(T(f, dev))
    assert rep["converged"] == 1
    assert abs(rep["iters"] - ref["iters"]) <= 1
    assert rel(N(u), ref["u"]) <= 1e-6
    assert rel(N(lam), ref["lam"]) <= 1e-5
    assert abs(rep["r_ref"] - ref["r_ref"]) <= 1e-9 * ref["r_ref"]


@pytest.mark.parametrize("S,n", [((1, 1, 1), (3, 3, 3)), ((3, 1, 2), (1, 1, 1))],
                         ids=["single_subdomain", "one_element_subdomains"])
def test_dual_pcg_degenerate_decompositions(S, n, dev):
    """Degenerate decompositions: one subdomain (B holds only the Dirichlet
    rows, G G^T is 6 x 6) and subdomains of a single element (24 DOFs padded
    to 64 rows, every node touched).  The solve matches the oracle's."""
    w = W.small_cube(S=S, n=n, amp=500.0, shear=100.0)
    P = Pair(w, dev, tile=16)
    f = P.mesh.torn_load(1.0) - P.a["fint"]
    ref = P.tf.solve(f, eps=1e-8)
    lam, u, rep, rc = P.g.dual_pcg(T(f, dev))
    assert rep["converged"] == 1
    assert abs(rep["iters"] - ref["iters"]) <= 1
    assert rel(N(u), ref["u"]) <= 1e-6
    assert rel(N(lam), ref["lam"]) <= 1e-5
    P.g.close()


@pytest.mark.parametrize("use_graph,check_every", [(0, 8), (1, 8), (1, 3)])
def test_dual_pcg_iteration_cap(use_graph, check_every, pair0, dev):
    """Stopped at max_pcg iterations (at the end of a replayed batch of 8, or
    inside a batch of 3), lambda and u are the oracle's after the same number
    of PCGP iterations: the updates folded into the next iteration's first
    projection are applied before the stopping test ends the loop."""
    from paper_1205_1926_amd import GpuSolver
    P = pair0
    g = GpuSolver(P.w, use_graph=use_graph, check_every=check_every, max_pcg=7, tile=32)
    g.assemble(T(P.du, dev))
    g.factorize()
    f = P.mesh.torn_load(1.0) - P.a["fint"]
    ref = P.tf.solve(f, eps=1e-8, maxit=7)
    assert not ref["converged"] and ref["iters"] == 7
    lam, u, rep, rc = g.dual_pcg(T(f, dev))
    assert rc == 2 and rep["converged"] == 0 and rep["iters"] == 7
    assert rel(N(lam), ref["lam"]) <= 1e-9
    assert rel(N(u), ref["u"]) <= 1e-9
    g.close()


def test_dual_pcg_warm_start_and_rejection(pair0, dev):
    P = pair0
    f = P.mesh.torn_load(1.0)
    ref = P.tf.solve(f, eps=1e-8)
    lam, u, rep, rc = P.g.dual_pcg(T(f, dev), guess=T(ref["lam"], dev))
    assert rep["iters"] <= 1 and rel(N(u), ref["u"]) <= 1e-6
    bad = torch.full((P.mesh.m,), float("nan"), dtype=torch.float64, device=dev)
    lam, u, rep, rc = P.g.dual_pcg(T(f, dev), guess=bad)
    from paper_1205_1926_amd import _capi
    assert rc == _capi.TFETI_W_WARMSTART_REJECTED
    assert rel(N(u), ref["u"]) <= 1e-6


@pytest.mark.parametrize("name", ["pair0", "pair_plastic", "pair_uneven"])
def test_fp32_fapply(name, request, dev):
    """FP32 panels of the FP64 factor: single F-applies and K^+ solves agree
    entry by entry with the oracle's and with the FP64 panels of the same
    factor (an FP64-mode handle on the same tangent) to FP32 level."""
    P64 = request.getfixturevalue(name)
    P = Pair(P64.w, dev, precision="fp32", plastic_step=(name == "pair_plastic"))
    rng = np.random.default_rng(5)
    lam = rng.standard_normal(P.mesh.m)
    q32 = N(P.g.fapply(T(lam, dev)))
    q64 = N(P64.g.fapply(T(lam, dev)))
    if name != "pair_uneven":
        # cubes: the oracle's fixing nodes, so F itself agrees
        assert emax(q32, P.tf.F(lam)) <= 1e-5
    else:
        # other fixing nodes: P F agrees on Ker G (Section 4.2)
        lk = P.tf.project(lam)
        assert emax(P.tf.project(N(P.g.fapply(T(lk, dev)))), P.tf.project(P.tf.F(lk))) <= 1e-5
    assert emax(q32, q64) <= 1e-5
    x = rng.standard_normal(P.mesh.n_torn)
    assert emax(N(P.g.kplus(T(x, dev))), N(P64.g.kplus(T(x, dev)))) <= 1e-5
    P.g.close()


@pytest.mark.parametrize("name", ["pair0", "pair_plastic", "pair_uneven"])
def test_fp32_refined_dual_pcg(name, request, dev):
    """FP32 inner PCGP with FP64 outer dual refinement reaches the FP64
    solution (displacement bar 1e-6) in a few outer sweeps."""
    P0 = request.getfixturevalue(name)
    P = Pair(P0.w, dev, precision="fp32", plastic_step=(name == "pair_plastic"))
    f = P.mesh.torn_load(1.0) - P.a["fint"]
    ref = P.tf.solve(f, eps=1e-8)
    lam, u, rep, rc = P.g.dual_pcg(T(f, dev))
    assert rep["converged"] == 1 and 1 <= rep["outer"] <= 4
    assert rel(N(u), ref["u"]) <= 1e-6
    assert rel(N(lam), ref["lam"]) <= 1e-5


def test_graph_replay_matches_eager(dev):
    """The PCGP iteration replayed from a HIP graph gives bitwise the eager
    result, solve after solve (several replays, eager work in between)."""
    from paper_1205_1926_amd import GpuSolver
    w = W.small_cube(S=(2, 2, 2), n=(3, 3, 3), amp=500.0, shear=100.0)
    # one fixed tile: the autotuner could pick different kernels per handle
    ge = GpuSolver(w, use_graph=0, tile=32)
    gg = GpuSolver(w, use_graph=1, tile=32)
    gt = GpuSolver(w, use_graph=1, tile=32)  # replay with timed solve kernels in one batch of four
    gt.set_timing(True)
    du = torch.zeros(ge.sizes["n_torn"], dtype=torch.float64, device=dev)
    for g in (ge, gg, gt):
        g.assemble(du)
        g.factorize()
    mesh = Mesh(w)
    rng = np.random.default_rng(9)
    total = 0
    for k in range(3):
        f = T(mesh.torn_load(1.0) * (1 + k) + 0.1 * rng.standard_normal(mesh.n_torn), dev)
        le, ue, re, _ = ge.dual_pcg(f)
        lg, ug, rg, _ = gg.dual_pcg(f)
        lt, ut, rt, _ = gt.dual_pcg(f)
        assert re["iters"] == rg["iters"] == rt["iters"]
        assert torch.equal(le, lg) and torch.equal(ue, ug)
        assert torch.equal(le, lt) and torch.equal(ue, ut)
        total += re["iters"]
    assert gg.graph_active() == 1 and gt.graph_active() == 1
    ms, cnt = gt.timing()
    # the solve kernels of the first batch of 8 iterations (and of every
    # fourth batch after it) are timed, the others replay without events
    assert min(total, 8) <= cnt < total and ms > 0


def test_newton_fp32_mode_matches_oracle(dev):
    from paper_1205_1926_amd import GpuSolver
    w = W.small_cube(S=(2, 2, 2), n=(3, 3, 3), amp=700.0, shear=150.0, steps=2)
    o = OracleSolver(w, "tfeti")
    g = GpuSolver(w, precision="fp32", use_graph=1)
    for k in range(w.steps):
        o.load_step()
        g.load_step()
        ug = N(g.state()["u"])
        assert rel(ug[o.untorn], o.u[o.untorn]) <= 1e-6, k


@pytest.mark.parametrize("tile,n,precision", [(16, (3, 4, 5), "fp64"), (32, (3, 4, 5), "fp64"),
                                              (64, (3, 4, 5), "fp64"), (16, (10, 10, 10), "fp64"),
                                              (16, (3, 4, 5), "fp32"), (64, (3, 4, 5), "fp32"),
                                              (32, (10, 10, 10), "fp32")])
def test_other_tiles(tile, n, precision, dev):
    """Tiles 16 and 32 have their panels written by the factorization
    itself, tile 64 by the separate packing pass; 10^3-element subdomains
    (half bandwidth 398) take the factorization's multi-pass panel path."""
    P = Pair(W.small_cube(S=(2, 1, 1) if n[0] == 10 else (2, 2, 1), n=n, amp=300.0), dev, tile=tile,
             precision=precision)
    rng = np.random.default_rng(6)
    lam = rng.standard_normal(P.mesh.m)
    tol = 1e-9 if precision == "fp64" else 1e-5
    assert emax(N(P.g.fapply(T(lam, dev))), P.tf.F(lam)) <= tol
    if precision == "fp32":
        # the outer refinement runs on the FP64 panels written alongside
        f = P.mesh.torn_load(1.0) - P.a["fint"]
        ref = P.tf.solve(f, eps=1e-8)
        lam, u, rep, rc = P.g.dual_pcg(T(f, dev))
        assert rep["converged"] == 1
        assert rel(N(u), ref["u"]) <= 1e-6


def test_autotuner_choice_and_cache(tmp_path, monkeypatch, dev):
    """tile = 0: the first factorization times every tile and schedule and
    keeps the fastest; F still matches the oracle; the choice is written to
    the cache and the next handle of the same problem takes it from there."""
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("TFETI_AUTOTUNE_CACHE", str(cache))
    P = Pair(W.config(0), dev, tile=0)
    sz = P.g.refresh_sizes()
    assert sz["autotuned"] == 1 and sz["tile"] in (16, 32, 64) and sz["schedule"] in (0, 1)
    rng = np.random.default_rng(12)
    lam = rng.standard_normal(P.mesh.m)
    assert emax(N(P.g.fapply(T(lam, dev))), P.tf.F(lam)) <= 1e-9
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and '"tile": %d' % sz["tile"] in lines[0]
    Q = Pair(W.config(0), dev, tile=0)
    sq = Q.g.refresh_sizes()
    assert sq["autotuned"] == 2 and sq["tile"] == sz["tile"] and sq["schedule"] == sz["schedule"]
    assert len(cache.read_text().splitlines()) == 1


def test_elastic_factor_reuse_is_exact(dev):
    """Keeping the factor of subdomains whose tangent is and was elastic, and
    copying back the kept elastic factor of subdomains that are elastic again,
    gives bit-identical results to factorizing every subdomain each
    iteration."""
    from paper_1205_1926_amd import GpuSolver
    w = W.small_cube(S=(3, 2, 2), n=(3, 3, 3), amp=650.0, shear=150.0, steps=3)
    runs = {}
    for flag in (0, 1):
        g = GpuSolver(w, refactor_all=flag, tile=32)
        hist = g.run()
        runs[flag] = (hist, N(g.state()["u"]), N(g.lam()))
    assert np.array_equal(runs[0][1], runs[1][1])
    assert np.array_equal(runs[0][2], runs[1][2])
    n_sub = 12
    counts = [r["refactored"] for h in runs[0][0] for r in h]
    assert counts[0] == n_sub
    assert min(counts) < n_sub          # elastic subdomains kept their factors
    assert all(r["refactored"] == n_sub for h in runs[1][0] for r in h)
    # the first iteration of a later load step is elastic everywhere: the
    # subdomains plastic at the end of the previous step get their kept
    # elastic factor back instead of a factorization
    assert sum(r["restored"] for h in runs[0][0] for r in h) > 0
    assert all(r["restored"] == 0 for h in runs[1][0] for r in h)
    assert [len(h) for h in runs[0][0]] == [len(h) for h in runs[1][0]]


def test_fapply_deterministic(pair0, dev):
    rng = np.random.default_rng(8)
    lam = T(rng.standard_normal(pair0.mesh.m), dev)
    a = N(pair0.g.fapply(lam))
    b = N(pair0.g.fapply(lam))
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- Newton / time stepping
def test_newton_config0_matches_oracle(dev):
    from paper_1205_1926_amd import GpuSolver
    w = W.config(0)
    o = OracleSolver(w, "tfeti")
    g = GpuSolver(w)
    for k in range(w.steps):
        ho = o.load_step()
        hg = g.load_step()
        ug = N(g.state()["u"])
        uo = o.u
        assert rel(ug[o.untorn], uo[o.untorn]) <= 1e-6, (k, rel(ug, uo))
        assert abs(len(hg) - len(ho)) <= 1
    st = g.state()
    assert np.abs(N(st["kappa"]) - o.kappa.ravel()).max() <= 1e-6 * max(np.abs(o.kappa).max(), 1e-12) + 1e-14


def test_newton_plastic_matches_oracle(dev):
    from paper_1205_1926_amd import GpuSolver
    w = W.small_cube(S=(2, 2, 2), n=(3, 3, 3), amp=700.0, shear=150.0, steps=3)
    o = OracleSolver(w, "tfeti")
    g = GpuSolver(w)
    for k in range(w.steps):
        ho = o.load_step()
        hg = g.load_step()
        ug = N(g.state()["u"])
        assert rel(ug[o.untorn], o.u[o.untorn]) <= 1e-6, k
    assert ho[-1]["plastic_el"] > 0
    assert hg[-1]["plastic_elements"] > 0
    st = g.state()
    assert np.abs(N(st["kappa"]) - o.kappa.ravel()).max() <= 1e-6 * np.abs(o.kappa).max()


def test_gpu_patch_test_closed_form(dev):
    """The elastoplastic patch test run entirely on the GPU reproduces the
    closed-form uniform state."""
    from paper_1205_1926_amd import GpuSolver
    q = 700.0
    w = W.patch_test(S=(2, 1, 2), n=(2, 2, 2), q=q, steps=3)
    g = GpuSolver(w, eps_pcg=1e-12, eps_newton=1e-12)
    g.run()
    m = w.material
    kap = (q - m.sigma_y) / m.H
    st = g.state()
    assert np.allclose(N(st["kappa"]), kap, rtol=1e-9)
    assert np.allclose(N(st["sigma"]).reshape(-1, 6), [0, 0, q, 0, 0, 0], atol=1e-7 * q)
