"""The paper's benchmark (Section 5) in its box-decomposable stand-in: an
eighth of the 20 x 20 x 2 plate on symmetry rollers, in tension on y = 10,
with a square hole through the thickness (one box of the decomposition left
out).  Pins of the absent-box handling and of the qualitative Newton
behaviour the paper reports for it (Table 2)."""

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import assembly
from oracle.mesh import Mesh
from oracle.newton import Solver
from oracle.tfeti import TFETI


def test_plate_geometry_and_constraints():
    """The hole's nodes belong to no subdomain, the rollers fix one
    component on each symmetry plane, and the notch faces are free."""
    w = W.plate_notch(1)
    m = Mesh(w)
    assert len(m.subs) == 15 and m.n_elems == 40 * 40 * 4 - 4 * 4 * 4
    Nx, Ny, Nz = m.N
    g = np.arange(m.n_gnodes)
    i, j, k = m.node_ijk(g)
    inside = (i < 4) & (j < 4)                    # strictly inside the 1 x 1 square hole
    assert not m.used[inside].any() and m.used[~inside].all()
    expect = np.stack([i == 0, j == 0, k == 0], axis=1) & m.used[:, None]
    assert np.array_equal(m.dir_mask & m.used[:, None], expect)
    notch = m.used & (((i == 4) & (j < 4)) | ((j == 4) & (i < 4))) & (i > 0) & (j > 0) & (k > 0)
    assert notch.sum() == 2 * 3 * 4 and not m.dir_mask[notch].any()
    f = m.torn_load(1.0)
    assert np.isclose(f[1::3].sum(), 400.0 * 10.0 * 1.0)    # traction 400 on the 10 x 1 face y = 10
    assert np.isclose(np.abs(f[0::3]).sum(), 0.0) and np.isclose(np.abs(f[2::3]).sum(), 0.0)


def test_plate_tfeti_equals_monolithic():
    """Elastic plate with the hole: TFETI (Algorithm 3) reproduces the
    Dirichlet-eliminated global solve on the nodes that exist."""
    w = W.plate_notch(1)
    mesh = Mesh(w)
    ed = assembly.element_dofs_torn(mesh)
    ne = mesh.n_elems
    a = assembly.assemble(mesh, ed, mesh.n_torn, np.zeros(mesh.n_torn), np.zeros((ne, 8, 6)), np.zeros((ne, 8)))
    tf = TFETI(mesh)
    tf.set_matrix(a["K"])
    f = mesh.torn_load(1.0)
    res = tf.solve(f, eps=1e-12)
    eg = assembly.element_dofs_global(mesh)
    ng = 3 * mesh.n_gnodes
    ag = assembly.assemble(mesh, eg, ng, np.zeros(ng), np.zeros((ne, 8, 6)), np.zeros((ne, 8)))
    fg = np.zeros(ng)
    for s in mesh.subs:
        np.add.at(fg.reshape(-1, 3), s.l2g, f[s.off:s.off + s.n_dofs].reshape(-1, 3))
    free = ~mesh.dir_mask.ravel() & np.repeat(mesh.used, 3)
    Kf = ag["K"][free][:, free]
    from oracle.tfeti import lower_band
    ab, _ = lower_band(Kf)
    ug = np.zeros(ng)
    ug[free] = sla.cho_solve_banded((sla.cholesky_banded(ab, lower=True), True), fg[free])
    ut = res["u"][mesh.untorn_index()]
    uu = ug[mesh.used_dofs()]
    assert np.linalg.norm(ut - uu) <= 1e-9 * np.linalg.norm(uu)
    assert res["converged"]


@pytest.mark.slow
def test_plate_newton_history_discretization_a():
    """Discretization (a) (one time step to t* = 1/4): the first Newton
    iteration solves the elastic problem (no plastic element, criterion 1),
    the plastic elements then grow and stabilize, and the criterion falls
    quadratically once the plastic set is fixed (the behaviour of the
    paper's Table 2)."""
    w = W.plate_notch(1, steps=1)
    o = Solver(w, "tfeti")
    h = o.load_step()
    crit = [r["crit"] for r in h]
    pl = [r["plastic_el"] for r in h]
    assert h[0]["plastic_gp"] == 0 and crit[0] == pytest.approx(1.0)
    assert 5 <= len(h) <= 9
    assert all(b >= a for a, b in zip(pl[1:], pl[2:])) and pl[-1] == pl[-2] > 0
    # quadratic tail: crit_{i+1} <= C crit_i^2 on the last iterations
    assert crit[-1] <= 100.0 * crit[-2] ** 2 and crit[-2] <= 100.0 * crit[-3] ** 2
    assert crit[-1] < 1e-8
