"""Pins of oracle.reference: the elastic stiffness assembled per distinct
subdomain shape equals the assembly of the whole mesh (Algorithm 5), and the
first load step it solves equals the Newton solver's first load step."""

import numpy as np

import workloads as W
from oracle import assembly, reference
from oracle.mesh import Mesh
from oracle.newton import Solver


def test_blocks_equal_whole_mesh_assembly():
    w = W.Workload("uneven", (2, 3, 2), [3, 5], [2, 4, 3], [6, 2])
    mesh = Mesh(w)
    ne = mesh.n_elems
    a = assembly.assemble(mesh, assembly.element_dofs_torn(mesh), mesh.n_torn, np.zeros(mesh.n_torn),
                          np.zeros((ne, 8, 6)), np.zeros((ne, 8)))
    Kb = reference.elastic_tangent_blocks(mesh)
    d = (Kb - a["K"]).tocoo()
    assert d.nnz == 0 or np.abs(d.data).max() <= 1e-14 * np.abs(a["K"].data).max()


def test_first_step_equals_newton_solver():
    w = W.config(0)
    r = reference.elastic_first_step(w, fapply_seed=1)
    o = Solver(w, "tfeti")
    hist = o.load_step()
    assert len(hist) == 1 and hist[0]["plastic_gp"] == 0
    idx = r["untorn"]
    assert np.linalg.norm(r["du"][idx] - o.u[idx]) <= 1e-12 * np.linalg.norm(o.u[idx])
    assert np.array_equal(r["F_lam"], r["tf"].F(r["lam_F"]))
