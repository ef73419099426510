"""Pins of the oracle's Q1 element: exact strains of linear fields, rigid body
modes in the kernel, rank, quadrature of the element volume and of a face."""

import numpy as np

from oracle import assembly, constitutive, q1
from oracle.mesh import Mesh
import workloads as W

H = (0.3, 0.5, 0.7)


def element_nodes(h):
    return q1.NODE_OFF * np.asarray(h)[None, :]


def test_linear_field_strain_exact():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 3))
    c = rng.standard_normal(3)
    X = element_nodes(H) + 0.1
    u = (X @ A.T + c).ravel()                       # u(x) = A x + c at the nodes
    B, w = q1.strain_matrices(H)
    eps_t = 0.5 * (A + A.T)
    expect = np.array([eps_t[0, 0], eps_t[1, 1], eps_t[2, 2], 2 * eps_t[0, 1], 2 * eps_t[1, 2], 2 * eps_t[0, 2]])
    for g in range(8):
        assert np.allclose(B[g] @ u, expect, atol=1e-12)


def test_weights_integrate_volume():
    _, w = q1.strain_matrices(H)
    assert abs(w.sum() - np.prod(H)) < 1e-15
    # partition of unity at the Gauss points
    assert np.allclose(q1.shape(q1.GAUSS).sum(axis=1), 1.0)


def test_element_stiffness_kernel_and_rank():
    mesh = Mesh(W.small_cube(S=(1, 1, 1), n=(1, 1, 1)))
    Ke = assembly.elastic_element_matrix(mesh)
    assert np.allclose(Ke, Ke.T, atol=1e-9 * np.abs(Ke).max())
    ev = np.linalg.eigvalsh(Ke)
    tol = 1e-10 * ev.max()
    assert (ev > -tol).all()
    assert int((ev > tol).sum()) == 18
    X = element_nodes(mesh.h)
    X = X - X.mean(axis=0)
    modes = []
    for t in np.eye(3):
        modes.append(np.tile(t, 8))
    for (i, j) in ((0, 1), (1, 2), (0, 2)):
        r = np.zeros((8, 3))
        r[:, i] = -X[:, j]
        r[:, j] = X[:, i]
        modes.append(r.ravel())
    for r in modes:
        assert np.linalg.norm(Ke @ r) <= 1e-12 * np.abs(Ke).max() * np.linalg.norm(r)


def test_face_load_totals():
    t = np.array([1.0, -2.0, 3.0])
    fl = q1.face_load((0.25, 0.5), t)
    assert np.allclose(fl.sum(axis=0), t * 0.125)
    assert np.allclose(fl, t[None] * 0.125 / 4)


def test_torn_load_total_force():
    w = W.small_cube(S=(2, 3, 2), n=(2, 2, 3), amp=250.0, shear=40.0)
    mesh = Mesh(w)
    f = mesh.torn_load(1.0).reshape(-1, 3)
    assert np.allclose(f.sum(axis=0), [40.0, 0.0, -250.0], rtol=1e-13)
