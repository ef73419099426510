"""Pins of the oracle's semismooth Newton / time stepping (Algorithms 1, 2, 4,
5): closed-form elastic and elastoplastic patch tests, TFETI against the
monolithic reference over plastic load steps, tangent = derivative of the
internal force, spectral equivalence of the tangent, the first Newton
iteration being elastic, and the quadratic tail."""

import numpy as np
import pytest

from oracle import assembly, constitutive
from oracle.newton import Solver
import workloads as W


def uniform_state_expect(q, mat, plastic_k):
    E, nu, sy, H = mat.E, mat.nu, mat.sigma_y, mat.H
    ezz = q / E + plastic_k
    exx = -nu * q / E - plastic_k / 2
    return exx, ezz


@pytest.mark.parametrize("linear", ["tfeti", "mono"])
def test_elastic_patch(linear):
    q = 120.0
    w = W.patch_test(S=(2, 2, 2), n=(2, 2, 2), q=q, steps=1)
    s = Solver(w, linear, eps_pcg=1e-12)
    s.run()
    mesh = s.mesh
    ug = s.global_displacement().reshape(-1, 3)
    i, j, k = mesh.node_ijk(np.arange(mesh.n_gnodes))
    x, y, z = i * mesh.h[0], j * mesh.h[1], k * mesh.h[2]
    exx, ezz = uniform_state_expect(q, w.material, 0.0)
    expect = np.stack([exx * x, exx * y, ezz * z], axis=1)
    assert np.abs(ug - expect).max() <= 1e-10 * np.abs(expect).max()
    sig = s.sigma.reshape(-1, 6)
    assert np.allclose(sig, [0, 0, q, 0, 0, 0], atol=1e-9 * q)


@pytest.mark.parametrize("linear", ["tfeti", "mono"])
def test_elastoplastic_patch(linear):
    """Uniaxial tension by q > sigma_y on rollers, ramped over 3 steps: the
    exact state is uniform with kappa = (q - sigma_y)/H,
    eps_zz = q/E + kappa, eps_xx = eps_yy = -nu q/E - kappa/2."""
    q = 700.0
    w = W.patch_test(S=(2, 1, 2), n=(2, 2, 2), q=q, steps=3)
    s = Solver(w, linear, eps_pcg=1e-12, eps_newton=1e-12)
    s.run()
    m = w.material
    kap = (q - m.sigma_y) / m.H
    assert np.allclose(s.kappa, kap, rtol=1e-10)
    mesh = s.mesh
    ug = s.global_displacement().reshape(-1, 3)
    i, j, k = mesh.node_ijk(np.arange(mesh.n_gnodes))
    x, y, z = i * mesh.h[0], j * mesh.h[1], k * mesh.h[2]
    exx, ezz = uniform_state_expect(q, m, kap)
    expect = np.stack([exx * x, exx * y, ezz * z], axis=1)
    assert np.abs(ug - expect).max() <= 1e-9 * np.abs(expect).max()
    assert np.allclose(s.sigma.reshape(-1, 6), [0, 0, q, 0, 0, 0], atol=1e-8 * q)


def test_tfeti_matches_monolithic_plastic():
    w = W.small_cube(S=(2, 2, 2), n=(2, 2, 3), amp=700.0, steps=3, shear=150.0)
    a = Solver(w, "tfeti")
    b = Solver(w, "mono")
    for _ in range(3):
        ha = a.load_step()
        hb = b.load_step()
        ua, ub = a.global_displacement(), b.global_displacement()
        assert np.linalg.norm(ua - ub) <= 1e-6 * np.linalg.norm(ub)
    assert ha[-1]["plastic_el"] > 0
    assert np.abs(a.kappa - b.kappa).max() <= 1e-6 * np.abs(b.kappa).max()


def test_tangent_is_derivative_of_internal_force():
    w = W.small_cube(S=(1, 1, 1), n=(2, 2, 2), amp=900.0, steps=1)
    s = Solver(w, "mono")
    rng = np.random.default_rng(0)
    # a state with many plastic points, then a random increment
    s.load_step()
    du = rng.standard_normal(s.n_global) * 1e-4
    du[~s.free] = 0.0
    a = assembly.assemble(s.mesh, s.edofs_g, s.n_global, du, s.sigma, s.kappa)
    assert a["plastic"].sum() > 0
    # skip if any point sits within the kink band
    phi = a["phi"]
    assert np.abs(phi).min() > 1e-3
    K = a["K"]
    v = rng.standard_normal(s.n_global)
    v[~s.free] = 0.0
    h = 1e-8
    fp = assembly.assemble(s.mesh, s.edofs_g, s.n_global, du + h * v, s.sigma, s.kappa, want_K=False)["fint"]
    fm = assembly.assemble(s.mesh, s.edofs_g, s.n_global, du - h * v, s.sigma, s.kappa, want_K=False)["fint"]
    fd = (fp - fm) / (2 * h)
    Kv = K @ v
    assert np.linalg.norm(fd - Kv) <= 1e-5 * np.linalg.norm(Kv)


def test_spectral_equivalence():
    w = W.small_cube(S=(1, 1, 1), n=(2, 2, 2), amp=900.0, steps=2)
    s = Solver(w, "mono")
    s.load_step()
    rng = np.random.default_rng(1)
    du = rng.standard_normal(s.n_global) * 2e-4
    du[~s.free] = 0.0
    a = assembly.assemble(s.mesh, s.edofs_g, s.n_global, du, s.sigma, s.kappa)
    ae = assembly.assemble(s.mesh, s.edofs_g, s.n_global, np.zeros(s.n_global),
                           np.zeros_like(s.sigma), np.zeros_like(s.kappa))
    assert a["plastic"].sum() > 0
    K = a["K"][s.free][:, s.free].toarray()
    Ke = ae["K"][s.free][:, s.free].toarray()
    lam, mu = constitutive.lame(w.material.E, w.material.nu)
    low = w.material.H / (3 * mu + w.material.H)
    L = np.linalg.cholesky(Ke)
    Li = np.linalg.inv(L)
    ev = np.linalg.eigvalsh(Li @ K @ Li.T)
    assert ev.min() >= low - 1e-9 and ev.max() <= 1 + 1e-9


def test_first_iteration_elastic_and_quadratic_tail():
    """Table 2 behaviour: iteration 1 solves an elastic problem (no plastic
    points, criterion 1); once the plastic set is fixed, the increment
    criterion decreases quadratically."""
    w = W.small_cube(S=(1, 1, 1), n=(3, 3, 3), amp=800.0, steps=1)
    s = Solver(w, "mono", eps_newton=1e-14)
    hist = s.load_step(criterion="increment")
    assert hist[0]["plastic_gp"] == 0 and hist[0]["crit"] == 1.0
    crit = [h["crit"] for h in hist]
    assert crit[-1] < 1e-12
    tail = [c for c in crit if c < 1e-2]
    ok = [tail[t + 1] <= 50.0 * tail[t] ** 2 for t in range(len(tail) - 1) if tail[t] > 1e-13]
    assert len(ok) >= 1 and all(ok)


def test_elastic_step_converges_in_one_solve():
    w = W.small_cube(S=(2, 1, 1), n=(2, 2, 2), amp=50.0, steps=1)
    s = Solver(w, "tfeti")
    hist = s.load_step()
    assert len(hist) == 1 and hist[0]["plastic_gp"] == 0
