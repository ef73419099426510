"""Pins of the oracle's constitutive step (Sections 2.2-2.4, Voigt forms of
Section 3.1) against definitions it does not itself evaluate: the tensor form
of Hooke's law, the discrete constitutive problem (discrete flow rule,
hardening law and loading/unloading conditions), finite differences of the
stress operator, and the bounds on its generalized derivative."""

import os

import numpy as np
import pytest

from oracle import constitutive as cm

HERE = os.path.dirname(__file__)
MAT = dict(E=206900.0, nu=0.29, sigma_y=450.0, H=10000.0)


def _golden():
    vals = {}
    for line in open(os.path.join(HERE, "golden", "paper_section5_material.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        vals[k] = float(v)
    return vals


def voigt_to_tensor_stress(s):
    return np.array([[s[0], s[3], s[5]], [s[3], s[1], s[4]], [s[5], s[4], s[2]]])


def voigt_to_tensor_strain(e):
    return np.array([[e[0], e[3] / 2, e[5] / 2], [e[3] / 2, e[1], e[4] / 2], [e[5] / 2, e[4] / 2, e[2]]])


def tensor_to_voigt_stress(t):
    return np.array([t[0, 0], t[1, 1], t[2, 2], t[0, 1], t[1, 2], t[0, 2]])


def tensor_to_voigt_strain(t):
    return np.array([t[0, 0], t[1, 1], t[2, 2], 2 * t[0, 1], 2 * t[1, 2], 2 * t[0, 2]])


def dev(t):
    return t - np.trace(t) / 3.0 * np.eye(3)


def test_lame_matches_paper_section5():
    g = _golden()
    lam, mu = cm.lame(g["E"], g["nu"])
    assert abs(lam - g["lambda"]) < 0.05
    assert abs(mu - g["mu"]) < 0.05


def test_hooke_voigt_equals_tensor_law():
    rng = np.random.default_rng(0)
    C = cm.hooke_matrix(MAT["E"], MAT["nu"])
    lam, mu = cm.lame(MAT["E"], MAT["nu"])
    for _ in range(20):
        a = rng.standard_normal((3, 3))
        eps = 0.5 * (a + a.T)
        sig_t = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps
        assert np.allclose(C @ tensor_to_voigt_strain(eps), tensor_to_voigt_stress(sig_t), rtol=1e-14, atol=1e-9)


def test_deviator_and_norm_match_tensor_definitions():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a = rng.standard_normal((3, 3))
        t = 0.5 * (a + a.T)
        tv = tensor_to_voigt_stress(t)
        assert np.allclose(cm.E_sigma() @ tv, tensor_to_voigt_stress(dev(t)), atol=1e-14)
        assert abs(cm.norm_sigma(tv) - np.linalg.norm(t)) < 1e-13
        # E_eps maps an engineering strain vector to the tensor deviator components
        e = 0.5 * (a + a.T)
        ev = tensor_to_voigt_strain(e)
        assert np.allclose(cm.E_eps() @ ev, tensor_to_voigt_stress(dev(e)), atol=1e-14)


def _random_states(n, seed, scale=2e-3):
    rng = np.random.default_rng(seed)
    sig = rng.standard_normal((n, 6)) * 150.0
    kap = np.abs(rng.standard_normal(n)) * 1e-3
    de = rng.standard_normal((n, 6)) * scale
    return sig, kap, de


def test_elastic_predictor_exact():
    sig, kap, de = _random_states(200, 2, scale=1e-6)
    sig *= 0.1
    ds, dk, D, pl, phi = cm.return_map(sig, kap, de, **MAT)
    C = cm.hooke_matrix(MAT["E"], MAT["nu"])
    assert not pl.any() and (phi <= 0).all()
    assert np.array_equal(ds, de @ C.T)
    assert np.all(dk == 0.0)
    assert np.array_equal(D, np.broadcast_to(C, D.shape))


def test_discrete_constitutive_problem_is_solved():
    """The return map must solve the discrete constitutive problem of Section 2.4:
    C^{-1}(trial - sigma) = dgamma sqrt(3/2) dev(sigma)/|dev(sigma)|,
    kappa - kappa_k = dgamma, dgamma >= 0, Phi(sigma, kappa) <= 0, dgamma Phi = 0."""
    sig, kap, de = _random_states(400, 3)
    E, nu, sy, H = MAT["E"], MAT["nu"], MAT["sigma_y"], MAT["H"]
    ds, dk, D, pl, _ = cm.return_map(sig, kap, de, E, nu, sy, H)
    assert pl.sum() > 50 and (~pl).sum() > 20
    lam, mu = cm.lame(E, nu)
    C = cm.hooke_matrix(E, nu)
    Cinv = np.linalg.inv(C)
    for p in range(len(sig)):
        s1 = sig[p] + ds[p]
        k1 = kap[p] + dk[p]
        trial = sig[p] + C @ de[p]
        T1 = voigt_to_tensor_stress(s1)
        phi1 = np.sqrt(1.5) * np.linalg.norm(dev(T1)) - (sy + H * k1)
        dgam = dk[p]
        assert dgam >= 0.0
        assert phi1 <= 1e-9 * sy
        assert abs(dgam * phi1) <= 1e-9 * sy * max(dgam, 1e-30)
        ep = voigt_to_tensor_strain(Cinv @ (trial - s1))      # plastic strain increment
        if pl[p]:
            flow = dgam * np.sqrt(1.5) * dev(T1) / np.linalg.norm(dev(T1))
            assert np.allclose(ep, flow, rtol=1e-9, atol=1e-14 + 1e-9 * np.abs(flow).max())
            assert abs(phi1) <= 1e-10 * sy
        else:
            assert np.allclose(s1, trial, rtol=0, atol=1e-12 * np.abs(trial).max())


def test_uniaxial_closed_form():
    """Uniaxial tension beyond yield (sigma_11 = s, other stresses zero) reached in
    one step from the virgin state: with linear hardening the plastic strain is
    eps_p = (s - sigma_y)/H along (1, -1/2, -1/2) and kappa = eps_p (Section 2.3
    flow and hardening laws integrated in closed form)."""
    E, nu, sy, H = MAT["E"], MAT["nu"], MAT["sigma_y"], MAT["H"]
    s = 600.0
    ep = (s - sy) / H
    eps_el = np.array([s / E, -nu * s / E, -nu * s / E, 0, 0, 0])
    eps_pl = np.array([ep, -ep / 2, -ep / 2, 0, 0, 0])
    de = eps_el + eps_pl
    ds, dk, D, pl, _ = cm.return_map(np.zeros((1, 6)), np.zeros(1), de[None], E, nu, sy, H)
    assert pl[0]
    assert np.allclose(ds[0], [s, 0, 0, 0, 0, 0], atol=1e-9 * s)
    assert abs(dk[0] - ep) < 1e-12


def _central_fd(sig, kap, de, h=1e-9):
    J = np.zeros((6, 6))
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        sp_, _, _, _, _ = cm.return_map(sig[None], kap[None], (de + e)[None], **MAT, want_tangent=False)
        sm_, _, _, _, _ = cm.return_map(sig[None], kap[None], (de - e)[None], **MAT, want_tangent=False)
        J[:, j] = (sp_[0] - sm_[0]) / (2 * h)
    return J


def test_tangent_equals_finite_difference():
    sig, kap, de = _random_states(60, 4)
    ds, dk, D, pl, phi = cm.return_map(sig, kap, de, **MAT)
    checked = 0
    for p in range(len(sig)):
        if abs(phi[p]) < 5.0:         # away from the kink Phi = 0
            continue
        J = _central_fd(sig[p], kap[p], de[p])
        assert np.allclose(D[p], J, rtol=1e-5, atol=1e-5 * np.abs(D[p]).max())
        checked += pl[p]
    assert checked > 10


def test_tangent_symmetric_and_bounded():
    """C >= T^o >= H/(3mu+H) C in the energy sense (Section 2.4)."""
    sig, kap, de = _random_states(300, 5)
    ds, dk, D, pl, _ = cm.return_map(sig, kap, de, **MAT)
    lam, mu = cm.lame(MAT["E"], MAT["nu"])
    low = MAT["H"] / (3 * mu + MAT["H"])
    C = cm.hooke_matrix(MAT["E"], MAT["nu"])
    L = np.linalg.cholesky(C)
    Li = np.linalg.inv(L)
    for p in np.nonzero(pl)[0]:
        assert np.allclose(D[p], D[p].T, atol=1e-9 * np.abs(D[p]).max())
        ev = np.linalg.eigvalsh(Li @ D[p] @ Li.T)
        assert ev.min() >= low - 1e-10 and ev.max() <= 1 + 1e-10
