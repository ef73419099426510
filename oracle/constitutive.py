"""Constitutive step of von Mises plasticity with linear isotropic hardening.

Oracle (test infrastructure).  Vectorised over points, float64.

Voigt convention (Section 3.1, stress/strain vector form): stresses are
(s11, s22, s33, s12, s23, s13); strains are (e11, e22, e33, 2e12, 2e23, 2e13).

* Hooke matrix C, deviatoric operators E_eps and E_sigma = P E_eps with
  P = diag(1,1,1,2,2,2), and the norm ||t||_sigma = sqrt(t^T P t)
  (Section 3.1, the matrix definitions that follow the vector form).
* Elastic predictor and plastic corrector (Section 2.4): the trial stress is
  sigma_k + C deps; if Phi(trial, kappa_k) <= 0 the step is elastic, else the
  plastic multiplier is Phi/(3 mu + H) and the stress is pulled back along the
  unit deviator by 3mu/(3mu+H) * sqrt(2/3) * Phi.
* Generalized derivative T^o (Section 2.4, its Voigt form in Section 3.1):
  C if elastic, else
  C - 2 mu beta E_eps - 2 mu beta sqrt(2/3) (sigma_y + H kappa_k)/||E_sigma tau||_sigma (n n^T - E_eps),
  with beta = 3 mu/(3 mu + H).  Note the hardening term uses kappa_k, the
  value at the start of the step.
"""

from __future__ import annotations

import numpy as np

SQRT23 = np.sqrt(2.0 / 3.0)
SQRT32 = np.sqrt(3.0 / 2.0)
YIELD_TIE = 1e-12  # relative margin of the elastic/plastic decision at Phi = 0


def lame(E: float, nu: float):
    """Lame coefficients from Young's modulus and Poisson's ratio (Section 5).

    The paper prints mu = 801938 for E = 206900, nu = 0.29; the formula gives
    80193.8..., which is what is used here."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def hooke_matrix(E: float, nu: float) -> np.ndarray:
    lam, mu = lame(E, nu)
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] = C[1, 1] = C[2, 2] = lam + 2.0 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def E_eps() -> np.ndarray:
    M = np.zeros((6, 6))
    M[:3, :3] = np.array([[2.0, -1.0, -1.0], [-1.0, 2.0, -1.0], [-1.0, -1.0, 2.0]]) / 3.0
    M[3, 3] = M[4, 4] = M[5, 5] = 1.5 / 3.0
    return M


def P_matrix() -> np.ndarray:
    return np.diag([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])


def E_sigma() -> np.ndarray:
    return P_matrix() @ E_eps()


def norm_sigma(t: np.ndarray) -> np.ndarray:
    """||t||_sigma = sqrt(t^T P t) over the last axis."""
    P = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])
    return np.sqrt(np.einsum("...i,i,...i->...", t, P, t))


def yield_function(tau: np.ndarray, kappa: np.ndarray, sigma_y: float, H: float) -> np.ndarray:
    """Phi(tau, kappa) = sqrt(3/2) ||E_sigma tau||_sigma - (sigma_y + H kappa)."""
    dev = tau @ E_sigma().T
    return SQRT32 * norm_sigma(dev) - (sigma_y + H * kappa)


def return_map(sigma_k: np.ndarray, kappa_k: np.ndarray, deps: np.ndarray,
               E: float, nu: float, sigma_y: float, H: float, want_tangent: bool = True):
    """Return mapping for arrays of points.

    sigma_k: (npts, 6) stress at t_k; kappa_k: (npts,); deps: (npts, 6) strain
    increment.  Returns (dsigma (npts,6), dkappa (npts,), D (npts,6,6) or None,
    plastic (npts,) bool, Phi (npts,) trial yield value).
    """
    sigma_k = np.asarray(sigma_k, dtype=np.float64).reshape(-1, 6)
    deps = np.asarray(deps, dtype=np.float64).reshape(-1, 6)
    kappa_k = np.asarray(kappa_k, dtype=np.float64).reshape(-1)
    lam, mu = lame(E, nu)
    C = hooke_matrix(E, nu)
    Ee = E_eps()
    Es = E_sigma()
    beta = 3.0 * mu / (3.0 * mu + H)

    Cde = deps @ C.T                       # C deps (elastic increment)
    tau = sigma_k + Cde                    # trial stress
    dev = tau @ Es.T                       # E_sigma tau
    ndev = norm_sigma(dev)
    phi = SQRT32 * ndev - (sigma_y + H * kappa_k)
    # Phi <= 0 is elastic.  A committed plastic point sits on the yield
    # surface, where rounding leaves Phi = O(1e-16) of either sign; the tie
    # is taken as elastic up to a relative margin of YIELD_TIE, so that the
    # tangent at a zero increment is always the elastic one.
    plastic = phi > YIELD_TIE * (sigma_y + H * kappa_k)

    safe = np.where(plastic, ndev, 1.0)
    nbar = dev / safe[:, None]
    phip = np.where(plastic, phi, 0.0)     # positive part of Phi
    dsigma = Cde - (beta * SQRT23 * phip)[:, None] * nbar
    dkappa = phip / (3.0 * mu + H)

    D = None
    if want_tangent:
        npts = sigma_k.shape[0]
        D = np.broadcast_to(C, (npts, 6, 6)).copy()
        if np.any(plastic):
            idx = np.nonzero(plastic)[0]
            nb = nbar[idx]
            coef = 2.0 * mu * beta * SQRT23 * (sigma_y + H * kappa_k[idx]) / ndev[idx]
            outer = np.einsum("pi,pj->pij", nb, nb)
            D[idx] = (C[None] - 2.0 * mu * beta * Ee[None]
                      - coef[:, None, None] * (outer - Ee[None]))
    return dsigma, dkappa, D, plastic, phi
