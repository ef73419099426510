"""Trilinear hexahedron (Q1) with the 2x2x2 Gauss rule.

Oracle (test infrastructure).  The paper uses linear tetrahedra with one
constant state per element (Section 3.1); the synthetic workloads use Q1
hexahedra, so the same per-element formulas (Algorithm 5: strain
G_T R_T u, stress increment by the return map, internal force and tangent
weighted by the element measure) are applied per Gauss point with weight
w_g det J instead of |T|.

Element node order on the reference cube [-1, 1]^3:
(0,0,0), (1,0,0), (1,1,0), (0,1,0), (0,0,1), (1,0,1), (1,1,1), (0,1,1),
where 0 -> -1 and 1 -> +1.  Element DOF 3a + c is component c of node a.
Gauss points +-1/sqrt(3) with xi fastest, all weights 1.
"""

from __future__ import annotations

import numpy as np

NODE_REF = np.array([
    [-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
    [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1],
], dtype=np.float64)

# local (i, j, k) offsets of the element nodes within the node lattice
NODE_OFF = ((NODE_REF + 1) // 2).astype(np.int64)

_g = 1.0 / np.sqrt(3.0)
GAUSS = np.array([[(-_g, _g)[i], (-_g, _g)[j], (-_g, _g)[k]]
                  for k in range(2) for j in range(2) for i in range(2)])


def shape(xi: np.ndarray) -> np.ndarray:
    """N_a(xi) = 1/8 (1 + xi xi_a)(1 + eta eta_a)(1 + zeta zeta_a)."""
    xi = np.atleast_2d(xi)
    return 0.125 * np.prod(1.0 + xi[:, None, :] * NODE_REF[None, :, :], axis=2)


def shape_grad_ref(xi: np.ndarray) -> np.ndarray:
    """dN_a/dxi_d at points xi: (npts, 8, 3)."""
    xi = np.atleast_2d(xi)
    f = 1.0 + xi[:, None, :] * NODE_REF[None, :, :]          # (npts, 8, 3)
    out = np.empty_like(f)
    for d in range(3):
        others = [e for e in range(3) if e != d]
        out[:, :, d] = 0.125 * NODE_REF[None, :, d] * f[:, :, others[0]] * f[:, :, others[1]]
    return out


def strain_matrices(h) -> tuple[np.ndarray, np.ndarray]:
    """Strain-displacement matrices B_g (8, 6, 24) and weights w_g det J (8,)
    for an axis-aligned box element with edge lengths h = (hx, hy, hz)."""
    h = np.asarray(h, dtype=np.float64)
    dref = shape_grad_ref(GAUSS)                 # (8 gp, 8 nodes, 3)
    dN = dref * (2.0 / h)[None, None, :]         # d/dx = d/dxi * 2/h
    B = np.zeros((8, 6, 24))
    for a in range(8):
        dx, dy, dz = dN[:, a, 0], dN[:, a, 1], dN[:, a, 2]
        B[:, 0, 3 * a + 0] = dx
        B[:, 1, 3 * a + 1] = dy
        B[:, 2, 3 * a + 2] = dz
        B[:, 3, 3 * a + 0] = dy          # 2 e12 = du1/dx2 + du2/dx1
        B[:, 3, 3 * a + 1] = dx
        B[:, 4, 3 * a + 1] = dz          # 2 e23 = du2/dx3 + du3/dx2
        B[:, 4, 3 * a + 2] = dy
        B[:, 5, 3 * a + 0] = dz          # 2 e13 = du1/dx3 + du3/dx1
        B[:, 5, 3 * a + 2] = dx
    w = np.full(8, np.prod(h) / 8.0)
    return B, w


def face_load(h2, t: np.ndarray) -> np.ndarray:
    """Consistent nodal loads of a uniform traction t (3,) on a bilinear face
    with edge lengths h2 = (ha, hb), by the 2x2 Gauss rule.  Returns (4, 3),
    face nodes ordered (0,0), (1,0), (1,1), (0,1) in the face's own axes."""
    ref = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
    out = np.zeros((4, 3))
    jac = h2[0] * h2[1] / 4.0
    for gj in (-_g, _g):
        for gi in (-_g, _g):
            N = 0.25 * (1 + gi * ref[:, 0]) * (1 + gj * ref[:, 1])
            out += N[:, None] * t[None, :] * jac
    return out
