"""Subdomain assembly (Algorithm 5) and the nonlinear operator / tangent
(Section 3.1, definitions of F_k and K_k).

Oracle (test infrastructure).  For every element T of every subdomain and
every Gauss point g (weight w_g det J playing the role of |T|):

    deps_g   = B_g R_T du                       strain increment
    dsigma_g = T_k(deps_g),  dkappa_g = T_kappa(deps_g)   (return map)
    f       -= w_g B_g^T dsigma_g                (internal force)
    K       += w_g B_g^T T^o_k(deps_g) B_g       (generalized tangent)

The paper's Algorithm 5 writes the force update with dsigma_{k,T}; it must be
the dsigma_{k+1,T} computed one line earlier, which is what is used here.

State arrays are ordered subdomain-major, then local element (x fastest),
then Gauss point (xi fastest): shape (n_elems, 8, 6) for stresses.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import constitutive, q1


def element_dofs_torn(mesh) -> np.ndarray:
    """(n_elems, 24) torn DOF indices of every element, subdomain-major."""
    out = []
    for s in mesh.subs:
        nodes = s.elems                              # (n_el, 8) local
        d = s.off + 3 * nodes[:, :, None] + np.arange(3)[None, None, :]
        out.append(d.reshape(-1, 24))
    return np.concatenate(out, axis=0)


def element_dofs_global(mesh) -> np.ndarray:
    """(n_elems, 24) global (untorn) DOF indices, same element order."""
    out = []
    for s in mesh.subs:
        g = s.l2g[s.elems]
        d = 3 * g[:, :, None] + np.arange(3)[None, None, :]
        out.append(d.reshape(-1, 24))
    return np.concatenate(out, axis=0)


def assemble(mesh, edofs: np.ndarray, ndof: int, du: np.ndarray,
             sigma_k: np.ndarray, kappa_k: np.ndarray, want_K: bool = True):
    """Evaluate the return map at every Gauss point for the displacement
    increment du (indexed by edofs) and assemble the internal force vector
    sum_T (B^T dsigma) and, if asked, the tangent matrix.

    Returns dict(fint (ndof,), K (csr or None), dsigma, dkappa, plastic, phi).
    """
    m = mesh.w.material
    B, w = q1.strain_matrices(mesh.h)                # (8,6,24), (8,)
    du_e = du[edofs]                                 # (ne, 24)
    deps = np.einsum("gij,ej->egi", B, du_e)         # (ne, 8, 6)
    ne = du_e.shape[0]
    ds, dk, D, plastic, phi = constitutive.return_map(
        sigma_k.reshape(-1, 6), kappa_k.reshape(-1), deps.reshape(-1, 6),
        m.E, m.nu, m.sigma_y, m.H, want_tangent=want_K)
    ds = ds.reshape(ne, 8, 6)
    fe = np.einsum("g,gij,egi->ej", w, B, ds)        # sum_g w B^T dsigma
    fint = np.zeros(ndof)
    np.add.at(fint, edofs.ravel(), fe.ravel())
    K = None
    if want_K:
        D = D.reshape(ne, 8, 6, 6)
        DB = np.einsum("egij,gjk->egik", D, B)       # (ne, 8, 6, 24)
        Ke = np.einsum("g,gia,egib->eab", w, B, DB)  # (ne, 24, 24)
        rows = np.repeat(edofs, 24, axis=1).ravel()
        cols = np.tile(edofs, (1, 24)).ravel()
        K = sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(ndof, ndof))
        K.sum_duplicates()
    return dict(fint=fint, K=K, dsigma=ds, dkappa=dk.reshape(ne, 8),
                plastic=plastic.reshape(ne, 8), phi=phi.reshape(ne, 8))


def elastic_element_matrix(mesh) -> np.ndarray:
    """K_e of one element with the Hooke matrix at all Gauss points (24, 24)."""
    m = mesh.w.material
    B, w = q1.strain_matrices(mesh.h)
    C = constitutive.hooke_matrix(m.E, m.nu)
    return np.einsum("g,gia,ij,gjb->ab", w, B, C, B)
