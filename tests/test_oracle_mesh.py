"""Pins of the oracle's decomposition and orthonormal gluing matrix B
(Section 4.1): row counts from a closed-form count of node multiplicities,
B B^T = I, B annihilates continuous fields, B_U selects exactly the
Dirichlet copies, full row rank."""

import numpy as np
import pytest

from oracle.mesh import Mesh
import workloads as W


def closed_form_counts(S, n, dirichlet_bottom=True):
    """Count multipliers of a cube of S^3 subdomains with n^3 elements each,
    clamped on z = 0: a node on k_a interior slab planes per axis belongs to
    prod(2^k_a) subdomains; a free (node, comp) with k copies gives k-1 gluing
    rows, a clamped one gives k Dirichlet rows."""
    N = S * n
    mult = np.array([2 if (0 < i < N and i % n == 0) else 1 for i in range(N + 1)])
    kk = mult[:, None, None] * mult[None, :, None] * mult[None, None, :]   # (i, j, k)
    bottom = np.zeros_like(kk, dtype=bool)
    bottom[:, :, 0] = True
    mG = 3 * int((kk[~bottom] - 1).sum())
    mU = 3 * int(kk[bottom].sum())
    n_torn = 3 * (n + 1) ** 3 * S ** 3
    return mG, mU, n_torn


@pytest.mark.parametrize("cfg,S,n", [(0, 2, 4), (1, 4, 8)])
def test_counts_closed_form(cfg, S, n):
    mesh = Mesh(W.config(cfg))
    mG, mU, nt = closed_form_counts(S, n)
    assert (mesh.m_G, mesh.m_U, mesh.n_torn) == (mG, mU, nt)


def test_counts_config0_values():
    mesh = Mesh(W.config(0))
    assert (mesh.m_G, mesh.m_U, mesh.m, mesh.n_torn) == (756, 300, 1056, 3000)


@pytest.mark.parametrize("w", [W.config(0), W.small_cube(S=(3, 2, 2), n=(2, 3, 2)), W.patch_test(S=(2, 2, 3), n=(2, 1, 2))])
def test_B_orthonormal_and_annihilates_continuous(w):
    mesh = Mesh(w)
    B = mesh.B
    BBt = (B @ B.T).toarray()
    assert np.abs(BBt - np.eye(mesh.m)).max() <= 1e-15
    rng = np.random.default_rng(0)
    ug = rng.standard_normal(3 * mesh.n_gnodes)
    ug.reshape(-1, 3)[mesh.dir_mask] = 0.0                 # admissible field
    ut = mesh.tear(ug)
    assert np.abs(B @ ut).max() < 1e-14
    # a torn field with one copy changed violates exactly the rows touching it
    ut2 = ut.copy()
    j = mesh.B_idx[0]
    ut2[j] += 1.0
    assert np.count_nonzero(np.abs(B @ ut2) > 1e-12) >= 1


def test_B_U_rows_select_dirichlet_copies():
    w = W.patch_test(S=(2, 2, 2), n=(2, 2, 2))
    mesh = Mesh(w)
    BU = mesh.B[mesh.m_G:]
    assert np.all(BU.getnnz(axis=1) == 1)
    assert np.all(BU.data == 1.0)
    # every Dirichlet copy is selected once, nothing else
    sel = set(BU.indices.tolist())
    expect = set()
    for s in mesh.subs:
        for a, g in enumerate(s.l2g):
            for c in range(3):
                if mesh.dir_mask[g, c]:
                    expect.add(s.off + 3 * a + c)
    assert sel == expect


def test_B_row_order_and_helmert_coefficients():
    mesh = Mesh(W.config(0))
    # rows of B_G come first; each glue row has coefficients summing to zero
    for r in range(mesh.m_G):
        a, b = mesh.B_indptr[r], mesh.B_indptr[r + 1]
        v = mesh.B_val[a:b]
        assert abs(v.sum()) < 1e-15
        assert v[-1] < 0 and np.all(v[:-1] > 0)
