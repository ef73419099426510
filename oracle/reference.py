"""Oracle results at the full sizes of the benchmark meshes.

Oracle (test infrastructure), float64.  Nothing in the product path may use
this module; the full-size parity tests and the accuracy leg of the benchmark
do.

At zero state every Gauss point takes the elastic branch of the return map
(Section 2.4), so the tangent of the first Newton iteration of the first load
step is the elastic stiffness K = diag(K_p) (Section 4.1).  The stiffness of
a box subdomain depends only on its element counts per axis, the element
size and the material: every element of the structured mesh has the same
element matrix, and the local numbering is the same lexicographic one.  The
blocks are therefore assembled once per distinct subdomain shape, by the
same assembly routine (Algorithm 5) on a one-subdomain mesh of that shape,
and placed on the diagonal (pinned against the assembly of the whole mesh in
tests/test_oracle_reference.py).

``elastic_first_step`` then follows Algorithm 4 for load step 1: Newton
iteration 1 solves K du = df by TFETI (Algorithm 3); iteration 2 evaluates
the return map at du and stops if the relative residual of the assembled
system is within the Newton tolerance (Algorithm 2 with the residual reading
of oracle.newton).  It refuses a step that is not elastic (a plastic first
step needs oracle.newton.Solver and its full tangent assembly).
"""

from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.sparse as sp

from . import assembly
from .mesh import Mesh
from .tfeti import TFETI


def elastic_tangent_blocks(mesh, log=None) -> sp.csr_matrix:
    """Torn elastic stiffness diag(K_p) of a box decomposition, each distinct
    subdomain shape assembled once on a one-subdomain mesh."""
    cache = {}
    blocks = []
    for s in mesh.subs:
        key = tuple(int(v) for v in s.n)
        if key not in cache:
            w1 = dataclasses.replace(mesh.w, name="one", S=(1, 1, 1), nx=[key[0]], ny=[key[1]], nz=[key[2]],
                                     extent=tuple(key[d] * mesh.h[d] for d in range(3)), absent=[])
            one = Mesh(w1)
            ed = assembly.element_dofs_torn(one)
            ne = one.n_elems
            a = assembly.assemble(one, ed, one.n_torn, np.zeros(one.n_torn), np.zeros((ne, 8, 6)),
                                  np.zeros((ne, 8)))
            cache[key] = a["K"].tocsr()
        blocks.append(cache[key])
    if log:
        log(f"oracle: {len(cache)} distinct subdomain shapes assembled")
    return sp.block_diag(blocks, format="csr")


def assembled_norm(mesh, v: np.ndarray) -> float:
    """Norm over free global DOFs of a torn force vector summed over the
    subdomain copies of each node."""
    rg = np.zeros(3 * mesh.n_gnodes)
    for s in mesh.subs:
        np.add.at(rg.reshape(-1, 3), s.l2g, v[s.off:s.off + s.n_dofs].reshape(-1, 3))
    return float(np.linalg.norm(rg[~mesh.dir_mask.ravel() & np.repeat(mesh.used, 3)]))


def elastic_first_step(w, log=None, fapply_seed: int | None = None):
    """Load step 1 of workload w from the zero state.  Returns the mesh, the
    TFETI object (factorized elastic K), du (torn), lambda, the PCGP
    iteration count, the relative residual at du and wall times; with
    fapply_seed also lam_F (seeded standard normal) and F lam_F."""
    say = log or (lambda msg: None)
    t = {}
    t0 = time.perf_counter()
    mesh = Mesh(w)
    t["mesh"] = time.perf_counter() - t0
    say(f"oracle: mesh of {w.name}: {len(mesh.subs)} subdomains, n={mesh.n_torn}, m={mesh.m}")
    t0 = time.perf_counter()
    K = elastic_tangent_blocks(mesh, say)
    t["assembly"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    tf = TFETI(mesh)
    t["coarse"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    tf.set_matrix(K)
    t["factorization"] = time.perf_counter() - t0
    say(f"oracle: {len(mesh.subs)} subdomain factorizations in {t['factorization']:.1f} s")
    out = dict(mesh=mesh, tf=tf, times=t)
    if fapply_seed is not None:
        lam = np.random.default_rng(fapply_seed).standard_normal(mesh.m)
        t0 = time.perf_counter()
        out["lam_F"] = lam
        out["F_lam"] = tf.F(lam)
        t["fapply"] = time.perf_counter() - t0
    df = mesh.torn_load(w.load_factor(1) - w.load_factor(0))
    t0 = time.perf_counter()
    res = tf.solve(df, eps=w.eps_pcg)
    t["solve"] = time.perf_counter() - t0
    say(f"oracle: PCGP {res['iters']} iterations in {t['solve']:.1f} s")
    if not res["converged"]:
        raise RuntimeError("oracle PCGP did not converge")
    du = res["u"]
    t0 = time.perf_counter()
    ne = mesh.n_elems
    a = assembly.assemble(mesh, assembly.element_dofs_torn(mesh), mesh.n_torn, du, np.zeros((ne, 8, 6)),
                          np.zeros((ne, 8)), want_K=False)
    t["return_map"] = time.perf_counter() - t0
    n_plastic = int(np.count_nonzero(a["plastic"]))
    relres = assembled_norm(mesh, df - a["fint"]) / assembled_norm(mesh, df)
    if n_plastic or relres > w.eps_newton:
        raise RuntimeError(f"load step 1 of {w.name} is not elastic ({n_plastic} plastic points, "
                           f"relative residual {relres:.2e})")
    out.update(du=du, lam=res["lam"], iters=res["iters"], relres=relres, untorn=mesh.untorn_index())
    return out
