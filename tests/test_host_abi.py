"""CPU tests of the HIP library's host side: the shared library loads and
exports every function declared in include/tfeti.h, and the host-built model
(decomposition, gluing matrix B, sizes) matches the oracle bit for bit.
No kernel is launched."""

import os
import re

import numpy as np
import pytest

import workloads as W
from oracle.mesh import Mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tfeti.h")
LIB = os.path.join(ROOT, "paper_1205_1926_amd", "libtfeti.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libtfeti.so not built (run __graft_entry__.build())")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("tfeti_setup", "tfeti_newton_step", "tfeti_dual_pcg", "return_map", "tfeti_fapply"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_1205_1926_amd import _capi
    assert set(_capi.SIGNATURES) == set(declared_functions())


def holed_cube():
    """3 x 3 x 2 boxes with the centre column and one corner box left out:
    nodes on the hole's faces are shared by fewer subdomains."""
    w = W.small_cube(S=(3, 3, 2), n=(2, 2, 2))
    w.absent = [(1, 1, 0), (1, 1, 1), (2, 2, 1)]
    return w


@pytest.mark.parametrize("w", [W.config(0), W.config(1), W.config(2), W.config(4),
                               W.small_cube(S=(3, 2, 2), n=(2, 3, 2)),
                               W.patch_test(S=(2, 2, 3), n=(2, 1, 2)),
                               W.Workload("uneven", (2, 3, 2), [3, 5], [2, 4, 3], [6, 2],
                                          dirichlet=[[1, 0, 0], [0, 0, 0], [0, 1, 0], [0, 0, 0], [1, 1, 1], [0, 0, 0]]),
                               W.plate_notch(1), W.plate_notch(2), holed_cube()])
def test_B_maps_bit_exact_with_oracle(w):
    from paper_1205_1926_amd import model_host
    sizes, rp, col, val = model_host(w)
    m = Mesh(w)
    assert (sizes["m"], sizes["m_G"], sizes["m_U"], sizes["n_torn"]) == (m.m, m.m_G, m.m_U, m.n_torn)
    assert np.array_equal(rp, m.B_indptr)
    assert np.array_equal(col, m.B_idx)
    assert np.array_equal(val.view(np.uint64), m.B_val.view(np.uint64))


def test_sizes_of_the_benchmark_mesh():
    """10x10x10 subdomains of 8^3 elements: multiplier counts and the skyline
    (envelope) of the factors, 535086 entries per subdomain."""
    from paper_1205_1926_amd import model_host
    sizes, *_ = model_host(W.config(4))
    assert sizes["n_sub"] == 1000 and sizes["n_torn"] == 2187000
    assert (sizes["m"], sizes["m_G"], sizes["m_U"]) == (612360, 588060, 24300)
    assert sizes["l"] == 6000
    assert sizes["skyline_entries"] == 535086 * 1000


def test_skyline_count_by_brute_force():
    """The library's envelope count equals the envelope of the oracle's
    assembled subdomain matrix (first nonzero column per row)."""
    from paper_1205_1926_amd import model_host
    from oracle import assembly
    w = W.small_cube(S=(1, 1, 1), n=(3, 2, 4))
    sizes, *_ = model_host(w)
    mesh = Mesh(w)
    ed = assembly.element_dofs_torn(mesh)
    a = assembly.assemble(mesh, ed, mesh.n_torn, np.zeros(mesh.n_torn), np.zeros((mesh.n_elems, 8, 6)),
                          np.zeros((mesh.n_elems, 8)))
    K = a["K"].tocsr()
    # factor ordering of the library: axes by increasing node count (here y, x, z)
    s = mesh.subs[0]
    N = [s.n[0] + 1, s.n[1] + 1, s.n[2] + 1]
    order = sorted(range(3), key=lambda ax: N[ax])
    perm = np.zeros(mesh.n_torn, dtype=np.int64)
    for a_ in range(s.n_nodes):
        ijk = [a_ % N[0], (a_ // N[0]) % N[1], a_ // (N[0] * N[1])]
        f = ijk[order[0]] + N[order[0]] * (ijk[order[1]] + N[order[1]] * ijk[order[2]])
        for c in range(3):
            perm[3 * a_ + c] = 3 * f + c
    Kp = K[np.argsort(perm)][:, np.argsort(perm)].tocsr()
    env = 0
    for r in range(Kp.shape[0]):
        cols = Kp.indices[Kp.indptr[r]:Kp.indptr[r + 1]]
        cols = cols[np.abs(Kp.data[Kp.indptr[r]:Kp.indptr[r + 1]]) > 0]
        env += r - cols.min() + 1
    assert sizes["skyline_entries"] == env


def test_holed_decomposition_refuses_only_dirichlet():
    """Where a hole's edge leaves interface nodes between free faces the
    interior of a subdomain is no box: the model still builds (lumped
    preconditioner), and the reason is kept for a Dirichlet set-up."""
    from paper_1205_1926_amd import model_host
    sizes, *_ = model_host(holed_cube())
    assert sizes["n_sub"] == 15


def test_invalid_problem_rejected():
    from paper_1205_1926_amd import model_host, TfetiError
    w = W.small_cube()
    w.material.H = 0.0
    with pytest.raises(TfetiError):
        model_host(w)
    w = W.small_cube(S=(1, 2, 1))
    w.absent = [(0, 0, 0), (0, 1, 0)]
    with pytest.raises(TfetiError):
        model_host(w)
    w = W.small_cube(S=(1, 2, 1))
    w.absent = [(0, 2, 0)]
    with pytest.raises(ValueError):
        model_host(w)


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes mirrors of the header's host structs have the C
    compiler's size and field offsets (a field added on one side only would
    shift every later one)."""
    import ctypes
    import shutil
    import subprocess
    from paper_1205_1926_amd import _capi
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"tfeti_options": _capi.Options, "tfeti_sizes": _capi.Sizes, "tfeti_pcg_report": _capi.PcgReport,
               "tfeti_newton_report": _capi.NewtonReport, "tfeti_problem": _capi.Problem,
               "tfeti_material": _capi.Material, "tfeti_mlp": _capi.Mlp}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tfeti.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        cname, f, v = line.split()
        py = structs[cname]
        want = ctypes.sizeof(py) if f == "sizeof" else getattr(py, f).offset
        assert int(v) == want, (cname, f, int(v), want)
        seen += 1
    assert seen == sum(len(p._fields_) + 1 for p in structs.values())
