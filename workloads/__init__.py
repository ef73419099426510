"""Seeded synthetic workload definitions shared by the oracle and the HIP path.

This module holds inputs only: box geometry, per-axis slab sizes, material
constants, face loads, Dirichlet masks, step counts and tolerances, and the
counter-based generator that draws the seeded values.  It contains none of the
solver's arithmetic (no element integration, no constitutive law, no gluing),
so that the oracle and the GPU library can both consume it without sharing any
of the method.

The paper's benchmark (a perforated plate meshed with tetrahedra, Section 5)
is not reproducible here: its meshes are not available.  The synthetic
stand-ins are unit cubes meshed with trilinear hexahedra and split into
box-shaped subdomains, loaded on the top face and clamped on the bottom face.
Material constants are the paper's (Section 5): E = 206900, nu = 0.29,
sigma_y = 450, H_m = 10000.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

MASK64 = (1 << 64) - 1

# Face indices: 0: x=0, 1: x=X, 2: y=0, 3: y=Y, 4: z=0, 5: z=Z.
FACE_X0, FACE_X1, FACE_Y0, FACE_Y1, FACE_Z0, FACE_Z1 = range(6)


class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): a 64-bit counter-based
    generator.  Each draw advances the state by the golden-ratio increment and
    mixes it with two xor-shift-multiply rounds."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float, hi: float) -> float:
        """lo + (hi - lo) * u with u the top 53 bits scaled to [0, 1)."""
        return lo + (hi - lo) * ((self.next_u64() >> 11) * 2.0 ** -53)

    def slab(self) -> int:
        """An element count per slab drawn from {6, 7, 8, 9, 10}."""
        return 6 + self.next_u64() % 5


@dataclass
class Material:
    E: float = 206900.0
    nu: float = 0.29
    sigma_y: float = 450.0
    H: float = 10000.0


@dataclass
class Workload:
    """One synthetic problem: geometry, material, boundary data and schedule."""
    name: str
    S: Tuple[int, int, int]                 # subdomains per axis
    nx: List[int]                           # elements per x-slab (len S[0])
    ny: List[int]
    nz: List[int]
    extent: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    material: Material = field(default_factory=Material)
    # dirichlet[face][comp] == 1: u_comp = 0 on that face
    dirichlet: List[List[int]] = field(default_factory=lambda: [[0, 0, 0] for _ in range(6)])
    # traction[face] = traction vector on that face at load factor 1
    traction: List[List[float]] = field(default_factory=lambda: [[0.0, 0.0, 0.0] for _ in range(6)])
    steps: int = 1
    eps_newton: float = 1e-10
    eps_pcg: float = 1e-8
    precision: str = "fp64"                 # "fp64" or "fp32" (factor precision)
    # boxes (I, J, K) of the decomposition left out of the body (a hole or
    # notch through it); their exposed faces carry no load and no constraint
    absent: List[Tuple[int, int, int]] = field(default_factory=list)
    # load path: "ramp" k/N, or "sine": sin(pi/2 k/N), the amplitude
    # 400 sin(2 pi t) of the paper's benchmark at t_k = k (1/4) / N
    load_kind: str = "ramp"

    @property
    def n_elements(self) -> int:
        return sum(self.nx) * sum(self.ny) * sum(self.nz)

    def load_factor(self, k: int) -> float:
        """Load factor at the end of step k (k = 1..N): k/N on the linear
        ramp, sin(pi/2 k/N) on the quarter sine."""
        if self.load_kind == "sine":
            return math.sin(0.5 * math.pi * k / self.steps)
        return k / self.steps


def _clamped_bottom() -> List[List[int]]:
    d = [[0, 0, 0] for _ in range(6)]
    d[FACE_Z0] = [1, 1, 1]
    return d


def config(index: int, load_seed: int = 0, mesh_seed: int = 2026) -> Workload:
    """The five synthetic configurations of the benchmark plan.

    0: 2x2x2 subdomains of 4^3 elements, top traction -z in [300, 500], 5 steps.
    1: 4x4x4 subdomains of 8^3 elements, top traction -z in [400, 600], 10 steps.
    2: 8x8x8 subdomains with per-axis slab sizes drawn from {6..10}
       (mesh_seed), top shear +x in [200, 400], 20 steps, FP32 factors.
    3: the mesh of 2 (learned warm start; same geometry, other load seeds).
    4: 10x10x10 subdomains of 8^3 elements, top compression in [300, 500]
       plus shear +x in [200, 400], 30 steps.
    """
    rng = SplitMix64(load_seed)
    if index == 0:
        amp = rng.uniform(300.0, 500.0)
        w = Workload("cube2x2x2_sub4", (2, 2, 2), [4] * 2, [4] * 2, [4] * 2,
                     dirichlet=_clamped_bottom(), steps=5)
        w.traction[FACE_Z1] = [0.0, 0.0, -amp]
        return w
    if index == 1:
        amp = rng.uniform(400.0, 600.0)
        w = Workload("cube4x4x4_sub8", (4, 4, 4), [8] * 4, [8] * 4, [8] * 4,
                     dirichlet=_clamped_bottom(), steps=10)
        w.traction[FACE_Z1] = [0.0, 0.0, -amp]
        return w
    if index in (2, 3):
        mrng = SplitMix64(mesh_seed)
        nx = [mrng.slab() for _ in range(8)]
        ny = [mrng.slab() for _ in range(8)]
        nz = [mrng.slab() for _ in range(8)]
        amp = rng.uniform(200.0, 400.0)
        w = Workload("cube8x8x8_uneven", (8, 8, 8), nx, ny, nz,
                     dirichlet=_clamped_bottom(), steps=20, precision="fp32")
        w.traction[FACE_Z1] = [amp, 0.0, 0.0]
        return w
    if index == 4:
        comp = rng.uniform(300.0, 500.0)
        shear = rng.uniform(200.0, 400.0)
        w = Workload("cube10x10x10_sub8", (10, 10, 10), [8] * 10, [8] * 10, [8] * 10,
                     dirichlet=_clamped_bottom(), steps=30)
        w.traction[FACE_Z1] = [shear, 0.0, -comp]
        return w
    raise ValueError(f"unknown config {index}")


def patch_test(S=(2, 2, 2), n=(2, 2, 2), q: float = 100.0, steps: int = 1) -> Workload:
    """Unit cube on symmetry rollers (u_x = 0 on x=0, u_y = 0 on y=0,
    u_z = 0 on z=0) with a uniform normal traction q on z = 1."""
    d = [[0, 0, 0] for _ in range(6)]
    d[FACE_X0] = [1, 0, 0]
    d[FACE_Y0] = [0, 1, 0]
    d[FACE_Z0] = [0, 0, 1]
    w = Workload("patch", tuple(S), [n[0]] * S[0], [n[1]] * S[1], [n[2]] * S[2],
                 dirichlet=d, steps=steps)
    w.traction[FACE_Z1] = [0.0, 0.0, q]
    return w


def small_cube(S=(2, 2, 2), n=(2, 2, 2), amp: float = 400.0, steps: int = 1,
               shear: float = 0.0) -> Workload:
    """A small clamped-bottom cube for fast tests (top traction -z, optional +x shear)."""
    w = Workload(f"cube{S[0]}x{S[1]}x{S[2]}_sub{n[0]}x{n[1]}x{n[2]}", tuple(S),
                 [n[0]] * S[0], [n[1]] * S[1], [n[2]] * S[2],
                 dirichlet=_clamped_bottom(), steps=steps)
    w.traction[FACE_Z1] = [shear, 0.0, -amp]
    return w


def plate_notch(level: int = 1, steps: int = 1, amp: float = 400.0, eps_newton: float = 1e-9,
                eps_pcg: float = 1e-12) -> Workload:
    """Stand-in for the paper's benchmark (Section 5): an eighth of a
    20 x 20 x 2 plate, x, y in [0, 10], z in [0, 1], with symmetry rollers on
    x = 0 (u_x), y = 0 (u_y) and z = 0 (u_z), loaded in tension by the
    traction (0, g(t), 0) on y = 10 with g(t) = amp sin(2 pi t), t in
    [0, 1/4], in `steps` equal time steps (the paper's discretizations (a)
    steps = 1 and (b) steps = 8).  The paper's hole of radius 1 and its
    tetrahedral meshes are not available; the hole here is the square
    [0, 1] x [0, 1] through the thickness, boxes of the decomposition left
    out, so that every subdomain stays a box.  Elements of 1 / (4 level).
    Level 1: boxes 1, 3, 3, 3 units wide in x and y, one in z (15
    subdomains, 6 336 elements).  Level >= 2: cubic boxes of at most 8
    elements per axis, k per unit length (level 2: 99 subdomains of 8^3,
    50 688 elements; level 4: 792 subdomains of 8^3, 405 504 elements)."""
    e = 4 * level                              # elements per unit length
    if level == 1:
        k, bx, bz = 1, [e, 3 * e, 3 * e, 3 * e], [e]
    else:
        k = next(k for k in range(1, e + 1) if e % k == 0 and e // k <= 8)
        bx, bz = [e // k] * (10 * k), [e // k] * k
    w = Workload(f"plate_notch_l{level}_n{steps}", (len(bx), len(bx), len(bz)), bx, list(bx), bz,
                 extent=(10.0, 10.0, 1.0), steps=steps, eps_newton=eps_newton, eps_pcg=eps_pcg,
                 load_kind="sine")
    w.dirichlet[FACE_X0] = [1, 0, 0]
    w.dirichlet[FACE_Y0] = [0, 1, 0]
    w.dirichlet[FACE_Z0] = [0, 0, 1]
    w.traction[FACE_Y1] = [0.0, amp, 0.0]
    w.absent = [(i, j, m) for m in range(len(bz)) for j in range(k) for i in range(k)]
    return w


def mlp_init(seed: int = 0, dims=(31, 256, 256, 21)):
    """Seeded He-style initial weights of the warm-start perceptron: W_l
    (out x in) normal with variance 2 / in, zero biases.  These are random
    inputs of the training run, shared by the oracle and the GPU path."""
    import numpy as np
    rng = np.random.default_rng(seed)
    params = {}
    for l in range(3):
        fan_in, fan_out = dims[l], dims[l + 1]
        params[f"W{l + 1}"] = rng.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in)
        params[f"b{l + 1}"] = np.zeros(fan_out)
    return params
