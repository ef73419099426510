"""FP64 CPU oracle for the TFETI semismooth-Newton elastoplastic solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the GPU library; both read
their inputs from the ``workloads`` module, which holds no solver arithmetic.

Everything here is plain numpy / scipy in float64, written from the paper
(Cermak, Kozubek, Sysala, Valdman, "A TFETI Domain Decomposition Solver for
Elastoplastic Problems"):

* ``constitutive`` - Hooke matrix, return mapping, generalized derivative
  (Sections 2.2-2.4 and their Voigt forms in Section 3.1).
* ``q1``           - trilinear hexahedron, 8-point Gauss rule.
* ``mesh``         - structured box mesh, box decomposition, orthonormal
  gluing matrix B (Section 4.1).
* ``tfeti``        - rigid modes, fixing-node generalized inverse (Remark 1),
  dual operator, projector, lumped preconditioner, PCGP (Algorithm 3).
* ``newton``       - subdomain assembly (Algorithm 5), semismooth Newton
  (Algorithms 2 and 4), time stepping (Algorithm 1), and the monolithic
  Dirichlet-eliminated reference solve (Section 3.1).
* ``mlp``          - FP64 reference of the warm-start network.

Pinned by the ``-m "not gpu"`` tests against closed forms, invariants and
brute-force solves; see tests/test_oracle_*.py.
"""
