"""CPU oracle for the vertex-patch multigrid smoother (test infrastructure only).

This package is a plain, slow, FP64 NumPy/SciPy restatement of the method of
Wichrowski, Munch, Kronbichler, Kanschat, "Smoothers with localized residual
computations for geometric multigrid methods" (arXiv 2407.02100).  It exists
to check the GPU library; it is not part of it.  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with ``paper_2407_02100_amd`` and imports
nothing from it; the only shared module is ``vps_inputs`` (seeded random data
and the nodal storage layout, no arithmetic of the method).

Modules
-------
fe           1D Q_k element: GLL nodes, Gauss rule, reference mass/stiffness
mesh         uniform Cartesian levels, vertex patches, colors
assemble     cell-by-cell sparse assembly (and the Kronecker-form operator)
transfer     prolongation by evaluation of coarse basis functions, restriction
smoother     exact/approximate dense local solvers and the sweeps of
             Algorithms 1, 2 and 3 (Section 3)
multigrid    V-cycle, PCG, flexible CG, stationary convergence factor
manufactured load vectors and L2 errors for the discretisation checks
learned      exact dense patch inverses -> per-eigenmode scaling targets
mlp          FP64 MLP forward/backward and Adam (checked by finite differences)

Parity status: every function is pinned by a CPU test under ``tests/`` (see
the test module names ``test_oracle_*``) except the mixed-precision and
learned *gains*, which are measured rather than pinned.
"""
