"""Reference oracle for octree local timestepping (LTS) — TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, FP64 CPU implementation of what the GPU hot path
computes, written from the paper "Scalable Local Timestepping on Octree Grids"
(Fernando & Sundar, arXiv 2011.10570).  Only the test-suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
The product package never imports it and shares no code with it: the only
common dependency is the seeded input generator package ``workloads`` (which
holds no arithmetic of the method).

Modules
  rk        Runge-Kutta tableaus, the stage/derivative relation K = C P D and the
            exact-rational stage-conversion weights (Sec. 3.6.2, eqs. rk_crrection,
            fc_1, fc_2).
  octree    linear octree, refinement criteria, ghost-reach balance, octree-to-block
            decomposition, neighbour search, canonical unzip map, LTS schedule and
            the speedup model (Sec. 3.2, 3.2.5, 3.3, 3.6.3, 3.7; eqs. w_nuts, w_uts, invS).
  fd        finite-difference stencils and the degree-4 Lagrange interpolant.
  solver    unzip / rhs / zip / RK update and the LTS (Alg. 2) and GTS (Alg. 1)
            drivers.
  analytic  closed-form solutions (Gaussian pulse, plane wave, 1D form of
            eq. lsm, Maxwell) and discrete norms.

Every function names the passage of the paper it follows.  Where the paper is
silent or garbled the reading taken is stated at the function.

Parity status: the adaptive-mesh LTS values (ghost ownership on shared
faces, c->f interpolation order, what a ghost holds between time levels) are
"parity unpinned" beyond the pins in tests/test_oracle_*.py: the paper prints
no adaptive solution values, so for them only this oracle defines the result.
"""
