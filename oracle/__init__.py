"""CPU oracle of the chemical-potential multiphase LBM (arXiv:1906.09530).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference the GPU
library is checked against.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it; the GPU library never does, and
the two share no code.

Two parts:

* ``cplbm_oracle.c`` -- the lattice Boltzmann scheme itself (naive loops,
  cyclic Thomas solves), built with ``gcc -O2 -ffp-contract=off`` into
  ``liboracle.so`` and reached here through ctypes;
* ``analytic.py`` -- thermodynamics in arbitrary precision (mpmath): critical
  points, the Maxwell construction, the planar-interface profile and surface
  tension;
* ``mlp.py`` -- the learned warm start in FP64 (numpy): the network, its
  backpropagated gradient, Adam, bfloat16 inference and the warm-start
  density field.
"""
from .lib import (  # noqa: F401
    EOS_CS, EOS_PR, EOS_RK, EOS_RKS, EOS_VDW, OracleParams, build, cfm_columns, cfm_columns_wall_value, cfm_line, collide_node,
    collide_node_mrt, feq, init, load, moments, mrt_inverse, mrt_matrix, mu0, mu0_capped, p0,
    alpha_T, run, run_until_converged, sc_psi, step, stream, threads,
)
