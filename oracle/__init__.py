"""FP64 CPU oracle for the even-parity RTE discretisation and its preconditioned
Richardson iteration (Doelz, Palii, Schlottbom, arXiv:2102.09038).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or run
anything here: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It is deliberately plain and slow: every operator is the
paper's definition written out with NumPy/SciPy primitives (dense matmul, sparse
matrices, Cholesky, sparse LU, symmetric eigensolver), with no blocking or fusion.

Modules
-------
quadrature   composite degree-5 rule on geodesic sphere triangles (a reading: the paper
             only says "higher-order integration rules", Sec. 6)
discretize   angular matrices (S+-, M_S+-, A_n, T_k, omega_k) and spatial P1/P0 matrices
             (Sec. 4)
operators    K+-, M+-, A, A^T, R, E, E_0, E_c, P_1^l, P_2 P_1 (Secs. 4-5)
solver       the outer Richardson iteration (Sec. 5, Alg. 3)
mixed        direct sparse LU of the full mixed system of Sec. 4 for tiny meshes
mg           geometric multigrid V-cycle for the E_0 blocks on lattice meshes and CG
             preconditioned by it (a reading of the multigrid remark of Sec. 5.5)

Pins: every function is checked in ``tests/test_oracle_*.py`` against closed forms,
invariants and special cases the paper or the mathematics fix (see each test's
docstring).  No function here is "parity unpinned".
"""
from .discretize import Discretization, discretize  # noqa: F401
from .operators import Operators  # noqa: F401
from .solver import richardson  # noqa: F401
