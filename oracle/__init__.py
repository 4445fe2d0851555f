"""FP64 CPU oracle of the chemical-potential lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Wen, Zhou, He, Zhang, Fang, "Chemical-potential-based
lattice Boltzmann method for nonideal fluids" (arXiv:1611.00907).  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it.
It shares no code with the GPU library and never imports it.

Pieces:
  * ``cplbm_oracle.c``  -- the time step in plain C loops (Eqs 8, 12, 13, 14, 28).
  * ``thermo``          -- EOS of Sec. III in numpy, critical point, Maxwell
                           equal-area coexistence, surface tension.
  * ``contact``         -- contact angle from a density field (Sec. V formula).
  * ``lattice``         -- ctypes binding of the C step and a small driver class.
  * ``cplbm3d_oracle.c`` / ``lattice3d`` -- the same step on D3Q19, periodic box.

Each function is pinned by ``tests/test_oracle_*.py`` against closed forms,
invariants or brute force; anything not pinned says "parity unpinned".
"""
from .lattice import OracleParams, OracleLattice, load_library, build_library  # noqa: F401
from . import thermo, contact  # noqa: F401
