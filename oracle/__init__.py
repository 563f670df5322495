"""Plain FP64 CPU oracle of the unfitted BAE / lattice Green's function method (arXiv 2502.05507).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this
package; only the tests, the graft smoke check and the benchmark's ``cpu_baseline`` leg
use it.  It shares no code with the HIP library: every function here is written from
the paper, in plain NumPy/SciPy, slowly and in the paper's order, so that a reader can
check it against the text by eye.

Modules
  lgf        lattice Green's function of the 7-point (modified) Laplacian (Sec. 2.2)
  geometry   point sets M+, M-, gamma+-, N+, D_n, E and the Dirichlet closure (Sec. 2.1, 3.2)
  operators  single/double layer potentials, the BAE operator, volume potential (Sec. 3.2-3.4)
  gmres      unrestarted GMRES with modified Gram-Schmidt and Givens rotations (Sec. 4)
  sparse     the plain sparse discrete Dirichlet problem the method is equivalent to (Sec. 2.2)
  box        the particular solution on the finite grid, G_h[chi_{M+} f] (Algorithm 1)
  bae        Algorithm 1 end to end

Every function is pinned by tests under tests/ (test_oracle_*.py) to values the paper
prints, closed forms, identities the paper proves, or library routines.
"""
