"""FP64 CPU oracle for the low-rank NUFFT of Ruiz-Antolin & Townsend (arXiv:1701.04492).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import anything from here.  The product
library never imports, links or calls this package, and this package imports
nothing from the product: the two share no code.

* ``oracle.nudft``   -- the definitions (direct O(N*M) sums in C, compensated,
  with exact phase reduction) and the nearest-grid assignment of Sec. 2.2.
* ``oracle.lowrank`` -- the paper's algorithm in plain numpy FP64: Bessel
  coefficients (Sec. 2.1.2), choice of K, factors u_r / v_r, the vectorized
  two-step form (Sec. 2.3), type I (Sec. 3.1), type III (Sec. 3.2) and the
  2-D transform (Sec. 4).
* ``oracle.inverse`` -- the inverse type-II transform of Sec. 3.3: conjugate
  gradients on the normal equations with the Toeplitz product through a 2N
  circulant embedding, and a dense least-squares reference for small sizes.
"""
