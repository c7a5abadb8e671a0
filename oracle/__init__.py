"""CPU oracle for modular polynomial multiplication (L. Meng, "Automatic Library
Generation for Modular Polynomial Multiplication").

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never calls it and
shares no code with it: not a kernel, a header, a helper or a constant table.

What it computes, each from its plain definition:
  poly.poly_mul          c_k = sum_{i+j=k} a_i b_j mod p         (Def. 2, eq. 2; Def. 3, eq. 3)
  poly.cyclic_conv       circular convolution mod p              (Def. 4, eq. 5)
  poly.dft_direct / ntt  evaluation at w^0..w^{N-1}              (section 3, Theorem 1, eq. 8-10)
  poly.tft               first n values in bit-reversed order    (section 3, TFT product, eq. 14)
  poly.crt3 / int_mul    three-primes integer product            (section 1)
  mlp.*                  float64 cost-model network (forward, backward, Adam)
Readings of the paper where it is silent are listed with each function.
"""

from . import poly, mlp  # noqa: F401
from ._clib import build  # noqa: F401
