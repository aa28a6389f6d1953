"""CPU reference ("oracle") for the fast QMC matrix product -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything from this package.  The product path (the HIP
library and its Python binding) never imports, calls or links it, and this
package imports nothing from the product.

What it computes (Dick, Kuo, Le Gia, Schwab, "Fast QMC matrix-vector
multiplication"):

* ``points``  -- the point set in conventional order, written out from its
  definition: rank-1 lattice points {n g_j / N} (Section 2.1), optionally with
  an equal shift Delta in every coordinate (Remark 2), polynomial lattice
  points over GF(2) (Remark 1, Niederreiter's construction) and the union of
  all Korobov lattice point sets {n b^j / K} (Section 2.2), each mapped by
  one univariate phi (Section 2.1: identity, the tent map, the inverse normal
  CDF; x - 1/2 as in Experiment 2).
* ``dense``   -- X = Y A and dA = Y^T G by forming Y explicitly and multiplying
  in FP64 (the "standard approach" of the paper's experiments), plus row- and
  entry-sampled versions for sizes where Y does not fit, and the elementwise
  epilogue of the PDE applications (Sections 3.2, 3.3).
* ``literal`` -- a second, independent route used only as a checker: the
  paper's own construction (primitive root beta, exponents c_j, the circulant
  Z and selection matrix P of eq. (ZPa), worked Example 1), evaluated as a
  plain O(N^2) product Z (P a) with the paper's row order mapped back.
* ``exact``   -- brute force over exact rationals for tiny N.
* ``composite`` -- a checker for lattice rules with a non-prime N: the
  product through the orbits d U(N/d) of the rows and the multilevel
  circulant over each unit group, with brute-force group structure.

The fast method reaches the plain product exactly in exact arithmetic
(eq. (ZPa) is an identity and the ordering does not change the quadrature sum,
Section 2.1), so the oracle is that plain product.  The inverse normal CDF is
the one library routine used (``scipy.special.ndtri``); it is pinned in the
tests against the standard library's ``statistics.NormalDist.inv_cdf`` and by
the round trip through ``math.erfc``.
"""

from .points import (PHI_IDENTITY, PHI_CENTERED, PHI_INVNORM, PHI_TENT,
                     RULE_LATTICE, RULE_POLY_GF2, RULE_KOROBOV_UNION, phi_apply, lattice_coords,
                     gf2_coords, gf2_digits_coords, coords, coords_rational, explicit_Y,
                     phi_residue_values, phi_rational)
from .dense import (matmul, adjoint, matmul_rows, adjoint_entries, Y_rows, epilogue, EPI_NONE,
                    EPI_AFFINE, EPI_EXP)
from . import literal, exact, composite

__all__ = [
    "PHI_IDENTITY", "PHI_CENTERED", "PHI_INVNORM", "PHI_TENT",
    "RULE_LATTICE", "RULE_POLY_GF2", "RULE_KOROBOV_UNION", "phi_apply", "lattice_coords", "gf2_coords",
    "gf2_digits_coords", "coords", "coords_rational", "explicit_Y",
    "phi_residue_values", "phi_rational",
    "matmul", "adjoint", "matmul_rows", "adjoint_entries", "Y_rows", "epilogue", "EPI_NONE",
    "EPI_AFFINE", "EPI_EXP",
    "literal", "exact", "composite",
]
