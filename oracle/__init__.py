"""Plain FP64 CPU oracle for the 2-D volume potential over triangle meshes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code, tables or constants with the
HIP library; both sides build their own quadrature rules, bases and geometry
from the definitions in the paper (Shen & Serkh, "Accelerating potential
evaluation over unstructured meshes in two dimensions").

Modules
-------
rules      reference-simplex quadrature and interpolation data (Sec. 2.1, 2.2,
           3.2, 3.4), built with SciPy / mpmath primitives.
potential  the evaluator itself, step by step in the paper's order: far sum
           over all quadrature nodes (Sec. 3.6), near/self classification
           (Def. of far/near field, Sec. 4.1), near corrections by adaptive
           subdivision (Sec. 3.3 with the Sec. 4.1 stopping rule), self
           corrections in radius-arc-length coordinates (Sec. 3.4), and the
           subtract-and-add coupling (Sec. 3.6).

Every function is pinned by a ``-m "not gpu"`` test against closed forms,
exactness identities, invariances or brute-force quadrature; see
``tests/test_oracle_*.py``.
"""

from . import rules, potential  # noqa: F401
