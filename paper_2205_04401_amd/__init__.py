"""MI355X (gfx950) 2-D volume-potential evaluator.

u(x) = (1/2pi) int_Omega log|x - y| f(y) dA_y over an unstructured triangle
mesh, following Shen & Serkh, "Accelerating potential evaluation over
unstructured meshes in two dimensions": a direct-sum far field over every
triangle's quadrature nodes, near-field lists from the Bernstein-ellipse
characterisation of each triangle's near region, and near/self corrections
applied as precomputed weights on per-triangle Koornwinder coefficients.

The compute path is the C-ABI library ``libvp.so`` (HIP kernels, see
``include/vp.h``); ``vp`` is its thin ctypes binding and ``workloads`` the
seeded synthetic input generators.  Importing the package loads nothing;
``vp.load()`` loads the library and fails loudly if it is missing.
"""

__all__ = ["vp", "workloads"]
