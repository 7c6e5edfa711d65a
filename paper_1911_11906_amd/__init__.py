"""fraclap: MI355X-native spectral fractional Poisson solver.

The discretised Laplace pencil K phi = theta M phi is solved for all
eigenpairs on the GPU (Cholesky, standard form, two-stage tridiagonalisation,
divide and conquer, back-transforms) and v = sum theta^(-alpha/2) <f,phi> phi
is applied to many forcings and fractional orders at once.

``inputs`` (seeded meshes/forcings) is importable without torch; the GPU API
(``Context``, ``Operator``, ``FracApply``) loads the HIP library on first use.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "Context", "Operator", "FracApply", "colmajor", "empty_colmajor"]


def __getattr__(name):
    if name in ("Context", "Operator", "FracApply", "colmajor", "empty_colmajor"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
