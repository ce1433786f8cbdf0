"""CPU oracle for the two-phase spectral-element LBM time step.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It wraps the plain-C FP64
implementation in ``semlbm_oracle.c`` (built by :mod:`oracle.build`) and adds a
numpy contact-angle measurement.  It shares no code with the GPU library.
"""
from .api import Oracle, load, set_threads  # noqa: F401
from .contact import contact_angle, interface_points, fit_circle  # noqa: F401
