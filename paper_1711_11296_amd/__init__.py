"""Clenshaw-Curtis spherical-harmonic transforms on AMD Instinct MI355X.

The transform pair (analysis, synthesis) and both adjoints run in the HIP
library libsht.so; see include/sht.h for the C ABI.
"""

from .plan import Plan, host_tables  # noqa: F401
from ._lib import SHTError  # noqa: F401
from .autograd import SHTForward, SHTInverse, sht_forward, sht_inverse  # noqa: F401
from .transfer import (spec_retruncate, grid_inject, grid_product, spec_laplacian,  # noqa: F401
                       grid_residual)
