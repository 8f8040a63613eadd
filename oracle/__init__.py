"""FP64 CPU oracle for the Clenshaw-Curtis spherical-harmonic transform pair.

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may use it; the product path never does.
"""
from .sht_oracle import *  # noqa: F401,F403
from .sht_oracle import (GRID_KINDS, ncoef, spec_index, nodes, weights, alf_m,
                         zonal_analysis, zonal_synthesis, forward, inverse,
                         forward_adjoint, inverse_adjoint, forward_sample,
                         inverse_sample_row, orthonormality_errors, retruncate, inject,
                         laplacian, helmholtz_residual)
