"""Residual and restriction steps of the two-grid cycle of App. C.

The elliptic problem (I - alpha L) X = F (eq. elliptic, alpha = dt/2) is
taken with a variable-coefficient Laplacian L X = kappa * lap(X), the
Laplacian evaluated pseudo-spectrally on the plan's grid.  Every step runs in
libsht.so on the current stream; the relaxation and the coarse solve are the
model's and are not part of this package.
"""

from .transfer import grid_inject, grid_residual, spec_laplacian


def helmholtz_residual(plan, x, kappa, f, alpha, scale=1.0):
    """R = x - alpha * kappa * lap(x) - f on a single-level plan's grid.

    x, f: grids [F, J, I] in the plan's dtype; kappa: [J, I]; scale: 1 /
    radius^2.  Analysis, spectral Laplacian, synthesis, fused update."""
    if len(plan.levels) != 1:
        raise ValueError("helmholtz_residual needs a single-level plan")
    N = plan.levels[0][0]
    lap = plan.inverse(spec_laplacian(plan.forward(x), N, scale))
    return grid_residual(x, kappa, lap, f, alpha)


def restrict_to_coarse_spectra(r_fine, coarse_plan, kind):
    """Restriction of a fine-grid field to the coarse level's spectral space
    (Sec. 3.2, App. C step 2): inject the coarse grid's nodes, then analyse
    on the coarse grid."""
    if len(coarse_plan.levels) != 1:
        raise ValueError("restrict_to_coarse_spectra needs a single-level coarse plan")
    _, Jc, Ic, _ = coarse_plan.levels[0]
    return coarse_plan.forward(grid_inject(r_fine, Jc, Ic, kind))
