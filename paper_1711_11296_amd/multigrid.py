"""Residual and restriction steps of the two-grid cycle of App. C.

The elliptic problem (I - alpha L) X = F (eq. elliptic, alpha = dt/2) is
taken with a variable-coefficient Laplacian L X = kappa * lap(X), the
Laplacian evaluated pseudo-spectrally on the plan's grid.  Every step runs in
libsht.so on the current stream; the relaxation and the coarse solve are the
model's and are not part of this package.

Both helpers take single-level plans and multi-level plans (the levels of a
hierarchy batched in one plan, Sec. 3.2): with several levels, the grids
and spectra are the plan's concatenated buffers (level k at
plan.grid_offsets[k] / plan.spec_offsets[k]) and the transforms run once
for all levels.
"""

from .transfer import grid_inject, grid_residual, spec_laplacian


def _per_level(v, n, name):
    if isinstance(v, (list, tuple)):
        if len(v) != n:
            raise ValueError("%s: one entry per level (%d)" % (name, n))
        return list(v)
    return [v] * n


def helmholtz_residual(plan, x, kappa, f, alpha, scale=1.0):
    """R = x - alpha * kappa * lap(x) - f on the plan's grid: analysis,
    spectral Laplacian, synthesis, fused update.

    Single-level plan: x, f grids [F, J, I] in the plan's dtype, kappa
    [J, I].  Multi-level plan: x, f the concatenated grids of all levels
    (plan.grid_elems values, any shape), kappa one [J_k, I_k] grid per level,
    scale a number or one per level (1 / radius^2); the result has x's
    shape."""
    levels = plan.levels
    if len(levels) == 1:
        N = levels[0][0]
        lap = plan.inverse(spec_laplacian(plan.forward(x), N, scale))
        return grid_residual(x, kappa, lap, f, alpha)
    import torch
    if not isinstance(kappa, (list, tuple)) or len(kappa) != len(levels):
        raise ValueError("kappa: one [J, I] grid per level (%d)" % len(levels))
    scales = _per_level(scale, len(levels), "scale")
    for k, (N, J, I, F) in enumerate(levels):
        if tuple(kappa[k].shape) != (J, I):
            raise ValueError("kappa[%d] must be [%d, %d]" % (k, J, I))
    xf, ff = x.contiguous().reshape(-1), f.contiguous().reshape(-1)
    if xf.numel() != plan.grid_elems or ff.numel() != plan.grid_elems:
        raise ValueError("x and f must hold the plan's %d grid values" % plan.grid_elems)
    s = plan.forward(xf)
    for k, (N, J, I, F) in enumerate(levels):
        o, n = plan.spec_offsets[k], F * (N + 1) * (N + 2)
        sk = s[o:o + n].view(F, (N + 1) * (N + 2) // 2, 2)
        spec_laplacian(sk, N, scales[k], out=sk)
    y = plan.inverse(s)
    r = torch.empty_like(xf)
    for k, (N, J, I, F) in enumerate(levels):
        o, n = plan.grid_offsets[k], F * J * I
        grid_residual(xf[o:o + n].view(F, J, I), kappa[k], y[o:o + n].view(F, J, I), ff[o:o + n].view(F, J, I),
                      alpha, out=r[o:o + n].view(F, J, I))
    return r.view(x.shape)


def restrict_to_coarse_spectra(r_fine, coarse_plan, kind):
    """Restriction of fine-grid fields to the coarse plan's spectral space
    (Sec. 3.2, App. C step 2): inject the coarse grid's nodes, then analyse
    on the coarse grid.

    Single-level coarse plan: r_fine [F, J_fine, I_fine].  Multi-level
    coarse plan: r_fine one fine grid [F_k, J_fine_k, I_fine_k] per coarse
    level (each nesting that level's grid); all levels are injected into one
    concatenated grid and analysed together (concatenated spectra)."""
    levels = coarse_plan.levels
    if len(levels) == 1:
        _, Jc, Ic, _ = levels[0]
        return coarse_plan.forward(grid_inject(r_fine, Jc, Ic, kind))
    import torch
    if not isinstance(r_fine, (list, tuple)) or len(r_fine) != len(levels):
        raise ValueError("r_fine: one fine grid per coarse level (%d)" % len(levels))
    for k, (N, J, I, F) in enumerate(levels):
        if r_fine[k].dim() != 3 or r_fine[k].shape[0] != F:
            raise ValueError("r_fine[%d] must be [%d, J_fine, I_fine]" % (k, F))
    g = torch.empty(coarse_plan.grid_elems, dtype=r_fine[0].dtype, device=r_fine[0].device)
    for k, (N, J, I, F) in enumerate(levels):
        o = coarse_plan.grid_offsets[k]
        grid_inject(r_fine[k], J, I, kind, out=g[o:o + F * J * I].view(F, J, I))
    return coarse_plan.forward(g)
