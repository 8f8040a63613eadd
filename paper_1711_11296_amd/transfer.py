"""Transfers between truncations and nested grids for multigrid cycles
(App. C): spectral re-truncation and grid injection; and the pointwise
product of grids (the nonlinear terms of Sec. 4.2).  Run by libsht.so on the
tensors' device and current stream."""

import ctypes

from . import _lib

_GRID = {"cc_poles": 0, "fejer2": 1, "fejer1": 2, "gauss": 3}


def _dbl(t):
    import torch
    if t.dtype == torch.float64:
        return 1
    if t.dtype == torch.float32:
        return 0
    raise TypeError("float32 or float64 tensors only")


def spec_retruncate(spec, N_in, N_out):
    """Spectra [F, (N_in+1)(N_in+2)/2, 2] -> [F, (N_out+1)(N_out+2)/2, 2]:
    coefficients with n <= min(N_in, N_out) copied, n > N_in set to zero
    (restriction when N_out < N_in, prolongation when N_out > N_in)."""
    import torch
    lib = _lib.load()
    spec = spec.contiguous()
    F = spec.shape[0]
    nc_in = (N_in + 1) * (N_in + 2) // 2
    if tuple(spec.shape) != (F, nc_in, 2):
        raise ValueError("spec must be [F, %d, 2]" % nc_in)
    out = torch.empty((F, (N_out + 1) * (N_out + 2) // 2, 2), dtype=spec.dtype, device=spec.device)
    stream = torch.cuda.current_stream(spec.device).cuda_stream
    _lib.check(lib.sht_spec_retruncate(N_in, N_out, F, _dbl(spec), ctypes.c_void_p(spec.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)))
    return out


def grid_inject(grid, J_coarse, I_coarse, kind="cc_poles"):
    """Grids [F, J_fine, I_fine] -> [F, J_coarse, I_coarse]: the nested rows
    and columns of the finer grid (see sht_grid_inject)."""
    import torch
    lib = _lib.load()
    grid = grid.contiguous()
    F, J, I = grid.shape
    out = torch.empty((F, J_coarse, I_coarse), dtype=grid.dtype, device=grid.device)
    stream = torch.cuda.current_stream(grid.device).cuda_stream
    _lib.check(lib.sht_grid_inject(J, I, J_coarse, I_coarse, F, _GRID[kind], _dbl(grid),
                                   ctypes.c_void_p(grid.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(stream)))
    return out


def grid_product(a, b):
    """Pointwise product a * b of two grids of the same shape and dtype."""
    import torch
    lib = _lib.load()
    if a.shape != b.shape or a.dtype != b.dtype or a.device != b.device:
        raise ValueError("a and b must match in shape, dtype and device")
    a = a.contiguous()
    b = b.contiguous()
    out = torch.empty_like(a)
    stream = torch.cuda.current_stream(a.device).cuda_stream
    _lib.check(lib.sht_grid_product(a.numel(), _dbl(a), ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)))
    return out

