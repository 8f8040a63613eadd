"""Transfers between truncations and nested grids for multigrid cycles
(App. C): spectral re-truncation and grid injection; the pieces of the
residual of the App. C elliptic problem (spectral Laplacian, grid update);
and the pointwise product of grids (the nonlinear terms of Sec. 4.2).  Run by libsht.so on the
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


def _check_out(out, shape, like):
    if tuple(out.shape) != tuple(shape) or out.dtype != like.dtype or out.device != like.device:
        raise ValueError("out must be %s of %s on %s" % (tuple(shape), like.dtype, like.device))
    if not out.is_contiguous():
        raise ValueError("out must be contiguous")
    return out


def grid_inject(grid, J_coarse, I_coarse, kind="cc_poles", out=None):
    """Grids [F, J_fine, I_fine] -> [F, J_coarse, I_coarse]: the nested rows
    and columns of the finer grid (see sht_grid_inject); into `out` when
    given (contiguous, not overlapping grid)."""
    import torch
    lib = _lib.load()
    grid = grid.contiguous()
    F, J, I = grid.shape
    if out is None:
        out = torch.empty((F, J_coarse, I_coarse), dtype=grid.dtype, device=grid.device)
    else:
        _check_out(out, (F, J_coarse, I_coarse), grid)
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



def spec_laplacian(spec, N, scale=1.0, out=None):
    """Spectra [F, (N+1)(N+2)/2, 2] -> c_n * spec with c_n = -scale n (n+1):
    the Laplacian on a sphere of radius 1/sqrt(scale); into `out` when given
    (contiguous; may be spec)."""
    import torch
    lib = _lib.load()
    spec = spec.contiguous()
    F = spec.shape[0]
    if tuple(spec.shape) != (F, (N + 1) * (N + 2) // 2, 2):
        raise ValueError("spec must be [F, %d, 2]" % ((N + 1) * (N + 2) // 2))
    out = torch.empty_like(spec) if out is None else _check_out(out, spec.shape, spec)
    stream = torch.cuda.current_stream(spec.device).cuda_stream
    _lib.check(lib.sht_spec_laplacian(N, F, _dbl(spec), float(scale), ctypes.c_void_p(spec.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)))
    return out


def grid_residual(x, kappa, y, f, alpha, out=None):
    """r = x - alpha * kappa * y - f; x, y, f [F, J, I] (or any shape whose
    trailing elements form whole copies of kappa), kappa [J, I] shared by
    all fields; into `out` when given (contiguous; may be x, y or f)."""
    import torch
    lib = _lib.load()
    ts = [x.contiguous(), kappa.contiguous(), y.contiguous(), f.contiguous()]
    if not (ts[0].shape == ts[2].shape == ts[3].shape):
        raise ValueError("x, y and f must have the same shape")
    if any(t.dtype != ts[0].dtype or t.device != ts[0].device for t in ts):
        raise ValueError("all tensors must share dtype and device")
    n, n_per = ts[0].numel(), ts[1].numel()
    if n_per < 1 or n % n_per:
        raise ValueError("kappa must tile x")
    r = torch.empty_like(ts[0]) if out is None else _check_out(out, ts[0].shape, ts[0])
    stream = torch.cuda.current_stream(x.device).cuda_stream
    _lib.check(lib.sht_grid_residual(n, n_per, _dbl(ts[0]), float(alpha), *[ctypes.c_void_p(t.data_ptr()) for t in ts],
                                     ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(stream)))
    return r
