"""sht_forward_noalloc, the analysis for callers that cannot allocate: the
same kernels as sht_forward with the workspace in the library's static
device array.  Called through the C ABI and compared with sht_forward of the
same plan (bitwise: same kernels, same order) and with the FP64 oracle, on
calls in a row whose second input is smaller, including a first call that
leaves NaN everywhere it wrote in the shared array."""

import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1711_11296_amd import _lib, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x6": 1e-6}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _noalloc(p, g, s):
    """sht_forward_noalloc(plan, grid, spec, stream) through ctypes."""
    stream = torch.cuda.current_stream(_dev()).cuda_stream
    return p._lib.sht_forward_noalloc(p._h, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(s.data_ptr()),
                                      ctypes.c_void_p(stream))


def _host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def _check_case(N, J, I, F, kind, form, seed, use_graph=False):
    from paper_1711_11296_amd import Plan
    p = Plan(N, J, I, F, grid=kind, form=form, use_graph=use_graph)
    dt = p.dtype
    g = torch.from_numpy(inputs.random_grid(F, J, I, seed=seed)).to(_dev(), dt)
    ref = p.forward(g)
    out = torch.full(p.spec_shape, float("nan"), device=_dev(), dtype=dt)
    assert _noalloc(p, g, out) == _lib.SHT_OK, _lib.last_error()
    torch.cuda.synchronize()
    assert torch.equal(out, ref), "noalloc differs from sht_forward (%s %s)" % (form, (N, J, I, F))
    e = np.linalg.norm(_host(out) - O.forward(_host(g), N, kind)) / np.linalg.norm(O.forward(_host(g), N, kind))
    assert e < TOL[form], e
    p.close()


@pytest.mark.parametrize("form", ["fp32", "fp64", "bf16x6"])
def test_noalloc_two_calls_second_smaller(form):
    # larger plan first, then a smaller one with another layout (even J: no
    # equator row, 15 padding rows per workspace plane)
    _check_case(100, 201, 216, 9, "cc_poles", form, seed=1)
    _check_case(40, 34, 96, 3, "fejer2", form, seed=2)


@pytest.mark.parametrize("form", ["fp32", "fp64"])
def test_noalloc_after_nan_call(form):
    """The first call analyses an all-NaN grid, so every workspace entry it
    wrote in the shared array is NaN; the next call, of a smaller plan whose
    padding rows fall inside that region, must still equal sht_forward."""
    from paper_1711_11296_amd import Plan
    pa = Plan(100, 201, 216, 64, grid="cc_poles", form=form)
    g = torch.full(pa.grid_shape, float("nan"), device=_dev(), dtype=pa.dtype)
    s = torch.empty(pa.spec_shape, device=_dev(), dtype=pa.dtype)
    assert _noalloc(pa, g, s) == _lib.SHT_OK, _lib.last_error()
    sh = _host(s)
    m0 = inputs.orders(100) == 0
    assert np.isnan(sh[:, :, 0]).all() and np.isnan(sh[:, ~m0, 1]).all()   # Im of m = 0 is written as 0
    pa.close()
    _check_case(40, 34, 96, 3, "fejer2", form, seed=3)
    _check_case(21, 43, 64, 2, "cc_poles", form, seed=4)


def test_noalloc_graph_plan_runs_eagerly():
    _check_case(30, 61, 64, 5, "fejer1", "fp32", seed=5, use_graph=True)


def test_noalloc_rejects_a_workspace_above_the_limit():
    from paper_1711_11296_amd import Plan
    p = Plan(300, 601, 640, 64, grid="cc_poles", form="fp32")
    assert p.workspace_bytes > (64 << 20)
    g = torch.zeros(p.grid_shape, device=_dev(), dtype=p.dtype)
    s = torch.zeros(p.spec_shape, device=_dev(), dtype=p.dtype)
    assert _noalloc(p, g, s) == _lib.SHT_EINVAL
    assert "static workspace" in _lib.last_error()
    torch.cuda.synchronize()
    assert torch.count_nonzero(s).item() == 0   # nothing was enqueued
    p.close()
