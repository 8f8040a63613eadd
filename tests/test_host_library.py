"""CPU checks of libsht.so: it loads, exports every entry point declared in
include/sht.h, validates arguments, and its host planner (nodes, weights,
table of P~_n^m) agrees with the oracle and with mpmath."""

import ctypes
import os
import re

import mpmath
import numpy as np
import pytest

import oracle as O
from paper_1711_11296_amd import _lib, host_tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sht.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sht_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load(require_torch=False)
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_invalid_arguments_are_rejected_without_a_gpu():
    lib = _lib.load(require_torch=False)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.sht_host_tables(-1, 5, 0, None, None, None) == _lib.SHT_EINVAL
    assert lib.sht_host_tables(3, 1, 0, None, None, None) == _lib.SHT_EINVAL   # cc_poles needs J >= 2
    assert lib.sht_host_tables(3, 0, 1, None, None, None) == _lib.SHT_EINVAL
    assert lib.sht_host_tables(3, 5, 7, None, None, None) == _lib.SHT_EINVAL
    assert "grid" in _lib.last_error() or "J" in _lib.last_error()
    # a handle that was never created is not a live plan
    bogus = ctypes.c_void_p(0x1000)
    buf = (ctypes.c_double * 4)()
    assert lib.sht_forward(None, buf, buf, None) == _lib.SHT_EINVAL
    assert lib.sht_forward(bogus, buf, buf, None) == _lib.SHT_ESTATE
    assert lib.sht_forward_noalloc(None, buf, buf, None) == _lib.SHT_EINVAL
    assert lib.sht_forward_noalloc(bogus, buf, buf, None) == _lib.SHT_ESTATE
    assert lib.sht_device_bytes(None) == _lib.SHT_EINVAL
    assert _lib.device_bytes() == 0      # no plan is live in this process
    assert lib.sht_plan_destroy(bogus) == _lib.SHT_ESTATE
    assert lib.sht_plan_query(bogus, 0, buf) == _lib.SHT_ESTATE
    opts = _lib.Options(0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert lib.sht_plan_ex(4, 9, 8, 1, ctypes.byref(opts), ctypes.byref(h)) == _lib.SHT_EINVAL  # I < 2N+1
    assert lib.sht_plan_ex(4, 9, 14, 1, ctypes.byref(opts), ctypes.byref(h)) == _lib.SHT_EINVAL  # 7 | I
    assert lib.sht_plan_ex(4, 9, 9, 0, ctypes.byref(opts), ctypes.byref(h)) == _lib.SHT_EINVAL  # F < 1
    assert lib.sht_plan_ex(4, 9, 9, 1, ctypes.byref(opts), None) == _lib.SHT_EINVAL
    n9 = (ctypes.c_int * 9)(*([8] * 9))
    i9 = (ctypes.c_int * 9)(*([32] * 9))
    j9 = (ctypes.c_int * 9)(*([17] * 9))
    f9 = (ctypes.c_int * 9)(*([1] * 9))
    assert lib.sht_plan_multi(9, n9, j9, i9, f9, ctypes.byref(opts), ctypes.byref(h)) == _lib.SHT_EINVAL
    assert "nlevels" in _lib.last_error()                                                  # at most 8 levels
    assert lib.sht_plan_ex(4, 9, 4800, 1, ctypes.byref(opts), ctypes.byref(h)) == _lib.SHT_EINVAL  # I > 4096
    bad = _lib.Options(0, 0, 0, 0, 0, 0, 3)     # no such zonal launch mode
    assert lib.sht_plan_ex(4, 9, 9, 1, ctypes.byref(bad), ctypes.byref(h)) == _lib.SHT_EINVAL
    assert "zonal" in _lib.last_error()
    assert not h.value
    del dp


@pytest.mark.parametrize("kind", O.GRID_KINDS)
@pytest.mark.parametrize("N,J", [(0, 3), (5, 11), (21, 43), (21, 42), (50, 101), (8, 16)])
def test_host_tables_match_oracle(kind, N, J):
    mu, w, alf = host_tables(N, J, kind)
    _, mo, so = O.nodes(J, kind)
    wo = O.weights(J, kind)
    Jh = (J + 1) // 2
    assert np.array_equal(mu, mo)
    assert np.allclose(w, wo, rtol=1e-13, atol=0)
    assert abs(w.sum() - 2.0) < 1e-14
    ref = np.concatenate([O.alf_m(N, m, mo[:Jh], so[:Jh]) for m in range(N + 1)])
    assert np.abs(alf - ref).max() < 1e-12


def test_host_table_high_degree_against_oracle_and_mpmath():
    N, J, kind = 479, 959, "fejer2"
    mu, w, alf = host_tables(N, J, kind)
    _, mo, so = O.nodes(J, kind)
    Jh = (J + 1) // 2
    for m in (0, 1, 100, 300, 479):
        ref = O.alf_m(N, m, mo[:Jh], so[:Jh])
        k0 = O.spec_index(N, m, m)
        assert np.abs(alf[k0:k0 + N - m + 1] - ref).max() < 1e-9
    # interior rows: mpmath's Legendre function at the stored mu
    mpmath.mp.dps = 40
    for (m, n, j) in [(0, 479, 200), (3, 400, 150), (200, 479, 300), (479, 479, 479), (10, 255, 330)]:
        x = mpmath.mpf(mu[j])
        ref = mpmath.legenp(n, m, x) * (-1) ** m * mpmath.sqrt(
            (2 * n + 1) / mpmath.mpf(2) * mpmath.factorial(n - m) / mpmath.factorial(n + m))
        v = alf[O.spec_index(N, m, n), j]
        assert abs(v - float(ref)) <= 1e-13 * max(1.0, abs(float(ref))), (m, n, j, v, float(ref))
    # next to the pole sqrt(1 - mu^2) of the rounded mu is not the rounded
    # sin(theta) the table uses (relative gap ~1e-13), so compare with the same
    # recurrence run in 40 digits from the same (mu, sin theta)
    _, _, so = O.nodes(J, kind)
    for (m, n, j) in [(0, 479, 0), (3, 400, 5), (100, 479, 2)]:
        x, sn = mpmath.mpf(mu[j]), mpmath.mpf(so[j])
        p = 1 / mpmath.sqrt(2)
        for k in range(1, m + 1):
            p *= mpmath.sqrt(mpmath.mpf(2 * k + 1) / (2 * k)) * sn
        p0, p1 = p, mpmath.sqrt(2 * m + 3) * x * p

        def a(k):
            return mpmath.sqrt((4 * mpmath.mpf(k) ** 2 - 1) / (mpmath.mpf(k) ** 2 - m * m))
        for k in range(m + 2, n + 1):
            p0, p1 = p1, a(k) * (x * p1 - p0 / a(k - 1))
        v = alf[O.spec_index(N, m, n), j]
        assert abs(v - float(p1)) <= 1e-14 * max(1.0, abs(float(p1))), (m, n, j, v, float(p1))


def test_host_table_no_underflow_at_high_order():
    """The sectoral start at m = N near the pole is far below the double
    range; the value stored is 0 there, but entries that return to the
    double range later in n are still right (carried exponent)."""
    N, J = 300, 601
    mu, _, alf = host_tables(N, J, "cc_poles")
    m = 300
    # row 1 (next to the pole): P~_300^300 ~ (sin theta_1)^300, below 1e-308
    assert alf[O.spec_index(N, m, m), 1] == 0.0
    mpmath.mp.dps = 60
    x = mpmath.mpf(mu[1])
    sn = mpmath.sqrt(1 - x * x)
    ref = mpmath.sqrt(mpmath.fprod(mpmath.mpf(2 * k + 1) / (2 * k) for k in range(1, m + 1)) / 2) * sn ** m
    assert abs(ref) < 1e-308
    # equator row: everything regular
    j = (J - 1) // 2
    assert mu[j] == 0.0
    assert np.all(alf[O.spec_index(N, m, m):O.spec_index(N, m, N) + 1, j][1::2] == 0.0)


def test_transfer_arguments_are_rejected_without_a_gpu():
    """Re-truncation, injection, the spectral Laplacian and the residual
    update check their arguments before any GPU call: bad sizes, grids that
    do not nest, non-finite scalars, NULL or misaligned pointers.
    (Every call here must fail validation: none may reach a launch, since
    the buffers are host memory.)"""
    lib = _lib.load(require_torch=False)
    buf = ctypes.create_string_buffer(4096 + 16)
    p = ctypes.c_void_p((ctypes.addressof(buf) + 15) // 16 * 16)
    q = ctypes.c_void_p(p.value + 2048)
    E = _lib.SHT_EINVAL
    assert lib.sht_spec_retruncate(-1, 3, 1, 0, p, q, None) == E
    assert lib.sht_spec_retruncate(3, 3, 0, 0, p, q, None) == E
    assert lib.sht_spec_retruncate(3, 3, 1, 0, None, q, None) == E
    assert lib.sht_spec_retruncate(3, 3, 1, 0, ctypes.c_void_p(p.value + 4), q, None) == E
    assert lib.sht_spec_retruncate(3, 3, 1, 0, p, p, None) == E
    assert lib.sht_grid_inject(33, 48, 16, 24, 1, 0, 0, p, q, None) == E    # 32 % 15
    assert lib.sht_grid_inject(34, 48, 17, 24, 1, 1, 0, p, q, None) == E    # 35 % 18
    assert lib.sht_grid_inject(33, 48, 17, 25, 1, 0, 0, p, q, None) == E    # 48 % 25
    assert lib.sht_grid_inject(33, 48, 17, 24, 1, 2, 0, p, q, None) == E    # shifted grid
    assert lib.sht_grid_inject(33, 48, 17, 24, 0, 0, 0, p, q, None) == E    # no fields
    assert lib.sht_grid_inject(33, 48, 17, 24, 1, 0, 0, None, q, None) == E
    # spectral Laplacian and residual update of the App. C residual
    assert lib.sht_spec_laplacian(-1, 1, 0, 1.0, p, q, None) == E
    assert lib.sht_spec_laplacian(3, 0, 0, 1.0, p, q, None) == E
    assert lib.sht_spec_laplacian(3, 1, 0, float("nan"), p, q, None) == E
    assert lib.sht_spec_laplacian(3, 1, 0, float("inf"), p, q, None) == E
    assert lib.sht_spec_laplacian(3, 1, 0, 1.0, None, q, None) == E
    assert lib.sht_spec_laplacian(3, 1, 1, 1.0, p, ctypes.c_void_p(q.value + 8), None) == E
    assert lib.sht_grid_residual(0, 1, 0, 1.0, p, p, q, q, q, None) == E
    assert lib.sht_grid_residual(10, 3, 0, 1.0, p, p, q, q, q, None) == E      # 10 % 3
    assert lib.sht_grid_residual(12, 0, 0, 1.0, p, p, q, q, q, None) == E
    assert lib.sht_grid_residual(12, 3, 0, float("nan"), p, p, q, q, q, None) == E
    assert lib.sht_grid_residual(12, 3, 0, 1.0, p, None, q, q, q, None) == E
    assert lib.sht_grid_residual(12, 3, 0, 1.0, p, p, q, q, None, None) == E

