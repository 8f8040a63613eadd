"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Bounds: rel-L2 <= 1e-12 for the FP64 form, <= 1e-6 for
the FP32 and split-bfloat16 forms (the oracle receives the FP32 inputs
promoted to FP64)."""

import numpy as np
import pytest

import oracle as O
from paper_1711_11296_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x6": 1e-6}
FORMS = ["fp64", "fp32", "bf16x6"]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _plan(N, J, I, F, kind, form):
    from paper_1711_11296_amd import Plan
    return Plan(N, J, I, F, grid=kind, form=form)


def _to_dev(x, form):
    dt = torch.float64 if form == "fp64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=_dev(), dtype=dt)


def _host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def _roundtrip_case(N, J, I, F, kind, form, profile="inv1", seed=0):
    p = _plan(N, J, I, F, kind, form)
    a = inputs.random_spectra(N, F, seed=seed, profile=profile)
    a_d = _to_dev(a, form)
    a_in = _host(a_d)                         # what the GPU received
    g_d = p.inverse(a_d)
    g_ref = O.inverse(a_in, N, J, I, kind)
    assert rel(_host(g_d), g_ref) < TOL[form], "inverse"
    g_in = _host(g_d)
    s_d = p.forward(g_d)
    s_ref = O.forward(g_in, N, kind)
    assert rel(_host(s_d), s_ref) < TOL[form], "forward"
    if J >= 2 * N + 1:
        assert rel(_host(s_d), a_in) < 10 * TOL[form], "round trip"
    p.close()


@pytest.mark.parametrize("kind", O.GRID_KINDS)
def test_c1_fp64_round_trip(kind):
    """N=21, J=43, I=64, one field, spectra with std (n+1)^-1, seed 0."""
    _roundtrip_case(21, 43, 64, 1, kind, "fp64")


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("kind", O.GRID_KINDS)
@pytest.mark.parametrize("N", [0, 1, 2, 5, 8])
def test_tiny_sweep(form, kind, N):
    """Every J from 2N-3 to 2N+3 (odd and even, aliasing or exact)."""
    for J in range(max(2, 2 * N - 3), 2 * N + 4):
        I = max(2 * N + 1, 1)
        I = {1: 1, 3: 3, 5: 5, 11: 12, 17: 18}.get(I, I)
        _roundtrip_case(N, J, I, 3, kind, form, seed=N * 100 + J)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("kind,N,J,I,F", [
    ("cc_poles", 100, 203, 216, 5),     # several row and K tiles, ragged tails, 2^3 3^3
    ("fejer2", 130, 250, 300, 9),       # even J (no equator row), F not a multiple of 8
    ("cc_poles", 64, 129, 200, 17),     # 5^2 radix, three field blocks
    ("fejer2", 33, 80, 81, 2),          # J > 2N+1, pure radix 3
    ("fejer1", 90, 183, 192, 6),        # shifted grid (Sec. 3.3), odd J
    ("fejer1", 71, 144, 150, 3),        # shifted grid, even J (no equator row)
])
def test_multi_tile_parity(form, kind, N, J, I, F):
    _roundtrip_case(N, J, I, F, kind, form, profile="k3", seed=N)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("kind,N,J,I,F", [
    ("cc_poles", 200, 101, 480, 5),     # I = 16*6*5, one wavenumber per thread
    ("fejer2", 239, 478, 480, 11),      # N = (I-1)/2, even J, ragged field block
    ("fejer2", 700, 97, 1440, 9),       # I = 16*9*10, two wavenumbers per thread
    ("cc_poles", 30, 33, 2880, 2),      # I = 16*12*15, most bins zero
    ("cc_poles", 40, 33, 2880, 19),     # I = 2880, three field blocks (FP64: five), ragged last block
    ("cc_poles", 1040, 40, 2880, 3),    # N + 1 > 1024: three wavenumbers per thread
    ("cc_poles", 150, 101, 400, 5),     # I = 16*5*5
    ("fejer2", 200, 60, 800, 3),        # I = 16*5*10, one wavenumber per thread
    ("fejer2", 300, 97, 800, 9),        # two wavenumbers per thread
    ("cc_poles", 600, 81, 1600, 3),     # I = 16*10*10, two wavenumbers per thread
    ("fejer1", 300, 64, 1600, 10),      # one wavenumber per thread, ragged field block
    ("gauss", 479, 80, 960, 3),         # I = 16*6*10 (the Tl479 Gaussian grid's length)
    ("fejer2", 600, 71, 1920, 5),       # I = 16*12*10, two wavenumbers per thread
])
def test_fixed_length_plans(form, kind, N, J, I, F):
    """Lengths with a compile-time three-pass FFT plan, away from the
    benchmark truncations: every wavenumber count per thread, ragged field
    blocks, both grids, odd and even J."""
    _roundtrip_case(N, J, I, F, kind, form, profile="k3", seed=N + J)
    p = _plan(N, J, I, F, kind, form)
    sb = _to_dev(inputs.random_spectra(N, F, seed=6, profile="inv1"), form)
    gb = _to_dev(inputs.random_grid(F, J, I, seed=7), form)
    x = p.forward_adjoint(sb)
    assert rel(_host(x), O.forward_adjoint(_host(sb), N, J, I, kind)) < TOL[form]
    y = p.inverse_adjoint(gb)
    assert rel(_host(y), O.inverse_adjoint(_host(gb), N, kind)) < TOL[form]
    p.close()


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("kind", O.GRID_KINDS)
def test_random_grid_forward(form, kind):
    """Analysis of a grid that is not band-limited is still the oracle's map."""
    N, J, I, F = 40, 81, 96, 4
    p = _plan(N, J, I, F, kind, form)
    g = _to_dev(inputs.random_grid(F, J, I, seed=3), form)
    s = p.forward(g)
    assert rel(_host(s), O.forward(_host(g), N, kind)) < TOL[form]
    p.close()


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("kind", O.GRID_KINDS)
def test_adjoints_against_oracle(form, kind):
    N, J, I, F = 30, 61, 64, 3
    p = _plan(N, J, I, F, kind, form)
    sb = _to_dev(inputs.random_spectra(N, F, seed=4, profile="inv1"), form)
    gb = _to_dev(inputs.random_grid(F, J, I, seed=5), form)
    x = p.forward_adjoint(sb)
    assert rel(_host(x), O.forward_adjoint(_host(sb), N, J, I, kind)) < TOL[form]
    y = p.inverse_adjoint(gb)
    assert rel(_host(y), O.inverse_adjoint(_host(gb), N, kind)) < TOL[form]
    p.close()


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_c2_full_batch(form):
    """N=159, J=319, I=480, 64 fields (16 levels x 4 variables), k^-3 spectra."""
    N, J, I, F = 159, 319, 480, 64
    for kind in O.GRID_KINDS:
        p = _plan(N, J, I, F, kind, form)
        a = inputs.random_spectra(N, F, seed=0, profile="k3")
        a_d = _to_dev(a, form)
        g_d = p.inverse(a_d)
        g_ref = O.inverse(_host(a_d), N, J, I, kind)
        assert rel(_host(g_d), g_ref) < TOL[form]
        g_in = _to_dev(g_ref, form)
        s_d = p.forward(g_in)
        assert rel(_host(s_d), O.forward(_host(g_in), N, kind)) < TOL[form]
        p.close()


def test_determinism_and_stream_order():
    N, J, I, F = 100, 201, 216, 8
    p = _plan(N, J, I, F, "cc_poles", "fp32")
    g = _to_dev(inputs.random_grid(F, J, I, seed=9), "fp32")
    s1 = p.forward(g).clone()
    s2 = p.forward(g).clone()
    torch.cuda.synchronize()
    assert torch.equal(s1, s2)
    x1 = p.inverse(s1).clone()
    x2 = p.inverse(s1).clone()
    torch.cuda.synchronize()
    assert torch.equal(x1, x2)
    p.close()


def test_nan_isolation_between_fields():
    N, J, I, F = 20, 41, 48, 8
    p = _plan(N, J, I, F, "fejer2", "fp64")
    g = inputs.random_grid(F, J, I, seed=10)
    g[3, 7, 11] = np.nan
    s = _host(p.forward(_to_dev(g, "fp64")))
    assert np.isnan(s[3]).any()
    others = np.delete(s, 3, axis=0)
    assert np.isfinite(others).all()
    p.close()


@pytest.mark.parametrize("form", FORMS)
def test_synthesis_nan_does_not_reach_a_later_analysis(form):
    # ceil(J/2) = 21 latitude rows, padded to 32.  Synthesis and analysis
    # share the plan's workspace in different layouts; what a synthesis
    # leaves there (NaN here) must not reach the padding rows the analysis
    # reads (their P~ entries are zero, and 0 * NaN is NaN).
    N, J, I, F = 20, 41, 48, 3
    p = _plan(N, J, I, F, "fejer2", form)
    a = inputs.random_spectra(N, F, seed=11)
    a[1, 5] = np.nan  # m = 0, n = 5: the odd-parity plane of m = 0
    gn = _host(p.inverse(_to_dev(a, form)))
    assert np.isnan(gn[1]).any() and np.isfinite(gn[[0, 2]]).all()
    g_d = _to_dev(inputs.random_grid(F, J, I, seed=12), form)
    s = _host(p.forward(g_d))
    assert np.isfinite(s).all()
    assert rel(s, O.forward(_host(g_d), N, "fejer2")) < TOL[form]
    p.close()


def test_error_paths_on_device():
    from paper_1711_11296_amd import Plan, SHTError
    p = Plan(10, 21, 24, 2, form="fp64")
    with pytest.raises(ValueError):
        p.forward(torch.zeros(5, device=_dev(), dtype=torch.float64))
    with pytest.raises(ValueError):
        p.forward(torch.zeros(p.grid_shape, device=_dev(), dtype=torch.float32))
    p.close()
    p.close()  # idempotent in Python
    with pytest.raises(SHTError):
        Plan(10, 21, 20, 2)      # I < 2N+1


@pytest.mark.parametrize("form", ["fp32", "bf16x6"])
def test_wide_items_first_launch_in_fresh_process(form):
    """A large single-level FP32-data plan with I = 480 and N + 1 <= 256
    runs the zonal stage with 16-field work items; its launch sizing must not
    depend on an earlier launch of another zonal kernel in the process, so
    the plan's first transform runs in a fresh interpreter (round trip,
    J >= 2N+1, spectra against their input; 201 latitude pairs x 25 field
    blocks of 16)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import torch\n"
        "from paper_1711_11296_amd import Plan, inputs\n"
        "N, J, I, F = 200, 401, 480, 400\n"
        "p = Plan(N, J, I, F, grid='cc_poles', form=%r)\n"
        "a = torch.from_numpy(inputs.random_spectra(N, F, seed=3, profile='k3')).to('cuda:0', torch.float32)\n"
        "s = p.forward(p.inverse(a))\n"
        "torch.cuda.synchronize()\n"
        "print('ERR', float((s - a).norm() / a.norm()))\n" % (root, form))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    err = float([ln for ln in r.stdout.splitlines() if ln.startswith("ERR")][-1].split()[1])
    assert err < 10 * TOL[form], err


@pytest.mark.parametrize("form", ["fp32", "bf16x6"])
def test_wide_items_with_80_column_tiles(form):
    """360 fields at I = 480: the zonal stage uses 16-field items (32
    workspace columns each) and the Legendre kernels 80-column tiles, so the
    workspace row must hold a whole number of both (800 columns, not 720):
    with 720 the last item of a row wrote 16 columns into the next row.  The
    fields of the last item and of the first items are compared with the
    oracle in both directions."""
    N, J, I, F = 200, 401, 480, 360
    sel = [0, 7, 8, 15, 351, 352, 359]
    p = _plan(N, J, I, F, "cc_poles", form)
    g = _to_dev(inputs.random_grid(F, J, I, seed=31), form)
    s = _host(p.forward(g))[sel]
    ref = O.forward(_host(g[sel]), N, "cc_poles")
    errs = [rel(s[k], ref[k]) for k in range(len(sel))]
    assert max(errs) < TOL[form], errs
    a = _to_dev(inputs.random_spectra(N, F, seed=32, profile="k3"), form)
    x = _host(p.inverse(a))[sel]
    ref = O.inverse(_host(a[sel]), N, J, I, "cc_poles")
    errs = [rel(x[k], ref[k]) for k in range(len(sel))]
    assert max(errs) < TOL[form], errs
    p.close()


def _kept_flops_from_oracle(N, J, F, kind, kb):
    """Legendre flops left after dropping, per m, the whole kb-latitude
    blocks at the pole where every |P~_n^m| < 1e-16 (scan of the oracle's P~)."""
    _, mu, s = O.nodes(J, kind)
    Jh = (J + 1) // 2
    kept = 0.0
    for m in range(N + 1):
        big = (np.abs(O.alf_m(N, m, mu[:Jh], s[:Jh])) >= 1e-16).any(axis=0)
        j0 = int(np.argmax(big)) if big.any() else Jh
        kept += 4.0 * (N - m + 1) * F * (Jh - j0 // kb * kb)
    return kept


@pytest.mark.parametrize("form", FORMS)
def test_reduced_transform(form):
    """Reduced transform (Sec. 4.1): for each m the polar latitudes where
    every |P~_n^m| < 1e-16 are left out of both sums.  The work left out
    matches a scan of the oracle's P~, and both directions still match the
    full transform of the oracle to the form's tolerance."""
    from paper_1711_11296_amd import Plan
    N, J, I, F, kind = 479, 959, 1440, 6, "fejer2"
    p = Plan(N, J, I, F, grid=kind, form=form, reduced=True)
    kept = _kept_flops_from_oracle(N, J, F, kind, 16 if form == "fp64" else 32)
    assert abs(p.legendre_flops_kept - kept) <= 1e-3 * kept
    assert p.legendre_flops_kept < 0.9 * p.legendre_flops
    a = inputs.random_spectra(N, F, seed=5, profile="k3")
    a_d = _to_dev(a, form)
    a_in = _host(a_d)
    g_d = p.inverse(a_d)
    g_in = _host(g_d)
    assert rel(g_in, O.inverse(a_in, N, J, I, kind)) < TOL[form], "inverse"
    s_d = p.forward(g_d)
    assert rel(_host(s_d), O.forward(g_in, N, kind)) < TOL[form], "forward"
    p.close()
    full = Plan(N, J, I, F, grid=kind, form=form)
    assert full.legendre_flops_kept == full.legendre_flops
    full.close()
