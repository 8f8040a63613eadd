"""The Gaussian grid and the aliasing of nonlinear terms (Sec. 4.2) on the
GPU: transforms on the Gaussian grid against the oracle, the pointwise
product kernel, and the quadratic-term aliasing that the linear CC grid
shows and the quadratic one removes (Sec. 3.1, eq. cc-condition)."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_1711_11296_amd import Plan, grid_product, inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x6": 1e-6}


def _rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().double().numpy()


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x6"])
@pytest.mark.parametrize("N,J,I,F", [(42, 43, 128, 3), (100, 101, 216, 5), (64, 80, 200, 2)])
def test_gauss_grid_round_trip(form, N, J, I, F):
    """Gauss-Legendre with J >= N+1 nodes is exact for the transform pair:
    both directions match the oracle and analysis inverts synthesis."""
    dt = torch.float64 if form == "fp64" else torch.float32
    p = Plan(N, J, I, F, grid="gauss", form=form)
    assert p.exact
    a = torch.from_numpy(inputs.random_spectra(N, F, seed=N, profile="k3")).to("cuda:0", dt)
    a_in = _host(a)
    g = p.inverse(a)
    g_in = _host(g)
    assert _rel(g_in, O.inverse(a_in, N, J, I, "gauss")) < TOL[form]
    s = p.forward(g)
    assert _rel(_host(s), O.forward(g_in, N, "gauss")) < TOL[form]
    assert _rel(_host(s), a_in) < 10 * TOL[form]
    p.close()


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("n", [1, 3, 4, 1000, 65537, 3 * 959 * 2880 + 1])
def test_grid_product_matches_numpy(dt, n):
    rng = np.random.default_rng(n)
    a = torch.from_numpy(rng.standard_normal(n)).to("cuda:0", dt)
    b = torch.from_numpy(rng.standard_normal(n)).to("cuda:0", dt)
    out = _host(grid_product(a, b))
    ref = a.cpu().numpy() * b.cpu().numpy()
    assert np.array_equal(out, ref.astype(np.float64))


def test_quadratic_term_aliasing():
    """Sec. 4.2 / Sec. 3.1: the spectrum of the product of two fields
    band-limited at N, analysed at N, is alias-free on the Gaussian grid
    with J >= (3N+1)/2 (the reference) and on the CC grid with J >= 3N+1
    (the quadratic grid), but aliased on the linear CC grid J = 2N+1."""
    N, F, I = 42, 2, 128                      # I >= 3N+1: the zonal products do not alias
    # the slowly decaying random spectra of the aliasing experiment; with a
    # steep spectrum the aliased part is far smaller (about 3e-7 for "k3")
    U = torch.from_numpy(inputs.random_spectra(N, F, seed=1, profile="uniform13")).to("cuda:0", torch.float64)
    V = torch.from_numpy(inputs.random_spectra(N, F, seed=2, profile="uniform13")).to("cuda:0", torch.float64)

    def uv_spectrum(kind, J):
        p = Plan(N, J, I, F, grid=kind, form="fp64")
        s = _host(p.forward(grid_product(p.inverse(U), p.inverse(V))))
        p.close()
        return s

    ref = uv_spectrum("gauss", (3 * N + 1 + 1) // 2)
    ref2 = uv_spectrum("gauss", 2 * N + 1)
    assert _rel(ref, ref2) < 1e-12               # both Gaussian grids are alias-free
    quad = uv_spectrum("cc_poles", 3 * N + 1)
    assert _rel(quad, ref) < 1e-12
    lin = uv_spectrum("cc_poles", 2 * N + 1)
    assert _rel(lin, ref) > 2e-5                  # the linear grid aliases the quadratic term
    # the aliased spectrum itself is the oracle's on the same grid
    Uh, Vh = _host(U), _host(V)
    lin_o = O.forward(O.inverse(Uh, N, 2 * N + 1, I, "cc_poles") * O.inverse(Vh, N, 2 * N + 1, I, "cc_poles"),
                      N, "cc_poles")
    assert _rel(lin, lin_o) < 1e-12
