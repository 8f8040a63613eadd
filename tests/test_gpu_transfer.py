"""Transfers between levels (App. C building blocks) on the GPU, through the
C ABI: spectral re-truncation and grid injection against the oracle (bit for
bit: they are copies), and the two-grid identity with the transforms."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_1711_11296_amd import Plan, grid_inject, inputs, spec_retruncate

pytestmark = pytest.mark.gpu


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", dt)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("N_in,N_out,F", [(21, 10, 3), (10, 21, 3), (17, 17, 1), (0, 5, 2), (300, 159, 5),
                                          (159, 300, 2), (5, 0, 4)])
def test_spec_retruncate_matches_oracle(dt, N_in, N_out, F):
    a = inputs.random_spectra(N_in, F, seed=N_in + 7 * N_out, profile="inv1")
    a_d = _dev(a, dt)
    out = spec_retruncate(a_d, N_in, N_out)
    torch.cuda.synchronize()
    ref = O.retruncate(a_d.cpu().double().numpy(), N_in, N_out)
    assert np.array_equal(out.cpu().double().numpy(), ref)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("kind,Jf,If,Jc,Ic,F", [("cc_poles", 1025, 1600, 513, 800, 2),
                                                ("cc_poles", 129, 200, 33, 50, 3),
                                                ("fejer2", 959, 1440, 479, 720, 2),
                                                ("fejer2", 959, 1440, 319, 480, 1),
                                                ("fejer2", 7, 9, 3, 3, 5)])
def test_grid_inject_matches_oracle(dt, kind, Jf, If, Jc, Ic, F):
    g = np.random.default_rng(Jf + Jc).standard_normal((F, Jf, If))
    g_d = _dev(g, dt)
    out = grid_inject(g_d, Jc, Ic, kind)
    torch.cuda.synchronize()
    ref = O.inject(g_d.cpu().double().numpy(), Jc, Ic, kind)
    assert np.array_equal(out.cpu().double().numpy(), ref)


@pytest.mark.parametrize("form,tol", [("fp64", 1e-12), ("fp32", 1e-6), ("bf16x6", 1e-6)])
def test_two_grid_restriction_identity(form, tol):
    """A field band-limited at the coarse truncation: injection then the
    coarse analysis equals the fine analysis restricted by re-truncation
    (Sec. 3.2, App. C), both on the GPU."""
    kind, Nc, Jc, Ic, Jf, If, F = "fejer2", 159, 319, 480, 959, 1440, 4
    Nf = 479
    dt = torch.float64 if form == "fp64" else torch.float32
    a = inputs.random_spectra(Nc, F, seed=3, profile="k3")
    a_f = spec_retruncate(_dev(a, dt), Nc, Nf)          # prolongation: zero-padded
    pf = Plan(Nf, Jf, If, F, grid=kind, form=form)
    pc = Plan(Nc, Jc, Ic, F, grid=kind, form=form)
    g_f = pf.inverse(a_f)
    via_grid = pc.forward(grid_inject(g_f, Jc, Ic, kind))
    via_spec = spec_retruncate(pf.forward(g_f), Nf, Nc)
    torch.cuda.synchronize()
    x = via_grid.cpu().double().numpy()
    y = via_spec.cpu().double().numpy()
    ref = a.astype(np.float64) if form == "fp64" else _dev(a, dt).cpu().double().numpy()
    for v in (x, y):
        assert np.linalg.norm(v - ref) / np.linalg.norm(ref) < 10 * tol
    pf.close()
    pc.close()
