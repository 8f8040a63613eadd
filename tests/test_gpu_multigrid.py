"""The residual and restriction steps of the App. C two-grid cycle on the
GPU, through the C ABI: the spectral Laplacian and the residual update
against the oracle, the composed residual on two nested levels of the
hierarchy (N = 32 and 64 on the grid with poles; N = 79 and 159 on the
paper's grid) in every form, and both steps on multi-level plans."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_1711_11296_amd import Plan, grid_residual, inputs, spec_laplacian
from paper_1711_11296_amd.multigrid import helmholtz_residual, restrict_to_coarse_spectra

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x6": 1e-6}


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().double().numpy()


def _rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


@pytest.mark.parametrize("N,F,scale", [(0, 2, 1.0), (21, 3, 1.0), (159, 5, 2.5e-14), (300, 1, 0.5)])
def test_spec_laplacian_matches_oracle(N, F, scale):
    a = inputs.random_spectra(N, F, seed=N + 1, profile="inv1")
    d64 = torch.from_numpy(a).to("cuda:0")
    out = _host(spec_laplacian(d64, N, scale))
    assert np.array_equal(out, O.laplacian(a, N, scale))      # same rounding: one product
    d32 = d64.float()
    out32 = _host(spec_laplacian(d32, N, scale))
    ref = O.laplacian(_host(d32), N, scale)
    assert np.allclose(out32, ref, rtol=2.4e-7, atol=0)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("F,J,I", [(1, 1, 5), (4, 3, 5), (3, 65, 100), (5, 1, 2), (2, 959, 1440)])
def test_grid_residual_matches_numpy(dt, F, J, I):
    rng = np.random.default_rng(J)
    x, y, f = (torch.from_numpy(rng.standard_normal((F, J, I))).to("cuda:0", dt) for _ in range(3))
    k = torch.from_numpy(1.0 + 0.5 * rng.random((J, I))).to("cuda:0", dt)
    r = _host(grid_residual(x, k, y, f, 0.37))
    xh, yh, fh, kh = (_host(t) for t in (x, y, f, k))
    ref = xh - 0.37 * kh[None] * yh - fh
    eps = 2.3e-16 if dt == torch.float64 else 1.2e-7
    scale = np.abs(xh) + 0.37 * np.abs(kh[None] * yh) + np.abs(fh)
    assert np.all(np.abs(r - ref) <= 4 * eps * scale)


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x6"])
@pytest.mark.parametrize("kind,Nc,Jc,Ic,Nf,Jf,If", [("cc_poles", 32, 65, 100, 64, 129, 200),
                                                    ("fejer2", 79, 159, 240, 159, 319, 480)])
def test_two_level_residual_and_restriction(form, kind, Nc, Jc, Ic, Nf, Jf, If):
    """Step 1 and the restriction of step 2 of the two-grid cycle: the
    residual R = X - alpha kappa lap(X) - F on the fine level, its injection
    and coarse analysis, and the residual on the coarse level, each against
    the oracle on the same inputs."""
    F = 3
    dt = torch.float64 if form == "fp64" else torch.float32
    alpha, scale = 0.2, 1e-4
    rng = np.random.default_rng(Nf)
    fine = Plan(Nf, Jf, If, F, grid=kind, form=form)
    coarse = Plan(Nc, Jc, Ic, F, grid=kind, form=form)
    X = fine.inverse(torch.from_numpy(inputs.random_spectra(Nf, F, seed=1, profile="inv1")).to("cuda:0", dt))
    Fr = fine.inverse(torch.from_numpy(inputs.random_spectra(Nf, F, seed=2, profile="inv1")).to("cuda:0", dt))
    kap = torch.from_numpy(1.0 + 0.5 * rng.random((Jf, If))).to("cuda:0", dt)
    R = helmholtz_residual(fine, X, kap, Fr, alpha, scale)
    Xh, Fh, kh = _host(X), _host(Fr), _host(kap)
    R_ref = O.helmholtz_residual(Xh, kh, Fh, alpha, Nf, kind, scale)
    Rh = _host(R)
    # the residual is a difference of O(1) terms: measure against the size
    # of what is subtracted
    assert np.linalg.norm(Rh - R_ref) / np.linalg.norm(Xh) < TOL[form]
    Rc = _host(restrict_to_coarse_spectra(R, coarse, kind))
    Rc_ref = O.forward(O.inject(Rh, Jc, Ic, kind), Nc, kind)
    assert _rel(Rc, Rc_ref) < TOL[form]
    # the coarse level's own residual (step 2 evaluates the same operator)
    Xc = O.inject(Xh, Jc, Ic, kind)
    Fc = O.inject(Fh, Jc, Ic, kind)
    kc = O.inject(kh[None], Jc, Ic, kind)[0]
    Rcg = _host(helmholtz_residual(coarse, torch.from_numpy(Xc).to("cuda:0", dt), torch.from_numpy(kc).to("cuda:0", dt),
                                   torch.from_numpy(Fc).to("cuda:0", dt), alpha, scale))
    Rcg_ref = O.helmholtz_residual(Xc, kc, Fc, alpha, Nc, kind, scale)
    assert np.linalg.norm(Rcg - Rcg_ref) / np.linalg.norm(Xc) < TOL[form]
    fine.close()
    coarse.close()


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x6"])
def test_multilevel_residual_and_restriction(form):
    """The residual on a multi-level plan (three nested levels of the grid
    with poles in one plan: one batched analysis and synthesis, a scale per
    level) against the oracle level by level, and the batched restriction
    of the two finer levels' residuals onto a two-level coarse plan against
    the oracle's injection and analysis.  The sizes leave some levels'
    slices of the concatenated buffers 8 bytes off a 16-byte boundary."""
    kind = "cc_poles"
    levels = [(32, 65, 90, 3), (64, 129, 180, 1), (128, 257, 360, 3)]
    dt = torch.float64 if form == "fp64" else torch.float32
    alpha, scales = 0.2, [1e-4, 2e-4, 5e-5]
    rng = np.random.default_rng(7)
    p = Plan(levels=levels, grid=kind, form=form)

    def concat(seed):
        return torch.from_numpy(np.concatenate([inputs.random_spectra(N, F, seed=seed + k, profile="inv1").ravel()
                                                for k, (N, J, I, F) in enumerate(levels)])).to("cuda:0", dt)

    X, Fr = p.inverse(concat(1)), p.inverse(concat(11))
    kap = [torch.from_numpy(1.0 + 0.5 * rng.random((J, I))).to("cuda:0", dt) for (N, J, I, F) in levels]
    R = helmholtz_residual(p, X, kap, Fr, alpha, scales)
    assert R.shape == X.shape
    Xh, Fh, Rh = _host(X), _host(Fr), _host(R)
    Rk = []
    for k, (N, J, I, F) in enumerate(levels):
        o, n = p.grid_offsets[k], F * J * I
        xk, fk, rk = (v[o:o + n].reshape(F, J, I) for v in (Xh, Fh, Rh))
        ref = O.helmholtz_residual(xk, _host(kap[k]), fk, alpha, N, kind, scales[k])
        assert np.linalg.norm(rk - ref) / np.linalg.norm(xk) < TOL[form], levels[k]
        Rk.append(rk)
    p.close()
    coarse = [(32, 65, 90, 1), (64, 129, 180, 3)]
    c = Plan(levels=coarse, grid=kind, form=form)
    Rc = _host(restrict_to_coarse_spectra([torch.from_numpy(Rk[k + 1]).to("cuda:0", dt) for k in range(2)], c, kind))
    for k, (N, J, I, F) in enumerate(coarse):
        o, n = c.spec_offsets[k], F * (N + 1) * (N + 2)
        ref = O.forward(O.inject(Rk[k + 1], J, I, kind), N, kind)
        assert _rel(Rc[o:o + n].reshape(ref.shape), ref) < TOL[form], coarse[k]
    c.close()


def test_multilevel_helpers_check_arguments():
    p = Plan(levels=[(8, 17, 32, 1), (16, 33, 64, 1)], grid="cc_poles", form="fp64")
    x = torch.zeros(p.grid_elems, dtype=torch.float64, device="cuda:0")
    k1, k2 = torch.ones(17, 32, dtype=torch.float64, device="cuda:0"), torch.ones(33, 64, dtype=torch.float64,
                                                                                    device="cuda:0")
    with pytest.raises(ValueError):
        helmholtz_residual(p, x, k1, x, 0.1)              # one kappa per level
    with pytest.raises(ValueError):
        helmholtz_residual(p, x, [k2, k1], x, 0.1)        # kappa shapes per level
    with pytest.raises(ValueError):
        helmholtz_residual(p, x[:-1], [k1, k2], x[:-1], 0.1)
    with pytest.raises(ValueError):
        restrict_to_coarse_spectra(x, p, "cc_poles")       # one fine grid per level
    p.close()
