"""The largest sizes the library takes: the longest zonal FFT (I = 4096,
runtime radices) with the largest truncation it allows (N = 2047, i.e. 2048
wavenumbers, four per thread of the zonal kernel, and 16 row tiles per m in
the Legendre kernels) on a short grid (J = 101 < 2N+1: the discrete maps
are still what the oracle computes), and a plan with the maximum of eight
levels, in both zonal launch modes.  Each against the oracle."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_1711_11296_amd import Plan, inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-6}


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().double().numpy()


def _rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def test_longest_fft_and_largest_truncation():
    N, J, I, F, kind = 2047, 101, 4096, 2, "cc_poles"
    a = inputs.random_spectra(N, F, seed=3, profile="inv1")
    g_ref = O.inverse(a, N, J, I, kind)
    s_ref = O.forward(g_ref, N, kind)
    for form in ("fp64", "fp32"):
        dt = torch.float64 if form == "fp64" else torch.float32
        p = Plan(N, J, I, F, grid=kind, form=form)
        ad = torch.from_numpy(a).to("cuda:0", dt)
        g = p.inverse(ad)
        # the forward map is applied to the oracle's grid (rounded to the
        # form's type), so that both directions are checked on their own
        s = p.forward(torch.from_numpy(g_ref).to("cuda:0", dt))
        if form == "fp64":
            gi_ref, sf_ref = g_ref, s_ref
        else:  # the oracle on the FP32-rounded inputs the GPU received
            gi_ref = O.inverse(_host(ad), N, J, I, kind)
            sf_ref = O.forward(_host(torch.from_numpy(g_ref).to(dt)), N, kind)
        ei = [_rel(x, r) for x, r in zip(_host(g), gi_ref)]
        ef = [_rel(x, r) for x, r in zip(_host(s), sf_ref)]
        print("N=2047 I=4096 %s: inverse %s forward %s" % (form, ["%.2e" % e for e in ei], ["%.2e" % e for e in ef]))
        assert max(ei) < TOL[form] and max(ef) < TOL[form]
        p.close()


@pytest.mark.parametrize("zonal", ["one_launch", "per_length"])
@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_eight_levels(form, zonal):
    levels = [(8, 17, 32, 1), (16, 33, 64, 2), (24, 49, 64, 3), (32, 65, 100, 1), (40, 81, 128, 2),
              (64, 129, 200, 3), (100, 201, 400, 2), (200, 401, 800, 1)]
    dt = torch.float64 if form == "fp64" else torch.float32
    p = Plan(levels=levels, grid="cc_poles", form=form, zonal=zonal)
    assert p.zonal_one_launch == ((True, True) if zonal == "one_launch" else (False, False))
    a = np.concatenate([inputs.random_spectra(N, F, seed=70 + k, profile="inv1").ravel()
                        for k, (N, J, I, F) in enumerate(levels)])
    g = p.inverse(torch.from_numpy(a).to("cuda:0", dt))
    s = p.forward(g)
    ah, gh, sh = _host(torch.from_numpy(a).to(dt)), _host(g), _host(s)
    for k, (N, J, I, F) in enumerate(levels):
        go, so = p.grid_offsets[k], p.spec_offsets[k]
        ak = ah[so:so + F * (N + 1) * (N + 2)].reshape(F, -1, 2)
        gk = gh[go:go + F * J * I].reshape(F, J, I)
        assert _rel(gk, O.inverse(ak, N, J, I, "cc_poles")) < TOL[form], ("inverse", levels[k])
        sk = sh[so:so + F * (N + 1) * (N + 2)].reshape(F, -1, 2)
        assert _rel(sk, O.forward(gk, N, "cc_poles")) < TOL[form], ("forward", levels[k])
    p.close()
