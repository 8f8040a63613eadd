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

TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x6": 1e-6}


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().double().numpy()


def _rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def test_longest_fft_and_largest_truncation():
    """Every form, with the table and with generated P~ (whose seed rows at
    this order include values below the double range)."""
    N, J, I, F, kind = 2047, 101, 4096, 2, "cc_poles"
    a = inputs.random_spectra(N, F, seed=3, profile="inv1")
    g64 = O.inverse(a, N, J, I, kind)
    refs = {torch.float64: (g64, O.forward(g64, N, kind))}
    for form in ("fp64", "fp32", "bf16x6"):
        dt = torch.float64 if form == "fp64" else torch.float32
        ad = torch.from_numpy(a).to("cuda:0", dt)
        gd = torch.from_numpy(g64).to("cuda:0", dt)
        if dt not in refs:  # the oracle on the FP32-rounded inputs the GPU receives
            refs[dt] = (O.inverse(_host(ad), N, J, I, kind), O.forward(_host(gd), N, kind))
        gi_ref, sf_ref = refs[dt]
        out = {}
        for otf in (False, True):
            p = Plan(N, J, I, F, grid=kind, form=form, otf=otf)
            # the forward map is applied to the oracle's grid, so that both
            # directions are checked on their own
            g, s = _host(p.inverse(ad)), _host(p.forward(gd))
            p.close()
            ei = [_rel(x, r) for x, r in zip(g, gi_ref)]
            ef = [_rel(x, r) for x, r in zip(s, sf_ref)]
            print("N=2047 I=4096 %s%s: inverse %s forward %s" % (form, " otf" if otf else "",
                                                                ["%.2e" % e for e in ei], ["%.2e" % e for e in ef]))
            assert max(ei) < TOL[form] and max(ef) < TOL[form]
            out[otf] = (g, s)
        # generated and stored P~ agree to a few roundings of the element type
        close = 1e-13 if form == "fp64" else 1e-7
        assert _rel(out[True][0], out[False][0]) < close and _rel(out[True][1], out[False][1]) < close


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


def test_workspace_beyond_4_gib():
    """T959 with 600 fields: the workspace (8.8 GB) is past 4 GiB, which the
    fixed-length zonal kernels address from a per-wave base; the first, a
    middle and the last field of both directions against the oracle."""
    N, J, I, F, kind = 959, 1919, 2880, 600, "cc_poles"
    p = Plan(N, J, I, F, grid=kind, form="fp32")
    assert p.workspace_bytes > 2 ** 32
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(11)
    a = torch.randn(p.spec_shape, generator=gen, device="cuda:0", dtype=torch.float32)
    g = p.inverse(a)
    s = p.forward(g)
    sel = [0, 299, F - 1]
    ah, gh, sh = _host(a[sel]), _host(g[sel]), _host(s[sel])
    del a, g, s
    p.close()
    torch.cuda.empty_cache()
    ei = [_rel(x, r) for x, r in zip(gh, O.inverse(ah, N, J, I, kind))]
    ef = [_rel(x, r) for x, r in zip(sh, O.forward(gh, N, kind))]
    print("T959 600 fields: inverse %s forward %s" % (["%.2e" % e for e in ei], ["%.2e" % e for e in ef]))
    assert max(ei) < 1e-6 and max(ef) < 1e-6
