"""The nested hierarchy batched in one plan (Sec. 3.2 nesting):
N = 32..512, J = 2N+1 on the grid with the poles, I = 100..1600, 32 fields
per level, FP32, autotuned Legendre tiles, graph replay.  Each level is
checked against the oracle; a coarse level fed the injected fine grid must
return the truncated spectrum."""

import os

import numpy as np
import pytest

import oracle as O
from paper_1711_11296_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LEVELS = [(32, 65, 100, 32), (64, 129, 200, 32), (128, 257, 400, 32),
          (256, 513, 800, 32), (512, 1025, 1600, 32)]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def plan(tmp_path_factory):
    from paper_1711_11296_amd import Plan
    _dev()
    os.environ["SHT_TUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "cache.txt")
    p = Plan(levels=LEVELS, grid="cc_poles", form="fp32", autotune=True, use_graph=True)
    yield p
    p.close()


def _split(p, buf, kind):
    out = []
    for k, (N, J, I, F) in enumerate(p.levels):
        if kind == "spec":
            o, n = p.spec_offsets[k], F * (N + 1) * (N + 2)
            out.append(buf[o:o + n].reshape(F, (N + 1) * (N + 2) // 2, 2))
        else:
            o, n = p.grid_offsets[k], F * J * I
            out.append(buf[o:o + n].reshape(F, J, I))
    return out


def test_hierarchy_against_oracle(plan):
    specs = [inputs.random_spectra(N, F, seed=k, profile="k3") for k, (N, J, I, F) in enumerate(LEVELS)]
    a = torch.from_numpy(np.concatenate([s.ravel() for s in specs])).to(_dev(), torch.float32)
    g = plan.inverse(a)
    s = plan.forward(g)
    gl = _split(plan, _np(g), "grid")
    sl = _split(plan, _np(s), "spec")
    al = _split(plan, _np(a), "spec")
    for k, (N, J, I, F) in enumerate(LEVELS):
        fs = slice(0, F) if N <= 128 else slice(0, 2)
        g_ref = O.inverse(al[k][fs], N, J, I, "cc_poles")
        assert rel(gl[k][fs], g_ref) < 1e-6, ("inverse", N)
        s_ref = O.forward(gl[k][fs], N, "cc_poles")
        assert rel(sl[k][fs], s_ref) < 1e-6, ("forward", N)
        assert rel(sl[k], al[k]) < 2e-6, ("round trip", N)


def test_graph_replay_matches_eager(plan):
    specs = [inputs.random_spectra(N, F, seed=10 + k, profile="k3") for k, (N, J, I, F) in enumerate(LEVELS)]
    a = torch.from_numpy(np.concatenate([s.ravel() for s in specs])).to(_dev(), torch.float32)
    g = torch.empty(plan.grid_elems, device=_dev(), dtype=torch.float32)
    s = torch.empty(plan.spec_elems, device=_dev(), dtype=torch.float32)
    plan.inverse(a, out=g)           # eager, then captured
    plan.forward(g, out=s)
    torch.cuda.synchronize()
    g0, s0 = g.clone(), s.clone()
    for _ in range(3):               # replays, with eager host work between
        g.zero_()
        s.zero_()
        torch.cuda.synchronize()
        plan.inverse(a, out=g)
        plan.forward(g, out=s)
        torch.cuda.synchronize()
        assert torch.equal(g, g0) and torch.equal(s, s0)


def test_injection_equals_truncation(plan):
    """Level k's grid taken as every other row and column of level k+1's grid
    (both synthesised from a spectrum band-limited to N_k) analyses back to
    that spectrum."""
    F = 32
    base = [inputs.random_spectra(N, F, seed=20 + k, profile="k3") for k, (N, J, I, F) in enumerate(LEVELS)]
    # level k+1 carries level k's spectrum zero-padded to N_{k+1}
    specs = [base[0]]
    for k in range(1, len(LEVELS)):
        Nc, Nf = LEVELS[k - 1][0], LEVELS[k][0]
        padded = np.zeros((F, O.ncoef(Nf), 2))
        for m in range(Nc + 1):
            padded[:, O.spec_index(Nf, m, m):O.spec_index(Nf, m, Nc) + 1] = \
                base[k - 1][:, O.spec_index(Nc, m, m):O.spec_index(Nc, m, Nc) + 1]
        specs.append(padded)
    a = torch.from_numpy(np.concatenate([s.ravel() for s in specs])).to(_dev(), torch.float32)
    g = plan.inverse(a)
    gl = _split(plan, g, "grid")
    inj = torch.empty_like(g)
    il = _split(plan, inj, "grid")
    il[-1].copy_(gl[-1])
    for k in range(len(LEVELS) - 1):
        il[k].copy_(gl[k + 1][:, ::2, ::2])
    s = _np(plan.forward(inj))
    sl = _split(plan, s, "spec")
    for k in range(len(LEVELS) - 1):
        assert rel(sl[k], base[k]) < 2e-6, LEVELS[k]


def test_autotune_cache_written(plan):
    path = os.environ["SHT_TUNE_CACHE"]
    txt = open(path).read()
    line = [ln for ln in txt.splitlines() if " lev5 " in ln][-1]
    # the plan runs the zonal launch modes the tuner stored
    assert plan.zonal_one_launch == tuple(bool(int(v)) for v in line.split("|")[1].split()[4:6])
    assert " form1 " in line and " v3 " in line and "|" in line
    vals = [int(x) for x in line.split("|")[1].split()]
    # Legendre blocking and order per direction, then the zonal launch
    # choice per direction (one launch or per FFT length)
    assert len(vals) == 6 and vals[4] in (0, 1) and vals[5] in (0, 1)


@pytest.mark.parametrize("form", ["fp64", "bf16x6"])
def test_mixed_length_levels_other_forms(form):
    """A multi-level plan whose levels mix lengths with a compile-time FFT
    plan (I = 400, 800) and without one (I = 200, 300), in the FP64 and
    split forms (one zonal launch per direction covers every level): each
    level against the oracle."""
    from paper_1711_11296_amd import Plan
    levels = [(64, 129, 200, 3), (128, 257, 400, 2), (149, 150, 300, 5), (399, 97, 800, 2)]
    dt = torch.float64 if form == "fp64" else torch.float32
    tol = 1e-12 if form == "fp64" else 1e-6
    p = Plan(levels=levels, grid="cc_poles", form=form)
    specs = [inputs.random_spectra(N, F, seed=30 + k, profile="inv1") for k, (N, J, I, F) in enumerate(levels)]
    a = torch.from_numpy(np.concatenate([s.ravel() for s in specs])).to(_dev(), dt)
    g = p.inverse(a)
    s = p.forward(g)
    al, gl, sl = _split(p, _np(a), "spec"), _split(p, _np(g), "grid"), _split(p, _np(s), "spec")
    for k, (N, J, I, F) in enumerate(levels):
        assert rel(gl[k], O.inverse(al[k], N, J, I, "cc_poles")) < tol, ("inverse", levels[k])
        assert rel(sl[k], O.forward(gl[k], N, "cc_poles")) < tol, ("forward", levels[k])
    p.close()


@pytest.mark.parametrize("zonal", ["one_launch", "per_length"])
@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16x6"])
def test_levels_ragged(form, zonal):
    """Both launch modes of a multi-level zonal stage (one launch over all
    levels; one per FFT length) with every kind of level the one-launch
    kernel takes (I = 1600, 800 and 400 with compile-time plans, I = 100 and
    128 with runtime radices), in plan order unlike their sizes, odd and even
    J, field counts that leave partial field blocks, all three forms: each
    level of both directions against the oracle."""
    from paper_1711_11296_amd import Plan
    levels = [(500, 1001, 1600, 11), (40, 81, 100, 9), (130, 262, 400, 13), (200, 401, 800, 3),
              (60, 121, 128, 17)]
    dt = torch.float64 if form == "fp64" else torch.float32
    tol = 1e-12 if form == "fp64" else 1e-6
    p = Plan(levels=levels, grid="cc_poles", form=form, zonal=zonal)
    assert p.zonal_one_launch == ((True, True) if zonal == "one_launch" else (False, False))
    specs = [inputs.random_spectra(N, F, seed=40 + k, profile="inv1") for k, (N, J, I, F) in enumerate(levels)]
    a = torch.from_numpy(np.concatenate([s.ravel() for s in specs])).to(_dev(), dt)
    g = p.inverse(a)
    s = p.forward(g)
    al, gl, sl = _split(p, _np(a), "spec"), _split(p, _np(g), "grid"), _split(p, _np(s), "spec")
    p.close()
    for k, (N, J, I, F) in enumerate(levels):
        assert rel(gl[k], O.inverse(al[k], N, J, I, "cc_poles")) < tol, ("inverse", levels[k])
        assert rel(sl[k], O.forward(gl[k], N, "cc_poles")) < tol, ("forward", levels[k])


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_per_length_levels(form):
    """A multi-level plan with a length outside the one-launch kernel (I =
    480) takes one zonal launch per compile-time length plus one for the
    runtime-radix levels: each level against the oracle."""
    from paper_1711_11296_amd import Plan
    levels = [(159, 319, 480, 5), (64, 129, 200, 3), (100, 201, 400, 10), (30, 40, 90, 2)]
    dt = torch.float64 if form == "fp64" else torch.float32
    tol = 1e-12 if form == "fp64" else 1e-6
    p = Plan(levels=levels, grid="cc_poles", form=form)
    specs = [inputs.random_spectra(N, F, seed=50 + k, profile="inv1") for k, (N, J, I, F) in enumerate(levels)]
    a = torch.from_numpy(np.concatenate([s.ravel() for s in specs])).to(_dev(), dt)
    g = p.inverse(a)
    s = p.forward(g)
    al, gl, sl = _split(p, _np(a), "spec"), _split(p, _np(g), "grid"), _split(p, _np(s), "spec")
    p.close()
    for k, (N, J, I, F) in enumerate(levels):
        assert rel(gl[k], O.inverse(al[k], N, J, I, "cc_poles")) < tol, ("inverse", levels[k])
        assert rel(sl[k], O.forward(gl[k], N, "cc_poles")) < tol, ("forward", levels[k])


def test_concurrent_levels_keep_stream_order():
    """A multi-level plan's several launches per direction stay ordered on
    the caller's stream: a chain on a side stream (input produced on that
    stream, synthesis, an in-place scaling of the grids, analysis, again)
    equals the same chain on the default stream bit for bit."""
    from paper_1711_11296_amd import Plan
    _dev()
    p = Plan(levels=LEVELS, grid="cc_poles", form="fp32")
    a = torch.from_numpy(np.concatenate([inputs.random_spectra(N, F, seed=20 + k, profile="k3").ravel()
                                         for k, (N, J, I, F) in enumerate(LEVELS)])).to(_dev(), torch.float32)

    def chain():
        x = a * 1.0
        for _ in range(3):
            g = p.inverse(x)
            g.mul_(2.0)
            x = p.forward(g)
            x.mul_(0.5)
        return x

    ref = chain()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        got = chain()
    side.synchronize()
    assert torch.equal(got, ref)
    assert rel(_np(got), _np(a)) < 1e-5   # the levels are exact (J = 2N+1): a round trip
    p.close()


@pytest.mark.parametrize("zonal", ["one_launch", "per_length"])
@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_levels_reduced_transform(form, zonal):
    """The reduced transform (Sec. 4.1) on a multi-level plan in both zonal
    launch modes: the synthesis leaves whole 128-latitude tiles of the high
    orders out of the workspace and the zonal synthesis reads them as zero;
    each level of both directions still matches the oracle's full
    transform."""
    from paper_1711_11296_amd import Plan
    levels = [(500, 1001, 1600, 5), (130, 262, 400, 3), (40, 81, 100, 2)]
    dt = torch.float64 if form == "fp64" else torch.float32
    tol = 1e-12 if form == "fp64" else 1e-6
    p = Plan(levels=levels, grid="cc_poles", form=form, reduced=True, zonal=zonal)
    assert p.legendre_flops_kept < p.legendre_flops
    specs = [inputs.random_spectra(N, F, seed=60 + k, profile="k3") for k, (N, J, I, F) in enumerate(levels)]
    a = torch.from_numpy(np.concatenate([s.ravel() for s in specs])).to(_dev(), dt)
    g = p.inverse(a)
    s = p.forward(g)
    al, gl, sl = _split(p, _np(a), "spec"), _split(p, _np(g), "grid"), _split(p, _np(s), "spec")
    p.close()
    for k, (N, J, I, F) in enumerate(levels):
        assert rel(gl[k], O.inverse(al[k], N, J, I, "cc_poles")) < tol, ("inverse", levels[k])
        assert rel(sl[k], O.forward(gl[k], N, "cc_poles")) < tol, ("forward", levels[k])
