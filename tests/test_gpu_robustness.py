"""Failure handling and plan-level machinery on the GPU: the graph cache of
use_graph plans past its 16 entries, the autotuner's cache when it holds an
inadmissible entry, and the out-of-memory path at plan time (forced from the
host with SHT_TEST_MAX_BYTES, so no allocation really fails)."""

import os

import numpy as np
import pytest

import oracle as O
from paper_1711_11296_amd import _lib, inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def test_graph_cache_cycles_past_its_capacity():
    """20 distinct (input, output) pairs per direction through a use_graph
    plan (graphs of the oldest pairs are destroyed while later launches may
    still be queued), then the first pairs again (captured anew): every
    result equals the eager plan's bit for bit."""
    from paper_1711_11296_amd import Plan
    N, J, I, F = 60, 121, 128, 6
    pg = Plan(N, J, I, F, grid="cc_poles", form="fp32", use_graph=True)
    pe = Plan(N, J, I, F, grid="cc_poles", form="fp32")
    grids = [torch.from_numpy(inputs.random_grid(F, J, I, seed=100 + k)).to(_dev(), torch.float32)
             for k in range(20)]
    outs = [torch.empty(pg.spec_shape, device=_dev(), dtype=torch.float32) for _ in range(20)]
    grids_back = [torch.empty(pg.grid_shape, device=_dev(), dtype=torch.float32) for _ in range(20)]
    for rep in range(2):
        for k in list(range(20)) + list(range(4)):
            pg.forward(grids[k], out=outs[k])
            pg.inverse(outs[k], out=grids_back[k])
        torch.cuda.synchronize()
        for k in range(20):
            assert torch.equal(outs[k], pe.forward(grids[k])), (rep, k)
            assert torch.equal(grids_back[k], pe.inverse(outs[k])), (rep, k)
    pg.close()
    pe.close()


def test_autotune_cache_with_an_inadmissible_entry(tmp_path, monkeypatch):
    """A cache line whose blocking does not fit the plan's workspace layout
    (here 64 column blocks, wider than any kernel takes), or whose zonal
    launch choice is neither 0 nor 1, is not used: the plan re-tunes, stores
    an admissible line and still matches the oracle."""
    from paper_1711_11296_amd import Plan
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SHT_TUNE_CACHE", str(cache))
    N, J, I, F = 80, 161, 180, 24
    p = Plan(N, J, I, F, grid="fejer2", form="fp32", autotune=True)
    p.close()
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and "|" in lines[0]
    key, vals = lines[0].split("|")
    assert "hip" in key and " v3 " in key
    good = [int(v) for v in vals.split()]
    assert len(good) == 6
    # a zonal launch choice outside {0, 1} with an otherwise good line
    cache.write_text("%s|%d %d %d %d 2 1\n" % (key, *good[:4]))
    Plan(N, J, I, F, grid="fejer2", form="fp32", autotune=True).close()
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and [int(v) for v in lines[1].split("|")[1].split()][4:] == [1, 1]
    cache.write_text("%s|64 0 64 1 1 1\n" % key)
    p = Plan(N, J, I, F, grid="fejer2", form="fp32", autotune=True)
    g = torch.from_numpy(inputs.random_grid(F, J, I, seed=21)).to(_dev(), torch.float32)
    s = p.forward(g)
    ref = O.forward(_host(g), N, "fejer2")
    assert np.linalg.norm(_host(s) - ref) / np.linalg.norm(ref) < 1e-6
    a = torch.from_numpy(inputs.random_spectra(N, F, seed=22, profile="k3")).to(_dev(), torch.float32)
    x = p.inverse(a)
    ref = O.inverse(_host(a), N, J, I, "fejer2")
    assert np.linalg.norm(_host(x) - ref) / np.linalg.norm(ref) < 1e-6
    p.close()
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and lines[1].startswith(key + "|")
    redo = [int(v) for v in lines[1].split("|")[1].split()]
    assert redo[0] in (1, 2, 4, 8, 10) and redo[2] in (1, 2, 4, 8) and redo[1] in (0, 1) and redo[3] in (0, 1)
    assert redo[4] == 1 and redo[5] == 1   # single-level plan: the zonal choice stays "one launch"
    del good


def test_out_of_memory_at_plan_time_leaks_nothing(monkeypatch):
    """With SHT_TEST_MAX_BYTES below what the plan needs, plan construction
    fails with SHT_ENOMEM, frees what it had allocated, and a later plan
    without the limit works."""
    from paper_1711_11296_amd import Plan, SHTError
    N, J, I, F = 200, 401, 480, 16
    before = _lib.device_bytes()
    probe = Plan(N, J, I, F, grid="cc_poles", form="fp32")
    need = _lib.device_bytes() - before
    probe.close()
    assert _lib.device_bytes() == before
    torch.cuda.synchronize()
    for frac in (0.1, 0.5, 0.99):
        monkeypatch.setenv("SHT_TEST_MAX_BYTES", str(before + int(frac * need)))
        with pytest.raises(SHTError) as ei:
            Plan(N, J, I, F, grid="cc_poles", form="fp32")
        assert ei.value.code == _lib.SHT_ENOMEM
        assert "SHT_TEST_MAX_BYTES" in str(ei.value)
        assert _lib.device_bytes() == before
    monkeypatch.delenv("SHT_TEST_MAX_BYTES")
    p = Plan(N, J, I, F, grid="cc_poles", form="fp32")
    a = torch.from_numpy(inputs.random_spectra(N, F, seed=23, profile="k3")).to(_dev(), torch.float32)
    s = p.forward(p.inverse(a))
    assert float((s - a).norm() / a.norm()) < 1e-5
    p.close()
    assert _lib.device_bytes() == before
    assert os.environ.get("SHT_TEST_MAX_BYTES") is None
