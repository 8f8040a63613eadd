"""Python face of the transform library: a plan object over the C ABI and
the host-only table export.  Every transform step runs in the HIP library;
this module only checks shapes and passes pointers and the current stream.
"""

import ctypes

import numpy as np

from . import _lib


def host_tables(N, J, grid="cc_poles"):
    """Nodes mu_j, weights w_j and the FP64 table of P~_n^m for the northern
    rows, as the library builds them (no GPU needed).
    Returns (mu [J], w [J], alf [ncoef, ceil(J/2)])."""
    lib = _lib.load(require_torch=False)
    Jh = (J + 1) // 2
    nc = (N + 1) * (N + 2) // 2
    mu = np.zeros(J)
    w = np.zeros(J)
    alf = np.zeros((nc, Jh))
    dp = ctypes.POINTER(ctypes.c_double)
    _lib.check(lib.sht_host_tables(N, J, _lib.GRID[grid], mu.ctypes.data_as(dp),
                                   w.ctypes.data_as(dp), alf.ctypes.data_as(dp)))
    return mu, w, alf


class Plan:
    """A transform plan on the current GPU.

    levels: one (N, J, I, nfields) tuple, or a list of them for a batched
    hierarchy run together (one Legendre launch per direction for all
    levels).  grid: "cc_poles", "fejer2", "fejer1" or "gauss";
    form: "fp64", "fp32" or "bf16x6".  reduced: leave out, per m, the polar
    latitudes where every |P~_n^m| < 1e-16 (the reduced transform of
    Sec. 4.1; see sht_options.reduced).  use_graph: each (direction, input
    buffer, output buffer) triple is captured into a hipGraph on its first
    call and replayed afterwards; at most 16 graphs are kept per plan, so pass
    the same out= buffers on every call (without out= a new output tensor,
    hence a new capture, may be made each time).  otf: both Legendre kernels
    generate P~ in FP64 from two stored seed rows per 16 degrees instead of
    reading a table, in every form (see sht_options.otf).  zonal (several
    levels): "auto", "one_launch" or "per_length", how the zonal stage is
    launched (see sht_zonal_t; with autotune, "auto" takes the faster).
    """

    def __init__(self, N=None, J=None, I=None, nfields=None, *, levels=None, grid="cc_poles",
                 form="fp64", autotune=False, use_graph=False, reduced=False, otf=False, zonal="auto"):
        import torch
        lib = _lib.load()
        if levels is None:
            levels = [(N, J, I, nfields)]
        self.levels = [tuple(int(v) for v in lv) for lv in levels]
        self.grid_kind = grid
        self.form = form
        self.dtype = torch.float64 if form == "fp64" else torch.float32
        opts = _lib.Options(_lib.GRID[grid], _lib.FORM[form], int(autotune), int(use_graph), int(reduced), int(otf),
                            _lib.ZONAL[zonal])
        h = ctypes.c_void_p()
        n = len(self.levels)
        arr = lambda k: (ctypes.c_int * n)(*[lv[k] for lv in self.levels])  # noqa: E731
        _lib.check(lib.sht_plan_multi(n, arr(0), arr(1), arr(2), arr(3), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.grid_elems = self._query(_lib.Q_GRID_ELEMS, ctypes.c_size_t)
        self.spec_elems = self._query(_lib.Q_SPEC_ELEMS, ctypes.c_size_t)
        self.legendre_flops = self._query(_lib.Q_LEGENDRE_FLOPS, ctypes.c_double)
        self.legendre_flops_kept = self._query(_lib.Q_LEGENDRE_FLOPS_KEPT, ctypes.c_double)
        # multi-level plans: (analysis, synthesis) zonal stage in one launch
        zo = self._query(_lib.Q_ZONAL_ONE_LAUNCH, ctypes.c_int)
        self.zonal_one_launch = (bool(zo & 1), bool(zo & 2))
        self.exact = bool(self._query(_lib.Q_EXACT, ctypes.c_int))
        self.workspace_bytes = self._query(_lib.Q_WORKSPACE_BYTES, ctypes.c_size_t)
        self.table_bytes = self._query(_lib.Q_TABLE_BYTES, ctypes.c_size_t)
        self.grid_offsets = [self._query(_lib.Q_GRID_OFFSET + k, ctypes.c_size_t) for k in range(n)]
        self.spec_offsets = [self._query(_lib.Q_SPEC_OFFSET + k, ctypes.c_size_t) for k in range(n)]

    # single-level conveniences
    @property
    def N(self):
        return self.levels[0][0]

    @property
    def ncoef(self):
        N = self.levels[0][0]
        return (N + 1) * (N + 2) // 2

    @property
    def grid_shape(self):
        N, J, I, F = self.levels[0]
        return (F, J, I) if len(self.levels) == 1 else (self.grid_elems,)

    @property
    def spec_shape(self):
        N, J, I, F = self.levels[0]
        return (F, (N + 1) * (N + 2) // 2, 2) if len(self.levels) == 1 else (self.spec_elems,)

    def _query(self, key, ctype):
        v = ctype()
        _lib.check(self._lib.sht_plan_query(self._h, key, ctypes.byref(v)))
        return v.value

    def _check(self, t, elems, name):
        import torch
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise ValueError("%s must be a CUDA (HIP) tensor" % name)
        if t.dtype != self.dtype:
            raise ValueError("%s must be %s for form %s" % (name, self.dtype, self.form))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if t.numel() != elems:
            raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), elems))

    def _run(self, fn, x, in_elems, out_elems, out_shape, out, names):
        import torch
        self._check(x, in_elems, names[0])
        if out is None:
            out = torch.empty(out_shape, dtype=self.dtype, device=x.device)
        self._check(out, out_elems, names[1])
        stream = torch.cuda.current_stream(x.device).cuda_stream
        _lib.check(fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                      ctypes.c_void_p(stream)))
        return out

    def forward(self, grid, out=None):
        """Analysis grid -> spec."""
        return self._run(self._lib.sht_forward, grid, self.grid_elems, self.spec_elems,
                         self.spec_shape, out, ("grid", "spec"))

    def forward_noalloc(self, grid, out=None):
        """Analysis grid -> spec through sht_forward_noalloc: the workspace is
        the library's static device array instead of the plan's (the plan's
        workspace must fit in 64 MiB); pass out= to allocate nothing."""
        return self._run(self._lib.sht_forward_noalloc, grid, self.grid_elems, self.spec_elems,
                         self.spec_shape, out, ("grid", "spec"))

    def inverse(self, spec, out=None):
        """Synthesis spec -> grid."""
        return self._run(self._lib.sht_inverse, spec, self.spec_elems, self.grid_elems,
                         self.grid_shape, out, ("spec", "grid"))

    def forward_adjoint(self, spec_bar, out=None):
        return self._run(self._lib.sht_forward_adjoint, spec_bar, self.spec_elems, self.grid_elems,
                         self.grid_shape, out, ("spec_bar", "grid_bar"))

    def inverse_adjoint(self, grid_bar, out=None):
        return self._run(self._lib.sht_inverse_adjoint, grid_bar, self.grid_elems, self.spec_elems,
                         self.spec_shape, out, ("grid_bar", "spec_bar"))

    def tables(self):
        """(mu, w, alf) of level 0 as built on the host in FP64."""
        N, J, _, _ = self.levels[0]
        nc = (N + 1) * (N + 2) // 2
        mu, w, alf = np.zeros(J), np.zeros(J), np.zeros((nc, (J + 1) // 2))
        dp = ctypes.POINTER(ctypes.c_double)
        _lib.check(self._lib.sht_plan_tables(self._h, mu.ctypes.data_as(dp), w.ctypes.data_as(dp),
                                             alf.ctypes.data_as(dp)))
        return mu, w, alf

    STAGES = ("zonal_analysis", "legendre_analysis", "legendre_synthesis", "zonal_synthesis")

    def profile(self, enable=True):
        """Time every kernel launch with events on the caller's stream."""
        _lib.check(self._lib.sht_plan_profile(self._h, int(enable)))

    def profile_read(self):
        """{stage: (total_ms, launches)} since the last read; waits for the GPU."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int * 4)()
        _lib.check(self._lib.sht_plan_profile_read(self._h, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.STAGES)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(self._lib.sht_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
