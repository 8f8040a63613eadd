"""The aliasing experiment of Sec. 4.2 on the GPU.

Three random fields U, V, W band-limited at N_trunc are synthesised on a
grid, their quadratic term UV and cubic term UVW are formed pointwise, and
both are analysed back to spectra truncated at N_trunc.  Done once on a test
grid and once on a reference grid fine enough to be alias-free, the two
results give the normalised aliasing error of every coefficient (n, m):
|X_test - X_ref| / |X_ref| (complex moduli).  Every transform, re-truncation
and product runs in libsht.so; only the final per-coefficient ratio is taken
on the host.
"""

import numpy as np

from . import inputs
from .plan import Plan
from .transfer import grid_product, spec_retruncate


class NonlinearTerms:
    """Spectra of UV and UVW computed on one grid (N, J, I, grid).

    Holds a three-field plan.  Called with device spectra U, V, W
    [1, (Nt+1)(Nt+2)/2, 2] band-limited at Nt <= N, it zero-pads them to
    truncation N (spectral prolongation), synthesises, multiplies pointwise,
    analyses at truncation N and cuts back to Nt; the result is a device
    tensor [2, (Nt+1)(Nt+2)/2, 2]: row 0 UV, row 1 UVW.  Runs on the current
    stream and does not synchronise.
    """

    def __init__(self, N, J, I, grid, form="fp64", otf=False):
        self.N = N
        self.plan = Plan(N, J, I, 3, grid=grid, form=form, otf=otf)

    def __call__(self, U, V, W):
        import torch
        nc = U.shape[1]
        Nt = int(round((np.sqrt(8 * nc + 1) - 3) / 2))
        if (Nt + 1) * (Nt + 2) // 2 != nc or Nt > self.N:
            raise ValueError("spectra must be triangular with truncation <= %d" % self.N)
        p = self.plan
        g = p.inverse(spec_retruncate(torch.cat([U, V, W]).to(p.dtype), Nt, self.N))
        q = grid_product(g[0], g[1])
        c = grid_product(q, g[2])
        # the plan holds three fields; the third analysed slot is unused
        x = p.forward(torch.stack([q, c, torch.zeros_like(q)]))
        return spec_retruncate(x[:2].contiguous(), self.N, Nt)

    def close(self):
        self.plan.close()


def nonlinear_spectra(U, V, W, N, J, I, grid, form="fp64", otf=False):
    """One-off NonlinearTerms(N, J, I, grid, form, otf)(U, V, W), synchronised."""
    import torch
    t = NonlinearTerms(N, J, I, grid, form, otf)
    try:
        out = t(U, V, W)
        torch.cuda.current_stream(out.device).synchronize()
    finally:
        t.close()
    return out


def normalised_error(test, ref):
    """|test - ref| / |ref| per coefficient, complex moduli; host arrays
    [F, ncoef, 2] -> [F, ncoef]."""
    t = np.asarray(test, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    return np.hypot(*(t - r).transpose(2, 0, 1)) / np.hypot(*r.transpose(2, 0, 1))


# Grids of the experiment (Sec. 4.2).  The paper gives N and J; the number
# of longitudes is the usual one for each truncation: I = 2J for the linear
# Gaussian grids (I >= 2N+1 for linear terms) and I = 2(J+1) for the cubic
# CC grid (I >= 4N+1, so products of three fields do not alias in longitude).
# Every I is a multiple of N_trunc + 1, which must factor into 2, 3 and 5.
def grids(N_trunc):
    Nref = 3 * N_trunc + 2
    return {
        "reference": (Nref, Nref + 1, 2 * (Nref + 1), "gauss"),
        "gauss_linear": (N_trunc, N_trunc + 1, 2 * (N_trunc + 1), "gauss"),
        "cc_cubic": (N_trunc, 2 * N_trunc + 1, 4 * (N_trunc + 1), "fejer2"),
    }


def experiment(N_trunc=479, seed=0, form="fp64", device="cuda:0", otf=False):
    """Run the experiment at truncation N_trunc with the random spectra of
    Sec. 4.2 (real and imaginary parts uniform on [(n+1)^(-1/3),
    2 (n+1)^(-1/3)]).  Returns a dict: for "gauss_linear" and "cc_cubic",
    the normalised errors [2 (quadratic, cubic), ncoef] against the
    reference grid, plus "spectra" (device tensors of every grid) and the
    input spectra.  otf: FP64 plans generate P~ instead of reading tables."""
    import torch
    U, V, W = [torch.from_numpy(inputs.random_spectra(N_trunc, 1, seed=seed + k, profile="uniform13")).to(device)
               for k in range(3)]
    out = {"U": U, "V": V, "W": W, "spectra": {}}
    for name, (N, J, I, kind) in grids(N_trunc).items():
        out["spectra"][name] = nonlinear_spectra(U, V, W, N, J, I, kind, form, otf)
    ref = out["spectra"]["reference"].cpu().double().numpy()
    for name in ("gauss_linear", "cc_cubic"):
        out[name] = normalised_error(out["spectra"][name].cpu().double().numpy(), ref)
    return out
