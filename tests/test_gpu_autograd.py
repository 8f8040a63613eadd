"""Adjoint transforms and autograd through the C ABI: dot-product tests,
gradients of a quadratic loss against the oracle's transposes, central
finite differences and torch.autograd.gradcheck in the FP64 form."""

import numpy as np
import pytest

import oracle as O
from paper_1711_11296_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _t(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev(), dt)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def _plan(N, J, I, F, kind, form):
    from paper_1711_11296_amd import Plan
    return Plan(N, J, I, F, grid=kind, form=form)


def _dot_bound(u, v, tol):
    """Bound for |<A x, y> - <x, A^T y>| with u = A x, v = y: rounding moves
    each side by at most about tol * |u| |v| (Cauchy-Schwarz); the inner
    product itself can be much smaller than that through cancellation."""
    return tol * torch.linalg.vector_norm(u.double()).item() * torch.linalg.vector_norm(v.double()).item()


@pytest.mark.parametrize("form,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
@pytest.mark.parametrize("kind", O.GRID_KINDS)
def test_dot_product(form, tol, kind):
    N, J, I, F = 63, 127, 192, 5
    dt = torch.float64 if form == "fp64" else torch.float32
    p = _plan(N, J, I, F, kind, form)
    x = _t(inputs.random_grid(F, J, I, seed=1), dt)
    y = _t(inputs.random_spectra(N, F, seed=2, profile="inv1"), dt)
    fx = p.forward(x)
    lhs = torch.sum(fx.double() * y.double()).item()
    rhs = torch.sum(x.double() * p.forward_adjoint(y).double()).item()
    assert abs(lhs - rhs) <= _dot_bound(fx, y, tol)
    iy = p.inverse(y)
    lhs = torch.sum(iy.double() * x.double()).item()
    rhs = torch.sum(y.double() * p.inverse_adjoint(x).double()).item()
    assert abs(lhs - rhs) <= _dot_bound(iy, x, tol)
    p.close()


@pytest.mark.parametrize("form,tol", [("fp64", 1e-12), ("fp32", 1e-6), ("bf16x6", 1e-6)])
@pytest.mark.parametrize("kind", O.GRID_KINDS)
def test_autograd_matches_oracle_transpose(form, tol, kind):
    from paper_1711_11296_amd import sht_forward, sht_inverse
    N, J, I, F = 40, 81, 96, 3
    dt = torch.float64 if form == "fp64" else torch.float32
    p = _plan(N, J, I, F, kind, form)
    g = _t(inputs.random_grid(F, J, I, seed=3), dt).requires_grad_(True)
    cs = inputs.loss_weights((F, O.ncoef(N), 2), seed=1)
    s = sht_forward(g, p)
    loss = torch.sum(_t(cs, dt) * s * s)
    loss.backward()
    cot = 2.0 * cs * _np(s)
    ref = O.forward_adjoint(cot, N, J, I, kind)
    assert np.linalg.norm(_np(g.grad) - ref) / np.linalg.norm(ref) < tol

    a = _t(inputs.random_spectra(N, F, seed=4, profile="inv1"), dt).requires_grad_(True)
    cg = inputs.loss_weights((F, J, I), seed=1)
    x = sht_inverse(a, p)
    loss = torch.sum(_t(cg, dt) * x * x)
    loss.backward()
    ref = O.inverse_adjoint(2.0 * cg * _np(x), N, kind)
    assert np.linalg.norm(_np(a.grad) - ref) / np.linalg.norm(ref) < tol
    assert np.all(_np(a.grad)[:, inputs.orders(N) == 0, 1] == 0.0)
    p.close()


def test_central_finite_differences_fp64():
    """The loss is quadratic, so a central difference has no truncation
    error: it must match the directional derivative to rounding."""
    from paper_1711_11296_amd import sht_forward, sht_inverse
    N, J, I, F = 31, 63, 64, 2
    p = _plan(N, J, I, F, "fejer2", "fp64")
    c = _t(inputs.loss_weights((F, O.ncoef(N), 2), seed=1), torch.float64)
    cg = _t(inputs.loss_weights((F, J, I), seed=1), torch.float64)

    def L1(g):
        s = sht_forward(g, p)
        return torch.sum(c * s * s)

    def L2(a):
        x = sht_inverse(a, p)
        return torch.sum(cg * x * x)

    rng = np.random.default_rng(7)
    for L, x0 in ((L1, _t(inputs.random_grid(F, J, I, seed=5), torch.float64)),
                  (L2, _t(inputs.random_spectra(N, F, seed=6, profile="inv1"), torch.float64))):
        x = x0.clone().requires_grad_(True)
        L(x).backward()
        for _ in range(4):
            d = _t(rng.standard_normal(tuple(x0.shape)), torch.float64)
            h = 1e-3
            with torch.no_grad():
                fd = (L(x0 + h * d) - L(x0 - h * d)).item() / (2 * h)
            an = torch.sum(x.grad * d).item()
            if L is L2:   # Im of m = 0 is ignored by the synthesis
                an = torch.sum(x.grad * d).item()
            assert abs(fd - an) <= 1e-9 * max(1.0, abs(an)), (fd, an)
    p.close()


def test_gradcheck_tiny():
    from paper_1711_11296_amd import sht_forward, sht_inverse
    N, J, I, F = 4, 9, 12, 2
    for kind in O.GRID_KINDS:
        p = _plan(N, J, I, F, kind, "fp64")
        g = _t(inputs.random_grid(F, J, I, seed=8), torch.float64).requires_grad_(True)
        assert torch.autograd.gradcheck(lambda x: sht_forward(x, p), (g,), eps=1e-6, atol=1e-9)
        a = _t(inputs.random_spectra(N, F, seed=9, profile="inv1"), torch.float64)
        a.requires_grad_(True)
        # Im of m = 0 does not enter the synthesis: its column of the
        # Jacobian is zero both numerically and analytically
        assert torch.autograd.gradcheck(lambda x: sht_inverse(x, p), (a,), eps=1e-6, atol=1e-9)
        p.close()


def test_t959_adjoint_autograd_fp32():
    """N=959, J=1919, I=2880, 64 fields, FP32: gradients of a random
    quadratic loss through forward and inverse; field 0 checked against the
    oracle's transpose (fields are independent), and a dot-product test on
    the whole batch."""
    from paper_1711_11296_amd import sht_forward, sht_inverse
    N, J, I, F = 959, 1919, 2880, 64
    p = _plan(N, J, I, F, "cc_poles", "fp32")
    a0 = _t(inputs.random_spectra(N, F, seed=0, profile="k3"), torch.float32)
    a = a0.clone().requires_grad_(True)
    cg = inputs.loss_weights((1, J, I), seed=1)
    x = sht_inverse(a, p)
    w = torch.ones_like(x)
    w[0] = _t(cg[0], torch.float32)
    loss = torch.sum(w * x * x)
    loss.backward()
    ref = O.inverse_adjoint(2.0 * cg * _np(x[0:1]), N, "cc_poles")
    err = np.linalg.norm(_np(a.grad[0:1]) - ref) / np.linalg.norm(ref)
    assert err < 1e-6, err
    # batch-wide dot products (on the device, in float64 accumulation)
    y = torch.randn(F, J, I, device=_dev(), dtype=torch.float32)
    ia = p.inverse(a0)
    lhs = torch.sum(ia.double() * y.double()).item()
    rhs = torch.sum(a0.double() * p.inverse_adjoint(y).double()).item()
    assert abs(lhs - rhs) <= _dot_bound(ia, y, 2e-6)
    s = p.forward(y)
    lhs = torch.sum(s.double() * a0.double()).item()
    rhs = torch.sum(y.double() * p.forward_adjoint(a0).double()).item()
    assert abs(lhs - rhs) <= _dot_bound(s, a0, 2e-6)
    p.close()
