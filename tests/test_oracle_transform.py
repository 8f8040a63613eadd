"""Pins of the oracle's Legendre functions and transform pair against
independent routes: closed forms, scipy/mpmath Legendre functions, numpy's
FFT and Gauss-Legendre rule, analytic symmetries and dense transposes."""

import math

import mpmath
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy import special

import oracle as O
from paper_1711_11296_amd import inputs

KINDS = O.GRID_KINDS


def _norm_alf_scipy(n, m, mu):
    """P~_n^m from scipy's associated Legendre function: remove the
    Condon-Shortley phase and normalise to unit L2 norm on [-1, 1]."""
    c = math.sqrt((2 * n + 1) / 2.0 * math.exp(math.lgamma(n - m + 1) - math.lgamma(n + m + 1)))
    return (-1) ** m * c * special.lpmv(m, n, mu)


# --------------------------------------------------------------------------
# associated Legendre functions
# --------------------------------------------------------------------------

def test_alf_low_degree_closed_forms():
    mu = np.linspace(-1, 1, 41)
    s = np.sqrt(1 - mu ** 2)
    P0 = O.alf_m(3, 0, mu, s)
    P1 = O.alf_m(3, 1, mu, s)
    P2 = O.alf_m(3, 2, mu, s)
    assert np.allclose(P0[0], 1 / math.sqrt(2), atol=1e-15)
    assert np.allclose(P0[1], math.sqrt(1.5) * mu, atol=1e-15)
    assert np.allclose(P0[2], math.sqrt(5 / 8) * (3 * mu ** 2 - 1), atol=1e-15)
    assert np.allclose(P1[0], math.sqrt(3) / 2 * s, atol=1e-15)
    assert np.allclose(P1[1], math.sqrt(15) / 2 * mu * s, atol=1e-15)
    assert np.allclose(P2[0], math.sqrt(15) / 4 * s ** 2, atol=1e-15)


def test_alf_vs_scipy_lpmv():
    N = 50
    mu = np.cos(np.linspace(0.01, math.pi - 0.01, 37))
    s = np.sqrt(1 - mu ** 2)
    for m in range(0, N + 1, 7):
        P = O.alf_m(N, m, mu, s)
        for n in range(m, N + 1):
            ref = _norm_alf_scipy(n, m, mu)
            assert np.allclose(P[n - m], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max() + 1e-300)


@pytest.mark.parametrize("n,m,th", [(959, 0, 0.0016), (959, 0, 1.1), (959, 300, 0.9),
                                    (700, 600, 1.5), (500, 17, 2.9), (959, 959, 1.2)])
def test_alf_vs_mpmath_high_degree(n, m, th):
    mpmath.mp.dps = 50
    mu = math.cos(th)
    s = math.sin(th)
    ref = mpmath.legenp(n, m, mpmath.mpf(mu)) * (-1) ** m
    ref *= mpmath.sqrt((2 * n + 1) / mpmath.mpf(2) * mpmath.factorial(n - m) / mpmath.factorial(n + m))
    P = O.alf_m(n, m, np.array([mu]), np.array([s]))[n - m, 0]
    assert abs(P - float(ref)) <= 1e-9 + 1e-10 * abs(float(ref))


@pytest.mark.parametrize("n,m,th,below", [(2047, 747, 12 * math.pi / 100, True), (2047, 760, 0.39, True),
                                          (2047, 900, 0.5 * math.pi, False)])
def test_alf_sectoral_start_below_double_range(n, m, th, below):
    """Orders whose sectoral start sin^m(theta) lies below the double range
    (0.368^747 ~ 1e-324) while P~_n^m grows back to O(1) by degree n: the
    values still match mpmath (the recurrence carries its exponent, as the
    paper's quadruple precision does)."""
    mpmath.mp.dps = 60
    mu = math.cos(th)
    s = math.sin(th)
    assert (m * math.log10(1.0 / s) > 308) == below
    ref = mpmath.legenp(n, m, mpmath.mpf(mu)) * (-1) ** m
    ref *= mpmath.sqrt((2 * n + 1) / mpmath.mpf(2) * mpmath.factorial(n - m) / mpmath.factorial(n + m))
    P = O.alf_m(n, m, np.array([mu]), np.array([s]))
    assert abs(P[n - m, 0] - float(ref)) <= 1e-9 + 1e-10 * abs(float(ref)), (P[n - m, 0], float(ref))
    # the same degrees at the same latitude: every entry finite, the sectoral
    # one rounded to 0 where it is below the double range
    assert np.all(np.isfinite(P))


def test_alf_orthonormal_under_gauss_rule():
    N = 30
    x, w = npleg.leggauss(40)
    for m in (0, 1, 5, 17, 30):
        P = O.alf_m(N, m, x, np.sqrt(1 - x ** 2))
        G = (P * w) @ P.T
        assert np.abs(G - np.eye(N - m + 1)).max() < 1e-13


def test_alf_parity():
    N = 40
    mu = np.linspace(0.05, 0.95, 11)
    s = np.sqrt(1 - mu ** 2)
    for m in (0, 3, 20):
        Pp = O.alf_m(N, m, mu, s)
        Pm = O.alf_m(N, m, -mu, s)
        sign = (-1.0) ** np.arange(N - m + 1)
        assert np.allclose(Pm, Pp * sign[:, None], rtol=1e-13, atol=1e-14)


# --------------------------------------------------------------------------
# quadrature + ALFs: numerical orthonormality (Sec. 4.1, Fig. 1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", KINDS)
def test_orthonormality_exact_when_cubic(kind):
    for N, J in ((21, 43), (63, 127)):
        en, eo = O.orthonormality_errors(N, J, kind)
        assert np.nanmax(en) < 1e-13 and np.nanmax(eo) < 1e-13


@pytest.mark.parametrize("kind", KINDS)
def test_orthonormality_breaks_below_cubic(kind):
    """J < 2N+1: rounding-level for n <= (J-1)/2, visibly larger beyond."""
    N, J = 21, 33
    en, _ = O.orthonormality_errors(N, J, kind)
    lim = (J - 1) // 2
    assert np.nanmax(en[:, :lim + 1]) < 1e-13
    assert np.nanmax(en[:, lim + 1:]) > 1e-6
    # as in Fig. 1, the largest errors are at small m and large n
    m, n = np.unravel_index(np.nanargmax(en), en.shape)
    assert m == 0 and n == N


# --------------------------------------------------------------------------
# zonal step against numpy's FFT
# --------------------------------------------------------------------------

def test_zonal_analysis_is_rfft_over_I():
    x = inputs.random_grid(3, 5, 48, seed=3)
    N = 20
    X = O.zonal_analysis(x, N)
    ref = np.fft.rfft(x, axis=-1)[..., :N + 1] / 48
    assert np.abs(X - ref).max() < 1e-15


def test_zonal_synthesis_is_hermitian_irfft():
    rng = np.random.default_rng(4)
    N, I = 20, 48
    X = rng.standard_normal((2, 5, N + 1)) + 1j * rng.standard_normal((2, 5, N + 1))
    full = np.zeros((2, 5, I // 2 + 1), dtype=complex)
    full[..., :N + 1] = X
    full[..., 0] = X[..., 0].real
    ref = np.fft.irfft(full, n=I, axis=-1) * I
    assert np.abs(O.zonal_synthesis(X, I) - ref).max() < 1e-13


# --------------------------------------------------------------------------
# the transform pair
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("N,J,I", [(21, 43, 64), (21, 45, 64), (10, 21, 21), (5, 11, 16)])
def test_round_trip_identity(kind, N, J, I):
    a = inputs.random_spectra(N, 2, seed=0, profile="inv1")
    g = O.inverse(a, N, J, I, kind)
    b = O.forward(g, N, kind)
    assert np.linalg.norm(b - a) / np.linalg.norm(a) < 1e-13


@pytest.mark.parametrize("kind", KINDS)
def test_aliasing_visible_below_2N_plus_1(kind):
    N, I = 21, 64
    a = inputs.random_spectra(N, 1, seed=0, profile="inv1")
    errs = {}
    for J in (33, 41, 42, 43, 44):
        g = O.inverse(a, N, J, I, kind)
        errs[J] = np.linalg.norm(O.forward(g, N, kind) - a) / np.linalg.norm(a)
    assert errs[43] < 1e-13 and errs[44] < 1e-13
    assert errs[42] > 1e-7 and errs[41] > 1e-7 and errs[33] > 1e-5


@pytest.mark.parametrize("kind", KINDS)
def test_quadratic_term_alias_free_on_quadratic_grid(kind):
    """Sec. 3.1 (eq. cc-condition) and Sec. 4.2: the degree-N spectrum of
    the product of two fields band-limited at N needs integrals of degree
    3N.  Gauss-Legendre with J >= (3N+1)/2 nodes integrates those exactly
    (textbook exactness 2J-1), so it fixes the alias-free spectrum; the CC
    grid with J = 3N+1 must reproduce it to rounding, the linear grid
    J = 2N+1 must not, and neither may a Gaussian grid one node short."""
    N, I = 21, 64                                 # I >= 3N+1: no zonal aliasing
    U = inputs.random_spectra(N, 1, seed=1, profile="uniform13")
    V = inputs.random_spectra(N, 1, seed=2, profile="uniform13")

    def uv(k, J):
        return O.forward(O.inverse(U, N, J, I, k) * O.inverse(V, N, J, I, k), N, k)

    def rel(x, y):
        return np.linalg.norm(x - y) / np.linalg.norm(y)

    ref = uv("gauss", (3 * N + 2) // 2)
    assert rel(uv(kind, 3 * N + 1), ref) < 1e-13
    assert rel(uv(kind, 2 * N + 1), ref) > 1e-4
    assert rel(uv("gauss", (3 * N + 2) // 2 - 1), ref) > 1e-4


def _poly_field(coef, mu, lam, sint):
    """Polynomial of total degree <= 3 in (x, y, z) on the sphere
    (z = mu = sin(latitude)), evaluated pointwise."""
    x = sint[:, None] * np.cos(lam)[None, :]
    y = sint[:, None] * np.sin(lam)[None, :]
    z = mu[:, None] * np.ones_like(lam)[None, :]
    out = np.zeros_like(x)
    k = 0
    for p in range(4):
        for q in range(4 - p):
            for r in range(4 - p - q):
                out += coef[k] * x ** p * y ** q * z ** r
                k += 1
    return out


@pytest.mark.parametrize("kind,J", [("cc_poles", 17), ("fejer2", 17), ("fejer2", 21),
                                    ("cc_poles", 13)])
def test_brute_force_vs_gauss_legendre(kind, J):
    """A degree-3 polynomial field is band-limited to n <= 3.  Its spectrum
    from the oracle (CC rule) must equal the one from an independent
    Gauss-Legendre transform built here from numpy's rule, numpy's FFT and
    scipy's Legendre functions."""
    N = 8
    I = 32
    rng = np.random.default_rng(11)
    coef = rng.standard_normal(20)
    lam = 2 * np.pi * np.arange(I) / I
    _, mu, sint = O.nodes(J, kind)
    spec = O.forward(_poly_field(coef, mu, lam, sint)[None], N, kind)[0]

    xg, wg = npleg.leggauss(N + 1)
    gg = _poly_field(coef, xg, lam, np.sqrt(1 - xg ** 2))
    Xg = np.fft.rfft(gg, axis=-1) / I
    ref = np.zeros_like(spec)
    for m in range(N + 1):
        for n in range(m, N + 1):
            v = np.sum(wg * _norm_alf_scipy(n, m, xg) * Xg[:, m])
            ref[O.spec_index(N, m, n)] = (v.real, v.imag if m else 0.0)
    assert np.abs(spec - ref).max() < 1e-13
    # and it really is band-limited to 3
    deg = inputs.degrees(N)
    assert np.abs(spec[deg > 3]).max() < 1e-13
    assert np.abs(spec[deg <= 3]).max() > 1e-2


@pytest.mark.parametrize("kind", KINDS)
def test_pure_harmonic_maps_to_unit_vector(kind):
    N, J, I = 12, 25, 32
    _, mu, _ = O.nodes(J, kind)
    lam = 2 * np.pi * np.arange(I) / I
    for (n, m, part) in [(0, 0, 0), (7, 0, 0), (5, 3, 0), (9, 4, 1), (12, 12, 1)]:
        P = _norm_alf_scipy(n, m, mu)
        if m == 0:
            g = P[:, None] * np.ones(I)[None, :]
        elif part == 0:
            g = 2 * P[:, None] * np.cos(m * lam)[None, :]
        else:
            g = -2 * P[:, None] * np.sin(m * lam)[None, :]
        spec = O.forward(g[None], N, kind)[0]
        ref = np.zeros_like(spec)
        ref[O.spec_index(N, m, n), part] = 1.0
        assert np.abs(spec - ref).max() < 1e-13


@pytest.mark.parametrize("kind", KINDS)
def test_meridional_flip(kind):
    """App. B: flipping the grid north-south multiplies a_n^m by (-1)^(n-m)."""
    N, J, I = 21, 43, 64
    g = inputs.random_grid(2, J, I, seed=5)
    a = O.forward(g, N, kind)
    b = O.forward(g[:, ::-1, :], N, kind)
    sign = (-1.0) ** (inputs.degrees(N) - inputs.orders(N))
    assert np.abs(b - a * sign[None, :, None]).max() < 1e-13


@pytest.mark.parametrize("kind", KINDS)
def test_longitude_shift(kind):
    N, J, I, k = 21, 43, 64, 5
    g = inputs.random_grid(1, J, I, seed=6)
    a = O.forward(g, N, kind)
    b = O.forward(np.roll(g, -k, axis=-1), N, kind)
    ph = np.exp(2j * np.pi * inputs.orders(N) * k / I)
    ac = (a[..., 0] + 1j * a[..., 1]) * ph[None]
    ac[:, inputs.orders(N) == 0] = ac[:, inputs.orders(N) == 0].real
    assert np.abs(b[..., 0] - ac.real).max() < 1e-13
    assert np.abs(b[..., 1] - ac.imag).max() < 1e-13


# --------------------------------------------------------------------------
# adjoints
# --------------------------------------------------------------------------

def _dense(fn, shape_in):
    size = int(np.prod(shape_in))
    cols = []
    for k in range(size):
        e = np.zeros(size)
        e[k] = 1.0
        cols.append(fn(e.reshape(shape_in)).ravel())
    return np.array(cols).T


@pytest.mark.parametrize("kind", KINDS)
def test_adjoints_are_dense_transposes(kind):
    N, J, I = 5, 11, 16
    nc = O.ncoef(N)
    Af = _dense(lambda g: O.forward(g[None], N, kind), (J, I))
    Afa = _dense(lambda s: O.forward_adjoint(s[None], N, J, I, kind), (nc, 2))
    assert np.abs(Afa - Af.T).max() < 1e-15
    Ai = _dense(lambda s: O.inverse(s[None], N, J, I, kind), (nc, 2))
    Aia = _dense(lambda g: O.inverse_adjoint(g[None], N, kind), (J, I))
    assert np.abs(Aia - Ai.T).max() < 1e-14
    # forward is a left inverse of inverse on the stored degrees of freedom
    # (Im a_n^0 is not a degree of freedom)
    P = Af @ Ai
    E = np.eye(2 * nc)
    for m0 in range(N + 1):
        E[2 * O.spec_index(N, 0, m0) + 1, 2 * O.spec_index(N, 0, m0) + 1] = 0.0
    assert np.abs(P - E).max() < 1e-14


@pytest.mark.parametrize("kind", KINDS)
def test_adjoint_dot_products(kind):
    N, J, I = 21, 43, 64
    g = inputs.random_grid(2, J, I, seed=7)
    s = inputs.random_spectra(N, 2, seed=8, profile="inv1")
    lhs = np.sum(O.forward(g, N, kind) * s)
    rhs = np.sum(g * O.forward_adjoint(s, N, J, I, kind))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs) + 1e-15
    lhs = np.sum(O.inverse(s, N, J, I, kind) * g)
    rhs = np.sum(s * O.inverse_adjoint(g, N, kind))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs) + 1e-15


# --------------------------------------------------------------------------
# nesting (Sec. 3.2): a coarse grid injected from a fine one
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind,Jc,Jf,step,off", [
    ("cc_poles", 17, 33, 2, 0), ("fejer2", 17, 35, 2, 1), ("fejer2", 17, 53, 3, 2)])
def test_injection_equals_truncation(kind, Jc, Jf, step, off):
    Nc, Ic, If = 8, 24, 48
    Nf = (Jf - 1) // 2
    a = inputs.random_spectra(Nc, 1, seed=9, profile="k3")
    g_f = O.inverse(a, Nc, Jf, If, kind)
    g_c = g_f[:, off::step, ::If // Ic]
    assert g_c.shape[1] == Jc
    b = O.forward(g_c, Nc, kind)
    assert np.abs(b - a).max() < 1e-13 * np.abs(a).max()
    # the fine analysis of the same field is a zero-padded copy
    bf = O.forward(g_f, Nf, kind)
    deg_f = inputs.degrees(Nf)
    ordf = inputs.orders(Nf)
    for m in range(Nc + 1):
        for n in range(m, Nf + 1):
            v = bf[0, O.spec_index(Nf, m, n)]
            if n <= Nc:
                assert np.abs(v - a[0, O.spec_index(Nc, m, n)]).max() < 1e-13
            else:
                assert np.abs(v).max() < 1e-13
    assert np.abs(bf[0, ordf > Nc]).max() < 1e-13 and deg_f.size == bf.shape[1]


# --------------------------------------------------------------------------
# sampled evaluation used at large sizes agrees with the full transforms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", KINDS)
def test_sampled_forms_match_full(kind):
    N, J, I = 21, 43, 64
    g = inputs.random_grid(2, J, I, seed=12)
    a = O.forward(g, N, kind)
    for m in (0, 1, 10, 21):
        ns = list(range(m, N + 1, 3))
        v = O.forward_sample(g[1], N, kind, m, ns)
        ref = np.array([a[1, O.spec_index(N, m, n)] for n in ns])
        assert np.abs(v - ref).max() < 1e-15
    s = inputs.random_spectra(N, 2, seed=13, profile="inv1")
    x = O.inverse(s, N, J, I, kind)
    for j in (0, 7, 21, 42):
        assert np.abs(O.inverse_sample_row(s[1], N, J, I, kind, j) - x[1, j]).max() < 1e-14


# --------------------------------------------------------------------------
# transfers between levels (App. C): re-truncation and injection
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind,Jc,Jf,Ic,If", [("cc_poles", 17, 33, 24, 48), ("fejer2", 17, 35, 24, 72),
                                              ("fejer2", 17, 53, 25, 50)])
def test_two_grid_transfers(kind, Jc, Jf, Ic, If):
    """Injection then coarse analysis, and fine analysis then restriction,
    both return the coarse spectrum of a field band-limited at the coarse
    truncation (Sec. 3.2, App. C); prolongation then restriction is the
    identity and prolongation pads with zeros."""
    Nc = 8
    Nf = (Jf - 1) // 2
    a = inputs.random_spectra(Nc, 2, seed=21, profile="k3")
    g_f = O.inverse(a, Nc, Jf, If, kind)
    g_c = O.inject(g_f, Jc, Ic, kind)
    assert g_c.shape == (2, Jc, Ic)
    assert np.abs(O.forward(g_c, Nc, kind) - a).max() < 1e-13 * np.abs(a).max()
    b = O.retruncate(O.forward(g_f, Nf, kind), Nf, Nc)
    assert np.abs(b - a).max() < 1e-13 * np.abs(a).max()
    up = O.retruncate(a, Nc, Nf)
    assert np.array_equal(O.retruncate(up, Nf, Nc), a)
    assert np.array_equal(O.retruncate(a, Nc, Nc), a)
    ordf = inputs.orders(Nf)
    deg_f = inputs.degrees(Nf)
    assert np.all(up[:, deg_f > Nc] == 0)
    assert ordf.size == up.shape[1]


@pytest.mark.parametrize("kind,Jc,Jf", [("cc_poles", 9, 33), ("fejer2", 15, 31), ("fejer2", 9, 29)])
def test_injection_rows_are_the_nested_nodes(kind, Jc, Jf):
    """Injected rows carry exactly the coarse grid's nodes: a grid holding
    mu_j of the fine grid injects to mu_j of the coarse one, bit for bit."""
    _, muf, _ = O.nodes(Jf, kind)
    _, muc, _ = O.nodes(Jc, kind)
    g = np.repeat(muf[None, :, None], 6, axis=2)
    assert np.array_equal(O.inject(g, Jc, 3, kind)[0, :, 0], muc)
    with pytest.raises(ValueError):
        O.inject(g, Jc + 1, 3, kind)
    with pytest.raises(ValueError):
        O.inject(g, Jc, 3, "fejer1")


def _xyz(J, I, kind):
    _, mu, sint = O.nodes(J, kind)
    lam = 2.0 * np.pi * np.arange(I) / I
    x = sint[:, None] * np.cos(lam)[None, :]
    y = sint[:, None] * np.sin(lam)[None, :]
    z = mu[:, None] * np.ones(I)[None, :]
    return x, y, z


@pytest.mark.parametrize("kind", KINDS)
def test_laplacian_closed_forms(kind):
    """On the unit sphere a harmonic homogeneous polynomial of degree l is an
    eigenfunction of the Laplacian with eigenvalue -l(l+1): z -> -2 z,
    xy -> -6 xy, x^3 - 3 x y^2 -> -12 (x^3 - 3 x y^2); z^2 = 1/3 + (z^2 - 1/3)
    gives 2 - 6 z^2; constants give 0.  The pseudo-spectral Laplacian
    (analysis, spectral factor, synthesis) reproduces each, and the factor
    scales with 1/radius^2."""
    N, J, I = 5, 11, 16
    x, y, z = _xyz(J, I, kind)
    cases = [(z, -2 * z), (x * y, -6 * x * y), (x ** 3 - 3 * x * y ** 2, -12 * (x ** 3 - 3 * x * y ** 2)),
             (z ** 2, 2 - 6 * z ** 2), (np.full_like(z, 3.0), np.zeros_like(z))]
    for g, lap in cases:
        out = O.inverse(O.laplacian(O.forward(g[None], N, kind), N), N, J, I, kind)[0]
        assert np.max(np.abs(out - lap)) < 1e-13
        out4 = O.inverse(O.laplacian(O.forward(g[None], N, kind), N, scale=0.25), N, J, I, kind)[0]
        assert np.max(np.abs(out4 - 0.25 * lap)) < 1e-13


@pytest.mark.parametrize("kind", KINDS)
def test_helmholtz_residual_of_manufactured_solution(kind):
    """App. C eq. elliptic with L X = kappa lap(X): for X = xy + z and a
    variable kappa = 1 + x/2, the right-hand side F = X - alpha kappa
    (-6 xy - 2 z) written out by hand makes the residual vanish; a wrong
    sign of alpha, kappa on the wrong side or a dropped term would not."""
    N, J, I = 5, 11, 16
    x, y, z = _xyz(J, I, kind)
    X = x * y + z
    kappa = 1.0 + 0.5 * x
    alpha = 0.3
    F = X - alpha * kappa * (-6 * x * y - 2 * z)
    R = O.helmholtz_residual(X[None], kappa, F[None], alpha, N, kind)
    assert np.max(np.abs(R)) < 1e-13
    # and the residual of another field is the hand-computed one
    X2 = z ** 2
    R2 = O.helmholtz_residual(X2[None], kappa, F[None], alpha, N, kind)
    assert np.max(np.abs(R2[0] - (X2 - alpha * kappa * (2 - 6 * z ** 2) - F))) < 1e-13
