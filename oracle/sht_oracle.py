"""Plain FP64 CPU oracle for the spherical-harmonic transform pair on the
Clenshaw-Curtis latitude grids (Hotta & Ujiie, "A nestable, multigrid-friendly
grid on a sphere for global spectral models based on Clenshaw-Curtis
quadrature").

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this module: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU library; the two meet
only through the seeded input generators.

Everything here is written straight from the definitions, slowly and in
float64: a DFT matrix instead of an FFT, the Legendre quadrature summed over
all J latitudes (no equatorial folding), associated Legendre functions from the
plain three-term recurrence.  Each function names the passage it follows.

Conventions (the readings of the paper used throughout):
  * grid kinds: "fejer2" is the paper's pole-free grid, theta_j = j*pi/(J+1),
    j = 1..J (Sec. 3.1, eq. cc-points); "cc_poles" is the classical
    Clenshaw-Curtis grid with the poles, theta_j = j*pi/(J-1), j = 0..J-1;
    "fejer1" is the shifted grid of Sec. 3.3, theta_j = (j - 1/2)*pi/J,
    j = 1..J (eq. fejer1-points); "gauss" is the Gaussian grid of Sec. 2
    (not in GRID_KINDS: a reference for the aliasing workload of Sec. 4.2).
    Row 0 is the one nearest the north pole.
  * P~_n^m is normalised so that its square integrates to 1 over mu in
    [-1, 1] (Sec. 2, eq. pnm-ortho), with no Condon-Shortley phase.
  * spectra are stored for m >= 0 only, as float pairs (re, im), m-major
    triangular: index(m, n) = m*(2N+3-m)/2 + (n-m).  Im a_n^0 is 0 on output
    and ignored on input (real fields).
  * the discrete zonal pair carries 1/I on the analysis side (Sec. 2, the
    discretised zonal integral); synthesis is the Hermitian sum over m.
"""

import math

import numpy as np

GRID_KINDS = ("cc_poles", "fejer2", "fejer1")


# --------------------------------------------------------------------------
# indexing helpers
# --------------------------------------------------------------------------

def ncoef(N):
    """Number of triangular coefficients with 0 <= m <= n <= N (Sec. 2)."""
    return (N + 1) * (N + 2) // 2


def spec_index(N, m, n):
    """Position of (m, n) in the m-major triangular spectral array."""
    return m * (2 * N + 3 - m) // 2 + (n - m)


# --------------------------------------------------------------------------
# nodes and weights
# --------------------------------------------------------------------------

def _sinpi_frac(a, b):
    """sin(pi*a/b) after reducing a/b by their gcd, odd in a bit for bit."""
    if a == 0:
        return 0.0
    g = math.gcd(abs(a), b)
    a //= g
    b //= g
    s = math.sin(math.pi * abs(a) / b)
    return s if a > 0 else -s


def _node_fraction(J, kind, j):
    """theta_j = pi*p/q as the integer pair (p, q)."""
    if kind == "cc_poles":
        if J < 2:
            raise ValueError("cc_poles needs J >= 2")
        return j, J - 1
    if kind == "fejer2":
        if J < 1:
            raise ValueError("fejer2 needs J >= 1")
        return j + 1, J + 1          # Sec. 3.1, eq. cc-points
    if kind == "fejer1":
        if J < 1:
            raise ValueError("fejer1 needs J >= 1")
        return 2 * j + 1, 2 * J      # Sec. 3.3, eq. fejer1-points
    raise ValueError("unknown grid kind %r" % (kind,))


_GAUSS_CACHE = {}


def _gauss_rule(J):
    """Gauss-Legendre nodes mu_j (descending), weights and sin(theta_j) of
    the J-point rule.

    The roots of P_J start from numpy's Gauss-Legendre routine and are
    refined by Newton's method on the three-term recurrence
    k P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2} in 40-digit decimal arithmetic;
    the weight is w = 2 (1 - x^2) / (J P_{J-1}(x))^2.  numpy's own weights
    lose about J * 1e-15 relative accuracy near the poles, too much for a
    1e-12 reference.  sin(theta_j) = sqrt(1 - x^2) is taken from the refined
    root too: near the poles, sqrt((1 - mu)(1 + mu)) of the rounded mu would
    be some 1e-10 off the node's own sine.  Nodes are mirrored so that
    mu_{J-1-j} = -mu_j.
    """
    if J in _GAUSS_CACHE:
        return _GAUSS_CACHE[J]
    import decimal
    ctx = decimal.Context(prec=40)
    D = decimal.Decimal
    x0, _ = np.polynomial.legendre.leggauss(J)
    mu = np.empty(J)
    w = np.empty(J)
    sint = np.empty(J)
    for j in range((J + 1) // 2):
        x = D(float(-x0[j]))                 # north-first: mu_j = -x_j > 0
        for _ in range(4):
            p0, p1 = D(1), x
            for k in range(2, J + 1):
                p0, p1 = p1, ctx.divide(ctx.subtract(ctx.multiply(ctx.multiply(D(2 * k - 1), x), p1),
                                                     ctx.multiply(D(k - 1), p0)), D(k))
            dp = ctx.divide(ctx.multiply(D(J), ctx.subtract(p0, ctx.multiply(x, p1))),
                            ctx.subtract(D(1), ctx.multiply(x, x)))
            x = ctx.subtract(x, ctx.divide(p1, dp))
        p0, p1 = D(1), x
        for k in range(2, J + 1):
            p0, p1 = p1, ctx.divide(ctx.subtract(ctx.multiply(ctx.multiply(D(2 * k - 1), x), p1),
                                                 ctx.multiply(D(k - 1), p0)), D(k))
        if J == 1:
            p0 = D(1)
        wj = ctx.divide(ctx.multiply(D(2), ctx.subtract(D(1), ctx.multiply(x, x))),
                        ctx.multiply(ctx.multiply(D(J), p0), ctx.multiply(D(J), p0)))
        if 2 * j + 1 == J:
            x = D(0)
        mu[j], mu[J - 1 - j] = float(x), -float(x)
        w[j] = w[J - 1 - j] = float(wj)
        sint[j] = sint[J - 1 - j] = float(ctx.sqrt(ctx.subtract(D(1), ctx.multiply(x, x))))
    _GAUSS_CACHE[J] = (mu, w, sint)
    return mu, w, sint


def nodes(J, kind):
    """Colatitudes theta_j, mu_j = cos(theta_j) = sin(phi_j) and sin(theta_j).

    Sec. 3.1 (eq. cc-points) for "fejer2"; Sec. 3.3 (eq. fejer1-points) for
    "fejer1"; the classical grid with the poles for "cc_poles".  mu is evaluated as sin(pi*(q-2p)/(2q)) with the fraction
    reduced by its gcd, so that the equator gets mu = 0 exactly, the mirror
    node gets exactly -mu and nested grids share their common nodes bit for
    bit.
    """
    if kind == "gauss":
        # Gaussian grid (Sec. 2, the comparison grid): the roots of P_J,
        # north first
        mu, _, sint = _gauss_rule(J)
        return np.arctan2(sint, mu), mu, sint
    theta = np.empty(J)
    mu = np.empty(J)
    sint = np.empty(J)
    for j in range(J):
        p, q = _node_fraction(J, kind, j)
        theta[j] = math.pi * p / q
        mu[j] = _sinpi_frac(q - 2 * p, 2 * q)
        sint[j] = _sinpi_frac(min(p, q - p), q)
    return theta, mu, sint


def weights(J, kind):
    """Quadrature weights w_j for integrals over mu in [-1, 1].

    "fejer2": the paper's closed form, Sec. 3.1 eq. cc-wgt (derived in
    App. A): w_j = 4 sin(theta_j)/(J+1) * sum over odd p <= J of
    sin(p theta_j)/p.

    "fejer1": Fejer's first rule, the interpolatory rule on the shifted nodes
    (Sec. 3.3, eq. fejer1-wgt): w_j = (2/J) [1 - 2 sum_{p=1}^{floor(J/2)}
    cos(2 p theta_j)/(4p^2-1)].  The printed form has no factor 2 before the
    sum; without it the rule is not exact even for mu^2 (J = 3), so the
    factor is taken as lost in print.

    "cc_poles": the classical Clenshaw-Curtis rule on n+1 = J points,
    w_k = (c_k/n) [1 - sum_{l=1}^{floor(n/2)} b_l cos(2 l theta_k)/(4l^2-1)]
    with c_0 = c_n = 1, c_k = 2 otherwise and b_l = 1 for l = n/2, 2 otherwise
    (the rule the paper cites from Trefethen 2008 and Waldvogel 2006).
    """
    if kind == "gauss":
        return _gauss_rule(J)[1].copy()
    w = np.empty(J)
    if kind == "fejer2":
        for j in range(J):
            p0, q = _node_fraction(J, kind, j)
            s = 0.0
            for p in range(1, J + 1, 2):
                s += _sinpi_frac((p * p0) % (2 * q), q) / p
            w[j] = 4.0 * _sinpi_frac(p0, q) / (J + 1) * s
        return w
    if kind == "fejer1":
        for j in range(J):
            s = 0.0
            for p in range(1, J // 2 + 1):
                # 2 p theta_j = pi * p (2j+1) / J, reduced mod 2 pi
                r = (p * (2 * j + 1)) % (2 * J)
                s += math.cos(math.pi * r / J) / (4.0 * p * p - 1.0)
            w[j] = 2.0 / J * (1.0 - 2.0 * s)
        return w
    if kind == "cc_poles":
        n = J - 1
        for k in range(J):
            c = 1.0 if (k == 0 or k == n) else 2.0
            s = 0.0
            for l in range(1, n // 2 + 1):
                b = 1.0 if 2 * l == n else 2.0
                # cos(2 l theta_k) with 2 l theta_k = 2 pi (l k mod n) / n
                r = (l * k) % n
                s += b * math.cos(2.0 * math.pi * r / n) / (4.0 * l * l - 1.0)
            w[k] = c / n * (1.0 - s)
        return w
    raise ValueError("unknown grid kind %r" % (kind,))


# --------------------------------------------------------------------------
# normalised associated Legendre functions
# --------------------------------------------------------------------------

def alf_m(N, m, mu, sint):
    """P~_n^m(mu_j) for n = m..N as an array [N-m+1, len(mu)].

    The standard three-term recurrence the paper uses (Sec. 4.1, after
    Enomoto 2015), in float64 and normalised as in eq. pnm-ortho:
      P~_0^0 = 1/sqrt(2)
      P~_m^m = sqrt((2m+1)/(2m)) sin(theta) P~_{m-1}^{m-1}
      P~_{m+1}^m = sqrt(2m+3) mu P~_m^m
      P~_n^m = a_n^m (mu P~_{n-1}^m - P~_{n-2}^m / a_{n-1}^m),
      a_n^m = sqrt((4n^2-1)/(n^2-m^2)).
    The paper runs it in quadruple precision, whose exponent range holds
    the sectoral start sin^m(theta) at any order used here; in float64 that
    start falls below the double range at high order (e.g. m = 747 at
    sin(theta) = 0.37), while P~_n^m grows back to O(1) before n = 2047.  So
    each latitude's values are carried as a float64 significand times 2^e
    with one integer exponent e per latitude (the recurrence is linear in
    the two values it carries, so both are rescaled together), and stored
    as significand * 2^e, which is 0 where the value is below the double
    range.
    """
    mu = np.asarray(mu, dtype=np.float64)
    sint = np.asarray(sint, dtype=np.float64)
    out = np.zeros((N - m + 1, mu.size))
    e = np.zeros(mu.size, dtype=np.int64)
    pmm = np.full(mu.size, 1.0 / math.sqrt(2.0))
    for k in range(1, m + 1):
        pmm, ex = np.frexp(math.sqrt((2.0 * k + 1.0) / (2.0 * k)) * sint * pmm)
        e += ex
    out[0] = np.ldexp(pmm, e)
    if N == m:
        return out
    p0, p1 = pmm, math.sqrt(2.0 * m + 3.0) * mu * pmm
    out[1] = np.ldexp(p1, e)

    def a(n):
        return math.sqrt((4.0 * n * n - 1.0) / (n * n - m * m))

    big = 2.0 ** 500
    for n in range(m + 2, N + 1):
        p0, p1 = p1, a(n) * (mu * p1 - p0 / a(n - 1))
        grow = np.abs(p1) > big
        if grow.any():
            p0 = np.where(grow, p0 / big, p0)
            p1 = np.where(grow, p1 / big, p1)
            e += np.where(grow, 500, 0)
        out[n - m] = np.ldexp(p1, e)
    return out


# --------------------------------------------------------------------------
# zonal (longitude) step
# --------------------------------------------------------------------------

def _phase(N, I):
    """alpha[m, i] = 2 pi ((m i) mod I) / I, for m = 0..N, i = 0..I-1."""
    m = np.arange(N + 1)[:, None]
    i = np.arange(I)[None, :]
    return 2.0 * np.pi * ((m * i) % I) / I


def zonal_analysis(x, N):
    """X^m(phi_j) = (1/I) sum_i x(lambda_i, phi_j) exp(-i m lambda_i), m <= N.

    Sec. 2, the discretised zonal integral, evaluated with an explicit DFT
    matrix.  x: [..., J, I] real -> [..., J, N+1] complex.
    """
    I = x.shape[-1]
    al = _phase(N, I)
    e = np.cos(al) - 1j * np.sin(al)
    return (x @ e.T) / I


def zonal_synthesis(X, I):
    """x(lambda_i) = Re X^0 + 2 sum_{m>=1} Re(X^m exp(i m lambda_i)).

    Sec. 2: the inverse DFT over m = -N..N with X^{-m} = conj(X^m) for a real
    field; Im X^0 is dropped.  X: [..., J, N+1] complex -> [..., J, I].
    """
    N = X.shape[-1] - 1
    al = _phase(N, I)
    c = np.cos(al)
    s = np.sin(al)
    c[1:] *= 2.0
    s[1:] *= 2.0
    # contiguous copies of the real and imaginary parts, so that the matrix
    # products run in BLAS (a strided view takes numpy's plain loop)
    return np.ascontiguousarray(X.real) @ c - np.ascontiguousarray(X.imag) @ s


# --------------------------------------------------------------------------
# the transform pair
# --------------------------------------------------------------------------

def _check_grid(grid):
    grid = np.asarray(grid, dtype=np.float64)
    if grid.ndim == 2:
        grid = grid[None]
    return grid


def _check_spec(spec, N):
    spec = np.asarray(spec, dtype=np.float64)
    if spec.ndim == 2:
        spec = spec[None]
    if spec.shape[-2:] != (ncoef(N), 2):
        raise ValueError("spec must be [F, ncoef, 2]")
    return spec


def forward(grid, N, kind):
    """Analysis (direct SHT), Sec. 2 eq. dSHT/dLT with the Clenshaw-Curtis
    quadrature of Sec. 3.1 eq. cc-quad:

        a_n^m = sum_{j=0}^{J-1} w_j P~_n^m(mu_j) X^m(phi_j).

    grid [F, J, I] -> spec [F, ncoef, 2]; Im a_n^0 set to 0.
    """
    grid = _check_grid(grid)
    F, J, I = grid.shape
    _, mu, sint = nodes(J, kind)
    w = weights(J, kind)
    X = zonal_analysis(grid, N)                  # [F, J, N+1]
    spec = np.zeros((F, ncoef(N), 2))
    for m in range(N + 1):
        P = alf_m(N, m, mu, sint)                # [n_m, J]
        a = (X[:, :, m] * w[None, :]) @ P.T      # [F, n_m]
        k0 = spec_index(N, m, m)
        spec[:, k0:k0 + N - m + 1, 0] = a.real
        spec[:, k0:k0 + N - m + 1, 1] = a.imag if m > 0 else 0.0
    return spec


def inverse(spec, N, J, I, kind):
    """Synthesis (inverse SHT), Sec. 2 eq. iSHT in its two steps: the
    Legendre sum eq. iLT, X^m(phi_j) = sum_n a_n^m P~_n^m(mu_j), then the
    zonal synthesis.  spec [F, ncoef, 2] -> grid [F, J, I].
    """
    spec = _check_spec(spec, N)
    F = spec.shape[0]
    _, mu, sint = nodes(J, kind)
    X = np.zeros((F, J, N + 1), dtype=np.complex128)
    for m in range(N + 1):
        P = alf_m(N, m, mu, sint)
        k0 = spec_index(N, m, m)
        a = spec[:, k0:k0 + N - m + 1, 0] + 1j * spec[:, k0:k0 + N - m + 1, 1]
        if m == 0:
            a = a.real + 0j
        X[:, :, m] = a @ P
    return zonal_synthesis(X, I)


def forward_adjoint(spec_bar, N, J, I, kind):
    """Transpose of `forward` under the Euclidean inner product of the stored
    real arrays (not a formula of the paper; needed for reverse-mode
    differentiation).  Written out from the definition of `forward`:

        d a_re(n,m) / d x_ji =  (w_j/I) P~_n^m(mu_j) cos(m lambda_i)
        d a_im(n,m) / d x_ji = -(w_j/I) P~_n^m(mu_j) sin(m lambda_i)  (m > 0)

    so x_bar_ji = (w_j/I) sum_m sum_n P~_n^m(mu_j)
                  (abar_re cos(m lambda_i) - abar_im sin(m lambda_i)),
    with the m = 0 imaginary part contributing nothing.
    """
    spec_bar = _check_spec(spec_bar, N)
    F = spec_bar.shape[0]
    _, mu, sint = nodes(J, kind)
    w = weights(J, kind)
    al = _phase(N, I)
    br = np.zeros((F, J, N + 1))       # sum_n abar_re(n, m) P~_n^m(mu_j)
    bi = np.zeros((F, J, N + 1))       # sum_n abar_im(n, m) P~_n^m(mu_j), 0 for m = 0
    for m in range(N + 1):
        P = alf_m(N, m, mu, sint)
        k0 = spec_index(N, m, m)
        br[:, :, m] = spec_bar[:, k0:k0 + N - m + 1, 0] @ P
        if m > 0:
            bi[:, :, m] = spec_bar[:, k0:k0 + N - m + 1, 1] @ P
    # the sum over m of br cos(m lambda_i) - bi sin(m lambda_i), as matrix products
    out = br @ np.cos(al) - bi @ np.sin(al)
    return out * (w / I)[None, :, None]


def inverse_adjoint(grid_bar, N, kind):
    """Transpose of `inverse` under the Euclidean inner product of the stored
    real arrays.  From x_ji = sum_n a_re(n,0) P~_n^0
    + 2 sum_{m>=1} sum_n P~_n^m (a_re cos - a_im sin):

        abar_re(n,m) =  c_m sum_j P~_n^m(mu_j) sum_i gbar_ji cos(m lambda_i)
        abar_im(n,m) = -c_m sum_j P~_n^m(mu_j) sum_i gbar_ji sin(m lambda_i)

    with c_0 = 1, c_m = 2 for m > 0, and abar_im(n, 0) = 0.
    """
    grid_bar = _check_grid(grid_bar)
    F, J, I = grid_bar.shape
    _, mu, sint = nodes(J, kind)
    al = _phase(N, I)
    cs = grid_bar @ np.cos(al).T                 # [F, J, N+1]
    sn = grid_bar @ np.sin(al).T
    out = np.zeros((F, ncoef(N), 2))
    for m in range(N + 1):
        P = alf_m(N, m, mu, sint)
        c = 1.0 if m == 0 else 2.0
        k0 = spec_index(N, m, m)
        out[:, k0:k0 + N - m + 1, 0] = c * (cs[:, :, m] @ P.T)
        if m > 0:
            out[:, k0:k0 + N - m + 1, 1] = -c * (sn[:, :, m] @ P.T)
    return out


# --------------------------------------------------------------------------
# pointwise evaluation for sampled checks at large sizes
# --------------------------------------------------------------------------

def forward_sample(grid_field, N, kind, m, n_list):
    """a_n^m of one field for one m and a few n, straight from the definition
    (same formula as `forward`, restricted).  grid_field [J, I] -> [len, 2]."""
    x = np.asarray(grid_field, dtype=np.float64)
    J, I = x.shape
    _, mu, sint = nodes(J, kind)
    w = weights(J, kind)
    al = 2.0 * np.pi * ((m * np.arange(I)) % I) / I
    Xm = (x @ np.cos(al) - 1j * (x @ np.sin(al))) / I       # [J]
    P = alf_m(N, m, mu, sint)
    out = np.zeros((len(n_list), 2))
    for k, n in enumerate(n_list):
        v = np.sum(w * P[n - m] * Xm)
        out[k] = (v.real, v.imag if m > 0 else 0.0)
    return out


def inverse_sample_row(spec_field, N, J, I, kind, j):
    """Row j of the synthesis of one field (same formula as `inverse`,
    restricted to one latitude).  spec_field [ncoef, 2] -> [I]."""
    spec = np.asarray(spec_field, dtype=np.float64)
    _, mu, sint = nodes(J, kind)
    X = np.zeros(N + 1, dtype=np.complex128)
    for m in range(N + 1):
        P = alf_m(N, m, mu[j:j + 1], sint[j:j + 1])[:, 0]
        k0 = spec_index(N, m, m)
        a = spec[k0:k0 + N - m + 1, 0] + 1j * spec[k0:k0 + N - m + 1, 1]
        if m == 0:
            a = a.real + 0j
        X[m] = a @ P
    return zonal_synthesis(X[None, :], I)[0]


# --------------------------------------------------------------------------
# numerical orthonormality (Sec. 4.1, eq. norm-err and eq. orth-err)
# --------------------------------------------------------------------------

def orthonormality_errors(N, J, kind):
    """Normality error |sum_j P~_n^m(mu_j)^2 w_j - 1| and orthogonality error
    max_{n' != n} |sum_j P~_n^m P~_n'^m w_j|, as arrays [N+1 (m), N+1 (n)]
    with NaN where n < m (Sec. 4.1, eq. norm-err, eq. orth-err)."""
    _, mu, sint = nodes(J, kind)
    w = weights(J, kind)
    en = np.full((N + 1, N + 1), np.nan)
    eo = np.full((N + 1, N + 1), np.nan)
    for m in range(N + 1):
        P = alf_m(N, m, mu, sint)
        G = (P * w[None, :]) @ P.T
        en[m, m:] = np.abs(np.diag(G) - 1.0)
        off = np.abs(G - np.diag(np.diag(G)))
        eo[m, m:] = off.max(axis=1) if G.shape[0] > 1 else 0.0
    return en, eo


# --------------------------------------------------------------------------
# transfers between levels (App. C building blocks)
# --------------------------------------------------------------------------

def retruncate(spec, N_in, N_out):
    """Spectral restriction / prolongation between truncations: coefficient
    (m, n) of the output is that of the input for n <= min(N_in, N_out) and
    zero for n > N_in.  spec: [F, ncoef(N_in), 2] -> [F, ncoef(N_out), 2]."""
    spec = np.asarray(spec, dtype=np.float64)
    F = spec.shape[0]
    out = np.zeros((F, ncoef(N_out), 2))
    for m in range(min(N_in, N_out) + 1):
        for n in range(m, min(N_in, N_out) + 1):
            out[:, spec_index(N_out, m, n)] = spec[:, spec_index(N_in, m, n)]
    return out


def inject(grid, Jc, Ic, kind):
    """Grid restriction by injection (Sec. 3.2): the coarse grid's nodes are
    a subset of the fine grid's.  "cc_poles": rows s*j with
    s = (Jf-1)/(Jc-1); "fejer2": rows s*(j+1)-1 with s = (Jf+1)/(Jc+1);
    columns t*i with t = If/Ic."""
    grid = np.asarray(grid, dtype=np.float64)
    _, Jf, If = grid.shape
    if If % Ic:
        raise ValueError("I_fine must be a multiple of I_coarse")
    t = If // Ic
    if kind == "cc_poles":
        if (Jf - 1) % (Jc - 1):
            raise ValueError("rows do not nest")
        s = (Jf - 1) // (Jc - 1)
        rows = [s * j for j in range(Jc)]
    elif kind == "fejer2":
        if (Jf + 1) % (Jc + 1):
            raise ValueError("rows do not nest")
        s = (Jf + 1) // (Jc + 1)
        rows = [s * (j + 1) - 1 for j in range(Jc)]
    else:
        raise ValueError("grid kind %r does not nest" % (kind,))
    return grid[:, rows, :][:, :, ::t].copy()



# --------------------------------------------------------------------------
# residual of the elliptic problem of App. C (eq. elliptic)
# --------------------------------------------------------------------------

def laplacian(spec, N, scale=1.0):
    """Spectral Laplacian: Y_n^m is an eigenfunction of the Laplacian on the
    unit sphere with eigenvalue -n(n+1); on a sphere of radius 1/sqrt(scale)
    the factor is -scale n(n+1).  spec [F, ncoef(N), 2] -> same shape."""
    spec = np.asarray(spec, dtype=np.float64)
    out = np.empty_like(spec)
    for m in range(N + 1):
        for n in range(m, N + 1):
            c = -scale * float(n * (n + 1))
            k = spec_index(N, m, n)
            out[:, k, 0] = c * spec[:, k, 0]
            out[:, k, 1] = c * spec[:, k, 1]
    return out


def helmholtz_residual(x, kappa, f, alpha, N, kind, scale=1.0):
    """R = (I - alpha L) x - f with L x = kappa * lap(x), the Laplacian
    evaluated pseudo-spectrally (analysis at truncation N, spectral
    Laplacian, synthesis on the same grid): the residual of step 1 of the
    two-grid cycle of App. C, alpha standing for dt/2.
    x, f [F, J, I]; kappa [J, I]."""
    x = np.asarray(x, dtype=np.float64)
    _, J, I = x.shape
    lap = inverse(laplacian(forward(x, N, kind), N, scale), N, J, I, kind)
    return x - alpha * np.asarray(kappa, dtype=np.float64)[None] * lap - np.asarray(f, dtype=np.float64)
