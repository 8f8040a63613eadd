"""Pins of the oracle's nodes and weights against what the paper and the
mathematics fix (closed forms, exactness degree, an independent moment solve,
the App. A cardinal-function integral, the numbers printed in Sec. 4.3)."""

import math
import os

import mpmath
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("kind", O.GRID_KINDS)
@pytest.mark.parametrize("J", [3, 4, 5, 8, 17, 43, 320])
def test_nodes_closed_form(kind, J):
    theta, mu, sint = O.nodes(J, kind)
    if kind == "cc_poles":
        ref = np.arange(J) * math.pi / (J - 1)
    elif kind == "fejer1":
        ref = (np.arange(1, J + 1) - 0.5) * math.pi / J   # Sec. 3.3, eq. fejer1-points
    else:
        ref = np.arange(1, J + 1) * math.pi / (J + 1)
    assert np.allclose(theta, ref, rtol=0, atol=1e-15)
    assert np.allclose(mu, np.cos(ref), rtol=0, atol=1e-15)
    assert np.allclose(sint, np.sin(ref), rtol=0, atol=1e-15)
    # north first, mirror antisymmetry bit for bit, equator exactly 0
    assert mu[0] > 0
    assert np.array_equal(mu[::-1], -mu)
    assert np.array_equal(sint[::-1], sint)
    if J % 2 == 1:
        assert mu[J // 2] == 0.0 and sint[J // 2] == 1.0
    if kind == "cc_poles":
        assert mu[0] == 1.0 and mu[-1] == -1.0 and sint[0] == 0.0


def test_nodes_nest_bitwise():
    # classical grid: J = 2^k + 1 nests by taking every other row
    prev = None
    for k in range(6, 11):
        J = 2 ** k + 1
        _, mu, s = O.nodes(J, "cc_poles")
        if prev is not None:
            assert np.array_equal(mu[::2], prev[0])
            assert np.array_equal(s[::2], prev[1])
        prev = (mu, s)
    # the paper's grid nests when J+1 is multiplied (Sec. 3.2): Tc159 in Tc479
    # (every 3rd row), Tc479 in Tc959 (every 2nd), Tc239 in Tc479 (every 2nd)
    cases = [(319, 959, 3), (479, 959, 2), (959, 1919, 2), (479, 1919, 4)]
    for Jc, Jf, s in cases:
        _, muc, sc = O.nodes(Jc, "fejer2")
        _, muf, sf = O.nodes(Jf, "fejer2")
        assert np.array_equal(muf[s - 1::s], muc)
        assert np.array_equal(sf[s - 1::s], sc)
    # the two grids are different: 65 and 129 on the paper's grid share only
    # the equator
    _, a, _ = O.nodes(65, "fejer2")
    _, b, _ = O.nodes(129, "fejer2")
    assert len(set(a.tolist()) & set(b.tolist())) == 1


def test_weights_hand_values():
    # fejer2, J = 3: theta = pi/4, pi/2, 3pi/4; eq. cc-wgt gives 2/3 each
    assert np.allclose(O.weights(3, "fejer2"), [2 / 3] * 3, rtol=1e-15)
    assert np.allclose(O.weights(5, "fejer2"),
                       np.array([14, 18, 26, 18, 14]) / 45, rtol=1e-15)
    # classical rule: Simpson for J = 3, and the 5-point rule
    assert np.allclose(O.weights(3, "cc_poles"), [1 / 3, 4 / 3, 1 / 3],
                       rtol=1e-15)
    assert np.allclose(O.weights(5, "cc_poles"),
                       np.array([1, 8, 12, 8, 1]) / 15, rtol=1e-15)
    # J = 2 on the classical grid is the trapezoid rule
    assert np.allclose(O.weights(2, "cc_poles"), [1.0, 1.0], rtol=1e-15)
    # Fejer's first rule: the midpoint rule in theta for J = 1; J = 2 has
    # nodes mu = +-1/sqrt(2) and weights 1, 1; J = 3 (theta = pi/6, pi/2,
    # 5pi/6) is exact for 1 and mu^2 only with weights 4/9, 10/9, 4/9
    assert np.allclose(O.weights(1, "fejer1"), [2.0], rtol=1e-15)
    assert np.allclose(O.weights(2, "fejer1"), [1.0, 1.0], rtol=1e-15)
    assert np.allclose(O.weights(3, "fejer1"), [4 / 9, 10 / 9, 4 / 9], rtol=1e-15)


def test_fejer1_printed_weights_lack_a_factor_two():
    """Sec. 3.3 prints eq. fejer1-wgt as (2/J)(1 - sum cos(2p theta)/(4p^2-1));
    that form sums to 2 but does not integrate mu^2 exactly, while the form
    with 2 * sum (Fejer's first rule, the oracle's) does: the reading taken."""
    J = 7
    theta, mu, _ = O.nodes(J, "fejer1")
    p = np.arange(1, J // 2 + 1)
    s = (np.cos(2 * np.outer(theta, p)) / (4 * p * p - 1)).sum(axis=1)
    printed = 2.0 / J * (1.0 - s)
    assert abs(printed.sum() - 2.0) < 1e-14
    assert abs(np.sum(printed * mu ** 2) - 2 / 3) > 1e-2
    w = O.weights(J, "fejer1")
    assert np.allclose(w, 2.0 / J * (1.0 - 2.0 * s), rtol=1e-14)
    assert abs(np.sum(w * mu ** 2) - 2 / 3) < 1e-15


@pytest.mark.parametrize("kind", O.GRID_KINDS)
@pytest.mark.parametrize("J", list(range(3, 18)) + [43, 319, 959])
def test_weights_sum_symmetry_positive(kind, J):
    w = O.weights(J, kind)
    assert abs(w.sum() - 2.0) < 1e-14 * max(1, J / 50)
    assert np.allclose(w, w[::-1], rtol=1e-13, atol=0)
    assert np.all(w > 0)


@pytest.mark.parametrize("kind", O.GRID_KINDS)
@pytest.mark.parametrize("J", list(range(3, 18)))
def test_weights_exact_degree(kind, J):
    """Exact for mu^d, d <= J-1 (and d = J when J is odd, by symmetry);
    not exact at the first even degree beyond that (Sec. 3.1,
    eq. cc-condition)."""
    _, mu, _ = O.nodes(J, kind)
    w = O.weights(J, kind)
    dmax = J if J % 2 == 1 else J - 1
    for d in range(dmax + 1):
        exact = 2.0 / (d + 1) if d % 2 == 0 else 0.0
        assert abs(np.sum(w * mu ** d) - exact) < 1e-14
    d = dmax + 1 if (dmax + 1) % 2 == 0 else dmax + 2
    assert abs(np.sum(w * mu ** d) - 2.0 / (d + 1)) > 1e-9


@pytest.mark.parametrize("kind", O.GRID_KINDS)
@pytest.mark.parametrize("J", [9, 17])
def test_weights_moment_system_mpmath(kind, J):
    """Independent route: the interpolatory rule on J distinct nodes is the
    unique solution of sum_j w_j T_k(mu_j) = int_{-1}^{1} T_k, k < J, here
    solved in 40-digit arithmetic."""
    mpmath.mp.dps = 40
    if kind == "cc_poles":
        th = [mpmath.pi * j / (J - 1) for j in range(J)]
    elif kind == "fejer1":
        th = [mpmath.pi * (2 * j + 1) / (2 * J) for j in range(J)]
    else:
        th = [mpmath.pi * (j + 1) / (J + 1) for j in range(J)]
    A = mpmath.matrix(J, J)
    b = mpmath.matrix(J, 1)
    for k in range(J):
        for j in range(J):
            A[k, j] = mpmath.cos(k * th[j])
        b[k] = mpmath.mpf(2) / (1 - k * k) if k % 2 == 0 else 0
    wref = mpmath.lu_solve(A, b)
    w = O.weights(J, kind)
    for j in range(J):
        assert abs(w[j] - float(wref[j])) <= 3e-15 * max(1.0, abs(float(wref[j]))) + 3e-16


@pytest.mark.parametrize("J", [9, 17])
def test_weights_appendix_a_cardinal_functions(J):
    """App. A: w_j = sin(theta_j) * integral_0^pi C_j(theta) dtheta with the
    cardinal functions C_j(theta) = 2/(J+1) sum_p sin(p theta_j) sin(p theta);
    the integral is done by mpmath quadrature, not in closed form."""
    mpmath.mp.dps = 30
    w = O.weights(J, "fejer2")
    for j in range(J):
        tj = mpmath.pi * (j + 1) / (J + 1)

        def C(t):
            return 2 / mpmath.mpf(J + 1) * mpmath.fsum(
                mpmath.sin(p * tj) * mpmath.sin(p * t) for p in range(1, J + 1))

        ref = mpmath.sin(tj) * mpmath.quad(C, [0, mpmath.pi])
        assert abs(w[j] - float(ref)) < 1e-15


def _read_sec43():
    rows = []
    with open(os.path.join(GOLDEN, "sec43_quadrature_errors.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rule, J, fam, deg, val, unit = line.split()
            rows.append((rule, int(J), fam, int(deg), float(val), float(unit)))
    return rows


def _family_at_nodes(fam, deg, theta, mu):
    if fam == "U":
        return np.sin((deg + 1) * theta) / np.sin(theta)
    if fam == "T":
        return np.cos(deg * theta)
    c = np.zeros(deg + 1)
    c[deg] = 1.0
    return npleg.legval(mu, c)


def _family_integral(fam, deg):
    if fam == "U":
        return 2.0 / (deg + 1) if deg % 2 == 0 else 0.0
    if fam == "T":
        return 2.0 / (1.0 - deg * deg) if deg % 2 == 0 else 0.0
    return 0.0


@pytest.mark.parametrize("row", _read_sec43(), ids=lambda r: "%s%d-%s%d" % r[:4])
def test_sec43_printed_quadrature_errors(row):
    """The paper prints these errors to one or two significant digits (some
    truncated, some rounded): accept printed - unit/2 <= value < printed + unit."""
    rule, J, fam, deg, printed, unit = row
    if rule == "fejer2":
        theta, mu, _ = O.nodes(J, "fejer2")
        w = O.weights(J, "fejer2")
    else:
        mu, w = npleg.leggauss(J)
        theta = np.arccos(mu)
    err = abs(_family_integral(fam, deg) - np.sum(w * _family_at_nodes(fam, deg, theta, mu)))
    assert printed - unit / 2 <= err < printed + unit, (err, printed)


@pytest.mark.parametrize("p", [1, 241, 481, 721])
def test_sec43_closed_form_error(p):
    """e_J(p) = 2/(J+1+p) + 2/(J+1-p) for U_{J+p}, J+p even (Sec. 4.3)."""
    J = 959
    theta, mu, _ = O.nodes(J, "fejer2")
    w = O.weights(J, "fejer2")
    deg = J + p
    err = _family_integral("U", deg) - np.sum(w * _family_at_nodes("U", deg, theta, mu))
    assert abs(err - (2.0 / (J + 1 + p) + 2.0 / (J + 1 - p))) < 1e-12
    # odd J+p is integrated exactly (error 0 up to rounding)
    err2 = _family_integral("U", deg + 1) - np.sum(w * _family_at_nodes("U", deg + 1, theta, mu))
    assert abs(err2) < 1e-12


@pytest.mark.parametrize("J", [1, 2, 3, 4, 7, 16, 33])
def test_gauss_grid_pins(J):
    """The Gaussian grid (Sec. 2, the comparison grid used as the aliasing
    reference): nodes are the roots of P_J (north first, mirror-symmetric),
    the weights integrate mu^d exactly for d <= 2J-1 and, for small J, not
    for d = 2J (eq. gauss-condition); J = 2 is the two-point rule
    +-1/sqrt(3)."""
    theta, mu, s = O.nodes(J, "gauss")
    w = O.weights(J, "gauss")
    assert np.all(np.diff(mu) < 0)
    assert np.allclose(mu, -mu[::-1], rtol=0, atol=1e-15)
    assert np.allclose(npleg.legval(mu, [0] * J + [1]), 0, atol=1e-13)
    assert np.allclose(mu ** 2 + s ** 2, 1, rtol=0, atol=1e-15)
    for d in range(2 * J):
        exact = 2.0 / (d + 1) if d % 2 == 0 else 0.0
        assert abs(np.sum(w * mu ** d) - exact) < 1e-13
    if J <= 7:  # (the error at degree 2J decays factorially with J)
        assert abs(np.sum(w * mu ** (2 * J)) - 2.0 / (2 * J + 1)) > 1e-12
    if J == 2:
        assert np.allclose(mu, [3 ** -0.5, -(3 ** -0.5)], rtol=1e-15)
        assert np.allclose(w, [1.0, 1.0], rtol=1e-15)


@pytest.mark.parametrize("J", [1, 2, 5, 16, 33, 160, 1440])
def test_gauss_host_nodes_match_oracle(J):
    """The library's extended-precision Newton nodes and weights (host code,
    no GPU) agree with the oracle's 40-digit ones, and so does its sine of
    the node: the sectoral P~_3^3 ~ sin^3(theta) of the library's table
    matches the oracle's near the poles too (J = 1440: 1 - mu_0 ~ 1e-6)."""
    from paper_1711_11296_amd import host_tables
    mu, w, alf = host_tables(3, J, "gauss")
    _, mo, so = O.nodes(J, "gauss")
    assert np.allclose(mu, mo, rtol=0, atol=2e-16)
    assert np.array_equal(mu, -mu[::-1])
    assert np.allclose(w, O.weights(J, "gauss"), rtol=1e-13, atol=0)
    Jh = (J + 1) // 2
    sect = O.alf_m(3, 3, mo[:Jh], so[:Jh])[0]
    # the library's root carries about 1e-19 absolute error, so its sine
    # near the pole is good to about 1e-19 / (1 - mu_0), some 1e-14 here
    assert np.allclose(alf[O.spec_index(3, 3, 3)], sect, rtol=1e-13, atol=0)
