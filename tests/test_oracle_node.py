"""Pins of the oracle's tables and node-level operations (no GPU).

Each test checks the oracle against something it does not compute itself:
closed forms, numpy's independent Gauss-HermiteE rule, the paper's explicit
second-order formulas Eq. (demoeq) / Eq. (demoforce), the Hermite generating
function, a finite-difference velocity derivative, conservation identities.
"""
import math

import numpy as np
import numpy.polynomial.hermite_e as HE
import pytest

SETS = (3, 4, 6)


def test_hermite_polynomials_match_numpy(oracle):
    # He_k (Sec. 2.1, Eq. hermipol in 1D) against numpy's HermiteE series
    xs = np.linspace(-4, 4, 17)
    for k in range(9):
        c = np.zeros(k + 1)
        c[k] = 1.0
        ref = HE.hermeval(xs, c)
        got = np.array([oracle.hermite(k, x) for x in xs])
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_gh_closed_forms(oracle):
    # 3-point: 0, +-sqrt(3), weights 2/3, 1/6; 4-point: +-sqrt(3 -+ sqrt 6),
    # weights (3 +- sqrt 6)/12 (roots of He_n, weights of Eq. weight)
    x, w = oracle.gh_rule(3)
    np.testing.assert_allclose(x, [-math.sqrt(3), 0.0, math.sqrt(3)], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 2 / 3, 1 / 6], rtol=1e-15)
    x, w = oracle.gh_rule(4)
    a, b = math.sqrt(3 - math.sqrt(6)), math.sqrt(3 + math.sqrt(6))
    np.testing.assert_allclose(x, [-b, -a, a, b], rtol=1e-15)
    wa, wb = (3 + math.sqrt(6)) / 12, (3 - math.sqrt(6)) / 12
    np.testing.assert_allclose(w, [wb, wa, wa, wb], rtol=1e-14)


@pytest.mark.parametrize("n", range(1, 9))
def test_gh_rule_matches_numpy_hermegauss(oracle, n):
    x, w = oracle.gh_rule(n)
    xr, wr = HE.hermegauss(n)
    np.testing.assert_allclose(x, xr, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(w, wr / math.sqrt(2 * math.pi), rtol=1e-12)
    # abscissae are the roots of He_n (D2Q36: He_6 = x^6 - 15x^4 + 45x^2 - 15)
    c = np.zeros(n + 1)
    c[n] = 1.0
    assert np.max(np.abs(HE.hermeval(x, c))) < 1e-11
    if n == 6:
        assert np.max(np.abs(x**6 - 15 * x**4 + 45 * x**2 - 15)) < 1e-11
    # exactly symmetric
    np.testing.assert_array_equal(x, -x[::-1])


@pytest.mark.parametrize("n", SETS)
def test_gh_degree(oracle, n):
    # degree 2n-1: sum w x^k = (k-1)!! for even k, 0 for odd k
    x, w = oracle.gh_rule(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else float(np.prod(np.arange(k - 1, 0, -2))) if k else 1.0
        assert abs(np.sum(w * x**k) - exact) < 1e-12 * max(1.0, exact)
    # and not exact at degree 2n
    k = 2 * n
    exact = float(np.prod(np.arange(k - 1, 0, -2)))
    assert abs(np.sum(w * x**k) - exact) > 1e-3


@pytest.mark.parametrize("n", SETS)
def test_vset_layout(oracle, n):
    cx, cy, w = oracle.vset(n)
    x, w1 = oracle.gh_rule(n)
    for q in range(n):
        for p in range(n):
            a = p + n * q
            assert cx[a] == x[p] and cy[a] == x[q] and w[a] == w1[p] * w1[q]
    assert abs(w.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("n", SETS)
def test_discrete_hermite_transform_is_invertible(oracle, n):
    rng = np.random.default_rng(n)
    f = rng.uniform(0.0, 1.0, n * n)
    a = oracle.hermite_coeffs(n, f)
    np.testing.assert_allclose(oracle.from_coeffs(n, a), f, rtol=1e-12, atol=1e-14)
    a2 = rng.normal(size=(n, n))
    np.testing.assert_allclose(oracle.hermite_coeffs(n, oracle.from_coeffs(n, a2)), a2,
                               rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("n,N", [(3, 2), (4, 2), (4, 3), (6, 2), (6, 3), (6, 4), (6, 5)])
def test_equilibrium_moments_exact_to_order(oracle, n, N):
    # the quadrature reproduces the equilibrium's Hermite coefficients
    # a_eq = rho u^k v^m exactly for k + m <= N (Eq. approxfeq + Eq. an)
    rho, ux, uy = 1.3, 0.07, -0.11
    feq = oracle.equilibrium(n, N, rho, ux, uy)
    a = oracle.hermite_coeffs(n, feq)
    for k in range(n):
        for m in range(n):
            want = rho * ux**k * uy**m if k + m <= N else 0.0
            assert abs(a[k, m] - want) < 1e-14, (k, m, a[k, m], want)


def test_continuous_maxwellian_coefficients(oracle):
    # a_eq,km = int f_M He_k He_m dxi = rho ux^k uy^m, checked by a 60-point
    # quadrature of the true Maxwellian (independent of the sets)
    rho, ux, uy = 0.9, 0.2, -0.15
    xg, wg = HE.hermegauss(60)
    wg = wg / math.sqrt(2 * math.pi)
    X, Y = np.meshgrid(xg, xg, indexing="ij")
    W = np.outer(wg, wg)
    # int g(xi) f_M dxi = sum W g(X,Y) f_M / omega(X,Y)
    ratio = rho * np.exp(X * ux + Y * uy - 0.5 * (ux * ux + uy * uy))
    for k in range(4):
        for m in range(4 - k):
            ck = np.zeros(k + 1); ck[k] = 1
            cm = np.zeros(m + 1); cm[m] = 1
            val = np.sum(W * ratio * HE.hermeval(X, ck) * HE.hermeval(Y, cm))
            assert abs(val - rho * ux**k * uy**m) < 1e-12
    # and the oracle's order-4 D2Q36 equilibrium has these coefficients
    a = oracle.hermite_coeffs(6, oracle.equilibrium(6, 4, rho, ux, uy))
    assert abs(a[2, 1] - rho * ux**2 * uy) < 1e-14


@pytest.mark.parametrize("n", SETS)
def test_second_order_equilibrium_is_eq_demoeq(oracle, n):
    # Eq. (demoeq) with T = 1, D = 2: w rho {1 + xi.u + [(xi.u)^2 - u^2]/2}
    cx, cy, w = oracle.vset(n)
    rho, ux, uy = 1.1, -0.08, 0.05
    xu = cx * ux + cy * uy
    ref = w * rho * (1 + xu + 0.5 * (xu**2 - (ux * ux + uy * uy)))
    np.testing.assert_allclose(oracle.equilibrium(n, 2, rho, ux, uy), ref, rtol=1e-14, atol=1e-17)


@pytest.mark.parametrize("n,N", [(4, 3), (6, 4), (6, 5)])
def test_equilibrium_generating_function_limit(oracle, n, N):
    # sum_k t^k He_k(x)/k! = exp(x t - t^2/2): the order-N equilibrium over
    # w rho approaches exp(xi.u - u^2/2) with error O(|u|^(N+1))
    cx, cy, w = oracle.vset(n)
    errs = []
    for s in (0.04, 0.02):
        ux, uy = s, -0.7 * s
        f = oracle.equilibrium(n, N, 1.0, ux, uy) / w
        ref = np.exp(cx * ux + cy * uy - 0.5 * (ux * ux + uy * uy))
        errs.append(np.max(np.abs(f - ref)))
    # halving u divides the error by ~2^(N+1)
    assert errs[0] / errs[1] > 2 ** (N + 1) * 0.7


@pytest.mark.parametrize("n,N", [(3, 2), (4, 3), (6, 4)])
def test_force_moments(oracle, n, N):
    cx, cy, w = oracle.vset(n)
    rho, ux, uy, gx, gy = 1.2, 0.03, -0.02, 1e-3, -4e-4
    g = oracle.force(n, N, rho, ux, uy, gx, gy)
    assert abs(g.sum()) < 1e-17
    assert abs((cx * g).sum() - rho * gx) < 1e-17
    assert abs((cy * g).sum() - rho * gy) < 1e-17
    # second moment: rho (g u + u g)
    assert abs((cx * cx * g).sum() - 2 * rho * gx * ux) < 1e-17
    assert abs((cx * cy * g).sum() - rho * (gx * uy + gy * ux)) < 1e-17


@pytest.mark.parametrize("n", SETS)
def test_second_order_force_is_eq_demoforce(oracle, n):
    # Eq. (demoforce): w rho {g.xi + (g.xi)(u.xi) - g.u}
    cx, cy, w = oracle.vset(n)
    rho, ux, uy, gx, gy = 0.95, 0.04, 0.01, 2e-3, 1e-3
    gxi, uxi = gx * cx + gy * cy, ux * cx + uy * cy
    ref = w * rho * (gxi + gxi * uxi - (gx * ux + gy * uy))
    np.testing.assert_allclose(oracle.force(n, 2, rho, ux, uy, gx, gy), ref, rtol=1e-13, atol=1e-19)


@pytest.mark.parametrize("n,N", [(4, 3), (6, 4)])
def test_force_is_minus_g_dot_velocity_gradient(oracle, n, N):
    # F = -g . grad_xi f with f the Hermite expansion of order N-1 (Eq. approxf
    # with a = a_eq): checked by central differences in xi at every abscissa
    cx, cy, w = oracle.vset(n)
    rho, ux, uy, gx, gy = 1.0, 0.06, -0.03, 0.5, 0.3

    def fcont(X, Y):
        om = np.exp(-(X * X + Y * Y) / 2) / (2 * math.pi)
        s = 0.0
        for k in range(N):
            for m in range(N - k):
                ck = np.zeros(k + 1); ck[k] = 1
                cm = np.zeros(m + 1); cm[m] = 1
                s = s + rho * ux**k * uy**m * HE.hermeval(X, ck) * HE.hermeval(Y, cm) / (
                    math.factorial(k) * math.factorial(m))
        return om * s

    h = 1e-5
    dfx = (fcont(cx + h, cy) - fcont(cx - h, cy)) / (2 * h)
    dfy = (fcont(cx, cy + h) - fcont(cx, cy - h)) / (2 * h)
    om = np.exp(-(cx * cx + cy * cy) / 2) / (2 * math.pi)
    ref = w * (-(gx * dfx + gy * dfy)) / om
    np.testing.assert_allclose(oracle.force(n, N, rho, ux, uy, gx, gy), ref, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("n,N", [(3, 2), (4, 3), (6, 4)])
def test_collision_conserves_mass_and_momentum(oracle, n, N):
    cx, cy, w = oracle.vset(n)
    rng = np.random.default_rng(7)
    f = w * (1 + 0.2 * rng.uniform(-1, 1, n * n))
    rho, ux, uy = oracle.moments(n, f)
    d = oracle.equilibrium(n, N, rho, ux, uy) - f
    assert abs(d.sum()) < 1e-15 and abs((cx * d).sum()) < 1e-15 and abs((cy * d).sum()) < 1e-15


def _noneq_state(oracle, n, N, seed):
    cx, cy, w = oracle.vset(n)
    rng = np.random.default_rng(seed)
    feq = oracle.equilibrium(n, N, 1.05, 0.03, -0.02)
    return feq + 1e-3 * w * rng.normal(size=n * n)


@pytest.mark.parametrize("lo,hi", [((3, 2), (6, 4)), ((4, 3), (6, 4)), ((3, 2), (4, 3))])
def test_projection_low_round_trip_exact(oracle, lo, hi):
    f = _noneq_state(oracle, lo[0], lo[1], 11)
    up = oracle.project(*lo, *hi, f)
    back = oracle.project(*hi, *lo, up)
    np.testing.assert_allclose(back, f, rtol=0, atol=1e-15)


@pytest.mark.parametrize("lo,hi", [((3, 2), (6, 4)), ((4, 3), (6, 4))])
def test_projection_invariants(oracle, lo, hi):
    f = _noneq_state(oracle, hi[0], hi[1], 12)
    down = oracle.project(*hi, *lo, f)
    assert np.allclose(oracle.moments(lo[0], down), oracle.moments(hi[0], f), rtol=0, atol=1e-15)
    # restriction then lift is idempotent
    p1 = oracle.project(*lo, *hi, down)
    p2 = oracle.project(*lo, *hi, oracle.project(*hi, *lo, p1))
    np.testing.assert_allclose(p2, p1, rtol=0, atol=1e-15)
    # the identity on one set
    np.testing.assert_array_equal(oracle.project(*hi, *hi, f), f)
    # equilibria map to equilibria of the target order
    feq = oracle.equilibrium(lo[0], lo[1], 0.9, 0.05, 0.02)
    np.testing.assert_allclose(oracle.project(*lo, *hi, feq),
                               oracle.equilibrium(hi[0], hi[1], 0.9, 0.05, 0.02), atol=1e-15)
    # the shared non-equilibrium components are carried over exactly
    a_lo = oracle.hermite_coeffs(lo[0], down)
    a_hi = oracle.hermite_coeffs(hi[0], oracle.project(*lo, *hi, down))
    r, ux, uy = oracle.moments(lo[0], down)
    for k in range(lo[0]):
        for m in range(lo[0]):
            eq_lo = r * ux**k * uy**m if k + m <= lo[1] else 0.0
            eq_hi = r * ux**k * uy**m if k + m <= hi[1] else 0.0
            assert abs((a_hi[k, m] - eq_hi) - (a_lo[k, m] - eq_lo)) < 1e-15


def test_projection_closure_fills_missing_components(oracle):
    f = _noneq_state(oracle, 3, 2, 13)
    c = np.zeros(36)
    c[3 * 6 + 0] = 1e-4   # (3,0)
    c[1 * 6 + 3] = -2e-4  # (1,3)
    c[0 * 6 + 1] = 5.0    # (0,1) is carried by D2Q9: the closure must not touch it
    up = oracle.project(3, 2, 6, 4, f, c)
    a = oracle.hermite_coeffs(6, up)
    r, ux, uy = oracle.moments(3, f)
    assert abs(a[3, 0] - (r * ux**3 + 1e-4)) < 1e-15
    assert abs(a[1, 3] - (r * ux * uy**3 - 2e-4)) < 1e-15
    assert abs(a[0, 1] - r * uy) < 1e-15
