"""Pins of the oracle's region switching, pressure boundary and density-
dependent relaxation time (no GPU).

* Switching indicator (Sec. 2.2, the 'B' breakdown parameter in isothermal
  form): a node built from chosen Hermite coefficients (Eq. an) gives exactly
  the largest second-order non-equilibrium component over rho, evaluated in
  the set of the node's own region; an equilibrium node gives zero.
* Band rule: hand-made indicator fields with answers worked out by hand,
  covering the strict threshold, the clamps, the mirrored top wall, the
  middle row that both halves scan, and a ragged last tile.
* Pressure boundary (ghost columns hold the equilibrium at the prescribed
  density with the edge node's velocity plus the edge node's
  non-equilibrium part, the virtual-boundary device of Sec. 2.2): equal inlet
  and outlet densities at rest are a fixed point, and after one step from an
  x-uniform state the edge columns gain exactly the half-range flux of the
  density jump, which the Gauss-Hermite rule fixes in closed form
  (numpy's hermegauss, not the oracle's rule).
* Density-dependent relaxation (Eq. dbgk: tau proportional to mu/p, with mu
  fixed): the shear-wave viscosity at rho = 2 is tau0 rho_ref / rho + dt/2.
"""
import math

import numpy as np
import pytest


# ------------------------------------------------------------ indicator
def _node_from_coeffs(oracle, n, rho, ux, uy, neq, rng):
    """Populations of set n whose Hermite coefficients are the equilibrium
    ones up to second order plus the given (n20, n11, n02), with arbitrary
    higher components (which the indicator must ignore)."""
    a = np.zeros((n, n))
    a[3:, :] = 0.0
    hi = rng.normal(scale=1e-3, size=(n, n))
    for k in range(n):
        for m in range(n):
            if k + m > 2:
                a[k, m] = hi[k, m]
    a[0, 0] = rho
    a[1, 0], a[0, 1] = rho * ux, rho * uy
    a[2, 0] = rho * ux * ux + neq[0]
    a[1, 1] = rho * ux * uy + neq[1]
    a[0, 2] = rho * uy * uy + neq[2]
    return oracle.from_coeffs(n, a)


@pytest.mark.parametrize("nl,nh", [(3, 6), (3, 4), (4, 6)])
def test_indicator_is_largest_second_order_neq_over_rho(oracle, nl, nh):
    nx, ny = 5, 12
    L = oracle.Lattice(nx, ny, kn=0.1, n_low=nl, n_high=nh, eq_low=2, eq_high=min(nh - 1, 4))
    L.set_regions(3, 2)
    reg = L.region()
    rng = np.random.default_rng(100 + nh)
    f = [np.zeros((nl * nl, ny + 1, nx)), np.zeros((nh * nh, ny + 1, nx))]
    want = np.zeros((ny + 1, nx))
    for j in range(ny + 1):
        for i in range(nx):
            rho = rng.uniform(0.6, 2.2)
            ux, uy = rng.uniform(-0.2, 0.2, 2)
            # different non-equilibrium parts in the two sets, with the
            # largest component (and its sign) rotating over the nodes
            for s, n in ((0, nl), (1, nh)):
                neq = rng.uniform(-1e-3, 1e-3, 3)
                big = (i + 2 * j + s) % 3
                neq[big] = (1 if (i + j) % 2 else -1) * rng.uniform(5e-3, 2e-2)
                f[s][:, j, i] = _node_from_coeffs(oracle, n, rho, ux, uy, neq, rng)
                if (reg[j, i] == 1) == (s == 1):
                    want[j, i] = np.max(np.abs(neq)) / rho
    L.set_populations(0, f[0])
    L.set_populations(1, f[1])
    B = L.indicator()
    np.testing.assert_allclose(B, want, rtol=1e-11, atol=0)


@pytest.mark.parametrize("n,N", [(3, 2), (4, 3), (6, 4)])
def test_indicator_vanishes_at_equilibrium(oracle, n, N):
    L = oracle.Lattice(6, 9, kn=0.1, n_low=n, n_high=n, eq_low=N)
    rng = np.random.default_rng(7)
    L.init_equilibrium(rng.uniform(0.5, 2.0, (10, 6)), rng.uniform(-0.2, 0.2, (10, 6)),
                       rng.uniform(-0.2, 0.2, (10, 6)))
    assert np.max(L.indicator()) < 1e-15


# ------------------------------------------------------------ band rule
def test_band_rule_hand_cases(oracle):
    # nx = 14 in tiles of 4: tiles 0..2 full, tile 3 ragged (columns 12, 13);
    # ny = 20: rows 0..20, the lower half is rows 0..10 and the upper half is
    # rows 20..10 (row 10 is scanned from both walls)
    nx, ny, th = 14, 20, 0.01
    L = oracle.Lattice(nx, ny, kn=0.1, n_low=3, n_high=6, eq_low=2, eq_high=4, tile_w=4)
    B = np.zeros((ny + 1, nx))
    # tile 0: lowest-wall hit in row 3 -> 4 rows; top hit 6 rows below the top
    # wall (row 14) -> 7 rows; a value equal to theta does not count
    B[3, 1] = 0.5
    B[1, 2] = 0.2
    B[14, 2] = 0.02
    B[8, 0] = th
    # tile 1: row 9 -> 10 rows; rows above the middle count for the top only:
    # row 12 is 8 below the top -> 9 rows
    B[9, 5] = 1.0
    B[12, 7] = 0.03
    # tile 2: the middle row (10) counts for both walls -> 11 rows each
    B[10, 9] = 0.02
    # tile 3 (ragged): the wall row itself -> 1 row at each wall; a value just
    # below theta does not count
    B[0, 12] = 0.02
    B[ny, 13] = 0.5
    B[5, 13] = th * (1 - 1e-12)
    raw_lo, raw_hi = [4, 10, 11, 1], [7, 9, 11, 1]
    blo, bhi = L.bands_from_indicator(B, th, 0, 1000)
    assert list(blo) == raw_lo and list(bhi) == raw_hi
    # clamped to [2, 9]
    blo, bhi = L.bands_from_indicator(B, th, 2, 9)
    assert list(blo) == [4, 9, 9, 2] and list(bhi) == [7, 9, 9, 2]
    # an all-quiet field gives the minimum band everywhere
    blo, bhi = L.bands_from_indicator(np.zeros_like(B), th, 3, 9)
    assert list(blo) == [3] * 4 and list(bhi) == [3] * 4


def test_band_rule_matches_brute_force_definition(oracle):
    # random sparse fields on several shapes against a direct reading of the
    # rule: per tile, one row past the highest lower-half row (distance from
    # the wall) whose indicator exceeds theta, mirrored at the top, clamped
    rng = np.random.default_rng(11)
    for nx, ny, tw in ((10, 15, 3), (64, 30, 16), (9, 8, 9), (7, 41, 2)):
        L = oracle.Lattice(nx, ny, kn=0.1, n_low=3, n_high=6, eq_low=2, eq_high=4, tile_w=tw)
        for _ in range(5):
            B = np.where(rng.uniform(size=(ny + 1, nx)) < 0.04, rng.uniform(0, 0.05, (ny + 1, nx)), 0.0)
            th, bmin, bmax = 0.01, int(rng.integers(0, 3)), int(rng.integers(3, ny))
            blo, bhi = L.bands_from_indicator(B, th, bmin, bmax)
            for t in range(-(-nx // tw)):
                cols = slice(t * tw, min((t + 1) * tw, nx))
                d_lo = [j + 1 for j in range(ny // 2 + 1) if np.any(B[j, cols] > th)]
                d_hi = [j + 1 for j in range(ny // 2 + 1) if np.any(B[ny - j, cols] > th)]
                lo = min(max(max(d_lo, default=0), bmin), bmax)
                hi = min(max(max(d_hi, default=0), bmin), bmax)
                assert (blo[t], bhi[t]) == (lo, hi), (nx, ny, tw, t)


# ------------------------------------------------------- pressure columns
def _half_range_moments(n):
    """sum over positive abscissae of x w and x^2 w, weights normalised to 1,
    from numpy's Gauss-Hermite_e rule."""
    x, w = np.polynomial.hermite_e.hermegauss(n)
    w = w / w.sum()
    pos = x > 0
    return float(np.sum(x[pos] * w[pos])), float(np.sum(x[pos] ** 2 * w[pos]))


@pytest.mark.parametrize("n,N", [(3, 2), (6, 4)])
def test_pressure_equal_densities_at_rest_is_fixed_point(oracle, n, N):
    rho0 = 1.3
    L = oracle.Lattice(9, 7, kn=0.1, n_low=n, n_high=n, eq_low=N, xbc=oracle.XBC_PRESSURE,
                       ybc=oracle.YBC_PERIODIC, rho_in=rho0, rho_out=rho0, rho_ref=1.0,
                       tau_mode=oracle.TAU_RHO)
    L.init_equilibrium(rho0, 0.0, 0.0)
    f0 = L.get_populations(0)
    L.step(20)
    # fixed to a few ulp: the rest velocity is a sum of opposite terms whose
    # rounding leaves ~1e-17, which the equilibria then carry
    np.testing.assert_allclose(L.get_populations(0), f0, rtol=1e-14, atol=0)


@pytest.mark.parametrize("n,N", [(3, 2), (4, 3), (6, 4)])
def test_pressure_columns_half_range_inflow(oracle, n, N):
    # x- and y-uniform state at rest with a non-equilibrium part that has no
    # mass or momentum (normal-stress difference), rho_in > rho0 > rho_out.
    # The ghost columns differ from the edge node by f_eq(rho_b, u) -
    # f_eq(rho0, u) = (rho_b - rho0) w at rest, so the limiter is inactive and
    # the edge column takes in dt (rho_b - rho0) times the half-range flux
    # sum_{xi_x > 0} xi_x w (and the same for x-momentum with xi_x^2);
    # every other column is unchanged.
    nx, ny, rho0, rin, rout = 8, 3, 1.5, 2.0, 1.0
    L = oracle.Lattice(nx, ny, kn=0.4, n_low=n, n_high=n, eq_low=N, xbc=oracle.XBC_PRESSURE,
                       ybc=oracle.YBC_PERIODIC, rho_in=rin, rho_out=rout)
    cx, cy, w = oracle.vset(n)
    eps = 2e-3
    he2 = lambda v: v * v - 1.0
    f = rho0 * w + eps * w * (he2(cx) - he2(cy))
    L.set_populations(0, np.broadcast_to(f[:, None, None], (n * n, ny + 1, nx)).copy())
    r0, _, _ = L.moments()
    L.step(1)
    r1, ux1, uy1 = L.moments()
    m1, m2 = _half_range_moments(n)
    dt = L.dt
    np.testing.assert_allclose(r1[:, 0], rho0 + dt * (rin - rho0) * m1, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r1[:, -1], rho0 + dt * (rout - rho0) * m1, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r1[:, 1:-1], r0[:, 1:-1], rtol=0, atol=1e-14)
    np.testing.assert_allclose(r1[:, 0] * ux1[:, 0], dt * (rin - rho0) * m2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r1[:, -1] * ux1[:, -1], -dt * (rout - rho0) * m2, rtol=0, atol=1e-14)
    assert np.max(np.abs(uy1)) < 1e-14


@pytest.mark.parametrize("n,N", [(3, 2), (6, 4)])
def test_pressure_columns_use_edge_velocity(oracle, n, N):
    # the same with a uniform velocity u0 along x: ghost - edge =
    # (rho_b - rho0) f_eq(1, u0), so the inflow of the right movers at the
    # inlet is dt (rho_b - rho0) sum_{xi_x > 0} xi_x f_eq(1, u0), with f_eq
    # the order-N equilibrium (pinned on its own by its moments)
    nx, ny, rho0, rin, rout, u0 = 8, 3, 1.5, 2.0, 1.0, 0.07
    L = oracle.Lattice(nx, ny, kn=0.4, n_low=n, n_high=n, eq_low=N, xbc=oracle.XBC_PRESSURE,
                       ybc=oracle.YBC_PERIODIC, rho_in=rin, rho_out=rout)
    cx, cy, w = oracle.vset(n)
    L.init_equilibrium(rho0, u0, 0.0)
    L.step(1)
    r1, _, _ = L.moments()
    e1 = oracle.equilibrium(n, N, 1.0, u0, 0.0)
    right, left = cx > 0, cx < 0
    din = L.dt * (rin - rho0) * np.sum(cx[right] * e1[right])
    dout = L.dt * (rout - rho0) * np.sum(-cx[left] * e1[left])
    # the interior columns next to the edge see no jump (x-uniform)
    np.testing.assert_allclose(r1[:, 0], rho0 + din, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r1[:, -1], rho0 + dout, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r1[:, 2:-2], rho0, rtol=0, atol=1e-14)


# ------------------------------------------------- rho-dependent tau
@pytest.mark.parametrize("n,N", [(3, 2), (6, 4)])
def test_rho_dependent_tau_shear_wave_viscosity(oracle, n, N):
    # Eq. (dbgk): the relaxation time is mu / p with p = rho T; at fixed mu
    # and T = 1 it is tau0 rho_ref / rho.  A shear wave on a uniform rho = 2
    # gas then decays with nu = tau0 rho_ref / rho + dt/2 (the forward-Euler
    # viscosity of the scheme, c_s = 1)
    nrow, tau0, rho = 256, 4.0, 2.0
    L = oracle.Lattice(4, nrow - 1, kn=tau0 / (nrow - 1), n_low=n, n_high=n, eq_low=N,
                       ybc=oracle.YBC_PERIODIC, tau_mode=oracle.TAU_RHO, rho_ref=1.0)
    y = np.arange(nrow)[:, None] * np.ones((1, 4))
    k = 2 * np.pi / nrow
    L.init_equilibrium(rho, 1e-3 * np.sin(k * y), 0.0 * y)
    L.step(100)

    def amp():
        _, ux, _ = L.moments()
        return 2 * np.mean(ux[:, 0] * np.sin(k * y[:, 0]))

    a0, t0 = amp(), L.steps * L.dt
    L.step(2000)
    a1, t1 = amp(), L.steps * L.dt
    nu = -math.log(a1 / a0) / (k * k * (t1 - t0))
    assert abs(nu / (tau0 / rho + 0.5 * L.dt) - 1) < 0.01, nu
