"""Pins of the oracle's thermal lattices (temperature in Eq. (demoeq), the wall
function S of Sec. 3.2, T_I of the interface of Sec. 2.2, the heat flux in the
'B' parameter of Sec. 2.2).

What fixes the expected values here, independently of the oracle's code:

* Gaussian moments.  The order-N equilibrium carries the Hermite coefficients
  of the Maxwellian up to order N, and the quadrature of degree 2n - 1 is exact
  for the moments sum f xi_x^a xi_y^b with a + b + N <= 2n - 1; those must
  equal rho E[X^a] E[Y^b] for X ~ N(ux, T), Y ~ N(uy, T) (closed form below).
* The printed second-order form of Eq. (demoeq), temperature term included.
* Chapman-Enskog.  Near rest at uniform pressure the first-order heat flux of
  the BGK equation is q = -tau/2 d/dy (sum xi_y^2 xi^2 f_eq).  With the set's
  moments m4 = sum w xi_y^2 xi^2 and M6 = sum w xi_y^2 xi^4 (taken from numpy's
  own Gauss-Hermite rule, not the oracle's), the order-2 thermal equilibrium
  gives sum xi_y^2 xi^2 f_eq = rho [m4 + (T - 1)(M6 - 2 m4)/2], so at constant
  p = rho T the conductivity read from the populations is
  kappa = tau (M6/4 - m4) p / T^2: 2 tau p for D2Q16 / D2Q36 (M6 = 24, the
  Maxwellian's), tau p / 2 for D2Q9 (M6 = 18).  The enthalpy flux gives
  c_p = m4 / 2 = 2, so an entropy (temperature) wave decays with the
  diffusivity kappa / (rho c_p); the time stepping adds dt/2 to tau, as for
  the viscosity (pinned in the isothermal flow tests): alpha = (tau + dt/2) *
  (M6 / (2 m4) - 2).
* Conservation.  BGK collisions towards an equilibrium with the node's own
  rho, u and energy conserve all three; the flux-form update conserves them
  on a periodic lattice.
* A closed box with both diffuse walls at T_w is in equilibrium only as the
  uniform Maxwellian at T_w at rest.
* The shear-wave viscosity mu = tau p (sum xi_x xi_y^2 f_eq = rho ux T for a
  set that resolves the third moment; rho ux for D2Q9) with the relaxation
  time tau = tau0 rho_ref / p of the collision frequency p / mu of Eq. (dbgk).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle

SETS = [(3, 2), (4, 2), (4, 3), (6, 2), (6, 4)]


def gauss_moment(a: int, u: float, T: float) -> float:
    """E[X^a] for X ~ N(u, T): sum_j C(a, 2j) u^(a-2j) T^j (2j-1)!!."""
    s = 0.0
    for j in range(a // 2 + 1):
        dfact = 1.0
        for k in range(1, 2 * j, 2):
            dfact *= k
        s += math.comb(a, 2 * j) * u ** (a - 2 * j) * T ** j * dfact
    return s


def set_moments_numpy(n: int):
    """m4 = sum w xi_y^2 xi^2 and M6 = sum w xi_y^2 xi^4 of the tensor-product
    n-point set, from numpy's Gauss-Hermite (probabilists') rule."""
    x, w = np.polynomial.hermite_e.hermegauss(n)
    w = w / w.sum()
    X, Y = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w)
    xi2 = X * X + Y * Y
    return float((W * Y * Y * xi2).sum()), float((W * Y * Y * xi2 * xi2).sum())


@pytest.mark.parametrize("n,eq", SETS)
def test_thermal_equilibrium_has_gaussian_moments(n, eq):
    cx, cy, _ = oracle.vset(n)
    rng = np.random.default_rng(7 + n + eq)
    for _ in range(4):
        rho, ux, uy = rng.uniform(0.5, 2.0), rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3)
        T = rng.uniform(0.7, 1.4)
        f = oracle.equilibrium(n, eq, rho, ux, uy, T=T)
        for a in range(eq + 1):
            for b in range(eq + 1 - a):
                if a + b + eq > 2 * n - 1:
                    continue
                got = float(np.sum(f * cx ** a * cy ** b))
                want = rho * gauss_moment(a, ux, T) * gauss_moment(b, uy, T)
                assert abs(got - want) <= 1e-13 * max(1.0, abs(want)), (a, b, got, want)


@pytest.mark.parametrize("n", [3, 4, 6])
def test_order2_thermal_equilibrium_is_eq_demoeq(n):
    """w rho {1 + xi.u + [(xi.u)^2 - u^2 + (T - 1)(xi^2 - D)] / 2}, D = 2."""
    cx, cy, w = oracle.vset(n)
    rho, ux, uy, T = 1.3, 0.11, -0.07, 1.17
    xu = cx * ux + cy * uy
    want = w * rho * (1 + xu + 0.5 * (xu ** 2 - (ux ** 2 + uy ** 2) + (T - 1) * (cx ** 2 + cy ** 2 - 2)))
    got = oracle.equilibrium(n, 2, rho, ux, uy, T=T)
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("n,eq", SETS)
def test_temperature_of_the_equilibrium_is_recovered(n, eq):
    rho, ux, uy, T = 0.9, -0.12, 0.05, 0.83
    r, vx, vy, t = oracle.moments_t(n, oracle.equilibrium(n, eq, rho, ux, uy, T=T))
    assert abs(r - rho) < 1e-14 and abs(vx - ux) < 1e-14 and abs(vy - uy) < 1e-14
    assert abs(t - T) < 1e-13


@pytest.mark.parametrize("n,eq", SETS)
def test_unit_temperature_is_the_isothermal_equilibrium(n, eq):
    a = oracle.equilibrium(n, eq, 1.1, 0.2, -0.1)
    b = oracle.equilibrium(n, eq, 1.1, 0.2, -0.1, T=1.0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n", [3, 4, 6])
def test_heat_flux_of_hand_built_populations(n):
    """At rest, sum xi_x^3 f = a_30 and sum xi_x xi_y^2 f = a_12 (the He_3 and
    He_1 He_2 coefficients), so q_x = (a_30 + a_12) / 2; likewise q_y."""
    a = np.zeros((n, n))
    a[0, 0] = 1.2
    a[2, 0] = a[0, 2] = 1.2 * 0.1   # T = 1.1
    if n > 3:
        a[3, 0], a[0, 3] = 0.02, -0.03
    a[1, 2], a[2, 1] = 0.005, 0.007
    f = oracle.from_coeffs(n, a)
    qx, qy = oracle.heat_flux(n, f)
    assert abs(qx - 0.5 * (a[3, 0] if n > 3 else 0.0) - 0.5 * a[1, 2]) < 1e-15
    assert abs(qy - 0.5 * (a[0, 3] if n > 3 else 0.0) - 0.5 * a[2, 1]) < 1e-15


@pytest.mark.parametrize("ns,es,nd,ed", [(3, 2, 6, 4), (6, 4, 3, 2), (3, 2, 4, 3), (4, 3, 6, 4), (6, 4, 4, 3)])
def test_thermal_projection_maps_equilibrium_to_equilibrium(ns, es, nd, ed):
    rho, ux, uy, T = 1.05, 0.08, -0.04, 1.25
    fs = oracle.equilibrium(ns, es, rho, ux, uy, T=T)
    fd = oracle.project(ns, es, nd, ed, fs, thermal=True)
    np.testing.assert_allclose(fd, oracle.equilibrium(nd, ed, rho, ux, uy, T=T), rtol=0, atol=2e-15)
    # and rho, u, T of any near-equilibrium node are carried exactly
    rng = np.random.default_rng(3)
    g = fs * (1 + 0.01 * rng.standard_normal(fs.size))
    m0 = oracle.moments_t(ns, g)
    m1 = oracle.moments_t(nd, oracle.project(ns, es, nd, ed, g, thermal=True))
    np.testing.assert_allclose(m1, m0, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("n,eq", [(3, 2), (4, 3), (6, 4)])
def test_periodic_thermal_lattice_conserves_mass_momentum_energy(n, eq):
    nx, ny = 16, 15
    L = oracle.Lattice(nx, ny, kn=0.05, n_low=n, n_high=n, eq_low=eq, thermal=True,
                       xbc=oracle.XBC_PERIODIC, ybc=oracle.YBC_PERIODIC)
    x = np.arange(nx)[None, :] * 2 * np.pi / nx
    y = np.arange(ny + 1)[:, None] * 2 * np.pi / (ny + 1)
    L.init_equilibrium(1 + 0.1 * np.sin(x + 2 * y), 0.05 * np.cos(y), 0.04 * np.sin(x),
                       1 + 0.15 * np.cos(x - y))
    c0, e0 = L.conservation(), L.energy()
    L.step(30)
    c1, e1 = L.conservation(), L.energy()
    assert abs(c1[0] / c0[0] - 1) < 1e-13
    assert np.all(np.abs(c1[1:] - c0[1:]) < 1e-12)
    assert abs(e1 / e0 - 1) < 1e-13
    T, _, _ = L.thermal_moments()
    assert T.std() > 1e-3   # the temperature field is still there


# (D2Q36's conductivity is pinned by the conduction test below: its entropy
# wave needs more columns than a quick test affords)
@pytest.mark.parametrize("n,eq,nx", [(3, 2, 128), (4, 3, 128)])
def test_entropy_wave_decays_with_the_chapman_enskog_diffusivity(n, eq, nx):
    tau, ny, eps = 0.5, 4, 1e-4
    L = oracle.Lattice(nx, ny, kn=tau / ny, n_low=n, n_high=n, eq_low=eq, thermal=True,
                       ybc=oracle.YBC_PERIODIC)
    m4, M6 = set_moments_numpy(n)
    ratio = M6 / (2 * m4) - 2
    k = 2 * np.pi / nx
    x = np.arange(nx)
    T0 = np.broadcast_to(1 + eps * np.sin(k * x), (ny + 1, nx))
    L.init_equilibrium(1.0 / T0, 0.0, 0.0, T0)   # uniform pressure, at rest
    alpha = (tau + L.dt / 2) * ratio
    chunk = int(0.05 / (alpha * k * k) / L.dt)
    ts, amp = [], []
    for s in range(20):
        L.step(chunk)
        T, _, _ = L.thermal_moments()
        ts.append((s + 1) * chunk * L.dt)
        amp.append(2 * np.mean((T[0] - 1) * np.sin(k * x)))
    rate = -np.polyfit(ts[10:], np.log(amp[10:]), 1)[0]
    assert abs(rate / (k * k) / alpha - 1) < 0.015, (rate / (k * k), alpha)


@pytest.mark.parametrize("n,eq", [(3, 2), (4, 3), (6, 4)])
def test_fourier_conduction_between_walls(n, eq):
    """Steady conduction between walls at 1.01 and 0.99: mid-channel heat flux
    over the temperature gradient is tau (M6/4 - m4) p / T^2, and there is
    no flow along the walls.  (Across the channel the wall condition of
    Sec. 3.2 leaves a small uniform mass current: resetting the populations
    that leave the wall node to the wall temperature's shape matches the
    particle fluxes but not that node's mass.)"""
    ny, nx, kn = 32, 4, 0.02
    tau = kn * ny
    L = oracle.Lattice(nx, ny, kn=kn, n_low=n, n_high=n, eq_low=eq, thermal=True, T_wall=(1.01, 0.99))
    L.init_equilibrium(1.0, 0.0, 0.0, 1.0)
    m4, M6 = set_moments_numpy(n)
    alpha = tau * (M6 / (2 * m4) - 2)
    L.step(int(8 * ny * ny / (np.pi ** 2 * alpha) / L.dt))
    T, _, qy = L.thermal_moments()
    rho, ux, uy = L.moments()
    j = ny // 2
    dTdy = (T[j + 1, 0] - T[j - 1, 0]) / 2
    p = rho[j, 0] * T[j, 0]
    kappa = -qy[j, 0] / dTdy
    assert abs(kappa / (tau * (M6 / 4 - m4) * p / T[j, 0] ** 2) - 1) < 2e-4
    assert np.abs(ux).max() < 1e-13 and np.abs(uy).max() < 0.2 * abs(qy[j, 0])
    assert T[0, 0] < 1.01 and T[-1, 0] > 0.99   # temperature jumps at the walls


def test_closed_box_relaxes_to_the_wall_temperature():
    n, ny, nx, tau, Tw = 4, 16, 4, 0.5, 1.05
    L = oracle.Lattice(nx, ny, kn=tau / ny, n_low=n, n_high=n, eq_low=2, thermal=True, T_wall=(Tw, Tw))
    L.init_equilibrium(1.0, 0.0, 0.0, 1.0)
    L.step(int(20 * ny * ny / (np.pi ** 2 * tau) / L.dt))
    f = L.get_populations(0)
    rho = f.sum(axis=0)
    rb = rho.mean()
    cx, cy, w = oracle.vset(n)
    S = w * (1 + 0.5 * (Tw - 1) * (cx ** 2 + cy ** 2 - 2))   # Eq. (demoeq) at rest, rho = 1
    assert np.abs(rho / rb - 1).max() < 1e-12
    np.testing.assert_allclose(f, np.broadcast_to(rb * S[:, None, None], f.shape), rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("n,eq,scale", [(4, 3, 1.2), (3, 2, 1.0)])
def test_shear_viscosity_at_constant_pressure(n, eq, scale):
    """Shear wave at T = 1.2, rho = 1/1.2 (p = 1) with tau = tau0 rho_ref / p:
    its viscosity over that at T = 1 is T for a set resolving the third
    moment (mu = tau p), 1 for D2Q9 (mu = tau rho)."""
    nus = []
    for Tm in (1.0, 1.2):
        nx, ny, tau0 = 4, 63, 0.5
        L = oracle.Lattice(nx, ny, kn=tau0 / ny, n_low=n, n_high=n, eq_low=eq, thermal=True,
                           ybc=oracle.YBC_PERIODIC, tau_mode=oracle.TAU_RHO)
        y = np.arange(ny + 1)
        k = 2 * np.pi / (ny + 1)
        L.init_equilibrium(1 / Tm, 1e-4 * np.sin(k * y)[:, None] * np.ones((1, nx)), 0.0, Tm)
        chunk = int(0.05 / ((tau0 + L.dt / 2) * Tm * k * k) / L.dt)
        ts, amp = [], []
        for s in range(20):
            L.step(chunk)
            _, ux, _ = L.moments()
            ts.append((s + 1) * chunk * L.dt)
            amp.append(2 * np.mean(ux[:, 0] * np.sin(k * y)))
        nus.append(-np.polyfit(ts[8:], np.log(amp[8:]), 1)[0] / (k * k))
    assert abs(nus[1] / nus[0] / scale - 1) < 5e-3, nus


def test_interpolation_interface_carries_the_average_temperature():
    nx, ny = 4, 24
    L = oracle.Lattice(nx, ny, kn=0.05, n_low=3, n_high=4, eq_low=2, eq_high=3, thermal=True,
                       iface=oracle.IFACE_PAPER, T_wall=(1.1, 0.95), u_wall=((0.05, 0.0), (-0.05, 0.0)))
    L.set_regions(5, 5)
    L.init_equilibrium(1.0, 0.0, 0.0, 1.0)
    L.step(200)
    T, _, _ = L.thermal_moments()
    rho, ux, uy = L.moments()
    for jI, jl, jh in [(5, 6, 4), (ny - 5, ny - 6, ny - 4)]:
        for fld in (T, rho, ux, uy):
            assert abs(fld[jI, 0] - 0.5 * (fld[jl, 0] + fld[jh, 0])) < 1e-14
    assert abs(T[5, 0] - 1.0) > 1e-3   # the walls have heated / cooled the gas


@pytest.mark.parametrize("n,eq", [(3, 2), (6, 4)])
def test_thermal_indicator(n, eq):
    """Zero at equilibrium (any T); a traceless stress or a heat flux added by
    hand shows up as |P_ij - p delta_ij| / p or |q| / (p sqrt(T))."""
    nx, ny = 4, 6
    L = oracle.Lattice(nx, ny, kn=0.1, n_low=n, n_high=n, eq_low=eq, thermal=True,
                       ybc=oracle.YBC_PERIODIC)
    rho, T = 1.3, 1.2
    L.init_equilibrium(rho, 0.0, 0.0, T)
    assert np.abs(L.indicator()).max() < 1e-14
    f = L.get_populations(0)
    a = np.zeros((n, n))
    a[2, 0], a[0, 2] = 0.01, -0.01      # P_xx - p = 0.01, P_yy - p = -0.01
    a[1, 2] = 0.03                       # q_x = 0.015
    d = oracle.from_coeffs(n, a)
    f[:, 2, 1] += d
    L.set_populations(0, f)
    B = L.indicator()
    p = rho * T
    assert abs(B[2, 1] - max(0.01 / p, 0.015 / (p * np.sqrt(T)))) < 1e-14
    assert np.abs(np.delete(B.reshape(-1), 2 * nx + 1)).max() < 1e-14


@pytest.mark.parametrize("iface", [oracle.IFACE_HERMITE, oracle.IFACE_PAPER])
def test_coupled_lattice_keeps_the_wall_maxwellian(iface):
    """Gas at rest at the walls' temperature is the uniform Maxwellian in
    either set: the coupled step (interface included) and a region change
    must leave it exactly as it is."""
    nx, ny, Tw = 6, 20, 1.2
    L = oracle.Lattice(nx, ny, kn=0.1, n_low=3, n_high=6, eq_low=2, eq_high=4, thermal=True,
                       T_wall=(Tw, Tw), iface=iface)
    L.set_regions(4, 4)
    L.init_equilibrium(0.9, 0.0, 0.0, Tw)
    L.step(20)
    if iface == oracle.IFACE_HERMITE:
        L.update_regions(7, 3)
        L.step(20)
    feq = [oracle.equilibrium(n, e, 0.9, 0.0, 0.0, T=Tw) for n, e in ((3, 2), (6, 4))]
    reg = L.region()
    for s in (0, 1):
        f = L.get_populations(s)
        mask = (reg == s) | ((reg == oracle.REG_IFACE) if s == 0 else False)
        got = f[:, mask]
        np.testing.assert_allclose(got, np.broadcast_to(feq[s][:, None], got.shape), rtol=0, atol=1e-14)
