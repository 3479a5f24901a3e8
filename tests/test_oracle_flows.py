"""Flow-level pins of the oracle (no GPU): Navier-Stokes limits and exact
steady-state invariants of the discrete scheme.

* Shear-wave decay on a periodic lattice: the Chapman-Enskog viscosity of the
  forward-Euler BGK update (Sec. 3.1) is nu = (tau + dt/2) c_s^2 with c_s = 1
  in units of sqrt(R T0).
* Steady Couette (Sec. 3.4): point antisymmetry, a steady velocity, the
  flux-form x-momentum balance of every row inside a band (exact to
  round-off), and the Navier-Stokes shear stress in the core.  Mass itself
  drifts slowly in coupled runs: the interface is not conservative.
* Steady Poiseuille: the face flux changes by dt rho g per row (exact steady
  momentum balance) and the core profile is the Navier-Stokes parabola with
  curvature -g / nu.
"""
import numpy as np
import pytest


def _face_flux_x_momentum(oracle, n, f, dt, rows):
    """Pi_{j+1/2} = sum_alpha xi_x nu_y F_{alpha, j+1/2} for faces j in rows
    (stencil rows j-1..j+2 must all hold set-n populations); column 0."""
    cx, cy, w = oracle.vset(n)
    out = []
    for j in rows:
        s = 0.0
        for a in range(n * n):
            nuy = cy[a] * dt
            if nuy == 0.0:
                continue
            F = oracle.face_value(nuy, f[a, j - 1, 0], f[a, j, 0], f[a, j + 1, 0], f[a, j + 2, 0])
            s += cx[a] * nuy * F
        out.append(s)
    return np.array(out)


@pytest.mark.parametrize("n,N", [(3, 2), (4, 3), (6, 4)])
def test_shear_wave_viscosity(oracle, n, N):
    nrow, tau = 256, 2.0
    L = oracle.Lattice(4, nrow - 1, kn=tau / (nrow - 1), n_low=n, n_high=n, eq_low=N,
                       ybc=oracle.YBC_PERIODIC)
    y = np.arange(nrow)[:, None] * np.ones((1, 4))
    k = 2 * np.pi / nrow
    L.init_equilibrium(1.0, 1e-3 * np.sin(k * y), 0.0 * y)
    L.step(100)

    def amp():
        _, ux, _ = L.moments()
        return 2 * np.mean(ux[:, 0] * np.sin(k * y[:, 0]))

    a0, t0 = amp(), L.steps * L.dt
    L.step(2000)
    a1, t1 = amp(), L.steps * L.dt
    nu = -np.log(a1 / a0) / (k * k * (t1 - t0))
    assert abs(nu / (tau + 0.5 * L.dt) - 1) < 0.01, nu


def test_couette_c1_steady_invariants(oracle):
    # D2Q16 (3rd-order equilibrium) in 8 rows at each wall, D2Q9 core,
    # Hermite interface, walls at -/+0.05, Kn = 0.1, 20k steps (steady)
    L = oracle.Lattice(4, 64, kn=0.1, n_low=3, n_high=4, eq_low=2, eq_high=3,
                       u_wall=((-0.05, 0.0), (0.05, 0.0)))
    L.set_regions(8, 8)
    L.init_equilibrium()
    L.step(20000)
    r, ux, uy = L.moments()
    u = ux[:, 0]
    # point antisymmetry of the steady state
    assert np.max(np.abs(u + u[::-1])) < 1e-12
    assert np.max(np.abs(r[:, 0] - r[::-1, 0])) < 1e-12
    assert np.max(np.abs(ux - ux[:, :1])) == 0.0
    # profile is monotone and bounded by the wall speeds (slip at the walls)
    assert np.all(np.diff(u) > 0) and u[0] > -0.05 and u[-1] < 0.05
    # flux form: inside a band, the x-momentum change of row j equals the
    # difference of the face fluxes (the collision conserves momentum)
    f9, f16 = L.get_populations(0), L.get_populations(1)
    cx9, _, _ = oracle.vset(3)
    cx16, _, _ = oracle.vset(4)
    L.step(1)
    g9, g16 = L.get_populations(0), L.get_populations(1)
    for n, f, g, cx, rows in ((3, f9, g9, cx9, range(10, 54)), (4, f16, g16, cx16, range(2, 6))):
        Pi = _face_flux_x_momentum(oracle, n, f, L.dt, range(rows.start - 1, rows.stop))
        dmom = np.einsum("a,aj->j", cx, (g - f)[:, list(rows), 0])
        np.testing.assert_allclose(dmom, -(Pi[1:] - Pi[:-1]), rtol=0, atol=2e-16)
    # the velocity is steady
    L.step(999)
    u2 = L.moments()[1][:, 0]
    assert np.max(np.abs(u2 - u)) < 1e-13
    # the core momentum flux is the Navier-Stokes shear stress
    # -(tau + dt/2) rho du/dy (viscosity of the forward-Euler update)
    Pi = _face_flux_x_momentum(oracle, 3, f9, L.dt, range(20, 45))
    tau = 0.1 * 64
    slope = np.polyfit(np.arange(20, 45), u[20:45], 1)[0]
    rho = r[32, 0]
    assert abs(Pi.mean() / L.dt / (-(tau + L.dt / 2) * rho * slope) - 1) < 0.02


def test_poiseuille_steady_balance_and_parabola(oracle):
    ny, kn, g = 24, 0.1, 1e-5
    L = oracle.Lattice(4, ny, kn=kn, n_low=3, n_high=3, eq_low=2, gx=g)
    L.init_equilibrium()
    L.step(12000)
    r, ux, _ = L.moments()
    f = L.get_populations(0)
    faces = range(1, ny - 2)
    Pi = _face_flux_x_momentum(oracle, 3, f, L.dt, faces)
    # row j = face j+1/2 minus face j-1/2 = dt rho_j g, for rows 2..ny-3
    d = np.diff(Pi)
    rows = np.arange(2, ny - 2)
    np.testing.assert_allclose(d, L.dt * r[rows, 0] * g, rtol=1e-8)
    # Navier-Stokes parabola: curvature -g / nu with nu = tau + dt/2
    u = ux[:, 0]
    yy = np.arange(ny + 1)
    c = np.polyfit(yy[3:-3], u[3:-3], 2)
    resid = u[3:-3] - np.polyval(c, yy[3:-3])
    assert np.max(np.abs(resid)) < 1e-3 * u.max()
    nu = kn * ny + 0.5 * L.dt
    assert abs(2 * c[0] / (-g / nu) - 1) < 0.01
