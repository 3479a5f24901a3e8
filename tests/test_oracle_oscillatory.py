"""Pins of the oracle's oscillating wall (oscillatory Couette flow, Sec. 3.5;
no GPU).

The bottom plate moves along x with u_w sin(omega t), the top plate is at
rest.  In the continuum limit the periodic state is Stokes' solution for a
plate oscillating under a parallel wall at distance H,
    u(y, t) = Im[u_w e^{i omega t} sinh(k (H - y)) / sinh(k H)],
    k = (1 + i) sqrt(omega / (2 nu)),
with the viscosity nu = tau + dt/2 of the forward-Euler update (pinned by
the shear-wave test).  The lattice solution differs from it by the wall slip,
which is first order in Kn: halving Kn at a fixed Stokes number
beta = sqrt(omega H^2 / nu) must halve the deviation.  A plate moving the
other way gives the mirror-image flow.
"""
import numpy as np
import pytest


def _stokes_run(oracle, ny, kn, beta, uw):
    dt = oracle.default_dt(3)
    nu = kn * ny + 0.5 * dt
    om = beta * beta * nu / (ny * ny)
    L = oracle.Lattice(4, ny, kn=kn, n_low=3, n_high=3, eq_low=2, u_osc=uw, omega_osc=om)
    L.init_equilibrium()
    nper = int(round(2 * np.pi / om / dt))
    L.step(3 * nper)
    y = np.arange(ny + 1)
    k = (1 + 1j) * np.sqrt(om / (2 * nu))
    err_all, err_core = 0.0, 0.0
    for _ in range(8):
        L.step(nper // 8)
        t = L.steps * dt
        ua = np.imag(uw * np.exp(1j * om * t) * np.sinh(k * (ny - y)) / np.sinh(k * ny))
        d = np.abs(L.moments()[1][:, 0] - ua) / uw
        err_all = max(err_all, float(d.max()))
        err_core = max(err_core, float(d[ny // 4: 3 * ny // 4].max()))
    return err_all, err_core


def test_oscillating_plate_converges_to_stokes_solution(oracle):
    e1, c1 = _stokes_run(oracle, 64, 0.01, 4.0, 0.02)
    e2, c2 = _stokes_run(oracle, 64, 0.005, 4.0, 0.02)
    assert e2 < 0.035 and c2 < 0.01, (e2, c2)
    # first-order slip: the deviation halves with Kn
    assert 1.6 < e1 / e2 < 2.6, (e1, e2)


def test_oscillating_plate_mirror_symmetry(oracle):
    # coupled D2Q9/D2Q36: reversing the plate's motion mirrors the flow
    kw = dict(kn=0.05, n_low=3, n_high=6, eq_low=2, eq_high=4, omega_osc=2e-3)
    A = oracle.Lattice(4, 30, u_osc=0.03, **kw)
    B = oracle.Lattice(4, 30, u_osc=-0.03, **kw)
    for L in (A, B):
        L.set_regions(5, 5)
        L.init_equilibrium()
        L.step(400)
    ra, ua, va = A.moments()
    rb, ub, vb = B.moments()
    assert np.max(np.abs(ua)) > 1e-3
    np.testing.assert_allclose(ub, -ua, rtol=0, atol=1e-15)
    np.testing.assert_allclose(rb, ra, rtol=0, atol=1e-15)
