"""Seeded synthetic inputs and workload recipes.

This module holds none of the method's arithmetic: it only draws seeded
random numbers (smooth density/velocity fields, noise arrays) and states the
sizes and parameters of the channel-flow workloads.  Both the GPU path and
the CPU oracle are fed from here.

Workloads (all synthetic: the paper's cases are analytic channel flows):
  couette_c1   planar Couette, nx = 4 (periodic) x ny = 64, walls -/+0.05,
               Kn = 0.1, D2Q16 (3rd-order equilibrium) in 8 rows at each
               wall, D2Q9 core, Hermite interface, FP64, 20k steps.
  poiseuille_c2  body-force channel nx = 1024 x ny = 512, g = 1e-6,
               Kn in {0.01, 0.05, 0.1}, D2Q36 (4th order) in 64 rows at each
               wall, D2Q9 elsewhere, FP32, 10k steps; all-D2Q36 comparison.
               Courant number 0.35 per axis for the fastest abscissa, inside
               the unsplit update's limit for flows that vary in x and y.
  pressure_c3  pressure-driven channel nx = 4096 x ny = 256, rho_in/rho_out
               = 2, outlet Kn = 0.2 (relaxation time ~ 1/rho), bands per
               64-column tile from the non-equilibrium indicator every 500
               steps, FP32 or BF16 storage.
  osc_couette  oscillatory Couette flow (Sec. 3.5): nx = 8 (periodic) x
               ny = 100, bottom plate moving along x with u_w sin(omega t),
               u_w = 0.05, top plate at rest, Stokes number
               beta = sqrt(omega H^2 / nu) = 4 with nu = Kn H (the BGK
               viscosity mu / rho = tau), Kn in {0.0178, 0.1, 0.3}; the
               low-order set in the middle 70 % (bands of 15 rows at each
               wall), M-D2Q9-36 and M-D2Q16-36 against all-D2Q36, FP64.
  kramers      Kramers' problem (Sec. 3.3): nx = 8 (periodic), a plate at
               rest on row 0 and a shear rate s = 1e-4 imposed above row
               ny = 400 = 200 mean free paths (lambda = tau = 2 nodes,
               Kn = 0.005 of the 400-node height), D2Q36 within 10 lambda
               of the plate (20 rows), D2Q9 beyond; started from the
               far-field shear flow, FP64.
  thermal_couette  thermal Couette channel, the C2 geometry (nx = 1024 x
               ny = 512): walls moving -/+0.05 at temperatures 1.05 / 0.95,
               Kn = 0.01, thermal D2Q36 (4th order) in 64 rows at each wall,
               thermal D2Q9 core, FP32, Courant 0.35, started at rest at
               T = 1.  Physics
               check on an x-uniform channel nx = 4 x ny = 128, Kn = 0.05,
               16-row bands: steady conduction (walls at rest, T 1.02 /
               0.98) and shear heating (walls -/+0.1 at T = 1), M-D2Q9-36
               and M-D2Q16-36 against all-D2Q36, FP64.
  batch_c5     128 independent channels, nx = 8 (periodic), ny uniform in
               [32, 512], Kn log-spaced in [0.01, 1], near-wall bands of
               8-64 rows (at most a third of the channel), velocity-set
               pairs D2Q9/D2Q16, D2Q9/D2Q36 and D2Q16/D2Q36 in turn,
               Couette and Poiseuille alternating, FP32, Courant 0.35,
               stepped as one batch in graph-captured segments of 5000
               steps.
"""
from __future__ import annotations

import numpy as np

D2Q9, D2Q16, D2Q36 = 3, 4, 6   # Gauss-Hermite points per axis


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def smooth_fields(nx: int, nrow: int, seed: int, rho_amp=0.02, u_amp=0.03, modes=3,
                  x_uniform=False):
    """rho, ux, uy on [nrow][nx]: 1 + / 0 + a few random low-wavenumber
    sinusoids (periodic in x; in y over nrow rows)."""
    g = rng(seed)
    y, x = np.mgrid[0:nrow, 0:nx].astype(np.float64)
    out = []
    for base, amp in ((1.0, rho_amp), (0.0, u_amp), (0.0, u_amp)):
        f = np.full((nrow, nx), base)
        for _ in range(modes):
            kx = 0 if x_uniform else int(g.integers(0, 3))
            ky = int(g.integers(1, 3))
            ph = g.uniform(0, 2 * np.pi, 2)
            a = amp * g.uniform(0.3, 1.0) / modes
            f = f + a * np.cos(2 * np.pi * kx * x / nx + ph[0]) * np.sin(np.pi * ky * y / max(nrow - 1, 1) + ph[1])
        out.append(f)
    return out


def noise(shape, seed: int, amp: float):
    """Uniform noise in [-amp, amp]."""
    return amp * rng(seed).uniform(-1.0, 1.0, shape)


def tile_bands(ntiles: int, seed: int, lo: int, hi: int):
    """Per-tile band widths, uniform integers in [lo, hi]."""
    g = rng(seed)
    return g.integers(lo, hi + 1, ntiles).astype(np.int32), g.integers(lo, hi + 1, ntiles).astype(np.int32)


COUETTE_C1 = dict(nx=4, ny=64, kn=0.1, n_low=D2Q9, n_high=D2Q16, eq_low=2, eq_high=3,
                  u_wall=((-0.05, 0.0), (0.05, 0.0)), bands=(8, 8), storage="f64", steps=20000)

POISEUILLE_C2 = dict(nx=1024, ny=512, kn=0.05, kn_sweep=(0.01, 0.05, 0.1), n_low=D2Q9, n_high=D2Q36,
                     eq_low=2, eq_high=4, gx=1e-6, bands=(64, 64), cfl=0.35, storage="f32", steps=10000)

PRESSURE_C3 = dict(nx=4096, ny=256, kn=0.2, n_low=D2Q9, n_high=D2Q36, eq_low=2, eq_high=4,
                   rho_in=2.0, rho_out=1.0, tile_w=64, theta=0.01, bmin=8, bmax=64, regrid=500,
                   cfl=0.3, storage="f32", steps=20000)

OSC_COUETTE = dict(nx=8, ny=100, kn=0.0178, kn_sweep=(0.0178, 0.1, 0.3), u_osc=0.05, beta=4.0,
                   bands=(15, 15), pairs=((3, 2, 6, 4), (4, 3, 6, 4)), storage="f64", periods=3)

KRAMERS = dict(nx=8, ny=400, kn=0.005, shear=1e-4, band=20, storage="f64")

THERMAL_COUETTE = dict(nx=1024, ny=512, kn=0.01, n_low=D2Q9, n_high=D2Q36, eq_low=2, eq_high=4,
                       u_wall=((-0.05, 0.0), (0.05, 0.0)), T_wall=(1.05, 0.95), bands=(64, 64), cfl=0.35,
                       storage="f32",
                       physics=dict(nx=4, ny=128, kn=0.05, bands=16, steps=80000, storage="f64",
                                    pairs=((3, 2, 6, 4), (4, 3, 6, 4)),
                                    cases={"conduction": dict(u_wall=((0.0, 0.0), (0.0, 0.0)), T_wall=(1.02, 0.98)),
                                           "shear_heating": dict(u_wall=((-0.1, 0.0), (0.1, 0.0)),
                                                                 T_wall=(1.0, 1.0))}))

BATCH_C5 = dict(count=128, nx=8, ny_range=(32, 512), kn_range=(0.01, 1.0), band_range=(8, 64),
                pairs=((3, 2, 4, 3), (3, 2, 6, 4), (4, 3, 6, 4)), u_wall=0.05, gx=1e-6, cfl=0.35, storage="f32",
                segment=5000, seed=51)


def batch_cases(c=BATCH_C5, count=None):
    """Seeded case list of the batch workload: per channel nx, ny, kn,
    bands, velocity-set pair, wall velocities and body force."""
    g = rng(c["seed"])
    n = c["count"] if count is None else count
    kns = np.geomspace(c["kn_range"][0], c["kn_range"][1], n)
    nys = g.integers(c["ny_range"][0], c["ny_range"][1] + 1, n)
    bands = g.integers(c["band_range"][0], c["band_range"][1] + 1, n)
    out = []
    for k in range(n):
        ny = int(nys[k])
        b = int(min(bands[k], ny // 3))
        nl, el, nh, eh = c["pairs"][k % len(c["pairs"])]
        couette = k % 2 == 0
        out.append(dict(nx=c["nx"], ny=ny, kn=float(kns[k]), n_low=nl, eq_low=el, n_high=nh, eq_high=eh,
                        bands=(b, b), storage=c["storage"], cfl=c["cfl"],
                        u_wall=((-c["u_wall"], 0.0), (c["u_wall"], 0.0)) if couette else ((0.0, 0.0), (0.0, 0.0)),
                        gx=0.0 if couette else c["gx"]))
    return out
