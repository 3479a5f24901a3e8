#!/usr/bin/env python3
"""Writes c3_oracle.npz: the FP64 oracle's state of the full-size pressure-
driven channel after 500 steps, a re-decomposition from the switching
indicator (Sec. 2.2), and 250 more steps.

Case (the pressure channel workload): 4096 x 257 nodes, walls at rows 0 and
256 (diffuse, at rest), pressure boundary columns with rho_in = 2 and
rho_out = 1 (equilibrium at the prescribed density with the edge node's
velocity plus its non-equilibrium part), relaxation time Kn ny rho_ref / rho
with Kn = 0.2 at rho_ref = 1 (Eq. dbgk with fixed viscosity), D2Q9 (order 2)
core and D2Q36 (order 4) bands per 64-column tile, Hermite interface,
per-axis Courant number 0.3.  Start: equilibrium at rest with a density
falling linearly from rho_in at column 0 to rho_out at column 4095, bands of
8 rows at each wall.  At step 500 the bands are recomputed from the
indicator (theta 0.002, clamped to [8, 64] rows: bands of 8 to 24 rows) and switched nodes are
converted by the Hermite projection; then 250 more steps.

Only the oracle computes here.  Stored: the sampled columns, the bands after
the re-decomposition, the oracle's indicator values nearest to theta (to
size the guard band of the map comparison), rho / ux / uy at the sampled
columns after 750 steps, and the FP64 sums of rho, rho ux, rho uy over every
node.  Run from the repository root:
    python tests/golden/make_c3_oracle.py
(OpenMP over rows; the result does not depend on the thread count.)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

NX, NY, KN = 4096, 256, 0.2
RHO_IN, RHO_OUT = 2.0, 1.0
THETA, BMIN, BMAX, TILE = 0.002, 8, 64, 64
STEPS1, STEPS2 = 500, 250
CFL = 0.3
COLS = np.unique(np.concatenate([np.arange(0, 8), np.arange(8, NX - 8, 61), np.arange(NX - 8, NX)]))
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle.npz")


def main():
    x, _ = oracle.gh_rule(6)
    dt = CFL / float(np.max(x))
    L = oracle.Lattice(NX, NY, kn=KN, n_low=3, eq_low=2, n_high=6, eq_high=4, dt=dt, xbc=oracle.XBC_PRESSURE,
                       rho_in=RHO_IN, rho_out=RHO_OUT, tau_mode=oracle.TAU_RHO, tile_w=TILE)
    L.set_regions(BMIN, BMIN)
    xx = np.arange(NX)[None, :] * np.ones((NY + 1, 1))
    L.init_equilibrium(RHO_IN - (RHO_IN - RHO_OUT) * xx / (NX - 1), 0 * xx, 0 * xx)
    t0 = time.time()
    for k in range(STEPS1 // 50):
        L.step(50)
        print(f"step {L.steps}  {time.time() - t0:.0f} s", flush=True)
    B = L.indicator()
    blo, bhi = L.bands_from_indicator(B, THETA, BMIN, BMAX)
    near = np.sort(np.abs(B.ravel() - THETA))[:16] / THETA
    L.update_regions(blo, bhi)
    for k in range(STEPS2 // 50):
        L.step(50)
        print(f"step {L.steps}  {time.time() - t0:.0f} s", flush=True)
    r, ux, uy = L.moments()
    sums = L.conservation()
    np.savez_compressed(OUT, cols=COLS, blo=blo, bhi=bhi, near_theta_rel=near, rho=r[:, COLS], ux=ux[:, COLS],
                        uy=uy[:, COLS], sums=sums, steps=np.array([STEPS1, STEPS2]), dt=np.array(dt),
                        threads=np.array(oracle.threads()))
    print(f"wrote {OUT}: bands lo {blo.min()}..{blo.max()}, hi {bhi.min()}..{bhi.max()}; "
          f"closest indicator to theta: {near[0]:.3e} theta", flush=True)


if __name__ == "__main__":
    main()
