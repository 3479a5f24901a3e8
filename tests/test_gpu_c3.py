"""Full-size pressure-driven channel (4096 x 257) against the FP64 oracle.

The oracle's state after 500 steps, a re-decomposition from the switching
indicator and 250 more steps is stored by tests/golden/make_c3_oracle.py
(the oracle alone computes it; the case is described there).  Here the GPU
runs the same case through the C ABI in the benchmark's launch
configuration (autotuned work shape) and is compared on:
  * the band map after the re-decomposition (theta 0.002: bands of 8 to 24
    rows), bit for bit for FP64 storage (the oracle's indicator values
    nearest to theta are stored, to size the guard band of the switching
    rule); the FP32 run takes the oracle's bands;
  * density and velocity at the stored columns (every 61st column and the
    8 next to each pressure boundary), relative L2 error: 1e-10 for FP64
    storage, 1e-5 for FP32 (stored as f - w s(i), s the imposed density
    ramp per group of 60 columns: 2.0e-6 measured; with a uniform s = 1 the
    stored deviations carried the ramp and the error was 1.5e-4);
  * the FP64 sums of rho, rho ux, rho uy over all nodes (FP64: 1e-12
    relative; they cover every node, not only the sampled columns).
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_oracle.npz")


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1007_4895_amd import lb as m
    m.lib()
    return m


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_c3_full_size_against_oracle(lb, storage, tol):
    g = np.load(GOLDEN)
    nx, ny = 4096, 256
    s1, s2 = (int(v) for v in g["steps"])
    print(f"c3 full size {storage}: {s1} + {s2} steps", flush=True)
    p = lb.make_params(nx, ny, kn=0.2, n_low=3, eq_low=2, n_high=6, eq_high=4, storage=storage,
                       xbc=lb.XBC_PRESSURE, rho_in=2.0, rho_out=1.0, tau_mode=lb.TAU_RHO, dt=float(g["dt"]),
                       tile_w=64)
    G = lb.Lattice(p)
    G.set_regions(8, 8)
    xx = np.arange(nx)[None, :] * np.ones((ny + 1, 1))
    G.init_equilibrium(2.0 - 1.0 * xx / (nx - 1), 0 * xx, 0 * xx)
    G.autotune(20)
    G.step(s1)
    if storage == "f64":
        # the GPU's own indicator and band rule: FP64 arithmetic on FP64
        # populations agrees with the oracle's to ~1e-15, far inside the
        # distance of the oracle's nearest indicator value to theta
        assert float(g["near_theta_rel"][0]) > 1e-12
        G.update_regions(0.002, 8, 64)
        lo, hi = G.get_regions()
        np.testing.assert_array_equal(lo, g["blo"])
        np.testing.assert_array_equal(hi, g["bhi"])
    else:
        # FP32 storage moves the indicator by ~1e-5 of theta, more than the
        # oracle's nearest values lie from it (stored): the FP32 run takes
        # the oracle's bands, converting switched nodes the same way
        G.change_regions(g["blo"], g["bhi"])
    G.step(s2)
    r, ux, uy = G.moments()
    cols = g["cols"]
    num = np.sqrt(np.sum((ux[:, cols] - g["ux"]) ** 2 + (uy[:, cols] - g["uy"]) ** 2))
    e_u = num / np.sqrt(np.sum(g["ux"] ** 2 + g["uy"] ** 2))
    e_r = np.max(np.abs(r[:, cols] - g["rho"]))
    print(f"c3 full size {storage}: velocity error {e_u:.3e}, density error {e_r:.3e}", flush=True)
    assert e_u < tol and e_r < tol
    if storage == "f64":
        sums = G.conservation()
        np.testing.assert_allclose(sums, g["sums"], rtol=1e-12, atol=1e-12 * abs(g["sums"][0]))
