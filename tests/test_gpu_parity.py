"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances: FP64 storage 1e-10 relative (rounding order, FMA contraction and
the minmod form of the limiter differ from the oracle, nothing else); FP32
(weight-shifted) storage 1e-5 relative velocity error.  Sizes span several
64-column waves with a ragged tail, and the full channel sizes in the
launch configuration of the benchmark.
"""
import numpy as np
import pytest

from paper_1007_4895_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1007_4895_amd import lb as m
    m.lib()
    return m


def pair(oracle, lb, nx, ny, *, storage="f64", bands=(0, 0), strip=0, dt=None, **kw):
    """Oracle and GPU lattices with identical parameters and dt."""
    n_hi = max(kw.get("n_low", 3), kw.get("n_high", kw.get("n_low", 3)))
    if dt is None:
        cfl = kw.pop("cfl", 0.5)
        x, _ = oracle.gh_rule(n_hi)
        dt = cfl / float(np.max(x))
    else:
        kw.pop("cfl", None)
    okw = dict(kw)
    for k in ("tile_w",):
        if okw.get(k, None) == 0:
            okw.pop(k)
    O = oracle.Lattice(nx, ny, dt=dt, **okw)
    G = lb.Lattice(lb.make_params(nx, ny, storage=storage, dt=dt, **kw))
    if strip:
        G.set_strip_rows(strip)
    O.set_regions(*bands)
    G.set_regions(*bands)
    return O, G


def rel_u(ux_a, uy_a, ux_b, uy_b, mask=None):
    if mask is None:
        mask = np.ones(ux_a.shape, bool)
    num = np.sqrt(np.sum((ux_a - ux_b)[mask] ** 2 + (uy_a - uy_b)[mask] ** 2))
    den = np.sqrt(np.sum(ux_b[mask] ** 2 + uy_b[mask] ** 2))
    return num / den


def pop_err(G, O, which):
    g, o = G.get_populations(which), O.get_populations(which)
    m = ~np.isnan(g[0])
    return np.max(np.abs(g[:, m] - o[:, m])) / np.max(np.abs(o[:, m])), m.sum()


# ------------------------------------------------------------ single sets
@pytest.mark.parametrize("n,N", [(3, 2), (4, 3), (6, 4)])
def test_single_set_periodic_2d(oracle, lb, n, N):
    # 150 columns = 2 full waves + a ragged 22-column tail; fully periodic
    # 2D data (Courant 0.3); non-equilibrium start from seeded noise
    nx, ny = 150, 19
    O, G = pair(oracle, lb, nx, ny, n_low=n, n_high=n, eq_low=N, kn=0.2, gx=2e-4, gy=-1e-4,
                ybc=oracle.YBC_PERIODIC, cfl=0.3)
    rho, ux, uy = W.smooth_fields(nx, ny + 1, seed=11, rho_amp=0.05, u_amp=0.05)
    O.init_equilibrium(rho, ux, uy)
    f = O.get_populations(0) * (1 + W.noise((n * n, ny + 1, nx), seed=12, amp=0.01))
    O.set_populations(0, f)
    G.set_populations(0, f)
    e0, cnt = pop_err(G, O, 0)
    assert cnt == nx * (ny + 1) and e0 < 1e-15
    for k in (1, 4, 25):
        O.step(k)
        G.step(k)
        e, _ = pop_err(G, O, 0)
        assert e < 1e-12, (k, e)
    _, uxo, uyo = O.moments()
    _, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-11


@pytest.mark.parametrize("n,N", [(3, 2), (6, 4)])
def test_single_set_walls_force(oracle, lb, n, N):
    # moving diffuse walls, body force, 2D start; 70 columns (ragged wave)
    nx, ny = 70, 24
    O, G = pair(oracle, lb, nx, ny, n_low=n, n_high=n, eq_low=N, kn=0.1, gx=1e-4,
                u_wall=((0.03, 0.0), (-0.02, 0.0)), cfl=0.3)
    rho, ux, uy = W.smooth_fields(nx, ny + 1, seed=21)
    O.init_equilibrium(rho, ux, uy)
    G.init_equilibrium(rho, ux, uy)
    O.step(60)
    G.step(60)
    e, _ = pop_err(G, O, 0)
    assert e < 1e-11
    r_o, uxo, uyo = O.moments()
    r_g, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-10
    assert np.max(np.abs(r_g - r_o)) < 1e-12


# ---------------------------------------------------------------- coupled
@pytest.mark.parametrize("lo,hi", [((3, 2), (4, 3)), ((3, 2), (6, 4)), ((4, 3), (6, 4))])
def test_coupled_hermite_2d(oracle, lb, lo, hi):
    nx, ny = 130, 40
    O, G = pair(oracle, lb, nx, ny, n_low=lo[0], eq_low=lo[1], n_high=hi[0], eq_high=hi[1], kn=0.08,
                gx=5e-5, u_wall=((-0.03, 0.0), (0.03, 0.0)), bands=(7, 9), cfl=0.3)
    rho, ux, uy = W.smooth_fields(nx, ny + 1, seed=31)
    O.init_equilibrium(rho, ux, uy)
    G.init_equilibrium(rho, ux, uy)
    for k in (1, 30):
        O.step(k)
        G.step(k)
        for s in (0, 1):
            e, _ = pop_err(G, O, s)
            assert e < 1e-11, (k, s, e)
    r_o, uxo, uyo = O.moments()
    r_g, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-10


def test_coupled_periodic_y_tile_bands(oracle, lb):
    # periodic in both directions with high-set bands that differ per tile:
    # row images and Hermite projection entries in the same step (one
    # launch for both), projection sources found across the y wrap
    nx, ny, tw = 130, 40, 64
    O, G = pair(oracle, lb, nx, ny, n_low=3, eq_low=2, n_high=6, eq_high=4, kn=0.08, gx=5e-5, gy=-2e-5,
                ybc=oracle.YBC_PERIODIC, tile_w=tw, bands=(5, 5), cfl=0.3)
    rho, ux, uy = W.smooth_fields(nx, ny + 1, seed=37)
    O.init_equilibrium(rho, ux, uy)
    G.init_equilibrium(rho, ux, uy)
    lo, hi = np.array([4, 0, 7], np.int32), np.array([2, 6, 0], np.int32)
    O.update_regions(lo, hi)
    G.change_regions(lo, hi)
    for k in (1, 25):
        O.step(k)
        G.step(k)
        for s in (0, 1):
            e, m = pop_err(G, O, s)
            assert m > 0 and e < 1e-11, (k, s, e)
    r_o, uxo, uyo = O.moments()
    r_g, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-10


def test_couette_c1_full_run(oracle, lb):
    c = W.COUETTE_C1
    O, G = pair(oracle, lb, c["nx"], c["ny"], n_low=c["n_low"], eq_low=c["eq_low"], n_high=c["n_high"],
                eq_high=c["eq_high"], kn=c["kn"], u_wall=c["u_wall"], bands=c["bands"])
    O.init_equilibrium()
    G.init_equilibrium()
    O.step(c["steps"])
    G.step(c["steps"])
    r_o, uxo, uyo = O.moments()
    r_g, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-10
    assert np.max(np.abs(r_g - r_o)) < 1e-12
    # steady profile is antisymmetric on the GPU too
    assert np.max(np.abs(uxg[:, 0] + uxg[::-1, 0])) < 1e-12


def test_paper_interface(oracle, lb):
    nx, ny = 70, 40
    O, G = pair(oracle, lb, nx, ny, n_low=3, eq_low=2, n_high=6, eq_high=2, kn=0.1,
                iface=oracle.IFACE_PAPER, u_wall=((-0.04, 0.0), (0.04, 0.0)), bands=(6, 8), cfl=0.3)
    rho, ux, uy = W.smooth_fields(nx, ny + 1, seed=41)
    O.init_equilibrium(rho, ux, uy)
    G.init_equilibrium(rho, ux, uy)
    O.step(50)
    G.step(50)
    for s in (0, 1):
        e, _ = pop_err(G, O, s)
        assert e < 1e-11
    r_o, uxo, uyo = O.moments()
    r_g, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-10


def test_pressure_channel_tile_bands(oracle, lb):
    # pressure x-boundary, relaxation time ~ 1/rho, per-tile bands (64-column
    # tiles, differing widths -> x-neighbours across tiles in the other set)
    nx, ny = 256, 40
    lo, hi = W.tile_bands(4, seed=51, lo=3, hi=9)
    O, G = pair(oracle, lb, nx, ny, n_low=3, eq_low=2, n_high=6, eq_high=4, kn=0.2,
                xbc=oracle.XBC_PRESSURE, rho_in=1.2, rho_out=1.0, tau_mode=oracle.TAU_RHO,
                tile_w=64, bands=(lo, hi), cfl=0.3)
    x = np.arange(nx)[None, :] * np.ones((ny + 1, 1))
    rho = 1.2 - 0.2 * x / (nx - 1)
    O.init_equilibrium(rho, 0 * x, 0 * x)
    G.init_equilibrium(rho, 0 * x, 0 * x)
    O.step(40)
    G.step(40)
    for s in (0, 1):
        e, _ = pop_err(G, O, s)
        assert e < 1e-11, (s, e)
    r_o, uxo, uyo = O.moments()
    r_g, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-10


# ---------------------------------------------------------------- storage
def test_fp32_coupled_channel(oracle, lb):
    nx, ny = 130, 64
    O, G = pair(oracle, lb, nx, ny, storage="f32", n_low=3, eq_low=2, n_high=6, eq_high=4, kn=0.05,
                gx=1e-5, u_wall=((-0.02, 0.0), (0.02, 0.0)), bands=(8, 8), cfl=0.3)
    rho, ux, uy = W.smooth_fields(nx, ny + 1, seed=61, rho_amp=0.01, u_amp=0.01)
    O.init_equilibrium(rho, ux, uy)
    G.init_equilibrium(rho, ux, uy)
    O.step(300)
    G.step(300)
    _, uxo, uyo = O.moments()
    _, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-5


def test_poiseuille_c2_full_width_x_uniform(oracle, lb):
    # the benchmark workload at full size (1024 x 513, D2Q36 in 64 rows at each
    # wall, FP32): the flow stays bit-for-bit x-uniform, so every column is
    # checked against the oracle run at nx = 4
    c = W.POISEUILLE_C2
    steps = 2000
    x, _ = oracle.gh_rule(6)
    dt = c["cfl"] / float(np.max(x))
    kw = dict(n_low=c["n_low"], eq_low=c["eq_low"], n_high=c["n_high"], eq_high=c["eq_high"], kn=c["kn"],
              gx=c["gx"])
    G = lb.Lattice(lb.make_params(c["nx"], c["ny"], storage=c["storage"], dt=dt, **kw))
    G.set_regions(*c["bands"])
    G.init_equilibrium()
    G.step(steps)
    r_g, uxg, uyg = G.moments()
    assert np.all(uxg == uxg[:, :1]) and np.all(r_g == r_g[:, :1])
    O = oracle.Lattice(4, c["ny"], dt=dt, **kw)
    O.set_regions(*c["bands"])
    O.init_equilibrium()
    O.step(steps)
    r_o, uxo, uyo = O.moments()
    assert rel_u(uxg[:, :4], uyg[:, :4], uxo, uyo) < 1e-5


def test_poiseuille_c2_wide_4096_x_uniform(oracle, lb):
    # the benchmark's 4096-column variant of the channel (4096 x 513, whose
    # populations exceed the Infinity Cache), in the work shape its autotuner
    # picks: bit-for-bit x-uniform, so every column is checked against the
    # oracle run at nx = 4
    c = W.POISEUILLE_C2
    steps = 1000
    x, _ = oracle.gh_rule(6)
    dt = c["cfl"] / float(np.max(x))
    kw = dict(n_low=c["n_low"], eq_low=c["eq_low"], n_high=c["n_high"], eq_high=c["eq_high"], kn=0.01,
              gx=c["gx"])
    G = lb.Lattice(lb.make_params(4 * c["nx"], c["ny"], storage=c["storage"], dt=dt, **kw))
    G.set_regions(*c["bands"])
    G.set_work_shape((7, 6), (1, 1))
    G.init_equilibrium()
    G.step(steps)
    r_g, uxg, uyg = G.moments()
    assert np.all(uxg == uxg[:, :1]) and np.all(r_g == r_g[:, :1])
    O = oracle.Lattice(4, c["ny"], dt=dt, **kw)
    O.set_regions(*c["bands"])
    O.init_equilibrium()
    O.step(steps)
    r_o, uxo, uyo = O.moments()
    assert rel_u(uxg[:, :4], uyg[:, :4], uxo, uyo) < 1e-5


def test_poiseuille_c2_damps_2d_perturbations(lb):
    # the benchmark workload at full size, in the benchmark's work shape and
    # at its Courant number, started from seeded density noise of 1e-6 that
    # varies in x and y: the x-varying part decays instead of growing (at
    # Courant 0.5 the channel is stable only while it stays exactly
    # x-uniform)
    c = W.POISEUILLE_C2
    ny1 = c["ny"] + 1
    noise = 1e-6 * W.rng(11).standard_normal((ny1, c["nx"]))
    G = lb.Lattice(lb.make_params(c["nx"], c["ny"], kn=0.01, n_low=c["n_low"], eq_low=c["eq_low"],
                                  n_high=c["n_high"], eq_high=c["eq_high"], gx=c["gx"], storage=c["storage"],
                                  cfl=c["cfl"]))
    G.set_regions(*c["bands"])
    G.set_work_shape((1, 2), (1, 1))
    G.init_equilibrium(rho=1.0 + noise)
    r0, _, _ = G.moments()
    a0 = float(np.max(np.abs(r0 - r0.mean(axis=1, keepdims=True))))
    G.step(3000)
    r, ux, uy = G.moments()
    assert np.all(np.isfinite(r)) and np.all(np.isfinite(ux)) and np.all(np.isfinite(uy))
    a = float(np.max(np.abs(r - r.mean(axis=1, keepdims=True))))
    assert a < 0.05 * a0, (a, a0)


# ------------------------------------------------------- runtime properties
def test_strip_rows_invariance_and_determinism(lb):
    def run(strip):
        G = lb.Lattice(lb.make_params(200, 60, kn=0.1, n_low=3, n_high=6, eq_low=2, eq_high=4, storage="f32",
                                      gx=1e-5, cfl=0.3, u_wall=((0.01, 0.0), (-0.01, 0.0))))
        G.set_regions(10, 12)
        if strip:
            G.set_strip_rows(strip)
        rho, ux, uy = W.smooth_fields(200, 61, seed=71)
        G.init_equilibrium(rho, ux, uy)
        G.step(50)
        return G.get_populations(0), G.get_populations(1)

    a = run(0)
    for strip in (1, 5, 64):
        b = run(strip)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_sampled_kernel_timing(lb):
    # timing mode with an interval N records events around the update
    # launches of the steps whose count is divisible by N only, and the
    # populations do not depend on it
    def make():
        G = lb.Lattice(lb.make_params(200, 60, kn=0.1, n_low=3, n_high=6, eq_low=2, eq_high=4, storage="f32",
                                      gx=1e-5, cfl=0.3))
        G.set_regions(10, 12)
        G.init_equilibrium()
        G.step(4)
        return G

    A, B = make(), make()
    A.set_timing(True, every=3)
    A.step(10)                      # steps 4..13: 6, 9 and 12 are timed
    ms_h, n_h, ms_all, n_all = A.kernel_times()
    assert n_h == 3 and n_all == 3 and ms_h > 0
    A.set_timing(True)
    A.step(5)
    assert A.kernel_times()[1] == 5
    A.set_timing(False)
    B.step(15)
    np.testing.assert_array_equal(A.get_populations(0), B.get_populations(0))
    np.testing.assert_array_equal(A.get_populations(1), B.get_populations(1))
    with pytest.raises(lb.LBError):
        A.set_timing(True, every=-2)


def test_autotune_restores_state(lb):
    G = lb.Lattice(lb.make_params(256, 60, kn=0.1, n_low=3, n_high=6, eq_low=2, eq_high=4, storage="f32",
                                  gx=1e-5, u_wall=((0.01, 0.0), (-0.01, 0.0))))
    G.set_regions(12, 12)
    G.init_equilibrium()
    G.step(20)
    before = (G.get_populations(0), G.get_populations(1), G.steps)
    rows = G.autotune(5)
    assert all(r >= 1 for r in rows) and G.strip_rows() == rows
    assert G.steps == before[2]
    np.testing.assert_array_equal(G.get_populations(0), before[0])
    np.testing.assert_array_equal(G.get_populations(1), before[1])


def test_checkpoint_resume_bitwise(lb):
    def make():
        G = lb.Lattice(lb.make_params(96, 40, kn=0.1, n_low=3, n_high=4, eq_low=2, eq_high=3, storage="f32",
                                      gx=1e-5, u_wall=((0.02, 0.0), (-0.02, 0.0))))
        G.set_regions(6, 6)
        G.init_equilibrium()
        return G

    A = make()
    A.step(300)
    B = make()
    B.step(150)
    st = B.get_state()
    C = make()
    C.set_state(st)
    assert C.steps == 150
    C.step(150)
    for s in (0, 1):
        np.testing.assert_array_equal(A.get_populations(s), C.get_populations(s))


def test_conservation_periodic(lb):
    nx, ny = 128, 31
    G = lb.Lattice(lb.make_params(nx, ny, kn=0.2, n_low=4, n_high=4, eq_low=3, gx=1e-4,
                                  ybc=lb.YBC_PERIODIC, cfl=0.3))
    rho, ux, uy = W.smooth_fields(nx, ny + 1, seed=81)
    G.init_equilibrium(rho, ux, uy)
    c0 = G.conservation()
    G.step(200)
    c1 = G.conservation()
    assert abs(c1[0] - c0[0]) / c0[0] < 1e-13
    assert abs((c1[1] - c0[1]) - 200 * G.dt * 1e-4 * c0[0]) < 1e-11


def test_projection_kernel(oracle, lb):
    import torch
    rng = np.random.default_rng(91)
    for (ns, es), (nd, ed) in (((3, 2), (6, 4)), ((6, 4), (3, 2)), ((4, 3), (6, 4)), ((6, 4), (4, 3))):
        n = 37
        f = np.stack([oracle.equilibrium(ns, es, 1 + 0.05 * rng.uniform(), 0.05 * rng.uniform(-1, 1),
                                         0.05 * rng.uniform(-1, 1)) for _ in range(n)])
        f = f * (1 + 0.01 * rng.uniform(-1, 1, f.shape))
        src = torch.tensor(f, device="cuda", dtype=torch.float64)
        dst = torch.zeros((n, nd * nd), device="cuda", dtype=torch.float64)
        lb.project(ns, es, nd, ed, src, dst)
        torch.cuda.synchronize()
        got = dst.cpu().numpy()
        want = np.stack([oracle.project(ns, es, nd, ed, f[k]) for k in range(n)])
        assert np.max(np.abs(got - want)) < 1e-15


def test_region_change_and_indicator(oracle, lb):
    nx, ny = 128, 48
    O, G = pair(oracle, lb, nx, ny, n_low=3, eq_low=2, n_high=6, eq_high=4, kn=0.1, tile_w=64,
                u_wall=((-0.05, 0.0), (0.05, 0.0)), bands=(6, 6), cfl=0.3)
    O.init_equilibrium()
    G.init_equilibrium()
    O.step(100)
    G.step(100)
    lo, hi = np.array([10, 4], np.int32), np.array([5, 12], np.int32)
    O.update_regions(lo, hi)
    G.change_regions(lo, hi)
    for s in (0, 1):
        e, _ = pop_err(G, O, s)
        assert e < 1e-12
    O.step(20)
    G.step(20)
    r_o, uxo, uyo = O.moments()
    r_g, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-10
    Bo, Bg = O.indicator(), G.indicator()
    assert np.max(np.abs(Bg - Bo)) < 1e-12 * max(1.0, np.max(Bo))
    # bands from the indicator, compared bit for bit.  The threshold sits in
    # a gap between indicator values (wider than 1e-9 relative, so rounding
    # differences cannot move a node across it), chosen among such gaps so
    # that the oracle's bands fall strictly between the clamps in as many
    # tiles as possible: the band rule itself decides them
    Bs = np.unique(Bo.ravel())
    best = None
    for k in range(len(Bs) - 1):
        if Bs[k + 1] - Bs[k] <= 1e-9 * Bs[k + 1]:
            continue
        th = float(0.5 * (Bs[k] + Bs[k + 1]))
        lo_o, hi_o = O.bands_from_indicator(Bo, th, 2, 20)
        inner = int(np.sum((lo_o > 2) & (lo_o < 20)) + np.sum((hi_o > 2) & (hi_o < 20)))
        if best is None or inner > best[0]:
            best = (inner, th)
    inner, theta = best
    assert inner >= 2, "no threshold gives bands between the clamps"
    bo = O.bands_from_indicator(Bo, theta, 2, 20)
    G.update_regions(theta, 2, 20)
    bg = G.get_regions()
    np.testing.assert_array_equal(bg[0], bo[0])
    np.testing.assert_array_equal(bg[1], bo[1])


def test_empty_wall_band_next_to_band(oracle, lb):
    # one tile has no high-set rows at a wall (band 0), its neighbour has a
    # band there: wall-row nodes beside the tile boundary are read across x
    # by the other set and must be projected although their y neighbours
    # beyond the wall do not exist
    nx, ny = 128, 32
    O, G = pair(oracle, lb, nx, ny, n_low=3, eq_low=2, n_high=6, eq_high=4, kn=0.1, tile_w=64,
                u_wall=((-0.05, 0.0), (0.05, 0.0)), bands=(6, 6), cfl=0.3)
    O.init_equilibrium()
    G.init_equilibrium()
    O.step(40)
    G.step(40)
    lo, hi = np.array([0, 7], np.int32), np.array([5, 0], np.int32)
    O.update_regions(lo, hi)
    G.change_regions(lo, hi)
    O.step(30)
    G.step(30)
    for s in (0, 1):
        e, m = pop_err(G, O, s)
        assert m > 0 and e < 1e-12
    _, uxo, uyo = O.moments()
    _, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-12


# ----------------------------------------------- pressure channel with regrid
def _c3_small(oracle, lb, storage, regrid):
    nx, ny, tw = 256, 48, 64
    x, _ = oracle.gh_rule(6)
    dt = 0.3 / float(np.max(x))
    kw = dict(n_low=3, eq_low=2, n_high=6, eq_high=4, kn=0.2, xbc=oracle.XBC_PRESSURE, rho_in=2.0,
              rho_out=1.0, tau_mode=oracle.TAU_RHO, tile_w=tw)
    G = lb.Lattice(lb.make_params(nx, ny, storage=storage, dt=dt, **kw))
    O = oracle.Lattice(nx, ny, dt=dt, **kw)
    xx = np.arange(nx)[None, :] * np.ones((ny + 1, 1))
    rho = 2.0 - 1.0 * xx / (nx - 1)
    for L in (G, O):
        L.set_regions(8, 8)
        L.init_equilibrium(rho, 0 * xx, 0 * xx)
    return G, O


def test_pressure_channel_regrid_fp64(oracle, lb):
    # the C3 procedure at reduced size: every 100 steps the indicator picks
    # per-tile bands (theta, clamp [4, 20]) and switched nodes are converted
    G, O = _c3_small(oracle, lb, "f64", 100)
    theta, bmin, bmax = 0.002, 4, 20
    for _ in range(3):
        O.step(100)
        G.step(100)
        Bo = O.indicator()
        guard = np.abs(Bo - theta) <= 1e-9 * theta
        assert guard.sum() == 0
        lo, hi = O.bands_from_indicator(Bo, theta, bmin, bmax)
        O.update_regions(lo, hi)
        G.update_regions(theta, bmin, bmax)
        glo, ghi = G.get_regions()
        np.testing.assert_array_equal(glo, lo)
        np.testing.assert_array_equal(ghi, hi)
    _, uxo, uyo = O.moments()
    _, uxg, uyg = G.moments()
    assert rel_u(uxg, uyg, uxo, uyo) < 1e-10


# Reduced-precision storage against FP64.  FP32 meets 1e-5 relative
# velocity error.  bf16 (8-bit significand, stochastic rounding) carries
# the velocity in population deviations of ~w |xi u|, so its error is set
# by 2^-9 of those: the bounds below are its measured behaviour (stated
# per result), and the 2e-3 goal is asserted separately as a known miss.
BF16_GOAL = 2e-3


def _c3_storage_error(oracle, lb, storage):
    G, O = _c3_small(oracle, lb, storage, 0)
    O.step(300)
    G.step(300)
    _, uxo, uyo = O.moments()
    _, uxg, uyg = G.moments()
    return rel_u(uxg, uyg, uxo, uyo)


def test_pressure_channel_storage_error(oracle, lb):
    # pressure-driven channel (density 2 -> 1, Courant 0.3), fixed bands,
    # FP32 storage (referenced to the imposed density ramp per column
    # group) against the FP64 oracle: the 1e-5 goal
    err = _c3_storage_error(oracle, lb, "f32")
    print(f"f32: relative velocity error vs FP64 oracle after 300 steps = {err:.3e}")
    assert err < 1e-5


def _c2_velocity(lb, storage, steps):
    c = W.POISEUILLE_C2
    p = lb.make_params(c["nx"], c["ny"], kn=c["kn"], n_low=3, eq_low=2, n_high=6, eq_high=4, gx=c["gx"],
                       storage=storage, cfl=c["cfl"])
    L = lb.Lattice(p)
    L.set_regions(*c["bands"])
    L.init_equilibrium()
    L.step(steps)
    _, ux, uy = L.moments()
    return ux, uy


def _c2_storage_error(lb, storage):
    # the full body-force channel (1024 x 513, 10k steps, Courant 0.35) in
    # reduced precision against the same run with FP64 storage (which the
    # coupled parity tests tie to the oracle at 1e-10)
    c = W.POISEUILLE_C2
    ref = _c2_velocity(lb, "f64", c["steps"])
    u = _c2_velocity(lb, storage, c["steps"])
    err = rel_u(u[0], u[1], ref[0], ref[1])
    print(f"{storage}: relative velocity error vs FP64 after {c['steps']} steps = {err:.3e}")
    return err


def test_poiseuille_c2_storage_error(lb):
    # FP32 storage: the 1e-5 goal
    assert _c2_storage_error(lb, "f32") < 1e-5


# bf16 storage: the 2e-3 goal is missed on both channels (measured 7.1e-3 on
# the body-force channel after 10k steps, 9.1e-3 on the pressure channel
# after 300): an 8-bit significand on the stored deviations, whose velocity
# part w xi u rho it must resolve.  These strict expected failures are the
# bf16 result; they turn into failures if the goal is ever met.
@pytest.mark.xfail(strict=True, reason="bf16 storage misses the 2e-3 velocity-error goal")
@pytest.mark.parametrize("case", ["pressure_channel", "poiseuille_c2"])
def test_bf16_storage_goal(oracle, lb, case):
    err = _c3_storage_error(oracle, lb, "bf16") if case == "pressure_channel" else _c2_storage_error(lb, "bf16")
    print(f"bf16 {case}: relative velocity error {err:.3e} (goal {BF16_GOAL})")
    assert err < BF16_GOAL


def test_bf16_storage_regression_bound(oracle, lb):
    # not the goal (see above): a guard that the stochastic rounding keeps
    # bf16 near its measured error (slow flows stall with round-to-nearest,
    # error 0.95)
    assert _c3_storage_error(oracle, lb, "bf16") < 2e-2


# ---------------------------------------------- execution modes, same bits
def test_concurrent_streams_bit_identical(lb):
    # the low set's kernels on a second stream (default) vs everything on
    # one stream: identical populations, also with the learned closure
    from paper_1007_4895_amd import closure
    import torch
    nx, ny = 300, 80
    Ls = []
    for conc in (True, False):
        p = lb.make_params(nx, ny, kn=0.05, n_low=3, eq_low=2, n_high=6, eq_high=4, storage="f32", gx=1e-5,
                           u_wall=((0.01, 0.0), (0.0, 0.0)), cfl=0.3)
        L = lb.Lattice(p)
        L.set_regions(12, 9)
        rho, ux, uy = W.smooth_fields(nx, ny + 1, seed=61)
        L.init_equilibrium(rho, ux, uy)
        L.set_concurrency(conc)
        Ls.append(L)
    for L in Ls:
        L.step(25)
    norm = np.array([0.0] * 10 + [0.3, 0.05, 0.05, 1.0] + [1e-3] * 6 + [0.0] * 6 + [3e-4] * 6, np.float32)
    params = torch.from_numpy(closure.init_params(3)).to("cuda:0")
    for L in Ls:
        L.set_closure(params, norm)
        L.step(25)
    for s in (0, 1):
        a, b = Ls[0].get_populations(s), Ls[1].get_populations(s)
        assert np.array_equal(np.isnan(a), np.isnan(b))
        m = ~np.isnan(a)
        assert np.array_equal(a[m], b[m]), s


def test_project_finish_launch_bit_identical(lb):
    # a pressure channel with tile bands has both a projection list and
    # pressure columns: one merged launch (single stream) against the
    # separate projection and finish kernels (second stream)
    nx, ny = 256, 48
    Ls = []
    for conc in (True, False):
        p = lb.make_params(nx, ny, kn=0.2, n_low=3, eq_low=2, n_high=6, eq_high=4, storage="f32",
                           xbc=lb.XBC_PRESSURE, rho_in=2.0, rho_out=1.0, tau_mode=lb.TAU_RHO, tile_w=64, cfl=0.3)
        L = lb.Lattice(p)
        L.set_regions(np.array([8, 12, 6, 10], np.int32), np.array([9, 5, 11, 8], np.int32))
        xx = np.arange(nx)[None, :] * np.ones((ny + 1, 1))
        L.init_equilibrium(2.0 - xx / (nx - 1), 0 * xx, 0 * xx)
        L.set_concurrency(conc)
        Ls.append(L)
    for L in Ls:
        L.step(40)
    for s in (0, 1):
        a, b = Ls[0].get_populations(s), Ls[1].get_populations(s)
        assert np.array_equal(np.isnan(a), np.isnan(b))
        m = ~np.isnan(a)
        assert m.sum() > 0 and np.array_equal(a[m], b[m]), s


def test_c3_full_size_regrid_bands(oracle, lb):
    # the pressure channel at its full size (4096 x 257, FP32, Courant 0.3):
    # at every regrid (each 500 steps) the bands the GPU derives from its
    # own indicator field equal the oracle's rule applied to that field
    # (bit-exact outside a guard band around theta), and the indicator of
    # every node in the D2Q36 set agrees with its definition evaluated by
    # the oracle on sampled nodes
    from paper_1007_4895_amd import closure
    c = W.PRESSURE_C3
    G = closure.channel(c["nx"], c["ny"], c["kn"], storage=c["storage"], all_high=False, bands=(c["bmin"], c["bmin"]),
                        rho_in=c["rho_in"], rho_out=c["rho_out"], cfl=c["cfl"], tile_w=c["tile_w"])
    O = oracle.Lattice(c["nx"], c["ny"], dt=G.dt, kn=c["kn"], n_low=3, eq_low=2, n_high=6, eq_high=4,
                       xbc=oracle.XBC_PRESSURE, rho_in=c["rho_in"], rho_out=c["rho_out"], tau_mode=oracle.TAU_RHO,
                       tile_w=c["tile_w"])
    theta, bmin, bmax = c["theta"], c["bmin"], c["bmax"]
    for _ in range(3):
        G.step(c["regrid"])
        B = G.indicator()
        assert np.all(np.isfinite(B))
        guard = np.abs(B - theta) <= 1e-9 * theta
        assert guard.sum() == 0
        lo, hi = O.bands_from_indicator(B, theta, bmin, bmax)
        G.update_regions(theta, bmin, bmax)
        glo, ghi = G.get_regions()
        np.testing.assert_array_equal(glo, lo)
        np.testing.assert_array_equal(ghi, hi)
    # indicator definition on sampled D2Q36 nodes
    f36 = G.get_populations(1)
    B = G.indicator()
    g = W.rng(71)
    rows = g.integers(0, c["ny"] + 1, 40)
    cols = g.integers(0, c["nx"], 40)
    for j, i in zip(rows, cols):
        f = f36[:, j, i]
        if np.isnan(f[0]):
            continue
        a = oracle.hermite_coeffs(6, f)
        r, ux, uy = a[0, 0], a[1, 0] / a[0, 0], a[0, 1] / a[0, 0]
        ref = max(abs(a[2, 0] - r * ux * ux), abs(a[1, 1] - r * ux * uy), abs(a[0, 2] - r * uy * uy)) / r
        assert abs(B[j, i] - ref) <= 1e-12 + 1e-9 * ref
