"""GPU tests of the learned interface closure: the FP32 training kernels
against the FP64 network oracle (forward, gradient, Adam), sample extraction
and bf16 inference against the oracle's features / targets / closure, the
coupled step with the learned lift against the oracle stepping with the same
closure, and what a network trained on the GPU gains over the analytic
lift.

Tolerances: FP32 arithmetic on O(1) standardised values gives ~1e-6
absolute per output (64-term sums); gradients are compared as a relative L2
norm over all 5384 entries (1e-4).  Features are FP64 on the GPU and rounded
to FP32 once (relative 1e-6).  The closure coefficients of the lift are FP32
network outputs with bf16 weights on both sides (relative 1e-4 of their
scale), which moves populations of one step by far less than 1e-9.
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


@pytest.fixture(scope="module")
def mlp():
    import oracle.mlp as m
    return m


def bf16_round(p):
    """Round float32 values to bf16 (nearest, ties to even), as float32."""
    u = np.ascontiguousarray(p, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _net(mlp, seed, B):
    g = W.rng(seed)
    p = mlp.init(W.noise((mlp.NPARAM,), seed, 1.0)) + 0.05 * g.normal(size=mlp.NPARAM)
    X = g.normal(size=(B, mlp.NIN))
    T = g.normal(size=(B, mlp.NREG))
    flag = g.integers(0, 2, B)
    return p.astype(np.float32), X.astype(np.float32), T.astype(np.float32), flag.astype(np.int32)


def _dev(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda:0")


@pytest.mark.parametrize("B", [1, 300, 4133])
def test_mlp_forward(lb, mlp, B):
    p, X, _, _ = _net(mlp, 1, B)
    net = lb.MLP(_dev(p), B)
    y = net.forward(_dev(X)).cpu().numpy()
    ref, _ = mlp.forward(p.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(y - ref)) < 2e-5 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("B", [7, 1000])
def test_mlp_gradient(lb, mlp, B):
    p, X, T, flag = _net(mlp, 2, B)
    net = lb.MLP(_dev(p), B)
    loss, g = net.loss_grad(_dev(X), _dev(T), _dev(flag))
    g1 = g.cpu().numpy().copy()
    l1 = float(loss.item())
    lref, gref = mlp.loss_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64), flag)
    assert abs(l1 - lref) < 1e-5 * abs(lref)
    rel = np.linalg.norm(g1 - gref) / np.linalg.norm(gref)
    print(f"B={B}: loss {l1:.6f} vs {lref:.6f}, gradient relative L2 error {rel:.2e}")
    assert rel < 1e-4
    # every block of the parameter vector, on its own
    o = 0
    for s in mlp.SIZES:
        n = int(np.prod(s))
        blk = np.linalg.norm(g1[o:o + n] - gref[o:o + n]) / max(np.linalg.norm(gref[o:o + n]), 1e-30)
        assert blk < 1e-4, (s, blk)
        o += n
    # deterministic: a second call gives the same bits
    _, g2 = net.loss_grad(_dev(X), _dev(T), _dev(flag))
    assert np.array_equal(g1, g2.cpu().numpy())


def test_mlp_adam(lb, mlp):
    import torch
    p, X, T, flag = _net(mlp, 3, 64)
    g = W.noise((mlp.NPARAM,), 4, 1e-2).astype(np.float32)
    net = lb.MLP(_dev(p), 64)
    pr, m, v = p.astype(np.float64), np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM)
    for t in range(1, 4):
        net.grad.copy_(_dev(g * t))
        net.adam(1e-3)
        pr, m, v = mlp.adam(pr, (g * t).astype(np.float64), m, v, t, lr=1e-3)
    torch.cuda.synchronize()
    assert np.max(np.abs(net.params.cpu().numpy() - pr)) < 1e-7


def _pressure_pair(oracle, lb, nx, ny, kn, storage, bands, all_high=False):
    from paper_1007_4895_amd import closure
    G = closure.channel(nx, ny, kn, storage=storage, all_high=all_high, bands=bands)
    O = oracle.Lattice(nx, ny, dt=G.dt, kn=kn, n_low=3, eq_low=2, n_high=6, eq_high=4,
                       xbc=oracle.XBC_PRESSURE, rho_in=2.0, rho_out=1.0, tau_mode=oracle.TAU_RHO, tile_w=64)
    O.set_regions(*((ny + 1, 0) if all_high else bands))
    xx = np.arange(nx)[None, :] * np.ones((ny + 1, 1))
    O.init_equilibrium(2.0 - xx / (nx - 1), 0 * xx, 0 * xx)
    return G, O


def test_closure_samples(oracle, lb, mlp):
    # features / targets / flags of an all-D2Q36 FP64 run vs the oracle's
    # definitions evaluated on the same populations
    import torch
    nx, ny, kn = 150, 40, 0.15
    G, _ = _pressure_pair(oracle, lb, nx, ny, kn, "f64", None, all_high=True)
    G.step(300)
    f36 = G.get_populations(1)
    g = W.rng(5)
    nodes = np.concatenate([[0, nx - 1, ny * nx, (ny + 1) * nx - 1],
                            g.choice(nx * (ny + 1), 700, replace=False)]).astype(np.int32)
    # threshold at the median indicator: both flag values occur
    def indicator(f):
        a = oracle.hermite_coeffs(6, f)
        r, ux, uy = a[0, 0], a[1, 0] / a[0, 0], a[0, 1] / a[0, 0]
        return max(abs(a[2, 0] - r * ux * ux), abs(a[1, 1] - r * ux * uy), abs(a[0, 2] - r * uy * uy)) / r
    fn = [f36[:, n // nx, n % nx] for n in nodes]
    B = np.array([indicator(f) for f in fn])
    theta = float(np.median(B)) * 1.0001
    x, t, fl = G.closure_samples(torch.from_numpy(nodes).to("cuda:0"), theta)
    x, t, fl = x.cpu().numpy(), t.cpu().numpy(), fl.cpu().numpy()
    for k, f in enumerate(fn):
        rho = float(np.sum(f))
        f9 = oracle.project(6, 4, 3, 2, f)
        xr = mlp.features(oracle, f9, kn * 1.0 / rho)
        tr = mlp.targets(oracle, f, 4)
        np.testing.assert_allclose(x[k], xr, rtol=2e-7, atol=1e-13)
        np.testing.assert_allclose(t[k], tr, rtol=2e-7, atol=1e-13)
    guard = np.abs(B - theta) <= 1e-9 * theta
    assert guard.sum() == 0
    np.testing.assert_array_equal(fl, (B > theta).astype(np.int32))
    assert 0 < fl.sum() < len(fl)


def _trial_norm():
    # plausible standardisation constants: O(1) network outputs become
    # closure coefficients of a few 1e-4
    return np.array([0.0] * 10 + [0.3, 0.05, 0.05, 1.0] + [1e-3] * 6 + [0.0] * 6 + [3e-4] * 6, np.float32)


def _oracle_closure(oracle, mlp, p, norm, kn, f9):
    """Oracle closure coefficients (nd = 6, row k*6 + m) of one D2Q9 node."""
    rho = float(np.sum(f9))
    x = mlp.features(oracle, f9, kn / rho)
    n = norm.astype(np.float64)
    xs = (x - n[0:10]) / n[10:20]
    y, _ = mlp.forward(bf16_round(p).astype(np.float64), xs[None, :])
    return mlp.closure_coeffs(y[0, :6], n[20:26], n[26:32], rho)


def test_closure_eval(oracle, lb, mlp):
    p, _, _, _ = _net(mlp, 6, 1)
    norm = _trial_norm()
    g = W.rng(7)
    f9 = []
    for k in range(257):
        f = oracle.equilibrium(3, 2, 1 + 0.5 * g.uniform(), 0.05 * g.normal(), 0.05 * g.normal())
        f9.append(f * (1 + W.noise((9,), 100 + k, 0.02)))
    f9 = np.array(f9)
    c = lb.closure_eval(_dev(p), norm, 0.2, True, 1.0, _dev(f9)).cpu().numpy()
    scale = 0.0
    for k in range(len(f9)):
        cr = _oracle_closure(oracle, mlp, p, norm, 0.2, f9[k])
        scale = max(scale, np.max(np.abs(cr)))
        assert np.max(np.abs(c[k] - cr)) < 1e-4 * np.max(np.abs(cr)) + 1e-12, k
    assert scale > 1e-4


def test_step_with_learned_closure(oracle, lb, mlp):
    # the lift of every step uses the network (bf16 weights) on the lifted
    # nodes' post-update D2Q9 populations; the oracle is given the same
    # closure coefficients, computed by the network oracle from its own state
    import torch
    nx, ny, kn = 130, 40, 0.2
    G, O = _pressure_pair(oracle, lb, nx, ny, kn, "f64", (6, 8))
    G.step(40)
    O.step(40)
    p, _, _, _ = _net(mlp, 8, 1)
    norm = _trial_norm()
    G.set_closure(_dev(p), norm)
    # step n -> n+1 uses the analytic halo on both sides; the GPU then lifts
    # with the network at the end of the step
    G.step(1)
    O.step(1)
    f9 = O.get_populations(0)
    reg = O.region()
    c = np.zeros((36, ny + 1, nx))
    for j in range(ny + 1):
        for i in range(nx):
            if reg[j, i] == oracle.REG_LOW:
                c[:, j, i] = _oracle_closure(oracle, mlp, p, norm, kn, f9[:, j, i])
    O.set_closure(c)
    O.step(1)
    G.step(1)
    for s in (0, 1):
        gpop, opop = G.get_populations(s), O.get_populations(s)
        m = ~np.isnan(gpop[0])
        e = np.max(np.abs(gpop[:, m] - opop[:, m])) / np.max(np.abs(opop[:, m]))
        assert e < 1e-9, (s, e)
    # the closure changed the step: analytic lift differs by far more
    _, O2 = _pressure_pair(oracle, lb, nx, ny, kn, "f64", (6, 8))
    O2.step(42)
    d = np.nanmax(np.abs(O2.get_populations(1) - O.get_populations(1)))
    assert d > 1e-7, d


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("channel", ["pressure", "periodic"])
def test_closure_in_the_projection_launch_bit_identical(oracle, lb, mlp, storage, channel):
    # a learned-closure step runs the inference inside the projection launch
    # (with the pressure columns' finish pass when the lattice has one); the
    # two-stream mode keeps the inference launch before the projection: the
    # same populations, bit for bit
    from paper_1007_4895_amd import closure
    nx, ny, kn = 130, 40, 0.2
    p, _, _, _ = _net(mlp, 8, 1)
    norm = _trial_norm()
    out = []
    for two_streams in (False, True):
        if channel == "pressure":
            G = closure.channel(nx, ny, kn, storage=storage, all_high=False, bands=(6, 8))
        else:
            G = lb.Lattice(lb.make_params(nx, ny, kn=kn, n_low=3, eq_low=2, n_high=6, eq_high=4, storage=storage,
                                          gx=1e-4, u_wall=((-0.02, 0.0), (0.02, 0.0)), cfl=0.3))
            G.set_regions(7, 5)
            rho, ux, uy = W.smooth_fields(nx, ny + 1, seed=91)
            G.init_equilibrium(rho, ux, uy)
        G.set_closure(_dev(p), norm)
        if two_streams:
            G.set_concurrency(True)
        G.step(30)
        out.append((G.get_populations(0), G.get_populations(1)))
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def test_region_change_with_learned_closure(oracle, lb, mlp):
    # nodes switched from D2Q9 to D2Q36 by a region change, and the halo
    # rebuilt after it, are lifted with the network; the oracle converts
    # with the same closure computed from its own D2Q9 state
    nx, ny, kn = 130, 40, 0.2
    G, O = _pressure_pair(oracle, lb, nx, ny, kn, "f64", (6, 8))
    G.step(40)
    O.step(40)
    p, _, _, _ = _net(mlp, 13, 1)
    norm = _trial_norm()
    G.set_closure(_dev(p), norm)
    f9 = O.get_populations(0)
    reg = O.region()
    c = np.zeros((36, ny + 1, nx))
    for j in range(ny + 1):
        for i in range(nx):
            if reg[j, i] == oracle.REG_LOW:
                c[:, j, i] = _oracle_closure(oracle, mlp, p, norm, kn, f9[:, j, i])
    O.set_closure(c)
    lo, hi = np.full(G.ntiles, 11, np.int32), np.full(G.ntiles, 12, np.int32)
    G.change_regions(lo, hi)
    O.update_regions(lo, hi)
    for s in (0, 1):
        gpop, opop = G.get_populations(s), O.get_populations(s)
        m = ~np.isnan(gpop[0])
        e = np.max(np.abs(gpop[:, m] - opop[:, m])) / np.max(np.abs(opop[:, m]))
        assert e < 1e-9, ("after the change", s, e)
    G.step(1)
    O.step(1)
    for s in (0, 1):
        gpop, opop = G.get_populations(s), O.get_populations(s)
        m = ~np.isnan(gpop[0])
        e = np.max(np.abs(gpop[:, m] - opop[:, m])) / np.max(np.abs(opop[:, m]))
        assert e < 1e-9, ("one step later", s, e)


def test_closure_training_gain(oracle, lb):
    # train on all-D2Q36 pressure-channel runs (Kn log-uniform in
    # [0.02, 0.5]) with the library's kernels; on a held-out Kn the learned
    # lift must beat the analytic one (which sets the missing coefficients
    # to zero)
    from paper_1007_4895_amd import closure
    nx, ny = 256, 48
    kns = np.exp(W.rng(9).uniform(np.log(0.02), np.log(0.5), 4))
    X, T, F, _ = closure.generate(nx, ny, kns, steps=2000, snaps=4, per_snap=4096, seed=10)
    norm = closure.standardisation(X, T)
    params, hist = closure.train(X, T, F, norm, steps=1500, batch=2048, lr=2e-3, seed=11)
    kh = 0.1
    Xh, Th, Fh, _, Ph = closure.generate(nx, ny, [kh], steps=2000, snaps=2, per_snap=4096, seed=12,
                                         keep_f36=True)
    e_tr, acc_tr = closure.target_errors(params, X, T, F, norm)
    e_h, acc_h = closure.target_errors(params, Xh, Th, Fh, norm)
    la, ll = closure.lift_errors(params, norm, kh, Ph)
    print(f"loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}; missing-coefficient relative error: train {e_tr:.3f}, "
          f"held-out {e_h:.3f} (analytic 1.0); flag accuracy train {acc_tr:.4f}, held-out {acc_h:.4f}; "
          f"lift L2 error analytic {la:.3e}, learned {ll:.3e} (ratio {ll / la:.3f})")
    assert hist[-1][1] < 0.5 * hist[0][1]
    assert e_h < 0.5
    assert ll < 0.8 * la


def test_update_regions_with_network_flags(oracle, lb, mlp):
    # the network's region flag counts beside the indicator in the band rule
    # (lb_set_closure_flags): the oracle evaluates the same network (bf16
    # weights, FP64 arithmetic) on its own state, flags the nodes whose
    # logits favour the high set, and applies its band rule to
    # "indicator above theta or flagged"
    import torch  # noqa: F401
    nx, ny, kn = 256, 48, 0.2
    G, O = _pressure_pair(oracle, lb, nx, ny, kn, "f64", (8, 8))
    G.step(300)
    O.step(300)
    p, _, _, _ = _net(mlp, 17, 1)
    norm = _trial_norm()
    G.set_closure(_dev(p), norm)
    G.set_closure_flags(True)
    B = O.indicator()
    f9, f36, reg = O.get_populations(0), O.get_populations(1), O.region()
    n = norm.astype(np.float64)
    X = np.zeros((ny + 1, nx, 10))
    for j in range(ny + 1):
        for i in range(nx):
            f = oracle.project(6, 4, 3, 2, f36[:, j, i]) if reg[j, i] == oracle.REG_HIGH else f9[:, j, i]
            X[j, i] = mlp.features(oracle, f, kn / float(np.sum(f)))
    y, _ = mlp.forward(bf16_round(p).astype(np.float64), ((X - n[0:10]) / n[10:20]).reshape(-1, 10))
    dz = (y[:, 7] - y[:, 6]).reshape(ny + 1, nx)
    # theta halfway into the widest gap between sorted indicator values
    # around their 95th percentile (rounding cannot move a node across it)
    sb = np.sort(B.ravel())
    k0 = int(0.95 * sb.size)
    k = k0 - 50 + int(np.argmax(np.diff(sb[k0 - 50:k0 + 50])))
    theta = 0.5 * (sb[k] + sb[k + 1])
    # nodes whose logit gap is within rounding of the GPU's bf16 / FP32
    # evaluation may go either way: tiles whose bands depend on them are
    # not compared
    sure_on, maybe_on = dz > 1e-3, dz > -1e-3
    want = [O.bands_from_indicator(np.where(fl, np.inf, B), theta, 8, 20) for fl in (sure_on, maybe_on)]
    base = O.bands_from_indicator(B, theta, 8, 20)
    G.update_regions(theta, 8, 20)
    got = G.get_regions()
    checked = 0
    for side in (0, 1):
        for t in range(len(got[side])):
            if want[0][side][t] == want[1][side][t]:
                assert got[side][t] == want[0][side][t], (side, t)
                checked += 1
    assert checked >= len(got[0])
    # the flags moved bands that the indicator alone would have left
    assert np.any(want[0][0] != base[0]) or np.any(want[0][1] != base[1])
    # switched off, the indicator alone decides again
    G.set_closure_flags(False)
    G.update_regions(theta, 8, 20)
    got = G.get_regions()
    np.testing.assert_array_equal(got[0], base[0])
    np.testing.assert_array_equal(got[1], base[1])
