"""GPU tests of batched stepping: many independent lattices advanced by one
launch per kernel and velocity-set pair (optionally replayed from captured
HIP graphs) must give bit-identical populations to stepping each lattice on
its own, which the single-lattice parity tests tie to the oracle; batched
channels of the 128-channel workload are also compared with the oracle
directly (the narrowest, and every 7th), and the full workload is checked
at its real sizes in the benchmark's launch configuration.
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


# (nx, ny, (n_low, eq_low, n_high, eq_high), bands, extra parameters)
MIXED = [
    (8, 40, (3, 2, 4, 3), (8, 8), dict(u_wall=((-0.05, 0.0), (0.05, 0.0)))),
    (8, 61, (3, 2, 6, 4), (9, 12), dict(gx=1e-5)),
    (8, 33, (4, 3, 6, 4), (10, 10), dict(gx=2e-5)),
    (70, 24, (3, 2, 6, 4), (5, 7), dict(u_wall=((0.03, 0.0), (-0.02, 0.0)))),
    (130, 30, (3, 2, 4, 3), (4, 6), dict(gx=5e-5, ybc=1)),
    (61, 20, (3, 2, 3, 2), (0, 0), dict(gx=1e-4)),
    (64, 26, (6, 4, 6, 4), (0, 0), dict(u_wall=((0.02, 0.0), (0.0, 0.0)))),
    (90, 28, (3, 2, 6, 4), (6, 6), dict(xbc=1, rho_in=1.02, rho_out=1.0, tau_mode=1, tile_w=64)),
]


def _make(lb, case, storage, seed):
    nx, ny, (nl, el, nh, eh), bands, extra = case
    p = lb.make_params(nx, ny, kn=0.1, n_low=nl, eq_low=el, n_high=nh, eq_high=eh, storage=storage, cfl=0.3,
                       **extra)
    L = lb.Lattice(p)
    L.set_regions(*bands)
    rho, ux, uy = W.smooth_fields(nx, ny + 1, seed=seed, rho_amp=0.02, u_amp=0.03)
    L.init_equilibrium(rho, ux, uy)
    return L


def _same(A, B):
    for s in (0, 1):
        a, b = A.get_populations(s), B.get_populations(s)
        if not np.array_equal(np.isnan(a), np.isnan(b)):
            return False
        m = ~np.isnan(a)
        if not np.array_equal(a[m], b[m]):
            return False
    return True


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_batch_bit_identical_to_single(lb, storage):
    cases = MIXED
    A = [_make(lb, c, storage, 100 + k) for k, c in enumerate(cases)]
    S = [_make(lb, c, storage, 100 + k) for k, c in enumerate(cases)]
    B = lb.Batch(A)
    nodes, launches, kinds = B.info()
    assert nodes == sum(c[0] * (c[1] + 1) for c in cases)
    assert kinds >= 5 and launches <= 4 * kinds
    # direct launches
    B.step(7)
    for L in S:
        L.step(7)
    assert all(_same(a, s) for a, s in zip(A, S))
    # graph segments of 4 steps: two replays (both parities) and a direct tail
    B.set_graph(4)
    B.step(11)
    for L in S:
        L.step(11)
    assert all(_same(a, s) for a, s in zip(A, S))
    B.step(8)
    for L in S:
        L.step(8)
    assert all(_same(a, s) for a, s in zip(A, S))
    # strips from the autotuner (states are restored)
    rows = B.autotune(3)
    assert all(_same(a, s) for a, s in zip(A, S)), rows
    B.step(5)
    for L in S:
        L.step(5)
    assert all(_same(a, s) for a, s in zip(A, S))
    assert all(a.steps == s.steps == 31 for a, s in zip(A, S))
    B.close()


# FP64 only: second-order D2Q16 / D2Q36 sets (a second merged update and
# projection launch) and a pair of equal sets with bands (a projection
# launch of its own), beside a pair of the first merged launch
SECOND_ORDER = [
    (8, 30, (4, 2, 6, 2), (6, 6), dict(gx=2e-5)),
    (70, 24, (3, 2, 6, 2), (5, 5), dict(u_wall=((-0.03, 0.0), (0.03, 0.0)))),
    (16, 40, (3, 2, 4, 2), (4, 4), dict(gx=1e-5)),
    (64, 20, (3, 2, 3, 2), (4, 4), dict(gx=3e-5)),
    (8, 33, (4, 3, 6, 4), (10, 10), dict(gx=2e-5)),
]


def test_batch_second_order_sets_and_equal_pairs(lb):
    A = [_make(lb, c, "f64", 300 + k) for k, c in enumerate(SECOND_ORDER)]
    S = [_make(lb, c, "f64", 300 + k) for k, c in enumerate(SECOND_ORDER)]
    B = lb.Batch(A)
    nodes, launches, kinds = B.info()
    assert kinds == len(SECOND_ORDER)
    # two merged updates, two merged projections, one projection of its own
    assert launches == 5, launches
    B.step(6)
    for L in S:
        L.step(6)
    assert all(_same(a, s) for a, s in zip(A, S))
    B.set_graph(3)
    B.step(7)
    for L in S:
        L.step(7)
    assert all(_same(a, s) for a, s in zip(A, S))
    B.close()


def test_batch_region_change_and_parity_guard(lb):
    A = [_make(lb, c, "f64", 200 + k) for k, c in enumerate(MIXED[:4])]
    S = [_make(lb, c, "f64", 200 + k) for k, c in enumerate(MIXED[:4])]
    B = lb.Batch(A)
    B.set_graph(2)
    B.step(4)
    for L in S:
        L.step(4)
    # a region change on one lattice is picked up by the batch
    A[1].change_regions(5, 15)
    S[1].change_regions(5, 15)
    B.step(6)
    for L in S:
        L.step(6)
    assert all(_same(a, s) for a, s in zip(A, S))
    # stepping a member on its own breaks the common parity: refused
    A[0].step(1)
    with pytest.raises(lb.LBError):
        B.step(1)
    B.close()


def test_batched_channel_vs_oracle(oracle, lb):
    # a narrow Couette channel (D2Q9 / D2Q16 order 3) inside a batch with two
    # other channels, against the oracle
    nx, ny = 8, 40
    x, _ = oracle.gh_rule(4)
    dt = 0.5 / float(np.max(x))
    kw = dict(kn=0.1, n_low=3, eq_low=2, n_high=4, eq_high=3, u_wall=((-0.05, 0.0), (0.05, 0.0)))
    O = oracle.Lattice(nx, ny, dt=dt, **kw)
    G = lb.Lattice(lb.make_params(nx, ny, storage="f64", dt=dt, **kw))
    others = [_make(lb, MIXED[1], "f64", 1), _make(lb, MIXED[3], "f64", 2)]
    for L in (O, G):
        L.set_regions(8, 8)
        L.init_equilibrium()
    B = lb.Batch([others[0], G, others[1]])
    B.set_graph(50)
    B.step(400)
    O.step(400)
    _, uxo, uyo = O.moments()
    _, uxg, uyg = G.moments()
    num = np.sqrt(np.sum((uxg - uxo) ** 2 + (uyg - uyo) ** 2))
    assert num / np.sqrt(np.sum(uxo ** 2 + uyo ** 2)) < 1e-10
    B.close()


def _c5(lb, count=None):
    cases = W.batch_cases(count=count)
    L = []
    for c in cases:
        p = lb.make_params(c["nx"], c["ny"], kn=c["kn"], n_low=c["n_low"], eq_low=c["eq_low"], n_high=c["n_high"],
                           eq_high=c["eq_high"], storage=c["storage"], u_wall=c["u_wall"], gx=c["gx"], cfl=c["cfl"])
        x = lb.Lattice(p)
        x.set_regions(*c["bands"])
        x.init_equilibrium()
        L.append(x)
    return cases, L


def test_c5_full_batch_bit_identical(lb):
    # the 128-channel workload at full size, graph segments + autotuned
    # strips as the benchmark runs it, against per-channel stepping
    cases, A = _c5(lb)
    _, S = _c5(lb)
    B = lb.Batch(A)
    B.autotune(5)
    B.set_graph(20)
    B.step(60)
    for L in S:
        L.step(60)
    bad = [k for k, (a, s) in enumerate(zip(A, S)) if not _same(a, s)]
    assert not bad, bad
    B.close()


def test_c5_channel_vs_oracle(oracle, lb):
    # one channel of the workload (the narrowest, FP32 storage) stepped in
    # the full batch, against the FP64 oracle: relative velocity error 1e-5
    cases, A = _c5(lb)
    k = int(np.argmin([c["ny"] for c in cases]))
    c = cases[k]
    G = A[k]
    O = oracle.Lattice(c["nx"], c["ny"], dt=G.dt, kn=c["kn"], n_low=c["n_low"], eq_low=c["eq_low"],
                       n_high=c["n_high"], eq_high=c["eq_high"], u_wall=c["u_wall"], gx=c["gx"])
    O.set_regions(*c["bands"])
    O.init_equilibrium()
    B = lb.Batch(A)
    B.set_graph(100)
    B.step(1000)
    O.step(1000)
    _, uxo, uyo = O.moments()
    _, uxg, uyg = G.moments()
    err = np.sqrt(np.sum((uxg - uxo) ** 2 + (uyg - uyo) ** 2) / np.sum(uxo ** 2 + uyo ** 2))
    print(f"channel {k} (ny={c['ny']}, Kn={c['kn']:.3g}): relative velocity error {err:.2e}")
    assert err < 1e-5
    B.close()


def test_c5_sampled_channels_vs_oracle(oracle, lb):
    # every 7th channel of the workload (both flow kinds, the three set
    # pairs, Kn across its range), stepped in the full batch in the
    # benchmark's launch configuration (autotuned strips, graph segments),
    # against the FP64 oracle run channel by channel
    cases, A = _c5(lb)
    B = lb.Batch(A)
    B.autotune(5)
    B.set_graph(100)
    B.step(300)
    worst = (0.0, -1)
    for k in range(0, len(cases), 7):
        c, G = cases[k], A[k]
        O = oracle.Lattice(c["nx"], c["ny"], dt=G.dt, kn=c["kn"], n_low=c["n_low"], eq_low=c["eq_low"],
                           n_high=c["n_high"], eq_high=c["eq_high"], u_wall=c["u_wall"], gx=c["gx"])
        O.set_regions(*c["bands"])
        O.init_equilibrium()
        O.step(300)
        _, uxo, uyo = O.moments()
        _, uxg, uyg = G.moments()
        err = np.sqrt(np.sum((uxg - uxo) ** 2 + (uyg - uyo) ** 2) / np.sum(uxo ** 2 + uyo ** 2))
        worst = max(worst, (float(err), k))
    print(f"sampled C5 channels: worst relative velocity error {worst[0]:.2e} (channel {worst[1]})")
    assert worst[0] < 1e-5
    B.close()


# persistent launches take lattices without a finish pass
PERSIST = [c for c in MIXED if not (c[4].get("ybc") or c[4].get("xbc"))]


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_persistent_batch_bit_identical_to_single(lb, storage):
    # one launch per run of steps, workgroups owning whole lattices: the same
    # bits as stepping every lattice on its own (stochastic-rounding seeds
    # included for bf16, whose kernels are built for D2Q9 and D2Q36 only)
    cases = PERSIST if storage != "bf16" else [c for c in PERSIST if set(c[2][::2]) <= {3, 6}]
    A = [_make(lb, c, storage, 400 + k) for k, c in enumerate(cases)]
    S = [_make(lb, c, storage, 400 + k) for k, c in enumerate(cases)]
    B = lb.Batch(A)
    B.set_persistent(True)
    _, launches, _ = B.info()
    assert launches == 0
    print(f"persistent batch {storage}: direct", flush=True)
    B.step(7)
    for L in S:
        L.step(7)
    assert all(_same(a, s) for a, s in zip(A, S))
    # graph segments of 4 steps (one captured launch each) and a tail; a
    # replayed segment repeats its stochastic-rounding seeds, so bf16 stays
    # on direct launches here
    if storage != "bf16":
        B.set_graph(4)
    B.step(11)
    for L in S:
        L.step(11)
    assert all(_same(a, s) for a, s in zip(A, S))
    # strips from the autotuner in this mode (states are restored)
    B.autotune(3)
    assert all(_same(a, s) for a, s in zip(A, S))
    B.step(6)
    for L in S:
        L.step(6)
    assert all(_same(a, s) for a, s in zip(A, S))
    # back to the per-step launches
    B.set_persistent(False)
    B.step(3)
    for L in S:
        L.step(3)
    assert all(_same(a, s) for a, s in zip(A, S))
    B.close()


def test_persistent_batch_refuses_finish_passes(lb):
    A = [_make(lb, c, "f64", 500 + k) for k, c in enumerate(MIXED)]
    B = lb.Batch(A)
    with pytest.raises(lb.LBError):
        B.set_persistent(True)
    # the batch keeps its per-step launches
    S = [_make(lb, c, "f64", 500 + k) for k, c in enumerate(MIXED)]
    B.step(3)
    for L in S:
        L.step(3)
    assert all(_same(a, s) for a, s in zip(A, S))
    B.close()


def test_c5_persistent_bit_identical(lb):
    # the 128-channel workload in persistent launches (graph segments, as the
    # benchmark runs it) against per-channel stepping
    cases, A = _c5(lb)
    _, S = _c5(lb)
    B = lb.Batch(A)
    B.set_persistent(True)
    B.autotune(5)
    B.set_graph(20)
    B.step(60)
    for L in S:
        L.step(60)
    bad = [k for k, (a, s) in enumerate(zip(A, S)) if not _same(a, s)]
    assert not bad, bad
    B.close()
