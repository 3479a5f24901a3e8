"""Training and evaluation of the learned interface closure.

When a D2Q9 node is lifted to D2Q36 (4th-order equilibrium) the Hermite
projection of Sec. 2.2 knows nothing of the non-equilibrium coefficients of
total order 3-4 that D2Q9 cannot carry and sets them to zero.  A small
network (10 -> 64 -> 64 -> 8, see include/lb.h) predicts the six of them
from node-local D2Q9 data, plus a flag telling whether the node's
non-equilibrium indicator exceeds the band threshold.

Everything numeric runs in the HIP library: sample extraction from
all-D2Q36 runs, the FP32 forward / backward / Adam kernels, bf16 inference
and the lift.  This module only drives it: it picks the runs and the nodes
(seeded), standardises the data set on the host, shuffles mini-batches and
reports errors.

Data: all-D2Q36 runs of the pressure-driven channel (inlet / outlet density
2 : 1, relaxation time ~ 1/rho, outlet Kn drawn log-uniformly in
[0.02, 0.5]), snapshots every few hundred steps, nodes drawn uniformly.
"""
from __future__ import annotations

import numpy as np

from . import lb
from . import workloads as W

NIN, NOUT, NREG = lb.MLP_NIN, lb.MLP_NOUT, lb.MLP_NREG
SIZES = [(64, 10), (64,), (64, 64), (64,), (8, 64), (8,)]


def init_params(seed: int) -> np.ndarray:
    """Xavier-uniform weights (limit sqrt(6 / (fan_in + fan_out))), zero
    biases, from seeded U(-1, 1) draws; float32."""
    u = W.noise((lb.mlp_param_count(),), seed, 1.0)
    p = np.zeros_like(u)
    o = 0
    for s in SIZES:
        n = int(np.prod(s))
        if len(s) == 2:
            p[o:o + n] = np.sqrt(6.0 / (s[0] + s[1])) * u[o:o + n]
        o += n
    return p.astype(np.float32)


def channel(nx, ny, kn, *, storage="f32", all_high=True, bands=(8, 8), rho_in=2.0, rho_out=1.0, cfl=0.3,
            tile_w=64):
    """Pressure-driven channel lattice (D2Q9 / D2Q36 order 4) started from a
    linear density ramp at rest."""
    p = lb.make_params(nx, ny, kn=kn, n_low=3, eq_low=2, n_high=6, eq_high=4, storage=storage,
                       xbc=lb.XBC_PRESSURE, rho_in=rho_in, rho_out=rho_out, tau_mode=lb.TAU_RHO, cfl=cfl,
                       tile_w=tile_w)
    L = lb.Lattice(p)
    if all_high:
        L.set_regions(ny + 1, 0)
    else:
        L.set_regions(*bands)
    xx = np.arange(nx)[None, :] * np.ones((ny + 1, 1))
    rho = rho_in - (rho_in - rho_out) * xx / (nx - 1)
    L.init_equilibrium(rho, 0 * xx, 0 * xx)
    return L


def generate(nx, ny, kns, *, steps, snaps, per_snap, seed, theta=0.01, storage="f32", keep_f36=False):
    """Samples from all-D2Q36 runs, one per Kn: after every steps // snaps
    steps, per_snap distinct nodes drawn uniformly.  Returns raw features,
    targets, flags and the run index of every sample (and, if asked, the
    samples' D2Q36 populations)."""
    import torch

    X, T, F, R, P = [], [], [], [], []
    g = W.rng(seed)
    every = max(1, steps // snaps)
    for r, kn in enumerate(kns):
        L = channel(nx, ny, float(kn), storage=storage)
        for _ in range(snaps):
            L.step(every)
            nodes = g.choice(nx * (ny + 1), size=min(per_snap, nx * (ny + 1)), replace=False).astype(np.int32)
            dn = torch.from_numpy(nodes).to(L.device)
            x, t, f = L.closure_samples(dn, theta)
            torch.cuda.synchronize()
            X.append(x.cpu().numpy())
            T.append(t.cpu().numpy())
            F.append(f.cpu().numpy())
            R.append(np.full(len(nodes), r, dtype=np.int32))
            if keep_f36:
                f36 = L.get_populations(1).reshape(36, -1)
                P.append(f36[:, nodes].T.copy())
        L.close()
    out = [np.concatenate(X), np.concatenate(T), np.concatenate(F), np.concatenate(R)]
    if keep_f36:
        out.append(np.concatenate(P))
    return tuple(out)


def standardisation(X, T):
    """32 constants: input means, input deviations, target means, target
    deviations (deviations floored at 1e-12 of the largest)."""
    X = np.asarray(X, np.float64)
    T = np.asarray(T, np.float64)
    xm, xs = X.mean(0), X.std(0)
    tm, ts = T.mean(0), T.std(0)
    xs = np.maximum(xs, 1e-12 * max(xs.max(), 1e-30))
    ts = np.maximum(ts, 1e-12 * max(ts.max(), 1e-30))
    return np.concatenate([xm, xs, tm, ts]).astype(np.float32)


def standardise(X, T, norm):
    n = np.asarray(norm, np.float64)
    Xs = (np.asarray(X, np.float64) - n[0:10]) / n[10:20]
    Ts = (np.asarray(T, np.float64) - n[20:26]) / n[26:32]
    return Xs.astype(np.float32), Ts.astype(np.float32)


def train(X, T, flag, norm, *, steps, batch=4096, lr=1e-3, seed=0, log_every=100, device="cuda:0"):
    """Adam on the standardised data set through the library's FP32
    kernels.  Returns (params as a device float32 tensor, loss history)."""
    import torch

    Xs, Ts = standardise(X, T, norm)
    fl = np.asarray(flag, np.int32)
    n = len(Xs)
    batch = min(batch, n)
    net = lb.MLP(torch.from_numpy(init_params(seed)).to(device), batch)
    g = W.rng(seed + 1)
    perm, pos = g.permutation(n), 0
    hist = []
    for k in range(steps):
        if pos + batch > n:
            perm, pos = g.permutation(n), 0
        idx = perm[pos:pos + batch]
        pos += batch
        xb = torch.from_numpy(np.ascontiguousarray(Xs[idx])).to(device)
        tb = torch.from_numpy(np.ascontiguousarray(Ts[idx])).to(device)
        fb = torch.from_numpy(np.ascontiguousarray(fl[idx])).to(device)
        loss, _ = net.loss_grad(xb, tb, fb)
        net.adam(lr)
        if log_every and (k % log_every == 0 or k == steps - 1):
            hist.append((k, float(loss.item())))
    torch.cuda.synchronize()
    return net.params, hist


def predict(params, X, norm, device="cuda:0"):
    """FP32 network outputs for raw features X: regression outputs
    de-standardised to raw targets, and flag probabilities."""
    import torch

    Xs, _ = standardise(X, np.zeros((len(X), NREG)), norm)
    out = np.zeros((len(X), NOUT), np.float32)
    step = 1 << 16
    net = lb.MLP(params, step)
    for a in range(0, len(X), step):
        xb = torch.from_numpy(np.ascontiguousarray(Xs[a:a + step])).to(device)
        out[a:a + len(xb)] = net.forward(xb).cpu().numpy()
    n = np.asarray(norm, np.float64)
    reg = n[20:26] + n[26:32] * out[:, :NREG].astype(np.float64)
    z = out[:, NREG:].astype(np.float64)
    p1 = 1.0 / (1.0 + np.exp(z[:, 0] - z[:, 1]))
    return reg, p1


def target_errors(params, X, T, flag, norm):
    """Relative L2 error of the predicted missing coefficients (the analytic
    closure predicts zero, error 1) and the flag accuracy."""
    reg, p1 = predict(params, X, norm)
    T = np.asarray(T, np.float64)
    e = float(np.sqrt(np.sum((reg - T) ** 2) / np.sum(T ** 2)))
    acc = float(np.mean((p1 > 0.5) == (np.asarray(flag) == 1)))
    return e, acc


def lift_errors(params, norm, kn, f36, rho_ref=1.0, tau_rho=True, device="cuda:0"):
    """D2Q36 nodes f36 [n, 36] (absolute, host) restricted to D2Q9 and lifted
    back, analytically and with the learned closure (bf16 weights).  Returns
    the L2 population errors of the two lifts against the original."""
    import torch

    src = torch.from_numpy(np.ascontiguousarray(f36, dtype=np.float64)).to(device)
    n = src.shape[0]
    f9 = torch.empty((n, 9), dtype=torch.float64, device=device)
    lb.project(6, 4, 3, 2, src, f9)
    c36 = lb.closure_eval(params, norm, kn, tau_rho, rho_ref, f9)
    fa = torch.empty((n, 36), dtype=torch.float64, device=device)
    fl = torch.empty((n, 36), dtype=torch.float64, device=device)
    lb.project(3, 2, 6, 4, f9, fa)
    lb.project(3, 2, 6, 4, f9, fl, closure=c36)
    torch.cuda.synchronize()
    a, l, t = fa.cpu().numpy(), fl.cpu().numpy(), src.cpu().numpy()
    return float(np.sqrt(np.sum((t - a) ** 2))), float(np.sqrt(np.sum((t - l) ** 2)))


def velocity_error(L, ref):
    """Relative L2 velocity error of lattice L against the field ref."""
    _, ux, uy = L.moments()
    return float(np.sqrt(np.sum((ux - ref[0]) ** 2 + (uy - ref[1]) ** 2) / np.sum(ref[0] ** 2 + ref[1] ** 2)))


def report(nx=4096, ny=256, runs=8, steps=20000, snaps=16, per_snap=16384, train_steps=4000, kn_eval=0.2,
           bands=(16, 16), seed=40, theta=0.01, regrid_every=500):
    """The learned closure on the pressure-driven channel: data from
    all-D2Q36 runs (Kn log-uniform in [0.02, 0.5]), training on the GPU,
    held-out sample and lift errors at kn_eval, and the coupled channel's
    velocity error against all-D2Q36 with the analytic and the learned lift
    (fixed bands), and with bands from the indicator every regrid_every
    steps (analytic lift, learned lift, learned lift with the network's
    region flag beside the indicator).  Returns a dict."""
    import time

    import torch

    out = {"geometry": f"{nx}x{ny + 1}", "runs": runs, "steps": steps}
    kns = np.exp(W.rng(seed).uniform(np.log(0.02), np.log(0.5), runs))
    t0 = time.perf_counter()
    X, T, F, _ = generate(nx, ny, kns, steps=steps, snaps=snaps, per_snap=per_snap, seed=seed + 1)
    out["samples"] = int(len(X))
    out["data_s"] = round(time.perf_counter() - t0, 2)
    out["kn_train"] = [round(float(k), 4) for k in kns]
    norm = standardisation(X, T)
    t0 = time.perf_counter()
    params, hist = train(X, T, F, norm, steps=train_steps, batch=4096, lr=2e-3, seed=seed + 2, log_every=500)
    out["train_s"] = round(time.perf_counter() - t0, 2)
    out["loss"] = [(k, round(v, 5)) for k, v in hist]
    e_tr, acc_tr = target_errors(params, X[:200000], T[:200000], F[:200000], norm)
    del X, T, F
    # held-out Kn: samples, lift errors, and the all-D2Q36 reference field
    Xh, Th, Fh, _, Ph = generate(nx, ny, [kn_eval], steps=steps, snaps=4, per_snap=per_snap, seed=seed + 3,
                                 keep_f36=True)
    e_h, acc_h = target_errors(params, Xh, Th, Fh, norm)
    la, ll = lift_errors(params, norm, kn_eval, Ph)
    out["missing_coeff_rel_error"] = {"train": round(e_tr, 4), "held_out": round(e_h, 4), "analytic": 1.0}
    out["flag_accuracy"] = {"train": round(acc_tr, 4), "held_out": round(acc_h, 4)}
    out["lift_l2_error"] = {"analytic": la, "learned": ll, "ratio": round(ll / la, 4)}
    A = channel(nx, ny, kn_eval, storage="f32")
    A.step(steps)
    _, ux, uy = A.moments()
    ref = (ux, uy)
    A.close()
    flow = {}
    for name, use in (("analytic", False), ("learned", True)):
        L = channel(nx, ny, kn_eval, storage="f32", all_high=False, bands=bands)
        if use:
            L.set_closure(params, norm)
        L.step(200)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.step(steps - 200)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t1
        flow[name] = {"e_model": velocity_error(L, ref),
                      "mlups": round(nx * (ny + 1) * (steps - 200) / sec / 1e6, 1)}
        L.close()
    out["coupled_vs_all_d2q36"] = {"kn_outlet": kn_eval, "bands": list(bands), **flow}
    # bands from the indicator every `regrid` steps: the analytic lift, and
    # the learned lift with the network's region flag beside the indicator
    regrid = {}
    for name, use, flags in (("analytic", False, False), ("learned", True, False), ("learned_flags", True, True)):
        L = channel(nx, ny, kn_eval, storage="f32", all_high=False, bands=(8, 8))
        if use:
            L.set_closure(params, norm)
            L.set_closure_flags(flags)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        done, mb = 0, []
        while done < steps:
            L.step(min(regrid_every, steps - done))
            done += regrid_every
            if done < steps:
                L.update_regions(theta, 8, 64)
                lo, hi = L.get_regions()
                mb.append(float(np.mean(np.concatenate([lo, hi]))))
        torch.cuda.synchronize()
        sec = time.perf_counter() - t1
        regrid[name] = {"e_model": velocity_error(L, ref), "mlups": round(nx * (ny + 1) * steps / sec / 1e6, 1),
                        "mean_band_rows": round(float(np.mean(mb)), 1) if mb else 8.0}
        L.close()
    out["regrid_vs_all_d2q36"] = {"kn_outlet": kn_eval, "theta": theta, "every": regrid_every, "bands": [8, 64],
                                  **regrid}
    return out


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description="learned-closure report on the pressure-driven channel")
    ap.add_argument("--small", action="store_true", help="reduced sizes (a quick check)")
    a = ap.parse_args()
    if a.small:
        r = report(nx=512, ny=64, runs=4, steps=3000, snaps=4, per_snap=4096, train_steps=800, bands=(8, 8))
    else:
        r = report()
    print(json.dumps(r))
