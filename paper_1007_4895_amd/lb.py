"""ctypes binding of liblb.so (include/lb.h).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI.  PyTorch supplies the device workspace and the stream.
The library must be built (``paper_1007_4895_amd.build``); loading fails
loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblb.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_EUNSTABLE, LB_EUNSUPPORTED, LB_ESTATE = 0, -1, -2, -3, -4, -5, -6
STORE_F64, STORE_F32, STORE_BF16 = 0, 1, 2
IFACE_HERMITE, IFACE_PAPER = 0, 1
TAU_CONST, TAU_RHO = 0, 1
XBC_PERIODIC, XBC_PRESSURE = 0, 1
YBC_WALLS, YBC_PERIODIC, YBC_SHEAR = 0, 1, 2

STORAGE = {"f64": STORE_F64, "f32": STORE_F32, "bf16": STORE_BF16}


class LBError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lb status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("n_low", C.c_int32), ("n_high", C.c_int32),
        ("eq_low", C.c_int32), ("eq_high", C.c_int32),
        ("force_low", C.c_int32), ("force_high", C.c_int32),
        ("tau_mode", C.c_int32), ("xbc", C.c_int32), ("ybc", C.c_int32),
        ("iface", C.c_int32), ("storage", C.c_int32), ("tile_w", C.c_int32),
        ("kn", C.c_double), ("rho_ref", C.c_double), ("cfl", C.c_double), ("dt", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double), ("u_wall", C.c_double * 4),
        ("rho_in", C.c_double), ("rho_out", C.c_double),
        ("u_osc", C.c_double), ("omega_osc", C.c_double), ("shear_top", C.c_double),
        ("T_wall", C.c_double * 2), ("thermal", C.c_int32), ("reserved_", C.c_int32),
    ]


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p


def lib():
    """Load liblb.so (never builds: a missing library is an error)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run paper_1007_4895_amd.build")
        L = C.CDLL(LIB_PATH)
        sig = {
            "lb_last_error": (C.c_char_p, []),
            "lb_params_default": (C.c_int, [C.POINTER(Params)]),
            "lb_workspace_bytes": (C.c_size_t, [C.POINTER(Params)]),
            "lb_create_lattice": (C.c_int, [C.POINTER(Params), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
            "lb_destroy_lattice": (None, [_vp]),
            "lb_get_info": (C.c_int, [_vp, _dp, _dp, _ip]),
            "lb_set_regions": (C.c_int, [_vp, _ip, _ip]),
            "lb_get_regions": (C.c_int, [_vp, _ip, _ip]),
            "lb_init_equilibrium": (C.c_int, [_vp, _dp, _dp, _dp]),
            "lb_init_equilibrium_thermal": (C.c_int, [_vp, _dp, _dp, _dp, _dp]),
            "lb_thermal_moments": (C.c_int, [_vp, _dp, _dp, _dp, C.c_int32]),
            "lb_energy": (C.c_int, [_vp, _dp]),
            "lb_step": (C.c_int, [_vp, C.c_int64]),
            "lb_moments": (C.c_int, [_vp, _dp, _dp, _dp, C.c_int32]),
            "lb_conservation": (C.c_int, [_vp, _dp]),
            "lb_get_populations": (C.c_int, [_vp, C.c_int32, _dp]),
            "lb_set_populations": (C.c_int, [_vp, C.c_int32, _dp]),
            "lb_state_bytes": (C.c_size_t, [_vp]),
            "lb_get_state": (C.c_int, [_vp, _vp, C.c_size_t]),
            "lb_set_state": (C.c_int, [_vp, _vp, C.c_size_t]),
            "lb_step_count": (C.c_int64, [_vp]),
            "lb_indicator": (C.c_int, [_vp, _dp, C.c_int32]),
            "lb_update_regions": (C.c_int, [_vp, C.c_double, C.c_int32, C.c_int32]),
            "lb_change_regions": (C.c_int, [_vp, _ip, _ip]),
            "lb_project": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, C.c_int64, _vp]),
            "lb_set_timing": (C.c_int, [_vp, C.c_int32]),
            "lb_kernel_times": (C.c_int, [_vp, _dp, C.POINTER(C.c_int64), _dp, C.POINTER(C.c_int64)]),
            "lb_set_strip_rows": (C.c_int, [_vp, C.c_int32]),
            "lb_region_counts": (C.c_int, [_vp, C.POINTER(C.c_int64)]),
            "lb_get_strip_rows": (C.c_int, [_vp, _ip]),
            "lb_set_work_shape": (C.c_int, [_vp, _ip, _ip]),
            "lb_set_concurrency": (C.c_int, [_vp, C.c_int32]),
            "lb_set_merged_update": (C.c_int, [_vp, C.c_int32]),
            "lb_get_work_shape": (C.c_int, [_vp, _ip, _ip]),
            "lb_autotune": (C.c_int, [_vp, C.c_int32, _ip]),
            "lb_mlp_param_count": (C.c_int64, []),
            "lb_mlp_workspace_bytes": (C.c_size_t, [C.c_int64]),
            "lb_mlp_forward": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, _vp]),
            "lb_mlp_forward_noalloc": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp]),
            "lb_mlp_loss_grad": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int64, _vp, _vp, _vp, _vp]),
            "lb_mlp_adam": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int64, C.c_float, _vp]),
            "lb_closure_eval": (C.c_int, [_vp, C.POINTER(C.c_float), C.c_double, C.c_int32, C.c_double, _vp,
                                          C.c_int64, _vp, _vp]),
            "lb_closure_samples": (C.c_int, [_vp, _vp, C.c_int64, C.c_double, _vp, _vp, _vp]),
            "lb_set_closure": (C.c_int, [_vp, _vp, C.POINTER(C.c_float)]),
            "lb_set_closure_flags": (C.c_int, [_vp, C.c_int32]),
            "lb_batch_create": (C.c_int, [C.POINTER(_vp), C.c_int32, _vp, C.POINTER(_vp)]),
            "lb_batch_destroy": (None, [_vp]),
            "lb_batch_set_graph": (C.c_int, [_vp, C.c_int32]),
            "lb_batch_set_persistent": (C.c_int, [_vp, C.c_int32]),
            "lb_batch_step": (C.c_int, [_vp, C.c_int64]),
            "lb_batch_set_strip_rows": (C.c_int, [_vp, C.c_int32, C.c_int32]),
            "lb_batch_autotune": (C.c_int, [_vp, C.c_int32, _ip]),
            "lb_batch_info": (C.c_int, [_vp, C.POINTER(C.c_int64), _ip, _ip]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != LB_OK:
        raise LBError(status, lib().lb_last_error().decode())


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(nx, ny, *, kn, n_low=3, n_high=3, eq_low=2, eq_high=None, storage="f64",
                iface=IFACE_HERMITE, tau_mode=TAU_CONST, xbc=XBC_PERIODIC, ybc=YBC_WALLS,
                tile_w=0, rho_ref=1.0, cfl=0.5, dt=0.0, gx=0.0, gy=0.0,
                u_wall=((0.0, 0.0), (0.0, 0.0)), rho_in=1.0, rho_out=1.0, u_osc=0.0,
                omega_osc=0.0, shear_top=0.0, thermal=False, T_wall=(1.0, 1.0)) -> Params:
    p = Params()
    _check(lib().lb_params_default(C.byref(p)))
    p.nx, p.ny = nx, ny
    p.n_low, p.n_high = n_low, n_high
    p.eq_low = eq_low
    p.eq_high = eq_low if eq_high is None else eq_high
    p.force_low = p.force_high = 0
    p.storage = STORAGE[storage] if isinstance(storage, str) else storage
    p.iface, p.tau_mode, p.xbc, p.ybc, p.tile_w = iface, tau_mode, xbc, ybc, tile_w
    p.kn, p.rho_ref, p.cfl, p.dt = kn, rho_ref, cfl, dt
    p.gx, p.gy = gx, gy
    for k, v in enumerate((u_wall[0][0], u_wall[0][1], u_wall[1][0], u_wall[1][1])):
        p.u_wall[k] = v
    p.rho_in, p.rho_out = rho_in, rho_out
    p.u_osc, p.omega_osc = u_osc, omega_osc
    p.shear_top = shear_top
    p.thermal = 1 if thermal else 0
    p.T_wall[0], p.T_wall[1] = T_wall
    return p


class Lattice:
    """A lattice living in a torch-allocated device workspace on the current
    torch stream (or the stream given)."""

    def __init__(self, params: Params, device="cuda:0", stream=None):
        import torch

        self.p = params
        self.nx, self.ny, self.nrow = params.nx, params.ny, params.ny + 1
        self.Q = (params.n_low ** 2, params.n_high ** 2)
        nbytes = lib().lb_workspace_bytes(C.byref(params))
        if nbytes == 0:
            _check(LB_EINVAL)
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        base = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _vp()
        _check(lib().lb_create_lattice(C.byref(params), _vp(base), nbytes, _vp(self.stream.cuda_stream),
                                       C.byref(h)))
        self._h = h
        dt, tau0, nt = C.c_double(), C.c_double(), C.c_int32()
        _check(lib().lb_get_info(h, C.byref(dt), C.byref(tau0), C.byref(nt)))
        self.dt, self.tau0, self.ntiles = dt.value, tau0.value, nt.value

    def close(self):
        if getattr(self, "_h", None):
            lib().lb_destroy_lattice(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- regions
    def _bands(self, lo, hi):
        lo = np.ascontiguousarray(np.broadcast_to(np.asarray(lo, dtype=np.int32), (self.ntiles,)))
        hi = np.ascontiguousarray(np.broadcast_to(np.asarray(hi, dtype=np.int32), (self.ntiles,)))
        return lo, hi

    def set_regions(self, lo, hi):
        lo, hi = self._bands(lo, hi)
        _check(lib().lb_set_regions(self._h, lo.ctypes.data_as(_ip), hi.ctypes.data_as(_ip)))

    def change_regions(self, lo, hi):
        lo, hi = self._bands(lo, hi)
        _check(lib().lb_change_regions(self._h, lo.ctypes.data_as(_ip), hi.ctypes.data_as(_ip)))

    def get_regions(self):
        lo = np.zeros(self.ntiles, dtype=np.int32)
        hi = np.zeros(self.ntiles, dtype=np.int32)
        _check(lib().lb_get_regions(self._h, lo.ctypes.data_as(_ip), hi.ctypes.data_as(_ip)))
        return lo, hi

    def update_regions(self, theta, bmin, bmax):
        _check(lib().lb_update_regions(self._h, theta, bmin, bmax))

    def region_counts(self):
        c = (C.c_int64 * 3)()
        _check(lib().lb_region_counts(self._h, c))
        return tuple(c)

    def set_strip_rows(self, rows):
        _check(lib().lb_set_strip_rows(self._h, rows))

    def strip_rows(self):
        r = (C.c_int32 * 2)()
        _check(lib().lb_get_strip_rows(self._h, r))
        return tuple(r)

    def set_merged_update(self, on=True):
        _check(lib().lb_set_merged_update(self._h, 1 if on else 0))

    def set_concurrency(self, on=True):
        _check(lib().lb_set_concurrency(self._h, 1 if on else 0))

    def work_shape(self):
        """((rows_low, rows_high), (order_low, order_high)) of the update kernels."""
        r, o = (C.c_int32 * 2)(), (C.c_int32 * 2)()
        _check(lib().lb_get_work_shape(self._h, r, o))
        return (r[0], r[1]), (o[0], o[1])

    def set_work_shape(self, rows, order):
        r, o = (C.c_int32 * 2)(*rows), (C.c_int32 * 2)(*order)
        _check(lib().lb_set_work_shape(self._h, r, o))

    def autotune(self, steps=50):
        """Pick the strip height of each set's update kernel by timing
        candidates; the lattice state is restored afterwards."""
        r = (C.c_int32 * 2)()
        _check(lib().lb_autotune(self._h, steps, r))
        return tuple(r)

    # ----------------------------------------------------------------- state
    def init_equilibrium(self, rho=None, ux=None, uy=None, T=None):
        """Equilibrium start; T (thermal lattices only) defaults to 1."""
        arrs = [None if a is None else _f64(np.broadcast_to(a, (self.nrow, self.nx))) for a in (rho, ux, uy, T)]
        ptrs = [None if a is None else _d(a) for a in arrs]
        if T is None:
            _check(lib().lb_init_equilibrium(self._h, *ptrs[:3]))
        else:
            _check(lib().lb_init_equilibrium_thermal(self._h, *ptrs))

    def step(self, n=1):
        _check(lib().lb_step(self._h, int(n)))

    @property
    def steps(self):
        return lib().lb_step_count(self._h)

    def moments(self):
        shp = (self.nrow, self.nx)
        r, ux, uy = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        _check(lib().lb_moments(self._h, _d(r), _d(ux), _d(uy), 0))
        return r, ux, uy

    def moments_device(self, rho, ux, uy):
        """Asynchronous moments into three float64 torch tensors on the device."""
        _check(lib().lb_moments(self._h, C.cast(rho.data_ptr(), _dp), C.cast(ux.data_ptr(), _dp),
                                C.cast(uy.data_ptr(), _dp), 1))

    def conservation(self):
        out = np.zeros(3)
        _check(lib().lb_conservation(self._h, _d(out)))
        return out

    def thermal_moments(self):
        """Temperature and heat flux (qx, qy) of every node, [ny+1][nx]."""
        shp = (self.nrow, self.nx)
        T, qx, qy = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        _check(lib().lb_thermal_moments(self._h, _d(T), _d(qx), _d(qy), 0))
        return T, qx, qy

    def energy(self):
        """Total energy: sum over nodes of 1/2 sum |xi|^2 f."""
        out = np.zeros(1)
        _check(lib().lb_energy(self._h, _d(out)))
        return float(out[0])

    def get_populations(self, which):
        f = np.zeros((self.Q[which], self.nrow, self.nx))
        _check(lib().lb_get_populations(self._h, which, _d(f)))
        return f

    def set_populations(self, which, f):
        f = _f64(f)
        assert f.shape == (self.Q[which], self.nrow, self.nx)
        _check(lib().lb_set_populations(self._h, which, _d(f)))

    def get_state(self) -> bytes:
        n = lib().lb_state_bytes(self._h)
        buf = C.create_string_buffer(n)
        _check(lib().lb_get_state(self._h, buf, n))
        return buf.raw

    def set_state(self, b: bytes):
        buf = C.create_string_buffer(b, len(b))
        _check(lib().lb_set_state(self._h, buf, len(b)))

    def indicator(self):
        B = np.zeros((self.nrow, self.nx))
        _check(lib().lb_indicator(self._h, _d(B), 0))
        return B

    # ---------------------------------------------------------------- timing
    def set_timing(self, on=True, every=1):
        """Events around the update launches of every `every`-th step."""
        _check(lib().lb_set_timing(self._h, int(every) if on else 0))

    def kernel_times(self):
        mh, ma = C.c_double(), C.c_double()
        nh, na = C.c_int64(), C.c_int64()
        _check(lib().lb_kernel_times(self._h, C.byref(mh), C.byref(nh), C.byref(ma), C.byref(na)))
        return mh.value, nh.value, ma.value, na.value

    # ------------------------------------------------------ learned closure
    def set_closure(self, params=None, norm=None):
        """Use the network (device float32 tensor of MLP_NPARAM values, norm =
        32 standardisation constants) in every D2Q9 -> D2Q36 lift; None
        restores the analytic projection."""
        if params is None:
            _check(lib().lb_set_closure(self._h, None, None))
            return
        nm = _norm(norm)
        _check(lib().lb_set_closure(self._h, _vp(params.data_ptr()), nm.ctypes.data_as(C.POINTER(C.c_float))))

    def set_closure_flags(self, on=True):
        """Count the nodes the network flags as above the threshold in
        update_regions (needs set_closure first)."""
        _check(lib().lb_set_closure_flags(self._h, 1 if on else 0))

    def closure_samples(self, nodes, theta):
        """Training samples at the listed nodes (device int32 tensor of
        j * nx + i) of the D2Q36 set: raw features [n, 10], raw targets
        [n, 6], flags [n] (device tensors, asynchronous)."""
        import torch

        n = nodes.numel()
        x = torch.empty((n, MLP_NIN), dtype=torch.float32, device=self.device)
        t = torch.empty((n, MLP_NREG), dtype=torch.float32, device=self.device)
        f = torch.empty((n,), dtype=torch.int32, device=self.device)
        _check(lib().lb_closure_samples(self._h, _vp(nodes.data_ptr()), n, theta, _vp(x.data_ptr()),
                                        _vp(t.data_ptr()), _vp(f.data_ptr())))
        return x, t, f


class Batch:
    """Independent lattices stepped together (lb_batch_*): one launch per
    kernel and velocity-set pair per step, optionally replayed from captured
    HIP graphs.  Runs on its own created stream (graphs cannot capture the
    null stream) and orders itself against the lattices' streams."""

    def __init__(self, lattices, stream=None):
        import torch

        self.lattices = list(lattices)
        n = len(self.lattices)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.lattices[0].device)
        arr = (_vp * n)(*[L._h.value for L in self.lattices])
        h = _vp()
        _check(lib().lb_batch_create(arr, n, _vp(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().lb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, segment_steps):
        _check(lib().lb_batch_set_graph(self._h, int(segment_steps)))

    def set_persistent(self, on=True):
        """One persistent launch per run of steps (workgroups own whole
        lattices and loop over the steps)."""
        _check(lib().lb_batch_set_persistent(self._h, 1 if on else 0))

    def step(self, n=1):
        _check(lib().lb_batch_step(self._h, int(n)))

    def set_strip_rows(self, low, high):
        _check(lib().lb_batch_set_strip_rows(self._h, int(low), int(high)))

    def autotune(self, steps=20):
        out = (C.c_int32 * 2)()
        _check(lib().lb_batch_autotune(self._h, int(steps), out))
        return out[0], out[1]

    def info(self):
        nodes, nl, nk = C.c_int64(), C.c_int32(), C.c_int32()
        _check(lib().lb_batch_info(self._h, C.byref(nodes), C.byref(nl), C.byref(nk)))
        return nodes.value, nl.value, nk.value


MLP_NIN, MLP_NH, MLP_NOUT, MLP_NREG = 10, 64, 8, 6


def _norm(norm):
    nm = np.ascontiguousarray(np.asarray(norm, dtype=np.float32).ravel())
    if nm.size != 32:
        raise ValueError("closure standardisation needs 32 values")
    return nm


def _stream(t, stream):
    import torch

    st = stream if stream is not None else torch.cuda.current_stream(t.device)
    return _vp(st.cuda_stream)


def mlp_param_count():
    return int(lib().lb_mlp_param_count())


class MLP:
    """Device FP32 training of the closure network through the C ABI (params,
    gradients and Adam moments are torch float32 tensors on one device)."""

    def __init__(self, params, max_batch, stream=None):
        import torch

        if params.numel() != mlp_param_count() or params.dtype != torch.float32:
            raise ValueError("params must be a float32 tensor of mlp_param_count() values")
        self.params = params.contiguous()
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        self.max_batch = max_batch
        self.ws = torch.empty(lib().lb_mlp_workspace_bytes(max_batch), dtype=torch.uint8, device=params.device)
        self.t = 0
        self.stream = stream

    def forward(self, x):
        import torch

        n = x.shape[0]
        if n > self.max_batch:
            raise ValueError("batch larger than the workspace")
        y = torch.empty((n, MLP_NOUT), dtype=torch.float32, device=x.device)
        _check(lib().lb_mlp_forward(_vp(self.params.data_ptr()), _vp(x.data_ptr()), _vp(y.data_ptr()), n,
                                    _vp(self.ws.data_ptr()), _stream(x, self.stream)))
        return y

    def loss_grad(self, x, t, flag):
        n = x.shape[0]
        if n > self.max_batch:
            raise ValueError("batch larger than the workspace")
        _check(lib().lb_mlp_loss_grad(_vp(self.params.data_ptr()), _vp(x.data_ptr()), _vp(t.data_ptr()),
                                      _vp(flag.data_ptr()), n, _vp(self.grad.data_ptr()),
                                      _vp(self.loss.data_ptr()), _vp(self.ws.data_ptr()),
                                      _stream(x, self.stream)))
        return self.loss, self.grad

    def adam(self, lr):
        self.t += 1
        _check(lib().lb_mlp_adam(_vp(self.params.data_ptr()), _vp(self.grad.data_ptr()), _vp(self.m.data_ptr()),
                                 _vp(self.v.data_ptr()), self.t, lr, _stream(self.params, self.stream)))


MLP_NOALLOC_MAX_N = 16384


def mlp_forward_noalloc(params, x, y, stream=None):
    """y[n, 8] = network(x[n, 10]) through the allocation-free entry point
    (float32 device tensors; n <= MLP_NOALLOC_MAX_N)."""
    _check(lib().lb_mlp_forward_noalloc(_vp(params.data_ptr()), _vp(x.data_ptr()), _vp(y.data_ptr()),
                                        x.shape[0], _stream(x, stream)))
    return y


def closure_eval(params, norm, kn_ref, tau_rho, rho_ref, f9, stream=None):
    """Closure coefficients [n, 36] of D2Q9 nodes f9 [n, 9] (float64 device
    tensor), network weights read through bf16 rounding."""
    import torch

    n = f9.shape[0]
    out = torch.empty((n, 36), dtype=torch.float64, device=f9.device)
    nm = _norm(norm)
    _check(lib().lb_closure_eval(_vp(params.data_ptr()), nm.ctypes.data_as(C.POINTER(C.c_float)), kn_ref,
                                 1 if tau_rho else 0, rho_ref, _vp(f9.data_ptr()), n, _vp(out.data_ptr()),
                                 _stream(f9, stream)))
    return out


def project(ns, eqs, nd, eqd, f_src, f_dst, closure=None, stream=None):
    """Hermite-moment projection of n nodes on the device: f_src [n, ns*ns],
    f_dst [n, nd*nd], closure [n, nd*nd] or None (float64 torch tensors)."""
    import torch

    n = f_src.shape[0]
    st = stream if stream is not None else torch.cuda.current_stream(f_src.device)
    cl = None if closure is None else _vp(closure.data_ptr())
    _check(lib().lb_project(ns, eqs, nd, eqd, _vp(f_src.data_ptr()), cl, _vp(f_dst.data_ptr()), n,
                            _vp(st.cuda_stream)))
