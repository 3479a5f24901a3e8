"""FP64 CPU oracle of the multiscale lattice Boltzmann step (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is written from the paper alone and shares no code,
header or table with the GPU library.  ``lbo.c`` holds the arithmetic; this
module only loads it with ctypes and marshals numpy arrays.

Each function names the passage of Meng, Zhang & Shan, "Multiscale lattice
Boltzmann approach to modeling gas flows", that it follows (see lbo.c).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbo.c")
_LIB = os.path.join(_HERE, "liblbo.so")

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-std=c11"]


def build() -> str:
    """Compile lbo.c into liblbo.so (always recompiles)."""
    cmd = ["gcc", *CFLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def _declare(L):
    L.lbo_he.restype = C.c_double
    L.lbo_he.argtypes = [C.c_int, C.c_double]
    L.lbo_gh_rule.argtypes = [C.c_int, _dp, _dp]
    L.lbo_vset.argtypes = [C.c_int, _dp, _dp, _dp]
    L.lbo_moments_node.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
    L.lbo_moments_node_t.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp]
    L.lbo_heat_flux_node.argtypes = [C.c_int, _dp, _dp, _dp]
    L.lbo_equilibrium_t.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, _dp]
    L.lbo_force_t.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                              C.c_double, C.c_double, _dp]
    L.lbo_project_t.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
    L.lbo_init_equilibrium_t.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
    L.lbo_thermal.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.lbo_energy.restype = C.c_double
    L.lbo_energy.argtypes = [C.c_void_p]
    L.lbo_hermite_coeffs.argtypes = [C.c_int, _dp, _dp]
    L.lbo_from_coeffs.argtypes = [C.c_int, _dp, _dp]
    L.lbo_equilibrium.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, _dp]
    L.lbo_force.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                            C.c_double, C.c_double, _dp]
    L.lbo_project.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp]
    L.lbo_face_value.restype = C.c_double
    L.lbo_face_value.argtypes = [C.c_double] * 5
    L.lbo_create.restype = C.c_void_p
    L.lbo_create.argtypes = [_dp, _ip]
    L.lbo_destroy.argtypes = [C.c_void_p]
    L.lbo_set_regions.argtypes = [C.c_void_p, _ip, _ip]
    L.lbo_update_regions.argtypes = [C.c_void_p, _ip, _ip]
    L.lbo_region.argtypes = [C.c_void_p, C.c_int, C.c_int]
    L.lbo_init_equilibrium.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.lbo_set_populations.argtypes = [C.c_void_p, C.c_int, _dp]
    L.lbo_get_populations.argtypes = [C.c_void_p, C.c_int, _dp]
    L.lbo_step.argtypes = [C.c_void_p, C.c_long]
    L.lbo_moments.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.lbo_conservation.argtypes = [C.c_void_p, _dp]
    L.lbo_set_closure.argtypes = [C.c_void_p, _dp]
    L.lbo_indicator.argtypes = [C.c_void_p, _dp]
    L.lbo_bands_from_indicator.argtypes = [C.c_void_p, _dp, C.c_double, C.c_int, C.c_int, _ip, _ip]
    L.lbo_step_count.restype = C.c_long
    L.lbo_step_count.argtypes = [C.c_void_p]
    L.lbo_set_threads.argtypes = [C.c_int]
    L.lbo_threads.restype = C.c_int


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- node level
def hermite(k: int, x: float) -> float:
    """Probabilists' Hermite polynomial He_k(x) (1D form of Eq. hermipol)."""
    return lib().lbo_he(int(k), float(x))


def gh_rule(n: int):
    """n-point Gauss-Hermite abscissae (roots of He_n) and Eq. (weight) weights."""
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().lbo_gh_rule(n, _d(x), _d(w)) != 0:
        raise ValueError(f"no {n}-point rule")
    return x, w


def vset(n: int):
    """Tensor-product D2Q(n*n) set: alpha = p + n q, xi = (x_p, x_q), w = w_p w_q."""
    Q = n * n
    cx, cy, w = np.zeros(Q), np.zeros(Q), np.zeros(Q)
    lib().lbo_vset(n, _d(cx), _d(cy), _d(w))
    return cx, cy, w


def moments(n: int, f):
    f = _f64(f)
    r, ux, uy = C.c_double(), C.c_double(), C.c_double()
    lib().lbo_moments_node(n, _d(f), C.byref(r), C.byref(ux), C.byref(uy))
    return r.value, ux.value, uy.value


def moments_t(n: int, f):
    """rho, ux, uy and the temperature T from sum xi^2 f = rho (u^2 + 2 T)."""
    f = _f64(f)
    r, ux, uy, T = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    lib().lbo_moments_node_t(n, _d(f), C.byref(r), C.byref(ux), C.byref(uy), C.byref(T))
    return r.value, ux.value, uy.value, T.value


def heat_flux(n: int, f):
    """q = 1/2 sum (xi - u) |xi - u|^2 f of one node."""
    f = _f64(f)
    qx, qy = C.c_double(), C.c_double()
    lib().lbo_heat_flux_node(n, _d(f), C.byref(qx), C.byref(qy))
    return qx.value, qy.value


def hermite_coeffs(n: int, f):
    """a[k, m] = sum_alpha f He_k(xi_x) He_m(xi_y) (Eq. an, component form)."""
    f = _f64(f)
    a = np.zeros(n * n)
    lib().lbo_hermite_coeffs(n, _d(f), _d(a))
    return a.reshape(n, n)


def from_coeffs(n: int, a):
    a = _f64(a).reshape(-1)
    f = np.zeros(n * n)
    lib().lbo_from_coeffs(n, _d(a), _d(f))
    return f


def equilibrium(n: int, order: int, rho, ux, uy, T=None):
    """Order-N Hermite equilibrium, Eq. (approxfeq); T = None is the
    isothermal form (T = 1)."""
    f = np.zeros(n * n)
    if T is None:
        lib().lbo_equilibrium(n, order, rho, ux, uy, _d(f))
    else:
        lib().lbo_equilibrium_t(n, order, rho, ux, uy, T, _d(f))
    return f


def force(n: int, order: int, rho, ux, uy, gx, gy, T=None):
    """Hermite body-force term g_alpha up to order N (Sec. 2.1)."""
    g = np.zeros(n * n)
    if T is None:
        lib().lbo_force(n, order, rho, ux, uy, gx, gy, _d(g))
    else:
        lib().lbo_force_t(n, order, rho, ux, uy, T, gx, gy, _d(g))
    return g


def project(ns: int, ords: int, nd: int, ordd: int, fs, closure=None, thermal=False):
    """Hermite-moment projection of one node's populations from set ns to nd
    (thermal: the equilibria at the node's own temperature)."""
    fs = _f64(fs)
    fd = np.zeros(nd * nd)
    cl = None if closure is None else _d(_f64(closure))
    fn = lib().lbo_project_t if thermal else lib().lbo_project
    fn(ns, ords, nd, ordd, _d(fs), cl, _d(fd))
    return fd


def face_value(nu, fm1, f0, fp1, fp2) -> float:
    """TVD/minmod face value F_{i+1/2} of Sec. 3.1 (mirrored for nu < 0)."""
    return lib().lbo_face_value(nu, fm1, f0, fp1, fp2)


def set_threads(n: int) -> None:
    """Threads of the oracle's node loops (OpenMP over rows); results are
    the same for any count."""
    lib().lbo_set_threads(int(n))


def threads() -> int:
    return int(lib().lbo_threads())


def default_dt(n_high: int, cfl: float = 0.5) -> float:
    """Time step with per-axis Courant number cfl for the fastest abscissa."""
    x, _ = gh_rule(n_high)
    return cfl / float(np.max(np.abs(x)))


# ------------------------------------------------------------------- lattice
TAU_CONST, TAU_RHO = 0, 1
XBC_PERIODIC, XBC_PRESSURE = 0, 1
YBC_WALLS, YBC_PERIODIC, YBC_SHEAR = 0, 1, 2
IFACE_HERMITE, IFACE_PAPER = 0, 1
REG_LOW, REG_HIGH, REG_IFACE = 0, 1, 2


class Lattice:
    """Oracle lattice: two velocity sets (low, high), bands of the high set at
    each wall per column tile, rows 0..ny.  Populations are [Q][ny+1][nx].
    u_osc, omega_osc: the bottom wall also moves along x with
    u_osc sin(omega_osc t), t the time of the level being computed
    (oscillatory Couette flow, Sec. 3.5).  ybc=YBC_SHEAR: a wall at the
    bottom and an imposed shear rate `shear` above the top row (Kramers'
    problem, Sec. 3.3).  thermal=True: every node's temperature comes from
    its energy moment and enters the equilibrium (Eq. demoeq), the
    relaxation rate (p / mu), the interface (T_I) and the indicator (heat
    flux); the walls are at T_wall = (bottom, top)."""

    def __init__(self, nx, ny, *, kn, n_low=3, n_high=3, eq_low=2, eq_high=None,
                 force_low=None, force_high=None, dt=None, rho_ref=1.0, tau_mode=TAU_CONST,
                 gx=0.0, gy=0.0, u_wall=((0.0, 0.0), (0.0, 0.0)), xbc=XBC_PERIODIC,
                 ybc=YBC_WALLS, rho_in=1.0, rho_out=1.0, iface=IFACE_HERMITE, tile_w=None,
                 u_osc=0.0, omega_osc=0.0, shear=0.0, thermal=False, T_wall=(1.0, 1.0)):
        eq_high = eq_low if eq_high is None else eq_high
        force_low = eq_low if force_low is None else force_low
        force_high = eq_high if force_high is None else force_high
        if dt is None:
            dt = default_dt(max(n_low, n_high))
        tile_w = nx if tile_w is None else tile_w
        self.nx, self.ny, self.nrow = nx, ny, ny + 1
        self.n = (n_low, n_high)
        self.Q = (n_low * n_low, n_high * n_high)
        self.dt = dt
        self.tile_w = tile_w
        self.ntiles = (nx + tile_w - 1) // tile_w
        dp = np.array([kn, rho_ref, dt, gx, gy, u_wall[0][0], u_wall[0][1], u_wall[1][0],
                       u_wall[1][1], rho_in, rho_out, u_osc, omega_osc, shear,
                       T_wall[0], T_wall[1]], dtype=np.float64)
        ip = np.array([nx, ny, n_low, n_high, eq_low, eq_high, force_low, force_high,
                       tau_mode, xbc, ybc, iface, tile_w, int(bool(thermal))], dtype=np.int32)
        self.thermal = bool(thermal)
        self._h = lib().lbo_create(_d(dp), _i(ip))
        if not self._h:
            raise ValueError("oracle lattice creation failed")
        self.set_regions(0, 0)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().lbo_destroy(h)
            self._h = None

    def _bands(self, blo, bhi):
        blo = np.broadcast_to(np.asarray(blo, dtype=np.int32), (self.ntiles,)).copy()
        bhi = np.broadcast_to(np.asarray(bhi, dtype=np.int32), (self.ntiles,)).copy()
        return blo, bhi

    def set_regions(self, blo, bhi):
        """High-set rows at the bottom (blo) and top (bhi) wall, per tile."""
        blo, bhi = self._bands(blo, bhi)
        lib().lbo_set_regions(self._h, _i(blo), _i(bhi))

    def update_regions(self, blo, bhi):
        """Re-decompose, converting switched nodes by the Hermite projection."""
        blo, bhi = self._bands(blo, bhi)
        lib().lbo_update_regions(self._h, _i(blo), _i(bhi))

    def region(self):
        r = np.zeros((self.nrow, self.nx), dtype=np.int32)
        for j in range(self.nrow):
            for i in range(self.nx):
                r[j, i] = lib().lbo_region(self._h, i, j)
        return r

    def init_equilibrium(self, rho=None, ux=None, uy=None, T=None):
        """Equilibrium start; T (thermal lattices) defaults to 1."""
        args = []
        for a in (rho, ux, uy, T):
            if a is None:
                args.append(None)
            else:
                a = _f64(np.broadcast_to(a, (self.nrow, self.nx)))
                args.append(a)
        ptrs = [None if a is None else _d(a) for a in args]
        lib().lbo_init_equilibrium_t(self._h, *ptrs)

    def set_populations(self, which, f):
        f = _f64(f)
        assert f.shape == (self.Q[which], self.nrow, self.nx)
        lib().lbo_set_populations(self._h, which, _d(f))

    def get_populations(self, which):
        f = np.zeros((self.Q[which], self.nrow, self.nx))
        lib().lbo_get_populations(self._h, which, _d(f))
        return f

    def set_closure(self, c):
        if c is None:
            lib().lbo_set_closure(self._h, None)
            return
        c = _f64(c)
        assert c.shape == (self.Q[1], self.nrow, self.nx)
        lib().lbo_set_closure(self._h, _d(c))

    def step(self, n=1):
        lib().lbo_step(self._h, int(n))

    @property
    def steps(self):
        return lib().lbo_step_count(self._h)

    def moments(self):
        shp = (self.nrow, self.nx)
        r, ux, uy = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        lib().lbo_moments(self._h, _d(r), _d(ux), _d(uy))
        return r, ux, uy

    def conservation(self):
        out = np.zeros(3)
        lib().lbo_conservation(self._h, _d(out))
        return out

    def thermal_moments(self):
        """Temperature and heat flux (qx, qy) of every node, [ny+1][nx]."""
        shp = (self.nrow, self.nx)
        T, qx, qy = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        lib().lbo_thermal(self._h, _d(T), _d(qx), _d(qy))
        return T, qx, qy

    def energy(self):
        """Total energy, the sum over nodes of 1/2 sum |xi|^2 f."""
        return float(lib().lbo_energy(self._h))

    def indicator(self):
        B = np.zeros((self.nrow, self.nx))
        lib().lbo_indicator(self._h, _d(B))
        return B

    def bands_from_indicator(self, B, theta, bmin, bmax):
        B = _f64(B)
        blo = np.zeros(self.ntiles, dtype=np.int32)
        bhi = np.zeros(self.ntiles, dtype=np.int32)
        lib().lbo_bands_from_indicator(self._h, _d(B), theta, bmin, bmax, _i(blo), _i(bhi))
        return blo, bhi
