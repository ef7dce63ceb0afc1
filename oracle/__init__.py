"""ctypes front end of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the product path never does.  Arrays are numpy,
row-major: a scalar field is ``(ny, nx)``, populations are ``(9, ny, nx)``.
``precision="f64"`` is the oracle proper; ``precision="f32"`` is its
single-precision twin, used only to size single-precision tolerances.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}
_DT = {"f64": np.float64, "f32": np.float32}
_NAME = {"f64": "liboracle.so", "f32": "liboracle_f32.so"}

_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_vp = ctypes.c_void_p


def lib(precision="f64"):
    if precision not in _LIBS:
        path = os.path.join(_HERE, _NAME[precision])
        if not os.path.exists(path):
            raise RuntimeError(f"oracle library {path} is not built; run oracle/build.py")
        L = ctypes.CDLL(path)
        L.orc_d2q9.argtypes = [_vp, _vp, _vp]
        L.orc_tables.argtypes = [_vp, _vp, _vp, _vp, _dbl, _dbl]
        L.orc_real_bytes.restype = ctypes.c_int
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_init.argtypes = [_i64, _i64, _vp, _vp, _vp, _vp]
        L.orc_moments.argtypes = [_i64, _i64, _vp, _vp, _vp, _vp]
        L.orc_psi.argtypes = [_i64, _dbl, _vp, _vp]
        L.orc_force.argtypes = [_i64, _i64, _dbl, _dbl, _vp, _vp, _vp]
        L.orc_collide.argtypes = [_i64, _i64, _dbl, _vp, _vp, _vp, _vp]
        L.orc_stream.argtypes = [_i64, _i64, _vp, _vp]
        L.orc_step.argtypes = [_i64, _i64, _dbl, _dbl, _dbl, _dbl, _vp, _i64]
        L.orc_step.restype = ctypes.c_int
        L.orc_observables.argtypes = [_i64, _i64, _dbl, _dbl, _dbl, _vp, _vp]
        L.orc_observables.restype = ctypes.c_int
        L.orc_run.argtypes = [_i64, _i64, _dbl, _dbl, _dbl, _dbl, _vp, _i64, _i64, _vp, _i64]
        L.orc_run.restype = ctypes.c_int64
        want = 8 if precision == "f64" else 4
        if L.orc_real_bytes() != want:
            raise RuntimeError(f"{path}: unexpected real size {L.orc_real_bytes()}")
        _LIBS[precision] = L
    return _LIBS[precision]


def _p(a):
    return a.ctypes.data_as(_vp)


def _field(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def threads(precision="f64"):
    """OpenMP threads the oracle's loops run on."""
    return lib(precision).orc_threads()


def set_threads(n, precision="f64"):
    """Run the oracle's loops on n OpenMP threads."""
    lib(precision).orc_set_threads(int(n))


def d2q9():
    cx = np.zeros(9, np.int8)
    cy = np.zeros(9, np.int8)
    w = np.zeros(9, np.float64)
    lib().orc_d2q9(_p(cx), _p(cy), _p(w))
    return cx, cy, w


def tables(G1, G2):
    """Link table of the two-belt force: (cx[24], cy[24], K[24], KE[25])."""
    cx = np.zeros(24, np.int8)
    cy = np.zeros(24, np.int8)
    K = np.zeros(24, np.float64)
    KE = np.zeros(25, np.float64)
    lib().orc_tables(_p(cx), _p(cy), _p(K), _p(KE), G1, G2)
    return cx, cy, K, KE


def init(rho, ux=None, uy=None, precision="f64"):
    rho = _field(rho, np.float64)
    ny, nx = rho.shape
    f = np.zeros((9, ny, nx), _DT[precision])
    ux = None if ux is None else _field(ux, np.float64)
    uy = None if uy is None else _field(uy, np.float64)
    lib(precision).orc_init(nx, ny, _p(rho), None if ux is None else _p(ux),
                            None if uy is None else _p(uy), _p(f))
    return f


def moments(f, precision="f64"):
    """(rho, jx, jy) with j = sum_i c_i f_i (momentum density)."""
    f = _field(f, _DT[precision])
    _, ny, nx = f.shape
    out = [np.zeros((ny, nx), _DT[precision]) for _ in range(3)]
    lib(precision).orc_moments(nx, ny, _p(f), *[_p(o) for o in out])
    return tuple(out)


def psi(rho, rho0=1.0, precision="f64"):
    rho = _field(rho, _DT[precision])
    out = np.zeros_like(rho)
    lib(precision).orc_psi(rho.size, rho0, _p(rho), _p(out))
    return out


def force(psi_field, G1, G2, precision="f64"):
    p = _field(psi_field, _DT[precision])
    ny, nx = p.shape
    Fx = np.zeros_like(p)
    Fy = np.zeros_like(p)
    lib(precision).orc_force(nx, ny, G1, G2, _p(p), _p(Fx), _p(Fy))
    return Fx, Fy


def collide(f, Fx, Fy, tau, precision="f64"):
    f = _field(f, _DT[precision])
    _, ny, nx = f.shape
    Fx = _field(Fx, _DT[precision])
    Fy = _field(Fy, _DT[precision])
    out = np.zeros_like(f)
    lib(precision).orc_collide(nx, ny, tau, _p(f), _p(Fx), _p(Fy), _p(out))
    return out


def stream(fpost, precision="f64"):
    fpost = _field(fpost, _DT[precision])
    _, ny, nx = fpost.shape
    out = np.zeros_like(fpost)
    lib(precision).orc_stream(nx, ny, _p(fpost), _p(out))
    return out


def step(f, nsteps, tau, rho0, G1, G2, precision="f64"):
    """Advance the pre-collision populations by nsteps; returns a new array."""
    f = np.array(f, dtype=_DT[precision], order="C", copy=True)
    _, ny, nx = f.shape
    if lib(precision).orc_step(nx, ny, tau, rho0, G1, G2, _p(f), nsteps) != 0:
        raise MemoryError("orc_step")
    return f


def observables(f, rho0, G1, G2, precision="f64"):
    """{M, E_s, E_m, sum psi^2, E_bulk} of the pre-collision state f."""
    f = _field(f, _DT[precision])
    _, ny, nx = f.shape
    out = np.zeros(5, np.float64)
    if lib(precision).orc_observables(nx, ny, rho0, G1, G2, _p(f), _p(out)) != 0:
        raise MemoryError("orc_observables")
    return out


def run(f, nsteps, tau, rho0, G1, G2, log_every, precision="f64"):
    """Run nsteps from f; returns (f_final, trace) with trace rows
    {t, M, E_s, E_m, sum psi^2, E_bulk} at every t % log_every == 0, t in [0, nsteps]."""
    f = np.array(f, dtype=_DT[precision], order="C", copy=True)
    _, ny, nx = f.shape
    cap = nsteps // log_every + 1 if log_every > 0 else 0
    trace = np.zeros((max(cap, 1), 6), np.float64)
    rows = lib(precision).orc_run(nx, ny, tau, rho0, G1, G2, _p(f), nsteps,
                                  log_every, _p(trace), cap)
    if rows < 0:
        raise MemoryError("orc_run")
    return f, trace[:rows]


# ---------------------------------------------------------------------------
# The lb_* entry points of the oracle libraries (oracle_abi.c): the same call
# sequence as the GPU library, on host memory.
# ---------------------------------------------------------------------------
class Params(ctypes.Structure):
    """The interface's parameter block (layout of the C declaration)."""
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("log_every", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("steps_per_launch", ctypes.c_int32),
                ("trace_cap", ctypes.c_int64),
                ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("G1", ctypes.c_double), ("G2", ctypes.c_double),
                ("rho_ref", ctypes.c_double)]


_ABI = {}


def abi(precision="f64"):
    """The oracle library with the lb_* signatures set."""
    if precision not in _ABI:
        L = lib(precision)
        P = ctypes.POINTER(Params)
        sig = {
            "lb_workspace_bytes": (ctypes.c_size_t, [P]),
            "lb_validate": (ctypes.c_int, [P]),
            "lb_launch_shape": (ctypes.c_int, [P, _vp, _vp, _vp, _vp]),
            "lb_two_step_shape": (ctypes.c_int, [P, _vp, _vp, _vp]),
            "lb_init": (ctypes.c_int, [ctypes.POINTER(_vp), P, _vp, ctypes.c_size_t,
                                       _vp, _vp, _vp, ctypes.c_int, _vp]),
            "lb_step": (ctypes.c_int, [_vp, _i64]),
            "lb_moments": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int]),
            "lb_pseudo_energy": (ctypes.c_int, [_vp, _vp]),
            "lb_trace": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
            "lb_time": (ctypes.c_int, [_vp, _vp]),
            "lb_get_state": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
            "lb_set_state": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _i64]),
            "lb_tables": (ctypes.c_int, [P, _vp, _vp, _vp, _vp]),
            "lb_destroy": (ctypes.c_int, [_vp]),
            "lb_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _ABI[precision] = L
    return _ABI[precision]


class AbiLattice:
    """One lattice driven through the oracle's lb_* entry points."""

    def __init__(self, rho_init, *, G1, G2, tau=1.0, rho0=1.0, log_every=0, trace_cap=0,
                 precision="f64", ux_init=None, uy_init=None):
        self.L = abi(precision)
        self.precision = precision
        rho = np.ascontiguousarray(rho_init, dtype=np.float64)
        self.ny, self.nx = rho.shape
        self.p = Params(nx=self.nx, ny=self.ny, storage=0 if precision == "f64" else 1,
                        log_every=log_every, trace_cap=trace_cap, tau=tau, rho0=rho0, G1=G1, G2=G2)
        nbytes = self.L.lb_workspace_bytes(ctypes.byref(self.p))
        if nbytes == 0:
            raise ValueError(self.L.lb_last_error().decode())
        self.ws = np.zeros(nbytes, np.uint8)
        self.ctx = _vp()
        u = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (ux_init, uy_init)]
        self._ok(self.L.lb_init(ctypes.byref(self.ctx), ctypes.byref(self.p), self.ws.ctypes.data,
                                nbytes, rho.ctypes.data, *[None if a is None else a.ctypes.data for a in u],
                                0, None))
        self.trace_cap = trace_cap

    def _ok(self, rc):
        if rc != 0:
            raise RuntimeError(f"oracle lb_* call failed ({rc}): {self.L.lb_last_error().decode()}")
        return rc

    def step(self, n):
        self._ok(self.L.lb_step(self.ctx, n))

    def moments(self):
        out = [np.empty((self.ny, self.nx)) for _ in range(3)]
        self._ok(self.L.lb_moments(self.ctx, *[a.ctypes.data for a in out], 0))
        return tuple(out)

    def pseudo_energy(self):
        out = np.empty(6)
        self._ok(self.L.lb_pseudo_energy(self.ctx, out.ctypes.data))
        return out

    def trace(self):
        out = np.empty((max(self.trace_cap, 1), 6))
        n = ctypes.c_int64()
        self._ok(self.L.lb_trace(self.ctx, out.ctypes.data, self.trace_cap, ctypes.byref(n)))
        return out[:n.value].copy()

    def get_state(self):
        out = np.empty((9, self.ny, self.nx), _DT[self.precision])
        self._ok(self.L.lb_get_state(self.ctx, out.ctypes.data, 0))
        return out

    def close(self):
        if self.ctx:
            self.L.lb_destroy(self.ctx)
            self.ctx = _vp()
