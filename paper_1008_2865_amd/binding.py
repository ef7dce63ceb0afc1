"""ctypes binding of liblb.so: the lb_* entry points of include/lb.h, same
names, argument marshalling only.

Every step of the method runs in the HIP library; this module converts
Python values to C arguments and C status codes to exceptions.  Importing it
fails loudly (``LBLibraryMissing``) when liblb.so has not been built: there is
no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LB_LIBRARY", os.path.join(HERE, "liblb.so"))

LB_F64, LB_F32, LB_F16DEV = 0, 1, 2
LB_OK, LB_ERR_INVALID, LB_ERR_HIP, LB_ERR_NONFINITE, LB_ERR_STATE = 0, -1, -2, -3, -4
STATUS_NAMES = {LB_ERR_INVALID: "LB_ERR_INVALID", LB_ERR_HIP: "LB_ERR_HIP",
                LB_ERR_NONFINITE: "LB_ERR_NONFINITE", LB_ERR_STATE: "LB_ERR_STATE"}
STORAGE_BYTES = {LB_F64: 8, LB_F32: 4, LB_F16DEV: 2}


class LBLibraryMissing(ImportError):
    pass


class LBError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


class lb_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("log_every", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("steps_per_launch", ctypes.c_int32),
                ("trace_cap", ctypes.c_int64),
                ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("G1", ctypes.c_double), ("G2", ctypes.c_double),
                ("rho_ref", ctypes.c_double)]


class lb_adj_loss(ctypes.Structure):
    _fields_ = [("E_target", ctypes.c_double), ("beta", ctypes.c_double),
                ("eps", ctypes.c_double)]


_vp = ctypes.c_void_p
_P = ctypes.POINTER(lb_params)

# name -> (restype, argtypes), in the order of include/lb.h
SIGNATURES = {
    "lb_workspace_bytes": (ctypes.c_size_t, [_P]),
    "lb_validate": (ctypes.c_int, [_P]),
    "lb_launch_shape": (ctypes.c_int, [_P, _vp, _vp, _vp, _vp]),
    "lb_two_step_shape": (ctypes.c_int, [_P, _vp, _vp, _vp]),
    "lb_init": (ctypes.c_int, [ctypes.POINTER(_vp), _P, _vp, ctypes.c_size_t,
                               _vp, _vp, _vp, ctypes.c_int, _vp]),
    "lb_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "lb_moments": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int]),
    "lb_pseudo_energy": (ctypes.c_int, [_vp, _vp]),
    "lb_trace": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, _vp]),
    "lb_time": (ctypes.c_int, [_vp, _vp]),
    "lb_get_state": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "lb_set_state": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int64]),
    "lb_tables": (ctypes.c_int, [_P, _vp, _vp, _vp, _vp]),
    "lb_destroy": (ctypes.c_int, [_vp]),
    "lb_last_error": (ctypes.c_char_p, []),
    "lb_batch_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int32]),
    "lb_batch_init": (ctypes.c_int, [ctypes.POINTER(_vp), _P, ctypes.c_int32, _vp, ctypes.c_size_t,
                                     ctypes.POINTER(_vp), ctypes.c_int, _vp]),
    "lb_batch_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "lb_batch_use_graphs": (ctypes.c_int, [_vp, ctypes.c_int]),
    "lb_batch_two_step_shape": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "lb_batch_two_step_tile": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "lb_batch_member": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(_vp)]),
    "lb_batch_destroy": (ctypes.c_int, [_vp]),
    "lb_adj_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int64, ctypes.c_int32]),
    "lb_adj_init": (ctypes.c_int, [ctypes.POINTER(_vp), _P, ctypes.c_int64, ctypes.c_int32, _vp,
                                   ctypes.c_size_t, _vp]),
    "lb_adj_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(lb_adj_loss), _vp]),
    "lb_adj_backward": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int]),
    "lb_adj_destroy": (ctypes.c_int, [_vp]),
    "lb_sk_shells": (ctypes.c_int, [ctypes.c_int32, _vp]),
    "lb_sk_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "lb_sk_init": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32, _vp, ctypes.c_size_t, _vp]),
    "lb_sk_compute": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_int32, _vp, _vp]),
    "lb_sk_destroy": (ctypes.c_int, [_vp]),
    "lb_pseudo_energy_state": (ctypes.c_int, [_P, _vp, ctypes.c_double, _vp, _vp]),
}

_lib = None


def lib():
    """The loaded liblb.so (raises LBLibraryMissing if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LBLibraryMissing(
                f"{LIB_PATH} not found: build it with `python -m paper_1008_2865_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != LB_OK:
        raise LBError(rc, lib().lb_last_error().decode(errors="replace"))
    return rc


def _ptr(a):
    """Address of a numpy array, a torch tensor, an int or None."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def make_params(nx, ny, *, storage=LB_F32, tau=1.0, rho0=1.0, G1=-4.9, G2=0.0,
                log_every=0, trace_cap=0, tile_x=0, tile_y=0, tile_rows=0, rho_ref=0.0,
                steps_per_launch=0):
    return lb_params(nx=nx, ny=ny, storage=storage, log_every=log_every,
                     tile_x=tile_x, tile_y=tile_y, tile_rows=tile_rows,
                     steps_per_launch=steps_per_launch,
                     trace_cap=trace_cap, tau=tau, rho0=rho0, G1=G1, G2=G2, rho_ref=rho_ref)


def lb_workspace_bytes(p):
    return lib().lb_workspace_bytes(ctypes.byref(p))


def lb_validate(p):
    return lib().lb_validate(ctypes.byref(p))


def lb_launch_shape(p):
    """(tile_x, tile_y, tile_rows, blocks) of the step kernel."""
    tx, ty, tr, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lb_launch_shape(ctypes.byref(p), ctypes.byref(tx), ctypes.byref(ty),
                                 ctypes.byref(tr), ctypes.byref(nb)))
    return tx.value, ty.value, tr.value, nb.value


def lb_two_step_shape(p):
    """(tile_x, tile_y, blocks) of the two-step launches, zeros if unused."""
    tx, ty, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lb_two_step_shape(ctypes.byref(p), ctypes.byref(tx), ctypes.byref(ty),
                                   ctypes.byref(nb)))
    return tx.value, ty.value, nb.value


def lb_init(p, workspace, nbytes, rho_init, ux_init=None, uy_init=None,
            inputs_on_device=False, stream=0):
    ctx = _vp()
    _check(lib().lb_init(ctypes.byref(ctx), ctypes.byref(p), _ptr(workspace), nbytes,
                         _ptr(rho_init), _ptr(ux_init), _ptr(uy_init),
                         int(bool(inputs_on_device)), stream or None))
    return ctx.value


def lb_step(ctx, n):
    return _check(lib().lb_step(ctx, n))


def lb_moments(ctx, rho=None, ux=None, uy=None, on_device=False):
    return _check(lib().lb_moments(ctx, _ptr(rho), _ptr(ux), _ptr(uy), int(bool(on_device))))


def lb_pseudo_energy(ctx, out):
    return _check(lib().lb_pseudo_energy(ctx, _ptr(out)))


def lb_trace(ctx, out, cap):
    n = ctypes.c_int64()
    _check(lib().lb_trace(ctx, _ptr(out), cap, ctypes.byref(n)))
    return n.value


def lb_time(ctx):
    t = ctypes.c_int64()
    _check(lib().lb_time(ctx, ctypes.byref(t)))
    return t.value


def lb_get_state(ctx, dst, on_device=False):
    return _check(lib().lb_get_state(ctx, _ptr(dst), int(bool(on_device))))


def lb_set_state(ctx, src, t, on_device=False):
    return _check(lib().lb_set_state(ctx, _ptr(src), int(bool(on_device)), t))


def lb_tables(p, cx, cy, K, KE):
    return _check(lib().lb_tables(ctypes.byref(p), _ptr(cx), _ptr(cy), _ptr(K), _ptr(KE)))


def lb_destroy(ctx):
    return _check(lib().lb_destroy(ctx))


def lb_last_error():
    return lib().lb_last_error().decode(errors="replace")


def _params_array(ps):
    arr = (lb_params * len(ps))()
    for i, p in enumerate(ps):
        arr[i] = p
    return arr


def lb_batch_workspace_bytes(ps):
    return lib().lb_batch_workspace_bytes(_params_array(ps), len(ps))


def lb_batch_init(ps, workspace, nbytes, rho_inits, inputs_on_device=False, stream=0):
    arr = _params_array(ps)
    ptrs = (_vp * len(ps))(*[_ptr(r) for r in rho_inits])
    b = _vp()
    _check(lib().lb_batch_init(ctypes.byref(b), arr, len(ps), _ptr(workspace), nbytes, ptrs,
                               int(bool(inputs_on_device)), stream or None))
    return b.value


def lb_batch_step(b, n):
    return _check(lib().lb_batch_step(b, n))


def lb_batch_use_graphs(b, enable):
    return _check(lib().lb_batch_use_graphs(b, int(bool(enable))))


def lb_batch_two_step_tile(b, tile_y):
    return _check(lib().lb_batch_two_step_tile(b, int(tile_y)))


def lb_batch_two_step_shape(b):
    """(tile_x, tile_y, blocks) of the batch's two-step launches, zeros if unused."""
    tx, ty, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lb_batch_two_step_shape(b, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(nb)))
    return tx.value, ty.value, nb.value


def lb_batch_member(b, i):
    m = _vp()
    _check(lib().lb_batch_member(b, i, ctypes.byref(m)))
    return m.value


def lb_batch_destroy(b):
    return _check(lib().lb_batch_destroy(b))


def lb_adj_workspace_bytes(p, nsteps, checkpoint_every):
    return lib().lb_adj_workspace_bytes(ctypes.byref(p), nsteps, checkpoint_every)


def lb_adj_init(p, nsteps, checkpoint_every, workspace, nbytes, stream=0):
    a = _vp()
    _check(lib().lb_adj_init(ctypes.byref(a), ctypes.byref(p), nsteps, checkpoint_every,
                             _ptr(workspace), nbytes, stream or None))
    return a.value


def lb_adj_forward(a, rho_init, G1, G2, E_target, beta, eps, on_device=False):
    """(L, E(T), A(T), M(T))."""
    out = (ctypes.c_double * 4)()
    loss = lb_adj_loss(E_target=E_target, beta=beta, eps=eps)
    _check(lib().lb_adj_forward(a, _ptr(rho_init), int(bool(on_device)), G1, G2,
                                ctypes.byref(loss), out))
    return tuple(out)


def lb_adj_backward(a, drho, on_device=False):
    """(dL/dG1, dL/dG2); dL/drho_init is written into drho."""
    dG = (ctypes.c_double * 2)()
    _check(lib().lb_adj_backward(a, dG, _ptr(drho), int(bool(on_device))))
    return dG[0], dG[1]


def lb_adj_destroy(a):
    return _check(lib().lb_adj_destroy(a))


def lb_sk_shells(L):
    n = ctypes.c_int32()
    _check(lib().lb_sk_shells(L, ctypes.byref(n)))
    return n.value


def lb_sk_workspace_bytes(L):
    return lib().lb_sk_workspace_bytes(L)


def lb_sk_init(L, workspace, nbytes, stream=0):
    s = _vp()
    _check(lib().lb_sk_init(ctypes.byref(s), L, _ptr(workspace), nbytes, stream or None))
    return s.value


def lb_sk_compute(s, rho, shell, counts, kbar_out=None, spectrum=None, on_device=False):
    """Fills shell / counts (numpy float64 / int64 arrays or None); returns kbar."""
    cap = len(shell) if shell is not None else (len(counts) if counts is not None else 0)
    kb = ctypes.c_double()
    _check(lib().lb_sk_compute(s, _ptr(rho), int(bool(on_device)), _ptr(shell), _ptr(counts),
                               cap, ctypes.byref(kb), _ptr(spectrum)))
    return kb.value


def lb_sk_destroy(s):
    return _check(lib().lb_sk_destroy(s))


def lb_pseudo_energy_state(p, state, t, stream):
    """{t, M, E_s, E_m, sum psi^2, E_bulk} of a dense [9][ny][nx] device
    population array, without a context or workspace (numpy float64[6])."""
    import numpy as np

    out = np.empty(6, np.float64)
    _check(lib().lb_pseudo_energy_state(ctypes.byref(p), _ptr(state), float(t), out.ctypes.data,
                                        stream or None))
    return out
