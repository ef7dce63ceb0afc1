"""LBSim: a two-belt Shan-Chen lattice on one GPU, driven through liblb.so.

PyTorch provides the device memory (the workspace and device-side outputs)
and the stream; every computation is a kernel of the HIP library.
"""
import numpy as np

from . import binding as B

STORAGE = {"f64": B.LB_F64, "f32": B.LB_F32, "f16dev": B.LB_F16DEV}


class LBSim:
    """A periodic nx-by-ny lattice started from rho_init (fluid at rest
    unless ux_init / uy_init are given).

    ``rho_init`` may be a numpy array (host) or a float64 CUDA tensor of
    shape (ny, nx).  All work runs on ``torch.cuda.current_stream()`` of
    the device current at construction.
    """

    def __init__(self, rho_init, *, G1, G2, tau=1.0, rho0=1.0, storage="f32",
                 log_every=0, trace_cap=None, tile_x=0, tile_y=0, tile_rows=0, rho_ref=None,
                 ux_init=None, uy_init=None, max_steps=None, steps_per_launch=0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("LBSim needs a HIP device (torch.cuda.is_available() is False)")
        self.torch = torch
        on_dev = isinstance(rho_init, torch.Tensor) and rho_init.is_cuda
        if on_dev:
            ny, nx = rho_init.shape
            rho_d = rho_init.to(torch.float64).contiguous()
            mean = float(rho_d.mean())
            ins = [rho_d] + [None if u is None else u.to(torch.float64).contiguous()
                             for u in (ux_init, uy_init)]
        else:
            rho_h = np.ascontiguousarray(rho_init, dtype=np.float64)
            ny, nx = rho_h.shape
            mean = float(rho_h.mean())
            ins = [rho_h] + [None if u is None else np.ascontiguousarray(u, dtype=np.float64)
                             for u in (ux_init, uy_init)]
        if trace_cap is None:
            trace_cap = (max_steps // log_every + 2) if (log_every and max_steps) else (
                1024 if log_every else 0)
        st = STORAGE[storage]
        self.p = B.make_params(nx, ny, storage=st, tau=tau, rho0=rho0, G1=G1, G2=G2,
                               log_every=log_every, trace_cap=trace_cap, tile_x=tile_x,
                               tile_y=tile_y, tile_rows=tile_rows, steps_per_launch=steps_per_launch,
                               rho_ref=(mean if rho_ref is None else rho_ref) if st == B.LB_F16DEV else 0.0)
        nbytes = B.lb_workspace_bytes(self.p)
        if nbytes == 0:
            B._check(B.lb_validate(self.p))
        self.nx, self.ny, self.storage = nx, ny, storage
        self.device = torch.cuda.current_device()
        self.stream = torch.cuda.current_stream()
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.ctx = B.lb_init(self.p, self.workspace, nbytes, *ins,
                             inputs_on_device=on_dev, stream=self.stream.cuda_stream)
        self.trace_cap = trace_cap

    # -- time stepping --------------------------------------------------
    def step(self, n=1):
        B.lb_step(self.ctx, n)

    @property
    def t(self):
        return B.lb_time(self.ctx)

    def launch_shape(self):
        return B.lb_launch_shape(self.p)

    # -- observables ----------------------------------------------------
    def moments(self, device=False):
        """(rho, ux, uy) of the state at t: numpy arrays, or CUDA tensors."""
        if device:
            t = self.torch
            out = [t.empty((self.ny, self.nx), dtype=t.float64, device="cuda") for _ in range(3)]
            B.lb_moments(self.ctx, *out, on_device=True)
            return tuple(out)
        out = [np.empty((self.ny, self.nx), np.float64) for _ in range(3)]
        B.lb_moments(self.ctx, *out, on_device=False)
        return tuple(out)

    def pseudo_energy(self):
        """{t, M, E_s, E_m, sum psi^2, E_bulk} of the state at t."""
        out = np.empty(6, np.float64)
        B.lb_pseudo_energy(self.ctx, out)
        return out

    def structure_factor(self, spectrum=False):
        """(S_n, counts, kbar, R) of the density at t (square lattices; see
        structure.StructureFactor)."""
        if getattr(self, "_sk", None) is None:
            from .structure import StructureFactor

            if self.nx != self.ny:
                raise ValueError("the structure factor is defined for square lattices")
            self._sk = StructureFactor(self.nx, stream=self.stream)
        rho = self.moments(device=True)[0]
        return self._sk(rho, spectrum=spectrum)

    def trace(self):
        out = np.empty((max(self.trace_cap, 1), 6), np.float64)
        n = B.lb_trace(self.ctx, out, self.trace_cap)
        return out[:n].copy()

    # -- checkpoint -----------------------------------------------------
    def state_dtype(self):
        return {"f64": np.float64, "f32": np.float32, "f16dev": np.float16}[self.storage]

    def get_state(self):
        out = np.empty((9, self.ny, self.nx), self.state_dtype())
        B.lb_get_state(self.ctx, out, on_device=False)
        return out

    def set_state(self, f, t):
        f = np.ascontiguousarray(f, dtype=self.state_dtype())
        assert f.shape == (9, self.ny, self.nx)
        B.lb_set_state(self.ctx, f, t, on_device=False)

    def close(self):
        if getattr(self, "_sk", None) is not None:
            self._sk.close()
            self._sk = None
        if getattr(self, "ctx", None):
            B.lb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Member(LBSim):
    """A lattice owned by an LBBatch: observables and state export only."""

    def __init__(self, batch, i, nx, ny, storage, trace_cap):
        self.torch = batch.torch
        self.ctx = B.lb_batch_member(batch.b, i)
        self.nx, self.ny, self.storage, self.trace_cap = nx, ny, storage, trace_cap
        self._batch = batch

    def step(self, n=1):
        raise RuntimeError("step the whole batch with LBBatch.step")

    def close(self):
        self.ctx = None


class LBBatch:
    """Many independent periodic lattices advanced by one launch per step.

    ``lattices`` is a list of dicts with keys rho_init (ny, nx) and G1, G2
    (optionally tau, rho0, tile_y, rho_ref).  Shared settings (storage,
    tile_x, tile_rows, log_every, trace_cap, steps_per_launch) are keyword
    arguments.  Plain steps are captured into HIP graphs when the current
    torch stream is not the null stream (not for half storage).
    """

    def __init__(self, lattices, *, storage="f32", tile_x=0, tile_rows=0, log_every=0,
                 trace_cap=None, max_steps=None, use_graphs=True, steps_per_launch=0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("LBBatch needs a HIP device")
        self.torch = torch
        if trace_cap is None:
            trace_cap = (max_steps // log_every + 2) if (log_every and max_steps) else (
                1024 if log_every else 0)
        st = STORAGE[storage]
        self.params, rhos, self.shapes = [], [], []
        for L in lattices:
            rho = np.ascontiguousarray(L["rho_init"], dtype=np.float64)
            ny, nx = rho.shape
            self.params.append(B.make_params(
                nx, ny, storage=st, tau=L.get("tau", 1.0), rho0=L.get("rho0", 1.0),
                G1=L["G1"], G2=L["G2"], log_every=log_every, trace_cap=trace_cap,
                tile_x=tile_x, tile_y=L.get("tile_y", 0), tile_rows=tile_rows,
                rho_ref=L.get("rho_ref", float(rho.mean())) if st == B.LB_F16DEV else 0.0,
                steps_per_launch=steps_per_launch))
            rhos.append(rho)
            self.shapes.append((ny, nx))
        nbytes = B.lb_batch_workspace_bytes(self.params)
        if nbytes == 0:
            for p in self.params:
                B._check(B.lb_validate(p))
            raise B.LBError(B.LB_ERR_INVALID, B.lb_last_error())
        self.stream = torch.cuda.current_stream()
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.b = B.lb_batch_init(self.params, self.workspace, nbytes, rhos,
                                 stream=self.stream.cuda_stream)
        if not use_graphs or self.stream.cuda_stream == 0:
            if self.stream.cuda_stream != 0 and st != B.LB_F16DEV:
                B.lb_batch_use_graphs(self.b, False)
        self.members = [_Member(self, i, nx, ny, storage, trace_cap)
                        for i, (ny, nx) in enumerate(self.shapes)]
        self.sites = sum(nx * ny for ny, nx in self.shapes)
        self.storage = storage

    def step(self, n=1):
        B.lb_batch_step(self.b, n)

    def two_step_shape(self):
        """(tile_x, tile_y, workgroups) of the two-step launches, zeros if unused."""
        return B.lb_batch_two_step_shape(self.b)

    def set_two_step_tile(self, tile_y):
        """Rows per workgroup of the two-step launches (0: the library's choice)."""
        B.lb_batch_two_step_tile(self.b, tile_y)

    def __getitem__(self, i):
        return self.members[i]

    def __len__(self):
        return len(self.members)

    def close(self):
        if getattr(self, "b", None):
            for m in self.members:
                m.close()
            B.lb_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
