"""Gradients of a droplet functional through the HIP adjoint (liblb.so).

``DropletLoss`` evaluates, for a run of T steps from a fluid at rest with
density rho_init and couplings (G1, G2),
    L = (E(T) - E_target)^2 + beta * A(T),
E = E_s + E_m (section V), A = sum_x sqrt(D_x rho^2 + D_y rho^2 + eps^2)
(central differences: an interface-length measure), and its gradients with
respect to G1, G2 and rho_init, by the reverse-mode kernels of the library
(lb_adj_forward / lb_adj_backward).  ``DropletLoss.__call__`` wraps the
pair in a ``torch.autograd.Function``.
"""
import numpy as np

from . import binding as B
from .sim import STORAGE


class DropletLoss:
    def __init__(self, nx, ny, steps, *, E_target, beta, eps=1e-6, tau=1.0, rho0=1.0,
                 storage="f32", checkpoint_every=100, tile_x=0, tile_y=0, tile_rows=0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("DropletLoss needs a HIP device (torch.cuda.is_available() is False)")
        self.torch = torch
        self.nx, self.ny, self.steps = nx, ny, steps
        self.E_target, self.beta, self.eps = float(E_target), float(beta), float(eps)
        self.p = B.make_params(nx, ny, storage=STORAGE[storage], tau=tau, rho0=rho0,
                               tile_x=tile_x, tile_y=tile_y, tile_rows=tile_rows)
        nbytes = B.lb_adj_workspace_bytes(self.p, steps, checkpoint_every)
        if nbytes == 0:
            B._check(B.lb_validate(self.p))
            raise B.LBError(B.LB_ERR_INVALID, "invalid adjoint configuration: " + B.lb_last_error())
        self.stream = torch.cuda.current_stream()
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.ctx = B.lb_adj_init(self.p, steps, checkpoint_every, self.workspace, nbytes,
                                 stream=self.stream.cuda_stream)
        self.generation = 0

    def forward(self, rho_init, G1, G2):
        """(L, E(T), A(T), M(T)); rho_init is a (ny, nx) array or CUDA tensor."""
        torch = self.torch
        if isinstance(rho_init, torch.Tensor) and rho_init.is_cuda:
            r = rho_init.detach().to(torch.float64).contiguous()
            on_dev = True
        else:
            r = np.ascontiguousarray(rho_init, dtype=np.float64)
            on_dev = False
        if tuple(r.shape) != (self.ny, self.nx):
            raise ValueError(f"rho_init has shape {tuple(r.shape)}, expected {(self.ny, self.nx)}")
        out = B.lb_adj_forward(self.ctx, r, float(G1), float(G2), self.E_target, self.beta,
                               self.eps, on_device=on_dev)
        self.generation += 1
        return out

    def backward(self):
        """(dL/dG1, dL/dG2, dL/drho_init as a float64 CUDA tensor)."""
        drho = self.torch.empty((self.ny, self.nx), dtype=self.torch.float64, device="cuda")
        dG1, dG2 = B.lb_adj_backward(self.ctx, drho, on_device=True)
        return dG1, dG2, drho

    def __call__(self, rho_init, G):
        """L as a 0-d float64 tensor, differentiable in rho_init (ny, nx) and
        G = (G1, G2)."""
        return _LossFunction.apply(rho_init, G, self)

    def close(self):
        if self.ctx is not None:
            B.lb_adj_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _function_class():
    import torch

    class LossFunction(torch.autograd.Function):
        @staticmethod
        def forward(ctx, rho_init, G, runner):
            L = runner.forward(rho_init, float(G[0]), float(G[1]))[0]
            ctx.runner, ctx.generation = runner, runner.generation
            ctx.G_device = G.device
            return torch.tensor(L, dtype=torch.float64, device=rho_init.device)

        @staticmethod
        def backward(ctx, gL):
            runner = ctx.runner
            if runner.generation != ctx.generation:
                raise RuntimeError("DropletLoss was evaluated again before this backward: "
                                   "one backward per forward")
            dG1, dG2, drho = runner.backward()
            gL = gL.to(torch.float64)
            dG = torch.tensor([dG1, dG2], dtype=torch.float64, device=ctx.G_device)
            return gL.to(drho.device) * drho, gL.to(ctx.G_device) * dG, None

    return LossFunction


class _Lazy:
    cls = None

    def apply(self, *args):
        if _Lazy.cls is None:
            _Lazy.cls = _function_class()
        return _Lazy.cls.apply(*args)


_LossFunction = _Lazy()
