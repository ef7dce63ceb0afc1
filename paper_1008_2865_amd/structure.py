"""Structure factor and droplet length scale through liblb.so (lb_sk_*).

``StructureFactor(L)`` evaluates, for a density field on an L x L periodic
lattice, the circularly averaged structure factor S_n, its first moment
kbar (eq. (rad), k in units of 2 pi / L) and the length scale
R = L / (2 kbar) of the section IV Fourier analysis.  Every pass runs in
the HIP library; this class only owns the workspace.
"""
import numpy as np

from . import binding as B


class StructureFactor:
    def __init__(self, L, stream=None):
        """stream: the torch CUDA stream to issue on (default: the current
        stream); inputs must be ready on it."""
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("StructureFactor needs a HIP device (torch.cuda.is_available() is False)")
        self.torch = torch
        self.L = L
        nbytes = B.lb_sk_workspace_bytes(L)
        if nbytes == 0:
            raise B.LBError(B.LB_ERR_INVALID, f"no structure factor for L = {L} (5 <= L <= 2048)")
        self.nshell = B.lb_sk_shells(L)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.ctx = B.lb_sk_init(L, self.workspace, nbytes, stream=self.stream.cuda_stream)

    def __call__(self, rho, spectrum=False):
        """(S_n, counts, kbar, R) of rho ((L, L) numpy array or float64 CUDA
        tensor); with spectrum=True also the full S(k) as an (L, L) CUDA
        tensor indexed [m][l]."""
        torch = self.torch
        on_dev = isinstance(rho, torch.Tensor) and rho.is_cuda
        r = rho.to(torch.float64).contiguous() if on_dev else np.ascontiguousarray(rho, np.float64)
        if tuple(r.shape) != (self.L, self.L):
            raise ValueError(f"rho has shape {tuple(r.shape)}, expected {(self.L, self.L)}")
        shell = np.empty(self.nshell, np.float64)
        counts = np.empty(self.nshell, np.int64)
        spec = torch.empty((self.L, self.L), dtype=torch.float64, device="cuda") if spectrum else None
        kbar = B.lb_sk_compute(self.ctx, r, shell, counts, spectrum=spec, on_device=on_dev)
        out = (shell, counts, kbar, self.L / (2.0 * kbar))
        return out + (spec,) if spectrum else out

    def close(self):
        if getattr(self, "ctx", None):
            B.lb_sk_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
