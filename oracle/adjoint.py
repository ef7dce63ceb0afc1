"""Reference gradients of a droplet functional (test infrastructure only).

A plain double-precision PyTorch (CPU) re-statement of the time step that
the C oracle implements (section II equilibrium and moments, eq. (FORCE)
with the section II sign, velocity-shift BGK collision, streaming of
eq. (1)), differentiated by autograd.  Only the tests load it.  Its forward
pass is checked against the C oracle step for step, and its gradients
against central finite differences, in tests/test_oracle_adjoint.py.

The functional of a state at time T (the loss of the adjoint workload):
    L = (E(T) - E_target)^2 + beta * A(T),
    E = E_s + E_m (section V energies, rest link included as in the C
        oracle),
    A = sum_x sqrt(D_x rho^2 + D_y rho^2 + eps^2), D central differences
        (an interface-length measure: |grad rho| is large only on
        interfaces).
Gradients are taken with respect to G1, G2 and the initial density
(populations start at rest equilibrium w_i rho_init).
"""
import math

import numpy as np
import torch

from . import d2q9, tables

_CX, _CY, _W = d2q9()
_LX, _LY, _KW, _KEW = tables(1.0, 0.0)  # unit G1: first-belt D2Q9 weights
_, _, _KP, _KEP = tables(0.0, 1.0)      # unit G2: Table 1 weights, rest p_s0


def _roll_to(psi, cx, cy):
    """psi(x + c) on the periodic lattice (array indexed [y, x])."""
    return torch.roll(psi, shifts=(-int(cy), -int(cx)), dims=(0, 1))


def step(f, G1, G2, tau, rho0=1.0):
    rho = f.sum(0)
    cx = torch.tensor(_CX, dtype=f.dtype)[:, None, None]
    cy = torch.tensor(_CY, dtype=f.dtype)[:, None, None]
    w = torch.tensor(_W, dtype=f.dtype)[:, None, None]
    jx = (cx * f).sum(0)
    jy = (cy * f).sum(0)
    psi = math.sqrt(rho0) * (1.0 - torch.exp(-rho / rho0))
    sx = torch.zeros_like(rho)
    sy = torch.zeros_like(rho)
    for k in range(24):
        Kk = G1 * float(_KW[k]) + G2 * float(_KP[k])
        nb = _roll_to(psi, _LX[k], _LY[k])
        sx = sx + Kk * float(_LX[k]) * nb
        sy = sy + Kk * float(_LY[k]) * nb
    Fx = -psi * sx
    Fy = -psi * sy
    ux = (jx + tau * Fx) / rho
    uy = (jy + tau * Fy) / rho
    cu = cx * ux + cy * uy
    uu = ux * ux + uy * uy
    feq = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
    fpost = f - (f - feq) / tau
    return torch.stack([torch.roll(fpost[i], shifts=(int(_CY[i]), int(_CX[i])), dims=(0, 1))
                        for i in range(9)])


def energy(f, G1, G2, rho0=1.0):
    """E_s + E_m of the pre-collision state f."""
    rho = f.sum(0)
    psi = math.sqrt(rho0) * (1.0 - torch.exp(-rho / rho0))
    acc = (G1 * float(_KEW[0]) + G2 * float(_KEP[0])) * psi
    for k in range(24):
        acc = acc + (G1 * float(_KEW[1 + k]) + G2 * float(_KEP[1 + k])) * _roll_to(psi, _LX[k], _LY[k])
    return 0.5 * (psi * acc).sum()


def interface_area(f, eps):
    rho = f.sum(0)
    dx = 0.5 * (torch.roll(rho, -1, dims=1) - torch.roll(rho, 1, dims=1))
    dy = 0.5 * (torch.roll(rho, -1, dims=0) - torch.roll(rho, 1, dims=0))
    return torch.sqrt(dx * dx + dy * dy + eps * eps).sum()


def loss(rho_init, G1, G2, steps, tau, E_target, beta, eps, rho0=1.0):
    w = torch.tensor(_W, dtype=rho_init.dtype)[:, None, None]
    f = w * rho_init
    for _ in range(steps):
        f = step(f, G1, G2, tau, rho0)
    E = energy(f, G1, G2, rho0)
    return (E - E_target) ** 2 + beta * interface_area(f, eps), f, E


def loss_and_grads(rho_init, G1, G2, steps, tau, E_target, beta, eps, rho0=1.0):
    """(L, dL/dG1, dL/dG2, dL/drho_init, E(T), f(T)) in double precision."""
    r = torch.tensor(np.asarray(rho_init, dtype=np.float64), requires_grad=True)
    g1 = torch.tensor(float(G1), dtype=torch.float64, requires_grad=True)
    g2 = torch.tensor(float(G2), dtype=torch.float64, requires_grad=True)
    L, f, E = loss(r, g1, g2, steps, tau, E_target, beta, eps, rho0)
    L.backward()
    return (float(L.detach()), float(g1.grad), float(g2.grad), r.grad.numpy().copy(), float(E.detach()),
            f.detach().numpy())
