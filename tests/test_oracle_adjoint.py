"""The reference gradients (oracle/adjoint.py) pinned to the C oracle and to
finite differences.

Its forward pass must reproduce the C oracle (itself pinned to the paper in
test_oracle_pins.py) and its energy the C oracle's section V observables;
its autograd gradients must match central finite differences of its own
loss, in double precision, on a horizon short enough for the loss to be
smooth at the step size.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import adjoint as A
from paper_1008_2865_amd import inputs


def test_forward_matches_c_oracle():
    G1, G2 = inputs.couplings(0.1)
    rho0 = inputs.rho_noise(16, 12, 3)
    w = torch.tensor(O.d2q9()[2])[:, None, None]
    f = w * torch.tensor(rho0)
    for _ in range(40):
        f = A.step(f, G1, G2, 0.9)
    fo = O.step(O.init(rho0), 40, 0.9, 1.0, G1, G2)
    assert np.max(np.abs(f.numpy() - fo)) < 1e-13
    E = float(A.energy(f, G1, G2))
    obs = O.observables(fo, 1.0, G1, G2)
    assert abs(E - (obs[1] + obs[2])) < 1e-12 * abs(E)


@pytest.mark.parametrize("tau,r", [(1.0, 0.1), (0.8, 0.05)])
def test_gradients_match_finite_differences(tau, r):
    G1, G2 = inputs.couplings(r)
    rho0 = inputs.rho_noise(12, 10, 5)
    steps, beta, eps = 30, 1.0 / 144, 1e-6
    E0 = float(A.loss(torch.tensor(rho0), G1, G2, steps, tau, 0.0, 0.0, eps)[2])
    Et = 1.01 * E0
    L, dG1, dG2, drho, _, _ = A.loss_and_grads(rho0, G1, G2, steps, tau, Et, beta, eps)

    def Lof(r_, g1, g2):
        return float(A.loss(torch.tensor(r_), g1, g2, steps, tau, Et, beta, eps)[0])

    h = 1e-6
    fd1 = (Lof(rho0, G1 + h, G2) - Lof(rho0, G1 - h, G2)) / (2 * h)
    fd2 = (Lof(rho0, G1, G2 + h) - Lof(rho0, G1, G2 - h)) / (2 * h)
    assert abs(fd1 - dG1) <= 1e-5 * abs(dG1) + 1e-9
    assert abs(fd2 - dG2) <= 1e-5 * abs(dG2) + 1e-9
    v = np.random.default_rng(1).standard_normal(rho0.shape)
    fdv = (Lof(rho0 + h * v, G1, G2) - Lof(rho0 - h * v, G1, G2)) / (2 * h)
    assert abs(fdv - float((drho * v).sum())) <= 1e-5 * abs(fdv)
    # The initial-density gradient is w-weighted: with populations w_i rho
    # it equals sum_i w_i dL/df_i(0); check one component by a one-hot FD.
    e = np.zeros_like(rho0)
    e[4, 7] = 1.0
    fde = (Lof(rho0 + h * e, G1, G2) - Lof(rho0 - h * e, G1, G2)) / (2 * h)
    assert abs(fde - drho[4, 7]) <= 1e-5 * abs(fde) + 1e-9


@pytest.mark.parametrize("l,m", [(1, 0), (3, 2), (0, 4)])
def test_interface_area_closed_form(l, m):
    # Central differences are exact on a cosine.  For
    # rho = a + b cos(kx x) + c cos(ky y), kx = 2 pi l / nx, ky = 2 pi m / ny:
    # D_x rho = -b sin(kx) sin(kx x), D_y rho = -c sin(ky) sin(ky y), so
    # A = sum_x sqrt(b^2 sin^2(kx) sin^2(kx x) + c^2 sin^2(ky) sin^2(ky y) + eps^2).
    # A one-sided difference or a dropped factor 1/2 fails this.
    nx, ny, a, b, c, eps = 24, 20, 0.7, 0.3, 0.2, 1e-3
    kx, ky = 2 * np.pi * l / nx, 2 * np.pi * m / ny
    y, x = np.mgrid[0:ny, 0:nx]
    rho = a + b * np.cos(kx * x) + c * np.cos(ky * y)
    dx = b * np.sin(kx) * np.sin(kx * x)
    dy = c * np.sin(ky) * np.sin(ky * y)
    A_ref = np.sqrt(dx * dx + dy * dy + eps * eps).sum()
    f = torch.zeros((9, ny, nx), dtype=torch.float64)
    f[0] = torch.tensor(rho)          # the measure reads the density only
    area = float(A.interface_area(f, eps))
    assert abs(area - A_ref) <= 1e-13 * A_ref


def test_interface_area_of_a_uniform_field():
    nx, ny, eps = 12, 9, 1e-6
    f = torch.zeros((9, ny, nx), dtype=torch.float64)
    f[:] = 0.7 / 9
    assert abs(float(A.interface_area(f, eps)) - nx * ny * eps) <= 1e-12 * nx * ny * eps
