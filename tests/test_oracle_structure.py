"""The structure-factor oracle (oracle/structure.py) pinned to closed forms.

A single Fourier mode has a structure factor known in closed form; the sum
of S(k) over all modes equals the variance sum (Parseval); on small
lattices the transform is checked against the defining double sum written
out, and shell membership against an enumeration of the shell inequality
in integer arithmetic.
"""
import math

import numpy as np
import pytest

from oracle import structure as SK


def brute_spectrum(rho):
    L = rho.shape[0]
    d = rho - rho.mean()
    S = np.zeros((L, L))
    xs = np.arange(L)
    for m in range(L):
        for l in range(L):
            ph = np.exp(2j * np.pi * (l * xs[None, :] + m * xs[:, None]) / L)
            S[m, l] = abs((d * ph).sum()) ** 2 / L ** 2
    return S


@pytest.mark.parametrize("L", [6, 8, 9])
def test_spectrum_is_the_defining_sum(L):
    rho = 0.7 + 0.05 * np.random.default_rng(L).standard_normal((L, L))
    assert np.allclose(SK.spectrum(rho), brute_spectrum(rho), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("L,l0,m0", [(64, 3, 0), (64, 5, 7), (48, 2, 9), (512, 40, 17)])
def test_single_mode_closed_form(L, l0, m0):
    # rho = mean + a cos(2 pi (l0 x + m0 y) / L): the modes +-(l0, m0) carry
    # |a N / 2|^2 / N = a^2 N / 4 each, every other mode nothing.
    a = 0.03
    y, x = np.mgrid[0:L, 0:L]
    rho = 0.7 + a * np.cos(2 * np.pi * (l0 * x + m0 * y) / L)
    S = SK.spectrum(rho)
    N = L * L
    peak = a * a * N / 4
    assert S[m0 % L, l0 % L] == pytest.approx(peak, rel=1e-12)
    assert S[-m0 % L, -l0 % L] == pytest.approx(peak, rel=1e-12)
    mask = np.ones_like(S, dtype=bool)
    mask[m0 % L, l0 % L] = mask[-m0 % L, -l0 % L] = False
    assert np.max(S[mask]) < 1e-20 * N
    Sn, counts = SK.shells(rho)
    n0 = int(math.floor(math.hypot(l0, m0) + 0.5))
    assert Sn[n0] == pytest.approx(2 * peak / counts[n0], rel=1e-12)
    assert SK.kbar(Sn) == pytest.approx(n0, rel=1e-12)
    assert SK.radius(rho) == pytest.approx(L / (2 * n0), rel=1e-12)


def test_parseval_and_translation_invariance():
    L = 40
    rho = 0.7 + 0.1 * np.random.default_rng(3).random((L, L))
    S = SK.spectrum(rho)
    assert S.sum() == pytest.approx(((rho - rho.mean()) ** 2).sum(), rel=1e-12)
    assert S[0, 0] < 1e-25
    shifted = np.roll(rho, (7, -11), axis=(0, 1))
    assert np.allclose(SK.spectrum(shifted), S, rtol=1e-10, atol=1e-14)
    # A real field: S(k) = S(-k).
    assert np.allclose(S, np.roll(S[::-1, ::-1], (1, 1), axis=(0, 1)), rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("L", [8, 15, 64])
def test_shell_membership_by_enumeration(L):
    idx = SK.shell_index(L)
    for m in range(L):
        for l in range(L):
            ls = l if l < (L + 1) // 2 else l - L   # fftfreq's signed index
            ms = m if m < (L + 1) // 2 else m - L
            q = ls * ls + ms * ms
            n = idx[m, l]
            # (n - 1/2)^2 <= q < (n + 1/2)^2 in integers: (2n-1)^2 <= 4q < (2n+1)^2.
            assert (n == 0 and q == 0) or ((2 * n - 1) ** 2 <= 4 * q < (2 * n + 1) ** 2)
    counts = np.bincount(idx.ravel())
    assert counts.sum() == L * L and counts[0] == 1
    if L >= 8:
        assert counts[1] == 8 and counts[2] == 12   # r = 1, sqrt 2; r = 2, sqrt 5
