"""Structure factor and droplet length scale (test infrastructure only).

Plain numpy statement of the Fourier analysis of section IV (the equation
defining S(k, t), its circular average and the first moment, eq. (rad)):

    S(k) = (1/N) |sum_x (rho(x) - mean rho) exp(i k.x)|^2,
    k = (2 pi / L) (l, m),  N = L^2,
    S_n = mean of S(k) over the shell (n - 1/2) <= |k| L / (2 pi) < n + 1/2,
    kbar = sum_n n S_n / sum_n S_n   (k in units of 2 pi / L, n >= 0),
    R = L / (2 kbar)                 (the reading in which k = 1 gives R = L/2).

The transform is numpy's FFT (a library primitive standing for the sum
over x); everything else is written out.  Only the tests and the benchmark's
CPU baseline load this module.  Its pins (a single cosine mode in closed
form, Parseval's identity, a brute-force DFT, shell membership by
enumeration) are in tests/test_oracle_structure.py.
"""
import numpy as np


def spectrum(rho):
    """S(k) on the L x L grid of modes, indexed [m][l] like the field
    (m, l the FFT frequency indices of y and x)."""
    rho = np.asarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    if nx != ny:
        raise ValueError("the structure factor is defined for square lattices")
    d = rho - rho.mean()
    F = np.fft.fft2(d)
    return (F.real ** 2 + F.imag ** 2) / d.size


def shell_index(L):
    """Shell n of every mode: the integer with n - 1/2 <= sqrt(l^2 + m^2) < n + 1/2,
    l, m the signed frequencies of an L-point transform."""
    f = np.fft.fftfreq(L, d=1.0 / L)  # 0, 1, ..., -1 (integers as floats)
    l = f[None, :]
    m = f[:, None]
    return np.floor(np.sqrt(l * l + m * m) + 0.5).astype(np.int64)


def shells(rho):
    """(S_n, counts) for n = 0 .. max shell."""
    S = spectrum(rho)
    idx = shell_index(S.shape[0])
    sums = np.bincount(idx.ravel(), weights=S.ravel())
    counts = np.bincount(idx.ravel())
    return sums / np.maximum(counts, 1), counts


def kbar(Sn):
    n = np.arange(len(Sn), dtype=np.float64)
    return float((n * Sn).sum() / Sn.sum())


def radius(rho):
    """R = L / (2 kbar) of a density field."""
    Sn, _ = shells(rho)
    return rho.shape[0] / (2.0 * kbar(Sn))
