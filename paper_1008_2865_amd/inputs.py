"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: it only draws the initial
density fields and the coupling constants of the workloads.

Initial state (section IV): a periodic fluid at rest with density
rho0 ln 2 + delta rho, delta rho / rho ~ 0.01, white noise.  The workloads use
rho = 0.7 (1 + 0.01 U(-1, 1)) drawn in double precision with numpy's PCG64
generator seeded per run.

Couplings: the paper scans G1, G2 at fixed A1 = G1 + G2 = -4.9 (section IV).
A workload labelled by the ratio r = G2 / |G1| therefore uses
G1 = A1 / (1 - r), G2 = r |G1|.
"""
import numpy as np

A1_PAPER = -4.9


def rho_noise(nx, ny, seed, mean=0.7, amp=0.01):
    """rho = mean * (1 + amp * U(-1, 1)), shape (ny, nx), float64."""
    rng = np.random.default_rng(seed)
    return mean * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(ny, nx)))


def couplings(r, A1=A1_PAPER):
    """(G1, G2) with G1 + G2 = A1 and G2 = r |G1|."""
    G1 = A1 / (1.0 - r)
    return G1, r * abs(G1)


def batched_lattices(count=96, seed=4, sizes=(128, 192, 256, 384, 512, 768, 1024),
                     r_max=0.15):
    """The batched sweep: `count` square lattices with sizes drawn uniformly
    from `sizes`, each with its own r ~ U[0, r_max] and its own noise seed.
    Returns a list of dicts {n, r, seed}."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.asarray(sizes), size=count)
    r = rng.uniform(0.0, r_max, size=count)
    seeds = rng.integers(1, 2**31 - 1, size=count)
    return [dict(n=int(a), r=float(b), seed=int(c)) for a, b, c in zip(n, r, seeds)]
