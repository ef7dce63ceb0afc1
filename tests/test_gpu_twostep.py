"""GPU: two plain steps per launch (temporal blocking, FP32 storage).

The two-step kernel applies to every site the same force and collision as
the one-step kernel, so its fields must be bit-identical to one step per
launch, for every tile shape, lattice size (small lattices whose tiles wrap
around them included) and chunking of the run; logging splits the pairs at
log points and records the same trace.
"""
import numpy as np
import pytest

import oracle as O
from paper_1008_2865_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1008_2865_amd.sim import LBSim  # noqa: E402

R01 = inputs.couplings(0.1)


def run(rho0, steps, spl, chunks=None, **kw):
    G1, G2 = R01
    sim = LBSim(rho0, G1=G1, G2=G2, storage="f32", max_steps=steps, steps_per_launch=spl, **kw)
    for n in (chunks or [steps]):
        sim.step(n)
    state, trace = sim.get_state(), sim.trace()
    sim.close()
    return state, trace


@pytest.mark.parametrize("nx,ny,tile_x,tile_y", [
    (300, 90, 256, 32),   # ragged in x (250-column output tiles) and y
    (256, 256, 256, 32),
    (100, 70, 64, 16),
    (130, 37, 128, 5),
    (5, 5, 64, 1),        # tiles wrap around the lattice several times
    (7, 9, 64, 3),
    (257, 11, 256, 4),
    (64, 64, 128, 64),
])
def test_two_steps_per_launch_bit_identical(nx, ny, tile_x, tile_y):
    print(f"two-step {nx}x{ny} tile {tile_x}x{tile_y}", flush=True)
    rho0 = inputs.rho_noise(nx, ny, 5)
    a, _ = run(rho0, 61, 1, tile_x=tile_x, tile_y=tile_y)
    b, _ = run(rho0, 61, 2, tile_x=tile_x, tile_y=tile_y)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_logging_and_chunks():
    rho0 = inputs.rho_noise(96, 80, 7)
    a, ta = run(rho0, 100, 1, log_every=7, tile_y=16)
    b, tb = run(rho0, 100, 2, log_every=7, chunks=[3, 50, 1, 46], tile_y=16)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert ta.shape == tb.shape and np.array_equal(ta, tb)


def test_full_size_against_oracle():
    # 2048^2, 256 x 32 tiles, 6 steps (3 two-step launches) against the oracle.
    G1, G2 = R01
    rho0 = inputs.rho_noise(2048, 2048, 1)
    fo = O.step(O.init(rho0), 6, 1.0, 1.0, G1, G2)
    a, _ = run(rho0, 6, 2)
    assert float(np.max(np.abs(a.astype(np.float64) - fo))) <= 2e-6
