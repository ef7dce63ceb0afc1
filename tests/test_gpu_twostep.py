"""GPU: two plain steps per launch (temporal blocking, FP32 and half storage).

The two-step kernel applies to every site the same force and collision as
the one-step kernel, so its fields must be bit-identical to one step per
launch, for every tile shape, lattice size (small lattices whose tiles wrap
around them included) and chunking of the run; logging splits the pairs at
log points and records the same trace.  In half storage the first step's
populations pass through LDS rounded exactly as they would be stored (the
rest population stochastically, from the same site hash), so the half
fields are bit-identical too.
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


def run(rho0, steps, spl, chunks=None, storage="f32", **kw):
    G1, G2 = R01
    sim = LBSim(rho0, G1=G1, G2=G2, storage=storage, max_steps=steps, steps_per_launch=spl, **kw)
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
    (600, 300, 256, 119),  # the tall tiles of large half-storage lattices, ragged
])
@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_two_steps_per_launch_bit_identical(nx, ny, tile_x, tile_y, storage):
    print(f"two-step {storage} {nx}x{ny} tile {tile_x}x{tile_y}", flush=True)
    rho0 = inputs.rho_noise(nx, ny, 5)
    a, _ = run(rho0, 61, 1, storage=storage, tile_x=tile_x, tile_y=tile_y)
    b, _ = run(rho0, 61, 2, storage=storage, tile_x=tile_x, tile_y=tile_y)
    bits = np.uint32 if storage == "f32" else np.uint16
    assert np.array_equal(a.view(bits), b.view(bits))


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_two_steps_per_launch_bit_identical_other_tau(storage, tau):
    # The relaxation f + (f_eq - f) / tau with tau != 1 (the paper's runs
    # use tau = 1, which takes the collision's other path).
    rho0 = inputs.rho_noise(150, 60, 8)
    a, _ = run(rho0, 41, 1, storage=storage, tau=tau, tile_x=128, tile_y=16)
    b, _ = run(rho0, 41, 2, storage=storage, tau=tau, tile_x=128, tile_y=16)
    bits = np.uint32 if storage == "f32" else np.uint16
    assert np.array_equal(a.view(bits), b.view(bits))


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_logging_and_chunks(storage):
    rho0 = inputs.rho_noise(96, 80, 7)
    a, ta = run(rho0, 100, 1, storage=storage, log_every=7, tile_y=16)
    b, tb = run(rho0, 100, 2, storage=storage, log_every=7, chunks=[3, 50, 1, 46], tile_y=16)
    bits = np.uint32 if storage == "f32" else np.uint16
    assert np.array_equal(a.view(bits), b.view(bits))
    assert ta.shape == tb.shape and np.array_equal(ta, tb)


def test_full_size_against_oracle():
    # 2048^2, 256 x 32 tiles, 6 steps (3 two-step launches) against the oracle.
    G1, G2 = R01
    rho0 = inputs.rho_noise(2048, 2048, 1)
    fo = O.step(O.init(rho0), 6, 1.0, 1.0, G1, G2)
    a, _ = run(rho0, 6, 2)
    assert float(np.max(np.abs(a.astype(np.float64) - fo))) <= 2e-6


def test_half_storage_decodes_identically_everywhere():
    # 512^2 x 61 steps: about 16M site updates, in which a single decode of a
    # stored half that rounded differently in one code path (the first rows
    # of a tile against the rows of the walk, one step per launch against
    # the LDS ring of two) would almost surely flip at least one
    # stochastically rounded rest population.
    rho0 = inputs.rho_noise(512, 512, 11)
    ref, _ = run(rho0, 61, 1, storage="f16dev", tile_x=256, tile_y=32)
    for spl, tx, ty, tr in [(1, 64, 7, 2), (1, 128, 1, 1), (2, 128, 24, 0), (2, 64, 5, 0)]:
        print(f"f16dev 512^2 steps/launch {spl} tile {tx}x{ty}x{tr}", flush=True)
        kw = dict(tile_x=tx, tile_y=ty) | ({"tile_rows": tr} if tr else {})
        s, _ = run(rho0, 61, spl, storage="f16dev", **kw)
        assert np.array_equal(s.view(np.uint16), ref.view(np.uint16))


def test_two_step_residency_matches_the_occupancy_query():
    # The two-step shape rule sizes tiles by the workgroups resident at once.
    # On the device it asks the runtime's occupancy query; without one it
    # uses the value for the kernel as built (6 workgroups of 128 lanes per
    # CU on 256 CUs).  Both must agree, or the CPU-side value is stale.
    from paper_1008_2865_amd import binding as B

    p = B.make_params(2048, 2048, storage=B.LB_F32, G1=-5.4, G2=0.54)
    assert B.lb_two_step_shape(p) == (128, 23, 1530)
    p = B.make_params(3000, 3000, storage=B.LB_F32, G1=-5.4, G2=0.54)
    assert B.lb_two_step_shape(p)[:2] == (256, 47)
    # The half storage's kernel has the same occupancy (three waves per SIMD).
    p = B.make_params(2048, 2048, storage=B.LB_F16DEV, G1=-5.4, G2=0.54, rho_ref=0.7)
    assert B.lb_two_step_shape(p) == (128, 23, 1530)
    p = B.make_params(8192, 8192, storage=B.LB_F16DEV, G1=-5.4, G2=0.54, rho_ref=0.7)
    assert B.lb_two_step_shape(p) == (256, 119, 2277)
