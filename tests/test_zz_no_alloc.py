"""GPU: lb_pseudo_energy_state, the entry point that allocates nothing.

It computes the section V observables of a dense population array with its
intermediate sums in the library's static device scratch.  Its output must
equal lb_pseudo_energy of a context holding the same state (the same site
values summed in another fixed order: double-precision sums of at most a
few 10^7 terms, within 1e-12 relative), on consecutive calls whose sizes
shrink (the scratch keeps the previous call's partials, which the smaller
call must not pick up).
"""
import numpy as np
import pytest

from paper_1008_2865_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1008_2865_amd import binding as B  # noqa: E402
from paper_1008_2865_amd.sim import LBSim  # noqa: E402

DT = {"f64": torch.float64, "f32": torch.float32, "f16dev": torch.float16}


def state_and_energy(n_x, n_y, storage, steps, seed):
    G1, G2 = inputs.couplings(0.1)
    sim = LBSim(inputs.rho_noise(n_x, n_y, seed), G1=G1, G2=G2, storage=storage)
    sim.step(steps)
    state = torch.empty((9, n_y, n_x), dtype=DT[storage], device="cuda")
    B.lb_get_state(sim.ctx, state, on_device=True)
    ref = sim.pseudo_energy()
    p = sim.p
    sim.close()
    return p, state, ref


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
def test_matches_lb_pseudo_energy_on_shrinking_calls(storage):
    stream = torch.cuda.current_stream().cuda_stream
    # Large first (more tiles than the 1024 workgroups: the grid-stride
    # path), then a ragged lattice smaller than one round of workgroups.
    for (nx, ny, steps, seed) in ((1030, 517, 40, 1), (70, 37, 25, 2)):
        print(f"no-alloc energy {storage} {nx}x{ny}", flush=True)
        p, state, ref = state_and_energy(nx, ny, storage, steps, seed)
        out = B.lb_pseudo_energy_state(p, state, float(steps), stream)
        assert out[0] == steps
        assert np.all(np.abs(out[1:] - ref[1:]) <= 1e-12 * np.abs(ref[1:])), (out, ref)


def test_rejects_bad_arguments():
    p = B.make_params(4, 16, storage=B.LB_F32, G1=-5.0, G2=0.5)
    x = torch.zeros(9 * 16 * 4, dtype=torch.float32, device="cuda")
    with pytest.raises(B.LBError) as e:
        B.lb_pseudo_energy_state(p, x, 0.0, 0)
    assert e.value.code == B.LB_ERR_INVALID
    p = B.make_params(8, 8, storage=B.LB_F32, G1=-5.0, G2=0.5)
    with pytest.raises(B.LBError) as e:
        B.lb_pseudo_energy_state(p, None, 0.0, 0)
    assert e.value.code == B.LB_ERR_INVALID
