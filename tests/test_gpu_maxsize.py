"""GPU: the largest lattice the library accepts, checked where the oracle can.

(nx + 192) ny must stay below 2^31 (in-plane offsets are 32-bit) and
ny <= 65535.  A 32768 x 65000 FP32 lattice sits just under the first limit:
its population planes hold 2.13e9 elements (8.5 GB each, 153 GB for both
buffers), so element offsets approach 2^31 and byte offsets reach 2^36.
The field is uniform except for a 16 x 16 noise patch straddling the
periodic corner; after 5 steps a disturbance has moved at most 15 sites
(one for streaming plus two for the psi stencil per step), so a 64 x 64
window around the corner must match the oracle run on a 64 x 64 periodic
lattice holding the same patch, and the total mass must be that of the
initial field.  The plain steps run in the library's default launch
configuration (two per launch at this size).
"""
import numpy as np
import pytest

import oracle as O
from paper_1008_2865_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1008_2865_amd import binding as B  # noqa: E402
from paper_1008_2865_amd.sim import LBSim  # noqa: E402

NX, NY, STEPS, W = 32768, 65000, 5, 64


def test_largest_lattice_window_against_oracle():
    assert (NX + 192) * NY < 2 ** 31 and NY <= 65535
    free, _ = torch.cuda.mem_get_info()
    need = 2 * 9 * (NX + 64) * NY * 4 + 4 * NX * NY * 8
    if free < need * 1.05:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} free")
    G1, G2 = inputs.couplings(0.1)
    patch = inputs.rho_noise(16, 16, 7)
    rows = np.arange(-W // 2, W // 2) % NY
    cols = np.arange(-W // 2, W // 2) % NX
    rho = np.full((NY, NX), 0.7)
    rho[np.ix_(rows[24:40], cols[24:40])] = patch
    mass0 = float(rho.sum())
    print(f"max size {NX}x{NY} f32, {STEPS} steps", flush=True)
    sim = LBSim(rho, G1=G1, G2=G2, storage="f32", max_steps=STEPS)
    del rho
    assert B.lb_two_step_shape(sim.p)[0] > 0
    sim.step(STEPS)
    dev = torch.empty((NY, NX), dtype=torch.float64, device="cuda")
    B.lb_moments(sim.ctx, dev, None, None, on_device=True)
    r = torch.as_tensor(rows, device="cuda")
    c = torch.as_tensor(cols, device="cuda")
    win = dev.index_select(0, r).index_select(1, c).cpu().numpy()
    del dev
    e = sim.pseudo_energy()
    sim.close()

    small = np.full((W, W), 0.7)
    small[24:40, 24:40] = patch
    fo = O.step(O.init(small), STEPS, 1.0, 1.0, G1, G2)
    assert float(np.max(np.abs(win - fo.sum(axis=0)))) <= 2e-6
    assert e[0] == STEPS and abs(e[1] - mass0) <= 1e-6 * mass0
