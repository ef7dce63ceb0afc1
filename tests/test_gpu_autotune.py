"""GPU: the launch-shape autotuner run for real on small cases.  Each tuner
times its candidates on the device, returns the fastest, caches it, and the
shape it returns runs and gives the same fields as the library's default."""
import json

import numpy as np
import pytest

from paper_1008_2865_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1008_2865_amd import autotune as A  # noqa: E402
from paper_1008_2865_amd.sim import LBBatch, LBSim  # noqa: E402


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "tiles.json"
    monkeypatch.setenv("LB_TUNE_CACHE", str(path))
    return path


def test_two_step_tuner_on_the_device(cache):
    n = 384
    print(f"tuning two-step shapes at {n}^2", flush=True)
    cands = [(128, 8), (128, 16), (256, 24)]
    tx, ty, tr = A.tune(n, n, "f32", candidates=cands, steps=10, steps_per_launch=2)
    assert (tx, ty) in cands and tr == 1
    entry = json.loads(cache.read_text())[f"f32:{n}x{n}:two-step"]
    assert (entry["tile_x"], entry["tile_y"]) == (tx, ty) and entry["us_per_step"] > 0
    # The tuned shape advances the lattice exactly as the default shape.
    G1, G2 = inputs.couplings(0.1)
    rho0 = inputs.rho_noise(n, n, 3)
    states = []
    for kw in (dict(tile_x=tx, tile_y=ty), {}):
        sim = LBSim(rho0, G1=G1, G2=G2, storage="f32", steps_per_launch=2, **kw)
        sim.step(20)
        states.append(sim.get_state())
        sim.close()
    assert np.array_equal(states[0].view(np.uint32), states[1].view(np.uint32))


def test_batch_two_step_tuner_on_the_device(cache):
    lats = []
    for k, n in enumerate((96, 160, 200)):
        G1, G2 = inputs.couplings(0.04 * k)
        lats.append(dict(rho_init=inputs.rho_noise(n, n, 40 + k), G1=G1, G2=G2, tile_y=16))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch = LBBatch(lats, storage="f32", tile_x=64, steps_per_launch=2)
        print("tuning the batch's two-step tile height", flush=True)
        ty = A.tune_batch_two_step(batch, heights=(8, 16, 24), steps=6)
        assert ty in (8, 16, 24)
        assert batch.two_step_shape()[:2] == (128, ty)
        (entry,) = json.loads(cache.read_text()).values()
        assert entry["tile_y"] == ty and entry["us_per_step"] > 0
        # From the cache on a second call, without stepping the batch.
        t0 = batch[0].t
        assert A.tune_batch_two_step(batch, heights=(8, 16, 24)) == ty
        assert batch[0].t == t0
        batch.close()
