"""Host tests of the launch-shape autotuner: which candidates it times, that it
keeps the fastest, and its cache.  The timing function is replaced by a
stand-in, so nothing here touches a GPU (the GPU test of the tuner is in
tests/test_gpu_autotune.py)."""
import json

import pytest

from paper_1008_2865_amd import autotune as A
from paper_1008_2865_amd import binding as B


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "tiles.json"
    monkeypatch.setenv("LB_TUNE_CACHE", str(path))
    return path


def fake_timer(monkeypatch, cost):
    """Replace the timing run by cost(tile_x, tile_y, tile_rows, spl); record the calls."""
    calls = []

    def time_shape(nx, ny, storage, tile_x, tile_y, tile_rows, steps=100, warmup=20,
                   steps_per_launch=1):
        calls.append((tile_x, tile_y, tile_rows, steps_per_launch))
        return cost(tile_x, tile_y, tile_rows, steps_per_launch)

    monkeypatch.setattr(A, "time_shape", time_shape)
    return calls


def test_one_step_tuner_keeps_the_fastest_and_caches(cache, monkeypatch):
    calls = fake_timer(monkeypatch, lambda tx, ty, tr, spl: {(128, 16, 1): 5.0}.get((tx, ty, tr), 9.0))
    cands = [(256, 32, 1), (128, 16, 1), (64, 4, 1), (256, 64, 2)]
    assert A.tune(300, 200, "f32", candidates=cands) == (128, 16, 1)
    assert [c[:3] for c in calls] == cands and all(c[3] == 1 for c in calls)
    stored = json.loads(cache.read_text())["f32:300x200"]
    assert (stored["tile_x"], stored["tile_y"], stored["tile_rows"], stored["us_per_step"]) == \
        (128, 16, 1, 5.0)
    # A second call answers from the cache; refresh times again.
    calls.clear()
    assert A.tune(300, 200, "f32", candidates=cands) == (128, 16, 1)
    assert calls == []
    assert A.tune(300, 200, "f32", candidates=cands, refresh=True) == (128, 16, 1)
    assert len(calls) == len(cands)


def test_one_step_tuner_clamps_and_filters(cache, monkeypatch):
    # Tiles taller than the lattice are clamped to it, tiles wider than the
    # lattice (beyond 64 lanes) are skipped, and double precision has no
    # two-rows-per-stage variant.
    calls = fake_timer(monkeypatch, lambda tx, ty, tr, spl: float(tx + ty + tr))
    A.tune(130, 10, "f64", candidates=[(256, 32, 1), (128, 32, 1), (64, 32, 1), (64, 8, 2)])
    assert [c[:3] for c in calls] == [(128, 10, 1), (64, 10, 1)]


def test_two_step_tuner_also_times_the_default_shape(cache, monkeypatch):
    # The library's default two-step shape is among the candidates even when
    # the list does not name it, so tuning never ends slower than the default.
    n = 4096
    dx, dy, _ = B.lb_two_step_shape(B.make_params(n, n, storage=B.LB_F32))
    assert (dx, dy) == (256, 92)
    calls = fake_timer(monkeypatch, lambda tx, ty, tr, spl: 1.0 if (tx, ty) == (dx, dy) else 2.0)
    assert A.tune(n, n, "f32", steps_per_launch=2) == (dx, dy, 1)
    assert (dx, dy, 1, 2) in calls and all(c[3] == 2 for c in calls)
    assert len(calls) == len(set(calls))
    assert json.loads(cache.read_text())[f"f32:{n}x{n}:two-step"]["tile_y"] == dy


def test_two_step_tuner_skips_shapes_larger_than_the_lattice(cache, monkeypatch):
    calls = fake_timer(monkeypatch, lambda tx, ty, tr, spl: float(ty))
    assert A.tune(200, 30, "f32", steps_per_launch=2) == (128, 8, 1)
    assert calls and all(tx - 6 <= 200 and ty <= 30 for tx, ty, _, _ in calls)
    # An explicit list is timed as given (no default shape added).
    calls.clear()
    A.tune(200, 30, "f32", steps_per_launch=2, candidates=[(128, 16), (128, 24)], refresh=True)
    assert [c[:2] for c in calls] == [(128, 16), (128, 24)]
