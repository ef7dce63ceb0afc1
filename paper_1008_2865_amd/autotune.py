"""Launch-shape autotuner for the step kernel.

Times candidate launch shapes (columns per workgroup, rows per workgroup,
rows per pipeline stage) on the GPU for a lattice size and storage, and
caches the fastest in a JSON file (``LB_TUNE_CACHE``, default
``~/.cache/paper_1008_2865_amd/tiles.json``).  Every candidate runs the
same library kernels; the tuner only chooses among launch shapes, which do
not change the computed fields.
"""
import json
import os

import numpy as np

# (tile_x, tile_y, tile_rows).  Tall tiles re-read fewer halo rows; short
# ones keep a lattice of a few hundred rows spread over all 256 CUs.
DEFAULT_CANDIDATES = [(256, 32, 1), (256, 16, 1), (128, 32, 1), (256, 32, 2), (128, 16, 1),
                      (64, 32, 1), (256, 64, 2), (256, 8, 1), (128, 8, 1), (256, 4, 1),
                      (64, 4, 1), (256, 2, 1)]
# Two-step launches, (tile_x, tile_y): a workgroup of tile_x lanes makes
# tile_x - 6 columns.  A workgroup walks its rows one after another, so the
# heights around "every tile resident in one round" matter most; on large
# lattices taller tiles recompute fewer halo rows.  The library's default
# shape for the lattice is always timed too.
TWO_STEP_CANDIDATES = [(128, h) for h in (8, 12, 16, 20, 23, 24, 28, 32, 40, 48)] + \
                      [(256, h) for h in (24, 32, 40, 44, 46, 48, 56, 64, 80, 96, 119, 128)]
# Two-step tile heights of a batch (its tiles are 128 lanes wide).
BATCH_TWO_STEP_HEIGHTS = (16, 24, 32, 40, 48, 56, 64)


def cache_path():
    return os.environ.get("LB_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1008_2865_amd",
                                       "tiles.json"))


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(d):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_shape(nx, ny, storage, tile_x, tile_y, tile_rows, steps=100, warmup=20,
               steps_per_launch=1):
    """Microseconds per step for one launch shape: of the one-step kernel
    (steps_per_launch = 1), or of the two-step kernel (2; tile_rows unused)."""
    import torch

    from . import inputs
    from .sim import LBSim

    G1, G2 = inputs.couplings(0.1)
    sim = LBSim(inputs.rho_noise(nx, ny, 1), G1=G1, G2=G2, storage=storage, tile_x=tile_x,
                tile_y=tile_y, tile_rows=tile_rows, steps_per_launch=steps_per_launch)
    sim.step(warmup)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    sim.step(steps)
    b.record()
    torch.cuda.synchronize()
    sim.close()
    return a.elapsed_time(b) * 1e3 / steps


def tune(nx, ny, storage="f32", candidates=None, refresh=False, steps=100, steps_per_launch=1):
    """Fastest (tile_x, tile_y, tile_rows) for this size and storage: of the
    one-step kernel, or with steps_per_launch = 2 of the two-step kernel
    (candidates (tile_x, tile_y); tile_rows is returned as 1)."""
    if steps_per_launch == 2:
        return _tune_two_step(nx, ny, storage, candidates, refresh, steps)
    key = f"{storage}:{nx}x{ny}"
    cache = _load()
    if not refresh and key in cache:
        c = cache[key]
        return c["tile_x"], c["tile_y"], c["tile_rows"]
    cands = candidates or DEFAULT_CANDIDATES
    if storage == "f64":
        cands = [c for c in cands if c[2] == 1]
    best = None
    for tx, ty, tr in cands:
        if tx > max(64, nx):
            continue
        us = time_shape(nx, ny, storage, tx, min(ty, ny), tr, steps=steps)
        if best is None or us < best[0]:
            best = (us, tx, min(ty, ny), tr)
    cache[key] = {"tile_x": best[1], "tile_y": best[2], "tile_rows": best[3], "us_per_step": best[0]}
    _save(cache)
    return best[1], best[2], best[3]


def _tune_two_step(nx, ny, storage, candidates, refresh, steps):
    key = f"{storage}:{nx}x{ny}:two-step"
    cache = _load()
    if not refresh and key in cache:
        c = cache[key]
        return c["tile_x"], c["tile_y"], 1
    from . import binding as B
    from .sim import STORAGE

    cands = list(candidates or TWO_STEP_CANDIDATES)
    if candidates is None:
        dx, dy, _ = B.lb_two_step_shape(B.make_params(nx, ny, storage=STORAGE[storage],
                                                      rho_ref=1.0))
        if dx and (dx, dy) not in cands:
            cands.append((dx, dy))
    best = None
    for tx, ty in cands:
        if tx - 6 > nx or ty > ny:
            continue
        us = time_shape(nx, ny, storage, tx, ty, 1, steps=steps, steps_per_launch=2)
        if best is None or us < best[0]:
            best = (us, tx, ty)
    cache[key] = {"tile_x": best[1], "tile_y": best[2], "us_per_step": best[0]}
    _save(cache)
    return best[1], best[2], 1


def tune_batch_two_step(batch, heights=BATCH_TWO_STEP_HEIGHTS, refresh=False, steps=20):
    """Set the fastest two-step tile height on a batch that runs plain steps
    two per launch (timed on the batch itself, every lattice in each launch)
    and return it; 0 when the batch runs one step per launch.  The batch
    advances while it is timed."""
    import hashlib

    import torch

    if batch.two_step_shape()[0] == 0:
        return 0
    sig = hashlib.sha1(repr(sorted(batch.shapes)).encode()).hexdigest()[:12]
    key = f"batch-two-step:{batch.storage}:{len(batch.shapes)}:{sig}"
    cache = _load()
    if not refresh and key in cache:
        batch.set_two_step_tile(cache[key]["tile_y"])
        return cache[key]["tile_y"]
    best = None
    for ty in heights:
        batch.set_two_step_tile(ty)
        batch.step(4)  # capture (graphs) and warm up
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        batch.step(steps)
        b.record()
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / steps
        if best is None or us < best[0]:
            best = (us, ty)
    batch.set_two_step_tile(best[1])
    cache[key] = {"tile_y": best[1], "us_per_step": best[0]}
    _save(cache)
    return best[1]


def tune_batch(lattices, storage="f32", tile_x=None, tile_ys=(8, 16, 32, 64), tile_rows=(1, 2),
               refresh=False, steps=40):
    """Shared (tile_x, tile_rows, tile_y) of the one-step kernel for a batch,
    timed on the whole batch at one step per launch (one launch covers every
    lattice, so the batch's own parallelism, not a single lattice's, decides
    the best tile height).  ``lattices``
    are LBBatch lattice dicts; tile_x defaults to the widest strip every
    lattice fills."""
    import hashlib

    import torch

    from .sim import LBBatch

    shapes = [tuple(np.shape(L["rho_init"])) for L in lattices]
    if tile_x is None:
        m = min(nx for _, nx in shapes)
        tile_x = 256 if m >= 256 else 128 if m >= 128 else 64
    sig = hashlib.sha1(repr(sorted(shapes)).encode()).hexdigest()[:12]
    key = f"batch:{storage}:{len(shapes)}:{sig}:x{tile_x}"
    cache = _load()
    if not refresh and key in cache:
        c = cache[key]
        return c["tile_x"], c["tile_rows"], c["tile_y"]
    best = None
    for tr in tile_rows:
        if storage == "f64" and tr != 1:
            continue
        for ty in tile_ys:
            lats = [dict(L, tile_y=min(ty, sh[0])) for L, sh in zip(lattices, shapes)]
            batch = LBBatch(lats, storage=storage, tile_x=tile_x, tile_rows=tr, steps_per_launch=1)
            batch.step(10)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            batch.step(steps)
            b.record()
            torch.cuda.synchronize()
            us = a.elapsed_time(b) * 1e3 / steps
            batch.close()
            del batch
            if best is None or us < best[0]:
                best = (us, ty, tr)
    cache[key] = {"tile_x": tile_x, "tile_rows": best[2], "tile_y": best[1], "us_per_step": best[0]}
    _save(cache)
    return tile_x, best[2], best[1]
