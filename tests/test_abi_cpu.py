"""Host-side checks of liblb.so that need no GPU.

The library loads and exports every entry point include/lb.h declares, the
host-side validation rejects what the header says it rejects, and the link
tables the kernels use are bit-identical to the oracle's (which are pinned to
Table 1 in test_oracle_tables.py).
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1008_2865_amd as P
from paper_1008_2865_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 14
    L = B.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.SIGNATURES), "binding and header disagree"


def test_params_struct_layout_matches_header():
    # int32 x8, int64, double x5 -> 80 bytes, trace_cap at 32, tau at 40.
    assert ctypes.sizeof(B.lb_params) == 80
    assert B.lb_params.trace_cap.offset == 32 and B.lb_params.tau.offset == 40


def good(**kw):
    d = dict(storage=P.LB_F32, G1=-5.444444444444445, G2=0.5444444444444445, log_every=10,
             trace_cap=5)
    d.update(kw)
    return P.make_params(kw.pop("nx", 64), kw.pop("ny", 48), **{k: v for k, v in d.items()
                                                                   if k not in ("nx", "ny")})


@pytest.mark.parametrize("field,value", [
    ("nx", 4), ("ny", 3), ("storage", 7), ("tau", 0.5), ("tau", float("nan")),
    ("rho0", 0.0), ("G1", float("inf")), ("log_every", -1), ("trace_cap", -2),
    ("tile_x", 96), ("tile_y", -1), ("tile_y", 5000), ("tile_rows", 3), ("steps_per_launch", 3),
    ("steps_per_launch", -1), ("ny", 65536)])
def test_validation_rejects(field, value):
    p = good()
    setattr(p, field, value)
    assert P.lb_validate(p) == B.LB_ERR_INVALID
    assert P.lb_workspace_bytes(p) == 0
    assert P.lb_last_error()


def test_f16_needs_positive_reference():
    p = good(storage=P.LB_F16DEV, rho_ref=0.0)
    assert P.lb_validate(p) == B.LB_ERR_INVALID
    p.rho_ref = 0.7
    assert P.lb_validate(p) == B.LB_OK


def test_workspace_and_launch_shape():
    p = good(nx=2048, ny=2048, trace_cap=41)
    tx, ty, tr, nb = P.lb_launch_shape(p)
    assert tx == 256 and ty >= 1 and tr in (1, 2) and nb == (2048 // tx) * math.ceil(2048 / ty)
    # Two population buffers of 9 planes plus bookkeeping.
    assert P.lb_workspace_bytes(p) >= 2 * 9 * 2048 * 2048 * 4
    small = good(nx=5, ny=5)
    assert P.lb_launch_shape(small)[0] == 64


@pytest.mark.parametrize("G1,G2", [(-5.444444444444445, 0.5444444444444445), (1.0, 0.0), (0.0, 1.0),
                                   (-4.9, 0.0), (-5.764705882352941, 0.8647058823529412)])
def test_tables_bit_identical_to_oracle(G1, G2):
    p = good(G1=G1, G2=G2)
    cx = np.zeros(24, np.int8)
    cy = np.zeros(24, np.int8)
    K = np.zeros(24)
    KE = np.zeros(25)
    P.lb_tables(p, cx, cy, K, KE)
    ocx, ocy, oK, oKE = O.tables(G1, G2)
    assert np.array_equal(cx, ocx) and np.array_equal(cy, ocy)
    assert np.array_equal(K.view(np.uint64), oK.view(np.uint64))
    assert np.array_equal(KE.view(np.uint64), oKE.view(np.uint64))


def test_init_rejects_bad_arguments_before_any_device_call():
    p = good(nx=8, ny=8)
    n = P.lb_workspace_bytes(p)
    rho = np.full((8, 8), 0.7)
    with pytest.raises(B.LBError) as e:
        P.lb_init(p, 256, n - 1, rho)  # short workspace
    assert e.value.code == B.LB_ERR_INVALID
    with pytest.raises(B.LBError) as e:
        P.lb_init(p, 256, n, None)
    assert e.value.code == B.LB_ERR_INVALID
    for bad in (np.nan, -0.1, 0.0, np.inf):
        r = rho.copy()
        r[3, 5] = bad
        with pytest.raises(B.LBError) as e:
            P.lb_init(p, 256, n, r)
        assert e.value.code == B.LB_ERR_INVALID
    u = np.zeros((8, 8))
    u[0, 0] = np.nan
    with pytest.raises(B.LBError) as e:
        P.lb_init(p, 256, n, rho, ux_init=u)
    assert e.value.code == B.LB_ERR_INVALID
    with pytest.raises(B.LBError) as e:
        P.lb_init(p, 255, n, rho)  # misaligned workspace
    assert e.value.code == B.LB_ERR_INVALID


def test_calls_on_unknown_context_fail_cleanly():
    bogus = 0x1234560
    for fn, args in [(P.lb_step, (1,)), (P.lb_time, ()), (P.lb_destroy, ()),
                     (P.lb_pseudo_energy, (np.zeros(6),))]:
        with pytest.raises(B.LBError) as e:
            fn(bogus, *args)
        assert e.value.code == B.LB_ERR_STATE


def test_init_without_device_reports_hip_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = good(nx=8, ny=8)
    with pytest.raises(B.LBError) as e:
        P.lb_init(p, 256, P.lb_workspace_bytes(p), np.full((8, 8), 0.7))
    assert e.value.code == B.LB_ERR_HIP


def test_batch_rejects_mismatched_settings():
    # Lattices of a batch must share storage, tile_x, tile_rows, log_every
    # and trace_cap; sizes and couplings may differ.
    ok = [B.make_params(64, 64, tile_x=64), B.make_params(100, 70, tile_x=64, G2=0.3)]
    assert B.lb_batch_workspace_bytes(ok) > sum(P.lb_workspace_bytes(p) for p in ok)
    for bad in ([B.make_params(64, 64, tile_x=64), B.make_params(64, 64, tile_x=128)],
                [B.make_params(64, 64, tile_x=64), B.make_params(64, 64, tile_x=64, log_every=3)],
                [B.make_params(64, 64, tile_x=64), B.make_params(64, 64, tile_x=64, storage=P.LB_F64)],
                [B.make_params(64, 64, tile_x=64), B.make_params(4, 64, tile_x=64)],
                [B.make_params(64, 64, tile_x=64), B.make_params(64, 64, tile_x=64,
                                                                 steps_per_launch=2)]):
        assert B.lb_batch_workspace_bytes(bad) == 0
        assert P.lb_last_error()
    # Two steps per launch add a second tile list to the workspace.
    two = [B.make_params(64, 64, tile_x=64, steps_per_launch=2) for _ in range(2)]
    one = [B.make_params(64, 64, tile_x=64, steps_per_launch=1) for _ in range(2)]
    assert B.lb_batch_workspace_bytes(two) > B.lb_batch_workspace_bytes(one)
    for fn in (B.lb_batch_two_step_shape, B.lb_batch_step):
        with pytest.raises(B.LBError) as e:
            fn(0x1234560) if fn is B.lb_batch_two_step_shape else fn(0x1234560, 1)
        assert e.value.code == B.LB_ERR_STATE


def test_adjoint_host_validation():
    p = B.make_params(64, 48, storage=P.LB_F32)
    nb = B.lb_adj_workspace_bytes(p, 300, 100)
    # The forward workspace, three 9-plane checkpoints and a 100-entry tape
    # of 4 values per site.
    assert nb > P.lb_workspace_bytes(p) + (3 * 9 + 100 * 4) * 64 * 48 * 4
    assert B.lb_adj_workspace_bytes(p, 600, 100) > nb         # more checkpoints
    assert B.lb_adj_workspace_bytes(p, 0, 1) > 0               # T = 0 is valid
    # Two segments re-step one into a second tape region while the other is
    # read; a single segment (the whole run taped forward) needs one region.
    one, two = B.lb_adj_workspace_bytes(p, 100, 100), B.lb_adj_workspace_bytes(p, 101, 100)
    region = 100 * 4 * 64 * 48 * 4
    assert region <= two - one <= region + 9 * 64 * 48 * 4 + 2 * 256 + 9 * 64 * 4 * 4
    for bad in [(B.make_params(64, 48, storage=P.LB_F16DEV), 10, 5),
                (p, -1, 5), (p, 10, 0), (B.make_params(4, 48), 10, 5),
                (B.make_params(32768, 32768, storage=P.LB_F32), 10, 5)]:  # > 2^29 sites
        assert B.lb_adj_workspace_bytes(*bad) == 0
    assert B.lb_adj_workspace_bytes(B.make_params(16384, 32768, storage=P.LB_F32), 10, 5) > 0
    for fn, args in [(B.lb_adj_backward, (np.zeros((48, 64)),)), (B.lb_adj_destroy, ()),
                     (B.lb_adj_forward, (np.full((48, 64), 0.7), -5.0, 0.5, 0.0, 0.0, 1e-6))]:
        with pytest.raises(B.LBError) as e:
            fn(0x1234560, *args)
        assert e.value.code == B.LB_ERR_STATE
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        with pytest.raises(B.LBError) as e:
            B.lb_adj_init(p, 300, 100, 256, nb)
        assert e.value.code == B.LB_ERR_HIP


def test_structure_factor_host_side():
    from oracle import structure as OS

    for L in (5, 8, 37, 64, 512, 2048):
        assert B.lb_sk_shells(L) == int(OS.shell_index(L).max()) + 1
        assert B.lb_sk_workspace_bytes(L) > 40 * L * L
    for L in (4, 2049, 0, -3):
        assert B.lb_sk_workspace_bytes(L) == 0
        with pytest.raises(B.LBError) as e:
            B.lb_sk_shells(L)
        assert e.value.code == B.LB_ERR_INVALID
    with pytest.raises(B.LBError) as e:
        B.lb_sk_compute(0x1234560, np.zeros((8, 8)), np.zeros(4), None)
    assert e.value.code == B.LB_ERR_STATE
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        with pytest.raises(B.LBError) as e:
            B.lb_sk_init(64, 256, B.lb_sk_workspace_bytes(64))
        assert e.value.code == B.LB_ERR_HIP


@pytest.mark.parametrize("n,shape", [
    (2048, (256, 32, 1, 512)),   # the tallest tile that keeps >= 512 workgroups
    (1024, (256, 8, 1, 512)),
    (512, (256, 2, 1, 512)),
    (8192, (256, 32, 1, 8192)),
    (100, (64, 2, 1, 100)),      # small lattices: 2-row tiles at least
])
def test_default_launch_shape(n, shape):
    assert B.lb_launch_shape(B.make_params(n, n)) == shape


@pytest.mark.parametrize("n,storage,spl,shape", [
    (1024, P.LB_F32, 0, (0, 0, 0)),          # tiles under 16 rows: one step per launch
    (2048, P.LB_F32, 0, (128, 23, 1530)),    # one round of resident 128-lane tiles
    (3500, P.LB_F32, 0, (256, 65, 756)),     # one round of 256-lane tiles (<= 96 rows)
    (4096, P.LB_F32, 0, (256, 92, 765)),
    (5120, P.LB_F32, 0, (256, 47, 2289)),    # about 48 rows, the last round full
    (6144, P.LB_F32, 0, (256, 51, 3025)),    # 48 rows would leave a 5th round 1/6 full
    (8192, P.LB_F32, 0, (256, 45, 6039)),
    (2048, P.LB_F32, 1, (0, 0, 0)),
    (1024, P.LB_F16DEV, 0, (0, 0, 0)),
    (2048, P.LB_F16DEV, 0, (128, 23, 1530)),  # half storage: one round as FP32
    (4096, P.LB_F16DEV, 0, (256, 92, 765)),
    (6144, P.LB_F16DEV, 0, (256, 101, 1525)),  # tallest <= 128 rows filling its rounds
    (8192, P.LB_F16DEV, 0, (256, 119, 2277)),  # three full rounds
    (8192, P.LB_F16DEV, 1, (0, 0, 0)),
    (8192, P.LB_F16DEV, 2, (256, 119, 2277)),
    (2048, P.LB_F64, 2, (0, 0, 0))])         # no double-precision two-step kernel
def test_two_step_default_shape(n, storage, spl, shape):
    p = good(nx=n, ny=n, storage=storage, steps_per_launch=spl, rho_ref=0.7)
    assert B.lb_two_step_shape(p) == shape
