"""GPU: the structure-factor kernels (lb_sk_*) against the oracle.

The oracle (oracle/structure.py, pinned to closed forms) and the kernels
see the same density fields: seeded random fields, a single Fourier mode
and the density of a lattice after spinodal growth.  Shell averages, shell
counts, kbar and the full spectrum are compared element by element, on
power-of-two sides (FFT path) and on other sides (direct transform).
"""
import numpy as np
import pytest

from oracle import structure as OS
from paper_1008_2865_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1008_2865_amd import binding as B  # noqa: E402
from paper_1008_2865_amd.sim import LBSim  # noqa: E402
from paper_1008_2865_amd.structure import StructureFactor  # noqa: E402


def compare(rho, sk, tol=1e-12):
    Sn_o, cnt_o = OS.shells(rho)
    spec_o = OS.spectrum(rho)
    Sn, cnt, kbar, R, spec = sk(rho, spectrum=True)
    assert np.array_equal(cnt, cnt_o)
    scale = float(spec_o.max())
    assert float(np.max(np.abs(Sn - Sn_o))) <= tol * scale
    assert float(np.max(np.abs(spec.cpu().numpy() - spec_o))) <= tol * scale
    kb = OS.kbar(Sn_o)
    assert abs(kbar - kb) <= tol * kb
    assert R == pytest.approx(rho.shape[0] / (2 * kb), rel=tol)
    return Sn, kbar


@pytest.mark.parametrize("L", [8, 37, 48, 64, 512, 2048])
def test_random_fields_match_oracle(L):
    print(f"structure factor random field L={L}", flush=True)
    rho = inputs.rho_noise(L, L, L, amp=0.2)
    sk = StructureFactor(L)
    compare(rho, sk, tol=1e-12 if L <= 512 else 1e-11)
    sk.close()


@pytest.mark.parametrize("L,l0,m0", [(512, 40, 17), (100, 3, 11)])
def test_single_mode(L, l0, m0):
    y, x = np.mgrid[0:L, 0:L]
    rho = 0.7 + 0.03 * np.cos(2 * np.pi * (l0 * x + m0 * y) / L)
    sk = StructureFactor(L)
    Sn, counts, kbar, R = sk(rho)
    n0 = int(np.floor(np.hypot(l0, m0) + 0.5))
    assert kbar == pytest.approx(n0, rel=1e-11)
    assert Sn[n0] == pytest.approx(2 * 0.03 ** 2 * L * L / 4 / counts[n0], rel=1e-11)
    sk.close()


def test_reproducible_and_device_input():
    rho = inputs.rho_noise(256, 256, 5, amp=0.1)
    sk = StructureFactor(256)
    a = sk(rho)
    b = sk(torch.tensor(rho, device="cuda"))
    c = sk(rho)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[0], c[0]) and a[2] == b[2] == c[2]
    flat = np.full((256, 256), 0.7)
    with pytest.raises(B.LBError) as e:
        sk(flat)
    assert e.value.code == B.LB_ERR_NONFINITE
    sk.close()


def test_lattice_after_spinodal_growth():
    """The density of a 256^2 FP64 lattice after 1500 steps (droplets formed)."""
    G1, G2 = inputs.couplings(0.1)
    sim = LBSim(inputs.rho_noise(256, 256, 1), G1=G1, G2=G2, storage="f64")
    sim.step(1500)
    rho = sim.moments()[0]
    Sn, counts, kbar, R = sim.structure_factor()
    Sn_o, _ = OS.shells(rho)
    assert float(np.max(np.abs(Sn - Sn_o))) <= 1e-12 * float(Sn_o.max())
    assert kbar == pytest.approx(OS.kbar(Sn_o), rel=1e-12)
    print(f"kbar {kbar:.3f}, R {R:.2f} lattice units at t = 1500", flush=True)
    assert 2.0 < R < 128.0
    sim.close()
