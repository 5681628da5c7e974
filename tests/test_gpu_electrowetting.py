"""Equilibrium electrowetting setup (Sec. 6.3) on the GPU: a conductive drop
with density and viscosity ratios 100 and permittivity ratio 81 on the bottom
electrode, Young angle 120 degrees plus the Lippmann shift eta / d in the wetting
condition.  Parity with the oracle in the normalisation and tolerances of
test_gpu_parity (FP32 1e-5, FP16S 1e-3, inner counts replayed), at a reduced
size and at the study's 200 x 100."""
import pytest

from paper_2407_01654_amd import workloads as W
from test_gpu_parity import assert_parity, run_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp16s", 1e-3)])
def test_electrowetting_parity_reduced(prec, tol):
    wl = W.electrowetting_drop(nx=100, ny=50, r=12.0, eta_over_d=0.3)
    ora, sim, K = run_pair(wl, 60, prec=prec, launch=dict(block_x=64, band_y=16, device_loop=1))
    assert_parity(ora, sim, wl.params, tol)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp16s", 1e-3)])
def test_electrowetting_parity_full_size(prec, tol):
    wl = W.electrowetting_drop(eta_over_d=0.5, eps_v=0.5)
    ora, sim, K = run_pair(wl, 8, prec=prec, launch=dict(block_x=64, band_y=16, device_loop=1))
    assert_parity(ora, sim, wl.params, tol)
