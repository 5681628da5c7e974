"""The drop-deformation study of Sec. 7.1 (Table 1, Fig. 8) on the GPU.
Parity of its workload (density ratio 2, W = 5, surface tension held at
1e-3 with the electrode difference following Ca_E) with the oracle at a reduced
cavity, in the normalisation and tolerances of test_gpu_parity (FP32 1e-5,
FP16S 1e-3, inner counts replayed)."""
import numpy as np
import pytest

from paper_2407_01654_amd import workloads as W
from test_gpu_parity import assert_parity, run_pair

pytestmark = pytest.mark.gpu

# Table 1 rows at a cavity of 8 radii, r = 10
CASES = {
    "R5_S5_Ca0.2": lambda: (W.deformation_drop(5.0, 5.0, 0.2, n=80), 60),
    "R5_S60_Ca0.2": lambda: (W.deformation_drop(5.0, 60.0, 0.2, n=80), 60),
    "R1.75_S3.5_Ca0.1": lambda: (W.deformation_drop(1.75, 3.5, 0.1, n=80), 60),
}


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp16s", 1e-3)])
@pytest.mark.parametrize("case", list(CASES))
def test_deformation_drop_parity_replay(case, prec, tol):
    wl, steps = CASES[case]()
    ora, sim, K = run_pair(wl, steps, prec=prec, launch=dict(block_x=64, band_y=16, device_loop=1))
    assert_parity(ora, sim, wl.params, tol)
    assert np.array_equal(sim.k_history(0), K)
