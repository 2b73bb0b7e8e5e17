"""The lambda calibration of Fig. 5 on the GPU path (paper Sec. 3.2): Phi(t)
(Eq. 4) of the sub-lattice algorithm at c = 0.42 against a near-serial
reference (one sub-lattice covering the lattice, lambda = 2).  Statistical, with
margins several times the spread seen over 120 realizations: the sub-lattice
algorithm with the paper's lambda = 16 and its balanced variant follow the
reference closely, while the checkerboard sweep does not (the paper's reason
for the sub-lattice algorithm)."""
import pytest

from paper_1209_0296_amd.calibrate import calibrate

pytestmark = pytest.mark.gpu


def test_lambda_calibration_at_c042():
    r = calibrate(64, 0.42, 32, [16], [1, 4, 16, 64], realizations=30, others=True)
    lam16 = r["candidates"][0]
    assert lam16["max_abs_dev"] < 0.04, lam16
    assert r["balanced"]["max_abs_dev"] < 0.025, r["balanced"]
    assert r["checkerboard"]["max_abs_dev"] > 0.1, r["checkerboard"]
    # Phi decays from 1 and stays positive over this window
    ref = r["reference"]["phi"]
    assert 1.0 > ref[0] > ref[-1] > 0.3
