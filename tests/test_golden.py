"""Values printed in the paper, stored as small text fixtures under tests/golden/."""
import os

import numpy as np

from oracle.ibm_oracle import RK_A, RK_B, RK_C

HERE = os.path.join(os.path.dirname(__file__), "golden")


def test_rk3_coefficients_match_paper():
    tab = np.loadtxt(os.path.join(HERE, "rk3_coefficients.txt"))
    assert np.array_equal(RK_A * 120.0, tab[:, 1])
    assert np.array_equal(RK_B * 120.0, tab[:, 2])
    assert abs(RK_C.sum() - 1.0) < 1e-15          # consistency: the stages cover one dt
    assert np.allclose(RK_C, [8 / 15, 2 / 15, 1 / 3], rtol=1e-15)
