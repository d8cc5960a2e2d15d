"""The bench's own inputs for the quasi-cylindrical column (no GPU): its
ion-column profile, which the library takes as a fixed background, equals
the oracle's neutralising background for both shape orders."""

import numpy as np
import pytest

import bench
from oracle import cylindrical as cy


@pytest.mark.parametrize("name", ["qc_column", "qc_column_cubic"])
def test_ion_profile_is_the_oracle_background(name):
    w = bench.QC_WORKLOADS[name]
    got = bench.qc_ion_profile(w)
    ref = cy.uniform_cylinder_background(1.0, w["rp"], 0.0, 1, w["nr"], w["dr"], 1, w["dz"],
                                         w.get("order", 1))[0][0][0].real
    assert np.max(np.abs(got - ref)) <= 1e-13
    # whole nodes inside the column take 1, nodes beyond it 0
    reach = (w.get("order", 1) + 1) // 2
    j = np.arange(w["nr"])
    assert np.all(got[(j + 0.5 + reach) * w["dr"] <= w["rp"]] == pytest.approx(1.0, abs=1e-14))
    assert np.all(got[(j + 0.5 - reach) * w["dr"] >= w["rp"]] == 0.0)
