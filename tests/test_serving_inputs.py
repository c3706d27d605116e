"""The serving workload's host-side pieces (no GPU): the seeded request
stream and the history count a request gets from the calibration."""
import math

import numpy as np
import pytest

from paper_0910_0329_amd import serving
from paper_0910_0329_amd.inputs import configs
from paper_0910_0329_amd.inputs.sources import ELECTRON, PHOTON


def test_request_stream_is_seeded_and_in_range():
    a = configs.serving_requests(20.0, 10.0, seed=5)
    b = configs.serving_requests(20.0, 10.0, seed=5)
    c = configs.serving_requests(20.0, 10.0, seed=6)
    assert [(r.t, r.phantom, r.particle, r.side, r.target) for r in a] == \
           [(r.t, r.phantom, r.particle, r.side, r.target) for r in b]
    assert [r.t for r in a] != [r.t for r in c]
    t = np.array([r.t for r in a])
    assert np.all(np.diff(t) >= 0) and t[-1] <= 10.0
    # Poisson count over 10 s at 20/s: 200 +- 4 sigma
    assert abs(len(a) - 200) <= 4 * math.sqrt(200)
    for r in a:
        assert r.phantom in (0, 1, 2) and r.particle in (PHOTON, ELECTRON)
        assert 1.0 <= r.side <= 10.0 and r.target in (0.01, 0.02)
        assert (6.0 <= r.energy <= 20.0) if r.particle == ELECTRON else r.energy == 0.0
    assert [r.index for r in a] == list(range(len(a)))


def test_history_count_follows_the_calibration_law():
    """N_cal is interpolated in log(side) and log(N) between calibration
    points and scaled by (1% / target)^2, then clipped."""
    cal = {(0, PHOTON): [(1.0, 4e6), (3.0, 1e6), (10.0, 2e5)]}
    req = configs.ServeRequest(0, 0.0, 0, PHOTON, 0.0, 3.0, 0.01)
    # (the count is truncated to an integer after exp/log, so +-1)
    assert serving.n_histories(cal, req) == pytest.approx(1_000_000, abs=1)
    req.target = 0.02
    assert serving.n_histories(cal, req) == pytest.approx(250_000, abs=1)
    # geometric mean between the nodes at the geometric-mean side
    req.target, req.side = 0.01, math.sqrt(3.0 * 10.0)
    assert serving.n_histories(cal, req) == pytest.approx(math.sqrt(1e6 * 2e5), rel=1e-9, abs=1)
    # clipping at both ends
    req.side, req.target = 10.0, 0.02
    assert serving.n_histories(cal, req) == 100_000
    req.side, req.target = 1.0, 0.001
    assert serving.n_histories(cal, req) == 50_000_000
