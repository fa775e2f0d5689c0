"""The oracle against its own stored outputs (regression guard; see tests/golden)."""
import json
import os

import numpy as np
import pytest

from tests.golden.make_golden import CASES, HERE, summary


@pytest.mark.parametrize("cfg,seed,scale", CASES)
def test_oracle_matches_golden(cfg, seed, scale):
    with open(os.path.join(HERE, f"oracle_{cfg}_seed{seed}.json")) as f:
        ref = json.load(f)
    got = summary(cfg, seed, scale)
    for k, v in ref.items():
        if k == "first_params_fp64":
            assert np.allclose(got[k], v, rtol=1e-12, atol=1e-12)
        else:
            assert got[k] == v, k
