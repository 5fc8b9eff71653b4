"""The oracle reproduces its committed trajectories (regression fixtures
written by tests/golden/make_golden.py, which calls only the oracle)."""
import os

import numpy as np
import pytest

from tests.golden import make_golden

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    lines = open(os.path.join(HERE, name)).read().splitlines()
    giter = int(lines[1].split()[-1])
    return giter, np.array([int(s, 16) for s in lines[2:]], dtype=np.uint64)


@pytest.mark.parametrize("name", sorted(make_golden.CASES))
def test_oracle_reproduces_golden_trajectory(name):
    giter, hist = load(name)
    r = make_golden.run(make_golden.CASES[name])
    assert r["giter"] == giter
    assert np.array_equal(r["hist"], hist)
