"""Regression fixtures of the CPU oracle (tests/golden/oracle_regression.json, written by
tests/golden/make_golden.py): digests of its outputs on small seeded cases. They guard the oracle against
unintended changes; what the oracle computes is pinned by the other tests/test_oracle_*.py files."""
import json
import os

import pytest

from tests.golden import make_golden

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_regression.json")


@pytest.fixture(scope="module")
def current():
    return make_golden.cases()


def test_oracle_matches_its_regression_fixture(current):
    want = json.load(open(GOLDEN))
    assert set(current) == set(want)
    for k in want:
        got = json.loads(json.dumps(current[k]))  # the same float formatting as the stored file
        assert got == want[k], k
