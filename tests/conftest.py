import json
import math
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _num(v):
    if isinstance(v, str):
        return float(v)
    return v


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def golden_lps():
    import synth

    out = {}
    for spec in load_golden("tiny_lps.json")["lps"]:
        out[spec["name"]] = (synth.tiny_lp(spec), spec)
    return out


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    return oracle


@pytest.fixture(scope="session")
def tiny():
    return golden_lps()
