import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _preload_runtime():
    # One HIP runtime per process: load the system runtime by its bare name before
    # anything imports torch (see paper_1908_01949_amd.rknscan.preload_hip_runtime).
    try:
        from paper_1908_01949_amd import rknscan
        rknscan.preload_hip_runtime()
    except OSError:
        pass


_preload_runtime()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def geo():
    from paper_1908_01949_amd import synth
    return synth.make_geometry()


@pytest.fixture(scope="session")
def ufield():
    from paper_1908_01949_amd import synth
    return synth.uniform_field(1.0)


@pytest.fixture(scope="session")
def sfield():
    from paper_1908_01949_amd import synth
    return synth.solenoid_field()


@pytest.fixture(scope="session")
def orc_u(geo, ufield):
    import oracle
    return oracle.Oracle(geo, ufield)


@pytest.fixture(scope="session")
def orc_s(geo, sfield):
    import oracle
    return oracle.Oracle(geo, sfield)


@pytest.fixture(scope="session")
def ev1(geo, ufield):
    from paper_1908_01949_amd import synth
    return synth.event_single_turn(geo, ufield, 0)
