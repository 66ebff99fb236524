import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")


_PROBLEMS = {}


def oracle_problem(name, N, k=None, **kw):
    """Build (once per session) the oracle problem of a reduced-size workload."""
    import synth
    from oracle.problem import Problem
    key = (name, N, k, tuple(sorted(kw.items())))
    if key not in _PROBLEMS:
        _PROBLEMS[key] = Problem(synth.get_config(name, N=N, k=k), **kw)
    return _PROBLEMS[key]


@pytest.fixture(scope="session")
def c1_small():
    return oracle_problem("c1", 8)


@pytest.fixture(scope="session")
def c2_small():
    return oracle_problem("c2", 8)


@pytest.fixture(scope="session")
def c3_small():
    return oracle_problem("c3", 8)


@pytest.fixture(scope="session")
def c4_small():
    return oracle_problem("c4", 8)


@pytest.fixture(scope="session")
def c1_16():
    """c1 at its named size, 16^3 (k = 1, Dirichlet top)."""
    return oracle_problem("c1", 16)


@pytest.fixture(scope="session")
def c3_16():
    return oracle_problem("c3", 16)


@pytest.fixture(scope="session")
def c4_16():
    return oracle_problem("c4", 16)


@pytest.fixture
def rng():
    return np.random.default_rng(1234)
