"""Shared test configuration.

`gpu` marks tests that need an MI355X (they call the HIP library through
its C ABI); everything else runs on the CPU.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than ~20 s on the CPU")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O

    O.lib()
    return O


_TABLES = {}


@pytest.fixture(scope="session")
def table_cache(oracle):
    """Oracle tables built once per session, keyed by their parameters."""

    def get(**kw):
        tp = oracle.table_params(**kw)
        key = tuple(getattr(tp, f) for f, _ in tp._fields_)
        if key not in _TABLES:
            _TABLES[key] = oracle.build_table(tp)
        return tp, _TABLES[key]

    return get
