"""Shared pytest setup.

Tests marked ``gpu`` need an MI355X and the built HIP library; everything else
runs on the CPU (the oracle, the input generators, host-side argument checks
and symbol exports of the GPU library)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    return oracle
