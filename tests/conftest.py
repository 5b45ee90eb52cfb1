import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def m13_path():
    from paper_1607_03884_amd import configs
    return configs.mech_path("M13")


@pytest.fixture(scope="session")
def m53_path():
    from paper_1607_03884_amd import configs
    return configs.mech_path("M53")


@pytest.fixture(scope="session")
def m13(oracle_mod, m13_path):
    return oracle_mod.Mech(m13_path)


@pytest.fixture(scope="session")
def m53(oracle_mod, m53_path):
    return oracle_mod.Mech(m53_path)
