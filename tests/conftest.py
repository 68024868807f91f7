import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    alt = os.environ.get("NBODY_ORACLE_LIB")  # a mutated build, see test_oracle_mutations
    if alt:
        oracle.load_library(alt)
    elif not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def nb():
    """The ctypes binding of libnbody.so (fails loudly if it is not built)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1803_01190_amd import nbody
    return nbody


@pytest.fixture(scope="session")
def ctx(nb):
    c = nb.Context(0)
    yield c.h
    c.close()
