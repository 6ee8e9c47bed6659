import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test taking more than ~20 s")


@pytest.fixture(scope="session")
def oracle():
    import oracle as O

    O.build()
    return O


@pytest.fixture(scope="session")
def inputs():
    from paper_1504_02577_amd import inputs as I

    return I


@pytest.fixture(scope="session")
def ba1k(inputs):
    return inputs.ba_graph(1000, 5)


@pytest.fixture(scope="session")
def ba1k_paths(oracle, ba1k):
    paths = oracle.walk(ba1k, 5, 100_000, 1)
    inv_ptr, inv_pid = oracle.index(ba1k.n, paths)
    return paths, inv_ptr, inv_pid


@pytest.fixture(scope="session")
def progress(request):
    """say(...) writes a progress line to the terminal at once, past output
    capture (long stages of the large-workload tests report as each ends)."""
    tr = request.config.pluginmanager.get_plugin("terminalreporter")
    capman = request.config.pluginmanager.get_plugin("capturemanager")

    def say(*a):
        msg = " ".join(str(x) for x in a)
        if tr is None or capman is None:
            print(msg, flush=True)
            return
        with capman.global_and_fixture_disabled():
            tr.write_line(msg)
            tr.flush()

    return say
