import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# A host-sanitizer run (tests/test_host_sanitizers.py) points the binding at the ASan/UBSan
# build of the library.
if os.environ.get("QSIM_TEST_LIB"):
    import paper_1412_2293_amd.qsim as _qsim
    _qsim.LIB_PATH = os.environ["QSIM_TEST_LIB"]


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    config.addinivalue_line("markers", "bigmem: GPU test that allocates states of 64 GiB or more")


def pytest_collection_modifyitems(config, items):
    # Keep GPU tests that allocate large state vectors late within the gpu run, and the
    # allocation-free entry point's test file after everything else.
    def order(it):
        if os.path.basename(str(it.fspath)).startswith("test_zz_"):
            return 2
        return 1 if it.get_closest_marker("bigmem") else 0
    items.sort(key=order)
