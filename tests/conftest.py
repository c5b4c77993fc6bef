import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C ABI)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _ensure_built():
    """Builds the CPU-side libraries only when nothing is built yet."""
    import netgen.build as nb
    import oracle.build as ob
    if not os.path.exists(os.path.join(ROOT, "netgen", "libdbnet.so")):
        nb.build()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        ob.build()


_ensure_built()
