"""Shared test set-up: the ``gpu`` marker, import paths and library builds."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _host_libs():
    """The generator and the oracle are plain C; build them if absent."""
    import oracle
    import synth
    for mod, name in ((synth, "libsynth.so"), (oracle, "librbsm_oracle.so")):
        if not os.path.exists(os.path.join(os.path.dirname(mod.__file__), name)):
            mod.build()
    yield
