import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")
    # progress lines of long GPU tests go to the terminal as they happen, not into the capture
    from tests import gpu_common
    gpu_common.set_capture_manager(config.pluginmanager.getplugin("capturemanager"))
