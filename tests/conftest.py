import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_capture = None


def pytest_configure(config):
    global _capture
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C ABI)")
    _capture = config.pluginmanager.getplugin("capturemanager")


def progress(msg):
    """Print a line to the terminal past pytest's output capture (long tests
    report their steps while they run)."""
    if _capture is not None:
        with _capture.global_and_fixture_disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)
