import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")
    config.addinivalue_line("markers", "slow: long CPU test")
    # the library's on-disk autotuning cache: a file of this test session, not
    # the user's cache directory
    if "NSMI_TUNE_CACHE" not in os.environ:
        import tempfile
        os.environ["NSMI_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="nsmi_tune_"), "tune.txt")
