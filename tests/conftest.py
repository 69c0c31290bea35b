import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Autotuning in the tests must not write a user tuning cache that later launches would read;
# tests of the cache point LTL_TUNE_CACHE at files of their own.
os.environ.setdefault("LTL_TUNE_CACHE", "off")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")
